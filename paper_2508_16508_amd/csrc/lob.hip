// lob.hip -- abm_lob_init / abm_lob_step: noisy traders on many limit order
// books, every book matched at once each step (Sec. 5.3, Fig. 5; the paper
// vectorises the matching over books, Table 4).
//
// One workgroup of 1024 threads owns one book for a whole call, with the
// book's order slots (side, price, qty, time, alive) in LDS.  A step:
//   expiry    orders placed E or more steps ago are cancelled;
//   orders    trader k (one per thread) orders when its draw is below
//             T_order; a block scan gives the new orders their rank in trader
//             order and the free slots theirs, and the free slot of rank j
//             takes new order j (the j-th lowest free slot, as add_agents);
//   rank      each live order's position in its side's price-time priority
//             (price, then time, then slot) is the number of same-side orders
//             with a smaller 64-bit priority key: a brute-force count over
//             the book (all lanes of a wave read the same key, so the LDS
//             serves it as a broadcast);
//   cumsum    block scans of the quantities in priority order give CB and CS;
//   volume    V = max over buys r of min(CB_r, CS(p_r)), CS(p) found by a
//             binary search of the sell prices (ascending along the list);
//   fills     an order fills the part of its share range below V: filled
//             orders are removed, partly filled ones keep the rest; the new
//             last price is the floor of the mean of the buy and sell prices
//             covering share V.
// Draws are keyed on (seed + book, step, trader, purpose).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "rng.hpp"

namespace abm {
namespace {

constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxCap = 1024;
constexpr int kMaxTraders = 1024;
constexpr int32_t kMaxPrice = (1 << 24) - 1;

enum LobPurpose : uint32_t { kLobOrder = 0x40, kLobSide = 0x41, kLobPrice = 0x42, kLobQty = 0x43 };
enum LobCol : int {
    kBuys = 0, kSells, kPlaced, kDropped, kExpired, kVolume, kFilled, kPrice, kCols
};

struct LobArgs {
    int32_t cap, traders;
    uint32_t T_order;
    int32_t spread, max_qty, expiry, price0;
    uint32_t seed;
    int32_t *side, *price, *qty, *time, *alive, *last_price;
    int64_t* stats;
    int32_t n_books;
    uint32_t step0;
    int32_t n_steps;
};

// Block-wide inclusive scan of one int32 per thread; `tot` receives the total.
__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t* wsum, int32_t* tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int q = 0; q < kWaves; ++q) {
        const int32_t s = wsum[q];
        before += q < w ? s : 0;
        all += s;
    }
    *tot = all;
    return before + x;
}

__device__ __forceinline__ int32_t block_max_i32(int32_t v, int32_t* wsum) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t m = 0;
    for (int q = 0; q < kWaves; ++q) m = max(m, wsum[q]);
    return m;
}

// Price-time priority key of a live order: smaller is matched first.
__device__ __forceinline__ uint64_t priority_key(int32_t side, int32_t price, int32_t time,
                                                 int32_t slot) {
    const uint64_t p = side == 0 ? uint64_t(kMaxPrice - price) : uint64_t(price);
    return (p << 40) | (uint64_t(uint32_t(time) & 0xFFFFFFu) << 16) | uint64_t(slot);
}

__global__ __launch_bounds__(kBlock) void k_lob_run(LobArgs a) {
    __shared__ int32_t o_side[kMaxCap], o_price[kMaxCap], o_qty[kMaxCap], o_time[kMaxCap],
        o_alive[kMaxCap];
    __shared__ uint64_t key[2 * kMaxCap];         // packed priority keys, buys then sells
    __shared__ int32_t list[2][kMaxCap];          // slot at each priority position, per side
    __shared__ int32_t cum[2][kMaxCap + 1];       // exclusive cumulative shares, per side
    __shared__ int32_t wsum[kWaves];
    __shared__ int32_t cnt[kCols], share_price[2];
    int32_t* new_side = list[0];                  // new orders reuse the matching arrays
    int32_t* new_price = list[1];
    int32_t* new_qty = cum[0];
    const int32_t C = a.cap, tid = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * C;
    const uint32_t seed = a.seed + blockIdx.x;
    int32_t last = a.last_price[blockIdx.x];
    if (tid < C) {
        o_side[tid] = a.side[base + tid];
        o_price[tid] = a.price[base + tid];
        o_qty[tid] = a.qty[base + tid];
        o_time[tid] = a.time[base + tid];
        o_alive[tid] = a.alive[base + tid];
    }
    __syncthreads();
    for (int32_t k = 0; k < a.n_steps; ++k) {
        const uint32_t t = a.step0 + uint32_t(k);
        const uint64_t skey = stream_key(seed, t);
        if (tid < kCols) cnt[tid] = 0;
        __syncthreads();
        // ---- expiry
        if (tid < C && o_alive[tid] && int64_t(t) - o_time[tid] >= a.expiry) {
            o_alive[tid] = 0;
            atomicAdd(&cnt[kExpired], 1);
        }
        // ---- new orders: rank among this step's orders in trader order
        bool want = false;
        int32_t side = 0, price = 0, qty = 0;
        if (tid < a.traders) {
            want = draw(skey, uint32_t(tid), kLobOrder) < a.T_order;
            int64_t p = int64_t(last) - a.spread +
                        scale(draw(skey, uint32_t(tid), kLobPrice), uint32_t(2 * a.spread + 1));
            price = int32_t(p < 1 ? 1 : (p > kMaxPrice ? kMaxPrice : p));
            side = draw(skey, uint32_t(tid), kLobSide) < 0x80000000u ? 0 : 1;
            qty = 1 + int32_t(scale(draw(skey, uint32_t(tid), kLobQty), uint32_t(a.max_qty)));
        }
        int32_t n_new;
        const int32_t j = block_incl_scan(want ? 1 : 0, wsum, &n_new) - 1;
        if (want) {
            new_side[j] = side;
            new_price[j] = price;
            new_qty[j] = qty;
        }
        __syncthreads();   // expiry is done before the free slots are ranked
        const bool is_free = tid < C && o_alive[tid] == 0;
        int32_t n_free;
        const int32_t f = block_incl_scan(is_free ? 1 : 0, wsum, &n_free) - 1;
        if (is_free && f < n_new) {
            o_side[tid] = new_side[f];
            o_price[tid] = new_price[f];
            o_qty[tid] = new_qty[f];
            o_time[tid] = int32_t(t);
            o_alive[tid] = 1;
        }
        if (tid == 0) {
            cnt[kPlaced] = n_new < n_free ? n_new : n_free;
            cnt[kDropped] = n_new - cnt[kPlaced];
        }
        __syncthreads();
        // ---- priority ranks: the live orders of each side are packed (in slot
        // order) into key[0, nb) and key[C, C + ns); an order's rank is the
        // number of keys of its side below its own (a brute-force count)
        const bool live = tid < C && o_alive[tid] != 0;
        const int32_t my_side = live ? o_side[tid] : -1;
        uint64_t my_key = ~0ull;
        if (live) my_key = priority_key(o_side[tid], o_price[tid], o_time[tid], tid);
        int32_t nb, ns;
        const int32_t jb = block_incl_scan(my_side == 0 ? 1 : 0, wsum, &nb) - 1;
        const int32_t js = block_incl_scan(my_side == 1 ? 1 : 0, wsum, &ns) - 1;
        if (my_side == 0) key[jb] = my_key;
        if (my_side == 1) key[C + js] = my_key;
        __syncthreads();
        int32_t rank = 0;
        if (live) {
            const uint64_t* k_side = key + (my_side ? C : 0);
            const int32_t n_side = my_side ? ns : nb;
            for (int32_t q = 0; q < n_side; ++q) rank += k_side[q] < my_key ? 1 : 0;
        }
        __syncthreads();   // new-order buffers (aliasing list / cum) are no longer read
        if (live) list[my_side][rank] = tid;
        __syncthreads();
        // ---- cumulative shares along each side's priority order
        for (int s = 0; s < 2; ++s) {
            const int32_t n = s ? ns : nb;
            const int32_t q = tid < n ? o_qty[list[s][tid]] : 0;
            int32_t total;
            const int32_t incl = block_incl_scan(q, wsum, &total);
            if (tid < n) cum[s][tid + 1] = incl;
            if (tid == 0) cum[s][0] = 0;
        }
        __syncthreads();
        // ---- volume: V = max over buys of min(CB_r, CS(p_r))
        int32_t v = 0;
        if (tid < nb) {
            const int32_t pb = o_price[list[0][tid]];
            int32_t lo = 0, hi = ns;                 // sells priced at most pb: [0, lo)
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (o_price[list[1][mid]] <= pb) lo = mid + 1; else hi = mid;
            }
            v = min(cum[0][tid + 1], cum[1][lo]);
        }
        const int32_t V = block_max_i32(v, wsum);
        // the orders covering share V set the new last price
        for (int s = 0; s < 2; ++s) {
            const int32_t n = s ? ns : nb;
            if (V > 0 && tid < n && cum[s][tid] < V && V <= cum[s][tid + 1])
                share_price[s] = o_price[list[s][tid]];
        }
        __syncthreads();
        if (V > 0) last = int32_t((int64_t(share_price[0]) + share_price[1]) / 2);
        // ---- fills
        for (int s = 0; s < 2; ++s) {
            const int32_t n = s ? ns : nb;
            if (tid < n) {
                const int32_t i = list[s][tid];
                const int32_t fill = V - cum[s][tid];
                if (fill > 0) {
                    if (fill >= o_qty[i]) o_alive[i] = 0; else o_qty[i] -= fill;
                    atomicAdd(&cnt[kFilled], 1);
                }
            }
        }
        __syncthreads();
        if (tid < C && o_alive[tid]) atomicAdd(&cnt[o_side[tid] ? kSells : kBuys], 1);
        __syncthreads();
        if (tid == 0) {
            cnt[kVolume] = V;
            cnt[kPrice] = last;
        }
        __syncthreads();
        if (a.stats && tid < kCols)
            a.stats[(int64_t(k) * a.n_books + blockIdx.x) * kCols + tid] = cnt[tid];
    }
    __syncthreads();
    if (tid < C) {
        a.side[base + tid] = o_side[tid];
        a.price[base + tid] = o_price[tid];
        a.qty[base + tid] = o_qty[tid];
        a.time[base + tid] = o_time[tid];
        a.alive[base + tid] = o_alive[tid];
    }
    if (tid == 0) a.last_price[blockIdx.x] = last;
}

__global__ __launch_bounds__(256) void k_lob_clear(LobArgs a, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        a.side[i] = 0;
        a.price[i] = 0;
        a.qty[i] = 0;
        a.time[i] = 0;
        a.alive[i] = 0;
        if (i < a.n_books) a.last_price[i] = a.price0;
    }
}

int check_lob(const abm_lob_params* p, const abm_lob_state* s) {
    if (!p || !s) return fail(ABM_E_INVALID, "params or state is NULL");
    if (p->cap < 1 || p->cap > kMaxCap) return fail(ABM_E_INVALID, "cap must be in [1, 1024]");
    if (p->traders < 0 || p->traders > kMaxTraders)
        return fail(ABM_E_INVALID, "traders must be in [0, 1024]");
    if (p->spread < 0 || p->spread > (1 << 22)) return fail(ABM_E_INVALID, "spread must be in [0, 2^22]");
    if (p->max_qty < 1 || p->max_qty > (1 << 20)) return fail(ABM_E_INVALID, "max_qty must be in [1, 2^20]");
    if (p->expiry < 1) return fail(ABM_E_INVALID, "expiry must be >= 1");
    if (p->price0 < 1 || p->price0 > kMaxPrice) return fail(ABM_E_INVALID, "price0 must be in [1, 2^24)");
    if (s->n_books < 1 || s->n_books > (1 << 20)) return fail(ABM_E_INVALID, "n_books must be in [1, 2^20]");
    if (!s->side || !s->price || !s->qty || !s->time || !s->alive || !s->last_price)
        return fail(ABM_E_INVALID, "book array is NULL");
    return ABM_OK;
}

LobArgs lob_args(const abm_lob_params* p, const abm_lob_state* s) {
    LobArgs a;
    a.cap = p->cap;
    a.traders = p->traders;
    a.T_order = p->T_order;
    a.spread = p->spread;
    a.max_qty = p->max_qty;
    a.expiry = p->expiry;
    a.price0 = p->price0;
    a.seed = p->seed;
    a.side = s->side;
    a.price = s->price;
    a.qty = s->qty;
    a.time = s->time;
    a.alive = s->alive;
    a.last_price = s->last_price;
    a.stats = s->stats;
    a.n_books = s->n_books;
    a.step0 = s->step;
    a.n_steps = 0;
    return a;
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_lob_init(const abm_lob_params* p, abm_lob_state* s, void* stream) {
    int rc = check_lob(p, s);
    if (rc != ABM_OK) return rc;
    rc = check_device();
    if (rc != ABM_OK) return rc;
    LobArgs a = lob_args(p, s);
    const int64_t n = int64_t(s->n_books) * p->cap;
    const int64_t m = n > s->n_books ? n : s->n_books;
    const int64_t blocks = (m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_lob_clear, dim3(uint32_t(blocks)), dim3(256), 0, as_stream(stream), a, m);
    rc = launch_status("lob_init");
    if (rc == ABM_OK) s->step = 0;
    return rc;
}

extern "C" int abm_lob_step(const abm_lob_params* p, abm_lob_state* s, int32_t n_steps,
                            void* stream) {
    int rc = check_lob(p, s);
    if (rc != ABM_OK) return rc;
    if (n_steps < 0) return fail(ABM_E_INVALID, "n_steps must be >= 0");
    if (uint64_t(s->step) + uint64_t(n_steps) > (1u << 24))
        return fail(ABM_E_INVALID, "steps beyond 2^24 are not supported (order times are 24-bit keys)");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    if (n_steps == 0) return ABM_OK;
    LobArgs a = lob_args(p, s);
    a.n_steps = n_steps;
    hipLaunchKernelGGL(k_lob_run, dim3(uint32_t(s->n_books)), dim3(kBlock), 0, as_stream(stream), a);
    rc = launch_status("lob_step");
    if (rc == ABM_OK) s->step += uint32_t(n_steps);
    return rc;
}
