// select.hip -- abm_select_update, abm_add_agents, abm_select_indices.
//
// One single-pass kernel per call: each tile ranks its selected slots (wave
// ballot + mbcnt, LDS scan of wave totals, decoupled look-back), then every
// selected slot of rank j < q PULLS record j and writes it into its own slot.
// Pulling (the slot owner reads the record) rather than pushing means every
// slot is written by the one thread that also read its mask/alive bit, so the
// scatter needs no synchronisation beyond the rank itself.  This is the O(n)
// counterpart of the paper's Rank-Match (Sec. 4, Alg. 1): the rank *is* the
// index of the matching record, so no n x m candidate matrix or argmax is built.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
constexpr int kSlotsPerLane = 32;
constexpr int64_t kTile = int64_t(kBlock) * kSlotsPerLane;   // 8192 slots

enum SelMode : int { kSelDense = 0, kSelIndirect = 1, kAddDense = 2, kCompact = 3 };

struct SelArgs {
    int32_t* dst[ABM_MAX_ATTRS];
    const int32_t* rec[ABM_MAX_ATTRS];
    const uint8_t* mask;      // select / compact: slot mask
    int32_t* alive;           // add: free = (alive == 0); placed slots set to 1
    const int32_t* rec_idx;   // indirect: ascending indices of the selected records
    const int64_t* d_q;       // indirect: number of selected records (device)
    int32_t* out_idx;         // compact: ascending selected indices
    int64_t q;                // dense: number of records
    int64_t n;                // slots
    int64_t* d_applied;       // placed records (compact: number selected)
    int64_t* d_dropped;
    uint64_t* status;
    EpochArg epoch;
    uint32_t ntiles;
    int32_t n_attrs;
    int32_t vec_ok;           // mask / alive allow 16-byte loads
};

// Selection bits of the 32 consecutive slots [first, first + 32): bit k is
// slot first + k.  Two 16-byte loads of the mask (or eight of alive) per lane.
template <int MODE>
__device__ __forceinline__ uint32_t load_bits(const SelArgs& a, int64_t first) {
    uint32_t bits = 0;
    if (a.vec_ok && first + kSlotsPerLane <= a.n) {
        if (MODE == kAddDense) {
            const int4* p = reinterpret_cast<const int4*>(a.alive + first);
            int4 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = p[q];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                bits |= uint32_t(v[q].x == 0) << (4 * q) | uint32_t(v[q].y == 0) << (4 * q + 1) |
                        uint32_t(v[q].z == 0) << (4 * q + 2) | uint32_t(v[q].w == 0) << (4 * q + 3);
        } else {
            const uint4* p = reinterpret_cast<const uint4*>(a.mask + first);
            const uint4 m0 = p[0], m1 = p[1];
            const uint32_t w[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bits |= uint32_t(((w[q] >> (8 * b)) & 0xFFu) != 0u) << (4 * q + b);
        }
    } else {
        for (int k = 0; k < kSlotsPerLane; ++k) {
            const int64_t s = first + k;
            if (s >= a.n) break;
            const bool sel = (MODE == kAddDense) ? a.alive[s] == 0 : a.mask[s] != 0;
            bits |= uint32_t(sel) << k;
        }
    }
    return bits;
}

// One tile of 8192 slots per block (a 2^24-slot launch is one round of
// resident blocks).  Phase 1 ranks the tile's selected slots (lane-major: lane
// t owns slots [32 t, 32 t + 32) of the tile) and writes their tile-local
// offsets, in rank order, into LDS.  Phase 2 walks those rank positions with
// consecutive threads, so the reads of records j, j+1, ... are contiguous and
// every load/store batch is branch-free.  (Rewriting whole destination lines
// instead would not pay: a partial 4-byte write costs the memory a line read
// and write, but so does reading the line to fill in the unselected slots.)
//
// NA is the attribute count rounded up to 1, 2, 4, 8 or 16; the host repeats
// the last attribute's pointers in the padding entries (the repeated copy
// writes the same value to the same slot).  A compile-time count keeps the
// load and store batches free of branches, so the compiler can overlap them.
template <int MODE, int NA>
__global__ __launch_bounds__(kBlock) void k_select(SelArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint16_t pos[kTile];
    const uint32_t tile = blockIdx.x;
    const uint32_t epoch = read_epoch(a.epoch);
    const int64_t tbase = int64_t(tile) * kTile;
    const int64_t lbase = tbase + int64_t(threadIdx.x) * kSlotsPerLane;
    const uint32_t bits0 = load_bits<MODE>(a, lbase);

    uint32_t r0, total;
    const uint32_t tile_excl = rank_counts<kWaves>(__popc(bits0), &r0, a.status, a.status - 1,
                                                   tile, a.ntiles, epoch, lds, &total);

    if (MODE == kCompact) {
        uint32_t bits = bits0, r = r0;
        while (bits) {
            const uint32_t k = __ffs(bits) - 1;
            bits &= bits - 1;
            a.out_idx[int64_t(tile_excl) + r++] = int32_t(lbase + k);
        }
        if (tile == a.ntiles - 1 && threadIdx.x == 0) *a.d_applied = int64_t(tile_excl) + total;
        return;
    }

    {
        uint32_t bits = bits0, r = r0;
        while (bits) {
            const uint32_t k = __ffs(bits) - 1;
            bits &= bits - 1;
            pos[r++] = uint16_t(threadIdx.x * kSlotsPerLane + k);
        }
    }
    __syncthreads();
    const int64_t q = (MODE == kSelIndirect) ? *a.d_q : a.q;
    const int64_t room = q - int64_t(tile_excl);
    const uint32_t lim = room <= 0 ? 0u : (room < int64_t(total) ? uint32_t(room) : total);
    // Two rank positions per thread and iteration (up to 32 loads in flight).
    // When the second position is past the end it aliases the first: the same
    // value goes to the same slot twice, which keeps the stores unconditional.
    for (uint32_t p0 = threadIdx.x; p0 < lim; p0 += 2 * kBlock) {
        const uint32_t p1 = p0 + kBlock;
        const bool has1 = p1 < lim;
        const int64_t j0 = int64_t(tile_excl) + p0;
        const int64_t j1 = int64_t(tile_excl) + (has1 ? p1 : p0);
        const int64_t s0 = (MODE == kSelIndirect) ? a.rec_idx[j0] : j0;
        const int64_t s1 = (MODE == kSelIndirect) ? a.rec_idx[j1] : j1;
        const int64_t d0 = tbase + pos[p0];
        const int64_t d1 = tbase + pos[has1 ? p1 : p0];
        int32_t v0[NA], v1[NA];
#pragma unroll
        for (int at = 0; at < NA; ++at) {
            v0[at] = a.rec[at][s0];
            v1[at] = a.rec[at][s1];
        }
#pragma unroll
        for (int at = 0; at < NA; ++at) {
            a.dst[at][d0] = v0[at];
            a.dst[at][d1] = v1[at];
        }
        if (MODE == kAddDense) {
            a.alive[d0] = 1;
            a.alive[d1] = 1;
        }
    }
    if (tile == a.ntiles - 1 && threadIdx.x == 0) {
        const int64_t p = int64_t(tile_excl) + total;
        const int64_t rr = p < q ? p : q;
        *a.d_applied = rr;
        if (a.d_dropped) *a.d_dropped = q - rr;
    }
}

// Writes the counts of a call that has nothing to scan.
__global__ void k_counts(const int64_t* d_q, int64_t q, int64_t* d_applied, int64_t* d_dropped) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t qq = d_q ? *d_q : q;
        if (d_applied) *d_applied = 0;
        if (d_dropped) *d_dropped = qq;
    }
}

int check_soa(const abm_soa* s, bool need_alive) {
    if (!s) return fail(ABM_E_INVALID, "collection is NULL");
    if (s->n_attrs < 1 || s->n_attrs > ABM_MAX_ATTRS)
        return fail(ABM_E_INVALID, "n_attrs must be in [1, 16]");
    if (s->capacity < 0 || s->capacity > kMaxIndex)
        return fail(ABM_E_INVALID, "capacity must be in [0, 2^31)");
    if (s->capacity > 0)
        for (int a = 0; a < s->n_attrs; ++a)
            if (!s->attr[a]) return fail(ABM_E_INVALID, "attribute pointer is NULL");
    if (need_alive && s->capacity > 0 && !s->alive)
        return fail(ABM_E_INVALID, "alive array is required");
    return ABM_OK;
}

int check_records(const abm_records* r, int32_t n_attrs) {
    if (!r) return fail(ABM_E_INVALID, "records are NULL");
    if (r->n_attrs != n_attrs) return fail(ABM_E_INVALID, "record and slot attribute counts differ");
    if (r->count < 0 || r->count > kMaxIndex)
        return fail(ABM_E_INVALID, "record count must be in [0, 2^31)");
    if (r->count > 0)
        for (int a = 0; a < r->n_attrs; ++a)
            if (!r->attr[a]) return fail(ABM_E_INVALID, "record attribute pointer is NULL");
    return ABM_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int padded_attrs(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : 16; }

// Fills the attribute pointer tables, repeating the last attribute up to the
// padded count.
void fill_attrs(SelArgs& a, const abm_soa* dst, const abm_records* rec) {
    const int n = dst->n_attrs, na = padded_attrs(n);
    for (int i = 0; i < na; ++i) {
        const int src = i < n ? i : n - 1;
        a.dst[i] = dst->attr[src];
        a.rec[i] = rec->attr[src];
    }
    a.n_attrs = na;
}

template <int MODE>
void launch_select(const SelArgs& a, hipStream_t st) {
    const dim3 grid(a.ntiles), block(kBlock);
    switch (a.n_attrs) {
        case 1: hipLaunchKernelGGL((k_select<MODE, 1>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_select<MODE, 2>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_select<MODE, 4>), grid, block, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_select<MODE, 8>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((k_select<MODE, 16>), grid, block, 0, st, a); break;
    }
}

int launch_compact(const uint8_t* mask, int64_t n, int32_t* out, int64_t* d_count,
                   const Workspace& w, hipStream_t st) {
    SelArgs c = {};
    c.mask = mask;
    c.out_idx = out;
    c.d_applied = d_count;
    c.n = n;
    c.status = w.status;
    int rc = next_epoch(w, st, &c.epoch);
    if (rc != ABM_OK) return rc;
    c.ntiles = static_cast<uint32_t>(tiles_for(n, kTile));
    c.vec_ok = aligned16(mask);
    hipLaunchKernelGGL((k_select<kCompact, 1>), dim3(c.ntiles), dim3(kBlock), 0, st, c);
    return launch_status("select_indices");
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_select_update(const abm_soa* dst, const uint8_t* sel_mask,
                                 const abm_records* upd, const uint8_t* upd_mask,
                                 int64_t* d_applied, int64_t* d_dropped, void* ws,
                                 size_t ws_bytes, void* stream) {
    int rc = check_soa(dst, false);
    if (rc != ABM_OK) return rc;
    rc = check_records(upd, dst->n_attrs);
    if (rc != ABM_OK) return rc;
    if (!d_applied) return fail(ABM_E_INVALID, "d_applied is NULL");
    if (dst->capacity > 0 && !sel_mask) return fail(ABM_E_INVALID, "sel_mask is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const int64_t cap = dst->capacity > upd->count ? dst->capacity : upd->count;
    rc = check_ws(ws, ws_bytes, cap);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, cap);
    hipStream_t st = as_stream(stream);

    const int64_t* d_q = nullptr;
    if (upd_mask && upd->count > 0) {
        d_q = reinterpret_cast<const int64_t*>(w.hdr + kHdrCountA);
        rc = launch_compact(upd_mask, upd->count, w.list_a,
                            reinterpret_cast<int64_t*>(w.hdr + kHdrCountA), w, st);
        if (rc != ABM_OK) return rc;
    }
    const bool nothing = dst->capacity == 0 || upd->count == 0;
    if (nothing) {
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, d_q, upd_mask ? 0 : upd->count,
                           d_applied, d_dropped);
        return launch_status("select_update");
    }
    SelArgs a = {};
    fill_attrs(a, dst, upd);
    a.mask = sel_mask;
    a.rec_idx = w.list_a;
    a.d_q = d_q;
    a.q = upd->count;
    a.n = dst->capacity;
    a.d_applied = d_applied;
    a.d_dropped = d_dropped;
    a.status = w.status;
    a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
    a.vec_ok = aligned16(sel_mask);
    rc = next_epoch(w, st, &a.epoch);
    if (rc != ABM_OK) return rc;
    if (d_q)
        launch_select<kSelIndirect>(a, st);
    else
        launch_select<kSelDense>(a, st);
    return launch_status("select_update");
}

extern "C" int abm_add_agents(const abm_soa* dst, const abm_records* newborn, int64_t* d_added,
                              int64_t* d_dropped, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_soa(dst, true);
    if (rc != ABM_OK) return rc;
    rc = check_records(newborn, dst->n_attrs);
    if (rc != ABM_OK) return rc;
    if (!d_added) return fail(ABM_E_INVALID, "d_added is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_ws(ws, ws_bytes, dst->capacity);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, dst->capacity);
    hipStream_t st = as_stream(stream);
    if (dst->capacity == 0 || newborn->count == 0) {
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, nullptr, newborn->count, d_added,
                           d_dropped);
        return launch_status("add_agents");
    }
    SelArgs a = {};
    fill_attrs(a, dst, newborn);
    a.alive = dst->alive;
    a.q = newborn->count;
    a.n = dst->capacity;
    a.d_applied = d_added;
    a.d_dropped = d_dropped;
    a.status = w.status;
    a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
    a.vec_ok = aligned16(dst->alive);
    rc = next_epoch(w, st, &a.epoch);
    if (rc != ABM_OK) return rc;
    launch_select<kAddDense>(a, st);
    return launch_status("add_agents");
}

extern "C" int abm_select_indices(const uint8_t* mask, int64_t n, int32_t* out_idx,
                                  int64_t* d_count, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || n > kMaxIndex) return fail(ABM_E_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && (!mask || !out_idx)) return fail(ABM_E_INVALID, "mask or out_idx is NULL");
    if (!d_count) return fail(ABM_E_INVALID, "d_count is NULL");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_ws(ws, ws_bytes, n);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, n);
    hipStream_t st = as_stream(stream);
    if (n == 0) {
        // the count of an empty mask is zero: written as "dropped" of a no-op
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, nullptr, 0, nullptr, d_count);
        return launch_status("select_indices");
    }
    return launch_compact(mask, n, out_idx, d_count, w, st);
}
