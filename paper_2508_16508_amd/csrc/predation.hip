// predation.hip -- abm_predation_init / abm_predation_step: the wolf-sheep-
// grass model of Sec. 5.1 (Fig. 2) on one GPU, one model per launch sequence.
//
// Step t is four launches (each arrow is a grid-wide dependency):
//   K1 move+claim   every live agent moves, pays 1 energy and posts its
//                   packed (draw << 32 | slot) key with a 64-bit atomicMin into
//                   the claim tables of its cell: grass (sheep on grown
//                   cells), prey (sheep) and eater (wolves).
//   K2 eat+breeders each live agent compares its keys with the reduced table
//                   entries (grass winner, eaten sheep, eating wolf), applies
//                   the energy gain / death, then decides whether it breeds;
//                   breeders are compacted into an ascending list with the
//                   single-pass scan (one scan chain per species).
//   K3 breed+die    free slots (alive == 0) are ranked by the same scan; the
//                   free slot of rank j < #breeders PULLS its child from
//                   breeder j (cell, half the energy) and the parent keeps the
//                   rest; live agents with negative energy die.
//   K4 regrow       every countdown above zero drops by one and the claim
//                   tables are re-armed for the next step.
// With multi_prey, K1 instead pushes every live sheep and wolf onto a list of
// its cell (64-bit atomicExch on the prey / eater words, which then hold list
// heads), and K1b, between K1 and K2, pairs the r-th wolf of each cell (eat
// key order) with the r-th sheep (prey key order): the wolf gains, the sheep
// is marked alive = 2 (eaten, still to take part in the grass rule of K2).
// Pulling into the free slot (rather than the parent pushing into some later
// tile) keeps every slot written by the thread that ranked it.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "rng.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kItems = 16;
constexpr int64_t kTile = int64_t(kWaves) * 64 * kItems;
constexpr int kBlock = 256;
constexpr uint64_t kNoClaim = ~0ull;

// Offsets of the eight neighbours, indexed by dir = draw >> 29, packed as
// (offset + 1) in two bits per direction:
//   dir: 0 (-1,-1) 1 (0,-1) 2 (1,-1) 3 (-1,0) 4 (1,0) 5 (-1,1) 6 (0,1) 7 (1,1)
constexpr uint32_t kDxPacked = 0x9224u;
constexpr uint32_t kDyPacked = 0xA940u;

enum StatCol : int {
    kLiveS = 0, kLiveW, kGrassEaten, kSheepEaten, kBirthsS, kBirthsW, kStarvedS, kStarvedW
};

struct Species {
    int32_t* x;
    int32_t* y;
    int32_t* e;
    int32_t* alive;
};

struct StepArgs {
    int32_t W, H, R, gain_s, gain_w;
    uint32_t T_s, T_w, seed;
    int64_t cap_s, cap_w;
    int32_t* grass;
    Species sp[2];        // 0 sheep, 1 wolves
    uint64_t* gclaim;     // grass: lowest sheep key per grown cell
    uint64_t* sclaim;     // prey: lowest sheep key per cell
    uint64_t* wclaim;     // eater: lowest wolf key per cell
    int64_t* stats;       // this step's row of 8, or null
    int64_t* acc;         // kAccCounters x kAccLanes spread accumulators
    uint32_t step;
    uint64_t* status;
    EpochArg epoch;
    int32_t* blist[2];    // breeder lists
    int64_t* d_nb[2];     // breeder counts
    uint32_t tiles[2];
    uint32_t chain_off[2];  // start of each species' scan chain in the status words
    int32_t multi;          // prey by rank within a cell (K1 builds lists, K1b matches)
};

__device__ __forceinline__ int32_t wrap_step(int32_t v, int32_t d, int32_t n) {
    v += d;
    return v < 0 ? n - 1 : (v >= n ? 0 : v);
}

// Cell of a position, or -1 when it lies off the lattice (a live agent is
// always on it in a state produced by this library; the test keeps a bad
// caller-supplied state from indexing outside the grid).
__device__ __forceinline__ int64_t cell_of(int32_t x, int32_t y, int32_t W, int32_t H) {
    return (x >= 0 && x < W && y >= 0 && y < H) ? int64_t(y) * W + x : -1;
}

__device__ __forceinline__ uint64_t agent_key(uint64_t skey, int64_t slot, uint32_t purpose) {
    return (uint64_t(draw(skey, uint32_t(slot), purpose)) << 32) | uint32_t(slot);
}

// Block-wide sum of one value per thread, added by thread 0 to this block's
// lane of the spread accumulator of counter `col` (256 lanes per counter, so
// no single address takes every block's atomic).
__device__ __forceinline__ void block_add(uint32_t v, int64_t* acc, int col, uint32_t* lds) {
    int64_t* dst = acc + int64_t(col) * kAccLanes + (blockIdx.x & (kAccLanes - 1));
    const uint32_t w = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < int(blockDim.x >> 6); ++i) s += lds[i];
        if (s) atomicAdd(reinterpret_cast<unsigned long long*>(dst), (unsigned long long)s);
    }
}

// ------------------------------------------------------------------ init
struct InitArgs {
    int32_t W, H, R, gain_s, gain_w;
    uint32_t seed;
    int64_t cap_s, cap_w, n_s0, n_w0, G;
    int32_t* grass;
    Species sp[2];
    uint64_t* claims;  // 3 * G
};

__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const uint64_t key = stream_key(a.seed, kInitStep);
    if (i < a.G) {
        const uint32_t h = draw(key, uint32_t(i), kGrassGrown);
        a.grass[i] = h < 0x80000000u
                         ? 0
                         : 1 + int32_t(scale(draw(key, uint32_t(i), kGrassCountdown), uint32_t(a.R)));
        a.claims[i] = kNoClaim;
        a.claims[a.G + i] = kNoClaim;
        a.claims[2 * a.G + i] = kNoClaim;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int64_t cap = s ? a.cap_w : a.cap_s;
        const int64_t n0 = s ? a.n_w0 : a.n_s0;
        const int32_t gain = s ? a.gain_w : a.gain_s;
        const uint32_t px = s ? kWolfX : kSheepX;
        if (i < cap) {
            int32_t x = 0, y = 0, e = 0, al = 0;
            if (i < n0) {
                x = int32_t(scale(draw(key, uint32_t(i), px), uint32_t(a.W)));
                y = int32_t(scale(draw(key, uint32_t(i), px + 1), uint32_t(a.H)));
                e = int32_t(scale(draw(key, uint32_t(i), px + 2), uint32_t(2 * gain)));
                al = 1;
            }
            a.sp[s].x[i] = x;
            a.sp[s].y[i] = y;
            a.sp[s].e[i] = e;
            a.sp[s].alive[i] = al;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fill64(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ K1
__global__ __launch_bounds__(kBlock) void k_move_claim(StepArgs a) {
    __shared__ uint32_t lds[kBlock / 64];
    const int64_t g = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int s = g < a.cap_s ? 0 : 1;
    const int64_t i = s ? g - a.cap_s : g;
    const int64_t cap = s ? a.cap_w : a.cap_s;
    const uint64_t skey = stream_key(a.seed, a.step);
    uint32_t live_s = 0, live_w = 0;
    if (i < cap && a.sp[s].alive[i] != 0) {
        (s ? live_w : live_s) = 1;
        const uint32_t d = draw(skey, uint32_t(i), s ? kWolfMove : kSheepMove) >> 29;
        const int32_t dx = int32_t((kDxPacked >> (2 * d)) & 3u) - 1;
        const int32_t dy = int32_t((kDyPacked >> (2 * d)) & 3u) - 1;
        const int32_t x = wrap_step(a.sp[s].x[i], dx, a.W);
        const int32_t y = wrap_step(a.sp[s].y[i], dy, a.H);
        a.sp[s].x[i] = x;
        a.sp[s].y[i] = y;
        a.sp[s].e[i] -= 1;
        const int64_t c = cell_of(x, y, a.W, a.H);
        if (c < 0) {
        } else if (a.multi) {
            // push slot i onto the list of its cell; the list ends at all-ones
            if (s == 0 && a.grass[c] == 0)
                atomicMin(reinterpret_cast<unsigned long long*>(a.gclaim + c),
                          (unsigned long long)agent_key(skey, i, kSheepGrassKey));
            uint64_t* head = (s ? a.wclaim : a.sclaim) + c;
            const uint64_t prev = atomicExch(reinterpret_cast<unsigned long long*>(head),
                                             (unsigned long long)i);
            a.blist[s][i] = int32_t(prev);   // all-ones -> -1
        } else if (s == 0) {
            if (a.grass[c] == 0)
                atomicMin(reinterpret_cast<unsigned long long*>(a.gclaim + c),
                          (unsigned long long)agent_key(skey, i, kSheepGrassKey));
            atomicMin(reinterpret_cast<unsigned long long*>(a.sclaim + c),
                      (unsigned long long)agent_key(skey, i, kSheepPreyKey));
        } else {
            atomicMin(reinterpret_cast<unsigned long long*>(a.wclaim + c),
                      (unsigned long long)agent_key(skey, i, kWolfEatKey));
        }
    }
    if (a.stats) {
        block_add(live_s, a.acc, kLiveS, lds);
        block_add(live_w, a.acc, kLiveW, lds);
    }
}

// K1b (multi_prey): wolf j of cell c takes rank r among the wolves of c (eat
// keys) and eats the sheep of rank r among the sheep of c (prey keys), if the
// cell has that many.  Ranks are counted over the cell's lists; the lists of a
// cell are short at the workloads' densities (a few agents), and the count is
// quadratic in the sheep of one cell at worst.  Distinct wolves of a cell
// have distinct ranks, so no sheep is taken twice.
__global__ __launch_bounds__(kBlock) void k_prey_match(StepArgs a) {
    const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (j >= a.cap_w || a.sp[1].alive[j] == 0) return;
    const int64_t c = cell_of(a.sp[1].x[j], a.sp[1].y[j], a.W, a.H);
    if (c < 0) return;
    const uint64_t skey = stream_key(a.seed, a.step);
    const uint64_t my_key = agent_key(skey, j, kWolfEatKey);
    uint32_t r = 0;
    for (int32_t w = int32_t(a.wclaim[c]); w >= 0; w = a.blist[1][w])
        r += agent_key(skey, w, kWolfEatKey) < my_key;
    const int32_t first = int32_t(a.sclaim[c]);
    for (int32_t q = first; q >= 0; q = a.blist[0][q]) {
        const uint64_t kq = agent_key(skey, q, kSheepPreyKey);
        uint32_t below = 0;
        for (int32_t u = first; u >= 0; u = a.blist[0][u])
            below += agent_key(skey, u, kSheepPreyKey) < kq;
        if (below == r) {
            a.sp[0].alive[q] = 2;
            a.sp[1].e[j] += a.gain_w;
            return;
        }
    }
}

// Maps workgroup t to (species, first tile of that species' scan chain).
__device__ __forceinline__ void species_tile(const StepArgs& a, uint32_t& tile, int& s,
                                             uint32_t& seg_first) {
    tile = blockIdx.x;
    s = tile < a.tiles[0] ? 0 : 1;
    seg_first = s ? a.tiles[0] : 0u;
}

// ------------------------------------------------------------------ K2
__global__ __launch_bounds__(kWaves * 64) void k_eat_breeders(StepArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    uint32_t tile, seg_first;
    int s;
    species_tile(a, tile, s, seg_first);
    const uint32_t epoch = read_epoch(a.epoch);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cap = s ? a.cap_w : a.cap_s;
    const int64_t base = int64_t(tile - seg_first) * kTile + int64_t(wave) * kItems * 64 + lane;
    const uint64_t skey = stream_key(a.seed, a.step);
    const Species sp = a.sp[s];
    uint32_t grass_eaten = 0, sheep_eaten = 0;
    bool f[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k * 64;
        f[k] = false;
        if (i >= cap || sp.alive[i] == 0) continue;
        const int64_t c = cell_of(sp.x[i], sp.y[i], a.W, a.H);
        int32_t e = sp.e[i];
        if (c < 0) {
            f[k] = e > 0 && draw(skey, uint32_t(i), s ? kWolfBreed : kSheepBreed) < (s ? a.T_w : a.T_s);
            continue;
        }
        if (s == 0) {
            if (a.gclaim[c] == agent_key(skey, i, kSheepGrassKey)) {
                e += a.gain_s;
                sp.e[i] = e;
                a.grass[c] = a.R;
                ++grass_eaten;
            }
            const bool eaten =
                a.multi ? sp.alive[i] == 2
                        : (a.wclaim[c] != kNoClaim &&
                           a.sclaim[c] == agent_key(skey, i, kSheepPreyKey));
            if (eaten) {
                sp.alive[i] = 0;
                ++sheep_eaten;
                continue;
            }
            f[k] = e > 0 && draw(skey, uint32_t(i), kSheepBreed) < a.T_s;
        } else {
            // (multi_prey: K1b has already added the gain)
            if (!a.multi && a.sclaim[c] != kNoClaim &&
                a.wclaim[c] == agent_key(skey, i, kWolfEatKey)) {
                e += a.gain_w;
                sp.e[i] = e;
            }
            f[k] = e > 0 && draw(skey, uint32_t(i), kWolfBreed) < a.T_w;
        }
    }
    uint32_t rank[kItems], total;
    const uint32_t tile_excl =
        rank_tile<kWaves, kItems>(f, rank, a.status + a.chain_off[s], a.status - 1,
                                  tile - seg_first, a.tiles[s], epoch, lds, &total);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (f[k]) a.blist[s][rank[k]] = int32_t(base + k * 64);
    const uint32_t last = seg_first + a.tiles[s] - 1;
    if (tile == last && threadIdx.x == 0) *a.d_nb[s] = int64_t(tile_excl) + total;
    if (a.stats && s == 0) {
        block_add(grass_eaten, a.acc, kGrassEaten, lds);
        block_add(sheep_eaten, a.acc, kSheepEaten, lds);
    }
}

// ------------------------------------------------------------------ K3
__global__ __launch_bounds__(kWaves * 64) void k_breed_die(StepArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    uint32_t tile, seg_first;
    int s;
    species_tile(a, tile, s, seg_first);
    const uint32_t epoch = read_epoch(a.epoch);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cap = s ? a.cap_w : a.cap_s;
    const int64_t base = int64_t(tile - seg_first) * kTile + int64_t(wave) * kItems * 64 + lane;
    const Species sp = a.sp[s];
    bool f[kItems], live[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k * 64;
        const bool in = i < cap;
        const int32_t al = in ? sp.alive[i] : 1;
        f[k] = in && al == 0;
        live[k] = in && al != 0;
    }
    uint32_t rank[kItems], total;
    const uint32_t tile_excl =
        rank_tile<kWaves, kItems>(f, rank, a.status + a.chain_off[s], a.status - 1,
                                  tile - seg_first, a.tiles[s], epoch, lds, &total);
    const int64_t nb = *a.d_nb[s];
    uint32_t starved = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k * 64;
        if (f[k] && int64_t(rank[k]) < nb) {
            const int32_t p = a.blist[s][rank[k]];
            const int32_t ep = sp.e[p];
            const int32_t ec = ep >> 1;
            sp.x[i] = sp.x[p];
            sp.y[i] = sp.y[p];
            sp.e[i] = ec;
            sp.e[p] = ep - ec;
            sp.alive[i] = 1;
        } else if (live[k] && sp.e[i] < 0) {
            // a breeder's energy stays positive, so no slot read by a child dies here
            sp.alive[i] = 0;
            ++starved;
        }
    }
    const uint32_t last = seg_first + a.tiles[s] - 1;
    if (a.stats) {
        if (tile == last && threadIdx.x == 0) {
            const int64_t nfree = int64_t(tile_excl) + total;
            a.stats[s ? kBirthsW : kBirthsS] = nfree < nb ? nfree : nb;
        }
        block_add(starved, a.acc, s ? kStarvedW : kStarvedS, lds);
    }
}

// ------------------------------------------------------------------ K4
// Workgroup 0 also folds the step's spread accumulators into its stats row
// and clears them for the next step (the births columns are written directly
// by the breed kernel).
__global__ __launch_bounds__(kBlock) void k_regrow_rearm(int32_t* __restrict__ grass,
                                                         uint64_t* __restrict__ claims, int64_t G,
                                                         int do_regrow, int64_t* acc,
                                                         int64_t* stats) {
    const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (stats && blockIdx.x == 0) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int col = wave; col < kAccCounters; col += kBlock / 64) {
            int64_t v = 0;
            for (int l = lane; l < kAccLanes; l += 64) {
                v += acc[col * kAccLanes + l];
                acc[col * kAccLanes + l] = 0;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && col != kBirthsS && col != kBirthsW) stats[col] = v;
        }
    }
    if (c >= G) return;
    if (do_regrow) {
        const int32_t g = grass[c];
        if (g > 0) grass[c] = g - 1;
    }
    claims[c] = kNoClaim;
    claims[G + c] = kNoClaim;
    claims[2 * G + c] = kNoClaim;
}

int check_params(const abm_predation_params* p) {
    if (!p) return fail(ABM_E_INVALID, "params are NULL");
    if (p->W < 1 || p->H < 1 || int64_t(p->W) * p->H > kMaxIndex)
        return fail(ABM_E_INVALID, "grid must satisfy W, H >= 1 and W*H < 2^31");
    if (p->R < 1) return fail(ABM_E_INVALID, "R must be >= 1");
    if (p->gain_s < 0 || p->gain_w < 0 || p->gain_s > (1 << 29) || p->gain_w > (1 << 29))
        return fail(ABM_E_INVALID, "gains must be in [0, 2^29]");
    if (p->cap_s < 1 || p->cap_w < 1 || p->cap_s > kMaxIndex || p->cap_w > kMaxIndex)
        return fail(ABM_E_INVALID, "capacities must be in [1, 2^31)");
    if (p->cap_s + p->cap_w > kMaxIndex)
        return fail(ABM_E_INVALID, "cap_s + cap_w must be below 2^31");
    if (p->n_s0 < 0 || p->n_w0 < 0 || p->n_s0 > p->cap_s || p->n_w0 > p->cap_w)
        return fail(ABM_E_INVALID, "initial counts must be in [0, capacity]");
    if (p->multi_prey != 0 && p->multi_prey != 1)
        return fail(ABM_E_INVALID, "multi_prey must be 0 or 1");
    return ABM_OK;
}

int check_state(const abm_predation_state* s) {
    if (!s) return fail(ABM_E_INVALID, "state is NULL");
    if (!s->grass || !s->claims) return fail(ABM_E_INVALID, "grass or claims is NULL");
    const abm_species* sp[2] = {&s->sheep, &s->wolves};
    for (int k = 0; k < 2; ++k)
        if (!sp[k]->x || !sp[k]->y || !sp[k]->e || !sp[k]->alive)
            return fail(ABM_E_INVALID, "species array is NULL");
    return ABM_OK;
}

Species species_of(const abm_species& s) { return Species{s.x, s.y, s.e, s.alive}; }

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_predation_init(const abm_predation_params* p, abm_predation_state* s,
                                  void* stream) {
    int rc = check_params(p);
    if (rc != ABM_OK) return rc;
    rc = check_state(s);
    if (rc != ABM_OK) return rc;
    rc = check_device();
    if (rc != ABM_OK) return rc;
    InitArgs a;
    a.W = p->W;
    a.H = p->H;
    a.R = p->R;
    a.gain_s = p->gain_s;
    a.gain_w = p->gain_w;
    a.seed = p->seed;
    a.cap_s = p->cap_s;
    a.cap_w = p->cap_w;
    a.n_s0 = p->n_s0;
    a.n_w0 = p->n_w0;
    a.G = int64_t(p->W) * p->H;
    a.grass = s->grass;
    a.sp[0] = species_of(s->sheep);
    a.sp[1] = species_of(s->wolves);
    a.claims = s->claims;
    int64_t m = a.G;
    if (a.cap_s > m) m = a.cap_s;
    if (a.cap_w > m) m = a.cap_w;
    hipLaunchKernelGGL(k_init, dim3(tiles_for(m, kBlock)), dim3(kBlock), 0, as_stream(stream), a);
    rc = launch_status("predation_init");
    if (rc == ABM_OK) s->step = 0;
    return rc;
}

extern "C" int abm_predation_step(const abm_predation_params* p, abm_predation_state* s,
                                  int32_t n_steps, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc != ABM_OK) return rc;
    rc = check_state(s);
    if (rc != ABM_OK) return rc;
    if (n_steps < 0) return fail(ABM_E_INVALID, "n_steps must be >= 0");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const int64_t cap = p->cap_s > p->cap_w ? p->cap_s : p->cap_w;
    rc = check_ws(ws, ws_bytes, cap);
    if (rc != ABM_OK) return rc;
    if (n_steps == 0) return ABM_OK;
    Workspace w = carve(ws, cap);
    hipStream_t st = as_stream(stream);
    const int64_t G = int64_t(p->W) * p->H;

    StepArgs a;
    a.W = p->W;
    a.H = p->H;
    a.R = p->R;
    a.gain_s = p->gain_s;
    a.gain_w = p->gain_w;
    a.T_s = p->T_s;
    a.T_w = p->T_w;
    a.seed = p->seed;
    a.cap_s = p->cap_s;
    a.cap_w = p->cap_w;
    a.grass = s->grass;
    a.sp[0] = species_of(s->sheep);
    a.sp[1] = species_of(s->wolves);
    a.gclaim = s->claims;
    a.sclaim = s->claims + G;
    a.wclaim = s->claims + 2 * G;
    a.status = w.status;
    a.acc = w.acc;
    a.blist[0] = w.list_a;
    a.blist[1] = w.list_b;
    a.d_nb[0] = reinterpret_cast<int64_t*>(w.hdr + kHdrCountA);
    a.d_nb[1] = reinterpret_cast<int64_t*>(w.hdr + kHdrCountB);
    a.tiles[0] = static_cast<uint32_t>(tiles_for(p->cap_s, kTile));
    a.tiles[1] = static_cast<uint32_t>(tiles_for(p->cap_w, kTile));
    a.chain_off[0] = 0;
    a.chain_off[1] = static_cast<uint32_t>(chain_words(a.tiles[0]));
    a.multi = p->multi_prey;

    const dim3 cell_grid(static_cast<uint32_t>(tiles_for(G, kBlock)));
    const dim3 agent_grid(static_cast<uint32_t>(tiles_for(p->cap_s + p->cap_w, kBlock)));
    const dim3 scan_grid(a.tiles[0] + a.tiles[1]);
    // the claim tables and accumulators start the call empty whatever the
    // caller did between calls
    hipLaunchKernelGGL(k_regrow_rearm, cell_grid, dim3(kBlock), 0, st, s->grass, s->claims, G, 0,
                       nullptr, nullptr);
    hipLaunchKernelGGL(k_fill64, dim3(tiles_for(kAccWords, kBlock)), dim3(kBlock), 0, st, w.acc,
                       kAccWords, int64_t(0));
    if (s->stats)
        hipLaunchKernelGGL(k_fill64, dim3(tiles_for(8 * int64_t(n_steps), kBlock)), dim3(kBlock),
                           0, st, s->stats, 8 * int64_t(n_steps), int64_t(0));
    for (int32_t k = 0; k < n_steps; ++k) {
        a.step = s->step + uint32_t(k);
        a.stats = s->stats ? s->stats + 8 * int64_t(k) : nullptr;
        hipLaunchKernelGGL(k_move_claim, agent_grid, dim3(kBlock), 0, st, a);
        if (a.multi)
            hipLaunchKernelGGL(k_prey_match, dim3(static_cast<uint32_t>(tiles_for(p->cap_w, kBlock))),
                               dim3(kBlock), 0, st, a);
        rc = next_epoch(w, st, &a.epoch);
        if (rc != ABM_OK) return rc;
        hipLaunchKernelGGL(k_eat_breeders, scan_grid, dim3(kWaves * 64), 0, st, a);
        rc = next_epoch(w, st, &a.epoch);
        if (rc != ABM_OK) return rc;
        hipLaunchKernelGGL(k_breed_die, scan_grid, dim3(kWaves * 64), 0, st, a);
        hipLaunchKernelGGL(k_regrow_rearm, cell_grid, dim3(kBlock), 0, st, s->grass, s->claims, G,
                           1, w.acc, a.stats);
    }
    rc = launch_status("predation_step");
    if (rc == ABM_OK) s->step += uint32_t(n_steps);
    return rc;
}
