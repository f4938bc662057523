// predation.hip -- abm_predation_init / abm_predation_step: the wolf-sheep-
// grass model of Sec. 5.1 (Fig. 2) on one GPU, one model per launch sequence.
//
// Inside a call the state is kept in two working forms (converted at the call's
// start and back at its end): grass holds the step at which a cell is grown
// again (grown at step t iff ready <= t), so no per-step regrow pass is needed,
// and a bitmask in the workspace marks the live slots, so the per-step kernels
// read 1 bit per slot instead of the 4-byte alive word and visit only live
// agents.  Each kernel works on tiles of 8192 slots (1024 threads, thread t <
// 256 owning the 32 slots of bitmask word t); a tile first compacts its live
// slots into a list in LDS and then spreads that list over all its threads,
// one agent per thread per batch, so dense and sparse tiles alike keep every
// lane busy.  Step t is three launches (each arrow a grid-wide dependency):
//   K1 move+claim   every live agent moves, pays 1 energy and posts its
//                   packed (step tag, draw, slot) key with a 64-bit atomicMin
//                   into the claim tables of its cell: grass (sheep on grown
//                   cells), prey (sheep) and eater (wolves).
//   K2 eat+breeders each live agent compares its keys with the reduced table
//                   entries (grass winner, eaten sheep, eating wolf), applies
//                   the energy gain and marks an eaten sheep alive = 2, then
//                   decides whether it breeds; the tile's breeders and its
//                   slots free for births (empty, or eaten this step) are
//                   ranked by the single-pass scan on two chains at once, the
//                   breeders compacted into an ascending list and the tile's
//                   free-slot prefix kept for K3.
//   K3 breed+die    the free slot of rank j < #breeders PULLS its child from
//                   breeder j (cell, half the energy) while the parent keeps
//                   the rest; live agents with negative energy die; at the end
//                   of a tag period the claim tables are re-armed (each
//                   workgroup streams its slice; within a period the falling
//                   tags make older words lose, see claim_key).
// Tiles past the last tile holding a live agent (the tile mark K3 leaves for
// the next step) skip their work: they hold no agent, K2's scans stop below
// them, and K3 computes their free-slot prefixes from the totals.
// With multi_prey, K1 instead pushes every live sheep and wolf onto a list of
// its cell (64-bit atomicExch on the prey / eater words, which then hold list
// heads), and K1b, between K1 and K2, pairs the r-th wolf of each cell (eat
// key order) with the r-th sheep (prey key order): the wolf gains, the sheep
// is marked alive = 2 (eaten, still to take part in the grass rule of K2).
// Pulling into the free slot (rather than the parent pushing into some later
// tile) keeps every slot written by one thread.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "rng.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 256;
constexpr int64_t kTile = int64_t(kBlock) * 32;   // 8192 slots: one bitmask word per thread
constexpr uint32_t kTagBits = 4;                  // claim-key tag: periods of 14 steps
// List entries per thread and batch.  With 1024 threads a tile, one each
// measured 102 us per 2048^2 step against 104 with two and 106 with four:
// the waves hide the latency of the random cell accesses better than a
// thread's own batch does.
#ifndef ABM_PRED_IN_FLIGHT
#define ABM_PRED_IN_FLIGHT 1
#endif
constexpr int kInFlight = ABM_PRED_IN_FLIGHT;
// Threads per tile: kBlock own the tile's bitmask words, and kHelpers times
// as many share the tile's list of agents.  Live agents crowd the low tiles
// (children take the lowest free slots), so a few hundred tiles hold all the
// work.  At 2048^2, twice the threads on each took 9% off the step and four
// times (1024-thread blocks, the most a block holds) a further 8%: the tiles
// past the last live one exit at once, so the larger blocks cost no extra
// dispatch rounds.
constexpr int kHelpers = 4;
// header words of the free-slot totals (words 4 and 5 are unused by the
// common layout)
constexpr int kHdrFreeA = 4, kHdrFreeB = 5;
// words 6-9: the tile marks of even and odd steps (two species each)
constexpr int kHdrMark = 6;
static_assert(kHdrFreeA > kHdrCountB && kHdrMark + 3 < kHdrError, "header word clash");
static_assert(kWaves * kHelpers >= 2 * kLevels, "the dual-chain prefix needs 2 kLevels waves");
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
    int32_t* ready;       // grass: step at which each cell is grown again
    Species sp[2];        // 0 sheep, 1 wolves
    uint32_t* bits[2];    // live-slot bitmasks
    int64_t G;            // cells
    uint64_t* claims;     // three words per cell c, at 3 c: grass (the lowest key
                          // of a sheep on the grown cell), prey (lowest sheep
                          // key), eater (lowest wolf key); together in one line
    uint32_t sb;          // slot bits of a claim key (see claim_key)
    uint64_t tag_hi;      // this step's tag, in place
    uint64_t tag_mask;    // the tag field
    int32_t rearm;        // K3 re-arms the whole table (the tag period ends)
    int64_t* stats;       // this step's row of 8, or null
    int64_t* acc;         // kAccCounters x kAccLanes spread accumulators: per counter, lanes
                          // [0, 128) for even steps of a call and [128, 256) for odd ones
    int32_t acc_par;      // this step's half (0 or 128)
    int64_t* fold_row;    // stats row of the previous step, folded by K1 (or null)
    uint32_t step;
    uint64_t* status;
    EpochArg epoch;
    int32_t* blist[2];    // breeder lists
    int64_t* d_nb[2];     // breeder counts
    int64_t* d_nf[2];     // free-slot counts (this step's births are min(nf, nb))
    int32_t* free_pre[2]; // per tile: exclusive free-slot prefix, written by K2 for K3
    uint32_t tiles[2];
    uint32_t chain_off[2];  // start of each species' breeder scan chain in the status words
    uint32_t fchain_off[2]; // ... and of its free-slot scan chain
    int32_t multi;          // prey by rank within a cell (K1 builds lists, K1b matches)
    uint64_t* mark_rd;      // [2] per species: no live agent in this tile or past it
    uint64_t* mark_wr;      // [2] the same for the next step, raised by K3 (cleared by K1)
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

// A claim word holds (tag, draw, slot) from the high bits down: slot in the
// low sb bits, the 32-bit draw above it and the step's tag on top.  Within a
// step, keys order as (draw, slot), the order of the method's claims.  Tags
// fall from step to step, so a word left by an earlier step of the same
// period (a larger tag) loses to every fresh claim and reads as unclaimed,
// and the table need not be re-armed between the steps of a period; all-ones
// (the re-armed word) carries a tag no step uses.
__device__ __forceinline__ uint64_t claim_key(const StepArgs& a, uint64_t skey, int64_t slot,
                                              uint32_t purpose) {
    return a.tag_hi | (uint64_t(draw(skey, uint32_t(slot), purpose)) << a.sb) | uint64_t(slot);
}

__device__ __forceinline__ bool claimed(const StepArgs& a, uint64_t word) {
    return (word & a.tag_mask) == a.tag_hi;
}

// Slot at the head of a multi-prey list word, or -1 (no push this step).
__device__ __forceinline__ int32_t head_slot(const StepArgs& a, uint64_t word) {
    return claimed(a, word) ? int32_t(word & ~a.tag_mask) : -1;
}

// Block-wide sum of one value per thread, added by thread 0 to this block's
// lane of the spread accumulator of counter `col` in the step's half (128
// lanes per counter and step, so no single address takes every block's
// atomic).  `acc` points at the step's half.
constexpr int kHalfLanes = kAccLanes / 2;
__device__ __forceinline__ void block_add(uint32_t v, int64_t* acc, int col, uint32_t* lds) {
    int64_t* dst = acc + int64_t(col) * kAccLanes + (blockIdx.x & (kHalfLanes - 1));
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

// Folds one step's half of the spread accumulators (`acc` points at it)
// into its stats row (the births columns are written by K3) and clears it for
// the step after next.  Any number of whole waves.
__device__ __forceinline__ void fold_stats(int64_t* acc, int64_t* stats) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int col = wave; col < kAccCounters; col += int(blockDim.x >> 6)) {
        int64_t v = 0;
        for (int l = lane; l < kHalfLanes; l += 64) {
            v += acc[col * kAccLanes + l];
            acc[col * kAccLanes + l] = 0;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0 && col != kBirthsS && col != kBirthsW) stats[col] = v;
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

// ------------------------------------------------------------------ tiles
// Tile t of a species covers slots [8192 t, 8192 t + 8192) and bitmask words
// [256 t, 256 t + 256), thread k owning word 256 t + k (slots 32 k .. 32 k + 31
// of the tile).  Bits of slots at or beyond the capacity are always zero.
// Workgroups take the tiles of both species interleaved -- sheep 0, wolves 0,
// sheep 1, wolves 1, ... until the shorter chain ends, then the rest of the
// longer one -- so that the low tiles, where children fill the lowest free
// slots and the live agents gather, are all in the first round of resident
// workgroups; within each chain tiles still run in increasing order.
struct TileRef {
    int s;            // species
    uint32_t tile;    // tile within the species' scan chain
    int64_t base;     // first slot
};

__device__ __forceinline__ TileRef tile_of(const StepArgs& a) {
    const uint32_t m = a.tiles[0] < a.tiles[1] ? a.tiles[0] : a.tiles[1];
    const uint32_t b = blockIdx.x;
    TileRef r;
    if (b < 2 * m) {
        r.s = int(b & 1u);
        r.tile = b >> 1;
    } else {
        r.s = a.tiles[0] > a.tiles[1] ? 0 : 1;
        r.tile = m + (b - 2 * m);
    }
    r.base = int64_t(r.tile) * kTile;
    return r;
}

// Block-wide list, in slot order, of the tile offsets of the set bits of each
// thread's mask (thread t owns offsets 32 t .. 32 t + 31).  Returns the list
// length (the same in every thread); *first receives the list index of this
// thread's first set bit.  Contains three block barriers; the list is
// complete when it returns.
template <int WAVES = kWaves>
__device__ __forceinline__ uint32_t block_list(uint32_t mask, uint16_t* list, uint32_t* wl,
                                               uint32_t* first) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t c = __popc(mask);
    uint32_t excl = 0, wtot = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        excl += lane_rank(bal) << b;
        wtot += static_cast<uint32_t>(__popcll(bal)) << b;
    }
    __syncthreads();   // earlier readers of wl and list are done
    if (lane == 0) wl[wave] = wtot;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t v = wl[w];
        before += w < wave ? v : 0u;
        total += v;
    }
    uint32_t r = before + excl;
    *first = r;
    for (uint32_t m = mask; m; m &= m - 1u) list[r++] = uint16_t(threadIdx.x * 32u + (__ffs(m) - 1));
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(total);
}

// A list entry is a 13-bit tile offset; a kernel may tag it with a 2-bit
// flag in bits 14-15 once it has read the offset.
__device__ __forceinline__ void tag(uint16_t* list, uint32_t j, uint32_t f) {
    list[j] = uint16_t((list[j] & 0x1FFFu) | (f << 14));
}

// The bits of `mask` whose list entries (in slot order from `first`) carry
// flag value v.
__device__ __forceinline__ uint32_t flagged(uint32_t mask, uint32_t first, const uint16_t* list,
                                            uint32_t v) {
    uint32_t out = 0, r = first;
    for (uint32_t m = mask; m; m &= m - 1u, ++r)
        if ((list[r] >> 14) == v) out |= m & (0u - m);
    return out;
}

__device__ __forceinline__ bool grown(int32_t ready, uint32_t step) {
    return int32_t(uint32_t(ready) - step) <= 0;
}

// Tile-local part of a rank: this thread's exclusive rank of its count c
// (0 <= c < 64) in thread order, and the tile total.  lds holds one word per
// wave.  Two block barriers.
template <int WAVES>
__device__ __forceinline__ uint32_t rank_block(uint32_t c, uint32_t* thread_excl, uint32_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t excl = 0, wtot = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        excl += lane_rank(bal) << b;
        wtot += static_cast<uint32_t>(__popcll(bal)) << b;
    }
    __syncthreads();
    if (lane == 0) lds[wave] = wtot;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t v = lds[w];
        before += w < wave ? v : 0u;
        total += v;
    }
    *thread_excl = before + excl;
    return total;
}

// Exclusive prefixes of two counts of this tile over two chains at once (the
// hierarchical look-back of the single-pass scan, one chain per group of
// kLevels waves: waves 0-3 walk chain A with count a, waves 4-7 chain B with
// count b).  Needs 2 kLevels waves; lds holds 2 kLevels words.  Two barriers.
__device__ __forceinline__ void hier_prefix2(uint64_t* chain_a, uint64_t* chain_b, uint64_t* err,
                                             uint32_t t, uint32_t T, uint32_t epoch, uint32_t a,
                                             uint32_t b, uint32_t* lds, uint32_t* pre_a,
                                             uint32_t* pre_b) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool second = wave >= kLevels;
    const int lv = second ? wave - kLevels : wave;
    const uint32_t count = second ? b : a;
    uint32_t part = 0;
    if (wave < 2 * kLevels) {
        uint64_t* level = second ? chain_b : chain_a;
        uint32_t n = T;
        for (int l = 0; l < lv; ++l) {
            level += n;
            n = (n + 63) >> 6;
        }
        const uint32_t g = t >> (6 * lv);
        const uint32_t d = g & 63u;
        const uint32_t pspan = 1u << (6 * (lv + 1));
        const bool publish = (((t & (pspan - 1)) == pspan - 1) || t == T - 1) && lv + 1 < kLevels;
        if (lv == 0 && lane == 0) st_agent(&level[g], pack_status(epoch, kFlagAgg, count));
        uint32_t v = 0;
        if (lane < d || (lane == d && lv > 0 && publish)) {
            const uint32_t idx = g - d + lane;
            v = static_cast<uint32_t>(poll_status(&level[idx], ld_agent(&level[idx]), epoch, err));
        }
        const uint32_t own = (lv == 0) ? count : 0u;
        part = wave_sum(lane < d ? v : 0u);
        if (publish) {
            const uint32_t incl = wave_sum(v) + own;
            if (lane == 0) st_agent(&(level + n)[g >> 6], pack_status(epoch, kFlagAgg, incl));
        }
    }
    __syncthreads();
    if (lane == 0 && wave < 2 * kLevels) lds[wave] = part;
    __syncthreads();
    uint32_t ta = 0, tb = 0;
#pragma unroll
    for (int l = 0; l < kLevels; ++l) {
        ta += lds[l];
        tb += lds[kLevels + l];
    }
    *pre_a = ta;
    *pre_b = tb;
}

// ------------------------------------------------------------------ K1
template <int H>
__global__ __launch_bounds__(kBlock * H) void k_move_claim(StepArgs a) {
    constexpr int kThreads = kBlock * H;
    __shared__ uint16_t list[kTile];
    __shared__ uint32_t wl[kWaves * H];
    __shared__ uint32_t lds[kWaves * H];
    const TileRef t = tile_of(a);
    const int s = t.s;
    const Species sp = a.sp[s];
    // the previous step's statistics, folded by the last workgroup (a tile
    // past the live agents, so it has time to spare); this step adds to the
    // other half of the accumulators
    if (a.fold_row && blockIdx.x == gridDim.x - 1)
        fold_stats(a.acc + (kHalfLanes - a.acc_par), a.fold_row);
    // the next step's tile marks start from zero (K3 raises them)
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x < 2) a.mark_wr[threadIdx.x] = 0;
    if (t.tile >= uint32_t(a.mark_rd[s])) return;   // past the last live tile
    const uint32_t mask =
        threadIdx.x < kBlock ? a.bits[s][int64_t(t.tile) * kBlock + threadIdx.x] : 0u;
    if (!__syncthreads_or(mask != 0u)) return;   // no live agent in the tile
    uint32_t first;
    const uint32_t n = block_list<kWaves * H>(mask, list, wl, &first);
    const uint64_t skey = stream_key(a.seed, a.step);
    for (uint32_t j0 = 0; j0 < n; j0 += kInFlight * kThreads) {
        int64_t i[kInFlight], c[kInFlight];
        int32_t x[kInFlight], y[kInFlight];
        bool on[kInFlight];
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            const uint32_t j = j0 + uint32_t(q * kThreads) + threadIdx.x;
            on[q] = j < n;
            i[q] = t.base + (on[q] ? list[j] : 0);
            if (on[q]) {
                x[q] = sp.x[i[q]];
                y[q] = sp.y[i[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q]) continue;
            const uint32_t d = draw(skey, uint32_t(i[q]), s ? kWolfMove : kSheepMove) >> 29;
            x[q] = wrap_step(x[q], int32_t((kDxPacked >> (2 * d)) & 3u) - 1, a.W);
            y[q] = wrap_step(y[q], int32_t((kDyPacked >> (2 * d)) & 3u) - 1, a.H);
            sp.x[i[q]] = x[q];
            sp.y[i[q]] = y[q];
            sp.e[i[q]] -= 1;
            c[q] = cell_of(x[q], y[q], a.W, a.H);
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q] || c[q] < 0) continue;
            if (a.multi) {
                // push slot i onto the list of its cell; the list ends at a word
                // of an earlier step (or all-ones)
                if (s == 0 && grown(a.ready[c[q]], a.step))
                    atomicMin(reinterpret_cast<unsigned long long*>(a.claims + 3 * c[q]),
                              (unsigned long long)claim_key(a, skey, i[q], kSheepGrassKey));
                uint64_t* head = a.claims + 3 * c[q] + (s ? 2 : 1);
                const uint64_t prev = atomicExch(reinterpret_cast<unsigned long long*>(head),
                                                 (unsigned long long)(a.tag_hi | uint64_t(i[q])));
                a.blist[s][i[q]] = head_slot(a, prev);
            } else if (s == 0) {
                if (grown(a.ready[c[q]], a.step))
                    atomicMin(reinterpret_cast<unsigned long long*>(a.claims + 3 * c[q]),
                              (unsigned long long)claim_key(a, skey, i[q], kSheepGrassKey));
                atomicMin(reinterpret_cast<unsigned long long*>(a.claims + 3 * c[q] + 1),
                          (unsigned long long)claim_key(a, skey, i[q], kSheepPreyKey));
            } else {
                atomicMin(reinterpret_cast<unsigned long long*>(a.claims + 3 * c[q] + 2),
                          (unsigned long long)claim_key(a, skey, i[q], kWolfEatKey));
            }
        }
    }
    if (a.stats) block_add(__popc(mask), a.acc + a.acc_par, s ? kLiveW : kLiveS, lds);
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
    for (int32_t w = head_slot(a, a.claims[3 * c + 2]); w >= 0; w = a.blist[1][w])
        r += agent_key(skey, w, kWolfEatKey) < my_key;
    const int32_t first = head_slot(a, a.claims[3 * c + 1]);
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

// ------------------------------------------------------------------ K2
// H x kBlock threads: threads below kBlock own the tile's bitmask words, all
// of them take part in the tile's list of agents (as in K1 and K3).
template <int H>
__global__ __launch_bounds__(kBlock * H) void k_eat_breeders(StepArgs a) {
    constexpr int kThreads = kBlock * H;
    __shared__ uint16_t list[kTile];
    __shared__ uint32_t wl[kWaves * H];
    __shared__ uint32_t lds[2 * kWaves * H + 1];
    const TileRef t = tile_of(a);
    const int s = t.s;
    const Species sp = a.sp[s];
    const uint32_t epoch = read_epoch(a.epoch);
    const int64_t cap = s ? a.cap_w : a.cap_s;
    // tiles at or past the mark hold no live agent: no breeder, every slot
    // free; they take no part in the scans (no tile below them reads their
    // words), and K3 derives their free-slot prefixes from the totals
    const uint32_t mark = uint32_t(a.mark_rd[s]);
    const uint32_t last = mark > 0 ? mark - 1 : 0;   // the tile that writes the totals
    const int64_t past = cap - int64_t(mark) * kTile > 0 ? cap - int64_t(mark) * kTile : 0;
    if (t.tile >= mark) {
        if (mark == 0 && t.tile == 0 && threadIdx.x == 0) {
            *a.d_nb[s] = 0;
            *a.d_nf[s] = cap;
        }
        return;
    }
    const uint32_t mask =
        threadIdx.x < kBlock ? a.bits[s][int64_t(t.tile) * kBlock + threadIdx.x] : 0u;
    // (a tile with no live agent skips the list: it still takes part in both scans)
    uint32_t first = 0, n = 0;
    if (__syncthreads_or(mask != 0u)) n = block_list<kWaves * H>(mask, list, wl, &first);
    const uint64_t skey = stream_key(a.seed, a.step);
    uint32_t grass_eaten = 0, sheep_eaten = 0;
    for (uint32_t j0 = 0; j0 < n; j0 += kInFlight * kThreads) {
        int64_t i[kInFlight], c[kInFlight];
        int32_t e[kInFlight];
        bool on[kInFlight], eaten[kInFlight];
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            const uint32_t j = j0 + uint32_t(q * kThreads) + threadIdx.x;
            on[q] = j < n;
            i[q] = t.base + (on[q] ? list[j] : 0);
            c[q] = on[q] ? cell_of(sp.x[i[q]], sp.y[i[q]], a.W, a.H) : -1;
            e[q] = on[q] ? sp.e[i[q]] : 0;
            eaten[q] = s == 0 && a.multi && on[q] && sp.alive[i[q]] == 2;
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q] || c[q] < 0) continue;
            if (s == 0) {
                if (a.claims[3 * c[q]] == claim_key(a, skey, i[q], kSheepGrassKey)) {
                    e[q] += a.gain_s;
                    sp.e[i[q]] = e[q];
                    a.ready[c[q]] = int32_t(a.step + uint32_t(a.R));
                    ++grass_eaten;
                }
                if (!a.multi)
                    eaten[q] = claimed(a, a.claims[3 * c[q] + 2]) &&
                               a.claims[3 * c[q] + 1] == claim_key(a, skey, i[q], kSheepPreyKey);
                if (eaten[q]) {
                    if (!a.multi) sp.alive[i[q]] = 2;
                    ++sheep_eaten;
                }
            } else if (!a.multi && claimed(a, a.claims[3 * c[q] + 1]) &&
                       a.claims[3 * c[q] + 2] == claim_key(a, skey, i[q], kWolfEatKey)) {
                // (multi_prey: K1b has already added the gain)
                e[q] += a.gain_w;
                sp.e[i[q]] = e[q];
            }
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q]) continue;
            const bool br = !eaten[q] && e[q] > 0 &&
                            draw(skey, uint32_t(i[q]), s ? kWolfBreed : kSheepBreed) <
                                (s ? a.T_w : a.T_s);
            // 1: breeder, 2: eaten (its slot is free for this step's births)
            tag(list, j0 + uint32_t(q * kThreads) + threadIdx.x, br ? 1u : (eaten[q] ? 2u : 0u));
        }
    }
    __syncthreads();
    // breeders (compacted in slot order for K3) and the slots free for this
    // step's births (empty, or eaten this step), ranked over two chains at once
    const bool owner = threadIdx.x < kBlock;
    const uint32_t bm = flagged(mask, first, list, 1);
    const uint32_t eaten_m = flagged(mask, first, list, 2);
    const int64_t lane0 = t.base + int64_t(threadIdx.x) * 32;
    const uint32_t in_cap = !owner || lane0 >= cap ? 0u
                          : (cap - lane0 >= 32 ? ~0u : (1u << (cap - lane0)) - 1u);
    const uint32_t free_m = ((~mask) & in_cap) | eaten_m;
    uint32_t r0, rf;
    const uint32_t total = rank_block<kWaves * H>(__popc(bm), &r0, lds);
    const uint32_t total_f = rank_block<kWaves * H>(__popc(free_m), &rf, lds + kWaves * H);
    uint32_t tile_excl, free_excl;
    hier_prefix2(a.status + a.chain_off[s], a.status + a.fchain_off[s], a.status - 1, t.tile,
                 a.tiles[s], epoch, total, total_f, lds, &tile_excl, &free_excl);
    uint32_t r = tile_excl + r0;
    for (uint32_t m = bm; m; m &= m - 1u)
        a.blist[s][r++] = int32_t(t.base + threadIdx.x * 32u + (__ffs(m) - 1));
    if (threadIdx.x == 0) a.free_pre[s][t.tile] = int32_t(free_excl);
    if (t.tile == last && threadIdx.x == 0) {
        *a.d_nb[s] = int64_t(tile_excl) + total;
        *a.d_nf[s] = int64_t(free_excl) + total_f + past;
    }
    if (a.stats && s == 0) {
        block_add(grass_eaten, a.acc + a.acc_par, kGrassEaten, lds);
        block_add(sheep_eaten, a.acc + a.acc_par, kSheepEaten, lds);
    }
}

// ------------------------------------------------------------------ K3
template <int H>
__global__ __launch_bounds__(kBlock * H) void k_breed_die(StepArgs a) {
    constexpr int kThreads = kBlock * H;
    __shared__ uint16_t list[kTile];
    __shared__ uint32_t wl[kWaves * H];
    __shared__ uint32_t lds[kWaves * H + 1];
    const bool owner = threadIdx.x < kBlock;      // owns bitmask word threadIdx.x
    const TileRef t = tile_of(a);
    const int s = t.s;
    const Species sp = a.sp[s];
    const int64_t cap = s ? a.cap_w : a.cap_s;
    const int64_t wi = int64_t(t.tile) * kBlock + threadIdx.x;
    const uint32_t mask = owner ? a.bits[s][wi] : 0u;   // live at K1, eaten sheep included
    // at the end of a tag period this workgroup's slice of the claim tables is
    // re-armed for the next step (K2, the last reader, has finished): whole
    // lines, streamed
    if (a.rearm) {
        const int64_t words = 3 * a.G, per = (words + gridDim.x - 1) / gridDim.x;
        const int64_t lo = int64_t(blockIdx.x) * per;
        const int64_t hi = lo + per < words ? lo + per : words;
        for (int64_t w = lo + threadIdx.x; w < hi; w += kThreads) a.claims[w] = kNoClaim;
    }
    const int64_t nb = *a.d_nb[s];
    if (a.stats && t.tile == a.tiles[s] - 1 && threadIdx.x == 0) {
        const int64_t nfree = *a.d_nf[s];
        a.stats[s ? kBirthsW : kBirthsS] = nfree < nb ? nfree : nb;
    }
    // the tile's free-slot prefix: from K2's scan below the mark; past it every
    // slot of every tile is free
    const uint32_t mark = uint32_t(a.mark_rd[s]);
    int64_t pre;
    if (t.tile < mark) {
        pre = a.free_pre[s][t.tile];
    } else {
        const int64_t past = cap - int64_t(mark) * kTile > 0 ? cap - int64_t(mark) * kTile : 0;
        pre = (*a.d_nf[s] - past) + int64_t(t.tile - mark) * kTile;
    }
    // a tile with no live agent and no birth (its free slots rank past the
    // breeders) has nothing to do
    const bool births_here = pre < nb;
    if (t.tile >= mark && !births_here) return;
    if (!__syncthreads_or(mask != 0u) && !births_here) return;
    uint32_t first;
    const uint32_t n = block_list<kWaves * H>(mask, list, wl, &first);
    // eaten sheep become free slots, starving agents die
    uint32_t starved = 0;
    for (uint32_t j0 = 0; j0 < n; j0 += kInFlight * kThreads) {
        int64_t i[kInFlight];
        int32_t al[kInFlight], e[kInFlight];
        bool on[kInFlight];
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            const uint32_t j = j0 + uint32_t(q * kThreads) + threadIdx.x;
            on[q] = j < n;
            i[q] = t.base + (on[q] ? list[j] : 0);
            al[q] = on[q] ? sp.alive[i[q]] : 0;
            e[q] = on[q] ? sp.e[i[q]] : 0;
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q]) continue;
            uint32_t f = 0;
            if (al[q] == 2) {
                f = 1;                      // eaten: a free slot for this step's births
                sp.alive[i[q]] = 0;
            } else if (e[q] < 0) {
                // a breeder's energy stays positive, so no slot read by a child dies here
                f = 2;
                sp.alive[i[q]] = 0;
                ++starved;
            }
            tag(list, j0 + uint32_t(q * kThreads) + threadIdx.x, f);
        }
    }
    __syncthreads();
    const uint32_t eaten_m = flagged(mask, first, list, 1);
    const uint32_t starved_m = flagged(mask, first, list, 2);
    const int64_t lane0 = t.base + int64_t(threadIdx.x) * 32;
    const uint32_t in_cap = !owner || lane0 >= cap ? 0u
                          : (cap - lane0 >= 32 ? ~0u : (1u << (cap - lane0)) - 1u);
    const uint32_t free_m = ((~mask) & in_cap) | eaten_m;
    // (the same free slots K2 ranked: its chain gave this tile's prefix)
    uint32_t r0;
    const uint32_t total = rank_block<kWaves * H>(__popc(free_m), &r0, lds);
    const uint32_t tile_excl = uint32_t(pre);
    const int64_t room = nb - int64_t(tile_excl);
    const uint32_t births = room <= 0 ? 0u : (room < int64_t(total) ? uint32_t(room) : total);
    // this lane's free slots of tile rank < births receive children
    const uint32_t mine = births > r0 ? (births - r0 < 32u ? births - r0 : 32u) : 0u;
    uint32_t born_m = 0;
    {
        uint32_t m = free_m;
        for (uint32_t k = 0; k < mine && m; ++k, m &= m - 1u) born_m |= m & (0u - m);
    }
    const uint32_t live_m = (mask & ~eaten_m & ~starved_m) | born_m;
    if (owner) a.bits[s][wi] = live_m;
    // the next step's mark: past the last tile left with a live agent
    if (__syncthreads_or(live_m != 0u) && threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(a.mark_wr + s),
                  (unsigned long long)(t.tile + 1));
    // the children, spread over the block: list the free slots that receive one
    uint32_t bfirst;
    const uint32_t nborn = block_list<kWaves * H>(born_m, list, wl, &bfirst);
    for (uint32_t j0 = 0; j0 < nborn; j0 += kInFlight * kThreads) {
        int64_t ci[kInFlight], p[kInFlight];
        int32_t px[kInFlight], py[kInFlight], pe[kInFlight];
        bool on[kInFlight];
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            const uint32_t j = j0 + uint32_t(q * kThreads) + threadIdx.x;
            on[q] = j < nborn;
            ci[q] = t.base + (on[q] ? list[j] : 0);
            p[q] = on[q] ? a.blist[s][tile_excl + j] : 0;
            if (on[q]) {
                px[q] = sp.x[p[q]];
                py[q] = sp.y[p[q]];
                pe[q] = sp.e[p[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < kInFlight; ++q) {
            if (!on[q]) continue;
            const int32_t ec = pe[q] >> 1;
            sp.x[ci[q]] = px[q];
            sp.y[ci[q]] = py[q];
            sp.e[ci[q]] = ec;
            sp.e[p[q]] = pe[q] - ec;
            sp.alive[ci[q]] = 1;
        }
    }
    if (a.stats) block_add(starved, a.acc + a.acc_par, s ? kStarvedW : kStarvedS, lds);
}

// ------------------------------------------------------------------ call edges
// Start of a call: grass countdowns -> ready steps, live bitmasks from alive,
// every claim word re-armed.  One thread per bitmask word (and cell).
__global__ __launch_bounds__(kBlock) void k_call_begin(StepArgs a, int64_t G, int64_t words_s,
                                                       int64_t words_w) {
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k < 2) a.mark_rd[k] = a.tiles[k];   // the first step visits every tile
    if (k < G) {
        a.ready[k] = int32_t(a.step + uint32_t(a.ready[k]));
        a.claims[3 * k] = kNoClaim;
        a.claims[3 * k + 1] = kNoClaim;
        a.claims[3 * k + 2] = kNoClaim;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int64_t words = s ? words_w : words_s;
        const int64_t cap = s ? a.cap_w : a.cap_s;
        if (k >= words) continue;
        const int32_t* al = a.sp[s].alive + k * 32;
        uint32_t m = 0;
        if (k * 32 + 32 <= cap && (reinterpret_cast<uintptr_t>(al) & 15) == 0) {
            int4 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = reinterpret_cast<const int4*>(al)[q];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                m |= uint32_t(v[q].x != 0) << (4 * q) | uint32_t(v[q].y != 0) << (4 * q + 1) |
                     uint32_t(v[q].z != 0) << (4 * q + 2) | uint32_t(v[q].w != 0) << (4 * q + 3);
        } else {
            for (int b = 0; b < 32 && k * 32 + b < cap; ++b) m |= uint32_t(al[b] != 0) << b;
        }
        a.bits[s][k] = m;
    }
}

// End of a call: ready steps -> countdowns at step `end`.
__global__ __launch_bounds__(kBlock) void k_call_end(int32_t* grass, int64_t G, uint32_t end) {
    const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (c < G) {
        const int32_t d = int32_t(uint32_t(grass[c]) - end);
        grass[c] = d > 0 ? d : 0;
    }
}

// The last step's fold (every other step's is done by the next step's K1).
__global__ __launch_bounds__(kBlock) void k_fold_stats(int64_t* acc, int64_t* stats) {
    fold_stats(acc, stats);
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
    a.ready = s->grass;
    a.sp[0] = species_of(s->sheep);
    a.sp[1] = species_of(s->wolves);
    a.bits[0] = w.bits_a;
    a.bits[1] = w.bits_b;
    a.G = G;
    a.claims = s->claims;
    a.status = w.status;
    a.acc = w.acc;
    a.blist[0] = w.list_a;
    a.blist[1] = w.list_b;
    a.d_nb[0] = reinterpret_cast<int64_t*>(w.hdr + kHdrCountA);
    a.d_nb[1] = reinterpret_cast<int64_t*>(w.hdr + kHdrCountB);
    a.d_nf[0] = reinterpret_cast<int64_t*>(w.hdr + kHdrFreeA);
    a.d_nf[1] = reinterpret_cast<int64_t*>(w.hdr + kHdrFreeB);
    a.tiles[0] = static_cast<uint32_t>(tiles_for(p->cap_s, kTile));
    a.tiles[1] = static_cast<uint32_t>(tiles_for(p->cap_w, kTile));
    // status words: the breeder chains of both species, then their free-slot
    // chains, then the per-tile free prefixes (int32) K2 leaves for K3; the
    // area is sized for 512-slot tiles, 16 times the chains of 8192-slot tiles
    const int64_t cw0 = chain_words(a.tiles[0]), cw1 = chain_words(a.tiles[1]);
    a.chain_off[0] = 0;
    a.chain_off[1] = static_cast<uint32_t>(cw0);
    a.fchain_off[0] = static_cast<uint32_t>(cw0 + cw1);
    a.fchain_off[1] = static_cast<uint32_t>(2 * cw0 + cw1);
    const int64_t pre_words = 2 * (cw0 + cw1) + (int64_t(a.tiles[0]) + a.tiles[1] + 1) / 2;
    if (pre_words > status_words(p->cap_s > p->cap_w ? p->cap_s : p->cap_w))
        return fail(ABM_E_WORKSPACE, "predation_step: scan state does not fit the workspace");
    a.free_pre[0] = reinterpret_cast<int32_t*>(w.status + 2 * (cw0 + cw1));
    a.free_pre[1] = a.free_pre[0] + a.tiles[0];
    a.multi = p->multi_prey;
    a.step = s->step;
    a.stats = nullptr;
    a.acc_par = 0;
    a.fold_row = nullptr;
    a.mark_rd = w.hdr + kHdrMark;
    a.mark_wr = w.hdr + kHdrMark + 2;
    // claim keys (claim_key): slots below 2^sb, a tag of up to kTagBits bits
    // sb + 32 bits up; a period of steps uses the tags t_max - 1 down to 1 (tag
    // 0 every step when only one tag bit is left), and its last step re-arms
    // the table.  Short periods re-arm often enough to cost little (one
    // streamed table per 14 steps) and keep every multi-step call crossing them.
    const int64_t max_cap = p->cap_s > p->cap_w ? p->cap_s : p->cap_w;
    uint32_t sb = 1;
    while (sb < 31 && (int64_t(1) << sb) < max_cap) ++sb;
    const uint32_t tag_bits = 32 - sb < kTagBits ? 32 - sb : kTagBits;
    const uint64_t t_max = (uint64_t(1) << tag_bits) - 1;
    const uint64_t period = t_max > 1 ? t_max - 1 : 1;
    a.sb = sb;
    a.tag_mask = ~uint64_t(0) << (32 + sb);

    const int64_t words_s = int64_t(a.tiles[0]) * kBlock, words_w = int64_t(a.tiles[1]) * kBlock;
    int64_t edge = G > words_s ? G : words_s;
    if (words_w > edge) edge = words_w;
    const dim3 tile_grid(a.tiles[0] + a.tiles[1]);
    // grass to ready steps, live bitmasks from alive, claim tables re-armed
    // (whatever the caller did to the state between calls)
    hipLaunchKernelGGL(k_call_begin, dim3(static_cast<uint32_t>(tiles_for(edge, kBlock))),
                       dim3(kBlock), 0, st, a, G, words_s, words_w);
    hipLaunchKernelGGL(k_fill64, dim3(tiles_for(kAccWords, kBlock)), dim3(kBlock), 0, st, w.acc,
                       kAccWords, int64_t(0));
    if (s->stats)
        hipLaunchKernelGGL(k_fill64, dim3(tiles_for(8 * int64_t(n_steps), kBlock)), dim3(kBlock),
                           0, st, s->stats, 8 * int64_t(n_steps), int64_t(0));
    for (int32_t k = 0; k < n_steps; ++k) {
        a.step = s->step + uint32_t(k);
        a.stats = s->stats ? s->stats + 8 * int64_t(k) : nullptr;
        a.acc_par = (k & 1) ? kHalfLanes : 0;
        a.mark_rd = w.hdr + kHdrMark + 2 * (k & 1);
        a.mark_wr = w.hdr + kHdrMark + 2 * ((k + 1) & 1);
        a.fold_row = s->stats && k > 0 ? s->stats + 8 * int64_t(k - 1) : nullptr;
        const uint64_t phase = uint64_t(k) % period;
        a.tag_hi = ((t_max > 1 ? t_max - 1 : 0) - phase) << (32 + sb);
        a.rearm = phase == period - 1;
        hipLaunchKernelGGL(k_move_claim<kHelpers>, tile_grid, dim3(kBlock * kHelpers), 0, st, a);
        if (a.multi)
            hipLaunchKernelGGL(k_prey_match, dim3(static_cast<uint32_t>(tiles_for(p->cap_w, kBlock))),
                               dim3(kBlock), 0, st, a);
        rc = next_epoch(w, st, &a.epoch);
        if (rc != ABM_OK) return rc;
        hipLaunchKernelGGL(k_eat_breeders<kHelpers>, tile_grid, dim3(kBlock * kHelpers), 0, st, a);
        hipLaunchKernelGGL(k_breed_die<kHelpers>, tile_grid, dim3(kBlock * kHelpers), 0, st, a);
    }
    if (s->stats)
        hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(kBlock), 0, st, w.acc + a.acc_par, a.stats);
    hipLaunchKernelGGL(k_call_end, dim3(static_cast<uint32_t>(tiles_for(G, kBlock))), dim3(kBlock),
                       0, st, s->grass, G, s->step + uint32_t(n_steps));
    rc = launch_status("predation_step");
    if (rc == ABM_OK) s->step += uint32_t(n_steps);
    return rc;
}
