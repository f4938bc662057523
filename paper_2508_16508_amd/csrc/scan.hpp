// scan.hpp -- single-pass exclusive prefix count over a selection mask:
// wave ballot/mbcnt ranks, an LDS scan of wave totals, and a hierarchical
// look-back across tiles (after the decoupled look-back of Merrill & Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016).
//
// This computes the paper's rank labels (Sec. 4, Alg. 1: cumulative sum of the
// mask times the mask) in one O(n) pass, 0-based: rank(i) = #{i' < i selected}.
//
// Tile order.  Tile t is processed by workgroup t.  A tile only waits on tiles
// with smaller ids, and each XCD dispatches its workgroups in increasing id
// order, so the smallest unfinished tile always has its workgroup resident and
// can finish.  (A ticket taken with one atomic per workgroup would not need
// that property, but same-address atomics serialise at about 12 ns each on
// MI355X: 4096 tiles would cost ~50 us.)  Waits are bounded: a wait that never
// ends sets the workspace error word and counts the missing tile as zero, so
// a broken assumption shows up as a reported error, never as a hung device.
//
// Hierarchy.  With ~2000 tiles resident at once, a flat look-back either polls
// O(T^2) status words in total or waits O(T / window) device round trips for
// the prefix frontier to arrive.  Instead tiles form groups of 64, groups form
// groups of 64, and so on.  Every tile publishes its own count (level 0); the
// last tile of each level-l group publishes the group's total at level l+1 as
// soon as it has summed that group's members, which depend only on lower
// levels -- never on earlier groups -- so no chain forms.  A tile's exclusive
// prefix is then, per level, the sum of at most 63 earlier siblings: one wave
// per level polls them in parallel (about two device round trips in total for
// 4096 tiles, and little polling traffic).
//
// Status words.  One uint64 per word: bits 63..34 epoch, 33..32 flag (1 =
// valid), 31..0 value.  The epoch is a per-launch generation number, so words
// left by earlier launches read as invalid and need no clearing pass.  Flag
// and value share one word, so relaxed agent-scope atomics suffice: no payload
// is published separately, and the 8 XCDs (separate L2s) see coherent values.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace abm {

constexpr uint32_t kFlagAgg = 1u;
constexpr uint32_t kFlagPfx = 2u;
constexpr uint32_t kEpochMask = 0x3FFFFFFFu;
// Upper bound on look-back polls of one status word (each poll is a device-
// scope load plus a short sleep, so this is on the order of a second).  A
// predecessor that never publishes is a bug; the wait then ends, the missing
// value counts as zero and *err is set, instead of hanging the device.
constexpr uint32_t kSpinLimit = 1u << 21;
// Pause between two polls of a status word (s_sleep units of 64 clocks).
#ifndef ABM_POLL_SLEEP
#define ABM_POLL_SLEEP 1
#endif

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t value) {
    return (static_cast<uint64_t>((epoch << 2) | flag) << 32) | value;
}

// Rank of this lane among the lanes whose bit is set in `ballot`.
__device__ __forceinline__ uint32_t lane_rank(uint64_t ballot) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(ballot), 0u));
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Epoch of a launch: a host-chosen value passed as an argument, or, for
// launches recorded into a graph (whose arguments are frozen), a device word
// that a one-thread kernel advances before each such launch.
struct EpochArg {
    uint32_t value;
    const uint32_t* dev;
};

__device__ __forceinline__ uint32_t read_epoch(const EpochArg& e) {
    return (e.dev ? __hip_atomic_load(e.dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : e.value) &
           kEpochMask;
}

__device__ __forceinline__ bool status_valid(uint64_t w, uint32_t epoch) {
    const uint32_t hi = static_cast<uint32_t>(w >> 32);
    return (hi >> 2) == epoch && (hi & 3u) != 0u;
}

// Polls one status word until it carries this launch's epoch (bounded).
__device__ __forceinline__ uint64_t poll_status(const uint64_t* p, uint64_t w, uint32_t epoch,
                                                uint64_t* err) {
    uint32_t spins = 0;
    while (!status_valid(w, epoch)) {
        if (++spins > kSpinLimit) {
            st_agent(err, 1ull);
            return pack_status(epoch, kFlagPfx, 0u);
        }
        __builtin_amdgcn_s_sleep(ABM_POLL_SLEEP);
        w = ld_agent(p);
    }
    return w;
}

// Number of status words one scan chain (segment) of T tiles uses: the tile
// words followed by each level's group words.
constexpr int kLevels = 4;  // 64^4 tiles per chain

__host__ __device__ __forceinline__ int64_t chain_words(int64_t T) {
    int64_t words = 0, n = T;
    for (int l = 0; l < kLevels; ++l) {
        words += n;
        n = (n + 63) >> 6;
    }
    return words;
}

// Exclusive prefix of `count` over the tiles of one chain, in tile order, for
// tile t of T.  `chain` points at the chain's status words.  Needs at least
// kLevels waves in the block; lds holds one word per wave.  Every thread gets
// the result.  Contains two block barriers.
__device__ __forceinline__ uint32_t hier_prefix(uint64_t* chain, uint64_t* err, uint32_t t,
                                                uint32_t T, uint32_t epoch, uint32_t count,
                                                uint32_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t part = 0;
    if (wave < kLevels) {
        // this level's word array and the tile's group index g at this level
        uint64_t* level = chain;
        uint32_t n = T;
        for (int l = 0; l < wave; ++l) {
            level += n;
            n = (n + 63) >> 6;
        }
        const uint32_t g = t >> (6 * wave);
        const uint32_t d = g & 63u;   // earlier siblings inside the parent group
        // this tile closes its parent group at this level (it is the group's
        // last tile, or the chain's last): it then publishes the group total
        const uint32_t pspan = 1u << (6 * (wave + 1));
        const bool publish = (((t & (pspan - 1)) == pspan - 1) || t == T - 1) && wave + 1 < kLevels;
        if (wave == 0 && lane == 0) st_agent(&level[g], pack_status(epoch, kFlagAgg, count));
        uint32_t v = 0;
        // lanes [0, d) read the earlier siblings; above level 0, lane d reads
        // the tile's own group word (published by the wave below) when the
        // parent total is needed
        if (lane < d || (lane == d && wave > 0 && publish)) {
            const uint32_t idx = g - d + lane;
            v = static_cast<uint32_t>(poll_status(&level[idx], ld_agent(&level[idx]), epoch, err));
        }
        const uint32_t own = (wave == 0) ? count : 0u;   // level 0: the tile's own count
        part = wave_sum(lane < d ? v : 0u);
        if (publish) {
            const uint32_t incl = wave_sum(v) + own;     // siblings + own group word
            if (lane == 0) st_agent(&(level + n)[g >> 6], pack_status(epoch, kFlagAgg, incl));
        }
    }
    __syncthreads();
    if (lane == 0) lds[wave] = part;
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int l = 0; l < kLevels; ++l) total += lds[l];
    return total;
}

// Ranks the ITEMS flags of every lane of a WAVES-wave block over one tile.
// Item i of lane l of wave w covers slot  tile_base + (w * ITEMS + i) * 64 + l,
// so consecutive lanes touch consecutive slots.  rank[i] receives the segment-
// wide exclusive rank of slot (i); the return value is the tile's exclusive
// prefix and *tile_total the number of selected slots in the tile.
// lds must hold WAVES + 1 words.  Ends with a block barrier.  The status
// array is preceded by the workspace header; status[-1] holds the error word.
template <int WAVES, int ITEMS>
__device__ __forceinline__ uint32_t rank_tile(const bool (&f)[ITEMS], uint32_t (&rank)[ITEMS],
                                              uint64_t* chain, uint64_t* err, uint32_t t,
                                              uint32_t T, uint32_t epoch, uint32_t* lds,
                                              uint32_t* tile_total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t b = __ballot(f[i]);
        rank[i] = run + lane_rank(b);
        run += static_cast<uint32_t>(__popcll(b));
    }
    if (lane == 0) lds[wave] = run;
    __syncthreads();
    uint32_t wave_excl = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t v = lds[w];
        wave_excl += (w < wave) ? v : 0u;
        total += v;
    }
    const uint32_t tile_excl = hier_prefix(chain, err, t, T, epoch, total, lds);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) rank[i] += tile_excl + wave_excl;
    *tile_total = total;
    return tile_excl;
}

// Tile-wide exclusive prefix of one count per thread (0 <= c < 64), in thread
// order: the wave part is a sum of bit-plane ballots (lane rank among lanes
// with bit b set, times 2^b), the block part an LDS scan of wave totals, the
// tile part the hierarchical look-back.  *thread_excl receives this thread's
// exclusive rank within the tile, *tile_total the tile's total; returns the
// tile's exclusive prefix within its chain.  lds holds WAVES + 1 words.
template <int WAVES>
__device__ __forceinline__ uint32_t rank_counts(uint32_t c, uint32_t* thread_excl,
                                                uint64_t* chain, uint64_t* err, uint32_t t,
                                                uint32_t T, uint32_t epoch, uint32_t* lds,
                                                uint32_t* tile_total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t excl = 0, wtot = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        excl += lane_rank(bal) << b;
        wtot += static_cast<uint32_t>(__popcll(bal)) << b;
    }
    if (lane == 0) lds[wave] = wtot;
    __syncthreads();
    uint32_t wave_excl = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t v = lds[w];
        wave_excl += (w < wave) ? v : 0u;
        total += v;
    }
    const uint32_t tile_excl = hier_prefix(chain, err, t, T, epoch, total, lds);
    *thread_excl = wave_excl + excl;
    *tile_total = total;
    return tile_excl;
}

// Sum of the values published (with this epoch) by status[0 .. count), read
// by the whole block with many polls in flight; the result is valid in every
// thread.  Used by reductions whose last workgroup produces the total, so the
// other workgroups never wait.  lds holds blockDim / 64 words.
__device__ __forceinline__ uint32_t block_sum_published(const uint64_t* status, int64_t count,
                                                        uint32_t epoch, uint64_t* err,
                                                        uint32_t* lds) {
    constexpr int kBatch = 8;
    uint32_t acc = 0;
    for (int64_t base = 0; base < count; base += int64_t(kBatch) * blockDim.x) {
        uint64_t w[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int64_t i = base + int64_t(k) * blockDim.x + threadIdx.x;
            w[k] = i < count ? ld_agent(&status[i]) : pack_status(epoch, kFlagAgg, 0u);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int64_t i = base + int64_t(k) * blockDim.x + threadIdx.x;
            if (i < count) w[k] = poll_status(&status[i], w[k], epoch, err);
            acc += static_cast<uint32_t>(w[k]);
        }
    }
    acc = wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    uint32_t total = 0;
    for (int i = 0; i < int(blockDim.x >> 6); ++i) total += lds[i];
    return total;
}

}  // namespace abm
