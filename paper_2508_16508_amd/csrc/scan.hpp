// scan.hpp -- single-pass exclusive prefix count over a selection mask:
// wave ballot/mbcnt ranks, an LDS scan of wave totals, and decoupled
// look-back across tiles (Merrill & Garland, "Single-pass Parallel Prefix Scan
// with Decoupled Look-back", 2016).
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
// Status words.  One uint64 per tile: bits 63..34 epoch, 33..32 flag
// (0 invalid, 1 aggregate, 2 inclusive prefix), 31..0 value.  The epoch is a
// per-launch generation number, so status words left by earlier launches read
// as invalid and need no clearing pass.  Flag and value share one word, so
// relaxed agent-scope atomics suffice: no payload is published separately, and
// the 8 XCDs (separate L2s) see coherent values.
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
        __builtin_amdgcn_s_sleep(1);
        w = ld_agent(p);
    }
    return w;
}

// Decoupled look-back, run by one whole wave.  Publishes this tile's aggregate,
// accumulates predecessors back to the nearest inclusive prefix (or to the
// first tile of the segment, which counts as prefix 0), publishes this tile's
// inclusive prefix and returns the exclusive prefix.
__device__ __forceinline__ uint32_t lookback(uint64_t* status, uint64_t* err, uint32_t tile,
                                             uint32_t seg_first, uint32_t epoch,
                                             uint32_t aggregate) {
    const int lane = threadIdx.x & 63;
    if (tile == seg_first) {
        if (lane == 0) st_agent(&status[tile], pack_status(epoch, kFlagPfx, aggregate));
        return 0;
    }
    if (lane == 0) st_agent(&status[tile], pack_status(epoch, kFlagAgg, aggregate));
    uint32_t exclusive = 0;
    int64_t pos = static_cast<int64_t>(tile) - 1;
    for (;;) {
        const int64_t idx = pos - lane;
        uint32_t flag = kFlagPfx, value = 0;
        if (idx >= static_cast<int64_t>(seg_first)) {
            const uint64_t w = poll_status(&status[idx], ld_agent(&status[idx]), epoch, err);
            flag = static_cast<uint32_t>(w >> 32) & 3u;
            value = static_cast<uint32_t>(w);
        }
        const uint64_t pfx = __ballot(flag == kFlagPfx);
        // lanes up to and including the nearest prefix contribute
        const int nearest = pfx ? (__ffsll(static_cast<unsigned long long>(pfx)) - 1) : 64;
        exclusive += wave_sum(lane <= nearest ? value : 0u);
        if (pfx) break;
        pos -= 64;
    }
    if (lane == 0) st_agent(&status[tile], pack_status(epoch, kFlagPfx, exclusive + aggregate));
    return exclusive;
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
                                              uint64_t* status, uint32_t tile, uint32_t seg_first,
                                              uint32_t epoch, uint32_t* lds,
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
    if (wave == 0) {
        const uint32_t ex = lookback(status, status - 1, tile, seg_first, epoch, total);
        if (lane == 0) lds[WAVES] = ex;
    }
    __syncthreads();
    const uint32_t tile_excl = lds[WAVES];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) rank[i] += tile_excl + wave_excl;
    *tile_total = total;
    return tile_excl;
}

// Tile-wide exclusive prefix of one count per thread (0 <= c < 32), in thread
// order: the wave part is a sum of bit-plane ballots (lane rank among lanes
// with bit b set, times 2^b), the block part an LDS scan of wave totals, the
// tile part the decoupled look-back.  *thread_excl receives this thread's
// exclusive rank within the tile, *tile_total the tile's total; returns the
// tile's exclusive prefix within its segment.  lds holds WAVES + 1 words.
// Ends with a block barrier.
template <int WAVES>
__device__ __forceinline__ uint32_t rank_counts(uint32_t c, uint32_t* thread_excl,
                                                uint64_t* status, uint32_t tile,
                                                uint32_t seg_first, uint32_t epoch, uint32_t* lds,
                                                uint32_t* tile_total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t excl = 0, wtot = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
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
    if (wave == 0) {
        const uint32_t ex = lookback(status, status - 1, tile, seg_first, epoch, total);
        if (lane == 0) lds[WAVES] = ex;
    }
    __syncthreads();
    *thread_excl = wave_excl + excl;
    *tile_total = total;
    return lds[WAVES];
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
