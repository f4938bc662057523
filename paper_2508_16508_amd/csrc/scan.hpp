// scan.hpp -- single-pass exclusive prefix count over a selection mask:
// wave ballot/mbcnt ranks, an LDS scan of wave totals, and decoupled
// look-back across tiles (Merrill & Garland, "Single-pass Parallel Prefix Scan
// with Decoupled Look-back", 2016).
//
// This computes the paper's rank labels (Sec. 4, Alg. 1: cumulative sum of the
// mask times the mask) in one O(n) pass, 0-based: rank(i) = #{i' < i selected}.
//
// Tile order.  Blocks take tile ids from an atomic ticket, so a tile only ever
// waits on tiles that some running block already holds: forward progress does
// not depend on the order in which the hardware dispatches workgroups.
//
// Status words.  One uint64 per tile: bits 63..34 epoch, 33..32 flag
// (0 invalid, 1 aggregate, 2 inclusive prefix), 31..0 value.  The epoch is a
// per-launch generation number kept next to the ticket, so status words from
// earlier launches read as invalid and need no clearing pass.  Flag and value
// share one word, so relaxed agent-scope atomics suffice: no payload is
// published separately, and the 8 XCDs (separate L2s) see coherent values.
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

// Takes the next tile ticket (one thread per block).  The block that takes the
// last ticket of the launch resets the counter and advances the epoch for the
// next launch on this workspace; every other block has already taken its
// ticket by then, and launches on one workspace are stream-ordered.
__device__ __forceinline__ void take_ticket(uint64_t* hdr, uint32_t ntiles, uint32_t& tile,
                                            uint32_t& epoch) {
    const uint64_t old = __hip_atomic_fetch_add(hdr, 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    tile = static_cast<uint32_t>(old);
    epoch = static_cast<uint32_t>(old >> 32) & kEpochMask;
    if (tile == ntiles - 1)
        st_agent(hdr, static_cast<uint64_t>((epoch + 1) & kEpochMask) << 32);
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
            uint64_t w;
            uint32_t spins = 0;
            for (;;) {
                w = ld_agent(&status[idx]);
                const uint32_t hi = static_cast<uint32_t>(w >> 32);
                if ((hi >> 2) == epoch && (hi & 3u) != 0u) break;
                if (++spins > kSpinLimit) {
                    st_agent(err, 1ull);
                    w = pack_status(epoch, kFlagPfx, 0u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
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

}  // namespace abm
