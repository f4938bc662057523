// remove.hip -- abm_remove_agents: the paper's set_agents_mask (Sec. 2), an
// independent masked update with no ranking: alive[i] = 0 wherever kill[i].
//
// A workgroup owns 8192 slots, 256 lines of 32 alive words (128 bytes).  The
// lanes take 16-byte chunks in order, eight lanes to a line, so one wave
// instruction covers eight whole lines (and the matching 256 kill bytes).  A
// line with a kill byte set is loaded whole and, when one of its slots was
// live, stored whole, the unchanged chunks with the values they hold: HBM3E
// has no byte mask, so a partly written sector costs the memory a
// read-modify-write, which a later kernel pays for when the partly dirty line
// leaves the caches.  Whether the line is wanted is one ballot over its eight
// lanes.  The conditional accesses are buffer instructions whose offset is
// moved out of range when not wanted -- the hardware then skips the access --
// so there are no branches and all of a lane's loads are in flight together.
// Every workgroup but the last publishes its removed count as an epoch-tagged
// status word; the last one sums them (no same-address atomics, which
// serialise).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kSlotsPerBlock = 8192;
constexpr int kPasses = int(kSlotsPerBlock / (4 * kBlock));   // chunks per lane
constexpr int kSkip = int(0x80000000u);   // out-of-range buffer offset: access skipped
constexpr int kRsrcWord3 = 0x00020000;    // raw buffer descriptor, 32-bit data format

__global__ __launch_bounds__(kBlock) void k_remove(const uint8_t* __restrict__ kill,
                                                   int32_t* __restrict__ alive, int64_t n,
                                                   uint64_t* status, EpochArg ep,
                                                   int64_t* d_removed) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    __shared__ uint32_t lds[kBlock / 64];
    const uint32_t epoch = read_epoch(ep);
    const int64_t bfirst = int64_t(blockIdx.x) * kSlotsPerBlock;
    uint32_t removed = 0;
    if (bfirst + kSlotsPerBlock <= n) {
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
            alive + bfirst, 0, int(kSlotsPerBlock * 4), kRsrcWord3);
        const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t*>(kill) + bfirst, 0, int(kSlotsPerBlock), kRsrcWord3);
        // lane l of a wave shares its line with lanes (l & ~7) .. (l | 7)
        const int first = int(threadIdx.x & 63u) & ~7;
        uint32_t kw[kPasses];
#pragma unroll
        for (int p = 0; p < kPasses; ++p)
            kw[p] = uint32_t(__builtin_amdgcn_raw_buffer_load_b32(
                rk, (p * kBlock + int(threadIdx.x)) * 4, 0, 0));
        v4i al[kPasses];
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            const bool line = ((__ballot(kw[p] != 0u) >> first) & 0xFFu) != 0u;
            al[p] = __builtin_amdgcn_raw_buffer_load_b128(
                ra, line ? (p * kBlock + int(threadIdx.x)) * 16 : kSkip, 0, 0);
        }
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            bool changed = false;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (((kw[p] >> (8 * b)) & 0xFFu) != 0u && al[p][b] != 0) {
                    ++removed;
                    al[p][b] = 0;
                    changed = true;
                }
            }
            const bool line = ((__ballot(changed) >> first) & 0xFFu) != 0u;
            __builtin_amdgcn_raw_buffer_store_b128(
                al[p], ra, line ? (p * kBlock + int(threadIdx.x)) * 16 : kSkip, 0, 0);
        }
    } else {
        // the partial last workgroup: slot by slot
        for (int64_t s = bfirst + threadIdx.x; s < n; s += kBlock) {
            if (kill[s] != 0 && alive[s] != 0) {
                ++removed;
                alive[s] = 0;
            }
        }
    }
    const uint32_t wsum = wave_sum(removed);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = wsum;
    __syncthreads();
    uint32_t bsum = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) bsum += lds[w];
    const uint32_t last = gridDim.x - 1;
    if (blockIdx.x != last) {
        if (threadIdx.x == 0) st_agent(&status[blockIdx.x], pack_status(epoch, kFlagAgg, bsum));
        return;
    }
    const uint32_t others = block_sum_published(status, last, epoch, status - 1, lds);
    if (threadIdx.x == 0) *d_removed = int64_t(others) + bsum;
}

__global__ void k_zero_count(int64_t* d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d = 0;
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_remove_agents(const abm_soa* dst, const uint8_t* kill_mask, int64_t* d_removed,
                                 void* ws, size_t ws_bytes, void* stream) {
    if (!dst) return fail(ABM_E_INVALID, "collection is NULL");
    if (dst->capacity < 0 || dst->capacity > kMaxIndex)
        return fail(ABM_E_INVALID, "capacity must be in [0, 2^31)");
    if (dst->capacity > 0 && (!dst->alive || !kill_mask))
        return fail(ABM_E_INVALID, "alive or kill_mask is NULL");
    if (!d_removed) return fail(ABM_E_INVALID, "d_removed is NULL");
    // 16-byte vector access of the mask and alive words
    if ((reinterpret_cast<uintptr_t>(kill_mask) & 15) || (reinterpret_cast<uintptr_t>(dst->alive) & 15))
        return fail(ABM_E_INVALID, "kill_mask and alive must be 16-byte aligned");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_ws(ws, ws_bytes, dst->capacity);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, dst->capacity);
    hipStream_t st = as_stream(stream);
    if (dst->capacity == 0) {
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, st, d_removed);
        return launch_status("remove_agents");
    }
    const uint32_t nblocks = static_cast<uint32_t>(tiles_for(dst->capacity, kSlotsPerBlock));
    EpochArg ep;
    rc = next_epoch(w, st, &ep);
    if (rc != ABM_OK) return rc;
    hipLaunchKernelGGL(k_remove, dim3(nblocks), dim3(kBlock), 0, st, kill_mask, dst->alive,
                       dst->capacity, w.status, ep, d_removed);
    return launch_status("remove_agents");
}
