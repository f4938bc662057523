// remove.hip -- abm_remove_agents: the paper's set_agents_mask (Sec. 2), an
// independent masked update with no ranking: alive[i] = 0 wherever kill[i].
//
// Each lane owns 16 consecutive slots: one 16-byte load of the kill mask, and
// only where some kill byte is set, 16-byte loads/stores of the matching alive
// words (so a sparse kill mask touches only the alive lines it needs).  Every
// workgroup but the last publishes its removed count as an epoch-tagged status
// word; the last one sums them (no same-address atomics, which serialise).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kBlock = 256;
constexpr int kSlotsPerLane = 16;
constexpr int64_t kSlotsPerBlock = int64_t(kBlock) * kSlotsPerLane;

__global__ __launch_bounds__(kBlock) void k_remove(const uint8_t* __restrict__ kill,
                                                   int32_t* __restrict__ alive, int64_t n,
                                                   uint64_t* status, EpochArg ep,
                                                   int64_t* d_removed) {
    __shared__ uint32_t lds[kBlock / 64];
    const uint32_t epoch = read_epoch(ep);
    const int64_t first = (int64_t(blockIdx.x) * kBlock + threadIdx.x) * kSlotsPerLane;
    uint32_t removed = 0;
    if (first + kSlotsPerLane <= n) {
        const uint4 km = *reinterpret_cast<const uint4*>(kill + first);
        const uint32_t kw[4] = {km.x, km.y, km.z, km.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (kw[q] == 0u) continue;
            int4* ap = reinterpret_cast<int4*>(alive + first + 4 * q);
            int4 al = *ap;
            int32_t v[4] = {al.x, al.y, al.z, al.w};
            bool changed = false;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (((kw[q] >> (8 * b)) & 0xFFu) != 0u && v[b] != 0) {
                    ++removed;
                    v[b] = 0;
                    changed = true;
                }
            }
            if (changed) *ap = make_int4(v[0], v[1], v[2], v[3]);
        }
    } else {
        for (int64_t s = first; s < n && s < first + kSlotsPerLane; ++s) {
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
