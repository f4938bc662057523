// remove.hip -- abm_remove_agents: the paper's set_agents_mask (Sec. 2), an
// independent masked update with no ranking: alive[i] = 0 wherever kill[i].
//
// Each lane owns 32 consecutive slots: two 16-byte loads of the kill mask,
// then, when one of its kill bytes is set, eight 16-byte loads and stores of
// alive -- its whole 128-byte line (a sparse kill mask touches only the alive
// lines it needs).  The line is always stored whole, the unchanged chunks with
// the values they hold, because HBM3E has no byte mask: a partly written
// sector costs the memory a read-modify-write, which a later kernel pays for
// when the partly dirty line leaves the caches.  The conditional
// accesses are buffer instructions whose offset is moved out of range when not
// wanted -- the hardware then skips the access -- so there are no branches and
// all eight loads are in flight together.  Every workgroup but the last
// publishes its removed count as an epoch-tagged status word; the last one
// sums them (no same-address atomics, which serialise).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kBlock = 256;
constexpr int kSlotsPerLane = 32;
constexpr int kSkip = int(0x80000000u);   // out-of-range buffer offset: access skipped
constexpr int64_t kSlotsPerBlock = int64_t(kBlock) * kSlotsPerLane;
// 16-byte chunks per stored group: the lane's whole 128-byte line
#ifndef ABM_REMOVE_GROUP_CHUNKS
#define ABM_REMOVE_GROUP_CHUNKS 8
#endif
constexpr int kGroupChunks = ABM_REMOVE_GROUP_CHUNKS;
static_assert(kGroupChunks == 1 || kGroupChunks == 2 || kGroupChunks == 4 || kGroupChunks == 8,
              "group of 1, 2, 4 or 8 chunks");

// Bits of the lane's eight chunks that share chunk q's group.
__device__ __forceinline__ constexpr uint32_t group_of(int q) {
    return ((1u << kGroupChunks) - 1u) << (q & ~(kGroupChunks - 1));
}

__global__ __launch_bounds__(kBlock) void k_remove(const uint8_t* __restrict__ kill,
                                                   int32_t* __restrict__ alive, int64_t n,
                                                   uint64_t* status, EpochArg ep,
                                                   int64_t* d_removed) {
    __shared__ uint32_t lds[kBlock / 64];
    const uint32_t epoch = read_epoch(ep);
    const int64_t first = (int64_t(blockIdx.x) * kBlock + threadIdx.x) * kSlotsPerLane;
    uint32_t removed = 0;
    if (first + kSlotsPerLane <= n) {
        typedef int v4i __attribute__((ext_vector_type(4)));
        const int64_t bfirst = int64_t(blockIdx.x) * kSlotsPerBlock;
        const int64_t bn = (n - bfirst) < kSlotsPerBlock ? (n - bfirst) : kSlotsPerBlock;
        const __amdgpu_buffer_rsrc_t ra =
            __builtin_amdgcn_make_buffer_rsrc(alive + bfirst, 0, int(bn * 4), 0x00020000);
        const uint4* kp = reinterpret_cast<const uint4*>(kill + first);
        const uint4 k0 = kp[0], k1 = kp[1];
        const uint32_t kw[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
        const int lo = int(threadIdx.x) * kSlotsPerLane * 4;
        uint32_t killc = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) killc |= uint32_t(kw[q] != 0u) << q;
        v4i al[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            al[q] = __builtin_amdgcn_raw_buffer_load_b128(
                ra, (killc & group_of(q)) ? lo + 16 * q : kSkip, 0, 0);
        uint32_t changed = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (((kw[q] >> (8 * b)) & 0xFFu) != 0u && al[q][b] != 0) {
                    ++removed;
                    al[q][b] = 0;
                    changed |= 1u << q;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            __builtin_amdgcn_raw_buffer_store_b128(al[q], ra,
                                                   (changed & group_of(q)) ? lo + 16 * q : kSkip, 0, 0);
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
