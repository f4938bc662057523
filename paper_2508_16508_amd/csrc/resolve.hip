// resolve.hip -- abm_resolve_conflicts: many claimants for one resource.
//
// The priority and the claim index are packed into one 64-bit key
// (prio << 32 | claim), so a single unsigned atomicMin per claim both picks the
// lowest priority and breaks ties by the lower index; the winner is then a
// plain equality test against the reduced key.  Three launches because each
// pass depends on the whole previous pass: reset, reduce, read back.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"

namespace abm {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_reset_keys(uint64_t* __restrict__ best, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) best[i] = ~0ull;
}

__device__ __forceinline__ bool claim_live(int64_t c, const int32_t* target, const uint8_t* active,
                                           int64_t n_targets, int32_t& t) {
    t = target[c];
    return (active == nullptr || active[c] != 0) && t >= 0 && int64_t(t) < n_targets;
}

__global__ __launch_bounds__(kBlock) void k_claim(const int32_t* __restrict__ target,
                                                  const uint32_t* __restrict__ prio,
                                                  const uint8_t* __restrict__ active,
                                                  int64_t n_claims, int64_t n_targets,
                                                  uint64_t* best) {
    const int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= n_claims) return;
    int32_t t;
    if (!claim_live(c, target, active, n_targets, t)) return;
    const uint64_t key = (uint64_t(prio[c]) << 32) | uint32_t(c);
    atomicMin(reinterpret_cast<unsigned long long*>(best + t), static_cast<unsigned long long>(key));
}

// Threads [0, n_claims) fill won[], threads [0, n_targets) fill winner[].
__global__ __launch_bounds__(kBlock) void k_readback(const int32_t* __restrict__ target,
                                                     const uint32_t* __restrict__ prio,
                                                     const uint8_t* __restrict__ active,
                                                     int64_t n_claims, int64_t n_targets,
                                                     const uint64_t* __restrict__ best,
                                                     int32_t* __restrict__ winner,
                                                     uint8_t* __restrict__ won) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n_claims) {
        int32_t t;
        uint8_t w = 0;
        if (claim_live(i, target, active, n_targets, t)) {
            const uint64_t key = (uint64_t(prio[i]) << 32) | uint32_t(i);
            w = best[t] == key ? 1 : 0;
        }
        won[i] = w;
    }
    if (i < n_targets) {
        const uint64_t b = best[i];
        winner[i] = b == ~0ull ? -1 : int32_t(uint32_t(b));
    }
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_resolve_conflicts(int64_t n_claims, const int32_t* target, const uint32_t* prio,
                                     const uint8_t* active, int64_t n_targets, uint64_t* best,
                                     int32_t* winner, uint8_t* won, void* stream) {
    // winner[] holds claim indices as int32, with -1 for "no claim"
    if (n_claims < 0 || n_claims > kMaxIndex)
        return fail(ABM_E_INVALID, "n_claims must be in [0, 2^31)");
    if (n_targets < 0 || n_targets > kMaxIndex)
        return fail(ABM_E_INVALID, "n_targets must be in [0, 2^31)");
    if (n_claims > 0 && (!target || !prio || !won))
        return fail(ABM_E_INVALID, "target, prio or won is NULL");
    if (n_targets > 0 && (!best || !winner)) return fail(ABM_E_INVALID, "best or winner is NULL");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    hipStream_t st = as_stream(stream);
    if (n_targets > 0)
        hipLaunchKernelGGL(k_reset_keys, dim3(tiles_for(n_targets, kBlock)), dim3(kBlock), 0, st,
                           best, n_targets);
    if (n_claims > 0 && n_targets > 0)
        hipLaunchKernelGGL(k_claim, dim3(tiles_for(n_claims, kBlock)), dim3(kBlock), 0, st, target,
                           prio, active, n_claims, n_targets, best);
    const int64_t m = n_claims > n_targets ? n_claims : n_targets;
    if (m > 0)
        hipLaunchKernelGGL(k_readback, dim3(tiles_for(m, kBlock)), dim3(kBlock), 0, st, target,
                           prio, active, n_claims, n_targets, best, winner, won);
    return launch_status("resolve_conflicts");
}
