// traffic.hip -- abm_traffic_init / abm_traffic_step: the three-lane traffic
// cellular automaton of Sec. 5.2 (Fig. 4), many roads at once (the paper
// vectorises it over roads with different car counts, Table 3).
//
// One workgroup owns one road for every step of a call: the road's car slots
// (lane, pos, alive) are loaded into LDS once, stepped there, and written back
// at the end, so a step is a few workgroup barriers and no global traffic
// besides the per-step statistics row.  A step:
//   occupancy   cell -> car slot for the start of the step (LDS);
//   decide      a car in the exit column leaves under a green light and waits
//               under red; any other car picks left / straight / right
//               uniformly (a lane off the road means straight) and, if that
//               cell one column ahead is free, posts its key
//               (direction priority << 24 | slot) by LDS atomicMin into the
//               cell: the cell, acting as an agent, admits the straight
//               arrival first, then the one from the lane below, then the one
//               from the lane above (the paper's priority mask);
//   move        winners move (the occupancy follows), losers wait, leaving
//               cars are removed (alive = 0, stale fields kept);
//   spawn       every free entry cell whose draw is below T_spawn gets a car;
//               spawned cars take the lowest free slots in lane order.
// Draws are keyed on (seed + road, step, agent, purpose): lights and spawns per
// lane, lane changes per car slot.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "rng.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxLength = 1024;   // 5 x 3L int32 of LDS per road stays below 64 KiB
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

enum TrafficCol : int {
    kCars = 0, kExited, kMoved, kBlocked, kLost, kWaitingRed, kSpawned, kLaneChanges, kCols
};

struct TrafficArgs {
    int32_t L;
    uint32_t T_green, T_spawn, seed;
    int32_t *lane, *pos, *alive;
    int64_t* stats;       // [n_steps][n_roads][kCols] or null
    int32_t n_roads;
    uint32_t step0;
    int32_t n_steps;
};

// Key of a claim on the cell ahead: the cell's priority of the arrival
// direction (straight 0, from the lane below 1, from the lane above 2) above
// the slot (slots are below 2^24).
__device__ __forceinline__ uint32_t claim_key(int32_t from, int32_t to, int32_t slot) {
    const uint32_t prio = to == from ? 0u : (from < to ? 1u : 2u);
    return (prio << 24) | uint32_t(slot);
}

// The lane a car at `lane` moves to: draw onto {-1, 0, +1}, off the road = stay.
__device__ __forceinline__ int32_t next_lane(uint64_t skey, int32_t slot, int32_t lane) {
    const int32_t nl = lane + int32_t(scale(draw(skey, uint32_t(slot), kTrafficLane), 3u)) - 1;
    return (nl < 0 || nl > 2) ? lane : nl;
}

__global__ __launch_bounds__(kBlock) void k_traffic_run(TrafficArgs a) {
    extern __shared__ int32_t sm[];
    __shared__ int32_t cnt[kCols];
    __shared__ int32_t want[3], spawn_slot[3], n_spawn;
    const int32_t L = a.L, n = 3 * L;
    int32_t* lane = sm;
    int32_t* pos = lane + n;
    int32_t* alive = pos + n;
    int32_t* occ = alive + n;                                  // start-of-step occupancy
    uint32_t* claim = reinterpret_cast<uint32_t*>(occ + n);    // lowest key per claimed cell
    const int64_t base = int64_t(blockIdx.x) * n;
    const uint32_t seed = a.seed + blockIdx.x;
    const int tid = threadIdx.x;

    for (int32_t i = tid; i < n; i += kBlock) {
        lane[i] = a.lane[base + i];
        pos[i] = a.pos[base + i];
        alive[i] = a.alive[base + i];
        claim[i] = kNoKey;
    }
    __syncthreads();
    for (int32_t k = 0; k < a.n_steps; ++k) {
        const uint32_t t = a.step0 + uint32_t(k);
        const uint64_t skey = stream_key(seed, t);
        // ---- occupancy at the start of the step
        for (int32_t c = tid; c < n; c += kBlock) occ[c] = -1;
        if (tid < kCols) cnt[tid] = 0;
        __syncthreads();
        for (int32_t i = tid; i < n; i += kBlock)
            if (alive[i]) occ[lane[i] * L + pos[i]] = i;
        __syncthreads();
        // ---- decide and claim (on the start-of-step occupancy)
        for (int32_t i = tid; i < n; i += kBlock) {
            if (!alive[i]) continue;
            atomicAdd(&cnt[kCars], 1);
            const int32_t l = lane[i], x = pos[i];
            if (x == L - 1) {
                if (draw(skey, uint32_t(l), kTrafficLight) >= a.T_green)
                    atomicAdd(&cnt[kWaitingRed], 1);
                continue;
            }
            const int32_t nl = next_lane(skey, i, l);
            const int32_t c = nl * L + x + 1;
            if (occ[c] >= 0) {
                atomicAdd(&cnt[kBlocked], 1);
                continue;
            }
            atomicMin(&claim[c], claim_key(l, nl, i));
        }
        __syncthreads();
        // ---- move the winners, remove the cars leaving under a green light
        for (int32_t i = tid; i < n; i += kBlock) {
            if (!alive[i]) continue;
            const int32_t l = lane[i], x = pos[i];
            if (x == L - 1) {
                if (draw(skey, uint32_t(l), kTrafficLight) < a.T_green) {
                    alive[i] = 0;
                    atomicAdd(&cnt[kExited], 1);
                }
                continue;
            }
            const int32_t nl = next_lane(skey, i, l);
            const int32_t c = nl * L + x + 1;
            if (occ[c] >= 0) continue;   // blocked
            if (claim[c] == claim_key(l, nl, i)) {
                lane[i] = nl;
                pos[i] = x + 1;
                atomicAdd(&cnt[kMoved], 1);
                if (nl != l) atomicAdd(&cnt[kLaneChanges], 1);
            } else {
                atomicAdd(&cnt[kLost], 1);
            }
        }
        __syncthreads();
        // entry cell l is taken after the moves iff the car that started there
        // stayed (nothing moves into column 0, and column 0 is not the exit)
        if (tid < 3) {
            const int32_t s = occ[tid * L];
            want[tid] = 0;
            if (!(s >= 0 && pos[s] == 0) &&
                draw(skey, uint32_t(tid), kTrafficSpawn) < a.T_spawn)
                want[tid] = 1;
        }
        __syncthreads();
        // ---- the lowest free slots for the spawning lanes (wave 0, by ballot)
        for (int32_t c = tid; c < n; c += kBlock) claim[c] = kNoKey;
        if (tid < 64) {
            const int32_t need = want[0] + want[1] + want[2];
            int32_t found = 0;
            for (int32_t c0 = 0; c0 < n && found < need; c0 += 64) {
                const int32_t i = c0 + tid;
                const bool is_free = i < n && alive[i] == 0;
                const uint64_t fm = __ballot(is_free);
                const int32_t r = found + int32_t(lane_rank(fm));
                if (is_free && r < need) spawn_slot[r] = i;
                found += __popcll(fm);
            }
            if (tid == 0) n_spawn = found < need ? found : need;
        }
        __syncthreads();
        if (tid < 3 && want[tid]) {
            const int32_t j = (tid > 0 ? want[0] : 0) + (tid > 1 ? want[1] : 0);
            if (j < n_spawn) {
                const int32_t s = spawn_slot[j];
                lane[s] = tid;
                pos[s] = 0;
                alive[s] = 1;
            }
        }
        if (tid == 0) cnt[kSpawned] = n_spawn;
        __syncthreads();
        if (a.stats && tid < kCols)
            a.stats[(int64_t(k) * a.n_roads + blockIdx.x) * kCols + tid] = cnt[tid];
    }
    __syncthreads();
    for (int32_t i = tid; i < n; i += kBlock) {
        a.lane[base + i] = lane[i];
        a.pos[base + i] = pos[i];
        a.alive[base + i] = alive[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_traffic_clear(int32_t* lane, int32_t* pos,
                                                         int32_t* alive, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        lane[i] = 0;
        pos[i] = 0;
        alive[i] = 0;
    }
}

int check_traffic(const abm_traffic_params* p, const abm_traffic_state* s) {
    if (!p || !s) return fail(ABM_E_INVALID, "params or state is NULL");
    if (p->length < 2 || p->length > kMaxLength)
        return fail(ABM_E_INVALID, "length must be in [2, 1024]");
    if (s->n_roads < 1 || s->n_roads > (1 << 20))
        return fail(ABM_E_INVALID, "n_roads must be in [1, 2^20]");
    if (!s->lane || !s->pos || !s->alive) return fail(ABM_E_INVALID, "car array is NULL");
    return ABM_OK;
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_traffic_init(const abm_traffic_params* p, abm_traffic_state* s, void* stream) {
    int rc = check_traffic(p, s);
    if (rc != ABM_OK) return rc;
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const int64_t n = int64_t(s->n_roads) * 3 * p->length;
    const int64_t blocks = tiles_for(n, kBlock) < 4096 ? tiles_for(n, kBlock) : 4096;
    hipLaunchKernelGGL(k_traffic_clear, dim3(uint32_t(blocks)), dim3(kBlock), 0, as_stream(stream),
                       s->lane, s->pos, s->alive, n);
    rc = launch_status("traffic_init");
    if (rc == ABM_OK) s->step = 0;
    return rc;
}

extern "C" int abm_traffic_step(const abm_traffic_params* p, abm_traffic_state* s,
                                int32_t n_steps, void* stream) {
    int rc = check_traffic(p, s);
    if (rc != ABM_OK) return rc;
    if (n_steps < 0) return fail(ABM_E_INVALID, "n_steps must be >= 0");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    if (n_steps == 0) return ABM_OK;
    TrafficArgs a;
    a.L = p->length;
    a.T_green = p->T_green;
    a.T_spawn = p->T_spawn;
    a.seed = p->seed;
    a.lane = s->lane;
    a.pos = s->pos;
    a.alive = s->alive;
    a.stats = s->stats;
    a.n_roads = s->n_roads;
    a.step0 = s->step;
    a.n_steps = n_steps;
    const size_t lds = size_t(5) * 3 * p->length * sizeof(int32_t);
    hipLaunchKernelGGL(k_traffic_run, dim3(uint32_t(s->n_roads)), dim3(kBlock), lds,
                       as_stream(stream), a);
    rc = launch_status("traffic_step");
    if (rc == ABM_OK) s->step += uint32_t(n_steps);
    return rc;
}
