// traffic.hip -- abm_traffic_init / abm_traffic_step: the three-lane traffic
// cellular automaton of Sec. 5.2 (Fig. 4), many roads at once (the paper
// vectorises it over roads with different car counts, Table 3).
//
// One workgroup owns one road for every step of a call: the road's car slots
// (lane, pos, alive) are loaded into LDS once, stepped there, and written back
// at the end, so a step is a few workgroup barriers and no global traffic
// besides the per-step statistics row.  A step:
//   occupancy   cell -> car slot at the start of the step (LDS, built once per
//               call and then carried from step to step by the moves);
//   decide      a car in the exit column leaves under a green light and waits
//               under red; any other car picks left / straight / right
//               uniformly (a lane off the road means straight) and, if that
//               cell one column ahead is free, posts its key
//               (direction priority << 24 | slot) by LDS atomicMin into the
//               cell: the cell, acting as an agent, admits the straight
//               arrival first, then the one from the lane below, then the one
//               from the lane above (the paper's priority mask);
//   move        winners move, losers wait, leaving cars are removed (alive =
//               0, stale fields kept); the cars left fill the next step's
//               occupancy map;
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
constexpr int kWaves = kBlock / 64;
constexpr int kMaxLength = 1024;   // 21 x 3L bytes of LDS per road stays below 64 KiB
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
constexpr int8_t kBlockedCar = 3;

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

// Per-wave event counts of one step, summed over the waves for the statistics.
struct WaveCounts {
    uint32_t v[kCols];
};

__device__ __forceinline__ uint32_t count_lanes(bool f) {
    return static_cast<uint32_t>(__popcll(__ballot(f)));
}

// LDS per road: lane, pos, alive, claim (3L each, int32), two occupancy maps
// (3L each, int16: the start-of-step map of this step and the map of the next
// step, which the moves and spawns fill) and each car's decision of the step
// (3L, int8), so that the moves do not draw again.  21 x 3L bytes (63 KiB at
// L = 1024).  A step is three barriers: after the claims, after the moves,
// after the spawns.
__global__ __launch_bounds__(kBlock) void k_traffic_run(TrafficArgs a) {
    extern __shared__ int32_t sm[];
    __shared__ uint32_t cntw[kWaves][kCols];
    const int32_t L = a.L, n = 3 * L;
    int32_t* lane = sm;
    int32_t* pos = lane + n;
    int32_t* alive = pos + n;
    uint32_t* claim = reinterpret_cast<uint32_t*>(alive + n);   // lowest key per claimed cell
    int16_t* occ_buf = reinterpret_cast<int16_t*>(claim + n);
    // exit column: 1 leaves (green), 0 waits (red); elsewhere the target lane
    // 0-2, or kBlockedCar
    int8_t* dec = reinterpret_cast<int8_t*>(occ_buf + 2 * n);
    const int64_t base = int64_t(blockIdx.x) * n;
    const uint32_t seed = a.seed + blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lid = tid & 63;

    for (int32_t i = tid; i < n; i += kBlock) {
        lane[i] = a.lane[base + i];
        pos[i] = a.pos[base + i];
        alive[i] = a.alive[base + i];
        claim[i] = kNoKey;
        occ_buf[i] = -1;
    }
    __syncthreads();
    for (int32_t i = tid; i < n; i += kBlock)
        if (alive[i]) occ_buf[lane[i] * L + pos[i]] = int16_t(i);
    __syncthreads();
    for (int32_t k = 0; k < a.n_steps; ++k) {
        const uint32_t t = a.step0 + uint32_t(k);
        const uint64_t skey = stream_key(seed, t);
        const int16_t* occ = occ_buf + (k & 1) * n;           // start of this step
        int16_t* nocc = occ_buf + ((k + 1) & 1) * n;          // start of the next step
        // the previous step's statistics (its counts are complete)
        if (k > 0 && a.stats && tid < kCols) {
            uint32_t c = 0;
            for (int w = 0; w < kWaves; ++w) c += cntw[w][tid];
            a.stats[(int64_t(k - 1) * a.n_roads + blockIdx.x) * kCols + tid] = c;
        }
        WaveCounts wc = {};
        // ---- decide and claim on the start-of-step occupancy; clear the next map
        for (int32_t i0 = 0; i0 < n; i0 += kBlock) {
            const int32_t i = i0 + tid;
            bool car = false, red = false, blocked = false;
            if (i < n) {
                nocc[i] = -1;
                if (alive[i]) {
                    car = true;
                    const int32_t l = lane[i], x = pos[i];
                    if (x == L - 1) {
                        red = draw(skey, uint32_t(l), kTrafficLight) >= a.T_green;
                        dec[i] = red ? 0 : 1;
                    } else {
                        const int32_t nl = next_lane(skey, i, l);
                        const int32_t c = nl * L + x + 1;
                        blocked = occ[c] >= 0;
                        dec[i] = blocked ? kBlockedCar : int8_t(nl);
                        if (!blocked) atomicMin(&claim[c], claim_key(l, nl, i));
                    }
                }
            }
            wc.v[kCars] += count_lanes(car);
            wc.v[kWaitingRed] += count_lanes(red);
            wc.v[kBlocked] += count_lanes(blocked);
        }
        __syncthreads();
        // ---- move the winners, remove the cars leaving under a green light;
        // every car still on the road enters the next map
        for (int32_t i0 = 0; i0 < n; i0 += kBlock) {
            const int32_t i = i0 + tid;
            bool exited = false, moved = false, changed = false, lost = false;
            if (i < n && alive[i]) {
                int32_t l = lane[i], x = pos[i];
                const int32_t d = dec[i];
                if (x == L - 1) {
                    exited = d == 1;
                } else if (d != kBlockedCar) {
                    const int32_t nl = d;
                    if (claim[nl * L + x + 1] == claim_key(l, nl, i)) {
                        moved = true;
                        changed = nl != l;
                        l = nl;
                        x = x + 1;
                        lane[i] = l;
                        pos[i] = x;
                    } else {
                        lost = true;
                    }
                }
                if (exited)
                    alive[i] = 0;
                else
                    nocc[l * L + x] = int16_t(i);
            }
            wc.v[kExited] += count_lanes(exited);
            wc.v[kMoved] += count_lanes(moved);
            wc.v[kLaneChanges] += count_lanes(changed);
            wc.v[kLost] += count_lanes(lost);
        }
        __syncthreads();
        // ---- reset the claims; wave 0 spawns: entry cell l is free after the
        // moves iff the next map has no car there (nothing moves into column 0),
        // and the r-th spawning lane takes the r-th lowest free slot
        for (int32_t c = tid; c < n; c += kBlock) claim[c] = kNoKey;
        if (wave == 0) {
            const bool want = lid < 3 && nocc[lid * L] < 0 &&
                              draw(skey, uint32_t(lid), kTrafficSpawn) < a.T_spawn;
            const uint64_t wm = __ballot(want);
            const int32_t need = __popcll(wm);
            int32_t found = 0;
            for (int32_t c0 = 0; c0 < n && found < need; c0 += 64) {
                const int32_t i = c0 + lid;
                const bool is_free = i < n && alive[i] == 0;
                const uint64_t fm = __ballot(is_free);
                const int32_t r = found + int32_t(lane_rank(fm));
                if (is_free && r < need) {
                    // the r-th set bit of wm is the lane that gets this slot
                    uint64_t m = wm;
                    for (int32_t q = 0; q < r; ++q) m &= m - 1;
                    const int32_t rl = __ffsll(static_cast<unsigned long long>(m)) - 1;
                    lane[i] = rl;
                    pos[i] = 0;
                    alive[i] = 1;
                    nocc[rl * L] = int16_t(i);
                }
                found += __popcll(fm);
            }
            wc.v[kSpawned] = uint32_t(found < need ? found : need);
        }
        if (lid < kCols) {
            uint32_t v = 0;
#pragma unroll
            for (int c = 0; c < kCols; ++c) v = c == lid ? wc.v[c] : v;
            cntw[wave][lid] = v;
        }
        __syncthreads();
    }
    if (a.n_steps > 0 && a.stats && tid < kCols) {
        uint32_t c = 0;
        for (int w = 0; w < kWaves; ++w) c += cntw[w][tid];
        a.stats[(int64_t(a.n_steps - 1) * a.n_roads + blockIdx.x) * kCols + tid] = c;
    }
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
    const size_t lds = size_t(21) * 3 * p->length;
    hipLaunchKernelGGL(k_traffic_run, dim3(uint32_t(s->n_roads)), dim3(kBlock), lds,
                       as_stream(stream), a);
    rc = launch_status("traffic_step");
    if (rc == ABM_OK) s->step += uint32_t(n_steps);
    return rc;
}
