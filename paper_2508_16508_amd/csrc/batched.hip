// batched.hip -- many independent predation models of uneven sizes in one
// persistent launch (the MI355X counterpart of vectorising whole models,
// paper Sec. 2 and Table 2, without requiring equal shapes).
//
// Each model is advanced by ONE workgroup for all of its steps, so every
// phase boundary is a workgroup barrier instead of a kernel launch.  Workgroups
// take models from a queue in a host-chosen order (largest first) until the
// queue is empty; a model whose work is done is skipped.
//
// Per step, three passes over the model's slots in chunks of blockDim x ITEMS:
//   A  move + claims   live agents move, pay one energy and post packed
//                      (draw << 32 | slot) keys by 64-bit atomicMin into the
//                      three claim words of their cell (grass, prey, eater);
//   B  eat + breeders  each live agent compares its keys with the reduced
//                      words; grass winners gain and set the cell's regrowth
//                      step, eaten sheep are marked alive = 2 (dead, claims not
//                      yet cleared); breeders are compacted in slot order;
//   C  re-arm + breed  every agent that was live at the start of the step
//                      resets the claim words it posted (so the tables return
//                      to all-ones after touching only occupied cells), then
//                      free slots (alive 0 or 2) are ranked, the free slot of
//                      rank j < #breeders pulls its child from breeder j, and
//                      live agents with negative energy die.
// Grass is stored as the step at which a cell is grown again (0 = grown from
// the start), so the per-cell regrowth pass of the one-model path disappears:
// a cell is grown at step t iff ready <= t; eating at step t sets ready = t + R.
// The countdown of the model definition is max(0, ready - steps_done).
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "rng.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr uint64_t kNoClaim = ~0ull;
constexpr uint32_t kDxPacked = 0x9224u;  // see predation.hip: dir -> dx + 1, 2 bits each
constexpr uint32_t kDyPacked = 0xA940u;

struct BatchArgs {
    abm_model_desc* models;
    const int32_t* order;      // queue order of model indices
    int32_t n_models;
    int32_t max_steps;         // per model, this launch
    int32_t* ready;            // packed per-cell regrowth step
    uint64_t* claims;          // packed, 3 words per cell
    int32_t *sx, *sy, *se, *sa;
    int32_t *wx, *wy, *we, *wa;
    uint32_t* queue;           // model queue counter (reset before the launch)
    int32_t* scratch;          // per-workgroup breeder list
    int64_t scratch_stride;    // ints per workgroup
};

__device__ __forceinline__ int32_t wrap_step(int32_t v, int32_t d, int32_t n) {
    v += d;
    return v < 0 ? n - 1 : (v >= n ? 0 : v);
}

__device__ __forceinline__ uint64_t ld_claim(const uint64_t* p) {
    // atomics execute in L2; a plain load could hit a stale line in the CU's L1
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void claim_min(uint64_t* p, uint64_t key) {
    atomicMin(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(key));
}

__device__ __forceinline__ void rearm(uint64_t* p) {
    __hip_atomic_store(p, kNoClaim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t key_of(uint64_t skey, int64_t slot, uint32_t purpose) {
    return (uint64_t(draw(skey, uint32_t(slot), purpose)) << 32) | uint32_t(slot);
}

__device__ __forceinline__ uint32_t block_sum32(uint32_t v, uint32_t* lds) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t s = 0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) s += lds[w];
    return s;
}

// Block-wide exclusive ranks of ITEMS flags per lane over one chunk (slot
// order = wave, item, lane); returns the chunk total.  lds holds one word per
// wave.  Two barriers.
template <int ITEMS>
__device__ __forceinline__ uint32_t chunk_rank(const bool (&f)[ITEMS], uint32_t (&rank)[ITEMS],
                                               uint32_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint64_t b = __ballot(f[k]);
        rank[k] = run + lane_rank(b);
        run += static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    if (lane == 0) lds[wave] = run;
    __syncthreads();
    uint32_t before = 0, all = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        const uint32_t v = lds[w];
        before += w < wave ? v : 0u;
        all += v;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) rank[k] += before;
    return all;
}

struct ModelView {
    int32_t W, H, R, gain[2];
    uint32_t T[2], seed;
    int32_t cap[2];
    int32_t* ready;
    uint64_t* claims;
    int32_t *x[2], *y[2], *e[2], *al[2];
};

__device__ __forceinline__ bool on_grid(const ModelView& v, int32_t x, int32_t y) {
    return x >= 0 && x < v.W && y >= 0 && y < v.H;
}

// One step t of model v.  A chunk is blockDim * ITEMS slots; item k of lane l
// of wave w is slot c0 + (w * ITEMS + k) * 64 + l, so each load instruction of
// a wave covers 64 consecutive slots and the ITEMS loads of a lane are issued
// together.  breeders: this workgroup's scratch list.
template <int ITEMS>
__device__ void model_step(const ModelView& v, uint32_t t, int32_t* breeders, uint32_t* lds,
                           uint32_t* live_out) {
    const uint64_t skey = stream_key(v.seed, t);
    const uint32_t move_p[2] = {kSheepMove, kWolfMove};
    const uint32_t breed_p[2] = {kSheepBreed, kWolfBreed};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t chunk = int32_t(blockDim.x) * ITEMS;
    const int32_t lbase = wave * ITEMS * 64 + lane;

    // ---- A: move + claims
    uint32_t live = 0;
    for (int s = 0; s < 2; ++s) {
        for (int32_t c0 = 0; c0 < v.cap[s]; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < v.cap[s] ? v.al[s][i] : 0;
            }
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (al[k] == 0) continue;
                const int32_t i = c0 + lbase + k * 64;
                ++live;
                const uint32_t d = draw(skey, uint32_t(i), move_p[s]) >> 29;
                const int32_t x =
                    wrap_step(v.x[s][i], int32_t((kDxPacked >> (2 * d)) & 3u) - 1, v.W);
                const int32_t y =
                    wrap_step(v.y[s][i], int32_t((kDyPacked >> (2 * d)) & 3u) - 1, v.H);
                v.x[s][i] = x;
                v.y[s][i] = y;
                v.e[s][i] -= 1;
                if (!on_grid(v, x, y)) continue;
                const int64_t c = int64_t(y) * v.W + x;
                uint64_t* cw = v.claims + 3 * c;
                if (s == 0) {
                    if (v.ready[c] <= int32_t(t)) claim_min(cw + 0, key_of(skey, i, kSheepGrassKey));
                    claim_min(cw + 1, key_of(skey, i, kSheepPreyKey));
                } else {
                    claim_min(cw + 2, key_of(skey, i, kWolfEatKey));
                }
            }
        }
    }
    *live_out = block_sum32(live, lds);   // (barrier: claims complete)

    // ---- B: eat + breeder compaction (per species, ascending slots)
    uint32_t nb[2];
    for (int s = 0; s < 2; ++s) {
        uint32_t base_rank = 0;
        for (int32_t c0 = 0; c0 < v.cap[s]; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < v.cap[s] ? v.al[s][i] : 0;
            }
            bool br[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                br[k] = false;
                if (al[k] == 0) continue;
                const int32_t i = c0 + lbase + k * 64;
                const int32_t x = v.x[s][i], y = v.y[s][i];
                int32_t e = v.e[s][i];
                bool eaten = false;
                if (on_grid(v, x, y)) {
                    const int64_t c = int64_t(y) * v.W + x;
                    const uint64_t* cw = v.claims + 3 * c;
                    if (s == 0) {
                        if (ld_claim(cw + 0) == key_of(skey, i, kSheepGrassKey)) {
                            e += v.gain[0];
                            v.e[0][i] = e;
                            v.ready[c] = int32_t(t) + v.R;
                        }
                        if (ld_claim(cw + 2) != kNoClaim &&
                            ld_claim(cw + 1) == key_of(skey, i, kSheepPreyKey)) {
                            v.al[0][i] = 2;   // eaten: dead, its claims still to be reset
                            eaten = true;
                        }
                    } else if (ld_claim(cw + 1) != kNoClaim &&
                               ld_claim(cw + 2) == key_of(skey, i, kWolfEatKey)) {
                        e += v.gain[1];
                        v.e[1][i] = e;
                    }
                }
                br[k] = !eaten && e > 0 && draw(skey, uint32_t(i), breed_p[s]) < v.T[s];
            }
            uint32_t rank[ITEMS];
            const uint32_t tot = chunk_rank<ITEMS>(br, rank, lds);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k)
                if (br[k]) breeders[(s ? v.cap[0] : 0) + base_rank + rank[k]] = c0 + lbase + k * 64;
            base_rank += tot;
        }
        nb[s] = base_rank;
    }
    __syncthreads();

    // ---- C: re-arm claims, breed into free slots, starve
    for (int s = 0; s < 2; ++s) {
        uint32_t base_rank = 0;
        for (int32_t c0 = 0; c0 < v.cap[s]; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < v.cap[s] ? v.al[s][i] : 1;
            }
            bool fr[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                fr[k] = i < v.cap[s] && (al[k] == 0 || al[k] == 2);
                if (i >= v.cap[s] || al[k] == 0) continue;
                // this agent posted claims in A: reset them
                const int32_t x = v.x[s][i], y = v.y[s][i];
                if (!on_grid(v, x, y)) continue;
                uint64_t* cw = v.claims + 3 * (int64_t(y) * v.W + x);
                if (s == 0) {
                    rearm(cw + 0);
                    rearm(cw + 1);
                } else {
                    rearm(cw + 2);
                }
            }
            uint32_t rank[ITEMS];
            const uint32_t tot = chunk_rank<ITEMS>(fr, rank, lds);   // barrier: x/y read first
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                const uint32_t j = base_rank + rank[k];
                if (fr[k] && j < nb[s]) {
                    const int32_t p = breeders[(s ? v.cap[0] : 0) + j];
                    const int32_t ep = v.e[s][p];
                    const int32_t ec = ep >> 1;
                    v.x[s][i] = v.x[s][p];
                    v.y[s][i] = v.y[s][p];
                    v.e[s][i] = ec;
                    v.e[s][p] = ep - ec;
                    v.al[s][i] = 1;
                } else if (i < v.cap[s]) {
                    if (al[k] == 2) {
                        v.al[s][i] = 0;
                    } else if (al[k] != 0 && v.e[s][i] < 0) {
                        // a breeder's energy stays positive, so no slot read by a child dies here
                        v.al[s][i] = 0;
                    }
                }
            }
            base_rank += tot;
        }
    }
    __syncthreads();
}

template <int ITEMS>
__global__ __launch_bounds__(1024) void k_batched_run(BatchArgs a) {
    __shared__ uint32_t lds[16];
    __shared__ int32_t s_model;
    int32_t* breeders = a.scratch + int64_t(blockIdx.x) * a.scratch_stride;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t q = atomicAdd(a.queue, 1u);
            s_model = q < uint32_t(a.n_models) ? a.order[q] : -1;
        }
        __syncthreads();
        const int32_t m = s_model;
        __syncthreads();
        if (m < 0) break;
        abm_model_desc* d = a.models + m;
        if (d->cap_s + d->cap_w > a.scratch_stride) {
            // the descriptor does not fit the breeder list (max_cap too small):
            // leave the model untouched and report it
            if (threadIdx.x == 0)
                __hip_atomic_store(reinterpret_cast<uint64_t*>(a.queue) + kHdrError, 1ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        ModelView v;
        v.W = d->W;
        v.H = d->H;
        v.R = d->R;
        v.gain[0] = d->gain_s;
        v.gain[1] = d->gain_w;
        v.T[0] = d->T_s;
        v.T[1] = d->T_w;
        v.seed = d->seed;
        v.cap[0] = int32_t(d->cap_s);
        v.cap[1] = int32_t(d->cap_w);
        v.ready = a.ready + d->cell_off;
        v.claims = a.claims + 3 * d->cell_off;
        v.x[0] = a.sx + d->sheep_off;
        v.y[0] = a.sy + d->sheep_off;
        v.e[0] = a.se + d->sheep_off;
        v.al[0] = a.sa + d->sheep_off;
        v.x[1] = a.wx + d->wolf_off;
        v.y[1] = a.wy + d->wolf_off;
        v.e[1] = a.we + d->wolf_off;
        v.al[1] = a.wa + d->wolf_off;
        const int32_t t0 = d->step;
        int32_t t1 = d->steps_target;
        if (t1 - t0 > a.max_steps) t1 = t0 + a.max_steps;
        uint64_t updates = 0;
        for (int32_t t = t0; t < t1; ++t) {
            uint32_t live;
            model_step<ITEMS>(v, uint32_t(t), breeders, lds, &live);
            updates += live;
        }
        if (threadIdx.x == 0 && t1 > t0) {
            d->step = t1;
            d->updates += int64_t(updates);
        }
        __syncthreads();
    }
}

// Initial state of every model (same definition as the one-model path).
__global__ __launch_bounds__(256) void k_batched_init(abm_model_desc* models, int32_t n_models,
                                                     int32_t* ready, uint64_t* claims,
                                                     int32_t* sx, int32_t* sy, int32_t* se,
                                                     int32_t* sa, int32_t* wx, int32_t* wy,
                                                     int32_t* we, int32_t* wa) {
    const abm_model_desc& d = models[blockIdx.y];
    const int64_t G = int64_t(d.W) * d.H;
    const uint64_t key = stream_key(d.seed, kInitStep);
    int64_t m = G;
    if (d.cap_s > m) m = d.cap_s;
    if (d.cap_w > m) m = d.cap_w;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < m; i += int64_t(gridDim.x) * 256) {
        if (i < G) {
            const uint32_t h = draw(key, uint32_t(i), kGrassGrown);
            ready[d.cell_off + i] =
                h < 0x80000000u ? 0
                                : 1 + int32_t(scale(draw(key, uint32_t(i), kGrassCountdown),
                                                    uint32_t(d.R)));
            uint64_t* cw = claims + 3 * (d.cell_off + i);
            cw[0] = kNoClaim;
            cw[1] = kNoClaim;
            cw[2] = kNoClaim;
        }
        for (int s = 0; s < 2; ++s) {
            const int64_t cap = s ? d.cap_w : d.cap_s;
            if (i >= cap) continue;
            const int64_t n0 = s ? d.n_w0 : d.n_s0;
            const int32_t gain = s ? d.gain_w : d.gain_s;
            const uint32_t px = s ? kWolfX : kSheepX;
            int32_t x = 0, y = 0, e = 0, al = 0;
            if (i < n0) {
                x = int32_t(scale(draw(key, uint32_t(i), px), uint32_t(d.W)));
                y = int32_t(scale(draw(key, uint32_t(i), px + 1), uint32_t(d.H)));
                e = int32_t(scale(draw(key, uint32_t(i), px + 2), uint32_t(2 * gain)));
                al = 1;
            }
            const int64_t o = (s ? d.wolf_off : d.sheep_off) + i;
            (s ? wx : sx)[o] = x;
            (s ? wy : sy)[o] = y;
            (s ? we : se)[o] = e;
            (s ? wa : sa)[o] = al;
        }
    }
}

// countdown[c] = max(0, ready[c] - step) for every cell of every model.
__global__ __launch_bounds__(256) void k_batched_grass(const abm_model_desc* models,
                                                      const int32_t* ready, int32_t* countdown) {
    const abm_model_desc& d = models[blockIdx.y];
    const int64_t G = int64_t(d.W) * d.H;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < G; i += int64_t(gridDim.x) * 256) {
        const int32_t r = ready[d.cell_off + i] - d.step;
        countdown[d.cell_off + i] = r > 0 ? r : 0;
    }
}

// Live counts per model (stored into the descriptors).
__global__ __launch_bounds__(256) void k_batched_count(abm_model_desc* models, const int32_t* sa,
                                                      const int32_t* wa) {
    __shared__ uint32_t lds[4];
    abm_model_desc& d = models[blockIdx.x];
    uint32_t ls = 0, lw = 0;
    for (int64_t i = threadIdx.x; i < d.cap_s; i += 256) ls += sa[d.sheep_off + i] != 0;
    for (int64_t i = threadIdx.x; i < d.cap_w; i += 256) lw += wa[d.wolf_off + i] != 0;
    ls = block_sum32(ls, lds);
    lw = block_sum32(lw, lds);
    if (threadIdx.x == 0) {
        d.live_s = ls;
        d.live_w = lw;
    }
}

__global__ void k_reset_queue(uint32_t* q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *reinterpret_cast<uint64_t*>(q) = 0;
}

int check_batch(const abm_batch* b) {
    if (!b) return fail(ABM_E_INVALID, "batch is NULL");
    if (b->n_models < 0 || b->n_models > 65535)
        return fail(ABM_E_INVALID, "n_models must be in [0, 65535]");
    if (b->n_models == 0) return ABM_OK;
    if (!b->models || !b->ready || !b->claims) return fail(ABM_E_INVALID, "batch array is NULL");
    const abm_species* sp[2] = {&b->sheep, &b->wolves};
    for (int k = 0; k < 2; ++k)
        if (!sp[k]->x || !sp[k]->y || !sp[k]->e || !sp[k]->alive)
            return fail(ABM_E_INVALID, "species array is NULL");
    if (b->max_cap < 1 || b->max_cap > (1 << 30))
        return fail(ABM_E_INVALID, "max_cap must be in [1, 2^30]");
    return ABM_OK;
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" size_t abm_batched_workspace_bytes(int64_t max_cap, int32_t n_workgroups) {
    if (max_cap < 1 || n_workgroups < 1) return 0;
    return size_t(kHeaderBytes) + size_t(n_workgroups) * size_t(2 * max_cap) * 4 + 256;
}

extern "C" int abm_predation_batched_init(const abm_batch* b, void* stream) {
    int rc = check_batch(b);
    if (rc != ABM_OK || b->n_models == 0) return rc;
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const dim3 grid(64, static_cast<uint32_t>(b->n_models));
    hipLaunchKernelGGL(k_batched_init, grid, dim3(256), 0, as_stream(stream), b->models,
                       b->n_models, b->ready, b->claims, b->sheep.x, b->sheep.y, b->sheep.e,
                       b->sheep.alive, b->wolves.x, b->wolves.y, b->wolves.e, b->wolves.alive);
    return launch_status("predation_batched_init");
}

extern "C" int abm_predation_run_batched(const abm_batch* b, const int32_t* order,
                                         int32_t max_steps, const abm_tuning* tune, void* ws,
                                         size_t ws_bytes, void* stream) {
    int rc = check_batch(b);
    if (rc != ABM_OK) return rc;
    if (max_steps < 0) return fail(ABM_E_INVALID, "max_steps must be >= 0");
    if (b->n_models == 0 || max_steps == 0) return ABM_OK;
    if (!order) return fail(ABM_E_INVALID, "order is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    int block = tune && tune->block_threads ? tune->block_threads : 512;
    if (block < 256 || block > 1024 || (block & 63))
        return fail(ABM_E_INVALID, "block_threads must be a multiple of 64 in [256, 1024]");
    const int items = tune && tune->items ? tune->items : 4;
    if (items != 1 && items != 2 && items != 4 && items != 8)
        return fail(ABM_E_INVALID, "items must be 1, 2, 4 or 8");
    const void* kern = items == 1 ? reinterpret_cast<const void*>(k_batched_run<1>)
                     : items == 2 ? reinterpret_cast<const void*>(k_batched_run<2>)
                     : items == 4 ? reinterpret_cast<const void*>(k_batched_run<4>)
                                  : reinterpret_cast<const void*>(k_batched_run<8>);
    int dev = 0, n_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0) != hipSuccess)
        return launch_status("predation_run_batched: device query");
    if (per_cu < 1) per_cu = 1;
    int grid = n_cu * per_cu;
    if (tune && tune->workgroups > 0 && tune->workgroups < grid) grid = tune->workgroups;
    if (grid > b->n_models) grid = b->n_models;
    const size_t need = abm_batched_workspace_bytes(b->max_cap, grid);
    if (!ws || ws_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", ws_bytes, need);
        return ABM_E_WORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(ABM_E_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = as_stream(stream);
    BatchArgs a;
    a.models = b->models;
    a.order = order;
    a.n_models = b->n_models;
    a.max_steps = max_steps;
    a.ready = b->ready;
    a.claims = b->claims;
    a.sx = b->sheep.x;
    a.sy = b->sheep.y;
    a.se = b->sheep.e;
    a.sa = b->sheep.alive;
    a.wx = b->wolves.x;
    a.wy = b->wolves.y;
    a.we = b->wolves.e;
    a.wa = b->wolves.alive;
    a.queue = reinterpret_cast<uint32_t*>(ws);
    a.scratch = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + kHeaderBytes);
    a.scratch_stride = 2 * b->max_cap;
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, a.queue);
    switch (items) {
        case 1: hipLaunchKernelGGL(k_batched_run<1>, dim3(grid), dim3(block), 0, st, a); break;
        case 2: hipLaunchKernelGGL(k_batched_run<2>, dim3(grid), dim3(block), 0, st, a); break;
        case 4: hipLaunchKernelGGL(k_batched_run<4>, dim3(grid), dim3(block), 0, st, a); break;
        default: hipLaunchKernelGGL(k_batched_run<8>, dim3(grid), dim3(block), 0, st, a); break;
    }
    hipLaunchKernelGGL(k_batched_count, dim3(b->n_models), dim3(256), 0, st, b->models,
                       b->sheep.alive, b->wolves.alive);
    return launch_status("predation_run_batched");
}

extern "C" int abm_predation_batched_grass(const abm_batch* b, int32_t* countdown, void* stream) {
    int rc = check_batch(b);
    if (rc != ABM_OK || b->n_models == 0) return rc;
    if (!countdown) return fail(ABM_E_INVALID, "countdown is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const dim3 grid(64, static_cast<uint32_t>(b->n_models));
    hipLaunchKernelGGL(k_batched_grass, grid, dim3(256), 0, as_stream(stream), b->models, b->ready,
                       countdown);
    return launch_status("predation_batched_grass");
}
