// batched.hip -- many independent predation models of uneven sizes in one
// persistent launch (the MI355X counterpart of vectorising whole models,
// paper Sec. 2 and Table 2, without requiring equal shapes).
//
// Each model is advanced by ONE workgroup for all of its steps, so every
// phase boundary is a workgroup barrier instead of a kernel launch.  Workgroups
// take models from a queue in a host-chosen order (largest first) until the
// queue is empty; a model whose work is done is skipped.
//
// Per step, three passes over the model's slots in chunks of blockDim x ITEMS
// (below each range's high-water mark, see model_step):
//   A  move + claims   live agents move, pay one energy and post packed
//                      (tag, draw, slot) keys by 64-bit atomicMin into the
//                      three claim words of their cell (grass, prey, eater);
//   B  eat + breeders  each live agent compares its keys with the reduced
//                      words; grass winners gain and set the cell's regrowth
//                      step, eaten sheep are marked alive = 2 (dead, claims not
//                      yet cleared); breeders are compacted in slot order;
//                      (multi-prey models: in A the agents push themselves onto
//                      lists of their cell instead of posting prey and eater
//                      keys, and a pass between A and B pairs each cell's
//                      wolves and sheep by rank; see prey_match)
//   C  breed           free slots (alive 0 or 2) are ranked, the free slot of
//                      rank j < #breeders pulls its child from breeder j, and
//                      live agents with negative energy die.
// Claim keys carry a step tag (see tagged_key): within a period of steps a
// word left by an earlier step reads as unclaimed and loses to every fresh
// key, so the model's claim table is re-armed (streamed back to all-ones) only
// in pass C of a period's last step and of the last step a launch runs, which
// keeps the tables all-ones between launches.
// A model run by one workgroup whose claim table (three words per cell) fits
// in the workgroup's dynamic LDS keeps it there (LOCAL): the table is set to
// all-ones when the model is taken, pass A posts into it with LDS atomics, and
// pass C clears it whole every step.  The global table of such a model is not touched.  The launch
// gives each workgroup the LDS its occupancy leaves free, so no workgroup
// is displaced for it.
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
constexpr uint32_t kTagBits = 4;     // claim-key tag: periods of 14 steps
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
    uint32_t* queue;           // two model queue counters (reset before the launch)
    int32_t* scratch;          // per-workgroup breeder list
    int64_t scratch_stride;    // ints per workgroup
    uint64_t* err;             // workspace error word
    int32_t *link_s, *link_w;  // per-cell list links of multi-prey models (or null)
    int32_t n_team;            // order[0, n_team) run in teams
    int32_t lds_words;         // dynamic LDS claim words per workgroup (0: none)
    uint32_t team_k;           // members per team
    uint32_t team_wgs;         // workgroups in teams (multiple of 8 * team_k)
    uint32_t* team_ctr;        // barrier counter per team
    int32_t* team_mail;        // model mailbox per team
    int32_t* team_counts;      // [workgroup][5] member counts
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

// A claim posted into the LOCAL table, through an LDS-qualified pointer (a
// generic pointer into LDS does not compile for this atomic here).
__device__ __forceinline__ void claim_min_lds(uint64_t* p, uint64_t key) {
    typedef __attribute__((address_space(3))) unsigned long long lds_u64;
    __hip_atomic_fetch_min((lds_u64*)p, static_cast<unsigned long long>(key), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Makes `word` (a slot with the step's tag) the head of the list whose head
// is *p; returns the previous head.
__device__ __forceinline__ uint64_t push_head(uint64_t* p, uint64_t word) {
    return __hip_atomic_exchange(p, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t push_head_lds(uint64_t* p, uint64_t word) {
    typedef __attribute__((address_space(3))) unsigned long long lds_u64;
    return __hip_atomic_exchange((lds_u64*)p, static_cast<unsigned long long>(word),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void rearm(uint64_t* p) {
    __hip_atomic_store(p, kNoClaim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The LOCAL claim table: the workgroup's dynamic LDS.
__device__ __forceinline__ uint64_t* local_claims() {
    extern __shared__ uint64_t dyn_claims[];
    return dyn_claims;
}

__device__ __forceinline__ void local_fill(uint64_t* lc, int32_t words) {
    for (int32_t i = threadIdx.x; i < words; i += blockDim.x) lc[i] = kNoClaim;
}

// (tag, draw, slot) from the high bits down: within a step these order as
// (draw, slot), the method's claim order; an earlier step of the period has
// a larger tag, so its words lose to fresh keys and read as unclaimed.
__device__ __forceinline__ uint64_t tagged_key(uint64_t tag_hi, uint32_t sb, uint64_t skey,
                                               int64_t slot, uint32_t purpose) {
    return tag_hi | (uint64_t(draw(skey, uint32_t(slot), purpose)) << sb) | uint64_t(slot);
}

// The ranking order of multi-prey (no tag: only keys of one step are compared).
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

// Block-wide maximum of one value per thread (every thread gets it); lds
// holds one word per wave.  Two barriers.
__device__ __forceinline__ int32_t block_max32(int32_t v, uint32_t* lds) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = uint32_t(v);
    __syncthreads();
    int32_t m = int32_t(lds[0]);
    for (int w = 1; w < int(blockDim.x >> 6); ++w) m = max(m, int32_t(lds[w]));
    return m;
}

// Block-wide inclusive scan of one value per thread: *incl gets this thread's
// inclusive prefix, the return value the block total.  lds holds one word per
// wave.
__device__ __forceinline__ uint32_t block_incl_scan32(uint32_t v, uint32_t* lds, uint32_t* incl) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) {
        const uint32_t s = lds[w];
        before += w < wave ? s : 0u;
        all += s;
    }
    *incl = before + x;
    return all;
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
    bool multi;                  // prey matched by rank within a cell
    uint32_t sb;                 // slot bits of a claim key
    uint32_t period;             // steps per tag period
    uint64_t tag_top;            // the first tag of a period
    uint64_t tag_mask;           // the tag field and the bits above it
    int32_t cap[2];
    int32_t* link[2];            // list links (multi), per species
    int32_t* ready;
    uint64_t* claims;
    int32_t *x[2], *y[2], *e[2], *al[2];
};

__device__ __forceinline__ bool on_grid(const ModelView& v, int32_t x, int32_t y) {
    return x >= 0 && x < v.W && y >= 0 && y < v.H;
}

// A team of K workgroups advancing one model together (K = 1: one workgroup
// alone).  Member r owns the r-th contiguous K-th of each species' slots and
// keeps its own breeder list; members exchange per-range counts.  Members of a
// team are the workgroups base, base + 8, ..., base + 8 (K - 1): workgroups are
// dispatched to the eight XCDs in turn, so the members normally share one L2.
// Correctness does not rest on that: the team barrier uses agent-scope fences.
constexpr int kMaxTeam = 16;
constexpr int kCountWords = 5;   // breeders of both species, free slots of both, live
constexpr int kMaxWorkgroups = 8 * 1024;

struct Team {
    int K, r;
    uint32_t gen;               // team barriers passed
    uint32_t* ctr;              // barrier counter (K > 1)
    int32_t* scratch;           // lists of all workgroups
    int64_t stride;             // ints per list
    int32_t* counts;            // [workgroup][kCountWords]
    uint32_t base;              // workgroup index of member 0
    uint64_t* err;
    int32_t* s_pre;             // LDS: breeder prefixes [2][kMaxTeam + 1], free prefix [2], live
    int32_t* s_ok;              // LDS: barrier outcome
    int32_t* s_bound;           // LDS: [2][kMaxTeam + 1] member range bounds of this launch
    int32_t* s_mark;            // LDS: [2] per species, 1 + the member's highest live slot after
                                // the last step (no live agent at or above it), or INT32_MAX
};

__device__ __forceinline__ int32_t* member_list(const Team& tm, int j) {
    return tm.scratch + int64_t(tm.base + 8u * uint32_t(j)) * tm.stride;
}

// Team-wide barrier; false if a member never arrived (the error word is set).
// Every wave waits until its own stores are performed at the L2, then the
// workgroup barrier; thread 0 alone makes the L2 contents visible device-wide
// (agent-scope release), counts the member in, waits for the others and
// acquires (agent scope, which also drops the CU's stale L1 lines) before the
// second workgroup barrier releases the other waves.  One release per member
// instead of one per wave: every wave writing back the L2 costs ~10x more
// when hundreds of workgroups are resident.
__device__ __forceinline__ bool team_sync(Team& tm) {
    if (tm.K == 1) {
        __syncthreads();
        return true;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(tm.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (tm.gen + 1) * uint32_t(tm.K);
        int32_t ok = 1;
        uint32_t spins = 0;
        while (__hip_atomic_load(tm.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit) {
                st_agent(tm.err, 1ull);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *tm.s_ok = ok;
    }
    __syncthreads();
    ++tm.gen;
    return *tm.s_ok != 0;
}

// Multi-prey rule for wolf j whose cell's words are cw (Sec. 4, Alg. 1 applied
// within one cell): j has rank r among the cell's wolves by eat key and takes
// the sheep of rank r among the cell's sheep by prey key, if there is one,
// marking it alive = 2 and gaining.  Ranks are counted by walking the cell's
// lists, whose heads are the prey (sheep) and eater (wolf) words; distinct
// wolves have distinct ranks, so no sheep is taken twice.  Quadratic in the
// sheep of one cell, which are few at the workloads' densities.
template <class Read, class Head>
__device__ __forceinline__ void prey_match(const ModelView& v, uint64_t skey, const uint64_t* cw,
                                           int32_t j, Read rd, Head head) {
    const int32_t first = head(rd(cw + 1));
    if (first < 0) return;
    const uint64_t mine = key_of(skey, j, kWolfEatKey);
    uint32_t r = 0;
    for (int32_t w = head(rd(cw + 2)); w >= 0; w = v.link[1][w])
        r += key_of(skey, w, kWolfEatKey) < mine ? 1u : 0u;
    for (int32_t q = first; q >= 0; q = v.link[0][q]) {
        const uint64_t kq = key_of(skey, q, kSheepPreyKey);
        uint32_t below = 0;
        for (int32_t u = first; u >= 0; u = v.link[0][u])
            below += key_of(skey, u, kSheepPreyKey) < kq ? 1u : 0u;
        if (below == r) {
            v.al[0][q] = 2;
            v.e[1][j] += v.gain[1];
            return;
        }
    }
}

// One step t of model v by team tm; false if the team barrier failed.  A chunk
// is blockDim * ITEMS slots; item k of lane l of wave w is slot
// c0 + (w * ITEMS + k) * 64 + l, so each load instruction of a wave covers 64
// consecutive slots and the ITEMS loads of a lane are issued together.
template <int ITEMS, bool LOCAL>
__device__ bool model_step(const ModelView& v, uint32_t t, uint32_t t0, bool last, Team& tm,
                           uint32_t* lds, uint32_t* live_out) {
    uint64_t* const claims = LOCAL ? local_claims() : v.claims;
    // LOCAL: the atomics of pass A are complete at the barrier that ends it
    auto rd = [](const uint64_t* p) { return LOCAL ? *p : ld_claim(p); };
    auto post = [](uint64_t* p, uint64_t key) {
        if constexpr (LOCAL)
            claim_min_lds(p, key);
        else
            claim_min(p, key);
    };
    // wave-uniform: kept in scalar registers
    const uint32_t phase = __builtin_amdgcn_readfirstlane((t - t0) % v.period);
    const uint32_t sb = __builtin_amdgcn_readfirstlane(v.sb);
    const uint64_t tag_hi =
        uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(v.tag_top - phase) << sb)) << 32;
    const uint64_t tag_mask =
        uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(v.tag_mask >> 32))) << 32;
    auto claimed = [tag_hi, tag_mask](uint64_t w) { return (w & tag_mask) == tag_hi; };
    // a list head's slot, or -1 (a word of an earlier step, or all-ones: the end)
    auto head = [tag_hi, tag_mask](uint64_t w) {
        return (w & tag_mask) == tag_hi ? int32_t(w & ~tag_mask) : -1;
    };
    // multi-prey: the agent's link is the cell's previous head
    auto push = [tag_hi, head](uint64_t* p, int32_t slot, int32_t* link) {
        const uint64_t word = tag_hi | uint64_t(uint32_t(slot));
        const uint64_t prev = LOCAL ? push_head_lds(p, word) : push_head(p, word);
        link[slot] = head(prev);
    };
    const uint64_t skey = stream_key(v.seed, t);
    const uint32_t move_p[2] = {kSheepMove, kWolfMove};
    const uint32_t breed_p[2] = {kSheepBreed, kWolfBreed};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t chunk = int32_t(blockDim.x) * ITEMS;
    const int32_t lbase = wave * ITEMS * 64 + lane;
    // this member's slot range of each species (the whole model when alone, the
    // launch's balanced bounds in a team); species 1's list follows species 0's
    int32_t lo[2], hi[2];
    if (tm.K == 1) {
        lo[0] = 0;
        hi[0] = v.cap[0];
        lo[1] = 0;
        hi[1] = v.cap[1];
    } else {
        lo[0] = tm.s_bound[tm.r];
        hi[0] = tm.s_bound[tm.r + 1];
        lo[1] = tm.s_bound[kMaxTeam + 1 + tm.r];
        hi[1] = tm.s_bound[kMaxTeam + 1 + tm.r + 1];
    }
    const int32_t list1 = v.cap[0];
    int32_t* my_list = member_list(tm, tm.r);
    // passes A and B visit [lo, eff): every live agent of the range lies below
    // the mark the last step left.  Each wave copies the mark into registers
    // here, after the barrier that ended the last step, and the mark is written
    // again only after every loop of this step (behind the barriers of the
    // reduction that computes it), so every wave runs the same trip counts.
    int32_t eff[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int32_t mk = tm.s_mark[s];
        eff[s] = __builtin_amdgcn_readfirstlane(max(lo[s], min(hi[s], mk)));
    }

    // ---- A: move + claims
    uint32_t live = 0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        for (int32_t c0 = lo[s]; c0 < eff[s]; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < eff[s] ? v.al[s][i] : 0;
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
                uint64_t* cw = claims + 3 * c;
                if (s == 0) {
                    if (v.ready[c] <= int32_t(t))
                        post(cw + 0, tagged_key(tag_hi, sb, skey, i, kSheepGrassKey));
                    if (v.multi)
                        push(cw + 1, i, v.link[0]);
                    else
                        post(cw + 1, tagged_key(tag_hi, sb, skey, i, kSheepPreyKey));
                } else if (v.multi) {
                    push(cw + 2, i, v.link[1]);
                } else {
                    post(cw + 2, tagged_key(tag_hi, sb, skey, i, kWolfEatKey));
                }
            }
        }
    }
    live = block_sum32(live, lds);
    if (!team_sync(tm)) return false;    // every claim of the step is posted

    // ---- multi-prey: wolves of this member take their prey
    if (v.multi) {
        for (int32_t c0 = lo[1]; c0 < eff[1]; c0 += chunk) {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t j = c0 + lbase + k * 64;
                if (j >= eff[1] || v.al[1][j] == 0) continue;
                const int32_t x = v.x[1][j], y = v.y[1][j];
                if (!on_grid(v, x, y)) continue;
                prey_match(v, skey, claims + 3 * (int64_t(y) * v.W + x), j, rd, head);
            }
        }
        if (!team_sync(tm)) return false;   // eaten sheep and wolves' gains are visible
    }

    // ---- B: eat, member-local breeder lists (ascending), free-slot counts
    uint32_t nb_local[2], nf_local[2], nf_below[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        uint32_t base_rank = 0, nfree = 0;
        int32_t* list = my_list + (s ? list1 : 0);
        for (int32_t c0 = lo[s]; c0 < eff[s]; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < eff[s] ? v.al[s][i] : -1;
            }
            bool br[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                br[k] = false;
                if (al[k] == 0) ++nfree;
                if (al[k] <= 0) continue;
                const int32_t i = c0 + lbase + k * 64;
                const int32_t x = v.x[s][i], y = v.y[s][i];
                int32_t e = v.e[s][i];
                bool eaten = false;
                if (on_grid(v, x, y)) {
                    const int64_t c = int64_t(y) * v.W + x;
                    const uint64_t* cw = claims + 3 * c;
                    if (s == 0) {
                        if (rd(cw + 0) == tagged_key(tag_hi, sb, skey, i, kSheepGrassKey)) {
                            e += v.gain[0];
                            v.e[0][i] = e;
                            v.ready[c] = int32_t(t) + v.R;
                        }
                        if (v.multi) {
                            eaten = al[k] == 2;   // taken by a wolf of its cell
                        } else if (claimed(rd(cw + 2)) &&
                                   rd(cw + 1) == tagged_key(tag_hi, sb, skey, i, kSheepPreyKey)) {
                            v.al[0][i] = 2;   // eaten: dead, its claims still to be reset
                            eaten = true;
                        }
                        nfree += eaten ? 1u : 0u;
                    } else if (!v.multi && claimed(rd(cw + 1)) &&
                               rd(cw + 2) == tagged_key(tag_hi, sb, skey, i, kWolfEatKey)) {
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
                if (br[k]) list[base_rank + rank[k]] = c0 + lbase + k * 64;
            base_rank += tot;
        }
        nb_local[s] = base_rank;
        nf_below[s] = block_sum32(nfree, lds);
        nf_local[s] = nf_below[s] + uint32_t(hi[s] - eff[s]);   // slots past the mark are free
    }
    // s_pre: [0, K] breeder prefix of species 0, [K+1, 2K+1] of species 1,
    // then the free-slot prefix of this member for both species and the live total
    int32_t* bpre0 = tm.s_pre;
    int32_t* bpre1 = tm.s_pre + tm.K + 1;
    int32_t* fpre = tm.s_pre + 2 * (tm.K + 1);
    if (tm.K == 1) {
        if (threadIdx.x == 0) {
            bpre0[0] = 0;
            bpre0[1] = int32_t(nb_local[0]);
            bpre1[0] = 0;
            bpre1[1] = int32_t(nb_local[1]);
            fpre[0] = 0;
            fpre[1] = 0;
            fpre[2] = int32_t(live);
        }
        __syncthreads();
    } else {
        if (threadIdx.x == 0) {
            int32_t* cnt = tm.counts + int64_t(tm.base + 8u * uint32_t(tm.r)) * kCountWords;
            cnt[0] = int32_t(nb_local[0]);
            cnt[1] = int32_t(nb_local[1]);
            cnt[2] = int32_t(nf_local[0]);
            cnt[3] = int32_t(nf_local[1]);
            cnt[4] = int32_t(live);
        }
        if (!team_sync(tm)) return false;   // every member's list and counts are visible
        if (threadIdx.x == 0) {
            int32_t b0 = 0, b1 = 0, f0 = 0, f1 = 0, lv = 0;
            for (int j = 0; j < tm.K; ++j) {
                const int32_t* cnt = tm.counts + int64_t(tm.base + 8u * uint32_t(j)) * kCountWords;
                bpre0[j] = b0;
                bpre1[j] = b1;
                b0 += cnt[0];
                b1 += cnt[1];
                if (j < tm.r) {
                    f0 += cnt[2];
                    f1 += cnt[3];
                }
                lv += cnt[4];
            }
            bpre0[tm.K] = b0;
            bpre1[tm.K] = b1;
            fpre[0] = f0;
            fpre[1] = f1;
            fpre[2] = lv;
        }
        __syncthreads();
    }
    *live_out = uint32_t(fpre[2]);

    int32_t top[2] = {0, 0};   // 1 + the highest slot this thread leaves alive
    // ---- C: breed into free slots, starve; re-arm the claims (every read of
    // the table in B is behind the barrier above): LOCAL every step, else at
    // the end of a tag period and at the last step of the launch, each team
    // member its share of the table
    if constexpr (LOCAL) {
        local_fill(claims, 3 * v.W * v.H);
    } else if (phase == v.period - 1 || last) {
        const int64_t words = 3 * int64_t(v.W) * v.H;
        const int64_t w0 = words * tm.r / tm.K, w1 = words * (tm.r + 1) / tm.K;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += blockDim.x) rearm(claims + w);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int32_t* bpre = s ? bpre1 : bpre0;
        const uint32_t nb = uint32_t(bpre[tm.K]);
        const int32_t list_off = s ? list1 : 0;
        uint32_t base_rank = uint32_t(fpre[s]);
        // births into this range: its free slots of model rank below nb; the
        // ones past the free slots below the mark take [eff, eff + above)
        const int64_t into = min(max(int64_t(nb) - int64_t(fpre[s]), int64_t(0)),
                                 int64_t(nf_local[s]));
        const int32_t above = int32_t(max(into - int64_t(nf_below[s]), int64_t(0)));
        const int32_t end = __builtin_amdgcn_readfirstlane(min(hi[s], eff[s] + above));
        for (int32_t c0 = lo[s]; c0 < end; c0 += chunk) {
            int32_t al[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                al[k] = i < end ? v.al[s][i] : 1;
            }
            bool fr[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                fr[k] = i < end && (al[k] == 0 || al[k] == 2);
            }
            uint32_t rank[ITEMS];
            const uint32_t tot = chunk_rank<ITEMS>(fr, rank, lds);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int32_t i = c0 + lbase + k * 64;
                const uint32_t j = base_rank + rank[k];
                if (fr[k] && j < nb) {
                    int q = 0;   // the member whose list holds breeder j
                    while (q + 1 < tm.K && uint32_t(bpre[q + 1]) <= j) ++q;
                    const int32_t p = member_list(tm, q)[list_off + int32_t(j) - bpre[q]];
                    const int32_t ep = v.e[s][p];
                    const int32_t ec = ep >> 1;
                    v.x[s][i] = v.x[s][p];
                    v.y[s][i] = v.y[s][p];
                    v.e[s][i] = ec;
                    v.e[s][p] = ep - ec;
                    v.al[s][i] = 1;
                    top[s] = i + 1;
                } else if (i < end) {
                    // a breeder's energy stays positive, so no slot read by a child dies
                    // here, whichever of its two values another member's child leaves
                    if (al[k] == 2 || (al[k] != 0 && v.e[s][i] < 0))
                        v.al[s][i] = 0;
                    else if (al[k] != 0)
                        top[s] = i + 1;
                }
            }
            base_rank += tot;
        }
    }
    // the next step's marks (every wave is past its loops: the reduction's
    // first barrier comes after them)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int32_t m = block_max32(top[s], lds);
        if (threadIdx.x == 0) tm.s_mark[s] = m;
    }
    // births, deaths and re-armed claims are visible to the next step
    return team_sync(tm);
}

__device__ ModelView view_of(const BatchArgs& a, const abm_model_desc* d) {
    ModelView v;
    v.W = d->W;
    v.H = d->H;
    v.R = d->R;
    v.gain[0] = d->gain_s;
    v.gain[1] = d->gain_w;
    v.T[0] = d->T_s;
    v.T[1] = d->T_w;
    v.seed = d->seed;
    v.multi = d->multi_prey != 0;
    // claim keys: slots below 2^sb (caps are at most 2^30), a tag of up to
    // kTagBits bits above the 32-bit draw; tags tag_top down to 1 (0 alone when
    // one tag bit is left, re-arming every step); all-ones has a tag no step uses
    const int64_t max_cap = d->cap_s > d->cap_w ? d->cap_s : d->cap_w;
    uint32_t sb = 1;
    while (sb < 31 && (int64_t(1) << sb) < max_cap) ++sb;
    const uint32_t tag_bits = 32 - sb < kTagBits ? 32 - sb : kTagBits;
    const uint64_t t_max = (uint64_t(1) << tag_bits) - 1;
    v.sb = sb;
    v.tag_top = t_max > 1 ? t_max - 1 : 0;
    v.period = t_max > 1 ? uint32_t(t_max - 1) : 1u;
    v.tag_mask = ~uint64_t(0) << (32 + sb);
    v.link[0] = a.link_s ? a.link_s + d->sheep_off : nullptr;
    v.link[1] = a.link_w ? a.link_w + d->wolf_off : nullptr;
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
    return v;
}

// Member ranges of a team for one launch, balanced by work: the members count
// the live agents of every 4096-slot block of their share of the model, and
// then every member computes the same bounds from the block costs (a slot
// costs 1 and a live agent 3 more: a dead slot is one coalesced load per pass,
// a live agent a draw, several gathers and atomics).  The live agents sit in
// the lowest slots (children take the lowest free slots), so equal slot
// counts would leave a few members with all the work.  False if a team barrier
// failed.
constexpr int32_t kBalBlock = 4096;

template <int ITEMS>
__device__ bool balance_team(const ModelView& v, Team& tm, uint32_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t chunk = int32_t(blockDim.x) * ITEMS;
    const int32_t lbase = wave * ITEMS * 64 + lane;
    int32_t* cost = member_list(tm, 0);   // lists are idle until the first step
    int32_t nblk[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) nblk[s] = (v.cap[s] + kBalBlock - 1) / kBalBlock;
    // live agents per block, each member over its share of the blocks
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int32_t per = (nblk[s] + tm.K - 1) / tm.K;
        const int32_t b0 = min(nblk[s], tm.r * per), b1 = min(nblk[s], b0 + per);
        for (int32_t blk = b0; blk < b1; ++blk) {
            const int32_t lo = blk * kBalBlock, hi = min(v.cap[s], lo + kBalBlock);
            uint32_t live = 0;
            for (int32_t c0 = lo; c0 < hi; c0 += chunk) {
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const int32_t i = c0 + lbase + k * 64;
                    live += (i < hi && v.al[s][i] != 0) ? 1u : 0u;
                }
            }
            live = block_sum32(live, lds);
            if (threadIdx.x == 0) cost[(s ? nblk[0] : 0) + blk] = (hi - lo) + 3 * int32_t(live);
        }
    }
    if (!team_sync(tm)) return false;
    // bounds: member r starts at the first block whose cost prefix reaches
    // r / K of the total
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int32_t* c = cost + (s ? nblk[0] : 0);
        int32_t* bound = tm.s_bound + s * (kMaxTeam + 1);
        uint32_t total = 0;
        for (int32_t b = threadIdx.x; b < nblk[s]; b += blockDim.x) total += uint32_t(c[b]);
        total = block_sum32(total, lds);
        if (threadIdx.x <= tm.K) bound[threadIdx.x] = threadIdx.x == 0 ? 0 : v.cap[s];
        __syncthreads();
        uint32_t carry = 0;
        for (int32_t b0 = 0; b0 < nblk[s]; b0 += int32_t(blockDim.x)) {
            const int32_t b = b0 + int32_t(threadIdx.x);
            const uint32_t mine = b < nblk[s] ? uint32_t(c[b]) : 0u;
            uint32_t incl;
            const uint32_t chunk_total = block_incl_scan32(mine, lds, &incl);
            const uint32_t before = carry + incl - mine;
            // the block where the prefix first reaches r * total / K
            for (int r = 1; r < tm.K; ++r) {
                const uint64_t target = (uint64_t(total) * uint32_t(r) + uint32_t(tm.K) - 1) /
                                        uint32_t(tm.K);
                if (b < nblk[s] && before < target && target <= before + mine)
                    bound[r] = min(v.cap[s], (b + 1) * kBalBlock);
            }
            carry += chunk_total;
        }
        __syncthreads();
        // bounds must not decrease (empty members keep a zero-width range)
        if (threadIdx.x == 0)
            for (int r = 1; r <= tm.K; ++r) bound[r] = max(bound[r], bound[r - 1]);
        __syncthreads();
    }
    return true;
}

// Runs model m's pending steps (at most max_steps) with team tm; member 0
// updates the descriptor.  A model of a single workgroup (no team) keeps its
// claim table in LDS when its 3 W H words fit in a.lds_words.  False if a
// team barrier failed.
template <int ITEMS>
__device__ bool run_model(const BatchArgs& a, int32_t m, Team& tm, uint32_t* lds) {
    abm_model_desc* d = a.models + m;
    if (d->cap_s + d->cap_w > a.scratch_stride || (d->multi_prey && !(a.link_s && a.link_w))) {
        // the descriptor does not fit the breeder list (max_cap too small), or
        // a multi-prey model has no list links: leave the model untouched and
        // report it
        if (threadIdx.x == 0 && tm.r == 0) st_agent(tm.err, 1ull);
        return true;
    }
    const ModelView v = view_of(a, d);
    const int32_t t0 = d->step;
    int32_t t1 = d->steps_target;
    if (t1 - t0 > a.max_steps) t1 = t0 + a.max_steps;
    if (tm.K > 1 && t1 > t0 && !balance_team<ITEMS>(v, tm, lds)) return false;
    uint64_t updates = 0;
    const bool local = tm.K == 1 && 3 * int64_t(v.W) * v.H <= a.lds_words;
    if (local && t1 > t0) local_fill(local_claims(), 3 * v.W * v.H);
    // no mark yet: the first step of the launch visits the whole range
    if (threadIdx.x == 0) {
        tm.s_mark[0] = INT32_MAX;
        tm.s_mark[1] = INT32_MAX;
    }
    __syncthreads();
    for (int32_t t = t0; t < t1; ++t) {
        uint32_t live;
        const bool last = t + 1 == t1;
        const bool ok =
            local ? model_step<ITEMS, true>(v, uint32_t(t), uint32_t(t0), last, tm, lds, &live)
                  : model_step<ITEMS, false>(v, uint32_t(t), uint32_t(t0), last, tm, lds, &live);
        if (!ok) return false;
        updates += live;
    }
    if (threadIdx.x == 0 && tm.r == 0 && t1 > t0) {
        d->step = t1;
        d->updates += int64_t(updates);
    }
    return true;
}

// Workgroups [0, team_wgs) form teams of team_k members and take models
// order[0, n_team) from queue 0; once that queue is empty they work alone like
// the other workgroups, which take order[n_team, n_models) from queue 1.
template <int ITEMS>
__global__ __launch_bounds__(1024) void k_batched_run(BatchArgs a) {
    __shared__ uint32_t lds[16];
    __shared__ int32_t s_pre[2 * (kMaxTeam + 1) + 3];
    __shared__ int32_t s_ok, s_model;
    __shared__ int32_t s_bound[2 * (kMaxTeam + 1)];
    __shared__ int32_t s_mark[2];
    const uint32_t b = blockIdx.x;
    Team tm;
    tm.gen = 0;
    tm.scratch = a.scratch;
    tm.stride = a.scratch_stride;
    tm.counts = a.team_counts;
    tm.err = a.err;
    tm.s_pre = s_pre;
    tm.s_ok = &s_ok;
    tm.s_bound = s_bound;
    tm.s_mark = s_mark;
    if (b < a.team_wgs) {
        const uint32_t xcd = b % 8, idx = b / 8;
        const uint32_t team = xcd + 8 * (idx / a.team_k);
        tm.K = int(a.team_k);
        tm.r = int(idx % a.team_k);
        tm.base = xcd + 8 * (idx - uint32_t(tm.r));
        tm.ctr = a.team_ctr + team;
        int32_t* mailbox = a.team_mail + team;
        for (;;) {
            if (threadIdx.x == 0 && tm.r == 0) {
                const uint32_t q = atomicAdd(a.queue + 0, 1u);
                __hip_atomic_store(mailbox, q < uint32_t(a.n_team) ? a.order[q] : -1,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!team_sync(tm)) return;
            if (threadIdx.x == 0)
                s_model = __hip_atomic_load(mailbox, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // every member has read the mailbox before the leader writes it again
            if (!team_sync(tm)) return;
            const int32_t m = s_model;
            // every wave has read s_model before thread 0 reuses it (the solo
            // loop below writes it straight away)
            __syncthreads();
            if (m < 0) break;
            if (!run_model<ITEMS>(a, m, tm, lds)) return;
        }
    }
    tm.K = 1;
    tm.r = 0;
    tm.base = b;
    tm.ctr = nullptr;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t q = uint32_t(a.n_team) + atomicAdd(a.queue + 1, 1u);
            s_model = q < uint32_t(a.n_models) ? a.order[q] : -1;
        }
        __syncthreads();
        const int32_t m = s_model;
        __syncthreads();
        if (m < 0) break;
        run_model<ITEMS>(a, m, tm, lds);
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

// Clears the queue counters and the team barrier counters of a run.
__global__ void k_reset_queue(uint32_t* q, uint32_t* team_ctr, int32_t n_teams) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i == 0) *reinterpret_cast<uint64_t*>(q) = 0;
    if (i < n_teams) team_ctr[i] = 0;
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

// Workspace of a batched run: a 256-byte header (queue counters; error word at
// byte 248), the team area (barrier counter and model mailbox per team, member
// counts per workgroup) and one breeder list (2 * max_cap ints) per workgroup.
constexpr int64_t kTeamAreaWords = int64_t(kMaxWorkgroups) * (2 + kCountWords);

extern "C" size_t abm_batched_workspace_bytes(int64_t max_cap, int32_t n_workgroups) {
    if (max_cap < 1 || max_cap > (int64_t(1) << 30) || n_workgroups < 1 ||
        n_workgroups > kMaxWorkgroups)
        return 0;
    return size_t(kHeaderBytes) + size_t(4 * kTeamAreaWords) +
           size_t(n_workgroups) * size_t(2 * max_cap) * 4 + 256;
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

namespace {

const void* run_kernel(int items) {
    return items == 1 ? reinterpret_cast<const void*>(k_batched_run<1>)
         : items == 2 ? reinterpret_cast<const void*>(k_batched_run<2>)
                      : reinterpret_cast<const void*>(k_batched_run<4>);
}

// Launch shape of a run: workgroups resident per CU at `block` threads and
// the dynamic LDS each can hold without lowering that count (the CU's LDS
// shared among them, less the kernel's static LDS; at most the per-workgroup
// limit).  False with the error set if a query fails.
bool run_shape(int items, int block, int* n_cu, int* per_cu, int64_t* lds_bytes) {
    const void* kern = run_kernel(items);
    int dev = 0, lds_cu = 0, lds_block = 0;
    hipFuncAttributes fa;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        hipFuncGetAttributes(&fa, kern) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, block, 0) != hipSuccess) {
        set_error("predation_run_batched: device query failed");
        return false;
    }
    if (*per_cu < 1) *per_cu = 1;
    int64_t dyn = int64_t(lds_cu) / *per_cu - int64_t(fa.sharedSizeBytes);
    if (dyn > int64_t(lds_block) - int64_t(fa.sharedSizeBytes))
        dyn = int64_t(lds_block) - int64_t(fa.sharedSizeBytes);
    dyn = dyn > 0 ? dyn / 1024 * 1024 : 0;
    // allocation granularity: step down until the occupancy is unchanged
    for (; dyn > 0; dyn -= 1024) {
        int with = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&with, kern, block, size_t(dyn)) !=
            hipSuccess) {
            set_error("predation_run_batched: occupancy query failed");
            return false;
        }
        if (with >= *per_cu) break;
    }
    *lds_bytes = dyn;
    return true;
}

}  // namespace

extern "C" int64_t abm_batched_lds_cells(int32_t block_threads, int32_t items) {
    if (block_threads < 256 || block_threads > 1024 || (block_threads & 63)) return 0;
    if (items != 1 && items != 2 && items != 4) return 0;
    if (check_device() != ABM_OK) return 0;
    int n_cu = 0, per_cu = 0;
    int64_t lds_bytes = 0;
    if (!run_shape(items, block_threads, &n_cu, &per_cu, &lds_bytes)) return 0;
    return lds_bytes / 24;
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
    if (items != 1 && items != 2 && items != 4)
        return fail(ABM_E_INVALID, "items must be 1, 2 or 4");
    int n_cu = 0, per_cu = 0;
    int64_t lds_bytes = 0;
    if (!run_shape(items, block, &n_cu, &per_cu, &lds_bytes)) return ABM_E_HIP;
    if (tune && tune->global_claims) lds_bytes = 0;
    int resident = n_cu * per_cu;
    if (tune && tune->workgroups > 0 && tune->workgroups < resident) resident = tune->workgroups;
    if (resident > kMaxWorkgroups) resident = kMaxWorkgroups;
    // teams: order[0, n_team) is run by teams of K workgroups, formed from the
    // first team_wgs workgroups (a multiple of 8 K)
    const int K = tune && tune->team_size > 1 ? tune->team_size : 1;
    int n_team = K > 1 && tune ? tune->team_models : 0;
    if (K > kMaxTeam) return fail(ABM_E_INVALID, "team_size must be at most 16");
    if (n_team < 0 || n_team > b->n_models)
        return fail(ABM_E_INVALID, "team_models must be in [0, n_models]");
    int team_wgs = 0;
    if (n_team > 0) {
        const int unit = 8 * K;
        const int fit = resident / unit * unit;
        if (fit == 0) {
            set_error("teams of %d need %d resident workgroups, %d are available", K, unit,
                      resident);
            return ABM_E_INVALID;
        }
        team_wgs = tune->team_workgroups > 0 ? tune->team_workgroups
                                             : (n_team * K + unit - 1) / unit * unit;
        if (team_wgs % unit != 0)
            return fail(ABM_E_INVALID, "team_workgroups must be a multiple of 8 * team_size");
        if (team_wgs > fit) team_wgs = fit;
    }
    int grid = resident - team_wgs;
    if (grid > b->n_models - n_team) grid = b->n_models - n_team;
    grid += team_wgs;
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
    a.link_s = b->link_s;
    a.link_w = b->link_w;
    char* base = static_cast<char*>(ws);
    a.queue = reinterpret_cast<uint32_t*>(base);
    a.err = reinterpret_cast<uint64_t*>(base + kHeaderBytes - 8);
    a.team_ctr = reinterpret_cast<uint32_t*>(base + kHeaderBytes);
    a.team_mail = reinterpret_cast<int32_t*>(a.team_ctr + kMaxWorkgroups);
    a.team_counts = a.team_mail + kMaxWorkgroups;
    a.scratch = reinterpret_cast<int32_t*>(base + kHeaderBytes + 4 * kTeamAreaWords);
    a.scratch_stride = 2 * b->max_cap;
    a.n_team = n_team;
    a.lds_words = int32_t(lds_bytes / 8);
    a.team_k = uint32_t(K);
    a.team_wgs = uint32_t(team_wgs);
    const int n_teams = team_wgs / K;
    hipLaunchKernelGGL(k_reset_queue, dim3((n_teams + 255) / 256 + 1), dim3(256), 0, st, a.queue,
                       a.team_ctr, n_teams);
    const size_t dyn = size_t(lds_bytes);
    switch (items) {
        case 1: hipLaunchKernelGGL(k_batched_run<1>, dim3(grid), dim3(block), dyn, st, a); break;
        case 2: hipLaunchKernelGGL(k_batched_run<2>, dim3(grid), dim3(block), dyn, st, a); break;
        default: hipLaunchKernelGGL(k_batched_run<4>, dim3(grid), dim3(block), dyn, st, a); break;
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
