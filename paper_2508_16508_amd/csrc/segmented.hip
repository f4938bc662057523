// segmented.hip -- batched (segmented) select_update, add_agents,
// remove_agents and resolve_conflicts: many independent collections of
// uneven sizes packed back to back and processed by one launch, each exactly
// as the single-collection call would process it alone (paper Sec. 2: the
// manipulation functions vectorise over Sets; here the Sets may differ in
// size).
//
// Segment m owns slots [slot_off[m], slot_off[m+1]) and records
// [rec_off[m], rec_off[m+1]) (device offset arrays, non-decreasing).  Tiles of
// 8192 slots run over the packed range regardless of segment boundaries, so
// uneven segments are load-balanced for free; ranks restart at every segment
// start through a segmented scan.  Its combine on (flag, count) pairs --
// (f1, c1) + (f2, c2) = (f1 | f2, f2 ? c2 : c1 + c2), flag = "a segment starts
// here" -- is associative but not commutative, so every level (lane, wave,
// block, tile hierarchy) combines strictly in slot order.  A pair is packed
// into the 32-bit status value: bit 31 flag, bits 30..0 count.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
constexpr int kSlotsPerLane = 32;
constexpr int64_t kTile = int64_t(kBlock) * kSlotsPerLane;
constexpr uint32_t kSegFlag = 0x80000000u;

__device__ __forceinline__ uint32_t seg_combine(uint32_t a, uint32_t b) {
    return (b & kSegFlag) ? (a & kSegFlag) | b : (a & kSegFlag) | ((a + b) & ~kSegFlag);
}

// Inclusive ordered scan over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_seg_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v = seg_combine(o, v);
    }
    return v;
}

// Segmented version of hier_prefix (scan.hpp): the exclusive ordered
// combination of the tile values of one chain, for tile t of T.
__device__ __forceinline__ uint32_t hier_prefix_seg(uint64_t* chain, uint64_t* err, uint32_t t,
                                                    uint32_t T, uint32_t epoch, uint32_t value,
                                                    uint32_t* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t part = 0;
    if (wave < kLevels) {
        uint64_t* level = chain;
        uint32_t n = T;
        for (int l = 0; l < wave; ++l) {
            level += n;
            n = (n + 63) >> 6;
        }
        const uint32_t g = t >> (6 * wave);
        const uint32_t d = g & 63u;
        const uint32_t pspan = 1u << (6 * (wave + 1));
        const bool publish = (((t & (pspan - 1)) == pspan - 1) || t == T - 1) && wave + 1 < kLevels;
        if (wave == 0 && lane == 0) st_agent(&level[g], pack_status(epoch, kFlagAgg, value));
        uint32_t v = 0;
        if (lane < d || (lane == d && wave > 0 && publish)) {
            const uint32_t idx = g - d + lane;
            v = static_cast<uint32_t>(poll_status(&level[idx], ld_agent(&level[idx]), epoch, err));
        }
        if (wave == 0 && lane == d) v = value;   // level 0: the tile's own value
        // exclusive part: lanes [0, d); inclusive (for the parent word): [0, d]
        const uint32_t excl_in = wave_seg_scan(lane < d ? v : 0u);
        const uint32_t incl_in = wave_seg_scan(lane <= d ? v : 0u);
        part = __shfl(excl_in, 63, 64);
        const uint32_t incl = __shfl(incl_in, 63, 64);
        if (publish && lane == 0)
            st_agent(&(level + n)[g >> 6], pack_status(epoch, kFlagAgg, incl));
    }
    __syncthreads();
    if (lane == 0) lds[wave] = part;
    __syncthreads();
    // farthest level first: S3 + S2 + S1 + S0
    uint32_t total = 0;
#pragma unroll
    for (int l = kLevels - 1; l >= 0; --l) total = seg_combine(total, lds[l]);
    return total;
}

enum SegMode : int { kSegSelect = 0, kSegAdd = 1, kSegRemove = 2 };

struct SegArgs {
    int32_t* dst[ABM_MAX_ATTRS];
    const int32_t* rec[ABM_MAX_ATTRS];
    const uint8_t* mask;        // select: slot mask; remove: kill mask
    int32_t* alive;             // add / remove
    const int64_t* slot_off;    // n_seg + 1
    const int64_t* rec_off;     // n_seg + 1 (select, add)
    int64_t* d_applied;         // per segment: applied / added / removed
    int64_t* d_dropped;         // per segment or null
    int64_t n;                  // packed slots
    uint64_t* status;
    EpochArg epoch;
    uint32_t ntiles;
    int32_t n_seg;
    int32_t n_attrs;
};

// Largest m with slot_off[m] <= s < slot_off[m + 1] (skipping empty segments).
__device__ __forceinline__ int32_t segment_of(const int64_t* off, int32_t n_seg, int64_t s) {
    int32_t lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_segmented(SegArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = blockIdx.x;
    const uint32_t epoch = read_epoch(a.epoch);
    const int64_t first = int64_t(tile) * kTile + int64_t(threadIdx.x) * kSlotsPerLane;
    const int64_t last = first + kSlotsPerLane < a.n ? first + kSlotsPerLane : a.n;

    // selection bits and segment-start bits of this lane's slots
    uint32_t sel = 0, starts = 0;
    int32_t m0 = 0;
    if (first < a.n) {
        for (int k = 0; k < last - first; ++k) {
            const int64_t s = first + k;
            bool f;
            if (MODE == kSegAdd)
                f = a.alive[s] == 0;
            else if (MODE == kSegRemove)
                f = a.mask[s] != 0 && a.alive[s] != 0;
            else
                f = a.mask[s] != 0;
            sel |= uint32_t(f) << k;
        }
        m0 = segment_of(a.slot_off, a.n_seg, first);
        if (a.slot_off[m0] == first) starts |= 1u;
        for (int32_t m = m0 + 1; m < a.n_seg; ++m) {
            const int64_t st = a.slot_off[m];
            if (st >= last) break;
            if (st < a.slot_off[m + 1]) starts |= 1u << (st - first);   // non-empty segment
        }
    }
    // the lane's (flag, count): selected slots after its last segment start
    uint32_t lane_val;
    if (starts) {
        const int hb = 31 - __clz(starts);
        lane_val = kSegFlag | __popc(sel >> hb);
    } else {
        lane_val = __popc(sel);
    }
    // block scan in lane order, then the tile prefix
    const uint32_t incl = wave_seg_scan(lane_val);
    uint32_t excl_w = __shfl_up(incl, 1, 64);
    if (lane == 0) excl_w = 0;
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t v = lds[w];
        if (w < wave) before = seg_combine(before, v);
        total = seg_combine(total, v);
    }
    const uint32_t tile_excl =
        hier_prefix_seg(a.status, a.status - 1, tile, a.ntiles, epoch, total, lds);
    const uint32_t lane_excl = seg_combine(seg_combine(tile_excl, before), excl_w);

    if (first >= a.n) return;
    // walk the lane's slots in order
    uint32_t running = lane_excl & ~kSegFlag;
    int32_t m = m0;
    int64_t seg_end = a.slot_off[m + 1];
    int64_t rbase = (MODE == kSegRemove) ? 0 : a.rec_off[m];
    int64_t q = (MODE == kSegRemove) ? 0 : a.rec_off[m + 1] - rbase;
    for (int k = 0; k < last - first; ++k) {
        const int64_t s = first + k;
        if ((starts >> k) & 1u) {
            // a new segment starts at s (skip empty segments in between)
            m = segment_of(a.slot_off, a.n_seg, s);
            seg_end = a.slot_off[m + 1];
            if (MODE != kSegRemove) {
                rbase = a.rec_off[m];
                q = a.rec_off[m + 1] - rbase;
            }
            running = 0;
        }
        if ((sel >> k) & 1u) {
            const uint32_t j = running++;
            if (MODE == kSegRemove) {
                a.alive[s] = 0;
            } else if (int64_t(j) < q) {
                const int64_t src = rbase + j;
                for (int at = 0; at < a.n_attrs; ++at) a.dst[at][s] = a.rec[at][src];
                if (MODE == kSegAdd) a.alive[s] = 1;
            }
        }
        if (s == seg_end - 1) {
            const int64_t p = running;
            if (MODE == kSegRemove) {
                a.d_applied[m] = p;
            } else {
                const int64_t r = p < q ? p : q;
                a.d_applied[m] = r;
                if (a.d_dropped) a.d_dropped[m] = q - r;
            }
        }
    }
}

// Counts of every segment as if empty (overwritten for non-empty segments).
__global__ void k_seg_counts(const int64_t* rec_off, int32_t n_seg, int64_t* applied,
                             int64_t* dropped) {
    const int32_t m = blockIdx.x * 256 + threadIdx.x;
    if (m >= n_seg) return;
    applied[m] = 0;
    if (dropped) dropped[m] = rec_off ? rec_off[m + 1] - rec_off[m] : 0;
}

// ------------------------------------------------------------------ resolve
struct SegResolveArgs {
    const int64_t* claim_off;   // n_seg + 1
    const int64_t* target_off;  // n_seg + 1
    const int32_t* target;      // segment-local target per claim
    const uint32_t* prio;
    const uint8_t* active;
    uint64_t* best;             // packed over all targets
    int32_t* winner;            // packed: segment-local claim index or -1
    uint8_t* won;
    int64_t n_claims, n_targets;
    int32_t n_seg;
};

__device__ __forceinline__ bool seg_claim(const SegResolveArgs& a, int64_t c, int64_t& gt,
                                          uint64_t& key) {
    const int32_t m = segment_of(a.claim_off, a.n_seg, c);
    const int32_t t = a.target[c];
    const int64_t nt = a.target_off[m + 1] - a.target_off[m];
    if ((a.active && a.active[c] == 0) || t < 0 || int64_t(t) >= nt) return false;
    gt = a.target_off[m] + t;
    key = (uint64_t(a.prio[c]) << 32) | uint32_t(c - a.claim_off[m]);
    return true;
}

__global__ __launch_bounds__(256) void k_seg_reset(uint64_t* best, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) best[i] = ~0ull;
}

__global__ __launch_bounds__(256) void k_seg_claim(SegResolveArgs a) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= a.n_claims) return;
    int64_t gt;
    uint64_t key;
    if (seg_claim(a, c, gt, key))
        atomicMin(reinterpret_cast<unsigned long long*>(a.best + gt),
                  static_cast<unsigned long long>(key));
}

__global__ __launch_bounds__(256) void k_seg_readback(SegResolveArgs a) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < a.n_claims) {
        int64_t gt;
        uint64_t key;
        a.won[i] = seg_claim(a, i, gt, key) && a.best[gt] == key ? 1 : 0;
    }
    if (i < a.n_targets) {
        const uint64_t b = a.best[i];
        a.winner[i] = b == ~0ull ? -1 : int32_t(uint32_t(b));
    }
}

int check_seg_soa(const abm_soa* s, bool attrs, bool alive) {
    if (!s) return fail(ABM_E_INVALID, "collection is NULL");
    if (s->capacity < 0 || s->capacity > kMaxIndex)
        return fail(ABM_E_INVALID, "capacity must be in [0, 2^31)");
    if (attrs) {
        if (s->n_attrs < 1 || s->n_attrs > ABM_MAX_ATTRS)
            return fail(ABM_E_INVALID, "n_attrs must be in [1, 16]");
        if (s->capacity > 0)
            for (int a = 0; a < s->n_attrs; ++a)
                if (!s->attr[a]) return fail(ABM_E_INVALID, "attribute pointer is NULL");
    }
    if (alive && s->capacity > 0 && !s->alive) return fail(ABM_E_INVALID, "alive array is required");
    return ABM_OK;
}

int launch_segmented(int mode, int32_t n_seg, const abm_soa* dst, const int64_t* slot_off,
                     const uint8_t* mask, const abm_records* rec, const int64_t* rec_off,
                     int64_t* applied, int64_t* dropped, void* ws, size_t ws_bytes,
                     void* stream) {
    if (n_seg < 0) return fail(ABM_E_INVALID, "n_segments must be >= 0");
    if (n_seg > 0 && (!slot_off || !applied)) return fail(ABM_E_INVALID, "offsets or counts are NULL");
    if (mode != kSegRemove && n_seg > 0 && !rec_off) return fail(ABM_E_INVALID, "rec_off is NULL");
    int rc = check_seg_soa(dst, mode != kSegRemove, mode != kSegSelect);
    if (rc != ABM_OK) return rc;
    if (mode != kSegRemove) {
        if (!rec || rec->n_attrs != dst->n_attrs)
            return fail(ABM_E_INVALID, "record and slot attribute counts differ");
        if (rec->count < 0 || rec->count > kMaxIndex)
            return fail(ABM_E_INVALID, "record count must be in [0, 2^31)");
    }
    if (mode != kSegAdd && dst->capacity > 0 && !mask) return fail(ABM_E_INVALID, "mask is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    if (n_seg == 0) return ABM_OK;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_seg_counts, dim3(tiles_for(n_seg, 256)), dim3(256), 0, st,
                       mode == kSegRemove ? nullptr : rec_off, n_seg, applied, dropped);
    if (dst->capacity == 0) return launch_status("segmented");
    rc = check_ws(ws, ws_bytes, dst->capacity);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, dst->capacity);
    SegArgs a = {};
    if (mode != kSegRemove)
        for (int i = 0; i < dst->n_attrs; ++i) {
            a.dst[i] = dst->attr[i];
            a.rec[i] = rec->attr[i];
        }
    a.mask = mask;
    a.alive = dst->alive;
    a.slot_off = slot_off;
    a.rec_off = rec_off;
    a.d_applied = applied;
    a.d_dropped = dropped;
    a.n = dst->capacity;
    a.status = w.status;
    a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
    a.n_seg = n_seg;
    a.n_attrs = mode == kSegRemove ? 0 : dst->n_attrs;
    rc = next_epoch(w, st, &a.epoch);
    if (rc != ABM_OK) return rc;
    const dim3 grid(a.ntiles), block(kBlock);
    if (mode == kSegSelect)
        hipLaunchKernelGGL(k_segmented<kSegSelect>, grid, block, 0, st, a);
    else if (mode == kSegAdd)
        hipLaunchKernelGGL(k_segmented<kSegAdd>, grid, block, 0, st, a);
    else
        hipLaunchKernelGGL(k_segmented<kSegRemove>, grid, block, 0, st, a);
    return launch_status("segmented");
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_select_update_batched(int32_t n_segments, const abm_soa* dst,
                                         const int64_t* slot_off, const uint8_t* sel_mask,
                                         const abm_records* upd, const int64_t* rec_off,
                                         int64_t* d_applied, int64_t* d_dropped, void* ws,
                                         size_t ws_bytes, void* stream) {
    return launch_segmented(kSegSelect, n_segments, dst, slot_off, sel_mask, upd, rec_off,
                            d_applied, d_dropped, ws, ws_bytes, stream);
}

extern "C" int abm_add_agents_batched(int32_t n_segments, const abm_soa* dst,
                                      const int64_t* slot_off, const abm_records* newborn,
                                      const int64_t* rec_off, int64_t* d_added,
                                      int64_t* d_dropped, void* ws, size_t ws_bytes,
                                      void* stream) {
    return launch_segmented(kSegAdd, n_segments, dst, slot_off, nullptr, newborn, rec_off,
                            d_added, d_dropped, ws, ws_bytes, stream);
}

extern "C" int abm_remove_agents_batched(int32_t n_segments, const abm_soa* dst,
                                         const int64_t* slot_off, const uint8_t* kill_mask,
                                         int64_t* d_removed, void* ws, size_t ws_bytes,
                                         void* stream) {
    return launch_segmented(kSegRemove, n_segments, dst, slot_off, kill_mask, nullptr, nullptr,
                            d_removed, nullptr, ws, ws_bytes, stream);
}

extern "C" int abm_resolve_conflicts_batched(int32_t n_segments, const int64_t* claim_off,
                                             int64_t n_claims, const int32_t* target,
                                             const uint32_t* prio, const uint8_t* active,
                                             const int64_t* target_off, int64_t n_targets,
                                             uint64_t* best, int32_t* winner, uint8_t* won,
                                             void* stream) {
    if (n_segments < 0) return fail(ABM_E_INVALID, "n_segments must be >= 0");
    if (n_claims < 0 || n_claims > kMaxIndex || n_targets < 0 || n_targets > kMaxIndex)
        return fail(ABM_E_INVALID, "n_claims and n_targets must be in [0, 2^31)");
    if (n_segments > 0 && (!claim_off || !target_off))
        return fail(ABM_E_INVALID, "offsets are NULL");
    if (n_claims > 0 && (!target || !prio || !won)) return fail(ABM_E_INVALID, "claim array is NULL");
    if (n_targets > 0 && (!best || !winner)) return fail(ABM_E_INVALID, "best or winner is NULL");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    if (n_segments == 0) return ABM_OK;
    hipStream_t st = as_stream(stream);
    SegResolveArgs a;
    a.claim_off = claim_off;
    a.target_off = target_off;
    a.target = target;
    a.prio = prio;
    a.active = active;
    a.best = best;
    a.winner = winner;
    a.won = won;
    a.n_claims = n_claims;
    a.n_targets = n_targets;
    a.n_seg = n_segments;
    if (n_targets > 0)
        hipLaunchKernelGGL(k_seg_reset, dim3(tiles_for(n_targets, 256)), dim3(256), 0, st, best,
                           n_targets);
    if (n_claims > 0 && n_targets > 0)
        hipLaunchKernelGGL(k_seg_claim, dim3(tiles_for(n_claims, 256)), dim3(256), 0, st, a);
    const int64_t m = n_claims > n_targets ? n_claims : n_targets;
    if (m > 0)
        hipLaunchKernelGGL(k_seg_readback, dim3(tiles_for(m, 256)), dim3(256), 0, st, a);
    return launch_status("resolve_conflicts_batched");
}
