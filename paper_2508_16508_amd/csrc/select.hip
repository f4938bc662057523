// select.hip -- abm_select_update, abm_add_agents, abm_select_indices.
//
// One single-pass kernel per call: each tile ranks its selected slots (wave
// ballot + mbcnt, LDS scan of wave totals, decoupled look-back), then the
// selected slot of rank j < q receives record j.  The rank *is* the index of
// the matching record, so this is the O(n) counterpart of the paper's
// Rank-Match (Sec. 4, Alg. 1): no n x m candidate matrix or argmax is built.
//
// Writing the records.  HBM3E keeps ECC per 32-byte sector and has no byte
// mask, so a store that covers part of a sector makes the memory read the
// sector, merge and write it back -- and those read-modify-writes, issued in
// random order, cost far more than streaming the same bytes.  The records are
// therefore merged on the GPU: the tile walks its slots in 16-byte chunks with
// consecutive threads on consecutive chunks, and every 32-byte sector that
// holds a receiving slot is loaded, merged with its records and stored whole
// (a sector whose slots all receive records is not loaded).  Sectors with no
// receiving slot are neither read nor written.  Unselected slots of a touched
// sector are rewritten with the values they hold, so no other writer may touch
// the destination during the call (the same rule as for the selected slots).
#include <hip/hip_runtime.h>

#include <mutex>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
constexpr int kSlotsPerLane = 32;
constexpr int64_t kTile = int64_t(kBlock) * kSlotsPerLane;   // 8192 slots

enum SelMode : int { kSelDense = 0, kSelIndirect = 1, kAddDense = 2, kCompact = 3 };

struct SelArgs {
    int32_t* dst[ABM_MAX_ATTRS];
    const int32_t* rec[ABM_MAX_ATTRS];
    const uint8_t* mask;      // select / compact: slot mask
    int32_t* alive;           // add: free = (alive == 0); placed slots set to 1
    const int32_t* rec_idx;   // indirect: ascending indices of the selected records
    const int64_t* d_q;       // indirect: number of selected records (device)
    int32_t* out_idx;         // compact: ascending selected indices
    int64_t q;                // dense: number of records
    int64_t n;                // slots
    int64_t* d_applied;       // placed records (compact: number selected)
    int64_t* d_dropped;
    uint64_t* status;
    EpochArg epoch;
    uint32_t ntiles;
    int32_t n_attrs;          // padded attribute count (1, 2, 4, 8 or 16)
    int32_t n_true;           // attribute count
    int32_t vec_ok;           // mask / alive allow 16-byte loads
};

// Selection bits of the 32 consecutive slots [first, first + 32): bit k is
// slot first + k.  Two 16-byte loads of the mask (or eight of alive) per lane.
template <int MODE>
__device__ __forceinline__ uint32_t load_bits(const SelArgs& a, int64_t first) {
    uint32_t bits = 0;
    if (a.vec_ok && first + kSlotsPerLane <= a.n) {
        if (MODE == kAddDense) {
            const int4* p = reinterpret_cast<const int4*>(a.alive + first);
            int4 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = p[q];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                bits |= uint32_t(v[q].x == 0) << (4 * q) | uint32_t(v[q].y == 0) << (4 * q + 1) |
                        uint32_t(v[q].z == 0) << (4 * q + 2) | uint32_t(v[q].w == 0) << (4 * q + 3);
        } else {
            const uint4* p = reinterpret_cast<const uint4*>(a.mask + first);
            const uint4 m0 = p[0], m1 = p[1];
            const uint32_t w[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bits |= uint32_t(((w[q] >> (8 * b)) & 0xFFu) != 0u) << (4 * q + b);
        }
    } else {
        for (int k = 0; k < kSlotsPerLane; ++k) {
            const int64_t s = first + k;
            if (s >= a.n) break;
            const bool sel = (MODE == kAddDense) ? a.alive[s] == 0 : a.mask[s] != 0;
            bits |= uint32_t(sel) << k;
        }
    }
    return bits;
}

// The scatter of k_select: the tile-local offsets of the selected slots sit in
// pos[] in rank order, and consecutive threads walk those rank positions, so
// the reads of records j, j+1, ... are contiguous and every load/store batch
// is branch-free.  Two rank positions per thread and iteration (up to 32
// loads in flight).  When the second position is past the end it aliases the
// first: the same value goes to the same slot twice, which keeps the stores
// unconditional.
template <int MODE, int NA>
__device__ __forceinline__ void scatter_tile(const SelArgs& a, const uint16_t* pos, int64_t tbase,
                                             uint32_t tile_excl, uint32_t lim) {
    for (uint32_t p0 = threadIdx.x; p0 < lim; p0 += 2 * kBlock) {
        const uint32_t p1 = p0 + kBlock;
        const bool has1 = p1 < lim;
        const int64_t j0 = int64_t(tile_excl) + p0;
        const int64_t j1 = int64_t(tile_excl) + (has1 ? p1 : p0);
        const int64_t s0 = (MODE == kSelIndirect) ? a.rec_idx[j0] : j0;
        const int64_t s1 = (MODE == kSelIndirect) ? a.rec_idx[j1] : j1;
        const int64_t d0 = tbase + pos[p0];
        const int64_t d1 = tbase + pos[has1 ? p1 : p0];
        int32_t v0[NA], v1[NA];
#pragma unroll
        for (int at = 0; at < NA; ++at) {
            v0[at] = a.rec[at][s0];
            v1[at] = a.rec[at][s1];
        }
#pragma unroll
        for (int at = 0; at < NA; ++at) {
            a.dst[at][d0] = v0[at];
            a.dst[at][d1] = v1[at];
        }
        if (MODE == kAddDense) {
            a.alive[d0] = 1;
            a.alive[d1] = 1;
        }
    }
}

// Tile-local offsets of this lane's selected slots (bits, from tile rank r),
// written to pos[] in rank order.
__device__ __forceinline__ void fill_pos(uint16_t* pos, uint32_t bits, uint32_t r) {
    while (bits) {
        const uint32_t k = __ffs(bits) - 1;
        bits &= bits - 1;
        pos[r++] = uint16_t(threadIdx.x * kSlotsPerLane + k);
    }
}

// One tile of 8192 slots per block (a 2^24-slot launch is one round of
// resident blocks).  Phase 1 ranks the tile's selected slots (lane-major: lane
// t owns slots [32 t, 32 t + 32) of the tile) and writes their tile-local
// offsets, in rank order, into LDS.  Phase 2 is scatter_tile.  This kernel
// serves select_indices, and select_update / add_agents on destinations whose
// arrays are not 16-byte aligned.
//
// NA is the attribute count rounded up to 1, 2, 4, 8 or 16; the host repeats
// the last attribute's pointers in the padding entries (the repeated copy
// writes the same value to the same slot).  A compile-time count keeps the
// load and store batches free of branches, so the compiler can overlap them.
template <int MODE, int NA>
__global__ __launch_bounds__(kBlock) void k_select(SelArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint16_t pos[kTile];
    const uint32_t tile = blockIdx.x;
    const uint32_t epoch = read_epoch(a.epoch);
    const int64_t tbase = int64_t(tile) * kTile;
    const int64_t lbase = tbase + int64_t(threadIdx.x) * kSlotsPerLane;
    const uint32_t bits0 = load_bits<MODE>(a, lbase);

    uint32_t r0, total;
    const uint32_t tile_excl = rank_counts<kWaves>(__popc(bits0), &r0, a.status, a.status - 1,
                                                   tile, a.ntiles, epoch, lds, &total);

    if (MODE == kCompact) {
        uint32_t bits = bits0, r = r0;
        while (bits) {
            const uint32_t k = __ffs(bits) - 1;
            bits &= bits - 1;
            a.out_idx[int64_t(tile_excl) + r++] = int32_t(lbase + k);
        }
        if (tile == a.ntiles - 1 && threadIdx.x == 0) *a.d_applied = int64_t(tile_excl) + total;
        return;
    }

    fill_pos(pos, bits0, r0);
    __syncthreads();
    const int64_t q = (MODE == kSelIndirect) ? *a.d_q : a.q;
    const int64_t room = q - int64_t(tile_excl);
    const uint32_t lim = room <= 0 ? 0u : (room < int64_t(total) ? uint32_t(room) : total);
    scatter_tile<MODE, NA>(a, pos, tbase, tile_excl, lim);
    if (tile == a.ntiles - 1 && threadIdx.x == 0) {
        const int64_t p = int64_t(tile_excl) + total;
        const int64_t rr = p < q ? p : q;
        *a.d_applied = rr;
        if (a.d_dropped) *a.d_dropped = q - rr;
    }
}

// Line-list merge.  A lane of the rank phase owns 32 consecutive slots of the
// tile, which are one 128-byte line of every attribute.  The lines holding a
// receiving slot are compacted into a list in LDS; eight consecutive threads
// then take one listed line (thread 8 i + k: chunk k, 16 bytes, of list entry
// i), so a wave covers eight whole lines per instruction.  Each line is
// loaded (a chunk whose four slots all receive is not), merged with its
// records and stored whole; unlisted lines are never visited.
constexpr int kLinesPerPass = 32;     // lines per work item (four chunk rows of a wave)

__device__ __forceinline__ uint32_t low_bits(uint32_t k) { return k >= 32u ? ~0u : (1u << k) - 1u; }

// The `keep` lowest set bits of b.
__device__ __forceinline__ uint32_t lowest_set(uint32_t b, uint32_t keep) {
    uint32_t out = 0;
    for (uint32_t i = 0; i < keep; ++i) {
        out |= b & (0u - b);
        b &= b - 1u;
    }
    return out;
}

// The receiving slots among the selected bits `b` whose first selected slot
// has tile rank `rk`: selected slots of rank < lim.  Ranks grow with the slot,
// so these are the lowest set bits of b.
__device__ __forceinline__ uint32_t receiving(uint32_t b, uint32_t rk, uint32_t lim,
                                              uint32_t total) {
    if (lim >= total) return b;
    const uint32_t nb = __popc(b);
    const uint32_t na = lim > rk ? (lim - rk < nb ? lim - rk : nb) : 0u;
    return na == nb ? b : lowest_set(b, na);
}

// Descriptor of chunk k (slots 4k .. 4k+3) of a listed line with selection
// bits `word` and first tile rank `pre`, packed into one word: the tile rank
// of the chunk's first receiving slot (bits 0-15), its receiving slots (bits
// 16-19, bit j = slot j of the chunk), valid (bit 20).
constexpr uint32_t kValid = 1u << 20, kAll = 0xFu << 16;

__device__ __forceinline__ uint32_t chunk_desc(uint32_t word, uint32_t pre, uint32_t k,
                                               uint32_t lim, uint32_t total) {
    const uint32_t sh = k << 2;
    const uint32_t rk = pre + __popc(word & low_bits(sh));
    const uint32_t ab = receiving((word >> sh) & 0xFu, rk, lim, total);
    return rk | (ab << 16) | kValid;
}

typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int kSkip = int(0x80000000u);     // out-of-range buffer offset: access skipped
constexpr int kRsrcWord3 = 0x00020000;      // raw buffer descriptor, 32-bit data format
// Cache policy of the merge's attribute line loads and stores: non-temporal
// (each line is read and written once per launch).  Measured on the 2^24 x 8
// microbenchmark: 7% less time per step than the default policy (p = 0.5: 247
// against 269 us for select_update, 267 against 297 for add_agents).  The
// records keep the default: several lanes' gathers read each of their lines.
constexpr int kStreamPolicy = 2;            // nt

// One work item of the line-list merge: attribute array `d` (ALIVE: the
// alive array, merged with the constant 1).  The thread handles chunk t mod 8
// of the lines at list entries i0 + j * istride (j < 4; entries past the list
// are skipped): it loads the old values (not for a chunk whose four slots all receive), reads
// the records of the receiving slots into them and stores the chunks whole.
// All accesses are buffer instructions with 32-bit offsets from a per-tile
// base (few registers); an access that is not wanted gets an out-of-range
// offset, which the hardware skips (a skipped load returns 0).
template <int MODE, bool ALIVE>
__device__ __forceinline__ void merge_item(const SelArgs& a, int32_t* d, const int32_t* rec,
                                           int64_t tbase, uint32_t tile_excl, uint32_t lim,
                                           uint32_t total, uint32_t n_lines, uint32_t i0,
                                           uint32_t istride, const uint16_t* list,
                                           const uint32_t* wbits, const uint32_t* wpre) {
    uint32_t dsc[4], off[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t i = i0 + uint32_t(j) * istride;
        const uint32_t k = threadIdx.x & 7u;
        const uint32_t line = i < n_lines ? list[i] : 0u;
        dsc[j] = i < n_lines ? chunk_desc(wbits[line], wpre[line], k, lim, total) : 0u;
        off[j] = (line * 8u + k) * 16u;
    }
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(d + tbase, 0, int(kTile * 4), kRsrcWord3);
    v4i v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool need = (dsc[j] & kValid) && (dsc[j] & kAll) != kAll;
        v[j] = __builtin_amdgcn_raw_buffer_load_b128(rd, need ? int(off[j]) : kSkip, 0,
                                                     kStreamPolicy);
    }
    if (ALIVE) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t ab = (dsc[j] >> 16) & 0xFu;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((ab >> k) & 1u) v[j][k] = 1;
        }
    } else {
        const int32_t* rt = rec + (MODE == kSelIndirect ? 0 : int64_t(tile_excl));
        const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int32_t*>(rt), 0, int(lim * 4u), kRsrcWord3);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t ab = (dsc[j] >> 16) & 0xFu, rk = dsc[j] & 0xFFFFu;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool on = (ab >> k) & 1u;
                const uint32_t r = rk + __popc(ab & low_bits(uint32_t(k)));
                int32_t x;
                if (MODE == kSelIndirect)
                    x = on ? rt[a.rec_idx[int64_t(tile_excl) + r]] : 0;
                else
                    x = __builtin_amdgcn_raw_buffer_load_b32(rr, on ? int(r * 4u) : kSkip, 0, 0);
                if (on) v[j][k] = x;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        __builtin_amdgcn_raw_buffer_store_b128(v[j], rd, (dsc[j] & kValid) ? int(off[j]) : kSkip,
                                               0, kStreamPolicy);
}

// One array of a dense tile: the thread's chunks are list entries 32 j + t / 8
// (j < 8) with descriptors and offsets precomputed in dsc / off; batches of
// four (loads, record reads, stores), `rows` of the eight being in use.
template <int MODE, bool ALIVE>
__device__ __forceinline__ void merge_dense(const SelArgs& a, int32_t* d, const int32_t* rec,
                                            int64_t tbase, uint32_t tile_excl, uint32_t lim,
                                            uint32_t (&dsc)[8], uint32_t (&off)[8], int rows) {
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(d + tbase, 0, int(kTile * 4), kRsrcWord3);
    const int32_t* rt = ALIVE ? nullptr
                              : rec + (MODE == kSelIndirect ? 0 : int64_t(tile_excl));
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(rt), 0, ALIVE ? 0 : int(lim * 4u), kRsrcWord3);
#pragma unroll
    for (int jb = 0; jb < 8; jb += 4) {
        if (jb >= rows) break;
        // the values below are the same for every array; recomputing them per
        // array keeps the compiler from holding all of them in registers
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            asm volatile("" : "+v"(dsc[jb + j]));
            asm volatile("" : "+v"(off[jb + j]));
        }
        v4i v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t dd = dsc[jb + j];
            const bool need = (dd & kValid) && (dd & kAll) != kAll;
            v[j] = __builtin_amdgcn_raw_buffer_load_b128(rd, need ? int(off[jb + j]) : kSkip, 0,
                                                         kStreamPolicy);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t ab = (dsc[jb + j] >> 16) & 0xFu, rk = dsc[jb + j] & 0xFFFFu;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool on = (ab >> k) & 1u;
                int32_t x = 1;
                if (!ALIVE) {
                    const uint32_t r = rk + __popc(ab & low_bits(uint32_t(k)));
                    if (MODE == kSelIndirect)
                        x = on ? rt[a.rec_idx[int64_t(tile_excl) + r]] : 0;
                    else
                        x = __builtin_amdgcn_raw_buffer_load_b32(rr, on ? int(r * 4u) : kSkip,
                                                                 0, 0);
                }
                if (on) v[j][k] = x;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            __builtin_amdgcn_raw_buffer_store_b128(
                v[j], rd, (dsc[jb + j] & kValid) ? int(off[jb + j]) : kSkip, 0, kStreamPolicy);
    }
}

// The listed lines of a full tile, every attribute (and, for add_agents,
// alive = 1 as one more).  A dense tile (more than 96 listed lines) runs the
// arrays one after another with the whole block on each: thread t takes list
// entries 32 j + t / 8 (j < 8, in two batches of four), so the four waves work
// on neighbouring lines of one array.  A sparse tile would then leave each
// wave a chain of one memory round trip per array; instead its work is cut
// into items of (array, 32 listed lines), wave w taking items w, w + 4, ...,
// so its arrays are in flight on the four waves at once.
template <int MODE>
__device__ __forceinline__ void merge_tile(const SelArgs& a, int64_t tbase, uint32_t tile_excl,
                                           uint32_t lim, uint32_t total, uint32_t n_lines,
                                           const uint16_t* list, const uint32_t* wbits,
                                           const uint32_t* wpre) {
    const int n_arr = a.n_true + (MODE == kAddDense ? 1 : 0);
    if (n_lines > 3 * kLinesPerPass) {
        uint32_t dsc[8], off[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t i = uint32_t(j * kLinesPerPass) + (threadIdx.x >> 3);
            const uint32_t k = threadIdx.x & 7u;
            const uint32_t line = i < n_lines ? list[i] : 0u;
            dsc[j] = i < n_lines ? chunk_desc(wbits[line], wpre[line], k, lim, total) : 0u;
            off[j] = (line * 8u + k) * 16u;
        }
        const int rows = int((n_lines + kLinesPerPass - 1) / kLinesPerPass);
        for (int at = 0; at < a.n_true; ++at)
            merge_dense<MODE, false>(a, a.dst[at], a.rec[at], tbase, tile_excl, lim, dsc, off,
                                     rows);
        if (MODE == kAddDense)
            merge_dense<MODE, true>(a, a.alive, nullptr, tbase, tile_excl, lim, dsc, off, rows);
        return;
    }
    // the wave index is uniform in the wave; said explicitly, so that the
    // array pointers picked by it stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int batches = int((n_lines + kLinesPerPass - 1) / kLinesPerPass);
    const int items = n_arr * batches;
    for (int it = wave; it < items; it += kWaves) {
        const int at = it / batches, b = it - at * batches;
        const uint32_t i0 = uint32_t(b * kLinesPerPass) + ((threadIdx.x & 63u) >> 3);
        if (MODE == kAddDense && at == a.n_true)
            merge_item<MODE, true>(a, a.alive, nullptr, tbase, tile_excl, lim, total, n_lines, i0,
                                   8, list, wbits, wpre);
        else
            merge_item<MODE, false>(a, a.dst[at], a.rec[at], tbase, tile_excl, lim, total,
                                    n_lines, i0, 8, list, wbits, wpre);
    }
}

// select_update / add_agents with whole-line writes.  The rank phase is that
// of k_select (lane t owns slots [32 t, 32 t + 32) of the 8192-slot tile,
// line t of every attribute); the merge is the line-list merge above, applied
// to every attribute and, for add_agents, to alive with the constant 1 (see
// merge_tile).  Every
// pointer is 16-byte aligned (checked on the host); the last tile, when
// partial, writes slot by slot.  The kernel stays within 64 VGPRs, so all
// 2048 tiles of a 2^24-slot launch are resident at once and the look-back
// waits one round.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_merge(SelArgs a) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint32_t wbits[kBlock];
    __shared__ uint32_t wpre[kBlock];
    __shared__ uint16_t list[kBlock];
    __shared__ uint32_t lcount[kWaves];
    const uint32_t tile = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t epoch = read_epoch(a.epoch);
    const int64_t tbase = int64_t(tile) * kTile;
    const int64_t lbase = tbase + int64_t(threadIdx.x) * kSlotsPerLane;
    const bool full_tile = tbase + kTile <= a.n;
    const uint32_t bits0 = load_bits<MODE>(a, lbase);

    uint32_t r0, total;
    uint32_t tile_excl = rank_counts<kWaves>(__popc(bits0), &r0, a.status, a.status - 1, tile,
                                             a.ntiles, epoch, lds, &total);
    // the tile's prefix and count are the same in every lane (read from LDS):
    // say so, so that the buffer descriptors built from them stay scalar
    tile_excl = __builtin_amdgcn_readfirstlane(tile_excl);
    total = __builtin_amdgcn_readfirstlane(total);
    const int64_t q = (MODE == kSelIndirect) ? *a.d_q : a.q;
    const int64_t room = q - int64_t(tile_excl);
    const uint32_t lim = room <= 0 ? 0u : (room < int64_t(total) ? uint32_t(room) : total);

    // compact the lines holding a receiving slot (in line order)
    const bool listed = bits0 != 0u && r0 < lim;
    const uint64_t bal = __ballot(listed);
    wbits[threadIdx.x] = bits0;
    wpre[threadIdx.x] = r0;
    if (lane == 0) lcount[wave] = uint32_t(__popcll(bal));
    __syncthreads();
    uint32_t before = 0, n_lines = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = lcount[w];
        before += w < wave ? c : 0u;
        n_lines += c;
    }
    n_lines = __builtin_amdgcn_readfirstlane(n_lines);
    if (listed) list[before + lane_rank(bal)] = uint16_t(threadIdx.x);
    __syncthreads();

    if (lim > 0 && full_tile) {
        merge_tile<MODE>(a, tbase, tile_excl, lim, total, n_lines, list, wbits, wpre);
    } else if (lim > 0 && listed) {
        // partial last tile: this lane's own receiving slots, one by one
        const uint32_t ab = receiving(bits0, r0, lim, total);
        for (uint32_t k = 0; k < 32; ++k) {
            if (!((ab >> k) & 1u)) continue;
            const int64_t g = int64_t(tile_excl) + r0 + __popc(ab & low_bits(k));
            const int64_t r = (MODE == kSelIndirect) ? int64_t(a.rec_idx[g]) : g;
            for (int at = 0; at < a.n_true; ++at) a.dst[at][lbase + k] = a.rec[at][r];
            if (MODE == kAddDense) a.alive[lbase + k] = 1;
        }
    }
    if (tile == a.ntiles - 1 && threadIdx.x == 0) {
        const int64_t p = int64_t(tile_excl) + total;
        const int64_t rr = p < q ? p : q;
        *a.d_applied = rr;
        if (a.d_dropped) *a.d_dropped = q - rr;
    }
}

// Writes the counts of a call that has nothing to scan.
__global__ void k_counts(const int64_t* d_q, int64_t q, int64_t* d_applied, int64_t* d_dropped) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t qq = d_q ? *d_q : q;
        if (d_applied) *d_applied = 0;
        if (d_dropped) *d_dropped = qq;
    }
}

int check_soa(const abm_soa* s, bool need_alive) {
    if (!s) return fail(ABM_E_INVALID, "collection is NULL");
    if (s->n_attrs < 1 || s->n_attrs > ABM_MAX_ATTRS)
        return fail(ABM_E_INVALID, "n_attrs must be in [1, 16]");
    if (s->capacity < 0 || s->capacity > kMaxIndex)
        return fail(ABM_E_INVALID, "capacity must be in [0, 2^31)");
    if (s->capacity > 0)
        for (int a = 0; a < s->n_attrs; ++a)
            if (!s->attr[a]) return fail(ABM_E_INVALID, "attribute pointer is NULL");
    if (need_alive && s->capacity > 0 && !s->alive)
        return fail(ABM_E_INVALID, "alive array is required");
    return ABM_OK;
}

int check_records(const abm_records* r, int32_t n_attrs) {
    if (!r) return fail(ABM_E_INVALID, "records are NULL");
    if (r->n_attrs != n_attrs) return fail(ABM_E_INVALID, "record and slot attribute counts differ");
    if (r->count < 0 || r->count > kMaxIndex)
        return fail(ABM_E_INVALID, "record count must be in [0, 2^31)");
    if (r->count > 0)
        for (int a = 0; a < r->n_attrs; ++a)
            if (!r->attr[a]) return fail(ABM_E_INVALID, "record attribute pointer is NULL");
    return ABM_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int padded_attrs(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : 16; }

// Fills the attribute pointer tables, repeating the last attribute up to the
// padded count.
void fill_attrs(SelArgs& a, const abm_soa* dst, const abm_records* rec) {
    const int n = dst->n_attrs, na = padded_attrs(n);
    for (int i = 0; i < na; ++i) {
        const int src = i < n ? i : n - 1;
        a.dst[i] = dst->attr[src];
        a.rec[i] = rec->attr[src];
    }
    a.n_attrs = na;
    a.n_true = n;
}

template <int MODE>
void launch_select(const SelArgs& a, hipStream_t st) {
    const dim3 grid(a.ntiles), block(kBlock);
    switch (a.n_attrs) {
        case 1: hipLaunchKernelGGL((k_select<MODE, 1>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_select<MODE, 2>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_select<MODE, 4>), grid, block, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_select<MODE, 8>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((k_select<MODE, 16>), grid, block, 0, st, a); break;
    }
}

// The merging kernel when every destination (and alive) pointer allows
// 16-byte access, else the scattering one.
template <int MODE>
void launch_write(SelArgs a, const abm_soa* dst, hipStream_t st) {
    bool vec = MODE != kAddDense || aligned16(dst->alive);
    for (int i = 0; i < dst->n_attrs; ++i) vec = vec && aligned16(dst->attr[i]);
    if (!vec) {
        launch_select<MODE>(a, st);
        return;
    }
    hipLaunchKernelGGL((k_merge<MODE>), dim3(a.ntiles), dim3(kBlock), 0, st, a);
}

// ------------------------------------------------------------ no-allocation form
// The scan state of abm_select_update_noalloc lives in this array: a 256-byte
// header (epoch word, error word at byte 248) followed by the tile status
// words of one scan chain for up to kNoallocMaxSlots slots.  Each device holds
// its own copy for the life of the process; every call on a device shares it.
constexpr int64_t kNoallocMaxSlots = int64_t(1) << 28;
// status words of one chain of T tiles: the tile words and each level's group
// words (as laid out by hier_prefix)
constexpr int64_t chain_words_c(int64_t T, int levels) {
    return levels == 0 ? 0 : T + chain_words_c((T + 63) / 64, levels - 1);
}
constexpr int64_t kScratchWords =
    kHeaderBytes / 8 + chain_words_c((kNoallocMaxSlots + kTile - 1) / kTile, kLevels) + 8;
static_assert(kScratchWords * 8 < (int64_t(1) << 19), "scratch stays under 512 KiB");
static __device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices] = {};

// Device address of this device's `scratch` (looked up once per device, with
// the device current; the array's host-side name is not a device address).
int scratch_for_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return ABM_E_HIP;
    }
    if (dev < 0 || dev >= kScratchDevices) return fail(ABM_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return ABM_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return ABM_OK;
}

// Hands the scratch error word to the caller and clears it for the next call.
__global__ void k_take_error(uint64_t* word, int64_t* d_error) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *d_error = int64_t(*word);
        *word = 0;
    }
}

int launch_compact(const uint8_t* mask, int64_t n, int32_t* out, int64_t* d_count,
                   const Workspace& w, hipStream_t st) {
    SelArgs c = {};
    c.mask = mask;
    c.out_idx = out;
    c.d_applied = d_count;
    c.n = n;
    c.status = w.status;
    int rc = next_epoch(w, st, &c.epoch);
    if (rc != ABM_OK) return rc;
    c.ntiles = static_cast<uint32_t>(tiles_for(n, kTile));
    c.vec_ok = aligned16(mask);
    hipLaunchKernelGGL((k_select<kCompact, 1>), dim3(c.ntiles), dim3(kBlock), 0, st, c);
    return launch_status("select_indices");
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" int abm_select_update(const abm_soa* dst, const uint8_t* sel_mask,
                                 const abm_records* upd, const uint8_t* upd_mask,
                                 int64_t* d_applied, int64_t* d_dropped, void* ws,
                                 size_t ws_bytes, void* stream) {
    int rc = check_soa(dst, false);
    if (rc != ABM_OK) return rc;
    rc = check_records(upd, dst->n_attrs);
    if (rc != ABM_OK) return rc;
    if (!d_applied) return fail(ABM_E_INVALID, "d_applied is NULL");
    if (dst->capacity > 0 && !sel_mask) return fail(ABM_E_INVALID, "sel_mask is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    const int64_t cap = dst->capacity > upd->count ? dst->capacity : upd->count;
    rc = check_ws(ws, ws_bytes, cap);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, cap);
    hipStream_t st = as_stream(stream);

    const int64_t* d_q = nullptr;
    if (upd_mask && upd->count > 0) {
        d_q = reinterpret_cast<const int64_t*>(w.hdr + kHdrCountA);
        rc = launch_compact(upd_mask, upd->count, w.list_a,
                            reinterpret_cast<int64_t*>(w.hdr + kHdrCountA), w, st);
        if (rc != ABM_OK) return rc;
    }
    const bool nothing = dst->capacity == 0 || upd->count == 0;
    if (nothing) {
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, d_q, upd_mask ? 0 : upd->count,
                           d_applied, d_dropped);
        return launch_status("select_update");
    }
    SelArgs a = {};
    fill_attrs(a, dst, upd);
    a.mask = sel_mask;
    a.rec_idx = w.list_a;
    a.d_q = d_q;
    a.q = upd->count;
    a.n = dst->capacity;
    a.d_applied = d_applied;
    a.d_dropped = d_dropped;
    a.status = w.status;
    a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
    a.vec_ok = aligned16(sel_mask);
    rc = next_epoch(w, st, &a.epoch);
    if (rc != ABM_OK) return rc;
    if (d_q)
        launch_write<kSelIndirect>(a, dst, st);
    else
        launch_write<kSelDense>(a, dst, st);
    return launch_status("select_update");
}

extern "C" int abm_add_agents(const abm_soa* dst, const abm_records* newborn, int64_t* d_added,
                              int64_t* d_dropped, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_soa(dst, true);
    if (rc != ABM_OK) return rc;
    rc = check_records(newborn, dst->n_attrs);
    if (rc != ABM_OK) return rc;
    if (!d_added) return fail(ABM_E_INVALID, "d_added is NULL");
    rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_ws(ws, ws_bytes, dst->capacity);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, dst->capacity);
    hipStream_t st = as_stream(stream);
    if (dst->capacity == 0 || newborn->count == 0) {
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, nullptr, newborn->count, d_added,
                           d_dropped);
        return launch_status("add_agents");
    }
    SelArgs a = {};
    fill_attrs(a, dst, newborn);
    a.alive = dst->alive;
    a.q = newborn->count;
    a.n = dst->capacity;
    a.d_applied = d_added;
    a.d_dropped = d_dropped;
    a.status = w.status;
    a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
    a.vec_ok = aligned16(dst->alive);
    rc = next_epoch(w, st, &a.epoch);
    if (rc != ABM_OK) return rc;
    launch_write<kAddDense>(a, dst, st);
    return launch_status("add_agents");
}

extern "C" int abm_select_indices(const uint8_t* mask, int64_t n, int32_t* out_idx,
                                  int64_t* d_count, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || n > kMaxIndex) return fail(ABM_E_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && (!mask || !out_idx)) return fail(ABM_E_INVALID, "mask or out_idx is NULL");
    if (!d_count) return fail(ABM_E_INVALID, "d_count is NULL");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_ws(ws, ws_bytes, n);
    if (rc != ABM_OK) return rc;
    Workspace w = carve(ws, n);
    hipStream_t st = as_stream(stream);
    if (n == 0) {
        // the count of an empty mask is zero: written as "dropped" of a no-op
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, nullptr, 0, nullptr, d_count);
        return launch_status("select_indices");
    }
    return launch_compact(mask, n, out_idx, d_count, w, st);
}

extern "C" int abm_select_update_noalloc(const abm_soa* dst, const uint8_t* sel_mask,
                                         const abm_records* upd, int64_t* d_applied,
                                         int64_t* d_dropped, int64_t* d_error, void* stream) {
    int rc = check_soa(dst, false);
    if (rc != ABM_OK) return rc;
    rc = check_records(upd, dst->n_attrs);
    if (rc != ABM_OK) return rc;
    if (!d_applied) return fail(ABM_E_INVALID, "d_applied is NULL");
    if (dst->capacity > 0 && !sel_mask) return fail(ABM_E_INVALID, "sel_mask is NULL");
    if (dst->capacity > kNoallocMaxSlots) {
        set_error("capacity %lld exceeds the no-allocation maximum of 2^28 slots",
                  static_cast<long long>(dst->capacity));
        return ABM_E_INVALID;
    }
    rc = check_device();
    if (rc != ABM_OK) return rc;
    void* base = nullptr;
    rc = scratch_for_device(&base);
    if (rc != ABM_OK) return rc;
    Workspace w = {};
    w.hdr = static_cast<uint64_t*>(base);
    w.status = w.hdr + kHeaderBytes / 8;
    hipStream_t st = as_stream(stream);
    if (dst->capacity == 0 || upd->count == 0) {
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, nullptr, upd->count, d_applied,
                           d_dropped);
    } else {
        SelArgs a = {};
        fill_attrs(a, dst, upd);
        a.mask = sel_mask;
        a.q = upd->count;
        a.n = dst->capacity;
        a.d_applied = d_applied;
        a.d_dropped = d_dropped;
        a.status = w.status;
        a.ntiles = static_cast<uint32_t>(tiles_for(dst->capacity, kTile));
        a.vec_ok = aligned16(sel_mask);
        rc = next_epoch(w, st, &a.epoch);
        if (rc != ABM_OK) return rc;
        launch_write<kSelDense>(a, dst, st);
    }
    if (d_error)
        hipLaunchKernelGGL(k_take_error, dim3(1), dim3(64), 0, st, w.hdr + kHdrError, d_error);
    return launch_status("select_update_noalloc");
}
