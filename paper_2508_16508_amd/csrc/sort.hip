// sort.hip -- abm_sort_agents and abm_select_agents (the Sec. 2 API's
// sort_agents and select_agents).
//
// sort_agents is a least-significant-digit radix sort of (key, slot) pairs
// with 8-bit digits, four passes over 32-bit keys, followed by a gather of
// every attribute column through the resulting permutation (the columns
// packed into one record per agent first).  Each pass is
//   histogram  per 4096-key tile, 256 bins in LDS, stored digit-major;
//   scan       one workgroup per digit scans that digit's tile counts (the
//              tile's offset within the digit's bucket), and one workgroup
//              turns the 256 digit totals into bucket bases;
//   scatter    each tile ranks its keys stably: a wave takes its 16 items in
//              order, finds the lanes holding the same digit with eight
//              ballots (one per digit bit), and ranks a lane after the
//              same-digit lanes below it and the same-digit keys of the
//              wave's earlier items (running per-wave counters in LDS); wave
//              offsets per digit follow from the wave totals.  A key's
//              destination is base[d] + tile offset[d] + wave offset[d] + rank.
// Keys in a tile are laid out wave-major, then item, then lane, so that the
// lane order inside an item is the index order and every pass is stable.  A
// signed key becomes an unsigned one with the sign bit flipped (ascending)
// and then all bits flipped (descending), so the descending sort keeps equal
// keys in index order too.
//
// select_agents is a stable partition, set flags first: a count of the set flags
// per 4096-flag tile, one scan of the tile counts, and a pass that stages
// each tile's indices in partition order in LDS and writes both runs.
#include <hip/hip_runtime.h>

#include "abm.h"
#include "common.hpp"
#include "scan.hpp"

namespace abm {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
constexpr int kItems = 16;
constexpr int64_t kTile = int64_t(kBlock) * kItems;   // 4096 keys
constexpr int kBins = 256;

enum KeySource : int {
    kFromKeys = 0,      // first pass: int32 keys, slot = index
    kFromBuffer = 1     // later passes: (ukey, slot) ping-pong buffers
};

struct PassArgs {
    const int32_t* key;        // kFromKeys
    const uint32_t* in_key;    // kFromBuffer
    const int32_t* in_val;
    uint32_t* out_key;
    int32_t* out_val;
    uint32_t* counts;          // [kBins][n_tiles]: tile counts, then tile offsets
    uint32_t* totals;          // [kBins]
    uint32_t* base;            // [kBins]
    int64_t n;
    uint32_t n_tiles;
    uint32_t shift;
    uint32_t flip;             // xor applied to the sign-flipped key (0 or ~0)
};

// Slot of item k of lane l of wave w in tile t.
__device__ __forceinline__ int64_t slot_of(uint32_t t, int w, int k, int l) {
    return int64_t(t) * kTile + int64_t(w) * (kItems * 64) + k * 64 + l;
}

template <int SRC>
__device__ __forceinline__ void load_item(const PassArgs& a, int64_t i, uint32_t& ukey,
                                          int32_t& val, uint32_t& digit) {
    if (SRC == kFromKeys) {
        ukey = (uint32_t(a.key[i]) ^ 0x80000000u) ^ a.flip;
        val = int32_t(i);
        digit = (ukey >> a.shift) & 0xFFu;
    } else {
        ukey = a.in_key[i];
        val = a.in_val[i];
        digit = (ukey >> a.shift) & 0xFFu;
    }
}

template <int SRC>
__global__ __launch_bounds__(kBlock) void k_hist(PassArgs a) {
    __shared__ uint32_t hist[kBins];
    const uint32_t t = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kBins; d += kBlock) hist[d] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = slot_of(t, w, k, lane);
        if (i >= a.n) continue;
        uint32_t ukey, digit;
        int32_t val;
        load_item<SRC>(a, i, ukey, val, digit);
        atomicAdd(&hist[digit], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBins; d += kBlock) a.counts[int64_t(d) * a.n_tiles + t] = hist[d];
}

// Exclusive scan in place of row r = blockIdx.x of n_tiles counts (the tile
// counts of one radix digit, or of the set flags); totals[r] = the row's sum.
// One workgroup of 1024 threads per row, four consecutive counts per thread
// (one round for up to 4096 tiles, i.e. 2^24 keys).
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan_rows(uint32_t* rows, uint32_t n_tiles,
                                                            uint32_t* totals) {
    uint32_t* counts = rows + int64_t(blockIdx.x) * n_tiles;
    __shared__ uint32_t wtot[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < n_tiles; c0 += 4 * kScanThreads) {
        const uint32_t i = c0 + 4 * threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = i + q < n_tiles ? counts[i + q] : 0u;
        const uint32_t mine = v[0] + v[1] + v[2] + v[3];
        uint32_t x = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wtot[w] = x;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kScanThreads / 64; ++q) {
            before += q < w ? wtot[q] : 0u;
            all += wtot[q];
        }
        uint32_t ex = carry + before + x - mine;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (i + q < n_tiles) {
                counts[i + q] = ex;
                ex += v[q];
            }
        carry += all;
        __syncthreads();   // wtot is reused by the next round
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBins) void k_digit_base(PassArgs a) {
    __shared__ uint32_t lds[kBins / 64 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t v = a.totals[threadIdx.x];
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int q = 0; q < w; ++q) before += lds[q];
    a.base[threadIdx.x] = before + x - v;
}

// Lanes of the wave whose digit equals this lane's (among the active lanes).
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t digit, bool active, int bits) {
    uint64_t m = __ballot(active);
#pragma unroll
    for (int b = 0; b < bits; ++b) {
        const uint64_t set = __ballot(active && ((digit >> b) & 1u));
        m &= ((digit >> b) & 1u) ? set : ~set;
    }
    return m;
}

template <int SRC>
__global__ __launch_bounds__(kBlock) void k_scatter(PassArgs a) {
    __shared__ uint32_t wcount[kWaves][kBins];   // running, then exclusive across waves
    __shared__ uint32_t dstart[kBins];           // start of each digit within the tile
    __shared__ uint32_t skey[kTile];             // the tile in digit order
    __shared__ int32_t sval[kTile];
    const uint32_t t = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * kBins; d += kBlock) (&wcount[0][0])[d] = 0;
    __syncthreads();
    uint32_t key[kItems], dig[kItems], rank[kItems];
    int32_t val[kItems];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = slot_of(t, w, k, lane);
        const bool active = i < a.n;
        key[k] = 0;
        val[k] = 0;
        dig[k] = 0;
        if (active) load_item<SRC>(a, i, key[k], val[k], dig[k]);
        const uint64_t peers = same_digit_lanes(dig[k], active, 8);
        // the lowest peer reads and advances the wave's counter for this digit
        const uint32_t before = active ? wcount[w][dig[k]] : 0u;
        rank[k] = before + uint32_t(__popcll(peers & below));
        // every peer has read the counter before the leader advances it
        __builtin_amdgcn_wave_barrier();
        if (active && (peers & below) == 0)
            wcount[w][dig[k]] = before + uint32_t(__popcll(peers));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive offsets of the waves, and the digit's tile total
    uint32_t dtot = 0;
    if (threadIdx.x < kBins) {
        const int d = threadIdx.x;
        for (int q = 0; q < kWaves; ++q) {
            const uint32_t c = wcount[q][d];
            wcount[q][d] = dtot;
            dtot += c;
        }
    }
    // exclusive scan of the digit totals: where each digit starts in the tile
    {
        uint32_t x = dtot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        __shared__ uint32_t wtot[kWaves];
        if (lane == 63) wtot[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int q = 0; q < w; ++q) before += wtot[q];
        if (threadIdx.x < kBins) dstart[threadIdx.x] = before + x - dtot;
    }
    __syncthreads();
    // where each digit's run of this tile goes, less its start in the tile
    // (read from global memory once per digit, not once per key)
    __shared__ int64_t goff[kBins];
    if (threadIdx.x < kBins) {
        const int d = threadIdx.x;
        goff[d] = int64_t(a.base[d]) + a.counts[int64_t(d) * a.n_tiles + t] - int64_t(dstart[d]);
    }
    // stage the tile in digit order
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = slot_of(t, w, k, lane);
        if (i >= a.n) continue;
        const uint32_t d = dig[k];
        const uint32_t p = dstart[d] + wcount[w][d] + rank[k];
        skey[p] = key[k];
        sval[p] = val[k];
    }
    __syncthreads();
    // consecutive threads write consecutive positions of a digit's run
    const int64_t left = a.n - int64_t(t) * kTile;
    const int32_t n_tile = left < kTile ? int32_t(left) : int32_t(kTile);
    for (int32_t p = threadIdx.x; p < n_tile; p += kBlock) {
        const uint32_t kk = skey[p];
        const int64_t dst = goff[(kk >> a.shift) & 0xFFu] + p;
        a.out_key[dst] = kk;
        a.out_val[dst] = sval[p];
    }
}

dim3 stream_grid(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return dim3(uint32_t(b < 8192 ? (b > 0 ? b : 1) : 8192));
}

// The columns go through the permutation packed into one record per agent:
// a coalesced pass writes record i = (col[0][i], ..., col[C-1][i]), padded to
// a power-of-two size (at most 128 bytes, so a record never straddles a
// 128-byte line), and the gather makes one random record read per agent and
// writes every column at position j.  Random reads, not bytes, bound a
// gather: each fetches a whole line whatever its width, so one read per agent
// replaces one per column and agent.
constexpr int kMaxCols = ABM_MAX_ATTRS + 1;   // attributes + alive
constexpr int kMaxRecWords = 32;

int rec_words(int n_cols) {
    int w = 1;
    while (w < n_cols) w <<= 1;
    return n_cols > 0 ? w : 0;
}

struct GatherArgs {
    int32_t* col[kMaxRecWords];   // the columns; entries from n_cols on are unused
    int32_t n_cols;
    int32_t* rec;                 // n records of RW words
    const int32_t* perm;
    int64_t n;
};

// Records of 1 or 2 words: one lane per record.
template <int RW>
__global__ __launch_bounds__(kBlock) void k_pack_small(GatherArgs g) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < g.n;
         i += int64_t(gridDim.x) * kBlock) {
        if (RW == 1)
            g.rec[i] = g.col[0][i];
        else
            reinterpret_cast<int2*>(g.rec)[i] = int2{g.col[0][i], g.n_cols > 1 ? g.col[1][i] : 0};
    }
}

template <int RW>
__global__ __launch_bounds__(kBlock) void k_gather_small(GatherArgs g) {
    for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < g.n;
         j += int64_t(gridDim.x) * kBlock) {
        const int64_t p = g.perm[j];
        if (RW == 1) {
            g.col[0][j] = g.rec[p];
        } else {
            const int2 t = reinterpret_cast<const int2*>(g.rec)[p];
            g.col[0][j] = t.x;
            if (g.n_cols > 1) g.col[1][j] = t.y;
        }
    }
}

// Records of 4 to 32 words (P = RW / 4 pieces of 16 bytes), 64 records per
// wave and round, transposed through LDS so that both sides of every global
// access are contiguous: pack reads each column at 64 consecutive positions
// (one lane per record) and writes the 64 records as 64 P consecutive pieces
// (lane-consecutive); gather reads 64 / P records per load instruction (P
// lanes per record, each record one 64-byte-aligned run) and writes each column
// at 64 consecutive positions.  The loop runs over whole blocks, so every wave
// meets the same barriers.
template <int RW>
__global__ __launch_bounds__(kBlock) void k_pack_cols(GatherArgs g) {
    constexpr int P = RW / 4;
    __shared__ int4 sbuf[kWaves * 64 * P];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int4* mine = sbuf + w * 64 * P;
    int4* rec4 = reinterpret_cast<int4*>(g.rec);
    for (int64_t b0 = int64_t(blockIdx.x) * kBlock; b0 < g.n; b0 += int64_t(gridDim.x) * kBlock) {
        const int64_t base = b0 + w * 64;
        const int64_t i = base + lane;
        int32_t r[RW];
#pragma unroll
        for (int c = 0; c < RW; ++c) r[c] = (c < g.n_cols && i < g.n) ? g.col[c][i] : 0;
#pragma unroll
        for (int v = 0; v < P; ++v) mine[lane * P + v] = int4{r[4 * v], r[4 * v + 1], r[4 * v + 2], r[4 * v + 3]};
        __syncthreads();
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int idx = k * 64 + lane;
            if (base + idx / P < g.n) rec4[base * P + idx] = mine[idx];
        }
        __syncthreads();
    }
}

template <int RW>
__global__ __launch_bounds__(kBlock) void k_gather_recs(GatherArgs g) {
    constexpr int P = RW / 4;
    __shared__ int4 sbuf[kWaves * 64 * P];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int4* mine = sbuf + w * 64 * P;
    const int4* rec4 = reinterpret_cast<const int4*>(g.rec);
    const int used = (g.n_cols + 3) / 4;   // pieces holding columns
    for (int64_t b0 = int64_t(blockIdx.x) * kBlock; b0 < g.n; b0 += int64_t(gridDim.x) * kBlock) {
        const int64_t base = b0 + w * 64;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int idx = k * 64 + lane;
            const int64_t j = base + idx / P;
            const int piece = idx % P;
            if (j < g.n && piece < used) mine[idx] = rec4[int64_t(g.perm[j]) * P + piece];
        }
        __syncthreads();
        const int64_t j = base + lane;
        if (j < g.n) {
            int32_t r[RW];
#pragma unroll
            for (int v = 0; v < P; ++v) {
                const int4 t = v < used ? mine[lane * P + v] : int4{0, 0, 0, 0};
                r[4 * v] = t.x;
                r[4 * v + 1] = t.y;
                r[4 * v + 2] = t.z;
                r[4 * v + 3] = t.w;
            }
#pragma unroll
            for (int c = 0; c < RW; ++c)
                if (c < g.n_cols) g.col[c][j] = r[c];
        }
        __syncthreads();
    }
}

template <int RW>
void gather_cols(const GatherArgs& ga, hipStream_t st) {
    if constexpr (RW <= 2) {
        hipLaunchKernelGGL(k_pack_small<RW>, stream_grid(ga.n), dim3(kBlock), 0, st, ga);
        hipLaunchKernelGGL(k_gather_small<RW>, stream_grid(ga.n), dim3(kBlock), 0, st, ga);
    } else {
        hipLaunchKernelGGL(k_pack_cols<RW>, stream_grid(ga.n), dim3(kBlock), 0, st, ga);
        hipLaunchKernelGGL(k_gather_recs<RW>, stream_grid(ga.n), dim3(kBlock), 0, st, ga);
    }
}

__global__ __launch_bounds__(kBlock) void k_copy(const int32_t* __restrict__ src,
                                                 int32_t* __restrict__ dst, int64_t n) {
    for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < n;
         j += int64_t(gridDim.x) * kBlock)
        dst[j] = src[j];
}

// ---- select_agents: a stable partition, trues first.  A tile is 4096
// flags, 16 per lane (one 16-byte load when the flags are 16-byte aligned).
constexpr int kSelPerLane = 16;
constexpr int64_t kSelTile = int64_t(kBlock) * kSelPerLane;

// Bit b set when flag first + b is in range and nonzero.
template <bool ALIGNED>
__device__ __forceinline__ uint32_t load_flags(const uint8_t* __restrict__ cond, int64_t first,
                                               int64_t n) {
    uint32_t bits = 0;
    if (ALIGNED && first + kSelPerLane <= n) {
        const uint4 v = *reinterpret_cast<const uint4*>(cond + first);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                bits |= ((w[q] >> (8 * b)) & 0xFFu) ? (1u << (4 * q + b)) : 0u;
    } else {
        for (int b = 0; b < kSelPerLane; ++b)
            if (first + b < n && cond[first + b]) bits |= 1u << b;
    }
    return bits;
}

// Exclusive scan of v over the workgroup (kBlock threads); *total = the sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wtot[kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        before += q < w ? wtot[q] : 0u;
        all += wtot[q];
    }
    *total = all;
    return before + x - v;
}

// counts[t] = flags set in tile t
template <bool ALIGNED>
__global__ __launch_bounds__(kBlock) void k_sel_count(const uint8_t* __restrict__ cond, int64_t n,
                                                      uint32_t* __restrict__ counts) {
    const int64_t first = int64_t(blockIdx.x) * kSelTile + int64_t(threadIdx.x) * kSelPerLane;
    uint32_t total;
    block_excl_scan(uint32_t(__popc(load_flags<ALIGNED>(cond, first, n))), &total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// The tile's set flags go to [counts[t], ...) and its clear flags to
// [total + (t * 4096 - counts[t]), ...), both in index order; the tile is
// staged in LDS in that order so that consecutive threads write consecutive
// positions.
template <bool ALIGNED>
__global__ __launch_bounds__(kBlock) void k_sel_scatter(const uint8_t* __restrict__ cond,
                                                        int64_t n,
                                                        const uint32_t* __restrict__ counts,
                                                        const uint32_t* __restrict__ totals,
                                                        int32_t* __restrict__ order,
                                                        int64_t* d_count) {
    __shared__ int32_t sidx[kSelTile];
    const uint32_t t = blockIdx.x;
    const int64_t tile0 = int64_t(t) * kSelTile;
    const int64_t first = tile0 + int64_t(threadIdx.x) * kSelPerLane;
    const uint32_t bits = load_flags<ALIGNED>(cond, first, n);
    uint32_t n_set;
    const uint32_t set_before = block_excl_scan(uint32_t(__popc(bits)), &n_set);
    const int64_t left = n - tile0;
    const int32_t n_tile = left < kSelTile ? int32_t(left) : int32_t(kSelTile);
    const int32_t lane0 = int32_t(threadIdx.x) * kSelPerLane;
    const int32_t valid_before = lane0 < n_tile ? lane0 : n_tile;
    uint32_t s_pos = set_before;
    uint32_t c_pos = n_set + uint32_t(valid_before) - set_before;
    for (int b = 0; b < kSelPerLane; ++b) {
        if (lane0 + b >= n_tile) break;
        const int32_t i = int32_t(first + b);
        if ((bits >> b) & 1u)
            sidx[s_pos++] = i;
        else
            sidx[c_pos++] = i;
    }
    __syncthreads();
    const int64_t total = int64_t(totals[0]);
    const int64_t set0 = int64_t(counts[t]);
    const int64_t clear0 = total + (tile0 - set0) - int64_t(n_set);
    for (int32_t p = threadIdx.x; p < n_tile; p += kBlock)
        order[(p < int32_t(n_set) ? set0 : clear0) + p] = sidx[p];
    if (t == 0 && threadIdx.x == 0) *d_count = total;
}

__global__ void k_count_out(const uint32_t* totals, int64_t* d_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_count = totals ? int64_t(totals[0]) : 0;
}

struct SortWs {
    int32_t* val_b;            // the last pass's slots: the permutation
    uint32_t *key_a, *key_b;   // the other ping-pong buffers ...
    int32_t* val_a;
    int32_t* rec;              // ... whose region the records reuse afterwards
    uint32_t *counts, *totals, *base;
};

uint32_t tiles_of(int64_t n) { return uint32_t((n + kTile - 1) / kTile); }

int64_t round256(int64_t bytes) { return (bytes + 255) / 256 * 256; }

// Bytes of the region shared by key_a, key_b, val_a and the records.
int64_t region_bytes(int64_t m, int n_cols) {
    const int64_t bufs = 3 * round256(4 * m);
    const int64_t recs = round256(m * 4 * rec_words(n_cols));
    return bufs > recs ? bufs : recs;
}

size_t sort_ws_bytes(int64_t n, int n_cols) {
    const int64_t m = n > 0 ? n : 1;
    return size_t(round256(4 * m) + region_bytes(m, n_cols) +
                  round256(4 * int64_t(kBins) * tiles_of(m)) + 2 * round256(4 * kBins));
}

SortWs carve_sort(void* ws, int64_t n, int n_cols) {
    const int64_t m = n > 0 ? n : 1;
    char* p = static_cast<char*>(ws);
    SortWs s;
    s.val_b = reinterpret_cast<int32_t*>(p);
    p += round256(4 * m);
    s.key_a = reinterpret_cast<uint32_t*>(p);
    s.key_b = reinterpret_cast<uint32_t*>(p + round256(4 * m));
    s.val_a = reinterpret_cast<int32_t*>(p + 2 * round256(4 * m));
    s.rec = reinterpret_cast<int32_t*>(p);
    p += region_bytes(m, n_cols);
    s.counts = reinterpret_cast<uint32_t*>(p);
    p += round256(4 * int64_t(kBins) * tiles_of(m));
    s.totals = reinterpret_cast<uint32_t*>(p);
    p += round256(4 * kBins);
    s.base = reinterpret_cast<uint32_t*>(p);
    return s;
}

template <int SRC>
void launch_pass(const PassArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hist<SRC>, dim3(a.n_tiles), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_scan_rows, dim3(kBins), dim3(kScanThreads), 0, st, a.counts, a.n_tiles,
                       a.totals);
    hipLaunchKernelGGL(k_digit_base, dim3(1), dim3(kBins), 0, st, a);
    hipLaunchKernelGGL(k_scatter<SRC>, dim3(a.n_tiles), dim3(kBlock), 0, st, a);
}

int check_sort_ws(void* ws, size_t ws_bytes, int64_t n, int n_cols) {
    const size_t need = sort_ws_bytes(n, n_cols);
    if (!ws || ws_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", ws_bytes, need);
        return ABM_E_WORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(ABM_E_WORKSPACE, "workspace must be 256-byte aligned");
    return ABM_OK;
}

}  // namespace
}  // namespace abm

using namespace abm;

extern "C" size_t abm_sort_workspace_bytes(int64_t n, int32_t n_cols) {
    if (n < 0 || n > kMaxIndex || n_cols < 0 || n_cols > kMaxCols) return 0;
    return sort_ws_bytes(n, n_cols);
}

extern "C" int abm_sort_agents(const abm_soa* dst, const int32_t* key, int32_t descending,
                               int32_t* perm, void* ws, size_t ws_bytes, void* stream) {
    if (!dst) return fail(ABM_E_INVALID, "dst is NULL");
    if (dst->n_attrs < 0 || dst->n_attrs > ABM_MAX_ATTRS)
        return fail(ABM_E_INVALID, "n_attrs must be in [0, 16]");
    if (dst->capacity < 0 || dst->capacity > kMaxIndex)
        return fail(ABM_E_INVALID, "capacity must be in [0, 2^31)");
    const int64_t n = dst->capacity;
    if (n > 0 && !key) return fail(ABM_E_INVALID, "key is NULL");
    for (int a = 0; a < dst->n_attrs; ++a)
        if (n > 0 && !dst->attr[a]) return fail(ABM_E_INVALID, "attribute array is NULL");
    int32_t* cols[kMaxCols];
    int n_cols = 0;
    for (int c = -1; c < dst->n_attrs; ++c) {
        int32_t* col = c < 0 ? dst->alive : dst->attr[c];
        if (col) cols[n_cols++] = col;
    }
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_sort_ws(ws, ws_bytes, n, n_cols);
    if (rc != ABM_OK) return rc;
    if (n == 0) return ABM_OK;
    hipStream_t st = as_stream(stream);
    SortWs s = carve_sort(ws, n, n_cols);
    PassArgs a{};
    a.key = key;
    a.counts = s.counts;
    a.totals = s.totals;
    a.base = s.base;
    a.n = n;
    a.n_tiles = tiles_of(n);
    a.flip = descending ? ~0u : 0u;
    uint32_t* kin = nullptr;
    int32_t* vin = nullptr;
    for (int pass = 0; pass < 4; ++pass) {
        a.shift = 8u * uint32_t(pass);
        a.in_key = kin;
        a.in_val = vin;
        a.out_key = (pass & 1) ? s.key_b : s.key_a;
        a.out_val = (pass & 1) ? s.val_b : s.val_a;
        if (pass == 0)
            launch_pass<kFromKeys>(a, st);
        else
            launch_pass<kFromBuffer>(a, st);
        kin = a.out_key;
        vin = a.out_val;
    }
    // vin = the permutation: the agent now at position j was at vin[j].  The
    // columns go through it packed into records, in the region of the buffers
    // the passes no longer need (vin is val_b, outside it).
    if (n_cols > 0) {
        GatherArgs ga{};
        for (int c = 0; c < n_cols; ++c) ga.col[c] = cols[c];
        ga.n_cols = n_cols;
        ga.rec = s.rec;
        ga.perm = vin;
        ga.n = n;
        switch (rec_words(n_cols)) {
            case 1: gather_cols<1>(ga, st); break;
            case 2: gather_cols<2>(ga, st); break;
            case 4: gather_cols<4>(ga, st); break;
            case 8: gather_cols<8>(ga, st); break;
            case 16: gather_cols<16>(ga, st); break;
            default: gather_cols<32>(ga, st); break;
        }
    }
    if (perm) hipLaunchKernelGGL(k_copy, stream_grid(n), dim3(kBlock), 0, st, vin, perm, n);
    return launch_status("sort_agents");
}

extern "C" int abm_select_agents(const uint8_t* cond, int64_t n, int32_t* order, int64_t* d_count,
                                 void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || n > kMaxIndex) return fail(ABM_E_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && (!cond || !order)) return fail(ABM_E_INVALID, "cond or order is NULL");
    if (!d_count) return fail(ABM_E_INVALID, "d_count is NULL");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    rc = check_sort_ws(ws, ws_bytes, n, 0);
    if (rc != ABM_OK) return rc;
    hipStream_t st = as_stream(stream);
    if (n == 0) {
        hipLaunchKernelGGL(k_count_out, dim3(1), dim3(64), 0, st, nullptr, d_count);
        return launch_status("select_agents");
    }
    SortWs s = carve_sort(ws, n, 0);
    const uint32_t n_tiles = uint32_t((n + kSelTile - 1) / kSelTile);
    if ((reinterpret_cast<uintptr_t>(cond) & 15) == 0) {
        hipLaunchKernelGGL(k_sel_count<true>, dim3(n_tiles), dim3(kBlock), 0, st, cond, n, s.counts);
        hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kScanThreads), 0, st, s.counts, n_tiles,
                           s.totals);
        hipLaunchKernelGGL(k_sel_scatter<true>, dim3(n_tiles), dim3(kBlock), 0, st, cond, n,
                           s.counts, s.totals, order, d_count);
    } else {
        hipLaunchKernelGGL(k_sel_count<false>, dim3(n_tiles), dim3(kBlock), 0, st, cond, n,
                           s.counts);
        hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(kScanThreads), 0, st, s.counts, n_tiles,
                           s.totals);
        hipLaunchKernelGGL(k_sel_scatter<false>, dim3(n_tiles), dim3(kBlock), 0, st, cond, n,
                           s.counts, s.totals, order, d_count);
    }
    return launch_status("select_agents");
}
