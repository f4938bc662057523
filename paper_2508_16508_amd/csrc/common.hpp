// common.hpp -- host-side plumbing shared by the libabm entry points:
// status/error reporting, device checks, workspace layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "abm.h"

namespace abm {

// Thread-local text of the last failure; returned by abm_last_error().
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// ABM_E_UNSUPPORTED unless the current device is gfx950 (cached per device).
int check_device();

inline int fail(int code, const char* what) {
    set_error("%s", what);
    return code;
}

// Checks the launch status of the kernels just enqueued.
inline int launch_status(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", where, hipGetErrorString(e));
        return ABM_E_HIP;
    }
    return ABM_OK;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- workspace
// [0, 256)                 header words (uint64); the last one is the scan
//                          error word, directly before the status array
// [256, 256 + 8*S)         tile status words of the single-pass scans
// [.., + 4*C)              int32 index list (compacted record indices or breeders)
// [.., + 4*C)              second int32 index list (second species)
// [.., + 8*kAccWords)      int64 spread accumulators (kAccLanes per counter)
// [.., + 2 * bitmask)      two live-slot bitmasks (predation: sheep, wolves)
// S covers two chains of ceil(C / kMinTile) tiles each.
constexpr int64_t kHeaderBytes = 256;
constexpr int64_t kMinTile = 512;
constexpr int kAccLanes = 256;             // accumulators per counter
constexpr int kAccCounters = 8;
constexpr int64_t kAccWords = int64_t(kAccLanes) * kAccCounters;

enum HeaderWord : int {
    kHdrEpoch = 0,    // device epoch word (uint32 in the low half) for graph-recorded launches
    kHdrCountA = 2,   // int64 count produced on the device (selected records / breeders)
    kHdrCountB = 3,   // int64 second count (second species)
    kHdrError = 31    // set to 1 when a bounded wait gave up (never expected)
};

inline int64_t tiles_for(int64_t n, int64_t tile) { return (n + tile - 1) / tile; }

// Room for two scan chains of ceil(C / kMinTile) tiles each plus their group
// words (a chain of T tiles needs less than T + T/63 + 4 words).
inline int64_t status_words(int64_t capacity) {
    const int64_t t = tiles_for(capacity, kMinTile);
    return 2 * (t + t / 63 + 8) + 2;
}

// Live-slot bitmask of one collection of up to `capacity` slots: one bit per
// slot, padded to whole 8192-slot tiles (1 KiB each).
inline int64_t bitmask_bytes(int64_t capacity) { return tiles_for(capacity, 8192) * 1024; }

inline size_t workspace_bytes(int64_t capacity) {
    if (capacity < 1) capacity = 1;
    return (size_t)(kHeaderBytes + 8 * status_words(capacity) + 8 * capacity + 8 * kAccWords +
                    2 * bitmask_bytes(capacity) + 64);
}

struct Workspace {
    uint64_t* hdr;
    uint64_t* status;
    int32_t* list_a;
    int32_t* list_b;
    int64_t* acc;
    uint32_t* bits_a;   // live-slot bitmasks (predation: sheep, wolves)
    uint32_t* bits_b;
};

inline Workspace carve(void* ws, int64_t capacity) {
    if (capacity < 1) capacity = 1;
    char* p = static_cast<char*>(ws);
    Workspace w;
    w.hdr = reinterpret_cast<uint64_t*>(p);
    w.status = reinterpret_cast<uint64_t*>(p + kHeaderBytes);
    char* lists = p + kHeaderBytes + 8 * status_words(capacity);
    w.list_a = reinterpret_cast<int32_t*>(lists);
    w.list_b = reinterpret_cast<int32_t*>(lists + 4 * capacity);
    w.acc = reinterpret_cast<int64_t*>(lists + 8 * capacity);
    w.bits_a = reinterpret_cast<uint32_t*>(lists + 8 * capacity + 8 * kAccWords);
    w.bits_b = w.bits_a + bitmask_bytes(capacity) / 4;
    return w;
}

// Validates a workspace argument for `capacity` slots.
inline int check_ws(const void* ws, size_t ws_bytes, int64_t capacity) {
    if (!ws) return fail(ABM_E_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(ABM_E_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = workspace_bytes(capacity);
    if (ws_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", ws_bytes, need);
        return ABM_E_WORKSPACE;
    }
    return ABM_OK;
}

constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;

}  // namespace abm

#include "scan.hpp"

namespace abm {

// Epoch for the next single-pass launch on workspace w: a fresh host value
// (launch argument), or -- when the stream is recording a graph, whose
// arguments replay unchanged -- the device epoch word, advanced in-stream by
// a one-thread kernel first.  Host epochs use bit 29 = 0 and device epochs
// bit 29 = 1, so the two never coincide on one workspace.
int next_epoch(const Workspace& w, hipStream_t st, EpochArg* out);

}  // namespace abm
