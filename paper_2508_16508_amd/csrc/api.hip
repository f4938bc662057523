// api.hip -- library-wide host entry points: errors, device check, workspace.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "abm.h"
#include "common.hpp"

namespace abm {

namespace {
thread_local char g_error[512] = "";
constexpr int kMaxDevices = 64;
std::atomic<int> g_device_ok[kMaxDevices];  // 0 unknown, 1 gfx950, 2 other
}  // namespace

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
}

int check_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return ABM_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(ABM_E_UNSUPPORTED, "device index out of range");
    int st = g_device_ok[dev].load(std::memory_order_relaxed);
    if (st == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) {
            set_error("hipGetDeviceProperties: %s", hipGetErrorString(e));
            return ABM_E_HIP;
        }
        st = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 2;
        g_device_ok[dev].store(st, std::memory_order_relaxed);
    }
    if (st != 1) return fail(ABM_E_UNSUPPORTED, "libabm is built for gfx950 (MI355X) only");
    return ABM_OK;
}

namespace {
std::atomic<uint32_t> g_host_epoch{1};

__global__ void k_bump_epoch(uint32_t* word) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t e = *word & 0x1FFFFFFFu;
        *word = ((e + 1u) & 0x1FFFFFFFu) | 0x20000000u;
    }
}
}  // namespace

int next_epoch(const Workspace& w, hipStream_t st, EpochArg* out) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) {
        set_error("hipStreamIsCapturing: %s", hipGetErrorString(e));
        return ABM_E_HIP;
    }
    if (cs == hipStreamCaptureStatusActive) {
        uint32_t* word = reinterpret_cast<uint32_t*>(w.hdr + kHdrEpoch);
        hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, st, word);
        out->value = 0;
        out->dev = word;
        return launch_status("epoch");
    }
    out->value = g_host_epoch.fetch_add(1, std::memory_order_relaxed) & 0x1FFFFFFFu;
    out->dev = nullptr;
    return ABM_OK;
}

}  // namespace abm

extern "C" {

const char* abm_last_error(void) { return abm::g_error; }

const char* abm_version(void) { return "abm 0.1.0 gfx950"; }

size_t abm_workspace_bytes(int op, int64_t capacity) {
    switch (op) {
        case ABM_OP_SELECT_UPDATE:
        case ABM_OP_ADD_AGENTS:
        case ABM_OP_REMOVE_AGENTS:
        case ABM_OP_SELECT_INDICES:
        case ABM_OP_PREDATION:
            return abm::workspace_bytes(capacity);
        default:
            return 0;
    }
}

int abm_workspace_init(void* ws, size_t ws_bytes, void* stream) {
    if (!ws || ws_bytes == 0) return abm::fail(ABM_E_WORKSPACE, "workspace is NULL or empty");
    int rc = abm::check_device();
    if (rc != ABM_OK) return rc;
    hipError_t e = hipMemsetAsync(ws, 0, ws_bytes, abm::as_stream(stream));
    if (e != hipSuccess) {
        abm::set_error("hipMemsetAsync: %s", hipGetErrorString(e));
        return ABM_E_HIP;
    }
    return ABM_OK;
}

}  // extern "C"
