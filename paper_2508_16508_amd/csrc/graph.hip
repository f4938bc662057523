// graph.hip -- multi-step batched rollouts captured once as a HIP graph and
// replayed: the counterpart of the paper's jit-compiled multi-step scans over
// vectorised models (Sec. 2), done here with one graph launch per rollout.
//
// The capture runs on a stream the library creates for it (a caller's
// default stream cannot be captured), records n_chunks launches of
// abm_predation_run_batched, and instantiates the graph.  Every pointer the
// launches use is baked into the graph: the handle owns the graph, not the
// buffers, which the caller keeps alive and in place until it destroys the
// handle.  The batched launches contain no memset nodes (queue counters are
// reset by a kernel), so replays need no re-arming.
#include <hip/hip_runtime.h>

#include <new>

#include "abm.h"
#include "common.hpp"

struct abm_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int device;
};

using namespace abm;

namespace {

int hip_fail(hipError_t e, const char* where) {
    set_error("%s: %s", where, hipGetErrorString(e));
    return ABM_E_HIP;
}

}  // namespace

extern "C" int abm_predation_batched_graph(const abm_batch* b, const int32_t* order,
                                           int32_t chunk_steps, int32_t n_chunks,
                                           const abm_tuning* tune, void* ws, size_t ws_bytes,
                                           abm_graph** out) {
    if (!out) return fail(ABM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!b) return fail(ABM_E_INVALID, "batch is NULL");
    if (chunk_steps < 1 || n_chunks < 1 || n_chunks > 65536)
        return fail(ABM_E_INVALID, "chunk_steps must be >= 1 and n_chunks in [1, 65536]");
    int rc = check_device();
    if (rc != ABM_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    for (int32_t i = 0; i < n_chunks && rc == ABM_OK; ++i)
        rc = abm_predation_run_batched(b, order, chunk_steps, tune, ws, ws_bytes, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (rc != ABM_OK) {   // the message of the failed launch stays the last error
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    abm_graph* h = new (std::nothrow) abm_graph{g, x, dev};
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(ABM_E_HIP, "out of host memory");
    }
    *out = h;
    return ABM_OK;
}

extern "C" int abm_graph_replay(abm_graph* g, void* stream) {
    if (!g) return fail(ABM_E_INVALID, "graph is NULL");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != g->device) return fail(ABM_E_INVALID, "graph was captured on another device");
    e = hipGraphLaunch(g->exec, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return ABM_OK;
}

extern "C" int abm_graph_destroy(abm_graph* g) {
    if (!g) return ABM_OK;
    hipError_t e1 = hipGraphExecDestroy(g->exec);
    hipError_t e2 = hipGraphDestroy(g->graph);
    delete g;
    if (e1 != hipSuccess) return hip_fail(e1, "hipGraphExecDestroy");
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphDestroy");
    return ABM_OK;
}
