// Recording of library calls into HIP graphs (stream capture) and replay.
#include <hip/hip_runtime.h>

#include "common.h"

struct mpwsd_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int mpwsd_graph_begin(hipStream_t* record_stream)
{
    mpwsd::clear_error();
    if (!record_stream) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_graph_begin: record_stream is NULL");
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_graph_begin: %s", hipGetErrorString(e));
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_graph_begin: %s", hipGetErrorString(e));
    }
    *record_stream = s;
    return MPWSD_OK;
}

extern "C" int mpwsd_graph_end(hipStream_t record_stream, mpwsd_graph** out)
{
    mpwsd::clear_error();
    if (!record_stream || !out) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_graph_end: null argument");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(record_stream, &g);
    (void)hipStreamDestroy(record_stream);
    if (e != hipSuccess || !g) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_graph_end: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_graph_end: instantiate: %s", hipGetErrorString(e));
    }
    *out = new mpwsd_graph{g, x};
    return MPWSD_OK;
}

extern "C" int mpwsd_graph_launch(const mpwsd_graph* graph, hipStream_t stream)
{
    mpwsd::clear_error();
    if (!graph) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_graph_launch: graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, stream);
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_graph_launch: %s", hipGetErrorString(e));
    return MPWSD_OK;
}

extern "C" int mpwsd_graph_destroy(mpwsd_graph* graph)
{
    mpwsd::clear_error();
    if (!graph) return MPWSD_OK;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return MPWSD_OK;
}
