// HIP graphs of library calls: a capture bracket around calls issued on a
// stream, and replay of the instantiated graph.  The entry points record
// kernel launches only (fills are kernels, not memset nodes), so a replay
// redoes every step of the captured calls, counters and queues included.
#include <new>

#include "../../include/sigkernel.h"
#include "internal.h"

struct sk_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

sk_status sigkernel_graph_begin(void* stream) {
  if (!stream) return SK_ERR_NULL;  // the NULL stream cannot be captured
  if (hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal) !=
      hipSuccess)
    return SK_ERR_HIP;
  return SK_OK;
}

sk_status sigkernel_graph_end(void* stream, sk_graph* graph) {
  if (!stream || !graph) return SK_ERR_NULL;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    return SK_ERR_HIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return SK_ERR_HIP;
  }
  sk_graph h = new (std::nothrow) sk_graph_s{g, x};
  if (!h) {
    hipGraphExecDestroy(x);
    hipGraphDestroy(g);
    return SK_ERR_HIP;
  }
  *graph = h;
  return SK_OK;
}

sk_status sigkernel_graph_launch(sk_graph graph, void* stream) {
  if (!graph) return SK_ERR_NULL;
  return hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? SK_OK
                                                                                      : SK_ERR_HIP;
}

sk_status sigkernel_graph_destroy(sk_graph graph) {
  if (!graph) return SK_ERR_NULL;
  const bool ok =
      hipGraphExecDestroy(graph->exec) == hipSuccess && hipGraphDestroy(graph->graph) == hipSuccess;
  delete graph;
  return ok ? SK_OK : SK_ERR_HIP;
}

}  // extern "C"
