// A forward pass recorded once as a HIP graph and replayed with one launch.
//
// At a small batch (one slot) the GPU finishes each of the forward's kernels faster than the
// host can enqueue the next, so the host's launch path sets the latency. A graph captures the
// whole launch sequence of conet_forward for fixed shapes and buffers (the kernels, their
// arguments and their order; no memsets or copies are recorded on this path) and replays it
// with a single hipGraphLaunch: the device walks the dependent kernels back to back.
#include <hip/hip_runtime.h>

#include <new>

#include "conet.h"
#include "conet_model.h"

struct conet_graph {
  conet_model* model = nullptr;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace conet;

static void graph_free(conet_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->capture) (void)hipStreamDestroy(g->capture);
  delete g;
}

extern "C" conet_status conet_graph_create(conet_model* M, const float* x, int32_t B, int32_t T, int32_t F,
                                           float* llr, conet_graph** out) {
  if (!out) return fail(CONET_EINVAL, "null output handle");
  *out = nullptr;
  if (!M || !x || !llr) return fail(CONET_EINVAL, "null argument");
  if (B < 1 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad shape B=%d T=%d F=%d", B, T, F);
  if ((int64_t)B * T * F > M->cfg.max_res) return fail(CONET_ESHAPE, "B*T*F exceeds max_res");
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales");
  conet_graph* g = new (std::nothrow) conet_graph();
  if (!g) return fail(CONET_ENOMEM, "host allocation failed");
  g->model = M;
  hipError_t e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    graph_free(g);
    return hip_fail(e, "graph capture start");
  }
  Geometry geo;
  geo.uniform = true; geo.B = B; geo.T = T; geo.F = F;
  const conet_status st = run_forward(M, M->arena, x, geo, llr, g->capture, nullptr);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->capture, &graph);  // ends the capture also when recording failed
  g->graph = graph;
  if (st != CONET_OK) {
    graph_free(g);
    return st;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    graph_free(g);
    return hip_fail(e, "graph capture");
  }
  *out = g;
  return CONET_OK;
}

extern "C" conet_status conet_graph_launch(conet_graph* g, void* stream) {
  if (!g || !g->exec) return fail(CONET_EINVAL, "null graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  return e == hipSuccess ? CONET_OK : hip_fail(e, "graph launch");
}

extern "C" conet_status conet_graph_destroy(conet_graph* g) {
  if (!g) return fail(CONET_EINVAL, "null graph");
  graph_free(g);
  return CONET_OK;
}
