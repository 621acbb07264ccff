// HIP graphs of a plan's step, and the launch-shape autotuner.
//
// Every count the kernels need (survivors, tiles, partial ranges) is computed
// and read on the device and the work-queue counters are cleared by a kernel,
// so the launches of a step do not depend on the poses: one graph replays the
// step for any poses written into the same query buffer.
#include <algorithm>

#include "runtime.h"

struct cm_graph {
  cm_context* ctx = nullptr;
  cm_plan* plan = nullptr;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace cm;

extern "C" {

cm_status cm_graph_create(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups out, cm_groups cot,
                          float* grad, const float* dir, float* hv, cm_graph** result) {
  if (!ctx || !pl || pl->ctx != ctx || !result) return fail(ctx, CM_E_INVALID, "bad arguments");
  *result = nullptr;
  auto* g = new cm_graph;
  g->ctx = ctx;
  g->plan = pl;
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return fail(ctx, CM_E_HIP, "graph stream creation failed");
  }
  const bool timing = pl->timing;
  pl->timing = false;  // events are not recorded into the graph
  cm_status st = CM_OK;
  hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = cm_contacts_step(ctx, pl, q, out, cot, grad, dir, hv, g->stream);
    e = hipStreamEndCapture(g->stream, &g->graph);
  }
  pl->timing = timing;
  if (st == CM_OK && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (st != CM_OK || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipStreamDestroy(g->stream);
    delete g;
    (void)hipGetLastError();
    return st != CM_OK ? st : hip_fail(ctx, e, "graph capture");
  }
  *result = g;
  return CM_OK;
}

cm_status cm_graph_launch(cm_graph* g, void* stream) {
  if (!g) return CM_E_INVALID;
  const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(g->ctx, e, "graph launch");
  return CM_OK;
}

cm_status cm_graph_destroy(cm_graph* g) {
  if (!g) return CM_E_INVALID;
  (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  (void)hipStreamDestroy(g->stream);
  delete g;
  return CM_OK;
}

cm_status cm_plan_autotune(cm_context* ctx, cm_plan* pl, const cm_query* q, cm_groups cot, float* grad,
                           const float* dir, float* hv, void* stream, int32_t* best) {
  if (!ctx || !pl || pl->ctx != ctx) return fail(ctx, CM_E_INVALID, "bad arguments");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(ctx, CM_E_HIP, "event creation failed");
  }
  // the sweeps this step runs: workgroups per CU and waves per workgroup
  int32_t& shape = dir ? pl->blocks_per_cu_dual : pl->blocks_per_cu;
  int32_t& waves = dir ? pl->wg_waves_dual : pl->wg_waves;
  const int32_t keep_shape = shape, keep_waves = waves;
  cm_status st = CM_OK;
  // one warm step, then two timed ones (records not written)
  auto time_it = [&](int32_t c, int32_t v, float* ms) -> bool {
    shape = c;
    waves = v;
    st = cm_contacts_step(ctx, pl, q, cm_groups{}, cot, grad, dir, hv, stream);
    if (st != CM_OK) return false;
    if (hipEventRecord(a, s) != hipSuccess) { st = CM_E_HIP; return false; }
    for (int r = 0; r < 2 && st == CM_OK; ++r) st = cm_contacts_step(ctx, pl, q, cm_groups{}, cot, grad, dir, hv, stream);
    if (st != CM_OK || hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(ms, a, b) != hipSuccess) {
      if (st == CM_OK) st = CM_E_HIP;
      return false;
    }
    return true;
  };
  // resident waves per CU first (workgroups of 4 waves), then the workgroup
  // size at that many waves (1 or 2 waves per workgroup: finer dispatch)
  const int32_t cand[] = {2, 4, 6, 8, 12, 16};
  float best_ms = 3.4e38f;
  int32_t pick_c = keep_shape, pick_v = keep_waves;
  bool ok = true;
  for (int32_t c : cand) {
    float ms = 0.f;
    if (!(ok = time_it(c, 4, &ms))) break;
    if (ms < best_ms) { best_ms = ms; pick_c = c; pick_v = 4; }
  }
  const int32_t per_cu = pick_c * 4;  // waves per CU of the pick
  for (int32_t v : {2, 1}) {
    if (!ok) break;
    float ms = 0.f;
    if (!(ok = time_it(per_cu / v, v, &ms))) break;
    if (ms < best_ms) { best_ms = ms; pick_c = per_cu / v; pick_v = v; }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  shape = ok ? pick_c : keep_shape;
  waves = ok ? pick_v : keep_waves;
  if (best) *best = shape;
  return ok ? CM_OK : fail(ctx, st, "autotune failed");
}

cm_status cm_plan_set_launch_shape(cm_plan* pl, int32_t float_per_cu, int32_t dual_per_cu) {
  if (!pl) return CM_E_INVALID;
  if (float_per_cu < 1 || float_per_cu > 64 || dual_per_cu < 1 || dual_per_cu > 64)
    return fail(pl->ctx, CM_E_INVALID, "launch shape outside [1, 64] workgroups per CU");
  pl->blocks_per_cu = float_per_cu;
  pl->blocks_per_cu_dual = dual_per_cu;
  return CM_OK;
}

cm_status cm_plan_launch_shape(const cm_plan* pl, int32_t* float_per_cu, int32_t* dual_per_cu) {
  if (!pl) return CM_E_INVALID;
  if (float_per_cu) *float_per_cu = pl->blocks_per_cu;
  if (dual_per_cu) *dual_per_cu = pl->blocks_per_cu_dual;
  return CM_OK;
}

cm_status cm_plan_set_wg_waves(cm_plan* pl, int32_t float_waves, int32_t dual_waves) {
  if (!pl) return CM_E_INVALID;
  auto ok = [](int32_t v) { return v == 1 || v == 2 || v == 4; };
  if (!ok(float_waves) || !ok(dual_waves)) return fail(pl->ctx, CM_E_INVALID, "waves per workgroup must be 1, 2 or 4");
  pl->wg_waves = float_waves;
  pl->wg_waves_dual = dual_waves;
  return CM_OK;
}

cm_status cm_plan_wg_waves(const cm_plan* pl, int32_t* float_waves, int32_t* dual_waves) {
  if (!pl) return CM_E_INVALID;
  if (float_waves) *float_waves = pl->wg_waves;
  if (dual_waves) *dual_waves = pl->wg_waves_dual;
  return CM_OK;
}

}  // extern "C"
