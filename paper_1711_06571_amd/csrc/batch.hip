// Batched building of many uneven events as one replayable HIP graph: the
// binning of every event and the single persistent build launch (which
// balances seeds of all events through its atomic queue, the GPU analogue of
// several events in flight and work stealing, sections 3.2, 4.2 and 4.3) are
// captured once from the caller's stream and replayed with hipGraphLaunch.
// The step plan adds the final fit of the built hit lists (section 2):
// gather of the lists into fit rows, then the fit.
#include <new>

#include "kfhost.h"

struct kf_batch_plan {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

// Capture of binning, build and (optionally) the final fit of the built
// lists from `stream`, then instantiation.
int plan_create(const kf_geometry* g, const kf_build_params* bp, int32_t n_events, const int32_t* event_offsets,
                int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov, const kf_hits* binned,
                int32_t* binned_offsets, float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig, void* bin_ws,
                size_t bin_ws_bytes, int32_t n_seeds, int32_t ld, const float* seed_par, const float* seed_cov,
                const int8_t* q, int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2,
                int32_t* out_nhits, int32_t* out_status, const kf_build_extra* extra, void* build_ws,
                size_t build_ws_bytes, const kf_fit_stage* fit, void* stream, kf_batch_plan** plan) {
  if (!plan || !binned || !g || !bp) return KF_E_INVALID_ARG;
  *plan = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return KF_E_INVALID_ARG;  // the null stream cannot be captured
  if (fit && (!fit->fit_hits || !fit->hole_mask || !fit->out_par || !fit->out_cov || !fit->out_chi2 ||
              !fit->out_ndof || !fit->out_status || (fit->arith != KF_ARITH_F32 && fit->arith != KF_ARITH_F64)))
    return KF_E_INVALID_ARG;
  if (fit && n_events > 1 && (!extra || !extra->seed_event)) return KF_E_INVALID_ARG;
  if (kf_check(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed))) return KF_E_HIP;
  int rc = hit_bin(g, n_events, event_offsets, binned->n_phi, binned->n_z, n_hits, layer, xyz, cov, binned_offsets,
                   sorted_xyzphi, sorted_cov, sorted_orig, nullptr, bin_ws, bin_ws_bytes, stream);
  if (rc == KF_OK)
    rc = kf_build(g, bp, binned, n_seeds, ld, seed_par, seed_cov, q, out_hits, out_par, out_cov, out_chi2, out_nhits,
                  out_status, extra, build_ws, build_ws_bytes, stream);
  if (rc == KF_OK && fit)
    rc = kf_gather_hits(g->n_layers, bp->first_layer, n_seeds, ld, out_hits, extra ? extra->seed_event : nullptr,
                        n_events, event_offsets, n_hits, xyz, cov, fit->fit_hits, fit->hole_mask, stream);
  if (rc == KF_OK && fit)  // the fit in the state of the build
    rc = (bp->state == 1 ? kf_fit_hybrid : kf_fit)(g, n_seeds, ld, bp->first_layer, fit->fit_hits, fit->hole_mask,
                                                   seed_par, seed_cov, q, fit->out_par, fit->out_cov, fit->out_chi2,
                                                   fit->out_ndof, fit->out_status, fit->arith, stream);
  hipGraph_t graph = nullptr;
  const int rc_end = kf_check(hipStreamEndCapture(s, &graph));
  if (rc != KF_OK || rc_end != KF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != KF_OK ? rc : rc_end;
  }
  hipGraphExec_t exec = nullptr;
  if (kf_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0))) {
    (void)hipGraphDestroy(graph);
    return KF_E_HIP;
  }
  kf_batch_plan* p = new (std::nothrow) kf_batch_plan;
  if (!p) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return KF_E_HIP;
  }
  p->graph = graph;
  p->exec = exec;
  *plan = p;
  return KF_OK;
}

}  // namespace

extern "C" int kf_batch_plan_create(const kf_geometry* g, const kf_build_params* bp, int32_t n_events,
                                    const int32_t* event_offsets, int32_t n_hits, const int32_t* layer,
                                    const float* xyz, const float* cov, const kf_hits* binned,
                                    int32_t* binned_offsets, float* sorted_xyzphi, float* sorted_cov,
                                    int32_t* sorted_orig, void* bin_ws, size_t bin_ws_bytes, int32_t n_seeds,
                                    int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q,
                                    int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2,
                                    int32_t* out_nhits, int32_t* out_status, const kf_build_extra* extra,
                                    void* build_ws, size_t build_ws_bytes, void* stream, kf_batch_plan** plan) {
  return plan_create(g, bp, n_events, event_offsets, n_hits, layer, xyz, cov, binned, binned_offsets, sorted_xyzphi,
                     sorted_cov, sorted_orig, bin_ws, bin_ws_bytes, n_seeds, ld, seed_par, seed_cov, q, out_hits,
                     out_par, out_cov, out_chi2, out_nhits, out_status, extra, build_ws, build_ws_bytes, nullptr,
                     stream, plan);
}

extern "C" int kf_step_plan_create(const kf_geometry* g, const kf_build_params* bp, int32_t n_events,
                                   const int32_t* event_offsets, int32_t n_hits, const int32_t* layer,
                                   const float* xyz, const float* cov, const kf_hits* binned,
                                   int32_t* binned_offsets, float* sorted_xyzphi, float* sorted_cov,
                                   int32_t* sorted_orig, void* bin_ws, size_t bin_ws_bytes, int32_t n_seeds,
                                   int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q,
                                   int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2,
                                   int32_t* out_nhits, int32_t* out_status, const kf_build_extra* extra,
                                   void* build_ws, size_t build_ws_bytes, const kf_fit_stage* fit, void* stream,
                                   kf_batch_plan** plan) {
  if (!fit) return KF_E_INVALID_ARG;
  return plan_create(g, bp, n_events, event_offsets, n_hits, layer, xyz, cov, binned, binned_offsets, sorted_xyzphi,
                     sorted_cov, sorted_orig, bin_ws, bin_ws_bytes, n_seeds, ld, seed_par, seed_cov, q, out_hits,
                     out_par, out_cov, out_chi2, out_nhits, out_status, extra, build_ws, build_ws_bytes, fit, stream,
                     plan);
}

extern "C" int kf_batch_plan_launch(kf_batch_plan* plan, void* stream) {
  if (!plan) return KF_E_INVALID_ARG;
  return kf_check(hipGraphLaunch(plan->exec, (hipStream_t)stream));
}

extern "C" int kf_batch_plan_destroy(kf_batch_plan* plan) {
  if (!plan) return KF_OK;
  int rc = kf_check(hipGraphExecDestroy(plan->exec));
  int rc2 = kf_check(hipGraphDestroy(plan->graph));
  delete plan;
  return rc != KF_OK ? rc : rc2;
}

extern "C" int kf_wall_clock_khz(int32_t* khz) {
  if (!khz) return KF_E_INVALID_ARG;
  int dev = 0, v = 0;
  if (kf_check(hipGetDevice(&dev))) return KF_E_HIP;
  if (kf_check(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev))) return KF_E_HIP;
  *khz = v;
  return KF_OK;
}
