// Combinatorial track building (placeholder until the kernel lands).
#include "kfhost.h"

extern "C" size_t kf_build_workspace_bytes(int32_t n_seeds, int32_t n_events) {
  (void)n_seeds;
  (void)n_events;
  return 256;
}

extern "C" int kf_build(const kf_geometry* g, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds,
                        int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q, int32_t* out_hits,
                        float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits, int32_t* out_status,
                        const kf_build_extra* extra, void* ws, size_t ws_bytes, void* stream) {
  return KF_E_UNSUPPORTED;
}
