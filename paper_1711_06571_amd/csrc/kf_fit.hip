// Seed (FP64) and fit (FP32) kernels: one lane per track over SoA buffers.
#include "kfdev.h"
#include "kfhost.h"

using namespace kfdev;

namespace {

struct GeomK {
  int n_layers;
  float r[32];
  float z_half, bz, x_over_x0, mass;
};

GeomK to_k(const kf_geometry* g) {
  GeomK k;
  k.n_layers = g->n_layers;
  for (int i = 0; i < 32; ++i) k.r[i] = g->r[i];
  k.z_half = g->z_half;
  k.bz = g->bz;
  k.x_over_x0 = g->x_over_x0;
  k.mass = g->mass;
  return k;
}

// Seed from layers 0..2 in FP64.  Circle through the three transverse
// points, direction tangent at hit 0 with the turning sense of the charge,
// tan(lambda) from the arc between hits 0 and 2, then the Kalman filter over
// the three hits from a broad prior on the surface.
__global__ void __launch_bounds__(256) seed_kernel(GeomK g, int n, int ld, const float* __restrict__ hits,
                                                   int8_t* __restrict__ q_out, float* __restrict__ seed_par,
                                                   float* __restrict__ seed_cov, int32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double h[3][9];
  bool fin = true;
  for (int l = 0; l < 3; ++l)
    for (int c = 0; c < 9; ++c) {
      h[l][c] = (double)hits[((size_t)l * 9 + c) * ld + i];
      fin = fin && k_finite(h[l][c]);
    }
  int st = fin ? 0 : KF_NONFINITE;
  int q = 1;
  double X[6] = {0, 0, 0, 0, 0, 0}, P[21];
  for (int k = 0; k < 21; ++k) P[k] = 0.0;
  if (!st) {
    const double x1 = h[0][0], y1 = h[0][1], z1 = h[0][2];
    const double bx = h[1][0] - x1, by = h[1][1] - y1;
    const double cx = h[2][0] - x1, cy = h[2][1] - y1;
    const double D = 2.0 * (bx * cy - by * cx);
    if (!(fabs(D) > 0.0)) st = KF_NO_CROSSING;
    if (!st) {
      const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
      const double ux = (cy * b2 - by * c2) / D, uy = (bx * c2 - cx * b2) / D;
      const double rho = sqrt(ux * ux + uy * uy);
      const double cross = bx * (h[2][1] - h[1][1]) - by * (h[2][0] - h[1][0]);
      q = cross < 0.0 ? 1 : -1;
      const double pt = kappa<double>() * fabs((double)g.bz) * rho;
      const double r1x = -ux, r1y = -uy;
      double tx, ty;
      if (cross > 0.0) { tx = -r1y / rho; ty = r1x / rho; }
      else { tx = r1y / rho; ty = -r1x / rho; }
      const double r3x = cx - ux, r3y = cy - uy;
      const double dal = fabs(atan2(r1x * r3y - r1y * r3x, r1x * r3x + r1y * r3y));
      const double tanl = (h[2][2] - z1) / (rho * dal);
      double X0[6] = {x1, y1, z1, pt * tx, pt * ty, pt * tanl};
      const double p2 = X0[3] * X0[3] + X0[4] * X0[4] + X0[5] * X0[5];
      const double r0 = sqrt(x1 * x1 + y1 * y1);
      const double ttx = -y1 / r0, tty = x1 / r0;
      for (int k = 0; k < 21; ++k) P[k] = 0.0;
      P[ut(0, 0)] = ttx * ttx;
      P[ut(0, 1)] = ttx * tty;
      P[ut(1, 1)] = tty * tty;
      P[ut(2, 2)] = 100.0;
      P[ut(3, 3)] = p2;
      P[ut(4, 4)] = p2;
      P[ut(5, 5)] = p2;
      // scattering on layer 0 (the prior sits at hit 0)
      if (g.x_over_x0 > 0.f) {
        const double p = sqrt(p2);
        const double cospsi = fabs((X0[0] * X0[3] + X0[1] * X0[4]) / (r0 * p));
        const double xe = (double)g.x_over_x0 / cospsi;
        const double beta2 = p2 / (p2 + (double)g.mass * (double)g.mass);
        const double th0 = 0.0136 / (sqrt(beta2) * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / beta2));
        const double t2 = th0 * th0;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) P[ut(3 + a, 3 + b)] += t2 * ((a == b ? p2 : 0.0) - X0[3 + a] * X0[3 + b]);
      }
      for (int k = 0; k < 6; ++k) X[k] = X0[k];
      for (int l = 0; l < 3 && !st; ++l) {
        if (l > 0) {
          double Xp[6], Pp[21];
          int rc = predict<double>(X, P, q, (double)g.r[l], (double)g.bz, (double)g.z_half, (double)g.x_over_x0,
                                   (double)g.mass, Xp, Pp);
          if (rc) { st = rc; break; }
          for (int k = 0; k < 6; ++k) X[k] = Xp[k];
          for (int k = 0; k < 21; ++k) P[k] = Pp[k];
        }
        Innov<double> in;
        const double V[6] = {h[l][3], h[l][4], h[l][5], h[l][6], h[l][7], h[l][8]};
        if (innovation<double>(X, P, h[l][0], h[l][1], h[l][2], V, in)) { st = KF_S_NOT_PD; break; }
        apply_update<double>(X, P, in);
      }
      if (!st && !(all_finite(X, 6) && all_finite(P, 21))) st = KF_NONFINITE;
    }
  }
  if (st) {  // failed seed: zero state and covariance, q = +1
    for (int k = 0; k < 6; ++k) X[k] = 0.0;
    for (int k = 0; k < 21; ++k) P[k] = 0.0;
    q = 1;
  }
  q_out[i] = (int8_t)q;
  status[i] = st;
  for (int k = 0; k < 6; ++k) seed_par[(size_t)k * ld + i] = (float)X[k];
  for (int k = 0; k < 21; ++k) seed_cov[(size_t)k * ld + i] = (float)P[k];
}

// Fit: one lane per track, layers looped in registers.  Storage is FP32;
// T is the arithmetic type (float, or double for the precise mode).
template <typename T>
__global__ void __launch_bounds__(256, (sizeof(T) == 8 ? 2 : 1)) fit_kernel(GeomK g, int n, int ld, int first_layer,
                                                  const float* __restrict__ hits,
                                                  const uint32_t* __restrict__ hole_mask,
                                                  const float* seed_par, const float* seed_cov,
                                                  const int8_t* __restrict__ qv, float* out_par, float* out_cov,
                                                  float* __restrict__ out_chi2, int32_t* __restrict__ out_ndof,
                                                  int32_t* __restrict__ out_status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T X[6], P[21];
#pragma unroll
  for (int k = 0; k < 6; ++k) X[k] = (T)seed_par[(size_t)k * ld + i];
#pragma unroll
  for (int k = 0; k < 21; ++k) P[k] = (T)seed_cov[(size_t)k * ld + i];
  const int q = qv[i];
  const uint32_t holes = hole_mask ? hole_mask[i] : 0u;
  T chi2 = 0;
  int ndof = 0;
  int st = (all_finite(X, 6) && all_finite(P, 21)) ? 0 : KF_NONFINITE;
  for (int l = first_layer; l < g.n_layers && !st; ++l) {
    const bool use = !((holes >> l) & 1u);
    float hv[9];  // kept in the storage type until the update
    if (use) {
      const float* hl = hits + (size_t)l * 9 * ld + i;
#pragma unroll
      for (int c = 0; c < 9; ++c) hv[c] = __builtin_nontemporal_load(hl + (size_t)c * ld);
      if (!all_finite(hv, 9)) { st = KF_NONFINITE; break; }
    }
    T Xp[6], Pp[21];
    int rc = predict<T>(X, P, q, (T)g.r[l], (T)g.bz, (T)g.z_half, (T)g.x_over_x0, (T)g.mass, Xp, Pp);
    if (rc) { st = rc; break; }
    if (use) {
      Innov<T> in;
      const T V[6] = {(T)hv[3], (T)hv[4], (T)hv[5], (T)hv[6], (T)hv[7], (T)hv[8]};
      if (innovation<T>(Xp, Pp, (T)hv[0], (T)hv[1], (T)hv[2], V, in)) { st = KF_S_NOT_PD; break; }
      const T c2 = chi2_of(in);
      apply_update<T>(Xp, Pp, in);
      if (!(all_finite(Xp, 6) && all_finite(Pp, 21) && k_finite(c2))) { st = KF_NONFINITE; break; }
      chi2 += c2;
      ndof += 2;
    } else if (!(all_finite(Xp, 6) && all_finite(Pp, 21))) {
      st = KF_NONFINITE;
      break;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = Xp[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = Pp[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) out_par[(size_t)k * ld + i] = (float)X[k];
#pragma unroll
  for (int k = 0; k < 21; ++k) out_cov[(size_t)k * ld + i] = (float)P[k];
  out_chi2[i] = (float)chi2;
  out_ndof[i] = ndof;
  out_status[i] = st;
}

int check_geometry(const kf_geometry* g) {
  if (!g || g->n_layers < 1 || g->n_layers > 32 || !(g->bz != 0.f) || !(g->z_half > 0.f)) return KF_E_INVALID_ARG;
  for (int l = 0; l < g->n_layers; ++l) {
    if (!(g->r[l] > 0.f)) return KF_E_INVALID_ARG;
    if (l > 0 && !(g->r[l] > g->r[l - 1])) return KF_E_INVALID_ARG;
  }
  return KF_OK;
}

}  // namespace

int kf_check_geometry(const kf_geometry* g) { return check_geometry(g); }

extern "C" int kf_seed(const kf_geometry* g, int32_t n, int32_t ld, const float* hits, int8_t* q_out,
                       float* seed_par, float* seed_cov, int32_t* status, void* stream) {
  if (check_geometry(g)) return KF_E_INVALID_ARG;
  if (n < 0 || ld < n || g->n_layers < 3) return KF_E_INVALID_ARG;
  if (n == 0) return KF_OK;
  if (!hits || !q_out || !seed_par || !seed_cov || !status) return KF_E_INVALID_ARG;
  const int bs = 256;
  hipLaunchKernelGGL(seed_kernel, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g), n, ld, hits,
                     q_out, seed_par, seed_cov, status);
  return kf_check_launch();
}

extern "C" int kf_fit(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
                      const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                      float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof, int32_t* out_status,
                      int32_t arith, void* stream) {
  if (check_geometry(g)) return KF_E_INVALID_ARG;
  if (n < 0 || ld < n || first_layer < 0 || first_layer > g->n_layers) return KF_E_INVALID_ARG;
  if (arith != KF_ARITH_F32 && arith != KF_ARITH_F64) return KF_E_INVALID_ARG;
  if (n == 0) return KF_OK;
  if (!hits || !seed_par || !seed_cov || !q || !out_par || !out_cov || !out_chi2 || !out_ndof || !out_status)
    return KF_E_INVALID_ARG;
  const int bs = 256;
  if (arith == KF_ARITH_F64)
    hipLaunchKernelGGL(fit_kernel<double>, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g), n, ld,
                       first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2, out_ndof,
                       out_status);
  else
    hipLaunchKernelGGL(fit_kernel<float>, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g), n, ld,
                       first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2, out_ndof,
                       out_status);
  return kf_check_launch();
}

namespace {

// Gather the hit rows of built tracks into the fit layout.  Layer l of seed i
// takes the built hit (event-local index) or, if none, a hole bit.
__global__ void __launch_bounds__(256) gather_kernel(int n_layers, int first_layer, int n, int ld,
                                                     const int32_t* __restrict__ built,
                                                     const int32_t* __restrict__ seed_event,
                                                     const int32_t* __restrict__ event_offsets, int n_events,
                                                     int n_hits, const float* __restrict__ xyz,
                                                     const float* __restrict__ cov, float* __restrict__ fit_hits,
                                                     uint32_t* __restrict__ hole_mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int e = seed_event ? seed_event[i] : 0;
  const bool ev_ok = e >= 0 && e < n_events;
  const int base = (ev_ok && event_offsets) ? event_offsets[e] : 0;
  const int end = (ev_ok && event_offsets) ? event_offsets[e + 1] : n_hits;
  uint32_t holes = 0;
  for (int l = first_layer; l < n_layers; ++l) {
    const int h = built[(size_t)(l - first_layer) * ld + i];
    const int g = base + h;
    float* row = fit_hits + (size_t)l * 9 * ld + i;
    if (!ev_ok || h < 0 || g >= end) {
      holes |= 1u << l;
      for (int c = 0; c < 9; ++c) row[(size_t)c * ld] = 0.f;
      continue;
    }
    for (int c = 0; c < 3; ++c) row[(size_t)c * ld] = xyz[(size_t)c * n_hits + g];
    for (int c = 0; c < 6; ++c) row[(size_t)(3 + c) * ld] = cov[(size_t)c * n_hits + g];
  }
  hole_mask[i] = holes;
}

}  // namespace

extern "C" int kf_gather_hits(int32_t n_layers, int32_t first_layer, int32_t n_seeds, int32_t ld,
                              const int32_t* built_hits, const int32_t* seed_event, int32_t n_events,
                              const int32_t* event_offsets, int32_t n_hits, const float* xyz, const float* cov,
                              float* fit_hits, uint32_t* hole_mask, void* stream) {
  if (n_layers < 1 || n_layers > 32 || first_layer < 0 || first_layer >= n_layers) return KF_E_INVALID_ARG;
  if (n_seeds < 0 || ld < n_seeds || n_events < 1 || n_hits < 0) return KF_E_INVALID_ARG;
  if (n_events > 1 && (!seed_event || !event_offsets)) return KF_E_INVALID_ARG;
  if (n_seeds == 0) return KF_OK;
  if (!built_hits || !fit_hits || !hole_mask || (n_hits > 0 && (!xyz || !cov))) return KF_E_INVALID_ARG;
  const int bs = 256;
  hipLaunchKernelGGL(gather_kernel, dim3((n_seeds + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, n_layers,
                     first_layer, n_seeds, ld, built_hits, seed_event, event_offsets, n_events, n_hits, xyz, cov,
                     fit_hits, hole_mask);
  return kf_check_launch();
}
