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

// Seed from layers 0..2 in FP64.  With a beam spot (bs > 0: tracks leave
// the z axis within bs cm transversely) the first circle passes through the
// axis point and hits 0 and 2, and the first Kalman step is the 1-D
// measurement "transverse impact parameter = 0" (variance bs^2); without it
// the circle passes through the three hits.  Direction tangent at hit 0 with
// the turning sense of the charge, tan(lambda) from the arc between hits 0
// and 2, then the Kalman filter over the three hits from a broad prior on
// the surface; the state at layer 2 is the seed.
__device__ inline void beam_constraint(double X[6], double P[21], int q, double bz, double bs, int& st) {
  // impact parameter f = |c| - rho of the circle about c = (x + py/k, y - px/k)
  const double k = (double)q * kappa<double>() * bz, ik = 1.0 / k, aik = fabs(ik);
  const double cx = X[0] + X[4] * ik, cy = X[1] - X[3] * ik;
  const double cn = sqrt(cx * cx + cy * cy), pt = sqrt(X[3] * X[3] + X[4] * X[4]);
  if (!(cn > 0.0) || !(pt > 0.0)) { st = KF_NO_CROSSING; return; }
  const double icn = 1.0 / cn, ipt = 1.0 / pt;
  const double f = cn - pt * aik;
  double H[6] = {cx * icn, cy * icn, 0.0, -cy * ik * icn - X[3] * ipt * aik, cx * ik * icn - X[4] * ipt * aik, 0.0};
  double PH[6];
  for (int i = 0; i < 6; ++i) {
    double a = 0.0;
    for (int j = 0; j < 6; ++j) a += P[ut(i, j)] * H[j];
    PH[i] = a;
  }
  double S = bs * bs;
  for (int i = 0; i < 6; ++i) S += H[i] * PH[i];
  if (!(S > 0.0)) { st = KF_S_NOT_PD; return; }
  const double iS = 1.0 / S;
  for (int i = 0; i < 6; ++i) X[i] -= PH[i] * iS * f;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) P[ut(i, j)] -= PH[i] * PH[j] * iS;
}

__global__ void __launch_bounds__(256) seed_kernel(GeomK g, int n, int ld, const float* __restrict__ hits, double bs,
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
  const bool beam = bs > 0.0;
  const double bz = (double)g.bz;
  if (!st) {
    // circle points A, B, C: the axis point (or hit 0), hit 0 (or hit 1), hit 2
    const double Ax = beam ? 0.0 : h[0][0], Ay = beam ? 0.0 : h[0][1];
    const double Bx = beam ? h[0][0] : h[1][0], By = beam ? h[0][1] : h[1][1];
    const double Cx = h[2][0], Cy = h[2][1];
    const double e1x = Bx - Ax, e1y = By - Ay, e2x = Cx - Ax, e2y = Cy - Ay;
    const double D = 2.0 * (e1x * e2y - e1y * e2x);
    if (!(fabs(D) > 0.0)) st = KF_NO_CROSSING;
    if (!st) {
      const double l1 = e1x * e1x + e1y * e1y, l2 = e2x * e2x + e2y * e2y;
      const double ox = Ax + (e2y * l1 - e1y * l2) / D, oy = Ay + (e1x * l2 - e2x * l1) / D;  // centre
      const double r1x = h[0][0] - ox, r1y = h[0][1] - oy, r3x = h[2][0] - ox, r3y = h[2][1] - oy;
      const double rho = sqrt(r1x * r1x + r1y * r1y);
      const double turn = e1x * (Cy - By) - e1y * (Cx - Bx);  // > 0: counter-clockwise
      q = ((turn < 0.0) == (bz > 0.0)) ? 1 : -1;
      const double pt = kappa<double>() * fabs(bz) * rho;
      const double tx = (turn > 0.0 ? -r1y : r1y) / rho, ty = (turn > 0.0 ? r1x : -r1x) / rho;
      const double dal = fabs(atan2(r1x * r3y - r1y * r3x, r1x * r3x + r1y * r3y));
      const double tanl = (h[2][2] - h[0][2]) / (rho * dal);
      X[0] = h[0][0]; X[1] = h[0][1]; X[2] = h[0][2];
      X[3] = pt * tx; X[4] = pt * ty; X[5] = pt * tanl;
      const double p2 = X[3] * X[3] + X[4] * X[4] + X[5] * X[5];
      const double r0 = sqrt(X[0] * X[0] + X[1] * X[1]);
      const double ttx = -X[1] / r0, tty = X[0] / r0;
      P[ut(0, 0)] = ttx * ttx;
      P[ut(0, 1)] = ttx * tty;
      P[ut(1, 1)] = tty * tty;
      P[ut(2, 2)] = 100.0;
      P[ut(3, 3)] = p2;
      P[ut(4, 4)] = p2;
      P[ut(5, 5)] = p2;
      if (beam) beam_constraint(X, P, q, bz, bs, st);
    }
    if (!st) {
      // scattering on layer 0 (the prior sits at hit 0)
      if (g.x_over_x0 > 0.f) {
        const double pp2 = X[3] * X[3] + X[4] * X[4] + X[5] * X[5];
        const double p = sqrt(pp2);
        const double r0 = sqrt(X[0] * X[0] + X[1] * X[1]);
        const double cospsi = fabs((X[0] * X[3] + X[1] * X[4]) / (r0 * p));
        const double xe = (double)g.x_over_x0 / cospsi;
        const double beta2 = pp2 / (pp2 + (double)g.mass * (double)g.mass);
        const double th0 = 0.0136 / (sqrt(beta2) * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / beta2));
        const double t2 = th0 * th0;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) P[ut(3 + a, 3 + b)] += t2 * ((a == b ? pp2 : 0.0) - X[3 + a] * X[3 + b]);
      }
      for (int l = 0; l < 3 && !st; ++l) {
        if (l > 0) {
          double Xp[6], Pp[21];
          int rc = predict<double>(X, P, q, (double)g.r[l], bz, (double)g.z_half, (double)g.x_over_x0,
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
// T is the arithmetic type (float, or double for the precise mode).  HYB:
// the state is the hybrid one (x, y, z, q/pT, phi, theta), entered from the
// Cartesian seed and returned as it is.
template <typename T, bool HYB>
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
  if constexpr (HYB) {
    T Y[6], B[9];
    hyb_from_cart(X, q, Y, B);
    congruence_mom(P, B);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = Y[k];
  }
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
    int rc;
    if constexpr (HYB)
      rc = predict_hyb<T>(X, P, (T)g.r[l], (T)g.bz, (T)g.z_half, (T)g.x_over_x0, (T)g.mass, Xp, Pp);
    else
      rc = predict<T>(X, P, q, (T)g.r[l], (T)g.bz, (T)g.z_half, (T)g.x_over_x0, (T)g.mass, Xp, Pp);
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

extern "C" int kf_seed(const kf_geometry* g, int32_t n, int32_t ld, const float* hits, float beam_sigma,
                       int8_t* q_out, float* seed_par, float* seed_cov, int32_t* status, void* stream) {
  if (check_geometry(g)) return KF_E_INVALID_ARG;
  if (n < 0 || ld < n || g->n_layers < 3 || !(beam_sigma >= 0.f)) return KF_E_INVALID_ARG;
  if (n == 0) return KF_OK;
  if (!hits || !q_out || !seed_par || !seed_cov || !status) return KF_E_INVALID_ARG;
  const int bs = 256;
  hipLaunchKernelGGL(seed_kernel, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g), n, ld, hits,
                     (double)beam_sigma, q_out, seed_par, seed_cov, status);
  return kf_check_launch();
}

namespace {

template <bool HYB>
int fit_launch(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
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
    hipLaunchKernelGGL((fit_kernel<double, HYB>), dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g),
                       n, ld, first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                       out_ndof, out_status);
  else
    hipLaunchKernelGGL((fit_kernel<float, HYB>), dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, to_k(g),
                       n, ld, first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                       out_ndof, out_status);
  return kf_check_launch();
}

}  // namespace

extern "C" int kf_fit(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
                      const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                      float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof, int32_t* out_status,
                      int32_t arith, void* stream) {
  return fit_launch<false>(g, n, ld, first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                           out_ndof, out_status, arith, stream);
}

extern "C" int kf_fit_hybrid(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
                             const uint32_t* hole_mask, const float* seed_par, const float* seed_cov,
                             const int8_t* q, float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof,
                             int32_t* out_status, int32_t arith, void* stream) {
  return fit_launch<true>(g, n, ld, first_layer, hits, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                          out_ndof, out_status, arith, stream);
}

namespace {

// Gather the hit rows of built tracks into the fit layout.  Layer l of seed i
// takes the built hit (event-local index) or, if none, a hole bit.  One lane
// per (seed, layer): the rows and the built indices are read and written
// coalesced along the seeds; the hit reads are the only scattered access.
// Blocks are dispatched to the 8 XCDs in turn (block index mod 8): block b
// takes seed chunk x * cpx + (k mod cpx) of layer first_layer + k / cpx
// (x = b mod 8, k = b / 8, cpx chunks per XCD), so each XCD gathers for its
// own eighth of the seeds, a few events at a time, whose hits stay in its L2.
__global__ void __launch_bounds__(256) gather_kernel(int n_layers, int first_layer, int n, int ld, int cpx,
                                                     const int32_t* __restrict__ built,
                                                     const int32_t* __restrict__ seed_event,
                                                     const int32_t* __restrict__ event_offsets, int n_events,
                                                     int n_hits, const float* __restrict__ xyz,
                                                     const float* __restrict__ cov, float* __restrict__ fit_hits) {
  const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int i = (x * cpx + k % cpx) * blockDim.x + threadIdx.x;
  const int l = first_layer + k / cpx;
  if (i >= n || l >= n_layers) return;
  const int e = seed_event ? seed_event[i] : 0;
  const bool ev_ok = e >= 0 && e < n_events;
  const int base = (ev_ok && event_offsets) ? event_offsets[e] : 0;
  const int end = (ev_ok && event_offsets) ? event_offsets[e + 1] : n_hits;
  const int h = built[(size_t)(l - first_layer) * ld + i];
  float* row = fit_hits + (size_t)l * 9 * ld + i;
  if (!ev_ok || h < 0 || h >= end - base) {  // (no overflow of base + h)
#pragma unroll
    for (int c = 0; c < 9; ++c) row[(size_t)c * ld] = 0.f;
    return;
  }
  const int g = base + h;
  float v[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = xyz[(size_t)c * n_hits + g];
#pragma unroll
  for (int c = 0; c < 6; ++c) v[3 + c] = cov[(size_t)c * n_hits + g];
#pragma unroll
  for (int c = 0; c < 9; ++c) row[(size_t)c * ld] = v[c];
}

// Hole mask of each built track: bit l set where layer l has no usable hit
// (the same test as the gather).
__global__ void __launch_bounds__(256) hole_mask_kernel(int n_layers, int first_layer, int n, int ld,
                                                        const int32_t* __restrict__ built,
                                                        const int32_t* __restrict__ seed_event,
                                                        const int32_t* __restrict__ event_offsets, int n_events,
                                                        int n_hits, uint32_t* __restrict__ hole_mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e = seed_event ? seed_event[i] : 0;
  const bool ev_ok = e >= 0 && e < n_events;
  const int base = (ev_ok && event_offsets) ? event_offsets[e] : 0;
  const int end = (ev_ok && event_offsets) ? event_offsets[e + 1] : n_hits;
  uint32_t holes = 0;
  for (int l = first_layer; l < n_layers; ++l) {
    const int h = built[(size_t)(l - first_layer) * ld + i];
    if (!ev_ok || h < 0 || h >= end - base) holes |= 1u << l;
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
  const int chunks = (n_seeds + bs - 1) / bs, cpx = (chunks + 7) / 8;
  hipLaunchKernelGGL(gather_kernel, dim3(8 * cpx * (n_layers - first_layer)), dim3(bs), 0, (hipStream_t)stream,
                     n_layers, first_layer, n_seeds, ld, cpx, built_hits, seed_event, event_offsets, n_events, n_hits,
                     xyz, cov, fit_hits);
  if (int rc = kf_check_launch()) return rc;
  hipLaunchKernelGGL(hole_mask_kernel, dim3((n_seeds + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, n_layers,
                     first_layer, n_seeds, ld, built_hits, seed_event, event_offsets, n_events, n_hits, hole_mask);
  return kf_check_launch();
}
