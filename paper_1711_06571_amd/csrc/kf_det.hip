// Fitting and combinatorial building over a general detector (section 4.1:
// the barrel closed by endcap disks, modules off the average surface of their
// layer), with two-step propagation in the build.
//
// The fit is one lane per track over SoA rows, as the barrel fit, with the
// step, Jacobian, scattering and update of the layer's kind.
//
// The build keeps the barrel builder's layout of the work (cand_cap
// consecutive lanes per seed, a persistent queue of seed groups, per-lane
// lists of the best accepted hits in LDS, a cooperative hit search, a merge
// of the seed's children by 64-bit rank keys, back-pointer tables) and
// changes what a step is:
//   - candidates of one seed may sit on different layers: each finds its own
//     next layer (the first after its current one whose average surface the
//     helix meets inside the layer's extent), so the history is indexed by
//     step and every entry records its layer;
//   - step 1 goes to the layer's average surface, where the window is formed
//     in (phi, w), w = z on a barrel layer and r on a disk;
//   - step 2 is inside the hit search: the lane that tests a (candidate, hit)
//     pair reads the candidate's state on the average surface from LDS,
//     moves it to the hit's own surface and computes the chi2 there;
//   - every candidate ends in the seed's best-finished record.
#include <stdint.h>

#include "kfdet.h"
#include "kfdev.h"
#include "kfhost.h"
#include "kfwave.h"

using namespace kfdev;

namespace {

struct DetK {
  int n_layers;
  int kind[32];
  float pos[32], lo[32], hi[32], dmod[32];
  float bz, x_over_x0, mass;
};

DetK det_k(const kf_detector* d) {
  DetK k = {};
  k.n_layers = d->n_layers;
  for (int i = 0; i < 32; ++i) {
    k.kind[i] = i < d->n_layers ? d->kind[i] : 0;
    k.pos[i] = d->pos[i];
    k.lo[i] = d->lo[i];
    k.hi[i] = d->hi[i];
    k.dmod[i] = d->dmod[i];
  }
  k.bz = d->bz;
  k.x_over_x0 = d->x_over_x0;
  k.mass = d->mass;
  return k;
}

__host__ __device__ inline bool finite_f(float v) { return __builtin_isfinite(v); }

// ------------------------------------------------------------------- fit

template <typename T>
__global__ void __launch_bounds__(256, (sizeof(T) == 8 ? 2 : 1))
    fit_det_kernel(DetK d, int n, int ld, int first_layer, const float* __restrict__ hits,
                   const uint32_t* __restrict__ visit_mask, const uint32_t* __restrict__ hole_mask,
                   const float* seed_par, const float* seed_cov, const int8_t* __restrict__ qv, float* out_par,
                   float* out_cov, float* __restrict__ out_chi2, int32_t* __restrict__ out_ndof,
                   int32_t* __restrict__ out_status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T X[6], P[21];
#pragma unroll
  for (int k = 0; k < 6; ++k) X[k] = (T)seed_par[(size_t)k * ld + i];
#pragma unroll
  for (int k = 0; k < 21; ++k) P[k] = (T)seed_cov[(size_t)k * ld + i];
  const int q = qv[i];
  const uint32_t visit = visit_mask[i];
  const uint32_t holes = hole_mask ? hole_mask[i] : 0u;
  T chi2 = 0;
  int ndof = 0;
  int st = (all_finite(X, 6) && all_finite(P, 21)) ? 0 : KF_NONFINITE;
  for (int l = first_layer; l < d.n_layers && !st; ++l) {
    if (!((visit >> l) & 1u)) continue;
    const int kind = d.kind[l];
    const bool use = !((holes >> l) & 1u);
    float hv[9];
    if (use) {
      const float* hl = hits + (size_t)l * 9 * ld + i;
#pragma unroll
      for (int c = 0; c < 9; ++c) hv[c] = __builtin_nontemporal_load(hl + (size_t)c * ld);
      if (!all_finite(hv, 9)) { st = KF_NONFINITE; break; }
    }
    // the surface: the hit's own (its radius or its z), else the layer's average
    T value = (T)d.pos[l];
    if (use) value = kind == KIND_DISK ? (T)hv[2] : k_sqrt((T)hv[0] * (T)hv[0] + (T)hv[1] * (T)hv[1]);
    T Xp[6], Pp[21];
    const int rc = surf_predict<T, false>(kind, X, P, q, value, (T)d.bz, true, (T)d.x_over_x0, (T)d.mass, Xp, Pp);
    if (rc) { st = rc; break; }
    if (use) {
      const T V[6] = {(T)hv[3], (T)hv[4], (T)hv[5], (T)hv[6], (T)hv[7], (T)hv[8]};
      T c2 = 0;
      if (update_kind<T>(kind, Xp, Pp, (T)hv[0], (T)hv[1], (T)hv[2], V, c2)) { st = KF_S_NOT_PD; break; }
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

// ----------------------------------------------------------------- build

struct DetBuildArgs {
  DetK d;
  float chi2_cut;
  int max_holes, cap;
  float nsigma, win_sig_rphi, win_sig_w;
  int first_layer;
  int n_events, n_phi, n_w;
  const int32_t* offsets;  // [events][layers][n_phi * n_w + 1]
  const float4* hpack;  // packed hits: (phi, x, y, z), (cov 0..3), (cov 4, cov 5, orig bits, 0)
  int refine;
  const int32_t* fine;  // [events][layers][n_w][n_phi * refine + 1]
  uint32_t* hist;       // [resident waves][steps][64] back-pointers
  int n_seeds, ld, n_groups;
  const float *seed_par, *seed_cov;
  const int8_t* q;
  const int32_t* seed_event;
  const int32_t* seed_order;
  int32_t* out_hits;
  uint32_t* out_visit;
  float *out_par, *out_cov, *out_chi2;
  int32_t *out_nhits, *out_status;
  unsigned long long* counters;
  int32_t* queue;
};

// history entry: parent slot (3 bits), layer (5 bits), hit index (24 bits)
__device__ inline uint32_t det_hist(int parent, int layer, uint32_t orig24) {
  return ((uint32_t)parent << 29) | ((uint32_t)layer << 24) | (orig24 & 0xFFFFFFu);
}

// LDS of one block (byte offsets), per wave:
//   stash    [27][64] f32   each slot's state before this step (for the record)
//   cand     [27][64] f32   each slot's state on its layer's average surface
//                           (step 1), read by the lanes that test its hits
//   record   [SEEDS][27] f32, recfield [SEEDS][5] i32 (valid, nhits, status,
//                           last step, slot)
//   starts   [64] i32       run starts of the cooperative hit search
//   publish  [64] f32 chi2, [64] u32 indices of a round's admissible hits
//   toplist  [cap][64] f32 chi2, i32 positions, u32 indices
struct DetLds {
  size_t stash, cand, rec, recf, acc, pub, tl, total;
};
__host__ __device__ inline size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }
__host__ __device__ inline DetLds det_lds(int nwaves, int cap) {
  const int seeds = 64 / cap;
  DetLds p;
  p.stash = 0;
  p.cand = al16(p.stash + (size_t)nwaves * 27 * 64 * 4);
  p.rec = al16(p.cand + (size_t)nwaves * 27 * 64 * 4);
  p.recf = al16(p.rec + (size_t)nwaves * seeds * 27 * 4);
  p.acc = al16(p.recf + (size_t)nwaves * seeds * 5 * 4);
  p.pub = al16(p.acc + (size_t)nwaves * 64 * 4);
  p.tl = al16(p.pub + (size_t)nwaves * 64 * 8);
  p.total = al16(p.tl + (size_t)nwaves * cap * 64 * 12);
  return p;
}

// The next layer of a candidate on layer `cur`: the first j > cur whose
// average surface the helix crosses ahead (a disk: moving outwards, within
// less than half a turn) inside the layer's extent.  Returns j and the state
// and covariance there (no material), or -1 when the candidate leaves.
template <typename T>
__device__ inline int next_layer(const DetK& d, int cur, const T X[6], const T P[21], int q, T Xa[6], T Pa[21]) {
  for (int j = cur + 1; j < d.n_layers; ++j) {
    const int kind = d.kind[j];
    Step<T> st;
    if (surf_step<T, false>(kind, X, q, (T)d.pos[j], (T)d.bz, Xa, st)) continue;
    T w;
    if (kind == KIND_DISK) {
      const T pr = Xa[0] * Xa[3] + Xa[1] * Xa[4];
      if (!(pr > T(0)) || !(fabs(st.alpha) < T(3.14159265358979323846))) continue;
      w = k_sqrt(Xa[0] * Xa[0] + Xa[1] * Xa[1]);
    } else {
      w = Xa[2];
    }
    if (!(w >= (T)d.lo[j] && w <= (T)d.hi[j])) continue;
#pragma unroll
    for (int k = 0; k < 21; ++k) Pa[k] = P[k];
    T J[6][6];
    if (kind == KIND_DISK) {
      surf_jacobian<T, true>(X, Xa, st, J);
      sandwich<T, true>(J, Pa);
    } else {
      surf_jacobian<T, false>(X, Xa, st, J);
      sandwich<T, false>(J, Pa);
    }
    return j;
  }
  return -1;
}

// chi2 of a hit for a candidate whose state on the layer's average surface
// is (Xa, Pa), after step 2 to the hit's surface (FP32).  The scattering added
// at the hit changes only the momentum block, which the measurement does not
// see, so S = M Pa M^T + V2 with M the measured rows of the surface Jacobian.
// Returns false where the step or S fails (the hit is then not accepted).
template <bool DISK>
__device__ inline bool pair_chi2(const float Xa[6], const float Pa[21], int q, float bz, float hx, float hy, float hz,
                                 const float V[6], float& c2) {
  float Xh[6];
  Step<float> st;
  if (DISK) {
    if (plane_step<float, true>(Xa, q, hz, bz, Xh, st)) return false;
  } else {
    if (propagate<float, true>(Xa, q, __builtin_sqrtf(hx * hx + hy * hy), bz, Xh, st)) return false;
  }
  float J[6][6];
  surf_jacobian<float, DISK>(Xa, Xh, st, J);
  float M0[6], M1[6], r0, r1, v00, v01, v11;
  if (DISK) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      M0[k] = jac_nz(true, 0, k) ? J[0][k] : 0.f;
      M1[k] = jac_nz(true, 1, k) ? J[1][k] : 0.f;
    }
    r0 = hx - Xh[0];
    r1 = hy - Xh[1];
    v00 = V[0];
    v01 = V[1];
    v11 = V[3];
  } else {
    const float ir = kfdev::k_rcp(__builtin_sqrtf(Xh[0] * Xh[0] + Xh[1] * Xh[1]));
    const float tx = -Xh[1] * ir, ty = Xh[0] * ir;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      M0[k] = jac_nz(false, 0, k) ? tx * J[0][k] + ty * J[1][k] : 0.f;
      M1[k] = J[2][k];
    }
    r0 = tx * (hx - Xh[0]) + ty * (hy - Xh[1]);
    r1 = hz - Xh[2];
    v00 = tx * tx * V[0] + 2.f * tx * ty * V[1] + ty * ty * V[3];
    v01 = tx * V[2] + ty * V[4];
    v11 = V[5];
  }
  float u0[6], u1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      a += Pa[ut(i, k)] * M0[k];
      b += Pa[ut(i, k)] * M1[k];
    }
    u0[i] = a;
    u1[i] = b;
  }
  float s00 = v00, s01 = v01, s11 = v11;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    s00 += M0[i] * u0[i];
    s01 += M0[i] * u1[i];
    s11 += M1[i] * u1[i];
  }
  const float det = s00 * s11 - s01 * s01;
  if (!(s00 > 0.f) || !(det > 0.f)) return false;
  c2 = (s11 * r0 * r0 - 2.f * s01 * r0 * r1 + s00 * r1 * r1) * k_rcp(det);  // hardware reciprocal
  return true;
}

// Hit search of every candidate of the wave on its own next layer: as the
// barrel builder's cooperative search (ranges of sorted positions from the
// fine phi index per (layer, w row) and phi interval, pairs of all candidates
// handed out 64 at a time, the pair's candidate from run-start marks,
// the round's admissible hits placed in the lists by rank), one pair per lane and
// round, with the window test in (phi, w) and the chi2 after step 2.
template <typename T>
__device__ inline void coop_scan_det(const DetBuildArgs& A, int ev, int lj, int kind, bool pok, int q, const T Xa[6],
                                     T dphi_w, T dw_w, T wp, const float* cand, TopList& tl, const AccBuf& ab,
                                     int lane) {
  const int nw = A.n_w, nf = A.n_phi * A.refine;
  const float inv = fine_inv(nf);
  const float tp = 6.283185307179586f;
  float a0 = 1.f, b0v = 0.f, a1 = 1.f, b1v = 0.f;
  int iw0 = 0, iw1 = -1;
  float fx = 0.f, fy = 0.f, fw = 0.f, fdw = 0.f, fdphi = 0.f, ftan = 0.f;
  if (pok) {
    fx = (float)Xa[0];
    fy = (float)Xa[1];
    fw = (float)wp;
    fdw = (float)dw_w;
    fdphi = (float)dphi_w;
    const float phip = wrap_2pi(atan2f(fy, fx));
    const float dphi = fdphi + 1e-5f, dw = fdw + 1e-4f;
    const float lo = A.d.lo[lj], hi = A.d.hi[lj];
    const float sc = (float)nw / (hi - lo);
    float f0 = floorf((fw - dw - lo) * sc), f1 = floorf((fw + dw - lo) * sc);
    // clamped in FP32 before the conversion: an infinite or undefined width
    // covers every row (the exact test then decides)
    f0 = f0 > 0.f ? (f0 < (float)(nw - 1) ? f0 : (float)(nw - 1)) : 0.f;
    f1 = f1 < (float)(nw - 1) ? (f1 > 0.f ? f1 : 0.f) : (float)(nw - 1);
    iw0 = (int)f0;
    iw1 = (int)f1;
    if (!(dphi < 3.14159f)) { a0 = 0.f; b0v = tp; }
    else {
      const float plo = phip - dphi, phi_ = phip + dphi;
      if (plo < 0.f) { a0 = 0.f; b0v = phi_; a1 = plo + tp; b1v = tp; }
      else if (phi_ >= tp) { a0 = plo; b0v = tp; a1 = 0.f; b1v = phi_ - tp; }
      else { a0 = plo; b0v = phi_; }
    }
    ftan = !(dphi_w < T(1.5707963267948966)) ? -1.f : tanf((float)dphi_w);
  }
  const int32_t* frow = A.fine + ((size_t)ev * A.d.n_layers + (pok ? lj : 0)) * nw * (nf + 1);
  const int nint = a1 <= b1v ? 2 : 1;
  const int R = pok ? (iw1 - iw0 + 1) * nint : 0;
  const int Rmax = wave_max(R);
  int n_acc = 0;  // accepted hits of this lane's candidate
  int held = 0;
  bool unsorted = false;  // entries appended out of order
  float thr_c2 = __builtin_inff();
  uint32_t thr_o = 0xFFFFFFFFu;
  const float cut = A.chi2_cut;
  const float bz = A.d.bz;
  auto range_of = [&](int r, float& a, float& b, int& q0, int& q1) {
    a = 1.f;
    b = 0.f;
    q0 = 0;
    q1 = 0;
    if (r < R) {
      const int ri = nint == 2 ? (r & 1) : 0, rr = nint == 2 ? (r >> 1) : r;
      a = ri ? a1 : a0;
      b = ri ? b1v : b0v;
      if (a <= b) {
        const int32_t* f = frow + (size_t)(iw0 + rr) * (nf + 1);
        q0 = f[fine_key(a, inv, nf)];
        q1 = f[fine_key(b, inv, nf) + 1];
      }
    }
  };
  float an = 1.f, bn = 0.f;
  int p0n = 0, p1n = 0;
  range_of(0, an, bn, p0n, p1n);
  for (int r = 0; r < Rmax; ++r) {
    const float a = an, b = bn;
    const int p0 = p0n, p1 = p1n;
    range_of(r + 1, an, bn, p0n, p1n);
    const int cnt = p1 > p0 ? p1 - p0 : 0;
    int total = 0;
    const int off = wave_excl_scan(cnt, lane, total);
    const int pb = p0 - off;
    int carry = 0;
    for (int base = 0; base < total; base += 64) {
      ab.start[lane] = -1;
      if (cnt > 0 && off >= base && off - base < 64) ab.start[off - base] = lane;
      __builtin_amdgcn_wave_barrier();
      const int stv = ab.start[lane];
      const unsigned long long sma = __ballot(stv >= 0);
      const unsigned long long sm = sma & ((2ull << lane) - 1ull);
      const int hb = sm ? 63 - (int)__builtin_clzll(sm) : 0;
      const int sc = __shfl(stv, hb, 64);
      const int c = sm ? sc : carry;
      const int my_lo = sm ? hb : 0;
      carry = __builtin_amdgcn_readlane(c, 63);
      const int k = base + lane;
      const bool valid = k < total;
      const int p = __shfl(pb, c, 64) + k;
      const float ca = __shfl(a, c, 64), cb = __shfl(b, c, 64);
      const float cx = __shfl(fx, c, 64), cy = __shfl(fy, c, 64), cw = __shfl(fw, c, 64);
      const float cdw = __shfl(fdw, c, 64), cdphi = __shfl(fdphi, c, 64), ctan = __shfl(ftan, c, 64);
      const int ckind = __shfl(kind, c, 64), cq = __shfl(q, c, 64);
      const float cthr = __shfl(thr_c2, c, 64);
      const uint32_t cthro = (uint32_t)__shfl((int)thr_o, c, 64);
      const int p_first = __builtin_amdgcn_readfirstlane(__shfl(p, 0, 64));
      const float4* hp = A.hpack + (size_t)(valid ? p : p_first) * 3;
      const float4 u0 = hp[0], u1 = hp[1], u2 = hp[2];
      bool keep = false, acc = false;
      float c2 = 0.f;
      uint32_t orig = 0;
      if (valid && u0.x >= ca && u0.x <= cb) {
        tl.scanned += 1;
        const float hx = u0.y, hy = u0.z, hz = u0.w;
        const float cr = cx * hy - cy * hx, dt = cx * hx + cy * hy;
        const bool in_phi = ctan < 0.f ? fabsf(atan2f(cr, dt)) <= cdphi : (dt > 0.f && fabsf(cr) <= ctan * dt);
        const float hw = ckind == KIND_DISK ? __builtin_sqrtf(hx * hx + hy * hy) : hz;
        if (fabsf(hw - cw) <= cdw && in_phi) {
          tl.tested += 1;
          float Xc[6], Pc[21];
#pragma unroll
          for (int m = 0; m < 6; ++m) Xc[m] = cand[m * 64 + c];
#pragma unroll
          for (int m = 0; m < 21; ++m) Pc[m] = cand[(6 + m) * 64 + c];
          const float V[6] = {u1.x, u1.y, u1.z, u1.w, u2.x, u2.y};
          const bool ok = ckind == KIND_DISK ? pair_chi2<true>(Xc, Pc, cq, bz, hx, hy, hz, V, c2)
                                             : pair_chi2<false>(Xc, Pc, cq, bz, hx, hy, hz, V, c2);
          if (ok && c2 < cut) {
            acc = true;
            orig = __float_as_uint(u2.z);
            keep = top_before(c2, orig, cthr, cthro);
          }
        }
      }
      // this lane's run as a candidate in the round: lanes [s0, e0); its
      // accepted hits are the accepted lanes of the run
      const int s0 = off - base > 0 ? off - base : 0;
      const int e0 = off + cnt - base < 64 ? off + cnt - base : 64;
      const unsigned long long am = __ballot(acc);
      if (s0 < e0) n_acc += __builtin_popcountll(am & run_mask(s0, e0));
      const unsigned long long m = __ballot(keep);
      if (m) {
        // the run of this lane's pair: from its candidate's mark to the next
        const unsigned long long above = sma & ~((2ull << lane) - 1ull);
        const int rhi = above ? (int)__builtin_ctzll(above) : 64;
        round_insert(tl, A.cap, lane, m, keep, c2, p, orig, c, my_lo, rhi, s0, e0, held, unsorted, thr_c2, thr_o,
                     ab.pub_c2, ab.pub_o);
      }
    }
  }
  if (unsorted) sort_own(tl, A.cap, held);
  tl.n = held;
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  tl.tot = n_acc;
}

// Waves per SIMD the register allocation aims at: the FP64 kernel at two
// spilled 888 bytes per lane and ran slower than at one without spills
// (16 lids events: 15.06 -> 13.26 ms); the FP32 kernel needs the second wave
// (12.0 ms against 17.0 at one).
#ifndef KF_BUILD_DET_F64_WAVES
#define KF_BUILD_DET_F64_WAVES 1
#endif
#ifndef KF_BUILD_DET_F32_WAVES
#define KF_BUILD_DET_F32_WAVES 2
#endif

template <typename T>
__global__ void __launch_bounds__(256, sizeof(T) == 8 ? KF_BUILD_DET_F64_WAVES : KF_BUILD_DET_F32_WAVES)
    build_det_kernel(DetBuildArgs A) {
  const int S = A.cap;
  const int SEEDS = 64 / S;
  extern __shared__ __align__(16) uint32_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int L = A.d.n_layers, F = A.first_layer, LB = L - F;
  const DetLds lp = det_lds(nwaves, S);
  char* base = (char*)lds;
  uint32_t* hist = A.hist + ((size_t)blockIdx.x * nwaves + wave) * LB * 64;
  float* stash = (float*)(base + lp.stash) + (size_t)wave * 27 * 64;
  float* cand = (float*)(base + lp.cand) + (size_t)wave * 27 * 64;
  float* fin = (float*)(base + lp.rec) + (size_t)wave * SEEDS * 27;
  int32_t* finm = (int32_t*)(base + lp.recf) + (size_t)wave * SEEDS * 5;
  char* wave_tl = base + lp.tl + (size_t)wave * S * 64 * 12;
  float* tl_c2 = (float*)wave_tl + lane;
  int32_t* tl_pos = (int32_t*)(wave_tl + (size_t)S * 64 * 4) + lane;
  uint32_t* tl_orig = (uint32_t*)(wave_tl + (size_t)S * 64 * 8) + lane;
  AccBuf ab;
  ab.start = (int32_t*)(base + lp.acc) + (size_t)wave * 64;
  ab.pub_c2 = (float*)(base + lp.pub) + (size_t)wave * 128;
  ab.pub_o = (uint32_t*)ab.pub_c2 + 64;
  const int sidx = lane / S, slot = lane - (lane / S) * S, sbase = sidx * S;
  const bool lane_used = sidx < SEEDS;
  const T bz = (T)A.d.bz, x0 = (T)A.d.x_over_x0, mass = (T)A.d.mass;

  for (;;) {
    int grp = 0;
    if (lane == 0) grp = atomicAdd(A.queue, 1);
    grp = __shfl(grp, 0, 64);
    if (grp >= A.n_groups) break;
    const int gi = grp * SEEDS + sidx;
    int seed = (lane_used && gi < A.n_seeds) ? (A.seed_order ? A.seed_order[gi] : gi) : -1;
    int ev = (seed >= 0 && seed < A.n_seeds && A.seed_event) ? A.seed_event[seed] : 0;
    const bool seed_ok = seed >= 0 && seed < A.n_seeds && ev >= 0 && ev < A.n_events;
    if (!seed_ok) { seed = 0; ev = 0; }
    const int q = seed_ok ? A.q[seed] : 1;
    T X[6], P[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = seed_ok ? (T)A.seed_par[(size_t)k * A.ld + seed] : T(0);
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = seed_ok ? (T)A.seed_cov[(size_t)k * A.ld + seed] : T(0);
    T chi2 = 0;
    int nhits = 0, holes = 0, cl = F - 1;
    int n_active = seed_ok ? 1 : 0;
    int seed_status = 0;
    if (lane_used && slot == 0) finm[sidx * 5 + 0] = 0;
    const int bad = !seed_ok ? 0
                    : event_too_large(A.offsets, ev, L, A.n_phi * A.n_w) ? KF_EVENT_TOO_LARGE
                    : !(all_finite(X, 6) && all_finite(P, 21))          ? KF_NONFINITE
                                                                        : 0;
    if (bad) {
      if (slot == 0) {
        finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = 0; finm[sidx * 5 + 2] = bad;
        finm[sidx * 5 + 3] = -1; finm[sidx * 5 + 4] = 0;
        for (int k = 0; k < 6; ++k) fin[sidx * 27 + k] = (float)X[k];
        for (int k = 0; k < 21; ++k) fin[sidx * 27 + 6 + k] = (float)P[k];
      }
      n_active = 0;
    }
    T fin_chi2_reg = 0;
    unsigned cnt_pred = 0, cnt_scan = 0, cnt_chi2 = 0, cnt_upd = 0;
    // each step moves every active candidate at least one layer outwards, so
    // LB + 1 steps stop them all
    for (int k = 0; k <= LB; ++k) {
      if (!__any(n_active > 0)) break;
      const bool live = slot < n_active;
      if (live) {
#pragma unroll
        for (int m = 0; m < 6; ++m) stash[m * 64 + lane] = (float)X[m];
#pragma unroll
        for (int m = 0; m < 21; ++m) stash[(6 + m) * 64 + lane] = (float)P[m];
      }
      // step 1: the next layer and the state on its average surface
      T Xa[6], Pa[21];
      int lj = -1;
      if (live) lj = next_layer<T>(A.d, cl, X, P, q, Xa, Pa);
      const bool pok = lj >= 0;
      if (!pok) {
#pragma unroll
        for (int m = 0; m < 6; ++m) Xa[m] = T(0);
#pragma unroll
        for (int m = 0; m < 21; ++m) Pa[m] = T(0);
      }
      const int kind = pok ? A.d.kind[lj] : 0;
      // window on the average surface, widened for the module offsets
      T dphi_w = T(0), dw_w = T(0), wp = T(0);
      if (pok) {
        const T ra = k_sqrt(Xa[0] * Xa[0] + Xa[1] * Xa[1]);
        const T tx = -Xa[1] / ra, ty = Xa[0] / ra, nx = Xa[0] / ra, ny = Xa[1] / ra;
        const T sr = (T)A.win_sig_rphi, sw = (T)A.win_sig_w;
        const T Stt = tx * tx * Pa[ut(0, 0)] + T(2) * tx * ty * Pa[ut(0, 1)] + ty * ty * Pa[ut(1, 1)] + sr * sr;
        const T pr = nx * Xa[3] + ny * Xa[4], pphi = tx * Xa[3] + ty * Xa[4];
        T Sww, slope_w, slope_phi;
        if (kind == KIND_DISK) {
          Sww = nx * nx * Pa[ut(0, 0)] + T(2) * nx * ny * Pa[ut(0, 1)] + ny * ny * Pa[ut(1, 1)] + sw * sw;
          slope_w = pr / Xa[5];
          slope_phi = pphi / (ra * Xa[5]);
        } else {
          Sww = Pa[ut(2, 2)] + sw * sw;
          slope_w = Xa[5] / pr;
          slope_phi = pphi / (ra * pr);
        }
        dphi_w = (T)A.nsigma * k_sqrt(Stt) / ra;
        dw_w = (T)A.nsigma * k_sqrt(Sww);
        const T dm = (T)A.d.dmod[lj];
        if (dm > T(0)) {
          dphi_w += dm * fabs(slope_phi);
          dw_w += dm * fabs(slope_w);
        }
        wp = kind == KIND_DISK ? ra : Xa[2];
#pragma unroll
        for (int m = 0; m < 6; ++m) cand[m * 64 + lane] = (float)Xa[m];
#pragma unroll
        for (int m = 0; m < 21; ++m) cand[(6 + m) * 64 + lane] = (float)Pa[m];
      }
      __builtin_amdgcn_wave_barrier();
      TopList tl;
      tl.c2 = tl_c2;
      tl.pos = tl_pos;
      tl.orig = tl_orig;
      tl.n = 0;
      tl.tot = 0;
      tl.scanned = 0;
      tl.tested = 0;
      coop_scan_det<T>(A, ev, lj, kind, pok, q, Xa, dphi_w, dw_w, wp, cand, tl, ab, lane);
      cnt_pred += pok ? 1u : 0u;
      cnt_scan += (unsigned)tl.scanned;
      cnt_chi2 += (unsigned)tl.tested;
      const bool hole_ok = pok && holes < A.max_holes;
      const int nchild = pok ? tl.tot + (hole_ok ? 1 : 0) : 0;
      // candidates that stop here (no next layer, or no child) compete for
      // the seed's record with their state before this step
      if (__any(live && nchild == 0)) {  // (most layers have none)
        const bool stopped = live && nchild == 0;
        const uint64_t fk = stopped ? make_key(nhits, (float)chi2, slot, 0) : kInfKey;
        const uint64_t best = group_min(fk, sbase, slot, S, lane_used);
        if (best != kInfKey) {
          const int ws = (int)((best >> 24) & 7);
          const int wl_ = sbase + ws;
          const T wc2 = shfl_t(chi2, wl_);
          const int wn = __shfl(nhits, wl_, 64);
          const int fvalid = finm[sidx * 5 + 0];
          const int fn = finm[sidx * 5 + 1];
          const T fc2 = shfl_t(fin_chi2_reg, sbase);
          const bool take = !fvalid || wn > fn || (wn == fn && wc2 < fc2);
          if (take) {
            if (slot == ws) {
              for (int m = 0; m < 27; ++m) fin[sidx * 27 + m] = stash[m * 64 + lane];
              finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = wn; finm[sidx * 5 + 2] = 0;
              finm[sidx * 5 + 3] = k - 1; finm[sidx * 5 + 4] = ws;
            }
            if (slot == 0) fin_chi2_reg = wc2;
          }
        }
      }
      // merge the seed's children, best first, into slots 0..cap-1
      int ptr = 0;
      bool hole_left = hole_ok;
      int my_parent = -1, my_pos = -1;
      uint32_t my_orig = kHoleIdx;
      T my_c2 = 0;
      int n_new = 0;
      for (int r = 0; r < A.cap; ++r) {
        uint64_t key = kInfKey;
        float hc2 = 0.f;
        int hpos = -1;
        uint32_t horig = kHoleIdx;
        if (pok) {
          if (ptr < tl.n) {
            top_get(tl, ptr, hc2, hpos, horig);
            key = make_key(nhits + 1, (float)(chi2 + (T)hc2), slot, horig);
          } else if (hole_left) {
            key = make_key(nhits, (float)chi2, slot, kHoleIdx);
          }
        }
        const uint64_t win = group_min(key, sbase, slot, S, lane_used);
        if (win == kInfKey) continue;
        const int ws = (int)((win >> 24) & 7);
        const int wl_ = sbase + ws;
        const int wpos = __shfl(hpos, wl_, 64);
        const T wc2 = (T)__shfl(hc2, wl_, 64);
        if (slot == ws) {
          if (ptr < tl.n) ptr += 1; else hole_left = false;
        }
        if (slot == r) {
          my_parent = ws;
          my_pos = wpos;
          my_orig = (uint32_t)(win & 0xFFFFFFu);
          my_c2 = wc2;
        }
        n_new = r + 1;
      }
      // children left after cap rounds (accepted hits beyond a full list
      // included): the seed's candidates were cut to cap
      {
        const bool left = pok && tl.tot - ptr + (hole_left ? 1 : 0) > 0;
        const unsigned long long lm = __ballot(left);
        if (lane_used && ((lm >> sbase) & ((1ull << S) - 1ull)) != 0ull) seed_status |= KF_CAP_TRUNC;
      }
      // new slots pull the parent's state on the average surface, then
      // step 2 to their hit's surface and the update (or the hole's scattering)
      const int src = sbase + (my_parent >= 0 ? my_parent : slot);
      T Xn[6], Pn[21];
#pragma unroll
      for (int m = 0; m < 6; ++m) Xn[m] = shfl_t(Xa[m], src);
#pragma unroll
      for (int m = 0; m < 21; ++m) Pn[m] = shfl_t(Pa[m], src);
      const T pchi2 = shfl_t(chi2, src);
      const int pnh = __shfl(nhits, src, 64), pho = __shfl(holes, src, 64), plj = __shfl(lj, src, 64);
      if (my_parent >= 0) {
        const int nk = A.d.kind[plj];
        const bool is_hole = my_orig == kHoleIdx;
        if (is_hole) {
          highland_add<T>(nk, Xn, Pn, x0, mass);
        } else {
          const float4* hp = A.hpack + (size_t)my_pos * 3;
          const float4 u0 = hp[0], u1 = hp[1], u2 = hp[2];
          const T hx = (T)u0.y, hy = (T)u0.z, hz = (T)u0.w;
          const T V[6] = {(T)u1.x, (T)u1.y, (T)u1.z, (T)u1.w, (T)u2.x, (T)u2.y};
          const T value = nk == KIND_DISK ? hz : k_sqrt(hx * hx + hy * hy);
          T Xh[6], Ph[21];
          // the step and S passed in the search's arithmetic; should either
          // fail here the candidate keeps its state on the average surface
          if (!surf_predict<T, true>(nk, Xn, Pn, q, value, bz, true, x0, mass, Xh, Ph)) {
            T c2u = 0;
            if (!update_kind<T>(nk, Xh, Ph, hx, hy, hz, V, c2u)) {
#pragma unroll
              for (int m = 0; m < 6; ++m) Xn[m] = Xh[m];
#pragma unroll
              for (int m = 0; m < 21; ++m) Pn[m] = Ph[m];
            }
          }
          cnt_upd += 1;
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) X[m] = Xn[m];
#pragma unroll
        for (int m = 0; m < 21; ++m) P[m] = Pn[m];
        chi2 = is_hole ? pchi2 : pchi2 + my_c2;
        nhits = is_hole ? pnh : pnh + 1;
        holes = is_hole ? pho + 1 : pho;
        cl = plj;
        hist[k * 64 + lane] = det_hist(my_parent, plj, my_orig);
      }
      n_active = n_new;
    }
    if (A.counters) {
      unsigned long long c[4] = {cnt_pred, cnt_scan, cnt_chi2, cnt_upd};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        unsigned long long v = c[m];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) atomicAdd(&A.counters[m], v);
      }
    }
    // every candidate has finished: the record is the result
    if (seed_ok && slot == 0) {
      const int fn = finm[sidx * 5 + 1];
      for (int m = 0; m < 6; ++m) A.out_par[(size_t)m * A.ld + seed] = fin[sidx * 27 + m];
      for (int m = 0; m < 21; ++m) A.out_cov[(size_t)m * A.ld + seed] = fin[sidx * 27 + 6 + m];
      A.out_chi2[seed] = (float)fin_chi2_reg;
      A.out_nhits[seed] = fn;
      A.out_status[seed] = finm[sidx * 5 + 2] | seed_status;
      for (int l = F; l < L; ++l) A.out_hits[(size_t)(l - F) * A.ld + seed] = -1;
      uint32_t visit = 0;
      int s = finm[sidx * 5 + 4];
      for (int st = finm[sidx * 5 + 3]; st >= 0; --st) {
        const uint32_t h = hist[st * 64 + sbase + s];
        const int layer = (int)((h >> 24) & 31u);
        const uint32_t o = h & 0xFFFFFFu;
        A.out_hits[(size_t)(layer - F) * A.ld + seed] = o == 0xFFFFFFu ? -1 : (int32_t)o;
        visit |= 1u << layer;
        s = (int)(h >> 29);
      }
      A.out_visit[seed] = visit;
    }
  }
}

template <typename T>
int launch_det(const DetBuildArgs& A, int lanes, int blocks, int hist_waves, hipStream_t s,
               kf_build_launch_info* info) {
  int dev = 0, max_lds = 0;
  if (kf_check(hipGetDevice(&dev))) return KF_E_HIP;
  if (kf_check(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev))) return KF_E_HIP;
  auto plan = [&](int ln) { return det_lds(ln / 64, A.cap).total; };
  if (lanes == 0) {
    lanes = 256;
    while (lanes > 64 && plan(lanes) > (size_t)max_lds) lanes /= 2;
  }
  const int nwaves = lanes / 64;
  const size_t lds = plan(lanes);
  if (lds > (size_t)max_lds) return KF_E_UNSUPPORTED;
  if (lds > (size_t)64 * 1024 &&
      kf_check(hipFuncSetAttribute((const void*)build_det_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds)))
    return KF_E_HIP;
  int cus = 0, per = 0;
  if (kf_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))) return KF_E_HIP;
  if (kf_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, build_det_kernel<T>, lanes, lds))) return KF_E_HIP;
  if (blocks <= 0) blocks = cus * (per > 0 ? per : 1);
  const int need = (A.n_groups + nwaves - 1) / nwaves;
  if (blocks > need) blocks = need;
  if (blocks > hist_waves / nwaves) blocks = hist_waves / nwaves;
  if (blocks < 1) return KF_E_WORKSPACE;
  if (info) {
    info->lanes_per_block = lanes;
    info->blocks = blocks;
    info->lds_bytes = (int32_t)lds;
    info->resident_blocks_per_cu = per;
    info->max_lds_per_block = max_lds;
  }
  hipLaunchKernelGGL(build_det_kernel<T>, dim3(blocks), dim3(lanes), lds, s, A);
  return kf_check_launch();
}

thread_local kf_build_launch_info g_last_det_launch = {};

int check_det(const kf_detector* d) {
  if (!d || d->n_layers < 1 || d->n_layers > 32 || !(d->bz != 0.f) || !finite_f(d->bz)) return KF_E_INVALID_ARG;
  for (int l = 0; l < d->n_layers; ++l) {
    if (d->kind[l] != KF_LAYER_BARREL && d->kind[l] != KF_LAYER_DISK) return KF_E_INVALID_ARG;
    if (!finite_f(d->pos[l]) || !finite_f(d->lo[l]) || !finite_f(d->hi[l]) || !(d->hi[l] > d->lo[l]))
      return KF_E_INVALID_ARG;
    if (d->kind[l] == KF_LAYER_BARREL && !(d->pos[l] > 0.f)) return KF_E_INVALID_ARG;
    if (!(d->dmod[l] >= 0.f) || !finite_f(d->dmod[l])) return KF_E_INVALID_ARG;
  }
  return KF_OK;
}

}  // namespace

int kf_check_detector(const kf_detector* d) { return check_det(d); }

extern "C" int kf_fit_det(const kf_detector* d, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
                          const uint32_t* visit_mask, const uint32_t* hole_mask, const float* seed_par,
                          const float* seed_cov, const int8_t* q, float* out_par, float* out_cov, float* out_chi2,
                          int32_t* out_ndof, int32_t* out_status, int32_t arith, void* stream) {
  if (check_det(d)) return KF_E_INVALID_ARG;
  if (n < 0 || ld < n || first_layer < 0 || first_layer > d->n_layers) return KF_E_INVALID_ARG;
  if (arith != KF_ARITH_F32 && arith != KF_ARITH_F64) return KF_E_INVALID_ARG;
  if (n == 0) return KF_OK;
  if (!hits || !visit_mask || !seed_par || !seed_cov || !q || !out_par || !out_cov || !out_chi2 || !out_ndof ||
      !out_status)
    return KF_E_INVALID_ARG;
  const int bs = 256;
  const DetK k = det_k(d);
  if (arith == KF_ARITH_F64)
    hipLaunchKernelGGL(fit_det_kernel<double>, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, k, n, ld,
                       first_layer, hits, visit_mask, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                       out_ndof, out_status);
  else
    hipLaunchKernelGGL(fit_det_kernel<float>, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream, k, n, ld,
                       first_layer, hits, visit_mask, hole_mask, seed_par, seed_cov, q, out_par, out_cov, out_chi2,
                       out_ndof, out_status);
  return kf_check_launch();
}

extern "C" int kf_build_det_last_launch(kf_build_launch_info* info) {
  if (!info) return KF_E_INVALID_ARG;
  *info = g_last_det_launch;
  return KF_OK;
}

extern "C" int kf_build_det(const kf_detector* d, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds,
                            int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q,
                            int32_t* out_hits, uint32_t* out_visit, float* out_par, float* out_cov, float* out_chi2,
                            int32_t* out_nhits, int32_t* out_status, const kf_build_extra* extra, void* ws,
                            size_t ws_bytes, void* stream) {
  if (check_det(d) || !bp || !hits) return KF_E_INVALID_ARG;
  if (n_seeds < 0 || ld < n_seeds) return KF_E_INVALID_ARG;
  if (bp->first_layer < 1 || bp->first_layer >= d->n_layers) return KF_E_INVALID_ARG;
  if (bp->cand_cap < 1 || bp->max_holes < 0 || !(bp->nsigma > 0.f) || !(bp->win_sig_rphi > 0.f) ||
      !(bp->win_sig_z > 0.f))
    return KF_E_INVALID_ARG;
  if (bp->cand_cap > 8) return KF_E_UNSUPPORTED;
  if (bp->phi_refine < 0 || bp->phi_refine > 64) return KF_E_INVALID_ARG;
  if (bp->arith != KF_ARITH_F32 && bp->arith != KF_ARITH_F64) return KF_E_INVALID_ARG;
  if (bp->window_mode != 0 || bp->state != 0) return KF_E_UNSUPPORTED;
  if (hits->n_layers != d->n_layers || hits->n_events < 1 || hits->n_phi < 1 || hits->n_z < 1 || hits->n_hits < 0)
    return KF_E_INVALID_ARG;
  kf_build_extra ex = {};
  if (extra) ex = *extra;
  if (ex.dump || ex.event_done_ticks || ex.start_tick) return KF_E_UNSUPPORTED;
  if (hits->n_events > 1 && !ex.seed_event) return KF_E_INVALID_ARG;
  if (n_seeds == 0) return KF_OK;
  if (!seed_par || !seed_cov || !q || !out_hits || !out_visit || !out_par || !out_cov || !out_chi2 || !out_nhits ||
      !out_status)
    return KF_E_INVALID_ARG;
  if (!hits->offsets || (hits->n_hits > 0 && (!hits->x || !hits->y || !hits->z || !hits->phi || !hits->cov ||
                                               !hits->orig)))
    return KF_E_INVALID_ARG;
  const int refine = bp->phi_refine > 0 ? bp->phi_refine : 64;
  if ((int64_t)hits->n_phi * refine > (1 << 20)) return KF_E_UNSUPPORTED;
  const size_t need = kf_build_workspace_bytes(bp, hits, n_seeds);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return KF_E_WORKSPACE;
  const int lanes = bp->lanes_per_block;
  if (lanes != 0 && lanes != 64 && lanes != 128 && lanes != 256) return KF_E_UNSUPPORTED;

  DetBuildArgs A;
  A.d = det_k(d);
  A.chi2_cut = bp->chi2_cut; A.max_holes = bp->max_holes; A.cap = bp->cand_cap;
  A.nsigma = bp->nsigma; A.win_sig_rphi = bp->win_sig_rphi; A.win_sig_w = bp->win_sig_z;
  A.first_layer = bp->first_layer;
  A.n_events = hits->n_events; A.n_phi = hits->n_phi; A.n_w = hits->n_z; A.offsets = hits->offsets;
  A.refine = refine;
  // workspace: the layout of kf_build's (queue head and event counters, fine
  // index, packed hits, history tables)
  const size_t fine_off = ws_head_bytes(hits->n_events);
  A.fine = (const int32_t*)((char*)ws + fine_off);
  const size_t pack_off =
      fine_off + ((fine_bytes(hits->n_events, hits->n_layers, hits->n_phi, hits->n_z, refine) + 255) & ~(size_t)255);
  A.hpack = (const float4*)((char*)ws + pack_off);
  const size_t hist_off = pack_off + pack_bytes(hits->n_hits);
  A.hist = (uint32_t*)((char*)ws + hist_off);
  const size_t LBw = (size_t)(d->n_layers - bp->first_layer) * 64 * 4;
  const int hist_waves = (int)((ws_bytes - hist_off) / LBw);
  const int seeds_per_wave = 64 / bp->cand_cap;
  A.n_seeds = n_seeds; A.ld = ld; A.n_groups = (n_seeds + seeds_per_wave - 1) / seeds_per_wave;
  A.seed_par = seed_par; A.seed_cov = seed_cov; A.q = q;
  A.seed_event = ex.seed_event; A.seed_order = ex.seed_order;
  A.out_hits = out_hits; A.out_visit = out_visit; A.out_par = out_par; A.out_cov = out_cov; A.out_chi2 = out_chi2;
  A.out_nhits = out_nhits; A.out_status = out_status;
  A.counters = (unsigned long long*)ex.counters;
  A.queue = (int32_t*)ws;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(build_clear, dim3(1), dim3(256), 0, s, A.queue, (int32_t*)((char*)ws + 256), hits->n_events,
                     (int64_t*)nullptr);
  if (int rc = kf_check_launch()) return rc;
  const int n_rows = hits->n_events * hits->n_layers * hits->n_z;
  hipLaunchKernelGGL(fine_kernel, dim3((n_rows + 3) / 4), dim3(256), 0, s, n_rows, hits->n_phi, hits->n_z,
                     hits->n_phi * refine, hits->offsets, hits->phi, (int32_t*)A.fine);
  if (int rc = kf_check_launch()) return rc;
  if (hits->n_hits > 0) {
    hipLaunchKernelGGL(pack_kernel, dim3((hits->n_hits + 255) / 256), dim3(256), 0, s, hits->n_hits, hits->x, hits->y,
                       hits->z, hits->phi, hits->cov, hits->orig, (float4*)A.hpack);
    if (int rc = kf_check_launch()) return rc;
  }
  return bp->arith == KF_ARITH_F64
             ? launch_det<double>(A, lanes, bp->persistent_blocks, hist_waves, s, &g_last_det_launch)
             : launch_det<float>(A, lanes, bp->persistent_blocks, hist_waves, s, &g_last_det_launch);
}
