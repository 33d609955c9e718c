// Combinatorial Kalman-filter track building (sections 2, 3.1, 4.3).
//
// Layout of the work: one lane per candidate slot, S slots per seed
// (S = 8, or 4 when cand_cap <= 4), 64/S seeds per wave.  One persistent
// launch: each wave takes groups of 64/S seeds from an atomic queue until the
// queue is empty, so uneven events and seeds balance across the chip.
//
// Per layer, per wave:
//   1. every live slot predicts its candidate (FP32 or FP64 arithmetic);
//   2. the search window is computed and the phi-sorted rows of the hit bins
//      that cover it are scanned (binary search to the window's low edge,
//      then a walk to its high edge); each in-window hit gets its chi2;
//   3. each lane keeps its best cand_cap children in registers;
//   4. the seed's children are merged across its S lanes, best first, by a
//      64-bit rank key (nhits, chi2, parent slot, hit index) with lane
//      shuffles; the winners take the slots 0..cap-1;
//   5. the new slots pull the parent's predicted state by shuffles and apply
//      the Kalman update with their hit;
//   6. back-pointers (parent slot, hit) go to an LDS history table; the best
//      hit list is recovered at the end by walking it backwards.
// Candidates with no child compete for a per-seed best-finished record (LDS).
#include <stdint.h>

#include "kfdev.h"
#include "kfhost.h"
#include "kfmlp.h"

using namespace kfdev;

namespace {

constexpr uint64_t kInfKey = ~0ull;
constexpr uint32_t kHoleIdx = 0xFFFFFFu;
constexpr int kMaxOrig = (1 << 24) - 2;

struct BuildArgs {
  // geometry
  int n_layers;
  float r[32];
  float z_half, bz, x_over_x0, mass;
  // cuts
  float chi2_cut;
  int max_holes, cap;
  float nsigma, win_sig_rphi, win_sig_z;
  int first_layer;
  int window_mode;
  const float* mlp;
  // hits
  int n_events, n_phi, n_z;
  const int32_t* offsets;
  const float *hx, *hy, *hz, *hphi, *hcov;
  const int32_t* horig;
  int n_hits;
  // seeds
  int n_seeds, ld, n_groups;
  const float *seed_par, *seed_cov;
  const int8_t* q;
  const int32_t* seed_event;
  const int32_t* seed_order;
  // outputs
  int32_t* out_hits;
  float *out_par, *out_cov, *out_chi2;
  int32_t *out_nhits, *out_status;
  // extras
  const int32_t* event_n_seeds;
  int64_t* event_done_ticks;
  int64_t* start_tick;
  const int32_t* true_hits;
  const float* true_xyz;
  float* dump;
  int32_t* dump_count;
  int dump_capacity;
  unsigned long long* counters;
  // workspace
  int32_t* queue;
  int32_t* event_done;
};

template <typename T> __device__ inline T shfl(T v, int src) { return __shfl(v, src, 64); }
__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src, 64), hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline double shfl_d(double v, int src) {
  uint64_t b = __double_as_longlong(v);
  return __longlong_as_double((long long)shfl_u64(b, src));
}
__device__ inline float shfl_t(float v, int src) { return __shfl(v, src, 64); }
__device__ inline double shfl_t(double v, int src) { return shfl_d(v, src); }

// minimum over the S lanes of one seed (S a power of two <= 64)
template <int S> __device__ inline uint64_t group_min(uint64_t k) {
#pragma unroll
  for (int m = 1; m < S; m <<= 1) {
    uint32_t lo = __shfl_xor((uint32_t)k, m, 64), hi = __shfl_xor((uint32_t)(k >> 32), m, 64);
    uint64_t o = ((uint64_t)hi << 32) | lo;
    k = o < k ? o : k;
  }
  return k;
}
template <int S> __device__ inline int group_sum(int v) {
#pragma unroll
  for (int m = 1; m < S; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ inline uint32_t chi2_bits(float c) {
  c = c > 0.f ? c : 0.f;  // chi2 >= 0; clears a negative rounding residue and -0
  return __float_as_uint(c);
}

// rank key: nhits desc, chi2 asc, parent slot asc, hit index asc (hole last)
__device__ inline uint64_t make_key(int nhits, float chi2, int slot, uint32_t orig24) {
  return ((uint64_t)(31 - nhits) << 59) | ((uint64_t)chi2_bits(chi2) << 27) | ((uint64_t)slot << 24) | orig24;
}

__device__ inline float wrap_2pi(float p) {
  const float tp = 6.283185307179586f;
  if (p < 0.f) p += tp;
  if (p >= tp) p -= tp;
  return p;
}

// first position in [lo, hi) with phi[pos] >= v (phi sorted ascending)
__device__ inline int lower_bound_phi(const float* __restrict__ phi, int lo, int hi, float v) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (phi[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename T, int CAPMAX> struct TopList {
  T c2[CAPMAX];
  int pos[CAPMAX];
  uint32_t orig[CAPMAX];
  int n;    // entries held (<= cap)
  int tot;  // accepted hits seen
  int scanned, tested;  // hits window-tested, hits given a chi2 (work counters)
};

template <typename T, int CAPMAX>
__device__ inline void top_insert(TopList<T, CAPMAX>& tl, int cap, T c2, int pos, uint32_t orig) {
  tl.tot += 1;
  // insertion into the sorted list (chi2 asc, index asc), keeping cap entries
  T cc = c2;
  int pp = pos;
  uint32_t oo = orig;
  bool carry = true;
#pragma unroll
  for (int k = 0; k < CAPMAX; ++k) {
    if (k < cap && carry) {
      if (k >= tl.n) {
        tl.c2[k] = cc; tl.pos[k] = pp; tl.orig[k] = oo;
        carry = false;
      } else {
        const bool before = (float)cc < (float)tl.c2[k] || ((float)cc == (float)tl.c2[k] && oo < tl.orig[k]);
        if (before) {
          T t0 = tl.c2[k]; int t1 = tl.pos[k]; uint32_t t2 = tl.orig[k];
          tl.c2[k] = cc; tl.pos[k] = pp; tl.orig[k] = oo;
          cc = t0; pp = t1; oo = t2;
        }
      }
    }
  }
  if (tl.n < cap) tl.n += 1;
}

template <typename T, int CAPMAX>
__device__ inline void top_get(const TopList<T, CAPMAX>& tl, int k, T& c2, int& pos, uint32_t& orig) {
  c2 = tl.c2[0]; pos = tl.pos[0]; orig = tl.orig[0];
#pragma unroll
  for (int j = 1; j < CAPMAX; ++j)
    if (j == k) { c2 = tl.c2[j]; pos = tl.pos[j]; orig = tl.orig[j]; }
}

// Scan one phi-sorted range [b0, b1) of hit positions restricted to stored
// phi in [plo, phi_hi], testing each hit exactly and collecting children.
template <typename T, int CAPMAX>
__device__ inline void scan_range(const BuildArgs& A, int b0, int b1, float plo, float phi_hi, const T Xp[6],
                                  const T Pp[21], T dphi_w, T dz_w, TopList<T, CAPMAX>& tl) {
  int p = lower_bound_phi(A.hphi, b0, b1, plo);
  for (; p < b1; ++p) {
    if (A.hphi[p] > phi_hi) break;
    tl.scanned += 1;
    const T hx = (T)A.hx[p], hy = (T)A.hy[p], hz = (T)A.hz[p];
    const T cr = Xp[0] * hy - Xp[1] * hx, dt = Xp[0] * hx + Xp[1] * hy;
    const T dph = k_atan2(cr, dt);
    if (!(fabs(dph) <= dphi_w) || !(fabs(hz - Xp[2]) <= dz_w)) continue;
    T V[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) V[c] = (T)A.hcov[(size_t)c * A.n_hits + p];
    Innov<T> in;
    tl.tested += 1;
    if (innovation<T>(Xp, Pp, hx, hy, hz, V, in)) continue;
    const T c2 = chi2_of(in);
    if (!(c2 < (T)A.chi2_cut)) continue;
    top_insert(tl, A.cap, c2, p, (uint32_t)A.horig[p]);
  }
}

template <typename T, int CAPMAX>
__device__ inline void scan_window(const BuildArgs& A, int ev, int l, const T Xp[6], const T Pp[21], T dphi_w,
                                   T dz_w, TopList<T, CAPMAX>& tl) {
  const int nphi = A.n_phi, nz = A.n_z, nb = nphi * nz;
  const int32_t* off = A.offsets + ((size_t)ev * A.n_layers + l) * (nb + 1);
  const float zh = A.z_half;
  const float zp = (float)Xp[2];
  const float phip = wrap_2pi((float)k_atan2(Xp[1], Xp[0]));
  const float eps_phi = 1e-5f, eps_z = 1e-4f;
  const float dphi = (float)dphi_w + eps_phi, dz = (float)dz_w + eps_z;
  int iz0 = (int)floorf((zp - dz + zh) * (float)nz / (2.f * zh));
  int iz1 = (int)floorf((zp + dz + zh) * (float)nz / (2.f * zh));
  iz0 = iz0 < 0 ? 0 : (iz0 > nz - 1 ? nz - 1 : iz0);
  iz1 = iz1 < 0 ? 0 : (iz1 > nz - 1 ? nz - 1 : iz1);
  const float tp = 6.283185307179586f;
  // up to two phi intervals within [0, 2pi)
  float a0, b0v, a1 = 1.f, b1v = 0.f;
  if (dphi >= 3.14159f) { a0 = 0.f; b0v = tp; }
  else {
    float lo = phip - dphi, hi = phip + dphi;
    if (lo < 0.f) { a0 = 0.f; b0v = hi; a1 = lo + tp; b1v = tp; }
    else if (hi >= tp) { a0 = lo; b0v = tp; a1 = 0.f; b1v = hi - tp; }
    else { a0 = lo; b0v = hi; }
  }
  for (int iz = iz0; iz <= iz1; ++iz) {
    for (int part = 0; part < 2; ++part) {
      const float a = part ? a1 : a0, b = part ? b1v : b0v;
      if (!(a <= b)) continue;
      int ip0 = (int)floorf(a * (float)nphi / tp), ip1 = (int)floorf(b * (float)nphi / tp);
      ip0 = ip0 < 0 ? 0 : (ip0 > nphi - 1 ? nphi - 1 : ip0);
      ip1 = ip1 < 0 ? 0 : (ip1 > nphi - 1 ? nphi - 1 : ip1);
      const int p0 = off[iz * nphi + ip0], p1 = off[iz * nphi + ip1 + 1];
      scan_range<T, CAPMAX>(A, p0, p1, a, b, Xp, Pp, dphi_w, dz_w, tl);
    }
  }
}

__device__ inline uint32_t pack_hist(int parent, uint32_t orig24) {
  return ((uint32_t)parent << 24) | (orig24 == kHoleIdx ? 0xFFFFFFu : orig24);
}

template <typename T, int S>
__global__ void __launch_bounds__(256) build_kernel(BuildArgs A) {
  constexpr int CAPMAX = S;
  constexpr int SEEDS = 64 / S;
  extern __shared__ __align__(16) uint32_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int LB = A.n_layers - A.first_layer;  // searched layers
  // LDS: history [waves][LB][64] u32 | record states [waves][SEEDS][27] T |
  //      record fields [waves][SEEDS][5] i32 (valid, nhits, status, last layer, slot)
  uint32_t* hist = lds + (size_t)wave * LB * 64;
  const size_t hist_words = (size_t)nwaves * LB * 64;
  const size_t fin_off = (hist_words * 4 + 15) & ~(size_t)15;
  T* fin = (T*)((char*)lds + fin_off) + (size_t)wave * SEEDS * 27;
  int32_t* finm = (int32_t*)((char*)lds + fin_off + (size_t)nwaves * SEEDS * 27 * sizeof(T)) + (size_t)wave * SEEDS * 5;
  const size_t mlp_off = (fin_off + (size_t)nwaves * SEEDS * 27 * sizeof(T) + (size_t)nwaves * SEEDS * 5 * 4 + 15) &
                         ~(size_t)15;
  uint16_t* mlp_buf = (uint16_t*)((char*)lds + mlp_off) + (size_t)wave * (KFMLP_LDS_BYTES / 2);
  const int sidx = lane / S, slot = lane % S, sbase = sidx * S;

  if (A.start_tick && lane == 0) atomicMin((unsigned long long*)A.start_tick, (unsigned long long)wall_clock64());

  for (;;) {
    int grp = 0;
    if (lane == 0) grp = atomicAdd(A.queue, 1);
    grp = __shfl(grp, 0, 64);
    if (grp >= A.n_groups) break;
    const int gi = grp * SEEDS + sidx;
    int seed = gi < A.n_seeds ? (A.seed_order ? A.seed_order[gi] : gi) : -1;
    int ev = (seed >= 0 && seed < A.n_seeds && A.seed_event) ? A.seed_event[seed] : 0;
    // caller-supplied indices outside their ranges: the seed is skipped
    const bool seed_ok = seed >= 0 && seed < A.n_seeds && ev >= 0 && ev < A.n_events;
    if (!seed_ok) { seed = 0; ev = 0; }
    const int q = seed_ok ? A.q[seed] : 1;
    // candidate state
    T X[6], P[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = seed_ok ? (T)A.seed_par[(size_t)k * A.ld + seed] : T(0);
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = seed_ok ? (T)A.seed_cov[(size_t)k * A.ld + seed] : T(0);
    T chi2 = 0;
    int nhits = 0, holes = 0;
    bool ontrack = true;
    int n_active = seed_ok ? 1 : 0;
    int seed_status = 0;
    if (slot == 0) finm[sidx * 5 + 0] = 0;
    if (seed_ok && !(all_finite(X, 6) && all_finite(P, 21))) {
      // non-finite seed: it is its own (finished) result
      if (slot == 0) {
        finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = 0; finm[sidx * 5 + 2] = KF_NONFINITE;
        finm[sidx * 5 + 3] = A.first_layer - 1; finm[sidx * 5 + 4] = 0;
        for (int k = 0; k < 6; ++k) fin[sidx * 27 + k] = X[k];
        for (int k = 0; k < 21; ++k) fin[sidx * 27 + 6 + k] = P[k];
      }
      n_active = 0;
    }
    T fin_chi2_reg = 0;  // chi2 of the finished record, kept by slot 0 of the seed
    unsigned cnt_pred = 0, cnt_scan = 0, cnt_chi2 = 0, cnt_upd = 0;
    int last_l = A.first_layer - 1;
    for (int l = A.first_layer; l < A.n_layers; ++l) {
      // all seeds of the wave done?
      if (!__any(n_active > 0)) break;
      last_l = l;
      const bool live = slot < n_active;
      T Xp[6], Pp[21];
      int rc = 1;
      if (live)
        rc = predict<T>(X, P, q, (T)A.r[l], (T)A.bz, (T)A.z_half, (T)A.x_over_x0, (T)A.mass, Xp, Pp);
      else {
#pragma unroll
        for (int k = 0; k < 6; ++k) Xp[k] = X[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) Pp[k] = P[k];
      }
      const bool pok = live && rc == 0;
      TopList<T, CAPMAX> tl;
      tl.n = 0;
      tl.tot = 0;
      tl.scanned = 0;
      tl.tested = 0;
#pragma unroll
      for (int k = 0; k < CAPMAX; ++k) { tl.c2[k] = 0; tl.pos[k] = 0; tl.orig[k] = 0; }
      // learned window: the whole wave evaluates the network on its 64 slots
      float wl[2] = {0.f, 0.f};
      if (A.window_mode == 1) {
        float feat[27];
#pragma unroll
        for (int k = 0; k < 6; ++k) feat[k] = pok ? (float)Xp[k] : 0.f;
#pragma unroll
        for (int k = 0; k < 21; ++k) feat[6 + k] = pok ? (float)Pp[k] : 0.f;
        kfmlp::wave_forward(A.mlp, mlp_buf, feat, wl);
        const float kap = A.mlp[KFMLP_OFF_KAPPA];
        wl[0] *= kap;
        wl[1] *= kap;
      }
      if (pok) {
        const T R = (T)A.r[l];
        const T rr = k_sqrt(Xp[0] * Xp[0] + Xp[1] * Xp[1]);
        const T tx = -Xp[1] / rr, ty = Xp[0] / rr;
        const T Suu = tx * tx * Pp[ut(0, 0)] + T(2) * tx * ty * Pp[ut(0, 1)] + ty * ty * Pp[ut(1, 1)] +
                      (T)A.win_sig_rphi * (T)A.win_sig_rphi;
        const T Sww = Pp[ut(2, 2)] + (T)A.win_sig_z * (T)A.win_sig_z;
        T w_rphi = (T)A.nsigma * k_sqrt(Suu), w_z = (T)A.nsigma * k_sqrt(Sww);
        if (A.window_mode == 1) {
          if (!(wl[0] < A.mlp[KFMLP_OFF_FLOOR])) w_rphi = (T)wl[0];
          if (!(wl[1] < A.mlp[KFMLP_OFF_FLOOR + 1])) w_z = (T)wl[1];
        }
        if (A.dump && ontrack && A.true_hits) {
          const int th = A.true_hits[(size_t)l * A.ld + seed];
          if (th >= 0) {
            const int row = atomicAdd(A.dump_count, 1);
            if (row < A.dump_capacity) {
              float* d = A.dump + (size_t)row * KFMLP_DUMP_ROW;
              for (int k = 0; k < 6; ++k) d[k] = (float)Xp[k];
              for (int k = 0; k < 21; ++k) d[6 + k] = (float)Pp[k];
              const T mx = (T)A.true_xyz[((size_t)l * 3 + 0) * A.ld + seed];
              const T my = (T)A.true_xyz[((size_t)l * 3 + 1) * A.ld + seed];
              const T mz = (T)A.true_xyz[((size_t)l * 3 + 2) * A.ld + seed];
              const T dph = k_atan2(Xp[0] * my - Xp[1] * mx, Xp[0] * mx + Xp[1] * my);
              d[27] = (float)(R * fabs(dph));
              d[28] = (float)fabs(mz - Xp[2]);
              d[29] = __int_as_float(seed);
              d[30] = __int_as_float(l);
              d[31] = __int_as_float(slot);
            }
          }
        }
        scan_window<T, CAPMAX>(A, ev, l, Xp, Pp, w_rphi / R, w_z, tl);
      }
      cnt_pred += live ? 1u : 0u;
      cnt_scan += (unsigned)tl.scanned;
      cnt_chi2 += (unsigned)tl.tested;
      const bool hole_ok = pok && holes < A.max_holes;
      const int nchild = tl.tot + (hole_ok ? 1 : 0);
      // finished candidates of this layer (live, no child) compete for the record
      {
        const bool stopped = live && nchild == 0;
        uint64_t fk = stopped ? make_key(nhits, (float)chi2, slot, 0) : kInfKey;
        const uint64_t best = group_min<S>(fk);
        if (best != kInfKey) {
          const int ws = (int)((best >> 24) & 7);
          const int wl_ = sbase + ws;
          // winner's chi2 in T and its fields
          const T wc2 = shfl_t(chi2, wl_);
          const int wn = __shfl(nhits, wl_, 64);
          const int wst = __shfl(live && rc ? rc : 0, wl_, 64);
          const int fvalid = finm[sidx * 5 + 0];
          const int fn = finm[sidx * 5 + 1];
          const T fc2 = shfl_t(fin_chi2_reg, sbase);
          const bool take = !fvalid || wn > fn || (wn == fn && wc2 < fc2);
          if (take) {
            if (slot == ws) {
              for (int k = 0; k < 6; ++k) fin[sidx * 27 + k] = X[k];
              for (int k = 0; k < 21; ++k) fin[sidx * 27 + 6 + k] = P[k];
              finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = wn; finm[sidx * 5 + 2] = wst;
              finm[sidx * 5 + 3] = l - 1; finm[sidx * 5 + 4] = ws;
            }
            if (slot == 0) fin_chi2_reg = wc2;
          }
        }
      }
      // merge the children of the seed, best first, into slots 0..cap-1
      const int tot = group_sum<S>(nchild);
      if (tot > A.cap) seed_status |= KF_CAP_TRUNC;
      int ptr = 0;
      bool hole_left = hole_ok;
      int my_parent = -1, my_pos = -1;
      uint32_t my_orig = kHoleIdx;
      T my_c2 = 0;
      int n_new = 0;
      for (int r = 0; r < A.cap; ++r) {
        uint64_t key = kInfKey;
        T hc2 = 0;
        int hpos = -1;
        uint32_t horig = kHoleIdx;
        if (pok) {
          if (ptr < tl.n) {
            top_get(tl, ptr, hc2, hpos, horig);
            key = make_key(nhits + 1, (float)(chi2 + hc2), slot, horig);
          } else if (hole_left) {
            key = make_key(nhits, (float)chi2, slot, kHoleIdx);
          }
        }
        const uint64_t win = group_min<S>(key);
        if (win == kInfKey) continue;  // no more children for this seed
        const int ws = (int)((win >> 24) & 7);
        const int wl_ = sbase + ws;
        const int wpos = __shfl(hpos, wl_, 64);
        const T wc2 = shfl_t(hc2, wl_);
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
      // new slots pull the parent's predicted state
      const int src = sbase + (my_parent >= 0 ? my_parent : slot);
      T Xn[6], Pn[21];
#pragma unroll
      for (int k = 0; k < 6; ++k) Xn[k] = shfl_t(Xp[k], src);
#pragma unroll
      for (int k = 0; k < 21; ++k) Pn[k] = shfl_t(Pp[k], src);
      const T pchi2 = shfl_t(chi2, src);
      const int pnh = __shfl(nhits, src, 64), pho = __shfl(holes, src, 64);
      const bool pon = __shfl((int)ontrack, src, 64) != 0;
      if (my_parent >= 0) {
        const bool is_hole = my_orig == kHoleIdx;
        if (!is_hole) {
          const T hx = (T)A.hx[my_pos], hy = (T)A.hy[my_pos], hz = (T)A.hz[my_pos];
          T V[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) V[c] = (T)A.hcov[(size_t)c * A.n_hits + my_pos];
          Innov<T> in;
          innovation<T>(Xn, Pn, hx, hy, hz, V, in);
          apply_update<T>(Xn, Pn, in);
          cnt_upd += 1;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) X[k] = Xn[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) P[k] = Pn[k];
        chi2 = is_hole ? pchi2 : pchi2 + my_c2;
        nhits = is_hole ? pnh : pnh + 1;
        holes = is_hole ? pho + 1 : pho;
        if (A.dump && A.true_hits) {
          const int th = seed_ok ? A.true_hits[(size_t)l * A.ld + seed] : -1;
          ontrack = pon && (is_hole || (int)my_orig == th);
        }
        hist[(l - A.first_layer) * 64 + lane] = pack_hist(my_parent, my_orig);
      }
      n_active = n_new;
    }
    if (A.counters) {
      unsigned long long c[4] = {cnt_pred, cnt_scan, cnt_chi2, cnt_upd};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        unsigned long long v = c[k];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
        if (lane == 0) atomicAdd(&A.counters[k], v);
      }
    }
    // final choice: best active (slot order), then the finished record
    {
      const bool act = slot < n_active;
      const uint64_t k = act ? make_key(nhits, (float)chi2, slot, 0) : kInfKey;
      const uint64_t best = group_min<S>(k);
      int bslot = -1;
      T bc2 = 0;
      int bn = 0;
      if (best != kInfKey) {
        bslot = (int)((best >> 24) & 7);
        bc2 = shfl_t(chi2, sbase + bslot);
        bn = __shfl(nhits, sbase + bslot, 64);
      } else {
        (void)shfl_t(chi2, sbase);
        (void)__shfl(nhits, sbase, 64);
      }
      const T fc2 = shfl_t(fin_chi2_reg, sbase);
      const int fvalid = finm[sidx * 5 + 0];
      const int fn = finm[sidx * 5 + 1];
      const bool use_fin = fvalid && (bslot < 0 || fn > bn || (fn == bn && fc2 < bc2));
      if (seed_ok) {
        // state: the best lane writes its own; slot 0 writes the record
        if (!use_fin && slot == bslot) {
          for (int k2 = 0; k2 < 6; ++k2) A.out_par[(size_t)k2 * A.ld + seed] = (float)X[k2];
          for (int k2 = 0; k2 < 21; ++k2) A.out_cov[(size_t)k2 * A.ld + seed] = (float)P[k2];
          A.out_chi2[seed] = (float)chi2;
          A.out_nhits[seed] = nhits;
          A.out_status[seed] = seed_status;
        }
        if (use_fin && slot == 0) {
          for (int k2 = 0; k2 < 6; ++k2) A.out_par[(size_t)k2 * A.ld + seed] = (float)fin[sidx * 27 + k2];
          for (int k2 = 0; k2 < 21; ++k2) A.out_cov[(size_t)k2 * A.ld + seed] = (float)fin[sidx * 27 + 6 + k2];
          A.out_chi2[seed] = (float)fin_chi2_reg;
          A.out_nhits[seed] = fn;
          A.out_status[seed] = finm[sidx * 5 + 2] | seed_status;
        }
        // hit list: walk the history backwards (one lane per seed)
        if (slot == 0) {
          int from_l = use_fin ? finm[sidx * 5 + 3] : last_l;
          int s = use_fin ? finm[sidx * 5 + 4] : bslot;
          if (bslot < 0 && !use_fin) from_l = A.first_layer - 1;
          for (int l = A.n_layers - 1; l > from_l; --l) A.out_hits[(size_t)(l - A.first_layer) * A.ld + seed] = -1;
          for (int l = from_l; l >= A.first_layer; --l) {
            const uint32_t h = hist[(l - A.first_layer) * 64 + sbase + s];
            const uint32_t o = h & 0xFFFFFFu;
            A.out_hits[(size_t)(l - A.first_layer) * A.ld + seed] = o == 0xFFFFFFu ? -1 : (int32_t)o;
            s = (int)(h >> 24);
          }
        }
        // per-event completion
        if (slot == 0 && A.event_done_ticks) {
          const int done = atomicAdd(&A.event_done[ev], 1);
          if (done == A.event_n_seeds[ev] - 1) A.event_done_ticks[ev] = (int64_t)wall_clock64();
        }
      }
    }
  }
}

__global__ void build_clear(int32_t* queue, int32_t* event_done, int n_events, int64_t* start_tick) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *queue = 0;
  if (i == 0 && start_tick) *start_tick = INT64_MAX;
  for (int e = i; e < n_events; e += gridDim.x * blockDim.x) event_done[e] = 0;
}

size_t lds_bytes(int LB, int nwaves, int S, size_t tsize, bool learned) {
  const int seeds = 64 / S;
  const size_t fin_off = ((size_t)nwaves * LB * 64 * 4 + 15) & ~(size_t)15;
  const size_t end = fin_off + (size_t)nwaves * seeds * 27 * tsize + (size_t)nwaves * seeds * 5 * 4;
  if (!learned) return end;
  return ((end + 15) & ~(size_t)15) + (size_t)nwaves * KFMLP_LDS_BYTES;
}

template <typename T, int S>
int launch(const BuildArgs& A, int lanes, int blocks, hipStream_t s) {
  const int nwaves = lanes / 64;
  const size_t lds = lds_bytes(A.n_layers - A.first_layer, nwaves, S, sizeof(T), A.window_mode == 1);
  if (lds > 64 * 1024) return KF_E_UNSUPPORTED;
  if (blocks <= 0) {
    int dev = 0, cus = 0, per = 0;
    if (kf_check(hipGetDevice(&dev))) return KF_E_HIP;
    if (kf_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))) return KF_E_HIP;
    if (kf_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, build_kernel<T, S>, lanes, lds))) return KF_E_HIP;
    blocks = cus * (per > 0 ? per : 1);
  }
  const int need = (A.n_groups + nwaves - 1) / nwaves;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((build_kernel<T, S>), dim3(blocks), dim3(lanes), lds, s, A);
  return kf_check_launch();
}

}  // namespace

extern "C" size_t kf_build_workspace_bytes(int32_t n_seeds, int32_t n_events) {
  (void)n_seeds;
  if (n_events < 1) n_events = 1;
  return 256 + (((size_t)n_events * 4 + 255) & ~(size_t)255);
}

extern "C" int kf_build(const kf_geometry* g, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds,
                        int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q, int32_t* out_hits,
                        float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits, int32_t* out_status,
                        const kf_build_extra* extra, void* ws, size_t ws_bytes, void* stream) {
  if (kf_check_geometry(g) || !bp || !hits) return KF_E_INVALID_ARG;
  if (n_seeds < 0 || ld < n_seeds) return KF_E_INVALID_ARG;
  if (bp->first_layer < 1 || bp->first_layer >= g->n_layers) return KF_E_INVALID_ARG;
  if (bp->cand_cap < 1 || bp->max_holes < 0 || !(bp->nsigma > 0.f) || !(bp->win_sig_rphi > 0.f) ||
      !(bp->win_sig_z > 0.f))
    return KF_E_INVALID_ARG;
  if (bp->cand_cap > 8) return KF_E_UNSUPPORTED;
  if (bp->arith != KF_ARITH_F32 && bp->arith != KF_ARITH_F64) return KF_E_INVALID_ARG;
  if (bp->window_mode != 0 && bp->window_mode != 1) return KF_E_INVALID_ARG;
  if (bp->window_mode == 1 && !bp->mlp) return KF_E_INVALID_ARG;
  if (hits->n_layers != g->n_layers || hits->n_events < 1 || hits->n_phi < 1 || hits->n_z < 1 || hits->n_hits < 0)
    return KF_E_INVALID_ARG;
  (void)kMaxOrig;  // hit indices are event-local: each event must hold fewer than 2^24 - 1 hits
  if (n_seeds == 0) return KF_OK;
  if (!seed_par || !seed_cov || !q || !out_hits || !out_par || !out_cov || !out_chi2 || !out_nhits || !out_status)
    return KF_E_INVALID_ARG;
  if (!hits->offsets || (hits->n_hits > 0 && (!hits->x || !hits->y || !hits->z || !hits->phi || !hits->cov ||
                                               !hits->orig)))
    return KF_E_INVALID_ARG;
  kf_build_extra ex = {};
  if (extra) ex = *extra;
  if (hits->n_events > 1 && !ex.seed_event) return KF_E_INVALID_ARG;
  if (ex.event_done_ticks && !ex.event_n_seeds) return KF_E_INVALID_ARG;
  if (ex.dump && (!ex.dump_count || !ex.true_hits || !ex.true_xyz || ex.dump_capacity < 0)) return KF_E_INVALID_ARG;
  const size_t need = kf_build_workspace_bytes(n_seeds, hits->n_events);
  if (!ws || ws_bytes < need) return KF_E_WORKSPACE;
  int lanes = bp->lanes_per_block ? bp->lanes_per_block : 256;
  if (lanes != 64 && lanes != 128 && lanes != 256) return KF_E_UNSUPPORTED;

  BuildArgs A;
  A.n_layers = g->n_layers;
  for (int i = 0; i < 32; ++i) A.r[i] = g->r[i];
  A.z_half = g->z_half; A.bz = g->bz; A.x_over_x0 = g->x_over_x0; A.mass = g->mass;
  A.chi2_cut = bp->chi2_cut; A.max_holes = bp->max_holes; A.cap = bp->cand_cap;
  A.nsigma = bp->nsigma; A.win_sig_rphi = bp->win_sig_rphi; A.win_sig_z = bp->win_sig_z;
  A.first_layer = bp->first_layer; A.window_mode = bp->window_mode; A.mlp = (const float*)bp->mlp;
  A.n_events = hits->n_events; A.n_phi = hits->n_phi; A.n_z = hits->n_z; A.offsets = hits->offsets;
  A.hx = hits->x; A.hy = hits->y; A.hz = hits->z; A.hphi = hits->phi; A.hcov = hits->cov; A.horig = hits->orig;
  A.n_hits = hits->n_hits;
  const int S = bp->cand_cap <= 4 ? 4 : 8;
  const int seeds_per_wave = 64 / S;
  A.n_seeds = n_seeds; A.ld = ld; A.n_groups = (n_seeds + seeds_per_wave - 1) / seeds_per_wave;
  A.seed_par = seed_par; A.seed_cov = seed_cov; A.q = q;
  A.seed_event = ex.seed_event; A.seed_order = ex.seed_order;
  A.out_hits = out_hits; A.out_par = out_par; A.out_cov = out_cov; A.out_chi2 = out_chi2;
  A.out_nhits = out_nhits; A.out_status = out_status;
  A.event_n_seeds = ex.event_n_seeds; A.event_done_ticks = ex.event_done_ticks; A.start_tick = ex.start_tick;
  A.true_hits = ex.true_hits; A.true_xyz = ex.true_xyz; A.dump = ex.dump; A.dump_count = ex.dump_count;
  A.dump_capacity = ex.dump_capacity;
  A.counters = (unsigned long long*)ex.counters;
  A.queue = (int32_t*)ws;
  A.event_done = (int32_t*)((char*)ws + 256);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(build_clear, dim3(1), dim3(256), 0, s, A.queue, A.event_done, hits->n_events, A.start_tick);
  if (int rc = kf_check_launch()) return rc;
  if (bp->arith == KF_ARITH_F64)
    return S == 4 ? launch<double, 4>(A, lanes, bp->persistent_blocks, s)
                  : launch<double, 8>(A, lanes, bp->persistent_blocks, s);
  return S == 4 ? launch<float, 4>(A, lanes, bp->persistent_blocks, s)
                : launch<float, 8>(A, lanes, bp->persistent_blocks, s);
}
