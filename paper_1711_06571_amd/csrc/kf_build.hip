// Combinatorial Kalman-filter track building (sections 2, 3.1, 4.3).
//
// Layout of the work: one lane per candidate slot, S = cand_cap consecutive
// lanes per seed, floor(64 / S) seeds per wave (lanes beyond the last seed
// idle).  One persistent launch: each wave takes groups of seeds from an
// atomic queue until the queue is empty, so uneven events and seeds balance
// across the chip.
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
//   6. back-pointers (parent slot, hit) go to the wave's history table in the
//      workspace; the best
//      hit list is recovered at the end by walking it backwards.
// Candidates with no child compete for a per-seed best-finished record (LDS).
#include <stdint.h>
#include <stdio.h>

#include <mutex>

#include "kfdev.h"
#include "kfhost.h"
#include "kfmlp.h"
#include "kfplan.h"
#include "kfwave.h"

using namespace kfdev;

namespace {


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
  // the hits packed per sorted position, three float4 each:
  // (phi, x, y, z), (cov 0..3), (cov 4, cov 5, orig bits, 0)
  const float4* hpack;
  int n_hits;
  int refine;            // sub-bins per phi bin in the fine index
  const int32_t* fine;   // [events][layers][n_z][n_phi * refine + 1]
  uint32_t* hist;        // [resident waves][searched layers][64] back-pointers
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

// ku / kv in FP64 builds only: there, kernel arguments and per-seed values
// that the layer loop uses are recomputed where they are used instead of
// being hoisted out of the loop and spilled (the FP32 build does not spill;
// the barriers would only cost it issue slots)
template <typename T, typename U> __device__ inline U ku64(U v) {
  if constexpr (sizeof(T) == 8) return ku(v);
  else return v;
}
template <typename T, typename U> __device__ inline U kv64(U v) {
  if constexpr (sizeof(T) == 8) return kv(v);
  else return v;
}

// Hit search of every candidate of the wave, shared by all 64 lanes.
//
// Each live candidate's window covers, per z row it overlaps and per phi
// interval (two where the window wraps at 2 pi), one range of sorted hit
// positions bracketed by the fine phi index.  Range r of every candidate is
// taken in turn; the (candidate, hit) pairs of all candidates' ranges r are
// numbered through a wave prefix sum and handed out 64 NP at a time, NP
// pairs per lane, so a candidate with a wide window no longer holds up the
// wave while the others wait.  A lane finds the pair's candidate from the
// marks the candidates set where their pairs start and reads what that
// candidate's tests share by lane shuffles.  Every hit whose stored phi lies in the candidate's interval
// gets the exact window test (z first, then the angle about the axis);
// in-window hits get their chi2; accepted hits (chi2 < cut) are counted for
// their candidate (a ballot over its run of lanes: a candidate's pairs occupy
// consecutive lanes) and, if they can enter its list of the best cap (a full
// list admits only hits that rank before its last entry), placed in it by
// their ranks, all of the round's at once (round_insert).  The ranking is
// total, so the result equals a serial scan.
//
// The tests and chi2 run in FP32 in both arithmetic modes, from the
// prediction rounded to FP32: their rounding (chi2 ~ 3e-5 at the cut,
// positions ~ 1e-5 cm) stays far below the chi2 gaps (1e-3) and window-edge
// distances (1e-4 cm) that separate decisions; the Kalman update of a
// chosen hit runs in the arithmetic of the mode.  NP (pairs per lane and
// round at most) is defined with the LDS plan.
template <typename T, int NPT>
__device__ inline void coop_scan(const BuildArgs& A, int ev, int l, bool pok, const T Xp[6], const T Pp[21],
                                 T dphi_w, T dz_w, TopList& tl, const AccBuf& ab, int lane) {
  static_assert(NPT >= 1 && NPT <= NP, "pairs per lane");
  const int nz = A.n_z, nf = A.n_phi * A.refine;
  const float inv = fine_inv(nf);
  const float tp = 6.283185307179586f;
  // this lane's window as conservative stored-value intervals (the exact
  // test decides): up to two phi intervals within [0, 2pi), z rows iz0..iz1
  float a0 = 1.f, b0v = 0.f, a1 = 1.f, b1v = 0.f;
  int iz0 = 0, iz1 = -1;
  // Per candidate, what every hit test shares: for dphi < pi/2 the angle
  // test |atan2(cross, dot)| <= dphi is dot > 0 and |cross| <= tan(dphi) dot
  // (ftan < 0 marks a wider window, which keeps the angle); the measurement
  // frame (tangent t = (-y, x) / r at the predicted point, from 1 / r) and
  // H P H^T of the prediction.
  float fx = 0.f, fy = 0.f, fz = 0.f, fdz = 0.f, fdphi = 0.f, ftan = 0.f;
  float firr = 0.f, suu = 0.f, suw = 0.f, sww = 0.f;
  if (pok) {
    const float zh = A.z_half;
    fx = (float)Xp[0];
    fy = (float)Xp[1];
    fz = (float)Xp[2];
    fdz = (float)dz_w;
    fdphi = (float)dphi_w;
    const float phip = wrap_2pi(atan2f(fy, fx));
    const float eps_phi = 1e-5f, eps_z = 1e-4f;
    const float dphi = fdphi + eps_phi, dz = fdz + eps_z;
    iz0 = (int)floorf((fz - dz + zh) * (float)ku64<T>(A.n_z) / (2.f * zh));
    iz1 = (int)floorf((fz + dz + zh) * (float)ku64<T>(A.n_z) / (2.f * zh));
    iz0 = iz0 < 0 ? 0 : (iz0 > nz - 1 ? nz - 1 : iz0);
    iz1 = iz1 < 0 ? 0 : (iz1 > nz - 1 ? nz - 1 : iz1);
    if (dphi >= 3.14159f) { a0 = 0.f; b0v = tp; }
    else {
      const float lo = phip - dphi, hi = phip + dphi;
      if (lo < 0.f) { a0 = 0.f; b0v = hi; a1 = lo + tp; b1v = tp; }
      else if (hi >= tp) { a0 = lo; b0v = tp; a1 = 0.f; b1v = hi - tp; }
      else { a0 = lo; b0v = hi; }
    }
    // (the angle test runs in FP32: so does the tangent of its bound)
    ftan = !(dphi_w < T(1.5707963267948966)) ? -1.f : tanf((float)dphi_w);
    const T rr = k_sqrt(Xp[0] * Xp[0] + Xp[1] * Xp[1]);
    const T irr = k_rcp(rr);
    const T tx = -Xp[1] * irr, ty = Xp[0] * irr;
    firr = (float)irr;
    suu = (float)(tx * tx * Pp[ut(0, 0)] + T(2) * tx * ty * Pp[ut(0, 1)] + ty * ty * Pp[ut(1, 1)]);
    suw = (float)(tx * Pp[ut(0, 2)] + ty * Pp[ut(1, 2)]);
    sww = (float)Pp[ut(2, 2)];
  }
  const int32_t* frow = A.fine + ((size_t)ev * A.n_layers + l) * nz * (nf + 1);
  // ranges: (row, interval) for every row, the second interval only where
  // the window wraps at 2 pi
  const int nint = a1 <= b1v ? 2 : 1;
  const int R = pok ? (iz1 - iz0 + 1) * nint : 0;
  const int Rmax = wave_max(R);
  int n_acc = 0;  // accepted hits of this lane's candidate
  int held = 0;           // entries in the list
  bool unsorted = false;  // entries appended out of order
  // the candidate's admission threshold: its last entry once its list is
  // full (before, +inf admits every accepted hit)
  float thr_c2 = __builtin_inff();
  uint32_t thr_o = 0xFFFFFFFFu;
  const float cut = A.chi2_cut;
  // range r of this candidate: its stored-value interval and its sorted
  // positions from the fine index (read one range ahead)
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
        const int32_t* f = frow + (size_t)(iz0 + rr) * (nf + 1);
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
    const int pb = p0 - off;  // sorted position of pair k of this candidate: pb + k
    int carry = 0;  // candidate of the previous round's last pair
    // each lane takes NP pairs per round (pair base + 64 h + lane): their
    // loads share one round trip
    for (int base = 0; base < total; base += 64 * NPT) {
      // candidate of a pair: candidates mark the slot where their pairs start
      // in this round; the pair's candidate is the nearest mark at or below
      // its slot in its half, else the one whose pairs run on from before
#pragma unroll
      for (int h = 0; h < NPT; ++h) ab.start[h * 64 + lane] = -1;
      if (cnt > 0 && off >= base && off - base < 64 * NPT) ab.start[off - base] = lane;
      __builtin_amdgcn_wave_barrier();
      int c[NPT], my_lo[NPT], p[NPT];
      unsigned long long sma[NPT];  // the half's marks
      bool valid[NPT];
      float ca[NPT], cb[NPT], cx[NPT], cy[NPT], cz[NPT], cdz[NPT], cdphi[NPT], ctan[NPT], cirr[NPT], csuu[NPT], csuw[NPT],
          csww[NPT], cthr[NPT];
      uint32_t cthro[NPT];
#pragma unroll
      for (int h = 0; h < NPT; ++h) {
        const int st = ab.start[h * 64 + lane];
        sma[h] = __ballot(st >= 0);
        const unsigned long long sm = sma[h] & ((2ull << lane) - 1ull);
        const int hb = sm ? 63 - (int)__builtin_clzll(sm) : 0;
        const int sc = __shfl(st, hb, 64);
        c[h] = sm ? sc : carry;
        my_lo[h] = sm ? hb : 0;  // first slot of this pair's candidate in the half
        carry = __builtin_amdgcn_readlane(c[h], 63);
        const int k = base + 64 * h + lane;
        valid[h] = k < total;
        p[h] = __shfl(pb, c[h], 64) + k;
        ca[h] = __shfl(a, c[h], 64);
        cb[h] = __shfl(b, c[h], 64);
        cx[h] = __shfl(fx, c[h], 64);
        cy[h] = __shfl(fy, c[h], 64);
        cz[h] = __shfl(fz, c[h], 64);
        cdz[h] = __shfl(fdz, c[h], 64);
        cdphi[h] = __shfl(fdphi, c[h], 64);
        ctan[h] = __shfl(ftan, c[h], 64);
        cirr[h] = __shfl(firr, c[h], 64);
        csuu[h] = __shfl(suu, c[h], 64);
        csuw[h] = __shfl(suw, c[h], 64);
        csww[h] = __shfl(sww, c[h], 64);
        cthr[h] = __shfl(thr_c2, c[h], 64);
        cthro[h] = (uint32_t)__shfl((int)thr_o, c[h], 64);
      }
      // everything each pair can need, in one round trip for all NP pairs
      // (a pair past the end reads the round's first pair, which exists)
      float ph[NPT], hx[NPT], hy[NPT], hz[NPT], V[NPT][6];
      uint32_t forig[NPT];
      const int p_first = __builtin_amdgcn_readfirstlane(__shfl(p[0], 0, 64));
#pragma unroll
      for (int h = 0; h < NPT; ++h) {
        const int ps = valid[h] ? p[h] : p_first;
        const float4* hp = A.hpack + (size_t)ps * 3;
        const float4 u0 = hp[0], u1 = hp[1], u2 = hp[2];
        ph[h] = u0.x;
        hx[h] = u0.y;
        hy[h] = u0.z;
        hz[h] = u0.w;
        V[h][0] = u1.x;
        V[h][1] = u1.y;
        V[h][2] = u1.z;
        V[h][3] = u1.w;
        V[h][4] = u2.x;
        V[h][5] = u2.y;
        forig[h] = __float_as_uint(u2.z);
      }
      // all loads in flight before the first test (the compiler would
      // otherwise wait for phi and issue the rest behind the phi test)
#pragma unroll
      for (int h = 0; h < NPT; ++h)
        asm volatile("" ::"v"(ph[h]), "v"(hx[h]), "v"(hy[h]), "v"(hz[h]), "v"(V[h][0]), "v"(V[h][1]), "v"(V[h][2]),
                     "v"(V[h][3]), "v"(V[h][4]), "v"(V[h][5]), "v"(forig[h]));
      bool keep[NPT], acc[NPT];
      float c2[NPT];
      uint32_t orig[NPT];
#pragma unroll
      for (int h = 0; h < NPT; ++h) {
        keep[h] = false;
        acc[h] = false;
        c2[h] = 0.f;
        orig[h] = 0;
        if (valid[h] && ph[h] >= ca[h] && ph[h] <= cb[h]) {
          tl.scanned += 1;
          const float cr = cx[h] * hy[h] - cy[h] * hx[h], dt = cx[h] * hx[h] + cy[h] * hy[h];
          const bool in_phi =
              ctan[h] < 0.f ? fabsf(atan2f(cr, dt)) <= cdphi[h] : (dt > 0.f && fabsf(cr) <= ctan[h] * dt);
          if (fabsf(hz[h] - cz[h]) <= cdz[h] && in_phi) {
            // innovation in the tangent-plane frame and its chi2 (2 dof)
            tl.tested += 1;
            const float ctx = -cy[h] * cirr[h], cty = cx[h] * cirr[h];
            const float r0 = ctx * (hx[h] - cx[h]) + cty * (hy[h] - cy[h]), r1 = hz[h] - cz[h];
            const float s00 = csuu[h] + ctx * ctx * V[h][0] + 2.f * ctx * cty * V[h][1] + cty * cty * V[h][3];
            const float s01 = csuw[h] + ctx * V[h][2] + cty * V[h][4];
            const float s11 = csww[h] + V[h][5];
            const float det = s00 * s11 - s01 * s01;
            if (s00 > 0.f && det > 0.f) {
              // (the hardware reciprocal: within a few ulp, no division sequence)
              c2[h] = (s11 * r0 * r0 - 2.f * s01 * r0 * r1 + s00 * r1 * r1) * k_rcp(det);
              if (c2[h] < cut) {
                acc[h] = true;
                orig[h] = forig[h];
                keep[h] = top_before(c2[h], orig[h], cthr[h], cthro[h]);
              }
            }
          }
        }
      }
      // the admissible hits of each half enter their candidates' lists
#pragma unroll
      for (int h = 0; h < NPT; ++h) {
        // this lane's run as a candidate in the half: lanes [s0, e0)
        const int bh = base + 64 * h;
        const int s0 = off - bh > 0 ? off - bh : 0;
        const int e0 = off + cnt - bh < 64 ? off + cnt - bh : 64;
        // accepted hits of each candidate: the accepted lanes of its run
        const unsigned long long am = __ballot(acc[h]);
        if (s0 < e0) n_acc += __builtin_popcountll(am & run_mask(s0, e0));
        const unsigned long long m = __ballot(keep[h]);
        if (m) {
          // the run of this lane's pair: from its candidate's mark to the next
          const unsigned long long above = sma[h] & ~((2ull << lane) - 1ull);
          const int rhi = above ? (int)__builtin_ctzll(above) : 64;
          round_insert(tl, A.cap, lane, m, keep[h], c2[h], p[h], orig[h], c[h], my_lo[h], rhi, s0, e0, held, unsorted,
                       thr_c2, thr_o, ab.pub_c2, ab.pub_o);
        }
      }
    }
  }
  if (unsorted) sort_own(tl, A.cap, held);
  tl.n = held;
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  tl.tot = n_acc;
}


// Waves per SIMD the register allocation aims at.  The build waits on
// memory and LDS most of the time, so a second resident wave pays even where
// it costs register spills (FP64: measured 26 % faster than one wave).  The
// macros allow a rebuild to compare.
#ifndef KF_BUILD_F32_WAVES
#define KF_BUILD_F32_WAVES 2
#endif
#ifndef KF_BUILD_F64_WAVES
#define KF_BUILD_F64_WAVES 2
#endif
#ifndef KF_BUILD_F64_LEARNED_WAVES
#define KF_BUILD_F64_LEARNED_WAVES 2
#endif

// Pairs per lane and round: NP in every build.  Learned FP64 builds took
// one while they spilled around the network (32 events: 17.35 -> 17.28 ms);
// with their state between layers in LDS two pay (11.45 -> 10.79 ms, hybrid
// state 11.40 -> 11.04 ms).  The macro allows a rebuild to compare.
#ifndef KF_LEARNED_F64_NPT
#define KF_LEARNED_F64_NPT 2
#endif
template <typename T, bool LEARNED>
constexpr int NPT_OF = (sizeof(T) == 8 && LEARNED) ? KF_LEARNED_F64_NPT : NP;

template <typename T, bool LEARNED, bool HYB>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? KF_BUILD_F32_WAVES
                                                       : (LEARNED ? KF_BUILD_F64_LEARNED_WAVES : KF_BUILD_F64_WAVES)))
    build_kernel(BuildArgs A) {
  const int S = A.cap;           // lanes per seed
  const int SEEDS = 64 / S;      // seeds per wave
  extern __shared__ __align__(16) uint32_t lds[];
  const int lane = threadIdx.x & 63;
  // the wave index as a uniform value in FP64 builds: the per-wave addresses
  // derived from it then stay in scalar registers (the FP32 build, which
  // does not spill, measured slower with it)
  const int wave = sizeof(T) == 8 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int LB = A.n_layers - A.first_layer;  // searched layers
  const LdsPlan lp = lds_plan(LB, nwaves, S, (int)sizeof(T), LEARNED, HYB);
  constexpr int NPL = xs_npl((int)sizeof(T), LEARNED, HYB);
  constexpr bool XS = NPL >= 0;  // state between layers in LDS
  char* base = (char*)lds;
  // this wave's back-pointer table (written once per new candidate and layer,
  // read once per seed at the end)
  uint32_t* hist = A.hist + ((size_t)blockIdx.x * nwaves + wave) * LB * 64;
  float* stash = (float*)(base + lp.stash) + (size_t)wave * (XS ? 21 - NPL : 27) * 64;
  T* xs = (T*)(base + lp.xs) + (size_t)wave * (XS ? 6 + NPL : 0) * 64 + lane;
  float* fin = (float*)(base + lp.rec) + (size_t)wave * SEEDS * 27;
  int32_t* finm = (int32_t*)(base + lp.recf) + (size_t)wave * SEEDS * 5;
  // per wave: the network buffer, or (after the network has run) the toplists
  char* wave_tl = base + lp.tl + (size_t)wave * lp.tl_stride;
  uint16_t* mlp_buf = (uint16_t*)wave_tl;
  float* tl_c2 = (float*)wave_tl + lane;
  int32_t* tl_pos = (int32_t*)(wave_tl + (size_t)S * 64 * 4) + lane;
  uint32_t* tl_orig = (uint32_t*)(wave_tl + (size_t)S * 64 * 8) + lane;
  AccBuf ab;
  ab.start = (int32_t*)(base + lp.acc) + (size_t)wave * 64 * NP;
  ab.pub_c2 = (float*)(base + lp.pub) + (size_t)wave * 128;
  ab.pub_o = (uint32_t*)ab.pub_c2 + 64;
  (void)mlp_buf;
  const int sidx = lane / S, slot = lane - (lane / S) * S, sbase = sidx * S;
  const bool lane_used = sidx < SEEDS;

  if (A.start_tick && lane == 0) atomicMin((unsigned long long*)A.start_tick, (unsigned long long)wall_clock64());

  for (;;) {
    int grp = 0;
    if (lane == 0) grp = atomicAdd(A.queue, 1);
    grp = __shfl(grp, 0, 64);
    if (grp >= A.n_groups) break;
    const int gi = grp * SEEDS + sidx;
    int seed = (lane_used && gi < A.n_seeds) ? (A.seed_order ? A.seed_order[gi] : gi) : -1;
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
    if constexpr (HYB) {  // the seed in the hybrid state
      if (seed_ok) {
        T Y[6], B[9];
        hyb_from_cart(X, q, Y, B);
        congruence_mom(P, B);
#pragma unroll
        for (int k = 0; k < 6; ++k) X[k] = Y[k];
      }
    }
    T chi2 = 0;
    int nhits = 0, holes = 0;
    bool ontrack = true;
    int n_active = seed_ok ? 1 : 0;
    int seed_status = 0;
    if (lane_used && slot == 0) finm[sidx * 5 + 0] = 0;
    // a non-finite seed, or one whose event holds more hits than 24-bit
    // event-local indices can name, is its own (finished) result
    const int bad = !seed_ok ? 0
                    : event_too_large(A.offsets, ev, A.n_layers, A.n_phi * A.n_z) ? KF_EVENT_TOO_LARGE
                    : !(all_finite(X, 6) && all_finite(P, 21))                     ? KF_NONFINITE
                                                                                   : 0;
    if (bad) {
      if (slot == 0) {
        finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = 0; finm[sidx * 5 + 2] = bad;
        finm[sidx * 5 + 3] = A.first_layer - 1; finm[sidx * 5 + 4] = 0;
        for (int k = 0; k < 6; ++k) fin[sidx * 27 + k] = (float)X[k];
        for (int k = 0; k < 21; ++k) fin[sidx * 27 + 6 + k] = (float)P[k];
      }
      n_active = 0;
    }
    if constexpr (XS) {
#pragma unroll
      for (int k = 0; k < 6; ++k) xs[k * 64] = X[k];
#pragma unroll
      for (int k = 0; k < NPL; ++k) xs[(6 + k) * 64] = P[21 - NPL + k];
    }
    T fin_chi2_reg = 0;  // chi2 of the finished record, kept by slot 0 of the seed
    unsigned cnt_pred = 0, cnt_scan = 0, cnt_chi2 = 0, cnt_upd = 0;
    int last_l = A.first_layer - 1;
    for (int l = A.first_layer; l < A.n_layers; ++l) {
      // all seeds of the wave done?
      if (!__any(n_active > 0)) break;
      last_l = l;
      const bool live = slot < n_active;
      if constexpr (XS) {
#pragma unroll
        for (int k = 0; k < 6; ++k) X[k] = xs[k * 64];
#pragma unroll
        for (int k = 0; k < NPL; ++k) P[21 - NPL + k] = xs[(6 + k) * 64];
      }
      // the state before prediction is kept (in the output precision) for
      // the finished record, so it need not stay in registers (the part held
      // in LDS is read from there)
      if (live) {
        if constexpr (XS) {
#pragma unroll
          for (int k = 0; k < 21 - NPL; ++k) stash[k * 64 + lane] = (float)P[k];
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k) stash[k * 64 + lane] = (float)X[k];
#pragma unroll
          for (int k = 0; k < 21; ++k) stash[(6 + k) * 64 + lane] = (float)P[k];
        }
      }
      T Xp[6], Pp[21];
      int rc = 1;
      if (live) {
        if constexpr (HYB)
          rc = predict_hyb<T>(X, P, (T)A.r[l], (T)ku64<T>(A.bz), (T)ku64<T>(A.z_half), (T)ku64<T>(A.x_over_x0),
                              (T)ku64<T>(A.mass), Xp, Pp);
        else
          rc = predict<T>(X, P, kv64<T>(q), (T)A.r[l], (T)ku64<T>(A.bz), (T)ku64<T>(A.z_half),
                          (T)ku64<T>(A.x_over_x0), (T)ku64<T>(A.mass), Xp, Pp);
      }
      else {
#pragma unroll
        for (int k = 0; k < 6; ++k) Xp[k] = T(0);
#pragma unroll
        for (int k = 0; k < 21; ++k) Pp[k] = T(0);
      }
      const bool pok = live && rc == 0;
      TopList tl;
      tl.c2 = tl_c2;
      tl.pos = tl_pos;
      tl.orig = tl_orig;
      tl.n = 0;
      tl.tot = 0;
      tl.scanned = 0;
      tl.tested = 0;
      // plain window from the predicted covariance
      T w_rphi = T(0), w_z = T(0);
      const T R = (T)A.r[l];
      if (pok) {
        const T rr = k_sqrt(Xp[0] * Xp[0] + Xp[1] * Xp[1]);
        const T tx = -Xp[1] / rr, ty = Xp[0] / rr;
        const T Suu = tx * tx * Pp[ut(0, 0)] + T(2) * tx * ty * Pp[ut(0, 1)] + ty * ty * Pp[ut(1, 1)] +
                      sq((T)ku64<T>(A.win_sig_rphi));
        const T Sww = Pp[ut(2, 2)] + sq((T)ku64<T>(A.win_sig_z));
        w_rphi = (T)ku64<T>(A.nsigma) * k_sqrt(Suu);
        w_z = (T)ku64<T>(A.nsigma) * k_sqrt(Sww);
        if (A.dump && ontrack && A.true_hits) {
          const int th = A.true_hits[(size_t)l * A.ld + seed];
          if (th >= 0) {
            const int row = atomicAdd(A.dump_count, 1);
            if (row < A.dump_capacity) {
              float* d = A.dump + (size_t)row * KFMLP_DUMP_ROW;
              if constexpr (HYB) {
                // the features the network reads: the Cartesian prediction
                T Xc[6], Am[9], Pc[21];
                (void)cart_from_hyb(Xp, Xc, Am);
                for (int k = 0; k < 21; ++k) Pc[k] = Pp[k];
                congruence_mom(Pc, Am);
                for (int k = 0; k < 6; ++k) d[k] = (float)Xc[k];
                for (int k = 0; k < 21; ++k) d[6 + k] = (float)Pc[k];
              } else {
                for (int k = 0; k < 6; ++k) d[k] = (float)Xp[k];
                for (int k = 0; k < 21; ++k) d[6 + k] = (float)Pp[k];
              }
              const T mx = (T)A.true_xyz[((size_t)l * 3 + 0) * A.ld + seed];
              const T my = (T)A.true_xyz[((size_t)l * 3 + 1) * A.ld + seed];
              const T mz = (T)A.true_xyz[((size_t)l * 3 + 2) * A.ld + seed];
              const T dph = k_atan2(Xp[0] * my - Xp[1] * mx, Xp[0] * mx + Xp[1] * my);
              d[27] = (float)(R * fabs(dph));
              d[28] = (float)fabs(mz - Xp[2]);
              // the plain half-widths this candidate's window has (the gates
              // of the learned window are set from them)
              d[29] = (float)w_rphi;
              d[30] = (float)w_z;
              d[31] = __int_as_float((int)(((uint32_t)seed << 8) | ((uint32_t)l << 3) | (uint32_t)slot));
            }
          }
        }
      }
      if constexpr (LEARNED) {
        // learned window where the plain one is wide (either half-width above
        // its gate): the wave evaluates the network on those slots only
        const bool gated = pok && (w_rphi > (T)A.mlp[KFMLP_OFF_GATE] || w_z > (T)A.mlp[KFMLP_OFF_GATE + 1]);
        // the features rounded to FP32 first and pinned there by an empty
        // asm: converted inside the row writes instead, the FP64 build's
        // register allocation spilled twice as much
        float feat[27];
        if constexpr (HYB) {
          // the network reads the Cartesian prediction: convert the hybrid
          // one (state, and covariance through d(X)/d(Y))
          T Xc[6], Am[9], Pc[21];
          (void)cart_from_hyb(Xp, Xc, Am);
#pragma unroll
          for (int k = 0; k < 21; ++k) Pc[k] = Pp[k];
          congruence_mom(Pc, Am);
#pragma unroll
          for (int k = 0; k < 27; ++k) feat[k] = (float)(k < 6 ? Xc[k] : Pc[k - 6]);
        } else {
#pragma unroll
          for (int k = 0; k < 27; ++k) feat[k] = (float)(k < 6 ? Xp[k] : Pp[k - 6]);
        }
#pragma unroll
        for (int k = 0; k < 27; ++k) asm volatile("" : "+v"(feat[k]));
        const uint64_t act = kfmlp::wave_stage(A.mlp, mlp_buf, [&](int k) { return feat[k]; }, gated);
        float o[2] = {0.f, 0.f};
        if (act) kfmlp::wave_tiles(A.mlp, mlp_buf, act, o);
        if (gated) {
          const float kap = A.mlp[KFMLP_OFF_KAPPA];
          float wl[2] = {A.mlp[KFMLP_OFF_SCALE] * kfmlp::softplus(o[0]),
                         A.mlp[KFMLP_OFF_SCALE + 1] * kfmlp::softplus(o[1])};
          wl[0] *= kap;
          wl[1] *= kap;
          if (!(wl[0] < A.mlp[KFMLP_OFF_FLOOR])) w_rphi = (T)wl[0];
          if (!(wl[1] < A.mlp[KFMLP_OFF_FLOOR + 1])) w_z = (T)wl[1];
        }
      }
      const T dphi_w = pok ? w_rphi / R : T(0), dz_w = pok ? w_z : T(0);
      coop_scan<T, NPT_OF<T, LEARNED>>(A, kv64<T>(ev), l, pok, Xp, Pp, dphi_w, dz_w, tl, ab, lane);
      const bool hole_ok = pok && holes < A.max_holes;
      const int nchild = tl.tot + (hole_ok ? 1 : 0);
      // finished candidates of this layer (live, no child) compete for the record
      if (__any(live && nchild == 0)) {  // (most layers have none)
        const bool stopped = live && nchild == 0;
        uint64_t fk = stopped ? make_key(nhits, (float)chi2, slot, 0) : kInfKey;
        const uint64_t best = group_min(fk, sbase, slot, S, lane_used);
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
              if constexpr (XS) {
                for (int k = 0; k < 6; ++k) fin[sidx * 27 + k] = (float)xs[k * 64];
                for (int k = 0; k < 21 - NPL; ++k) fin[sidx * 27 + 6 + k] = stash[k * 64 + lane];
                for (int k = 21 - NPL; k < 21; ++k) fin[sidx * 27 + 6 + k] = (float)xs[(6 + k - 21 + NPL) * 64];
              } else {
                for (int k = 0; k < 27; ++k) fin[sidx * 27 + k] = stash[k * 64 + lane];
              }
              finm[sidx * 5 + 0] = 1; finm[sidx * 5 + 1] = wn; finm[sidx * 5 + 2] = wst;
              finm[sidx * 5 + 3] = l - 1; finm[sidx * 5 + 4] = ws;
            }
            if (slot == 0) fin_chi2_reg = wc2;
          }
        }
      }
      // merge the children of the seed, best first, into slots 0..cap-1
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
        if (win == kInfKey) continue;  // no more children for this seed
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
          const float4* hp = A.hpack + (size_t)my_pos * 3;
          const float4 u0 = hp[0], u1 = hp[1], u2 = hp[2];
          const T hx = (T)u0.y, hy = (T)u0.z, hz = (T)u0.w;
          const T V[6] = {(T)u1.x, (T)u1.y, (T)u1.z, (T)u1.w, (T)u2.x, (T)u2.y};
          Innov<T> in;
          innovation<T>(Xn, Pn, hx, hy, hz, V, in);
          apply_update<T>(Xn, Pn, in);
        }
        if constexpr (XS) {
#pragma unroll
          for (int k = 0; k < 6; ++k) xs[k * 64] = Xn[k];
#pragma unroll
          for (int k = 0; k < NPL; ++k) xs[(6 + k) * 64] = Pn[21 - NPL + k];
#pragma unroll
          for (int k = 0; k < 21 - NPL; ++k) P[k] = Pn[k];
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k) X[k] = Xn[k];
#pragma unroll
          for (int k = 0; k < 21; ++k) P[k] = Pn[k];
        }
        chi2 = is_hole ? pchi2 : pchi2 + my_c2;
        nhits = is_hole ? pnh : pnh + 1;
        holes = is_hole ? pho + 1 : pho;
        if (A.dump && A.true_hits) {
          const int th = seed_ok ? A.true_hits[(size_t)l * A.ld + seed] : -1;
          ontrack = pon && (is_hole || (int)my_orig == th);
        }
        hist[(l - A.first_layer) * 64 + lane] = pack_hist(my_parent, my_orig);
      }
      cnt_pred += live ? 1u : 0u;
      cnt_scan += (unsigned)tl.scanned;
      cnt_chi2 += (unsigned)tl.tested;
      cnt_upd += my_parent >= 0 && my_orig != kHoleIdx ? 1u : 0u;
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
      const uint64_t best = group_min(k, sbase, slot, S, lane_used);
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
      const int fvalid = lane_used ? finm[sidx * 5 + 0] : 0;
      const int fn = lane_used ? finm[sidx * 5 + 1] : 0;
      const bool use_fin = fvalid && (bslot < 0 || fn > bn || (fn == bn && fc2 < bc2));
      if (seed_ok) {
        // state: the best lane writes its own; slot 0 writes the record
        if (!use_fin && slot == bslot) {
          for (int k2 = 0; k2 < 6; ++k2) A.out_par[(size_t)k2 * A.ld + seed] = (float)(XS ? xs[k2 * 64] : X[k2]);
          for (int k2 = 0; k2 < 21; ++k2)
            A.out_cov[(size_t)k2 * A.ld + seed] =
                (float)(XS && k2 >= 21 - NPL ? xs[(6 + k2 - 21 + NPL) * 64] : P[k2]);
          A.out_chi2[seed] = (float)chi2;
          A.out_nhits[seed] = nhits;
          A.out_status[seed] = seed_status;
        }
        if (use_fin && slot == 0) {
          for (int k2 = 0; k2 < 6; ++k2) A.out_par[(size_t)k2 * A.ld + seed] = fin[sidx * 27 + k2];
          for (int k2 = 0; k2 < 21; ++k2) A.out_cov[(size_t)k2 * A.ld + seed] = fin[sidx * 27 + 6 + k2];
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

int refine_of(const kf_build_params* bp) { return bp->phi_refine > 0 ? bp->phi_refine : 64; }

// the launch shape of the last kf_build call of this host thread
thread_local kf_build_launch_info g_last_launch = {};

template <typename T, bool LEARNED, bool HYB>
int launch(const BuildArgs& A, int lanes, int blocks, int hist_waves, hipStream_t s) {
  const int LB = A.n_layers - A.first_layer;
  int dev = 0, max_lds = 0;
  if (kf_check(hipGetDevice(&dev))) return KF_E_HIP;
  if (kf_check(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev))) return KF_E_HIP;
  auto plan = [&](int ln) { return lds_plan(LB, ln / 64, A.cap, (int)sizeof(T), LEARNED, HYB).total; };
  if (lanes == 0) {  // automatic: the widest block whose LDS fits
    lanes = 256;
    while (lanes > 64 && plan(lanes) > (size_t)max_lds) lanes /= 2;
  }
  const int nwaves = lanes / 64;
  const size_t lds = plan(lanes);
  if (lds > (size_t)max_lds) return KF_E_UNSUPPORTED;
  if (lds > (size_t)64 * 1024 &&
      kf_check(hipFuncSetAttribute((const void*)build_kernel<T, LEARNED, HYB>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)))
    return KF_E_HIP;
  int cus = 0, per = 0;
  if (kf_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))) return KF_E_HIP;
  if (kf_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, build_kernel<T, LEARNED, HYB>, lanes, lds)))
    return KF_E_HIP;
  if (blocks <= 0) blocks = cus * (per > 0 ? per : 1);
  const int need = (A.n_groups + nwaves - 1) / nwaves;
  if (blocks > need) blocks = need;
  if (blocks > hist_waves / nwaves) blocks = hist_waves / nwaves;  // history tables in the workspace
  if (blocks < 1) return KF_E_WORKSPACE;
  g_last_launch.lanes_per_block = lanes;
  g_last_launch.blocks = blocks;
  g_last_launch.lds_bytes = (int32_t)lds;
  g_last_launch.resident_blocks_per_cu = per;
  g_last_launch.max_lds_per_block = max_lds;
  hipLaunchKernelGGL((build_kernel<T, LEARNED, HYB>), dim3(blocks), dim3(lanes), lds, s, A);
  return kf_check_launch();
}

}  // namespace

extern "C" int kf_build_last_launch(kf_build_launch_info* info) {
  if (!info) return KF_E_INVALID_ARG;
  *info = g_last_launch;
  return KF_OK;
}

extern "C" size_t kf_build_workspace_bytes(const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds) {
  (void)n_seeds;
  if (!bp || !hits || hits->n_events < 1 || hits->n_layers < 1 || hits->n_phi < 1 || hits->n_z < 1) return 0;
  if (bp->first_layer < 1 || bp->first_layer >= hits->n_layers) return 0;
  const size_t LB = (size_t)(hits->n_layers - bp->first_layer);
  if (hits->n_hits < 0) return 0;
  return ws_head_bytes(hits->n_events) +
         ((fine_bytes(hits->n_events, hits->n_layers, hits->n_phi, hits->n_z, refine_of(bp)) + 255) & ~(size_t)255) +
         pack_bytes(hits->n_hits) + (size_t)hist_waves_of_device() * LB * 64 * 4;
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
  if (bp->phi_refine < 0 || bp->phi_refine > 64) return KF_E_INVALID_ARG;
  if (bp->arith != KF_ARITH_F32 && bp->arith != KF_ARITH_F64) return KF_E_INVALID_ARG;
  if (bp->window_mode != 0 && bp->window_mode != 1) return KF_E_INVALID_ARG;
  if (bp->window_mode == 1 && !bp->mlp) return KF_E_INVALID_ARG;
  if (bp->state != 0 && bp->state != 1) return KF_E_INVALID_ARG;
  if (hits->n_layers != g->n_layers || hits->n_events < 1 || hits->n_phi < 1 || hits->n_z < 1 || hits->n_hits < 0)
    return KF_E_INVALID_ARG;
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
  const int refine = refine_of(bp);
  if ((int64_t)hits->n_phi * refine > (1 << 20)) return KF_E_UNSUPPORTED;
  const size_t need = kf_build_workspace_bytes(bp, hits, n_seeds);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return KF_E_WORKSPACE;
  const int lanes = bp->lanes_per_block;
  if (lanes != 0 && lanes != 64 && lanes != 128 && lanes != 256) return KF_E_UNSUPPORTED;

  BuildArgs A;
  A.n_layers = g->n_layers;
  for (int i = 0; i < 32; ++i) A.r[i] = g->r[i];
  A.z_half = g->z_half; A.bz = g->bz; A.x_over_x0 = g->x_over_x0; A.mass = g->mass;
  A.chi2_cut = bp->chi2_cut; A.max_holes = bp->max_holes; A.cap = bp->cand_cap;
  A.nsigma = bp->nsigma; A.win_sig_rphi = bp->win_sig_rphi; A.win_sig_z = bp->win_sig_z;
  A.first_layer = bp->first_layer; A.window_mode = bp->window_mode; A.mlp = (const float*)bp->mlp;
  A.n_events = hits->n_events; A.n_phi = hits->n_phi; A.n_z = hits->n_z; A.offsets = hits->offsets;
  A.n_hits = hits->n_hits;
  A.refine = refine;
  const size_t fine_off = ws_head_bytes(hits->n_events);
  A.fine = (const int32_t*)((char*)ws + fine_off);
  const size_t pack_off =
      fine_off + ((fine_bytes(hits->n_events, hits->n_layers, hits->n_phi, hits->n_z, refine) + 255) & ~(size_t)255);
  A.hpack = (const float4*)((char*)ws + pack_off);
  const size_t hist_off = pack_off + pack_bytes(hits->n_hits);
  A.hist = (uint32_t*)((char*)ws + hist_off);
  const size_t LBw = (size_t)(g->n_layers - bp->first_layer) * 64 * 4;
  const int hist_waves = (int)((ws_bytes - hist_off) / LBw);
  const int seeds_per_wave = 64 / bp->cand_cap;
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
  {
    const int n_rows = hits->n_events * hits->n_layers * hits->n_z;
    hipLaunchKernelGGL(fine_kernel, dim3((n_rows + 3) / 4), dim3(256), 0, s, n_rows, hits->n_phi, hits->n_z,
                       hits->n_phi * refine, hits->offsets, hits->phi, (int32_t*)A.fine);
    if (int rc = kf_check_launch()) return rc;
    if (hits->n_hits > 0) {
      hipLaunchKernelGGL(pack_kernel, dim3((hits->n_hits + 255) / 256), dim3(256), 0, s, hits->n_hits, hits->x,
                         hits->y, hits->z, hits->phi, hits->cov, hits->orig, (float4*)A.hpack);
      if (int rc = kf_check_launch()) return rc;
    }
  }
  if (bp->arith == KF_ARITH_F64)
    return bp->state == 1
               ? (bp->window_mode == 1 ? launch<double, true, true>(A, lanes, bp->persistent_blocks, hist_waves, s)
                                       : launch<double, false, true>(A, lanes, bp->persistent_blocks, hist_waves, s))
               : (bp->window_mode == 1 ? launch<double, true, false>(A, lanes, bp->persistent_blocks, hist_waves, s)
                                       : launch<double, false, false>(A, lanes, bp->persistent_blocks, hist_waves, s));
  return bp->state == 1
             ? (bp->window_mode == 1 ? launch<float, true, true>(A, lanes, bp->persistent_blocks, hist_waves, s)
                                     : launch<float, false, true>(A, lanes, bp->persistent_blocks, hist_waves, s))
             : (bp->window_mode == 1 ? launch<float, true, false>(A, lanes, bp->persistent_blocks, hist_waves, s)
                                     : launch<float, false, false>(A, lanes, bp->persistent_blocks, hist_waves, s));
}

// ------------------------------------------------- allocation-free variant
//
// kf_build_noalloc runs kf_build with its workspace in `scratch`, a static
// device array of this library: every GPU the library runs on holds its own
// copy (kScratchBytes) until the process ends.  In host code the array's
// name stands for a host-side shadow, not a device address: the device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that pointer is handed to kernels.  What the
// build needs zeroed (queue head, per-event counters) is cleared by a kernel
// of every call; the fine index and the packed hits are rebuilt by every
// call; so the contents left by the previous call do not matter.  Calls that
// overlap on one GPU share the array and race.

static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of this device's copy of `scratch`
int scratch_of_current_device(void** out) {
  int dev = 0;
  if (kf_check(hipGetDevice(&dev))) return KF_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return kf_fail(KF_E_UNSUPPORTED, "kf_build_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (kf_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return KF_E_HIP;
    if (!p) return kf_fail(KF_E_HIP, "kf_build_noalloc: no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return KF_OK;
}

}  // namespace

extern "C" size_t kf_build_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int kf_build_noalloc(const kf_geometry* g, const kf_build_params* bp, const kf_hits* hits,
                                int32_t n_seeds, int32_t ld, const float* seed_par, const float* seed_cov,
                                const int8_t* q, int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2,
                                int32_t* out_nhits, int32_t* out_status, const kf_build_extra* extra, void* stream) {
  if (kf_check_geometry(g) || !bp || !hits) return KF_E_INVALID_ARG;
  const size_t need = kf_build_workspace_bytes(bp, hits, n_seeds);
  if (need == 0) return KF_E_INVALID_ARG;
  if (need > kScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof(msg), "kf_build_noalloc: this call needs %zu workspace bytes, the static scratch holds %zu",
             need, kScratchBytes);
    return kf_fail(KF_E_WORKSPACE, msg);
  }
  void* ws = nullptr;
  if (int rc = scratch_of_current_device(&ws)) return rc;
  return kf_build(g, bp, hits, n_seeds, ld, seed_par, seed_cov, q, out_hits, out_par, out_cov, out_chi2, out_nhits,
                  out_status, extra, ws, kScratchBytes, stream);
}
