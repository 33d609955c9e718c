// Device-side Kalman-filter arithmetic for barrel tracking on gfx950.
//
// Everything here works on one candidate held in registers of one lane:
// state X[6] = (x, y, z, px, py, pz), covariance P[21] (upper triangle, row
// order).  The functions are templated on the scalar type: the fit and build
// kernels use float, or double in their precise mode; the seed kernel double.
//
// Formulation choices for FP32 (the FP64 oracle uses textbook closed forms):
//   - the crossing with the cylinder is solved for tan(alpha/2) of the turning
//     angle from a quadratic whose coefficients carry no large cancelling
//     terms (the circle-intersection form cancels |C|^2 - rho^2 ~ 1e6 cm^2 at
//     10 GeV);
//   - the transverse displacement is written with sin(alpha)/h and
//     2 sin^2(alpha/2)/h, so it stays accurate as h -> 0;
//   - the Jacobian uses only nonzero blocks; the covariance update touches
//     only the upper triangle;
//   - quotients by one denominator share its reciprocal (FP32: the hardware
//     reciprocal, within 1 ulp; FP64: a correctly rounded 1/x).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// The arithmetic is also compiled for the host (a CPU build of the same
// functions is used to inspect individual candidates).
#define KFD __host__ __device__

namespace kfdev {

constexpr int KF_NO_CROSSING = 1;
constexpr int KF_OUT_OF_Z = 2;
constexpr int KF_NONFINITE = 4;
constexpr int KF_S_NOT_PD = 8;
constexpr int KF_CAP_TRUNC = 16;
constexpr int KF_EVENT_TOO_LARGE = 32;

// GeV / (T cm): pT = KAPPA * B * rho
template <typename T> KFD constexpr T kappa() { return T(0.299792458e-2); }

// index of (i, j), i <= j, in the 21-entry upper triangle
__host__ __device__ constexpr int ut(int i, int j) {
  return i <= j ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j);
}

template <typename T> KFD inline T sq(T v) { return v * v; }

KFD inline float k_sqrt(float v) { return __builtin_sqrtf(v); }
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline float k_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
#else
inline float k_rcp(float v) { return 1.0f / v; }
#endif
KFD inline double k_rcp(double v) { return 1.0 / v; }
KFD inline double k_sqrt(double v) { return __builtin_sqrt(v); }
KFD inline void k_sincos(float a, float* s, float* c) { sincosf(a, s, c); }
KFD inline void k_sincos(double a, double* s, double* c) { sincos(a, s, c); }
KFD inline float k_atan2(float y, float x) { return atan2f(y, x); }
KFD inline double k_atan2(double y, double x) { return atan2(y, x); }
KFD inline float k_tan(float v) { return tanf(v); }
KFD inline double k_tan(double v) { return tan(v); }
KFD inline float k_atan(float v) { return atanf(v); }
KFD inline float k_log(float v) { return logf(v); }

// A double constant materialised where it is used: the empty asm (scalar
// registers) keeps the compiler from hoisting it out of the layer loop,
// where every series coefficient would hold two registers throughout.
KFD inline double kc(double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(c));
#endif
  return c;
}

// A kernel argument read where it is used (the empty asm on its scalar
// register): what is computed from it in vector registers (an FP64
// conversion, a square) is then recomputed inside the layer loop, not
// hoisted out of it and spilled to scratch memory.
template <typename U> KFD inline U ku(U v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(v));
#endif
  return v;
}

// A per-lane value made opaque where it is used (the empty asm on its
// vector register): what is computed from it is recomputed there, not held
// through the layer loop (or spilled) as a loop-invariant value.
template <typename U> KFD inline U kv(U v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#endif
  return v;
}

// FP64 arctangent and logarithm written out from textbook identities: inside
// the build kernels, which are short of registers, the library routines made
// the compiler spill around every call (the arctangent alone cost 15 % of
// the FP64 build).  Their series coefficients go through kc().  Both stay
// within a few ulp of the correctly rounded value (a CPU test checks them
// against the host library).
//
// atan: |x| > 1 folds to pi/2 - atan(1/|x|); arguments above 0.05 are
// halved (at most four times) by atan(x) = 2 atan(x / (1 + sqrt(1 + x^2)));
// on |x| <= 0.05 the odd Taylor series x sum (-1)^k x^2k / (2k + 1) to x^13
// (the first term left out is below 1e-19 of the sum).  The propagation's
// arguments (tangents of half the turning angle between layers) are mostly
// below 0.05, where no halving runs.
KFD inline double k_atan(double v) {
  double x = fabs(v);
  const bool inv = x > 1.0;
  if (inv) x = 1.0 / x;
  double scale = 1.0;
  while (x > 0.05) {
    x = x / (1.0 + __builtin_sqrt(1.0 + x * x));
    scale *= 2.0;
  }
  const double u = x * x;
  double p = 1.0 / 13.0;
  p = __builtin_fma(p, u, kc(-1.0 / 11.0));
  p = __builtin_fma(p, u, kc(1.0 / 9.0));
  p = __builtin_fma(p, u, kc(-1.0 / 7.0));
  p = __builtin_fma(p, u, kc(1.0 / 5.0));
  p = __builtin_fma(p, u, kc(-1.0 / 3.0));
  double r = scale * __builtin_fma(x * u, p, x);
  if (inv) r = 1.5707963267948966 - r;
  return __builtin_copysign(r, v);
}

// log: v = m 2^e with m in [sqrt(1/2), sqrt(2)), log m = 2 atanh(f) with
// f = (m - 1) / (m + 1), |f| <= 0.172, the series 2 f sum f^2k / (2k + 1) to
// f^23; e ln 2 added in two parts (Cody and Waite's split of ln 2, whose
// leading part times a small integer is exact).  Zero, negative, infinite and
// NaN arguments give the IEEE results.
KFD inline double k_log(double v) {
  if (!(v > 0.0)) return v == 0.0 ? -__builtin_inf() : __builtin_nan("");
  if (!__builtin_isfinite(v)) return v;
  int e = 0;
  double m = __builtin_frexp(v, &e);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = (m - 1.0) / (m + 1.0), f2 = f * f;
  double p = 1.0 / 23.0;
  p = __builtin_fma(p, f2, kc(1.0 / 21.0));
  p = __builtin_fma(p, f2, kc(1.0 / 19.0));
  p = __builtin_fma(p, f2, kc(1.0 / 17.0));
  p = __builtin_fma(p, f2, kc(1.0 / 15.0));
  p = __builtin_fma(p, f2, kc(1.0 / 13.0));
  p = __builtin_fma(p, f2, kc(1.0 / 11.0));
  p = __builtin_fma(p, f2, kc(1.0 / 9.0));
  p = __builtin_fma(p, f2, kc(1.0 / 7.0));
  p = __builtin_fma(p, f2, kc(1.0 / 5.0));
  p = __builtin_fma(p, f2, kc(1.0 / 3.0));
  const double lm = 2.0 * __builtin_fma(f * f2, p, f);
  const double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
  return (double)e * ln2_hi + ((double)e * ln2_lo + lm);
}
KFD inline bool k_finite(float v) { return __builtin_isfinite(v); }
KFD inline bool k_finite(double v) { return __builtin_isfinite(v); }

// Helix in B = bz * zhat after a turn alpha = h*s (h = -q*KAPPA*bz/pT,
// s = transverse path):
//   pos(s) = pos + t * sin(a)/h + n * (1 - cos(a))/h,   t = p_T/pT, n = zhat x t
//   p_T(s) = rotation of p_T by a,   z(s) = z + pz * s / pT.
// Crossing with r = R.  With u = pos.t, v = pos.n, D = R^2 - r0^2, the
// condition |pos(s)|^2 = R^2 becomes, for tau = tan(alpha/2),
//   (2b - c) tau^2 + 2 a tau - c = 0,  a = h u, b = 1 + h v, c = h^2 D / 2.
// tau covers one full turn (alpha in (-pi, pi)); both roots are formed in
// the cancellation-free pair q/A, -c/q with q = -(a + sign(a) sqrt(disc)).
// The first crossing along the motion is the root whose turn, taken with the
// sign of h and in (0, 2 pi) in magnitude, is smallest.  NEAREST: the
// crossing reached by the smallest turn forwards or backwards (|alpha| < pi,
// the root of smallest |tau|); s then has either sign.
template <typename T> struct Step {
  T s;      // transverse path
  T alpha;  // turning angle
  T sa, ca; // sin(alpha), cos(alpha)
  T A, B;   // sin(alpha)/h, (1 - cos(alpha))/h
  T h, pt, ipt;  // ipt = 1 / pt
};

template <typename T, bool NEAREST = false>
KFD inline int propagate(const T X[6], int q, T R, T bz, T Xo[6], Step<T>& st) {
  const T px = X[3], py = X[4], pz = X[5];
  const T pt2 = px * px + py * py;
  const T pt = k_sqrt(pt2);
  if (!(pt > T(0))) return KF_NO_CROSSING;
  const T ipt = k_rcp(pt);
  const T h = -T(q) * kappa<T>() * bz * ipt;
  const T tx = px * ipt, ty = py * ipt;
  const T u = X[0] * tx + X[1] * ty;
  const T v = -X[0] * ty + X[1] * tx;
  const T r02 = X[0] * X[0] + X[1] * X[1];
  const T D = R * R - r02;
  const T a = h * u;
  const T b = T(1) + h * v;
  const T c = T(0.5) * h * h * D;
  const T A2 = T(2) * b - c;
  const T disc = a * a + c * A2;
  if (!(disc >= T(0))) return KF_NO_CROSSING;
  const T sd = k_sqrt(disc);
  const T qq = -(a + (a >= T(0) ? sd : -sd));
  const T sg = h > T(0) ? T(1) : T(-1);
  // the two roots, oriented so that the motion turns towards positive tau
  const T t1 = sg * (qq / A2), t2 = sg * (-c / qq);
  // first along the motion: the smallest positive oriented root if any,
  // otherwise the most negative one (a turn beyond pi)
  T t;
  if constexpr (NEAREST) {
    t = (fabs(t2) < fabs(t1) || !(t1 == t1)) ? t2 : t1;
  } else {
    if (t1 > T(0) && t2 > T(0)) t = t1 < t2 ? t1 : t2;
    else if (t1 > T(0)) t = t1;
    else if (t2 > T(0)) t = t2;
    else t = t1 < t2 ? t1 : t2;
  }
  if (!(t == t)) return KF_NO_CROSSING;  // both roots undefined (degenerate circle)
  T half = k_atan(t);
  if constexpr (!NEAREST) {
    if (!(half > T(0))) half += T(3.14159265358979323846);
  }
  half *= sg;
  const T alpha = T(2) * half;
  // sin(alpha) and 1 - cos(alpha) from tau = tan(alpha / 2) = sg * t (tan has
  // period pi, so the turn beyond pi shares t): 2 tau / (1 + tau^2) and
  // 2 tau^2 / (1 + tau^2); an infinite t is the half turn
  T sa, omc;
  if (fabs(t) < T(1e18)) {  // t * t stays finite in FP32
    const T iw = k_rcp(T(1) + t * t);
    sa = T(2) * sg * t * iw;
    omc = T(2) * t * t * iw;
  } else {
    sa = T(0);
    omc = T(2);
  }
  const T ca = T(1) - omc;
  const T ih = k_rcp(h);
  const T s = alpha * ih;
  if (!NEAREST && !(s > T(0))) return KF_NO_CROSSING;
  const T Ah = sa * ih, Bh = omc * ih;
  Xo[0] = X[0] + tx * Ah - ty * Bh;
  Xo[1] = X[1] + ty * Ah + tx * Bh;
  Xo[2] = X[2] + pz * s * ipt;
  Xo[3] = px * ca - py * sa;
  Xo[4] = py * ca + px * sa;
  Xo[5] = pz;
  st.s = s; st.alpha = alpha; st.sa = sa; st.ca = ca; st.A = Ah; st.B = Bh; st.h = h; st.pt = pt; st.ipt = ipt;
  return 0;
}

// Covariance transport P <- J P J^T for the map "state -> state at the
// crossing" (J = Js + w g^T: Js at fixed path, w = dX/ds, g = ds/dX keeps the
// end point on the cylinder), then + Q (Highland scattering at the new point).
// Nonzero pattern of J: rows x, y, px, py use columns {x, y, px, py}; row z
// uses all six; row pz is the identity.
template <typename T>
KFD inline void transport(const T X0[6], const T X1[6], const Step<T>& st, T P[21], T x_over_x0, T mass) {
  const T px = X0[3], py = X0[4], pz = X0[5];
  const T ipt = st.ipt, ipt2 = ipt * ipt, ipt3 = ipt2 * ipt;
  const T s = st.s;
  const T px1 = X1[3], py1 = X1[4];
  const T aox = st.alpha * ipt2;  // d(alpha)/d(px) = -aox*px
  // Js entries (rows x, y, z, px, py at columns px, py, pz)
  const T sp3 = s * ipt3;
  const T j03 = st.A * ipt - px1 * px * sp3;
  const T j04 = -st.B * ipt - px1 * py * sp3;
  const T j13 = st.B * ipt - py1 * px * sp3;
  const T j14 = st.A * ipt - py1 * py * sp3;
  const T j23 = -pz * px * sp3;
  const T j24 = -pz * py * sp3;
  const T j25 = s * ipt;
  const T j33 = st.ca + py1 * aox * px;
  const T j34 = -st.sa + py1 * aox * py;
  const T j43 = st.sa - px1 * aox * px;
  const T j44 = st.ca - px1 * aox * py;
  // surface term
  const T w0 = px1 * ipt, w1 = py1 * ipt, w2 = pz * ipt, w3 = -st.h * py1, w4 = st.h * px1;
  const T r = k_sqrt(X1[0] * X1[0] + X1[1] * X1[1]);
  const T ir = k_rcp(r);
  const T nx = X1[0] * ir, ny = X1[1] * ir;
  const T den = nx * w0 + ny * w1;
  const T mid = -k_rcp(den);
  const T g0 = nx * mid, g1 = ny * mid;
  const T g3 = (nx * j03 + ny * j13) * mid, g4 = (nx * j04 + ny * j14) * mid;
  // J rows as (c0, c1, c3, c4) for rows 0, 1, 3, 4; row 2 has all six columns
  const T J0[4] = {T(1) + w0 * g0, w0 * g1, j03 + w0 * g3, j04 + w0 * g4};
  const T J1[4] = {w1 * g0, T(1) + w1 * g1, j13 + w1 * g3, j14 + w1 * g4};
  const T J3[4] = {w3 * g0, w3 * g1, j33 + w3 * g3, j34 + w3 * g4};
  const T J4[4] = {w4 * g0, w4 * g1, j43 + w4 * g3, j44 + w4 * g4};
  const T J2[6] = {w2 * g0, w2 * g1, T(1), j23 + w2 * g3, j24 + w2 * g4, j25};
  // full copy of P (symmetric)
  T F[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) F[i][j] = P[ut(i, j)];
  // Tm = J P (rows 0..5)
  constexpr int c4[4] = {0, 1, 3, 4};
  T Tm[6][6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T a0 = 0, a1 = 0, a3 = 0, a4 = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      a0 += J0[m] * F[c4[m]][k];
      a1 += J1[m] * F[c4[m]][k];
      a3 += J3[m] * F[c4[m]][k];
      a4 += J4[m] * F[c4[m]][k];
    }
    Tm[0][k] = a0; Tm[1][k] = a1; Tm[3][k] = a3; Tm[4][k] = a4;
    T a2 = 0;
#pragma unroll
    for (int m = 0; m < 6; ++m) a2 += J2[m] * F[m][k];
    Tm[2][k] = a2;
    Tm[5][k] = F[5][k];
  }
  // P' = Tm J^T, upper triangle
  const T* Jr[6] = {J0, J1, J2, J3, J4, nullptr};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = i; j < 6; ++j) {
      T acc = 0;
      if (j == 2) {
#pragma unroll
        for (int m = 0; m < 6; ++m) acc += Tm[i][m] * J2[m];
      } else if (j == 5) {
        acc = Tm[i][5];
      } else {
        const T* Jj = j == 0 ? J0 : j == 1 ? J1 : j == 3 ? J3 : J4;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc += Tm[i][c4[m]] * Jj[m];
      }
      P[ut(i, j)] = acc;
    }
  }
  (void)Jr;
  // Highland multiple scattering at the crossing (momentum block)
  if (x_over_x0 > T(0)) {
    const T p2 = X1[3] * X1[3] + X1[4] * X1[4] + X1[5] * X1[5];
    const T p = k_sqrt(p2);
    const T ip = k_rcp(p);
    const T cospsi = fabs((X1[0] * X1[3] + X1[1] * X1[4]) * ir * ip);
    const T xe = x_over_x0 * k_rcp(cospsi);
    const T e2 = p2 + mass * mass;             // energy squared
    const T ibeta2 = e2 * ip * ip;             // 1 / beta^2
    const T th0 = T(0.0136) * k_sqrt(ibeta2) * ip * k_sqrt(xe) * (T(1) + T(0.038) * k_log(xe * ibeta2));
    const T t2 = th0 * th0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) P[ut(3 + i, 3 + j)] += t2 * ((i == j ? p2 : T(0)) - X1[3 + i] * X1[3 + j]);
  }
}

// Predict: propagate + transport.  Returns a status bit or 0.
template <typename T>
KFD inline int predict(const T X[6], const T P[21], int q, T R, T bz, T z_half, T x_over_x0, T mass,
                              T Xo[6], T Po[21]) {
  Step<T> st;
  int rc = propagate(X, q, R, bz, Xo, st);
  if (rc) return rc;
  if (fabs(Xo[2]) > z_half) return KF_OUT_OF_Z;
#pragma unroll
  for (int i = 0; i < 21; ++i) Po[i] = P[i];
  transport(X, Xo, st, Po, x_over_x0, mass);
  return 0;
}

// Measurement frame on the plane tangent to the cylinder at the predicted
// point (section 4.1): u along t = (-y, x)/r, w along z.
template <typename T> struct Innov {
  T r0, r1;          // residual (t.(m - pos), m_z - z)
  T S00, S01, S11;   // innovation covariance
  T det;
  T tx, ty;
};

template <typename T>
KFD inline int innovation(const T X[6], const T P[21], T mx, T my, T mz, const T V[6], Innov<T>& in) {
  const T r = k_sqrt(X[0] * X[0] + X[1] * X[1]);
  const T ir = k_rcp(r);
  const T tx = -X[1] * ir, ty = X[0] * ir;
  in.tx = tx; in.ty = ty;
  in.r0 = tx * (mx - X[0]) + ty * (my - X[1]);
  in.r1 = mz - X[2];
  const T Vuu = tx * tx * V[0] + T(2) * tx * ty * V[1] + ty * ty * V[3];
  const T Vuw = tx * V[2] + ty * V[4];
  const T Vww = V[5];
  in.S00 = tx * tx * P[ut(0, 0)] + T(2) * tx * ty * P[ut(0, 1)] + ty * ty * P[ut(1, 1)] + Vuu;
  in.S01 = tx * P[ut(0, 2)] + ty * P[ut(1, 2)] + Vuw;
  in.S11 = P[ut(2, 2)] + Vww;
  in.det = in.S00 * in.S11 - in.S01 * in.S01;
  if (!(in.S00 > T(0)) || !(in.det > T(0))) return KF_S_NOT_PD;
  return 0;
}

template <typename T> KFD inline T chi2_of(const Innov<T>& in) {
  const T idet = k_rcp(in.det);
  const T i00 = in.S11 * idet, i01 = -in.S01 * idet, i11 = in.S00 * idet;
  return in.r0 * (i00 * in.r0 + i01 * in.r1) + in.r1 * (i01 * in.r0 + i11 * in.r1);
}

// Kalman update: K = P H^T S^-1, X += K r, P -= K (H P) (upper triangle).
template <typename T> KFD inline void apply_update(T X[6], T P[21], const Innov<T>& in) {
  const T idet = k_rcp(in.det);
  const T i00 = in.S11 * idet, i01 = -in.S01 * idet, i11 = in.S00 * idet;
  T U[6], W[6];  // columns of P H^T: U = P t, W = P zhat
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    U[i] = in.tx * P[ut(i, 0)] + in.ty * P[ut(i, 1)];
    W[i] = P[ut(i, 2)];
  }
  T K0[6], K1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    K0[i] = U[i] * i00 + W[i] * i01;
    K1[i] = U[i] * i01 + W[i] * i11;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) X[i] += K0[i] * in.r0 + K1[i] * in.r1;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) P[ut(i, j)] -= K0[i] * U[j] + K1[i] * W[j];
}

template <typename T> KFD inline bool all_finite(const T* a, int n) {
  bool ok = true;
  for (int i = 0; i < n; ++i) ok = ok && k_finite(a[i]);
  return ok;
}

// Hybrid state (section 3: Cartesian position, polar momentum):
// Y = (x, y, z, k, phi, theta), k = q / pT signed.  The prediction of Y is
// the Cartesian prediction at the same point with the covariance carried
// through the changes of variables; they leave the position alone, so only
// the momentum blocks of their Jacobians are kept (3 x 3, row-major).
//
// Y -> Cartesian state; A = d(px, py, pz) / d(k, phi, theta); returns q.
template <typename T> KFD inline int cart_from_hyb(const T Y[6], T X[6], T A[9]) {
  const T k = Y[3];
  const T ak = k < T(0) ? -k : k;
  const T pt = k_rcp(ak);
  const T sg = k < T(0) ? T(-1) : T(1);
  T sf, cf, st, ct;
  k_sincos(Y[4], &sf, &cf);
  k_sincos(Y[5], &st, &ct);
  const T ist = k_rcp(st);
  const T cot = ct * ist;
  X[0] = Y[0];
  X[1] = Y[1];
  X[2] = Y[2];
  X[3] = pt * cf;
  X[4] = pt * sf;
  X[5] = pt * cot;
  const T dpt = -sg * pt * pt;  // d pT / d k
  A[0] = dpt * cf; A[1] = -pt * sf; A[2] = T(0);
  A[3] = dpt * sf; A[4] = pt * cf;  A[5] = T(0);
  A[6] = dpt * cot; A[7] = T(0);    A[8] = -pt * ist * ist;
  return k < T(0) ? -1 : 1;
}

// Cartesian state (charge q) -> Y; B = d(k, phi, theta) / d(px, py, pz).
template <typename T> KFD inline void hyb_from_cart(const T X[6], int q, T Y[6], T B[9]) {
  const T px = X[3], py = X[4], pz = X[5];
  const T pt2 = px * px + py * py;
  const T pt = k_sqrt(pt2);
  const T ipt = k_rcp(pt), ipt2 = ipt * ipt;
  const T ip2 = k_rcp(pt2 + pz * pz);
  const T k = (q < 0 ? T(-1) : T(1)) * ipt;
  Y[0] = X[0];
  Y[1] = X[1];
  Y[2] = X[2];
  Y[3] = k;
  Y[4] = k_atan2(py, px);
  Y[5] = k_atan2(pt, pz);
  B[0] = -k * px * ipt2;       B[1] = -k * py * ipt2;       B[2] = T(0);
  B[3] = -py * ipt2;           B[4] = px * ipt2;            B[5] = T(0);
  B[6] = px * pz * ipt * ip2;  B[7] = py * pz * ipt * ip2;  B[8] = -pt * ip2;
}

// P <- M P M^T with M = diag(I3, Mp) on the 21-entry upper triangle: the
// position block stays, position-momentum becomes Ppm Mp^T, momentum Mp Pmm Mp^T.
template <typename T> KFD inline void congruence_mom(T P[21], const T M[9]) {
  T pm[3][3], mm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) pm[i][b] = P[ut(i, 3 + b)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) mm[a][b] = P[ut(3 + a, 3 + b)];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) P[ut(i, 3 + a)] = pm[i][0] * M[a * 3] + pm[i][1] * M[a * 3 + 1] + pm[i][2] * M[a * 3 + 2];
  // T1 = Mp Pmm, then T1 Mp^T (upper triangle)
  T t1[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) t1[a][b] = M[a * 3] * mm[0][b] + M[a * 3 + 1] * mm[1][b] + M[a * 3 + 2] * mm[2][b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = a; c < 3; ++c)
      P[ut(3 + a, 3 + c)] = t1[a][0] * M[c * 3] + t1[a][1] * M[c * 3 + 1] + t1[a][2] * M[c * 3 + 2];
}

// Prediction of a hybrid state: to Cartesian, predict, back.
template <typename T>
KFD inline int predict_hyb(const T Y[6], const T P[21], T R, T bz, T z_half, T x_over_x0, T mass, T Yo[6],
                           T Po[21]) {
  if (!(Y[3] != T(0))) return KF_NONFINITE;
  T X[6], A[9], Pc[21], Xo[6], B[9];
#pragma unroll
  for (int k = 0; k < 21; ++k) Pc[k] = P[k];
  const int q = cart_from_hyb(Y, X, A);
  congruence_mom(Pc, A);
  const int rc = predict<T>(X, Pc, q, R, bz, z_half, x_over_x0, mass, Xo, Po);
  if (rc) return rc;
  hyb_from_cart(Xo, q, Yo, B);
  congruence_mom(Po, B);
  return 0;
}

}  // namespace kfdev
