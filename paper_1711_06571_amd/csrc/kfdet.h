// Device arithmetic of the general detector (section 4.1): barrel cylinders
// closed by endcap disks (planes z = const), with modules that may sit off a
// layer's average surface.  One candidate per lane, state X[6], covariance
// P[21] (upper triangle, row order), as in kfdev.h.
//
// A step moves a state to a surface along the helix:
//   - cylinder r = R: the first crossing along the motion (as the barrel
//     propagation), or the nearest crossing either way (the second step from
//     a layer's average radius to the radius of one of its hits);
//   - plane z = Z: transverse path s = (Z - z) pT / pz, ahead only or either
//     way.
// The covariance follows with the surface Jacobian J = Js + w g^T (Js at a
// fixed path, w = dX/ds, g = ds/dX0 keeps the end point on the surface), and
// a thin layer's Highland noise is added with the incidence measured from the
// surface normal (radial for a cylinder, z for a plane).
#pragma once
#include "kfdev.h"

namespace kfdev {

constexpr int KIND_BARREL = 0;
constexpr int KIND_DISK = 1;

// The helix after a transverse path s (any sign): Step and end state.
// sin(alpha) and 1 - cos(alpha) = 2 sin^2(alpha / 2) come from the half angle,
// so both stay accurate for small turns.
template <typename T>
KFD inline int helix_step(const T X[6], int q, T bz, T s, T Xo[6], Step<T>& st) {
  const T px = X[3], py = X[4], pz = X[5];
  const T pt = k_sqrt(px * px + py * py);
  if (!(pt > T(0))) return KF_NO_CROSSING;
  const T ipt = k_rcp(pt);
  const T h = -T(q) * kappa<T>() * bz * ipt;
  const T alpha = h * s;
  T sh, ch;
  k_sincos(T(0.5) * alpha, &sh, &ch);
  const T sa = T(2) * sh * ch, omc = T(2) * sh * sh;
  const T ih = k_rcp(h);
  const T Ah = sa * ih, Bh = omc * ih;
  const T tx = px * ipt, ty = py * ipt;
  Xo[0] = X[0] + tx * Ah - ty * Bh;
  Xo[1] = X[1] + ty * Ah + tx * Bh;
  Xo[2] = X[2] + pz * s * ipt;
  Xo[3] = px * (T(1) - omc) - py * sa;
  Xo[4] = py * (T(1) - omc) + px * sa;
  Xo[5] = pz;
  st.s = s; st.alpha = alpha; st.sa = sa; st.ca = T(1) - omc; st.A = Ah; st.B = Bh; st.h = h; st.pt = pt;
  st.ipt = ipt;
  return 0;
}

// Step to the plane z = Z (ahead only unless NEAREST).  A track parallel to
// the plane has no crossing.
template <typename T, bool NEAREST>
KFD inline int plane_step(const T X[6], int q, T Z, T bz, T Xo[6], Step<T>& st) {
  const T pt = k_sqrt(X[3] * X[3] + X[4] * X[4]);
  if (!(pt > T(0)) || !(X[5] != T(0))) return KF_NO_CROSSING;
  const T s = (Z - X[2]) * pt / X[5];
  if (!k_finite(s)) return KF_NO_CROSSING;
  if (!NEAREST && !(s > T(0))) return KF_NO_CROSSING;
  return helix_step<T>(X, q, bz, s, Xo, st);
}

// Step to a surface of either kind: value = radius (barrel) or z (disk).
template <typename T, bool NEAREST>
KFD inline int surf_step(int kind, const T X[6], int q, T value, T bz, T Xo[6], Step<T>& st) {
  return kind == KIND_DISK ? plane_step<T, NEAREST>(X, q, value, bz, Xo, st)
                           : propagate<T, NEAREST>(X, q, value, bz, Xo, st);
}

// Which entries of the surface Jacobian can be non-zero (compile-time after
// unrolling): a cylinder leaves the position-z and pz columns of the
// transverse rows empty; a plane empties the z row.
KFD constexpr bool jac_nz(bool disk, int i, int j) {
  if (i == 5) return j == 5;
  if (disk) {
    if (i == 2) return false;
    if (j == 0) return i == 0;
    if (j == 1) return i == 1;
    return true;
  }
  if (i == 2) return true;
  return j == 0 || j == 1 || j == 3 || j == 4;
}

// Full surface Jacobian of "state -> state on the surface" after step st from
// X0 to X1 (entries outside jac_nz are left unset).
template <typename T, bool DISK>
KFD inline void surf_jacobian(const T X0[6], const T X1[6], const Step<T>& st, T J[6][6]) {
  const T px = X0[3], py = X0[4], pz = X0[5];
  const T ipt = st.ipt, ipt2 = ipt * ipt, ipt3 = ipt2 * ipt;
  const T s = st.s;
  const T px1 = X1[3], py1 = X1[4];
  const T aox = st.alpha * ipt2;
  const T sp3 = s * ipt3;
  // Js at fixed path: position rows pick up the momentum through the arc and
  // through alpha ~ 1 / pT; the momentum rotates by alpha
  const T j03 = st.A * ipt - px1 * px * sp3, j04 = -st.B * ipt - px1 * py * sp3;
  const T j13 = st.B * ipt - py1 * px * sp3, j14 = st.A * ipt - py1 * py * sp3;
  const T j23 = -pz * px * sp3, j24 = -pz * py * sp3, j25 = s * ipt;
  const T j33 = st.ca + py1 * aox * px, j34 = -st.sa + py1 * aox * py;
  const T j43 = st.sa - px1 * aox * px, j44 = st.ca - px1 * aox * py;
  const T w[5] = {px1 * ipt, py1 * ipt, pz * ipt, -st.h * py1, st.h * px1};
  T g[6];
  if constexpr (DISK) {
    // n = zhat: g = -(z row of Js) / w_z
    const T mid = -k_rcp(w[2]);
    g[0] = T(0); g[1] = T(0); g[2] = mid; g[3] = j23 * mid; g[4] = j24 * mid; g[5] = j25 * mid;
  } else {
    // n = radial unit vector at the end point
    const T ir = k_rcp(k_sqrt(X1[0] * X1[0] + X1[1] * X1[1]));
    const T nx = X1[0] * ir, ny = X1[1] * ir;
    const T mid = -k_rcp(nx * w[0] + ny * w[1]);
    g[0] = nx * mid; g[1] = ny * mid; g[2] = T(0);
    g[3] = (nx * j03 + ny * j13) * mid; g[4] = (nx * j04 + ny * j14) * mid; g[5] = T(0);
  }
  const T Js[5][6] = {{T(1), T(0), T(0), j03, j04, T(0)},
                      {T(0), T(1), T(0), j13, j14, T(0)},
                      {T(0), T(0), T(1), j23, j24, j25},
                      {T(0), T(0), T(0), j33, j34, T(0)},
                      {T(0), T(0), T(0), j43, j44, T(0)}};
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (jac_nz(DISK, i, j)) J[i][j] = Js[i][j] + w[i] * g[j];
  J[5][5] = T(1);
}

// P <- J P J^T on the upper triangle, skipping the known zeros of J.
template <typename T, bool DISK> KFD inline void sandwich(const T J[6][6], T P[21]) {
  T F[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) F[i][j] = P[ut(i, j)];
  T Tm[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      T a = T(0);
#pragma unroll
      for (int m = 0; m < 6; ++m)
        if (jac_nz(DISK, i, m)) a += J[i][m] * F[m][k];
      Tm[i][k] = a;
    }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      T a = T(0);
#pragma unroll
      for (int m = 0; m < 6; ++m)
        if (jac_nz(DISK, j, m)) a += Tm[i][m] * J[j][m];
      P[ut(i, j)] = a;
    }
}

// Highland noise of a thin layer (x_over_x0 at normal incidence) crossed at
// X, incidence from the surface normal; added to the momentum block.
template <typename T> KFD inline void highland_add(int kind, const T X[6], T P[21], T x_over_x0, T mass) {
  if (!(x_over_x0 > T(0))) return;
  const T p2 = X[3] * X[3] + X[4] * X[4] + X[5] * X[5];
  const T p = k_sqrt(p2);
  const T ip = k_rcp(p);
  T cospsi;
  if (kind == KIND_DISK) {
    cospsi = fabs(X[5] * ip);
  } else {
    const T ir = k_rcp(k_sqrt(X[0] * X[0] + X[1] * X[1]));
    cospsi = fabs((X[0] * X[3] + X[1] * X[4]) * ir * ip);
  }
  const T xe = x_over_x0 * k_rcp(cospsi);
  const T ibeta2 = (p2 + mass * mass) * ip * ip;
  const T th0 = T(0.0136) * k_sqrt(ibeta2) * ip * k_sqrt(xe) * (T(1) + T(0.038) * k_log(xe * ibeta2));
  const T t2 = th0 * th0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) P[ut(3 + i, 3 + j)] += t2 * ((i == j ? p2 : T(0)) - X[3 + i] * X[3 + j]);
}

// One step to a surface with the covariance transported (and the layer's
// scattering added at the end point when `material`).
template <typename T, bool NEAREST>
KFD inline int surf_predict(int kind, const T X[6], const T P[21], int q, T value, T bz, bool material,
                            T x_over_x0, T mass, T Xo[6], T Po[21]) {
  Step<T> st;
  const int rc = surf_step<T, NEAREST>(kind, X, q, value, bz, Xo, st);
  if (rc) return rc;
#pragma unroll
  for (int k = 0; k < 21; ++k) Po[k] = P[k];
  T J[6][6];
  if (kind == KIND_DISK) {
    surf_jacobian<T, true>(X, Xo, st, J);
    sandwich<T, true>(J, Po);
  } else {
    surf_jacobian<T, false>(X, Xo, st, J);
    sandwich<T, false>(J, Po);
  }
  if (material) highland_add<T>(kind, Xo, Po, x_over_x0, mass);
  return 0;
}

// Disk measurement: (x, y) in the disk's plane, V2 the (x, y) block of the
// hit covariance (V = xx, xy, xz, yy, yz, zz).
template <typename T>
KFD inline int innovation_disk(const T X[6], const T P[21], T mx, T my, const T V[6], Innov<T>& in) {
  in.tx = T(1);
  in.ty = T(0);
  in.r0 = mx - X[0];
  in.r1 = my - X[1];
  in.S00 = P[ut(0, 0)] + V[0];
  in.S01 = P[ut(0, 1)] + V[1];
  in.S11 = P[ut(1, 1)] + V[3];
  in.det = in.S00 * in.S11 - in.S01 * in.S01;
  if (!(in.S00 > T(0)) || !(in.det > T(0))) return KF_S_NOT_PD;
  return 0;
}

// K = P H^T S^-1 with H picking (x, y); X += K r, P -= K (H P).
template <typename T> KFD inline void apply_update_disk(T X[6], T P[21], const Innov<T>& in) {
  const T idet = k_rcp(in.det);
  const T i00 = in.S11 * idet, i01 = -in.S01 * idet, i11 = in.S00 * idet;
  T U[6], W[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    U[i] = P[ut(i, 0)];
    W[i] = P[ut(i, 1)];
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

// Update with a hit of a layer of the given kind (barrel: the plane tangent
// to the cylinder at the predicted point; disk: the disk's plane); returns a
// status bit or 0 and the hit's chi2.
template <typename T>
KFD inline int update_kind(int kind, T X[6], T P[21], T mx, T my, T mz, const T V[6], T& chi2) {
  Innov<T> in;
  const int rc = kind == KIND_DISK ? innovation_disk<T>(X, P, mx, my, V, in) : innovation<T>(X, P, mx, my, mz, V, in);
  if (rc) return rc;
  chi2 = chi2_of(in);
  if (kind == KIND_DISK) apply_update_disk<T>(X, P, in);
  else apply_update<T>(X, P, in);
  return 0;
}

}  // namespace kfdev
