/*
 * kforacle — plain FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY: the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may call it;
 * the product path never does.  See kforacle.h for the conventions.
 *
 * Everything here is written for clarity, not speed: full 6x6 matrices,
 * plain loops, brute-force hit scans.
 */
#include "kforacle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KAPPA 0.299792458e-2 /* GeV / (T cm) */
#define TWO_PI 6.283185307179586476925286766559
#define PI 3.1415926535897932384626433832795

/* ------------------------------------------------------------ helpers */

static void matmul(const double* A, const double* B, double* C, int n, int m, int p) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[i * m + k] * B[k * p + j];
      C[i * p + j] = s;
    }
}

static void transpose(const double* A, double* T, int n, int m) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) T[j * n + i] = A[i * m + j];
}

static void sym_from_upper(const double* u, double* P) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) { P[i * 6 + j] = u[k]; P[j * 6 + i] = u[k]; ++k; }
}

static void upper_from_sym(const double* P, double* u) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) u[k++] = P[i * 6 + j];
}

static int all_finite(const double* a, int n) {
  for (int i = 0; i < n; ++i) if (!isfinite(a[i])) return 0;
  return 1;
}

/* ----------------------------------------------- helix (section 3) */

/*
 * Motion of a unit charge q in B = bz * zhat (section 3: uniform
 * longitudinal field).  With pT = |(px,py)| and the signed curvature
 * h = -q*KAPPA*bz/pT, after a transverse path s the momentum has turned by
 * alpha = h*s and
 *   x(s) = x + [px sin(a) - py (1-cos(a))] / (pT h)
 *   y(s) = y + [py sin(a) + px (1-cos(a))] / (pT h)
 *   z(s) = z + pz s / pT.
 */
void orc_state_at(const double X[6], int q, double bz, double s, double Xo[6]) {
  double px = X[3], py = X[4], pz = X[5];
  double pt = sqrt(px * px + py * py);
  double h = -(double)q * KAPPA * bz / pt;
  double a = h * s, ca = cos(a), sa = sin(a);
  double c = pt * h;
  Xo[0] = X[0] + (px * sa - py * (1.0 - ca)) / c;
  Xo[1] = X[1] + (py * sa + px * (1.0 - ca)) / c;
  Xo[2] = X[2] + pz * s / pt;
  Xo[3] = px * ca - py * sa;
  Xo[4] = py * ca + px * sa;
  Xo[5] = pz;
}

/*
 * Propagation to the cylinder of radius R: the first crossing along the
 * motion, found by intersecting the transverse circle (centre C, radius
 * rho = 1/|h|) with the circle r = R.  Returns ORC_TRK_NO_CROSSING if the
 * circles do not meet.  *disc receives (R^2 - a^2)/R^2, the normalised
 * half-chord squared, which tends to 0 at tangency.
 */
int orc_propagate(const double X[6], int q, double R, double bz, double Xo[6], double* s_out, double* disc) {
  double px = X[3], py = X[4];
  double pt = sqrt(px * px + py * py);
  if (disc) *disc = INFINITY;
  if (!(pt > 0.0) || bz == 0.0) return ORC_TRK_NO_CROSSING;
  double h = -(double)q * KAPPA * bz / pt;
  double cx = X[0] - py / (pt * h), cy = X[1] + px / (pt * h);
  double rho = 1.0 / fabs(h);
  double d = sqrt(cx * cx + cy * cy);
  if (!(d > 0.0) || d > R + rho || d < fabs(R - rho)) return ORC_TRK_NO_CROSSING;
  double a = (R * R - rho * rho + d * d) / (2.0 * d);
  double b2 = R * R - a * a;
  if (b2 < 0.0) b2 = 0.0;
  if (disc) *disc = b2 / (R * R);
  double b = sqrt(b2);
  double best = INFINITY;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    double Px = (a / d) * cx + sgn * (b / d) * (-cy);
    double Py = (a / d) * cy + sgn * (b / d) * cx;
    double ux = X[0] - cx, uy = X[1] - cy; /* start, seen from the centre */
    double vx = Px - cx, vy = Py - cy;     /* crossing, seen from the centre */
    double alpha = atan2(ux * vy - uy * vx, ux * vx + uy * vy);
    if (h > 0.0 && alpha <= 0.0) alpha += TWO_PI;
    if (h < 0.0 && alpha >= 0.0) alpha -= TWO_PI;
    double s = alpha / h;
    if (s < best) best = s;
  }
  orc_state_at(X, q, bz, best, Xo);
  if (s_out) *s_out = best;
  return 0;
}

/* Js = dX(s)/dX0 at fixed transverse path s, and w = dX/ds at the end point
 * (the end state is returned in Xo). */
static void jacobian_fixed_path(const double X[6], int q, double bz, double s, double Js[36], double w[6],
                                double Xo[6]) {
  double px = X[3], py = X[4], pz = X[5];
  double pt2 = px * px + py * py, pt = sqrt(pt2);
  double h = -(double)q * KAPPA * bz / pt;
  double a = h * s, ca = cos(a), sa = sin(a);
  double c = pt * h; /* = -q KAPPA bz, independent of pT */
  orc_state_at(X, q, bz, s, Xo);
  double px1 = Xo[3], py1 = Xo[4];
  double da_dpx = -a * px / pt2, da_dpy = -a * py / pt2;
  memset(Js, 0, sizeof(double) * 36);
  Js[0 * 6 + 0] = 1.0; Js[1 * 6 + 1] = 1.0; Js[2 * 6 + 2] = 1.0;
  Js[0 * 6 + 3] = (sa + px1 * da_dpx) / c;
  Js[0 * 6 + 4] = (-(1.0 - ca) + px1 * da_dpy) / c;
  Js[1 * 6 + 3] = ((1.0 - ca) + py1 * da_dpx) / c;
  Js[1 * 6 + 4] = (sa + py1 * da_dpy) / c;
  Js[2 * 6 + 3] = -pz * s * px / (pt2 * pt);
  Js[2 * 6 + 4] = -pz * s * py / (pt2 * pt);
  Js[2 * 6 + 5] = s / pt;
  Js[3 * 6 + 3] = ca - py1 * da_dpx;
  Js[3 * 6 + 4] = -sa - py1 * da_dpy;
  Js[4 * 6 + 3] = sa + px1 * da_dpx;
  Js[4 * 6 + 4] = ca + px1 * da_dpy;
  Js[5 * 6 + 5] = 1.0;
  w[0] = px1 / pt; w[1] = py1 / pt; w[2] = pz / pt; w[3] = -h * py1; w[4] = h * px1; w[5] = 0.0;
}

/*
 * Jacobian of "state -> state at the crossing with the cylinder".
 * J = Js + w g^T, where Js = dX(s)/dX0 at fixed path s, w = dX/ds at the
 * crossing, and g = ds/dX0 = -(n . Js[x,y rows]) / (n . w[x,y]) keeps the
 * end point on the cylinder (n = radial unit vector at the crossing).
 */
void orc_jacobian(const double X[6], int q, double bz, double s, double J[36]) {
  double Js[36], w[6], Xo[6];
  jacobian_fixed_path(X, q, bz, s, Js, w, Xo);
  double r = sqrt(Xo[0] * Xo[0] + Xo[1] * Xo[1]);
  double nx = Xo[0] / r, ny = Xo[1] / r;
  double den = nx * w[0] + ny * w[1];
  double g[6];
  for (int j = 0; j < 6; ++j) g[j] = -(nx * Js[0 * 6 + j] + ny * Js[1 * 6 + j]) / den;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) J[i * 6 + j] = Js[i * 6 + j] + w[i] * g[j];
}

/*
 * Multiple-scattering process noise (section 2: the Kalman filter carries
 * multiple-scattering estimates in the trajectory).  PDG Highland width for
 * unit charge, thin scatterer with effective thickness x/X0 / cos(psi)
 * (psi: angle between the track and the layer normal), beta from the given
 * mass.  Two independent projected angles of variance theta0^2 give the
 * momentum covariance theta0^2 (|p|^2 I - p p^T); the position block is 0.
 */
void orc_ms_cov(const double X[6], double x_over_x0, double mass, double Q[36]) {
  memset(Q, 0, sizeof(double) * 36);
  if (!(x_over_x0 > 0.0)) return;
  double p2 = X[3] * X[3] + X[4] * X[4] + X[5] * X[5];
  double p = sqrt(p2);
  double r = sqrt(X[0] * X[0] + X[1] * X[1]);
  double cospsi = fabs((X[0] * X[3] + X[1] * X[4]) / (r * p));
  double xe = x_over_x0 / cospsi;
  double beta = p / sqrt(p2 + mass * mass);
  double th0 = 0.0136 / (beta * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / (beta * beta)));
  double t2 = th0 * th0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Q[(3 + i) * 6 + 3 + j] = t2 * ((i == j ? p2 : 0.0) - X[3 + i] * X[3 + j]);
}

/*
 * Predict step: propagate to layer `layer`, transport the covariance with
 * the Jacobian and add the scattering noise of that layer evaluated on the
 * predicted state.  Returns ORC_TRK_NO_CROSSING or ORC_TRK_OUT_OF_Z on
 * failure (outputs then unspecified).
 */
int orc_predict(const orc_geometry* g, int layer, const double X[6], int q, const double P[36], double Xo[6],
                double Po[36], double* disc) {
  double s;
  int rc = orc_propagate(X, q, (double)g->r[layer], (double)g->bz, Xo, &s, disc);
  if (rc) return rc;
  if (fabs(Xo[2]) > (double)g->z_half) return ORC_TRK_OUT_OF_Z;
  double J[36], JT[36], T[36], Q[36];
  orc_jacobian(X, q, (double)g->bz, s, J);
  transpose(J, JT, 6, 6);
  matmul(J, P, T, 6, 6, 6);
  matmul(T, JT, Po, 6, 6, 6);
  orc_ms_cov(Xo, (double)g->x_over_x0, (double)g->mass, Q);
  for (int i = 0; i < 36; ++i) Po[i] += Q[i];
  return 0;
}

/*
 * Kalman update on the plane tangent to the cylinder at the predicted
 * point (section 4.1).  The measurement frame is (t, zhat) with
 * t = (-y, x, 0)/r; H picks (t . pos, z).  Residual r = (t.(m - pos),
 * m_z - z); the hit's 3x3 covariance V is projected to V2 = F V F^T with
 * F = [t; zhat].  S = H P H^T + V2, K = P H^T S^-1, X' = X + K r,
 * P' = P - K H P, chi2 = r^T S^-1 r (2 degrees of freedom).
 * hit = (x, y, z, Vxx, Vxy, Vxz, Vyy, Vyz, Vzz).  Returns ORC_TRK_S_NOT_PD
 * if S is not positive definite.
 */
int orc_update(const double X[6], const double P[36], const double hit[9], double Xo[6], double Po[36],
               double* chi2) {
  double r = sqrt(X[0] * X[0] + X[1] * X[1]);
  double tx = -X[1] / r, ty = X[0] / r;
  double H[12] = {tx, ty, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0};
  double V[9] = {hit[3], hit[4], hit[5], hit[4], hit[6], hit[7], hit[5], hit[7], hit[8]};
  double F[9] = {tx, ty, 0, 0, 0, 1, 0, 0, 0}; /* rows t, zhat (third row unused) */
  double FV[6], V2[4];
  matmul(F, V, FV, 2, 3, 3);
  double FT[6] = {F[0], F[3], F[1], F[4], F[2], F[5]};
  matmul(FV, FT, V2, 2, 3, 2);
  double res[2] = {tx * (hit[0] - X[0]) + ty * (hit[1] - X[1]), hit[2] - X[2]};
  double HT[12], PHT[12], S[4];
  transpose(H, HT, 2, 6);
  matmul(P, HT, PHT, 6, 6, 2);
  matmul(H, PHT, S, 2, 6, 2);
  for (int i = 0; i < 4; ++i) S[i] += V2[i];
  double det = S[0] * S[3] - S[1] * S[2];
  if (!(S[0] > 0.0) || !(det > 0.0)) return ORC_TRK_S_NOT_PD;
  double Si[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
  double K[12], HP[12], KHP[36];
  matmul(PHT, Si, K, 6, 2, 2);
  for (int i = 0; i < 6; ++i) Xo[i] = X[i] + K[i * 2 + 0] * res[0] + K[i * 2 + 1] * res[1];
  matmul(H, P, HP, 2, 6, 6);
  matmul(K, HP, KHP, 6, 2, 6);
  for (int i = 0; i < 36; ++i) Po[i] = P[i] - KHP[i];
  double Sir[2] = {Si[0] * res[0] + Si[1] * res[1], Si[2] * res[0] + Si[3] * res[1]};
  *chi2 = res[0] * Sir[0] + res[1] * Sir[1];
  return 0;
}

static void load_hit(const float* hits, int ld, int layer, int i, double h[9]) {
  for (int c = 0; c < 9; ++c) h[c] = (double)hits[((size_t)layer * 9 + c) * (size_t)ld + (size_t)i];
}

/* ------------------------------------------------------------- seed */

/*
 * Transverse impact parameter of the helix of state X (charge q, field bz),
 * as the signed distance of the z axis from the circle: f = |c| - rho, with
 * the circle centre c = (x + py/k, y - px/k), k = q*KAPPA*bz (the helix
 * above turns about that point) and rho = pT/|k|.  H = df/dX (z and pz do
 * not enter).  Returns nonzero when the centre sits on the axis.
 */
int orc_beam_d0(const double X[6], int q, double bz, double* f, double H[6]) {
  double k = (double)q * KAPPA * bz;
  double cx = X[0] + X[4] / k, cy = X[1] - X[3] / k;
  double cn = sqrt(cx * cx + cy * cy);
  double pt = sqrt(X[3] * X[3] + X[4] * X[4]);
  if (!(cn > 0.0) || !(pt > 0.0)) return 1;
  double ak = fabs(k);
  *f = cn - pt / ak;
  H[0] = cx / cn;
  H[1] = cy / cn;
  H[2] = 0.0;
  H[3] = -cy / (k * cn) - X[3] / (pt * ak);
  H[4] = cx / (k * cn) - X[4] / (pt * ak);
  H[5] = 0.0;
  return 0;
}

/*
 * Seed from the hits on layers 0, 1, 2.  Seeding itself is outside the
 * paper's scope (section 2: seeds are given); this is the test convention
 * that turns three hits into a starting state and covariance.
 *
 * With a beam spot (beam_sigma > 0: the track comes from the z axis within
 * beam_sigma cm transversely):
 *   1. the circle through the axis point (0, 0) and the transverse points of
 *      hits 0 and 2 gives the centre and rho, hence pT = KAPPA*|bz|*rho; its
 *      turning sense with the sign of bz gives q;
 *   2. the momentum at hit 0 is tangent to that circle, along the motion;
 *      tan(lambda) from the z change over the arc from hit 0 to hit 2;
 *   3. starting at hit 0 with a broad prior (1 cm tangential, 10 cm in z,
 *      |p| per momentum component), one Kalman update with the measurement
 *      "impact parameter = 0" of variance beam_sigma^2 (orc_beam_d0);
 *   4. add the layer-0 scattering and run the Kalman filter over hits 0, 1,
 *      2; the state and covariance at layer 2 are the seed.
 * Without a beam spot (beam_sigma <= 0) step 1 uses the circle through the
 * three hits and step 3 is skipped.
 */
static int seed_one(const orc_geometry* g, const double h[3][9], double beam_sigma, int* q_out, double X[6],
                    double P[36]) {
  const int beam = beam_sigma > 0.0;
  /* the three circle points: (0,0), hit 0, hit 2 or hit 0, hit 1, hit 2 */
  double p0x = beam ? 0.0 : h[0][0], p0y = beam ? 0.0 : h[0][1];
  double p1x = beam ? h[0][0] : h[1][0], p1y = beam ? h[0][1] : h[1][1];
  double p2x = h[2][0], p2y = h[2][1];
  /* centre from |c - p0| = |c - p1| = |c - p2| */
  double ax = p1x - p0x, ay = p1y - p0y, bx = p2x - p0x, by = p2y - p0y;
  double D = 2.0 * (ax * by - ay * bx);
  if (!(fabs(D) > 0.0)) return ORC_TRK_NO_CROSSING;
  double a2 = ax * ax + ay * ay, b2 = bx * bx + by * by;
  double cx = p0x + (by * a2 - ay * b2) / D, cy = p0y + (ax * b2 - bx * a2) / D;
  /* hit 0 and hit 2 seen from the centre */
  double r1x = h[0][0] - cx, r1y = h[0][1] - cy;
  double r3x = h[2][0] - cx, r3y = h[2][1] - cy;
  double rho = sqrt(r1x * r1x + r1y * r1y);
  /* turning sense of p0 -> p1 -> p2: counter-clockwise if cross > 0 */
  double cross = (p1x - p0x) * (p2y - p1y) - (p1y - p0y) * (p2x - p1x);
  double bz = (double)g->bz;
  /* the helix turns clockwise (seen from +z) when q*bz > 0 */
  int q = (cross < 0.0) == (bz > 0.0) ? 1 : -1;
  double pt = KAPPA * fabs(bz) * rho;
  double tx, ty;
  if (cross > 0.0) { tx = -r1y / rho; ty = r1x / rho; }
  else { tx = r1y / rho; ty = -r1x / rho; }
  double dalpha = fabs(atan2(r1x * r3y - r1y * r3x, r1x * r3x + r1y * r3y));
  double tanl = (h[2][2] - h[0][2]) / (rho * dalpha);
  double X0[6] = {h[0][0], h[0][1], h[0][2], pt * tx, pt * ty, pt * tanl};
  double p2 = X0[3] * X0[3] + X0[4] * X0[4] + X0[5] * X0[5];
  double r0 = sqrt(X0[0] * X0[0] + X0[1] * X0[1]);
  double ttx = -X0[1] / r0, tty = X0[0] / r0;
  double P0[36];
  memset(P0, 0, sizeof(P0));
  P0[0 * 6 + 0] = ttx * ttx; P0[0 * 6 + 1] = ttx * tty;
  P0[1 * 6 + 0] = ttx * tty; P0[1 * 6 + 1] = tty * tty;
  P0[2 * 6 + 2] = 100.0;
  P0[3 * 6 + 3] = p2; P0[4 * 6 + 4] = p2; P0[5 * 6 + 5] = p2;
  if (beam) {
    double f, H[6], PH[6];
    if (orc_beam_d0(X0, q, bz, &f, H)) return ORC_TRK_NO_CROSSING;
    matmul(P0, H, PH, 6, 6, 1);
    double S = beam_sigma * beam_sigma;
    for (int i = 0; i < 6; ++i) S += H[i] * PH[i];
    if (!(S > 0.0)) return ORC_TRK_S_NOT_PD;
    for (int i = 0; i < 6; ++i) X0[i] += PH[i] / S * (0.0 - f);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) P0[i * 6 + j] -= PH[i] * PH[j] / S;
  }
  double Q[36];
  orc_ms_cov(X0, (double)g->x_over_x0, (double)g->mass, Q);
  for (int i = 0; i < 36; ++i) P0[i] += Q[i];
  double chi2;
  if (orc_update(X0, P0, h[0], X, P, &chi2)) return ORC_TRK_S_NOT_PD;
  for (int l = 1; l < 3; ++l) {
    double Xp[6], Pp[36];
    int rc = orc_predict(g, l, X, q, P, Xp, Pp, NULL);
    if (rc) return rc;
    if (orc_update(Xp, Pp, h[l], X, P, &chi2)) return ORC_TRK_S_NOT_PD;
  }
  *q_out = q;
  return all_finite(X, 6) && all_finite(P, 36) ? 0 : ORC_TRK_NONFINITE;
}

static int seed_rows(const orc_geometry* g, int n, int ld, const float* hits32, const double* hits64,
                     double beam_sigma, int8_t* q_out, float* seed_par, float* seed_cov, double* seed_par64,
                     double* seed_cov64, int32_t* status) {
  if (n < 0 || ld < n || g->n_layers < 3) return 1;
  for (int i = 0; i < n; ++i) {
    double h[3][9];
    for (int l = 0; l < 3; ++l) {
      if (hits32) load_hit(hits32, ld, l, i, h[l]);
      else for (int c = 0; c < 9; ++c) h[l][c] = hits64[((size_t)l * 9 + c) * (size_t)ld + (size_t)i];
    }
    int q = 1;
    double X[6], P[36], u[21];
    int st = all_finite(&h[0][0], 27) ? seed_one(g, h, beam_sigma, &q, X, P) : ORC_TRK_NONFINITE;
    if (st) { for (int c = 0; c < 6; ++c) X[c] = 0.0; for (int c = 0; c < 36; ++c) P[c] = 0.0; }
    upper_from_sym(P, u);
    q_out[i] = (int8_t)q;
    status[i] = st;
    for (int c = 0; c < 6; ++c) {
      if (seed_par) seed_par[(size_t)c * ld + i] = (float)X[c];
      if (seed_par64) seed_par64[(size_t)c * ld + i] = X[c];
    }
    for (int c = 0; c < 21; ++c) {
      if (seed_cov) seed_cov[(size_t)c * ld + i] = (float)u[c];
      if (seed_cov64) seed_cov64[(size_t)c * ld + i] = u[c];
    }
  }
  return 0;
}

int orc_seed(const orc_geometry* g, int n, int ld, const float* hits, double beam_sigma, int8_t* q_out,
             float* seed_par, float* seed_cov, double* seed_par64, double* seed_cov64, int32_t* status) {
  return seed_rows(g, n, ld, hits, NULL, beam_sigma, q_out, seed_par, seed_cov, seed_par64, seed_cov64, status);
}

int orc_seed64(const orc_geometry* g, int n, int ld, const double* hits, double beam_sigma, int8_t* q_out,
               double* seed_par64, double* seed_cov64, int32_t* status) {
  return seed_rows(g, n, ld, NULL, hits, beam_sigma, q_out, NULL, NULL, seed_par64, seed_cov64, status);
}

/* -------------------------------------------------------------- fit */

/*
 * Track fit (section 2: with the hit list fixed after building, the Kalman
 * filter is applied layer after layer without branching).  From the seed,
 * for each layer l >= first_layer: predict, then update with the track's
 * hit on l (or skip the update where hole_mask has bit l set).  chi2 is the
 * sum of the per-hit chi2, ndof = 2 per hit used.  A failed step sets its
 * status bit and freezes the track at its last good state.
 */
static void fit_one(const orc_geometry* g, int first_layer, const double* hitrows /*[L][9]*/,
                    uint32_t holes, const double Xs[6], const double Ps[36], int q, double Xout[6],
                    double Pout[36], double* chi2_out, int* ndof_out, int* status_out) {
  double X[6], P[36];
  memcpy(X, Xs, sizeof(X));
  memcpy(P, Ps, sizeof(P));
  double chi2 = 0.0;
  int ndof = 0, st = 0;
  if (!all_finite(X, 6) || !all_finite(P, 36)) st = ORC_TRK_NONFINITE;
  for (int l = first_layer; l < g->n_layers && !st; ++l) {
    const double* h = hitrows + (size_t)l * 9;
    int use = !((holes >> l) & 1u);
    if (use && !all_finite(h, 9)) { st = ORC_TRK_NONFINITE; break; }
    double Xp[6], Pp[36];
    int rc = orc_predict(g, l, X, q, P, Xp, Pp, NULL);
    if (rc) { st = rc; break; }
    if (!use) {
      if (!all_finite(Xp, 6) || !all_finite(Pp, 36)) { st = ORC_TRK_NONFINITE; break; }
      memcpy(X, Xp, sizeof(X)); memcpy(P, Pp, sizeof(P));
      continue;
    }
    double Xu[6], Pu[36], c2;
    rc = orc_update(Xp, Pp, h, Xu, Pu, &c2);
    if (rc) { st = rc; break; }
    if (!all_finite(Xu, 6) || !all_finite(Pu, 36) || !isfinite(c2)) { st = ORC_TRK_NONFINITE; break; }
    memcpy(X, Xu, sizeof(X)); memcpy(P, Pu, sizeof(P));
    chi2 += c2;
    ndof += 2;
  }
  memcpy(Xout, X, sizeof(X));
  memcpy(Pout, P, sizeof(P));
  *chi2_out = chi2;
  *ndof_out = ndof;
  *status_out = st;
}

/* ------------------------------------------------- hybrid-state fit */

/*
 * Hybrid state (section 3: global Cartesian coordinates for the position,
 * polar coordinates for the momentum): Y = (x, y, z, k, phi, theta) with
 * k = q / pT (signed, so the charge is a continuous part of the state),
 * phi the azimuth and theta the polar angle of the momentum:
 *   px = cos(phi) / |k|, py = sin(phi) / |k|, pz = cos(theta) / (sin(theta) |k|),
 *   q = sign(k).
 * The helix depends on the state only through k (its curvature is
 * proportional to k), the direction and the position, so a prediction is the
 * Cartesian one taken at the same point: Y -> X (Cartesian), predict,
 * X' -> Y'; its covariance is carried through the Jacobians of the two
 * changes of variables (exact linearisation of the composed map).  The
 * update is the tangent-plane update of section 4.1 applied to Y: it only
 * measures the position, whose components are common to both states, but
 * its linear correction now acts on (k, phi, theta), and k may change sign.
 */
void orc_hyb_from_cart(const double X[6], int q, double Y[6]) {
  double pt = sqrt(X[3] * X[3] + X[4] * X[4]);
  Y[0] = X[0]; Y[1] = X[1]; Y[2] = X[2];
  Y[3] = (double)q / pt;
  Y[4] = atan2(X[4], X[3]);
  Y[5] = atan2(pt, X[5]);
}

int orc_cart_from_hyb(const double Y[6], double X[6]) {
  double pt = 1.0 / fabs(Y[3]);
  X[0] = Y[0]; X[1] = Y[1]; X[2] = Y[2];
  X[3] = pt * cos(Y[4]);
  X[4] = pt * sin(Y[4]);
  X[5] = pt * cos(Y[5]) / sin(Y[5]);
  return Y[3] > 0.0 ? 1 : -1;
}

/* d(X)/d(Y) at Y (6x6, row-major): identity on the position, and the
 * derivatives of (px, py, pz) with respect to (k, phi, theta). */
void orc_hyb_jac_cart_from_hyb(const double Y[6], double A[36]) {
  memset(A, 0, sizeof(double) * 36);
  for (int i = 0; i < 3; ++i) A[i * 6 + i] = 1.0;
  double k = Y[3], pt = 1.0 / fabs(k), s = k > 0.0 ? 1.0 : -1.0;
  double cf = cos(Y[4]), sf = sin(Y[4]), ct = cos(Y[5]), st = sin(Y[5]);
  double dpt = -s * pt * pt; /* d pT / d k */
  A[3 * 6 + 3] = dpt * cf;  A[3 * 6 + 4] = -pt * sf;  A[3 * 6 + 5] = 0.0;
  A[4 * 6 + 3] = dpt * sf;  A[4 * 6 + 4] = pt * cf;   A[4 * 6 + 5] = 0.0;
  A[5 * 6 + 3] = dpt * ct / st; A[5 * 6 + 4] = 0.0;   A[5 * 6 + 5] = -pt / (st * st);
}

/* d(Y)/d(X) at X (charge q): identity on the position, and the derivatives
 * of (k, phi, theta) with respect to (px, py, pz). */
void orc_hyb_jac_hyb_from_cart(const double X[6], int q, double B[36]) {
  memset(B, 0, sizeof(double) * 36);
  for (int i = 0; i < 3; ++i) B[i * 6 + i] = 1.0;
  double px = X[3], py = X[4], pz = X[5];
  double pt2 = px * px + py * py, pt = sqrt(pt2), p2 = pt2 + pz * pz;
  double k = (double)q / pt;
  B[3 * 6 + 3] = -k * px / pt2;       B[3 * 6 + 4] = -k * py / pt2;       B[3 * 6 + 5] = 0.0;
  B[4 * 6 + 3] = -py / pt2;           B[4 * 6 + 4] = px / pt2;            B[4 * 6 + 5] = 0.0;
  B[5 * 6 + 3] = px * pz / (pt * p2); B[5 * 6 + 4] = py * pz / (pt * p2); B[5 * 6 + 5] = -pt / p2;
}

/* M P M^T */
static void congruence(const double M[36], const double P[36], double Po[36]) {
  double MT[36], T[36];
  transpose(M, MT, 6, 6);
  matmul(M, P, T, 6, 6, 6);
  matmul(T, MT, Po, 6, 6, 6);
}

int orc_predict_hyb(const orc_geometry* g, int layer, const double Y[6], const double P[36], double Yo[6],
                    double Po[36], double* disc) {
  double X[6], A[36], Pc[36], Xo[6], Pco[36], B[36];
  if (disc) *disc = NAN;
  if (!(Y[3] != 0.0)) return ORC_TRK_NONFINITE;
  int q = orc_cart_from_hyb(Y, X);
  orc_hyb_jac_cart_from_hyb(Y, A);
  congruence(A, P, Pc);
  int rc = orc_predict(g, layer, X, q, Pc, Xo, Pco, disc);
  if (rc == ORC_TRK_OUT_OF_Z) memcpy(Yo, Xo, sizeof(double) * 3); /* the crossing point, for the caller's margin */
  if (rc) return rc;
  orc_hyb_from_cart(Xo, q, Yo);
  orc_hyb_jac_hyb_from_cart(Xo, q, B);
  congruence(B, Pco, Po);
  return 0;
}

/*
 * Fit in the hybrid state: the Cartesian seed (X, P, q) is converted to Y
 * (covariance through d(Y)/d(X)), then per layer: hybrid prediction, update
 * with the hit (or none on a hole).  Outputs are hybrid: (x, y, z, k, phi,
 * theta) and their covariance (21 upper-triangle entries).
 */
static void fit_one_hyb(const orc_geometry* g, int first_layer, const double* hitrows /*[L][9]*/, uint32_t holes,
                        const double Xs[6], const double Ps[36], int q, double Yout[6], double Pout[36],
                        double* chi2_out, int* ndof_out, int* status_out) {
  double B[36], Y[6], P[36];
  orc_hyb_from_cart(Xs, q, Y);
  orc_hyb_jac_hyb_from_cart(Xs, q, B);
  congruence(B, Ps, P);
  double chi2 = 0.0;
  int ndof = 0, st = 0;
  if (!all_finite(Y, 6) || !all_finite(P, 36)) st = ORC_TRK_NONFINITE;
  for (int l = first_layer; l < g->n_layers && !st; ++l) {
    const double* h = hitrows + (size_t)l * 9;
    int use = !((holes >> l) & 1u);
    if (use && !all_finite(h, 9)) { st = ORC_TRK_NONFINITE; break; }
    double Yp[6], Pp[36];
    int rc = orc_predict_hyb(g, l, Y, P, Yp, Pp, NULL);
    if (rc) { st = rc; break; }
    if (!use) {
      if (!all_finite(Yp, 6) || !all_finite(Pp, 36)) { st = ORC_TRK_NONFINITE; break; }
      memcpy(Y, Yp, sizeof(Y)); memcpy(P, Pp, sizeof(P));
      continue;
    }
    double Yu[6], Pu[36], c2;
    rc = orc_update(Yp, Pp, h, Yu, Pu, &c2);
    if (rc) { st = rc; break; }
    if (!all_finite(Yu, 6) || !all_finite(Pu, 36) || !isfinite(c2)) { st = ORC_TRK_NONFINITE; break; }
    memcpy(Y, Yu, sizeof(Y)); memcpy(P, Pu, sizeof(P));
    chi2 += c2;
    ndof += 2;
  }
  memcpy(Yout, Y, sizeof(Y));
  memcpy(Pout, P, sizeof(P));
  *chi2_out = chi2;
  *ndof_out = ndof;
  *status_out = st;
}

static void store_fit(int ld, int i, const double Y[6], const double P[36], double c2, int ndof, int st,
                      double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  double u[21];
  upper_from_sym(P, u);
  for (int c = 0; c < 6; ++c) out_par[(size_t)c * ld + i] = Y[c];
  for (int c = 0; c < 21; ++c) out_cov[(size_t)c * ld + i] = u[c];
  out_chi2[i] = c2;
  out_ndof[i] = ndof;
  out_status[i] = st;
}

int orc_fit_hybrid(const orc_geometry* g, int n, int ld, int first_layer, const float* hits,
                   const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                   double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || g->n_layers > 32 || first_layer < 0) return 1;
  double rows[9 * 32];
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < g->n_layers; ++l) load_hit(hits, ld, l, i, rows + l * 9);
    double Xs[6], u[21], Ps[36], Y[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = (double)seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = (double)seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one_hyb(g, first_layer, rows, hole_mask ? hole_mask[i] : 0u, Xs, Ps, q[i], Y, P, &c2, &ndof, &st);
    store_fit(ld, i, Y, P, c2, ndof, st, out_par, out_cov, out_chi2, out_ndof, out_status);
  }
  return 0;
}

/* FP64 inputs throughout (used by the exactness pins). */
int orc_fit_hybrid64(const orc_geometry* g, int n, int ld, int first_layer, const double* hits,
                     const double* seed_par, const double* seed_cov, const int8_t* q, double* out_par,
                     double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || g->n_layers > 32 || first_layer < 0) return 1;
  double rows[9 * 32];
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < g->n_layers; ++l)
      for (int c = 0; c < 9; ++c) rows[l * 9 + c] = hits[((size_t)l * 9 + c) * (size_t)ld + (size_t)i];
    double Xs[6], u[21], Ps[36], Y[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one_hyb(g, first_layer, rows, 0u, Xs, Ps, q[i], Y, P, &c2, &ndof, &st);
    store_fit(ld, i, Y, P, c2, ndof, st, out_par, out_cov, out_chi2, out_ndof, out_status);
  }
  return 0;
}

int orc_fit(const orc_geometry* g, int n, int ld, int first_layer, const float* hits, const uint32_t* hole_mask,
            const float* seed_par, const float* seed_cov, const int8_t* q, double* out_par, double* out_cov,
            double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || g->n_layers > 32 || first_layer < 0) return 1;
  double* rows = (double*)malloc(sizeof(double) * 9 * 32);
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < g->n_layers; ++l) load_hit(hits, ld, l, i, rows + l * 9);
    double Xs[6], u[21], Ps[36], X[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = (double)seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = (double)seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one(g, first_layer, rows, hole_mask ? hole_mask[i] : 0u, Xs, Ps, q[i], X, P, &c2, &ndof, &st);
    upper_from_sym(P, u);
    for (int c = 0; c < 6; ++c) out_par[(size_t)c * ld + i] = X[c];
    for (int c = 0; c < 21; ++c) out_cov[(size_t)c * ld + i] = u[c];
    out_chi2[i] = c2;
    out_ndof[i] = ndof;
    out_status[i] = st;
  }
  free(rows);
  return 0;
}

/* FP64 inputs throughout (used by the exactness pins). */
int orc_fit64(const orc_geometry* g, int n, int ld, int first_layer, const double* hits,
              const double* seed_par, const double* seed_cov, const int8_t* q, double* out_par, double* out_cov,
              double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || g->n_layers > 32 || first_layer < 0) return 1;
  double rows[9 * 32];
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < g->n_layers; ++l)
      for (int c = 0; c < 9; ++c) rows[l * 9 + c] = hits[((size_t)l * 9 + c) * ld + i];
    double Xs[6], u[21], Ps[36], X[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one(g, first_layer, rows, 0u, Xs, Ps, q[i], X, P, &c2, &ndof, &st);
    upper_from_sym(P, u);
    for (int c = 0; c < 6; ++c) out_par[(size_t)c * ld + i] = X[c];
    for (int c = 0; c < 21; ++c) out_cov[(size_t)c * ld + i] = u[c];
    out_chi2[i] = c2;
    out_ndof[i] = ndof;
    out_status[i] = st;
  }
  return 0;
}

/* ---------------------------------------------------------- binning */

/*
 * Hit binning (the hit-selection structure of section 3.1): per layer,
 * n_z x n_phi bins, bin = iz * n_phi + iphi, with
 *   phi  = atan2(y, x) in [0, 2 pi), computed in FP64, rounded to FP32;
 *   iphi = min(n_phi - 1, floor(phi_f32 * n_phi / (2 pi)))  (FP64);
 *   iz   = clamp(floor((z + z_half) * n_z / (2 z_half)), 0, n_z - 1) (FP64).
 * Hits are ordered by (layer, bin, phi_f32, original index).
 * offsets[l*(nb+1) + b] is the position of the first hit of bin b of layer
 * l in that order (nb = n_phi*n_z; entry nb closes the layer).  A hit on a
 * layer outside [0, L) or with a non-finite coordinate has no place in the
 * binned structure: it sorts after every layer (reading: such a hit is
 * rejected, not binned).
 */
typedef struct { int32_t layer, bin; float phi; int32_t idx; } bin_key;

static int bin_key_cmp(const void* pa, const void* pb) {
  const bin_key* a = (const bin_key*)pa;
  const bin_key* b = (const bin_key*)pb;
  if (a->layer != b->layer) return a->layer < b->layer ? -1 : 1;
  if (a->bin != b->bin) return a->bin < b->bin ? -1 : 1;
  if (a->phi != b->phi) return a->phi < b->phi ? -1 : 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

int orc_hit_bin(const orc_geometry* g, int n_phi, int n_z, int n_hits, const int32_t* layer, const float* xyz,
                int32_t* offsets, int32_t* order, float* phi_sorted) {
  if (n_phi < 1 || n_z < 1 || n_hits < 0) return 1;
  int nb = n_phi * n_z, L = g->n_layers;
  bin_key* k = (bin_key*)malloc(sizeof(bin_key) * (size_t)(n_hits > 0 ? n_hits : 1));
  double zh = (double)g->z_half;
  for (int i = 0; i < n_hits; ++i) {
    double x = (double)xyz[i], y = (double)xyz[(size_t)n_hits + i], z = (double)xyz[2 * (size_t)n_hits + i];
    if (layer[i] < 0 || layer[i] >= L || !isfinite(x) || !isfinite(y) || !isfinite(z)) {
      k[i].layer = INT32_MAX; k[i].bin = 0; k[i].phi = 0.0f; k[i].idx = i;
      continue;
    }
    double ph = atan2(y, x);
    if (ph < 0.0) ph += TWO_PI;
    float phf = (float)ph;
    int ip = (int)floor((double)phf * (double)n_phi / TWO_PI);
    if (ip > n_phi - 1) ip = n_phi - 1;
    if (ip < 0) ip = 0;
    int iz = (int)floor((z + zh) * (double)n_z / (2.0 * zh));
    if (iz < 0) iz = 0;
    if (iz > n_z - 1) iz = n_z - 1;
    k[i].layer = layer[i];
    k[i].bin = iz * n_phi + ip;
    k[i].phi = phf;
    k[i].idx = i;
  }
  qsort(k, (size_t)n_hits, sizeof(bin_key), bin_key_cmp);
  for (int i = 0; i < n_hits; ++i) { order[i] = k[i].idx; phi_sorted[i] = k[i].phi; }
  /* offsets: first sorted position with (layer, bin) >= (l, b) */
  int pos = 0;
  for (int l = 0; l < L; ++l)
    for (int b = 0; b <= nb; ++b) {
      while (pos < n_hits && (k[pos].layer < l || (k[pos].layer == l && k[pos].bin < b))) ++pos;
      offsets[l * (nb + 1) + b] = pos;
    }
  free(k);
  return 0;
}

/* ------------------------------------------------------ learned window */

/*
 * Parameter block of the window network (FP64 values of the BF16 weights):
 *   mu[27] sd[27] W1[64][27] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]
 *   scale[2] kappa floor_rphi floor_z gate_rphi gate_z
 */
#define MLP_OFF_MU 0
#define MLP_OFF_SD 27
#define MLP_OFF_W1 54
#define MLP_OFF_B1 (MLP_OFF_W1 + 64 * 27)
#define MLP_OFF_W2 (MLP_OFF_B1 + 64)
#define MLP_OFF_B2 (MLP_OFF_W2 + 64 * 64)
#define MLP_OFF_W3 (MLP_OFF_B2 + 64)
#define MLP_OFF_B3 (MLP_OFF_W3 + 2 * 64)
#define MLP_OFF_SCALE (MLP_OFF_B3 + 2)
#define MLP_OFF_KAPPA (MLP_OFF_SCALE + 2)
#define MLP_OFF_FLOOR (MLP_OFF_KAPPA + 1)
#define MLP_OFF_GATE (MLP_OFF_FLOOR + 2)
#define MLP_SIZE (MLP_OFF_GATE + 2)

int orc_mlp_blob_size(void) { return MLP_SIZE; }

/* round to the nearest bfloat16 (ties to even), via FP32 */
static double bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double softplus(double o) { return o > 30.0 ? o : log1p(exp(o)); }

/*
 * Window network: x_hat = (x - mu)/sd rounded to BF16; two GELU layers of
 * width 64 whose outputs are rounded to BF16 (they feed BF16 products);
 * a linear head; widths = scale * softplus(o) (arc half-width at the
 * layer radius in cm, z half-width in cm).  kappa is applied by the caller.
 */
int orc_mlp_forward(const double* m, const double x[27], double w[2]) {
  double xh[27], h1[64], h2[64];
  for (int k = 0; k < 27; ++k) xh[k] = bf16_round((x[k] - m[MLP_OFF_MU + k]) / m[MLP_OFF_SD + k]);
  for (int j = 0; j < 64; ++j) {
    double s = m[MLP_OFF_B1 + j];
    for (int k = 0; k < 27; ++k) s += m[MLP_OFF_W1 + j * 27 + k] * xh[k];
    h1[j] = bf16_round(gelu(s));
  }
  for (int j = 0; j < 64; ++j) {
    double s = m[MLP_OFF_B2 + j];
    for (int k = 0; k < 64; ++k) s += m[MLP_OFF_W2 + j * 64 + k] * h1[k];
    h2[j] = bf16_round(gelu(s));
  }
  for (int j = 0; j < 2; ++j) {
    double s = m[MLP_OFF_B3 + j];
    for (int k = 0; k < 64; ++k) s += m[MLP_OFF_W3 + j * 64 + k] * h2[k];
    w[j] = m[MLP_OFF_SCALE + j] * softplus(s);
  }
  return 0;
}

/* ------------------------------------------------------------ build */

typedef struct {
  double X[6], P[36];
  int nhits, holes, status;
  double chi2;
  int32_t hits[32]; /* per searched layer: original hit index, -1 none */
} cand_t;

typedef struct {
  int nhits, parent, hit, holes;
  double chi2;
  double X[6], P[36];
} child_t;

/* rank order: nhits desc, chi2 asc, parent slot asc, hit index asc, hole last */
static int child_cmp(const void* pa, const void* pb) {
  const child_t* a = (const child_t*)pa;
  const child_t* b = (const child_t*)pb;
  if (a->nhits != b->nhits) return a->nhits > b->nhits ? -1 : 1;
  if (a->chi2 != b->chi2) return a->chi2 < b->chi2 ? -1 : 1;
  if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
  long ha = a->hit < 0 ? 0x7fffffffL : a->hit, hb = b->hit < 0 ? 0x7fffffffL : b->hit;
  return ha < hb ? -1 : (ha > hb ? 1 : 0);
}

static int better(int n1, double c1, int n2, double c2) { return n1 > n2 || (n1 == n2 && c1 < c2); }

static double wrap_pi(double d) {
  while (d > PI) d -= TWO_PI;
  while (d <= -PI) d += TWO_PI;
  return d;
}

static double minf(double a, double b) { return a < b ? a : b; }

/*
 * Combinatorial track building (section 2; fixed candidate slots per seed
 * ranked best-first, section 4.3).  For each seed, layer by layer from
 * first_layer:
 *   1. predict every active candidate; a failed propagation (no crossing or
 *      |z| > z_half) stops it;
 *   2. window: plain = nsigma * sqrt(S) per coordinate with S = H P H^T +
 *      diag(win_sig_rphi^2, win_sig_z^2), as dphi = w_rphi / R, dz = w_z;
 *      learned (only where the plain arc half-width exceeds gate_rphi or
 *      the plain z half-width exceeds gate_z; the plain window elsewhere)
 *      = kappa * network widths where they are not below the floors, the
 *      plain width otherwise;
 *   3. scan every hit of the layer in original-index order; a hit is in
 *      the window iff |wrap(phi_h - phi_p)| <= dphi and |z_h - z_p| <= dz;
 *      it is accepted iff its update chi2 < chi2_cut;
 *   4. children: one updated child per accepted hit, plus a hole child
 *      (predicted state, no update) while holes < max_holes;
 *   5. all children of the seed are ranked (nhits desc, chi2 asc, parent
 *      slot asc, hit asc, hole last); the first cand_cap become the new
 *      candidates in that order (CAP_TRUNC marks a cut);
 *   6. a candidate with no child is finished and competes for the seed's
 *      single best-finished record under (nhits desc, chi2 asc), replacing
 *      it only when strictly better.
 * The result is the best of (active candidates in slot order, then the
 * finished record) under (nhits desc, chi2 asc), first wins ties.  nhits
 * counts hits on the searched layers only.
 *
 * With state = 1 the candidates carry the hybrid state (x, y, z, q/pT, phi,
 * theta): the seed is converted on entry, predictions are hybrid ones (the
 * charge follows the sign of q/pT), the update and the window are unchanged
 * (they use the position and its covariance block), and the outputs are
 * hybrid.
 *
 * out_margin[5][ld] records, per seed, the smallest distance of any
 * decision from its threshold, one row per kind of decision:
 *   [0] chi2 (absolute: |chi2 - cut| of in-window hits, chi2 gaps at equal
 *       nhits for cap cuts, record replacements and the final choice);
 *   [1] plain window edges (cm: R*| |dphi| - dphi_w | or | |dz| - dz_w | of
 *       the coordinate whose test decided, where that coordinate's width is
 *       the covariance window's);
 *   [2] geometry (normalised crossing discriminant, | |z| - z_half |/z_half);
 *   [3] gate of the learned window (cm: distance of the plain half-widths
 *       from the gates that decide whether the network is consulted);
 *   [4] learned widths (cm: window edges of a coordinate whose width came
 *       from the network, and learned width vs floor).
 * A window decision is "in" iff both coordinates pass: if both pass, each
 * coordinate's distance goes to its own row; if one fails, that one's; if
 * both fail, the larger of the two (flipping the decision needs both) goes to
 * the learned row when either width is learned, else to the plain row.
 */
int orc_build(const orc_geometry* g, const orc_build_params* bp, int n_hits, const int32_t* layer,
              const float* xyz, const float* cov, int n_seeds, int ld, const float* seed_par,
              const float* seed_cov, const int8_t* q, int n_list, const int32_t* seed_list,
              int32_t* out_hits, double* out_par, double* out_cov, double* out_chi2, int32_t* out_nhits,
              int32_t* out_status, double* out_margin) {
  const int L = g->n_layers, F = bp->first_layer;
  if (n_seeds < 0 || ld < n_seeds || L > 32 || F < 0 || F >= L || bp->cand_cap < 1 || n_list < 0 || n_list > ld)
    return 1;
  if (bp->window_mode == 1 && !bp->mlp) return 1;
  if (bp->state != 0 && bp->state != 1) return 1;
  /* group hit indices by layer, increasing original index */
  int* lay_cnt = (int*)calloc((size_t)L, sizeof(int));
  int* lay_off = (int*)calloc((size_t)L + 1, sizeof(int));
  int* lay_idx = (int*)malloc(sizeof(int) * (size_t)(n_hits > 0 ? n_hits : 1));
  for (int i = 0; i < n_hits; ++i) if (layer[i] >= 0 && layer[i] < L) lay_cnt[layer[i]]++;
  for (int l = 0; l < L; ++l) lay_off[l + 1] = lay_off[l] + lay_cnt[l];
  for (int l = 0; l < L; ++l) lay_cnt[l] = 0;
  for (int i = 0; i < n_hits; ++i)
    if (layer[i] >= 0 && layer[i] < L) lay_idx[lay_off[layer[i]] + lay_cnt[layer[i]]++] = i;

  int cap = bp->cand_cap;
  cand_t* act = (cand_t*)malloc(sizeof(cand_t) * (size_t)cap);
  cand_t* nxt = (cand_t*)malloc(sizeof(cand_t) * (size_t)cap);
  int* stopped = (int*)malloc(sizeof(int) * (size_t)cap);
  int* stop_status = (int*)malloc(sizeof(int) * (size_t)cap);
  size_t ch_cap = 64;
  child_t* ch = (child_t*)malloc(sizeof(child_t) * ch_cap);
  const size_t N = (size_t)n_hits;

  for (int li = 0; li < n_list; ++li) {
    int i = seed_list ? seed_list[li] : li;
    double mc2 = INFINITY, mwin = INFINITY, mgeo = INFINITY, mgate = INFINITY, mlrn = INFINITY;
    int seed_status = 0;
    cand_t fin;
    int have_fin = 0;
    int qi = q[i];
    int n_act = 1;
    memset(&act[0], 0, sizeof(cand_t));
    double u[21];
    for (int c = 0; c < 6; ++c) act[0].X[c] = (double)seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = (double)seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, act[0].P);
    if (bp->state == 1) { /* the seed in the hybrid state */
      double Y[6], B[36], Pc[36];
      memcpy(Pc, act[0].P, sizeof(Pc));
      orc_hyb_from_cart(act[0].X, qi, Y);
      orc_hyb_jac_hyb_from_cart(act[0].X, qi, B);
      congruence(B, Pc, act[0].P);
      memcpy(act[0].X, Y, sizeof(Y));
    }
    for (int l = 0; l < 32; ++l) act[0].hits[l] = -1;
    if (!all_finite(act[0].X, 6) || !all_finite(act[0].P, 36)) {
      act[0].status = ORC_TRK_NONFINITE;
      n_act = 0;
      fin = act[0];
      have_fin = 1;
    }
    for (int l = F; l < L && n_act > 0; ++l) {
      double R = (double)g->r[l];
      size_t nch = 0;
      int n_stop = 0;
      for (int a = 0; a < n_act; ++a) {
        cand_t* c = &act[a];
        double Xp[6], Pp[36], disc = INFINITY;
        int rc = bp->state == 1 ? orc_predict_hyb(g, l, c->X, c->P, Xp, Pp, &disc)
                                : orc_predict(g, l, c->X, qi, c->P, Xp, Pp, &disc);
        if (isfinite(disc)) mgeo = minf(mgeo, disc);
        if (rc != ORC_TRK_NO_CROSSING && rc != ORC_TRK_NONFINITE) mgeo = minf(mgeo, fabs(fabs(Xp[2]) - (double)g->z_half) / (double)g->z_half);
        if (rc) { stopped[n_stop] = a; stop_status[n_stop++] = rc; continue; }
        /* window */
        double rr = sqrt(Xp[0] * Xp[0] + Xp[1] * Xp[1]);
        double tx = -Xp[1] / rr, ty = Xp[0] / rr;
        double Suu = tx * tx * Pp[0] + 2.0 * tx * ty * Pp[1] + ty * ty * Pp[7] +
                     (double)bp->win_sig_rphi * (double)bp->win_sig_rphi;
        double Sww = Pp[14] + (double)bp->win_sig_z * (double)bp->win_sig_z;
        double w_rphi = (double)bp->nsigma * sqrt(Suu), w_z = (double)bp->nsigma * sqrt(Sww);
        /* learned window: consulted where the covariance window is wide (its
           arc or z half-width above the gate); elsewhere the plain window */
        int gated = 0, lrn_rphi = 0, lrn_z = 0; /* a width from the network */
        if (bp->window_mode == 1) {
          double dr = w_rphi - bp->mlp[MLP_OFF_GATE], dz = w_z - bp->mlp[MLP_OFF_GATE + 1];
          gated = dr > 0.0 || dz > 0.0;
          /* distance of the gate decision from flipping (cm) */
          double gm = gated ? fmax(dr > 0.0 ? dr : 0.0, dz > 0.0 ? dz : 0.0) : fmin(-dr, -dz);
          mgate = minf(mgate, gm);
        }
        if (gated) {
          /* features: the Cartesian prediction and covariance (a hybrid
             prediction is converted: state, and covariance through
             d(X)/d(Y)) */
          double feat[27], wl[2], pu[21], Xf[6], Pf[36];
          memcpy(Xf, Xp, sizeof(Xf));
          memcpy(Pf, Pp, sizeof(Pf));
          if (bp->state == 1) {
            double A[36];
            orc_cart_from_hyb(Xp, Xf);
            orc_hyb_jac_cart_from_hyb(Xp, A);
            congruence(A, Pp, Pf);
          }
          for (int k = 0; k < 6; ++k) feat[k] = Xf[k];
          upper_from_sym(Pf, pu);
          for (int k = 0; k < 21; ++k) feat[6 + k] = pu[k];
          orc_mlp_forward(bp->mlp, feat, wl);
          double kap = bp->mlp[MLP_OFF_KAPPA];
          double fl[2] = {bp->mlp[MLP_OFF_FLOOR], bp->mlp[MLP_OFF_FLOOR + 1]};
          double lw[2] = {kap * wl[0], kap * wl[1]};
          mlrn = minf(mlrn, fabs(lw[0] - fl[0]));
          mlrn = minf(mlrn, fabs(lw[1] - fl[1]));
          if (!(lw[0] < fl[0])) { w_rphi = lw[0]; lrn_rphi = 1; }
          if (!(lw[1] < fl[1])) { w_z = lw[1]; lrn_z = 1; }
        }
        double dphi_w = w_rphi / R, dz_w = w_z;
        double php = atan2(Xp[1], Xp[0]), zp = Xp[2];
        int n_own = 0;
        for (int k = lay_off[l]; k < lay_off[l + 1]; ++k) {
          int hi = lay_idx[k];
          double hx = (double)xyz[hi], hy = (double)xyz[N + hi], hz = (double)xyz[2 * N + hi];
          double dph = wrap_pi(atan2(hy, hx) - php), dz = hz - zp;
          double aph = fabs(dph), az = fabs(dz);
          int pph = aph <= dphi_w, pz = az <= dz_w;
          double mph = R * fabs(aph - dphi_w), mz = fabs(az - dz_w);
          double* row_ph = lrn_rphi ? &mlrn : &mwin;
          double* row_z = lrn_z ? &mlrn : &mwin;
          if (pph && pz) { *row_ph = minf(*row_ph, mph); *row_z = minf(*row_z, mz); }
          else if (!pph && !pz) {
            double* row = (lrn_rphi || lrn_z) ? &mlrn : &mwin;
            *row = minf(*row, mph > mz ? mph : mz);
          } else if (!pph) *row_ph = minf(*row_ph, mph);
          else *row_z = minf(*row_z, mz);
          if (!(pph && pz)) continue;
          double hit[9] = {hx, hy, hz};
          for (int cc = 0; cc < 6; ++cc) hit[3 + cc] = (double)cov[(size_t)cc * N + hi];
          double Xu[6], Pu[36], c2;
          if (orc_update(Xp, Pp, hit, Xu, Pu, &c2)) continue;
          mc2 = minf(mc2, fabs(c2 - (double)bp->chi2_cut));
          if (!(c2 < (double)bp->chi2_cut)) continue;
          if (nch == ch_cap) { ch_cap *= 2; ch = (child_t*)realloc(ch, sizeof(child_t) * ch_cap); }
          child_t* d = &ch[nch++];
          d->nhits = c->nhits + 1; d->parent = a; d->hit = hi; d->holes = c->holes;
          d->chi2 = c->chi2 + c2;
          memcpy(d->X, Xu, sizeof(Xu)); memcpy(d->P, Pu, sizeof(Pu));
          ++n_own;
        }
        if (c->holes < bp->max_holes) {
          if (nch == ch_cap) { ch_cap *= 2; ch = (child_t*)realloc(ch, sizeof(child_t) * ch_cap); }
          child_t* d = &ch[nch++];
          d->nhits = c->nhits; d->parent = a; d->hit = -1; d->holes = c->holes + 1;
          d->chi2 = c->chi2;
          memcpy(d->X, Xp, sizeof(Xp)); memcpy(d->P, Pp, sizeof(Pp));
          ++n_own;
        }
        if (n_own == 0) { stopped[n_stop] = a; stop_status[n_stop++] = 0; }
      }
      /* finished candidates compete for the record, in slot order */
      for (int s = 0; s < n_stop; ++s) {
        cand_t* c = &act[stopped[s]];
        c->status |= stop_status[s];
        if (!have_fin) { fin = *c; have_fin = 1; continue; }
        if (c->nhits == fin.nhits) mc2 = minf(mc2, fabs(c->chi2 - fin.chi2));
        if (better(c->nhits, c->chi2, fin.nhits, fin.chi2)) fin = *c;
      }
      qsort(ch, nch, sizeof(child_t), child_cmp);
      size_t keep = nch < (size_t)cap ? nch : (size_t)cap;
      if (nch > (size_t)cap) {
        seed_status |= ORC_TRK_CAP_TRUNC;
        if (ch[cap - 1].nhits == ch[cap].nhits) mc2 = minf(mc2, fabs(ch[cap].chi2 - ch[cap - 1].chi2));
      }
      for (size_t k = 0; k < keep; ++k) {
        cand_t* d = &nxt[k];
        const cand_t* p = &act[ch[k].parent];
        memcpy(d->hits, p->hits, sizeof(d->hits));
        d->hits[l - F] = ch[k].hit;
        memcpy(d->X, ch[k].X, sizeof(d->X)); memcpy(d->P, ch[k].P, sizeof(d->P));
        d->nhits = ch[k].nhits; d->holes = ch[k].holes; d->chi2 = ch[k].chi2; d->status = 0;
      }
      cand_t* t = act; act = nxt; nxt = t;
      n_act = (int)keep;
    }
    /* final choice */
    const cand_t* best = NULL;
    for (int a = 0; a < n_act; ++a) {
      if (!best) { best = &act[a]; continue; }
      if (better(act[a].nhits, act[a].chi2, best->nhits, best->chi2)) best = &act[a];
    }
    if (have_fin && (!best || better(fin.nhits, fin.chi2, best->nhits, best->chi2))) best = &fin;
    for (int a = 0; a < n_act; ++a)
      if (&act[a] != best && act[a].nhits == best->nhits) mc2 = minf(mc2, fabs(act[a].chi2 - best->chi2));
    if (have_fin && &fin != best && fin.nhits == best->nhits) mc2 = minf(mc2, fabs(fin.chi2 - best->chi2));
    double ub[21];
    upper_from_sym(best->P, ub);
    for (int l = F; l < L; ++l) out_hits[(size_t)(l - F) * ld + li] = best->hits[l - F];
    for (int c = 0; c < 6; ++c) out_par[(size_t)c * ld + li] = best->X[c];
    for (int c = 0; c < 21; ++c) out_cov[(size_t)c * ld + li] = ub[c];
    out_chi2[li] = best->chi2;
    out_nhits[li] = best->nhits;
    out_status[li] = best->status | seed_status;
    if (out_margin) {
      out_margin[li] = mc2;
      out_margin[(size_t)ld + li] = mwin;
      out_margin[2 * (size_t)ld + li] = mgeo;
      out_margin[3 * (size_t)ld + li] = mgate;
      out_margin[4 * (size_t)ld + li] = mlrn;
    }
  }
  free(act); free(nxt); free(ch); free(stopped); free(stop_status); free(lay_cnt); free(lay_off); free(lay_idx);
  return 0;
}

/* ===================================================================
 * General detector (section 4.1): barrel cylinders and endcap disks (the
 * "cylinder with lids"), whose modules may sit off the layer's average
 * surface.  Track building propagates in two steps: to the layer's average
 * surface (average radius of a barrel layer, average z of a disk), then from
 * there to the surface of each candidate hit; the update is made at the
 * hit.  A barrel hit is measured on the plane tangent to the cylinder
 * through the hit (section 4.1), a disk hit in the disk's plane (x, y).
 * =================================================================== */

static int det_kind_ok(const orc_detector* d, int l) { return d->kind[l] == ORC_BARREL || d->kind[l] == ORC_DISK; }

/*
 * Crossing of the helix with the cylinder r = R.  nearest = 0: the first
 * crossing along the motion (s > 0, as orc_propagate); nearest = 1: the
 * crossing reached by the shortest path forwards or backwards (s of either
 * sign), the second step from a layer's average surface to a hit's.
 * Returns ORC_TRK_NO_CROSSING if the circles do not meet; *disc as
 * orc_propagate.
 */
int orc_cyl_path(const double X[6], int q, double R, double bz, int nearest, double* s_out, double* disc) {
  double px = X[3], py = X[4];
  double pt = sqrt(px * px + py * py);
  if (disc) *disc = INFINITY;
  if (!(pt > 0.0) || bz == 0.0) return ORC_TRK_NO_CROSSING;
  double h = -(double)q * KAPPA * bz / pt;
  double cx = X[0] - py / (pt * h), cy = X[1] + px / (pt * h);
  double rho = 1.0 / fabs(h);
  double d = sqrt(cx * cx + cy * cy);
  if (!(d > 0.0) || d > R + rho || d < fabs(R - rho)) return ORC_TRK_NO_CROSSING;
  double a = (R * R - rho * rho + d * d) / (2.0 * d);
  double b2 = R * R - a * a;
  if (b2 < 0.0) b2 = 0.0;
  if (disc) *disc = b2 / (R * R);
  double b = sqrt(b2);
  double best = INFINITY;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    double Px = (a / d) * cx + sgn * (b / d) * (-cy);
    double Py = (a / d) * cy + sgn * (b / d) * cx;
    double ux = X[0] - cx, uy = X[1] - cy;
    double vx = Px - cx, vy = Py - cy;
    double alpha = atan2(ux * vy - uy * vx, ux * vx + uy * vy); /* (-pi, pi] */
    if (!nearest) {
      if (h > 0.0 && alpha <= 0.0) alpha += TWO_PI;
      if (h < 0.0 && alpha >= 0.0) alpha -= TWO_PI;
    }
    double s = alpha / h;
    if (nearest ? fabs(s) < fabs(best) : s < best) best = s;
  }
  *s_out = best;
  return 0;
}

/*
 * Crossing with the plane z = Z: z(s) = z + pz s / pT gives s = (Z - z) pT / pz.
 * nearest = 0 requires s > 0 (the plane lies ahead); nearest = 1 takes s of
 * either sign.  A track parallel to the plane (pz = 0) has no crossing.
 */
int orc_plane_path(const double X[6], double Z, int nearest, double* s_out) {
  double pt = sqrt(X[3] * X[3] + X[4] * X[4]);
  if (!(pt > 0.0) || X[5] == 0.0) return ORC_TRK_NO_CROSSING;
  double s = (Z - X[2]) * pt / X[5];
  if (!nearest && !(s > 0.0)) return ORC_TRK_NO_CROSSING;
  if (!isfinite(s)) return ORC_TRK_NO_CROSSING;
  *s_out = s;
  return 0;
}

/* Unit normal of a surface at point x: radial for a cylinder, zhat for a plane. */
static void surface_normal(int kind, const double x[3], double n[3]) {
  if (kind == ORC_DISK) { n[0] = 0.0; n[1] = 0.0; n[2] = 1.0; return; }
  double r = sqrt(x[0] * x[0] + x[1] * x[1]);
  n[0] = x[0] / r; n[1] = x[1] / r; n[2] = 0.0;
}

/*
 * Jacobian of "state -> state on the surface" (cylinder: kind = barrel,
 * plane: kind = disk) after the path s: J = Js + w g^T with
 * g = ds/dX0 = -(n . Js[position rows]) / (n . w[position]), n the surface
 * normal at the end point.  The end point stays on the surface, so every
 * transported covariance has the null vector (n, 0, 0, 0).
 */
void orc_jacobian_surf(const double X[6], int q, double bz, double s, int kind, double J[36]) {
  double Js[36], w[6], Xo[6], n[3];
  jacobian_fixed_path(X, q, bz, s, Js, w, Xo);
  surface_normal(kind, Xo, n);
  double den = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
  double g[6];
  for (int j = 0; j < 6; ++j) g[j] = -(n[0] * Js[0 * 6 + j] + n[1] * Js[1 * 6 + j] + n[2] * Js[2 * 6 + j]) / den;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) J[i * 6 + j] = Js[i * 6 + j] + w[i] * g[j];
}

/* Highland noise of a thin layer crossed at X: as orc_ms_cov with the
 * incidence measured from the normal of the surface (radial or zhat). */
void orc_ms_cov_surf(const double X[6], int kind, double x_over_x0, double mass, double Q[36]) {
  memset(Q, 0, sizeof(double) * 36);
  if (!(x_over_x0 > 0.0)) return;
  double p2 = X[3] * X[3] + X[4] * X[4] + X[5] * X[5];
  double p = sqrt(p2);
  double n[3];
  surface_normal(kind, X, n);
  double cospsi = fabs((n[0] * X[3] + n[1] * X[4] + n[2] * X[5]) / p);
  double xe = x_over_x0 / cospsi;
  double beta = p / sqrt(p2 + mass * mass);
  double th0 = 0.0136 / (beta * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / (beta * beta)));
  double t2 = th0 * th0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Q[(3 + i) * 6 + 3 + j] = t2 * ((i == j ? p2 : 0.0) - X[3 + i] * X[3 + j]);
}

/*
 * One propagation step to a surface (kind, value = radius or z): the helix
 * to the crossing (first along the motion, or nearest when `nearest`), the
 * covariance transported with the surface Jacobian, and, when `material`,
 * the scattering noise of a thin layer at the end point.
 */
int orc_step_surf(const orc_detector* d, int kind, double value, int nearest, int material, const double X[6],
                  int q, const double P[36], double Xo[6], double Po[36], double* disc) {
  double s;
  int rc = kind == ORC_DISK ? orc_plane_path(X, value, nearest, &s)
                            : orc_cyl_path(X, q, value, (double)d->bz, nearest, &s, disc);
  if (rc) return rc;
  orc_state_at(X, q, (double)d->bz, s, Xo);
  double J[36], JT[36], T[36];
  orc_jacobian_surf(X, q, (double)d->bz, s, kind, J);
  transpose(J, JT, 6, 6);
  matmul(J, P, T, 6, 6, 6);
  matmul(T, JT, Po, 6, 6, 6);
  if (material) {
    double Q[36];
    orc_ms_cov_surf(Xo, kind, (double)d->x_over_x0, (double)d->mass, Q);
    for (int i = 0; i < 36; ++i) Po[i] += Q[i];
  }
  return 0;
}

/*
 * Kalman update with a disk hit, measured in the disk's plane: H picks
 * (x, y), residual (m_x - x, m_y - y), V2 the (x, y) block of the hit's
 * covariance; otherwise as orc_update.
 */
int orc_update_disk(const double X[6], const double P[36], const double hit[9], double Xo[6], double Po[36],
                    double* chi2) {
  double H[12] = {1, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0};
  double V2[4] = {hit[3], hit[4], hit[4], hit[6]};
  double res[2] = {hit[0] - X[0], hit[1] - X[1]};
  double HT[12], PHT[12], S[4];
  transpose(H, HT, 2, 6);
  matmul(P, HT, PHT, 6, 6, 2);
  matmul(H, PHT, S, 2, 6, 2);
  for (int i = 0; i < 4; ++i) S[i] += V2[i];
  double det = S[0] * S[3] - S[1] * S[2];
  if (!(S[0] > 0.0) || !(det > 0.0)) return ORC_TRK_S_NOT_PD;
  double Si[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
  double K[12], HP[12], KHP[36];
  matmul(PHT, Si, K, 6, 2, 2);
  for (int i = 0; i < 6; ++i) Xo[i] = X[i] + K[i * 2 + 0] * res[0] + K[i * 2 + 1] * res[1];
  matmul(H, P, HP, 2, 6, 6);
  matmul(K, HP, KHP, 6, 2, 6);
  for (int i = 0; i < 36; ++i) Po[i] = P[i] - KHP[i];
  double Sir[2] = {Si[0] * res[0] + Si[1] * res[1], Si[2] * res[0] + Si[3] * res[1]};
  *chi2 = res[0] * Sir[0] + res[1] * Sir[1];
  return 0;
}

/* the surface a hit lies on: its radius (barrel) or its z (disk) */
static double hit_surface(int kind, const double hit[9]) {
  return kind == ORC_DISK ? hit[2] : sqrt(hit[0] * hit[0] + hit[1] * hit[1]);
}

/* update with a hit of a layer of the given kind, at the predicted state */
static int update_kind(int kind, const double X[6], const double P[36], const double hit[9], double Xo[6],
                       double Po[36], double* chi2) {
  return kind == ORC_DISK ? orc_update_disk(X, P, hit, Xo, Po, chi2) : orc_update(X, P, hit, Xo, Po, chi2);
}

/* coordinate along a layer's extent: z on a barrel layer, r on a disk */
static double extent_coord(int kind, const double x[3]) {
  return kind == ORC_DISK ? sqrt(x[0] * x[0] + x[1] * x[1]) : x[2];
}

/*
 * Fit over a general detector (section 2: the Kalman filter over a fixed hit
 * list).  For each layer l >= first_layer (in index order) whose bit is set
 * in visit_mask[i]: with a hit (bit clear in hole_mask[i]) the state goes in
 * one step to the hit's own surface (its radius on a barrel layer, its z on a
 * disk; first crossing along the motion), takes the layer's scattering there
 * and is updated with the hit; on a hole it goes to the layer's average
 * surface and takes the scattering there.  The extents are not checked: the
 * list says which layers the track crossed.  Outputs as orc_fit.
 */
static void fit_one_det(const orc_detector* d, int first_layer, const double* hitrows, uint32_t visit,
                        uint32_t holes, const double Xs[6], const double Ps[36], int q, double Xout[6],
                        double Pout[36], double* chi2_out, int* ndof_out, int* status_out) {
  double X[6], P[36];
  memcpy(X, Xs, sizeof(X));
  memcpy(P, Ps, sizeof(P));
  double chi2 = 0.0;
  int ndof = 0, st = 0;
  if (!all_finite(X, 6) || !all_finite(P, 36)) st = ORC_TRK_NONFINITE;
  for (int l = first_layer; l < d->n_layers && !st; ++l) {
    if (!((visit >> l) & 1u)) continue;
    const double* h = hitrows + (size_t)l * 9;
    const int kind = d->kind[l];
    int use = !((holes >> l) & 1u);
    if (use && !all_finite(h, 9)) { st = ORC_TRK_NONFINITE; break; }
    double Xp[6], Pp[36];
    int rc = orc_step_surf(d, kind, use ? hit_surface(kind, h) : (double)d->pos[l], 0, 1, X, q, P, Xp, Pp, NULL);
    if (rc) { st = rc; break; }
    if (!use) {
      if (!all_finite(Xp, 6) || !all_finite(Pp, 36)) { st = ORC_TRK_NONFINITE; break; }
      memcpy(X, Xp, sizeof(X)); memcpy(P, Pp, sizeof(P));
      continue;
    }
    double Xu[6], Pu[36], c2;
    rc = update_kind(kind, Xp, Pp, h, Xu, Pu, &c2);
    if (rc) { st = rc; break; }
    if (!all_finite(Xu, 6) || !all_finite(Pu, 36) || !isfinite(c2)) { st = ORC_TRK_NONFINITE; break; }
    memcpy(X, Xu, sizeof(X)); memcpy(P, Pu, sizeof(P));
    chi2 += c2;
    ndof += 2;
  }
  memcpy(Xout, X, sizeof(X));
  memcpy(Pout, P, sizeof(P));
  *chi2_out = chi2;
  *ndof_out = ndof;
  *status_out = st;
}

static int det_ok(const orc_detector* d) {
  if (d->n_layers < 1 || d->n_layers > 32) return 0;
  for (int l = 0; l < d->n_layers; ++l)
    if (!det_kind_ok(d, l) || !(d->hi[l] > d->lo[l])) return 0;
  return 1;
}

int orc_fit_det(const orc_detector* d, int n, int ld, int first_layer, const float* hits, const uint32_t* visit_mask,
                const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || !det_ok(d) || first_layer < 0 || !visit_mask) return 1;
  double rows[9 * 32];
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < d->n_layers; ++l) load_hit(hits, ld, l, i, rows + l * 9);
    double Xs[6], u[21], Ps[36], X[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = (double)seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = (double)seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one_det(d, first_layer, rows, visit_mask[i], hole_mask ? hole_mask[i] : 0u, Xs, Ps, q[i], X, P, &c2, &ndof,
                &st);
    store_fit(ld, i, X, P, c2, ndof, st, out_par, out_cov, out_chi2, out_ndof, out_status);
  }
  return 0;
}

/* FP64 inputs throughout (used by the exactness pins). */
int orc_fit_det64(const orc_detector* d, int n, int ld, int first_layer, const double* hits,
                  const uint32_t* visit_mask, const double* seed_par, const double* seed_cov, const int8_t* q,
                  double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status) {
  if (n < 0 || ld < n || !det_ok(d) || first_layer < 0 || !visit_mask) return 1;
  double rows[9 * 32];
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l < d->n_layers; ++l)
      for (int c = 0; c < 9; ++c) rows[l * 9 + c] = hits[((size_t)l * 9 + c) * (size_t)ld + (size_t)i];
    double Xs[6], u[21], Ps[36], X[6], P[36], c2;
    int ndof, st;
    for (int c = 0; c < 6; ++c) Xs[c] = seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, Ps);
    fit_one_det(d, first_layer, rows, visit_mask[i], 0u, Xs, Ps, q[i], X, P, &c2, &ndof, &st);
    store_fit(ld, i, X, P, c2, ndof, st, out_par, out_cov, out_chi2, out_ndof, out_status);
  }
  return 0;
}

/*
 * Binning over a general detector: per layer n_w x n_phi bins, bin =
 * iw * n_phi + iphi, with phi as orc_hit_bin and the extent coordinate w = z
 * (barrel) or w = r = sqrt(x^2 + y^2) (disk), both in FP64 from the FP32
 * inputs: iw = clamp(floor((w - lo) * n_w / (hi - lo)), 0, n_w - 1).  Order
 * and offsets as orc_hit_bin.
 */
int orc_hit_bin_det(const orc_detector* d, int n_phi, int n_w, int n_hits, const int32_t* layer, const float* xyz,
                    int32_t* offsets, int32_t* order, float* phi_sorted) {
  if (n_phi < 1 || n_w < 1 || n_hits < 0 || !det_ok(d)) return 1;
  int nb = n_phi * n_w, L = d->n_layers;
  bin_key* k = (bin_key*)malloc(sizeof(bin_key) * (size_t)(n_hits > 0 ? n_hits : 1));
  for (int i = 0; i < n_hits; ++i) {
    double x = (double)xyz[i], y = (double)xyz[(size_t)n_hits + i], z = (double)xyz[2 * (size_t)n_hits + i];
    int l = layer[i];
    if (l < 0 || l >= L || !isfinite(x) || !isfinite(y) || !isfinite(z)) { /* rejected, as orc_hit_bin */
      k[i].layer = INT32_MAX; k[i].bin = 0; k[i].phi = 0.0f; k[i].idx = i;
      continue;
    }
    double ph = atan2(y, x);
    if (ph < 0.0) ph += TWO_PI;
    float phf = (float)ph;
    int ip = (int)floor((double)phf * (double)n_phi / TWO_PI);
    if (ip > n_phi - 1) ip = n_phi - 1;
    if (ip < 0) ip = 0;
    int iw = 0;
    if (l >= 0 && l < L) {
      double w = d->kind[l] == ORC_DISK ? sqrt(x * x + y * y) : z;
      double lo = (double)d->lo[l], hi = (double)d->hi[l];
      iw = (int)floor((w - lo) * (double)n_w / (hi - lo));
      if (iw < 0) iw = 0;
      if (iw > n_w - 1) iw = n_w - 1;
    }
    k[i].layer = layer[i];
    k[i].bin = iw * n_phi + ip;
    k[i].phi = phf;
    k[i].idx = i;
  }
  qsort(k, (size_t)n_hits, sizeof(bin_key), bin_key_cmp);
  for (int i = 0; i < n_hits; ++i) { order[i] = k[i].idx; phi_sorted[i] = k[i].phi; }
  int pos = 0;
  for (int l = 0; l < L; ++l)
    for (int b = 0; b <= nb; ++b) {
      while (pos < n_hits && (k[pos].layer < l || (k[pos].layer == l && k[pos].bin < b))) ++pos;
      offsets[l * (nb + 1) + b] = pos;
    }
  free(k);
  return 0;
}

typedef struct {
  double X[6], P[36];
  int nhits, holes, status, layer; /* layer: the last layer the candidate visited */
  double chi2;
  int32_t hits[32];                /* per layer: original hit index, -1 none */
  uint32_t visit;                  /* layers visited (hit or hole) */
} dcand_t;

typedef struct {
  int nhits, parent, hit, holes, layer;
  double chi2;
  double X[6], P[36];
} dchild_t;

static int dchild_cmp(const void* pa, const void* pb) {
  const dchild_t* a = (const dchild_t*)pa;
  const dchild_t* b = (const dchild_t*)pb;
  if (a->nhits != b->nhits) return a->nhits > b->nhits ? -1 : 1;
  if (a->chi2 != b->chi2) return a->chi2 < b->chi2 ? -1 : 1;
  if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
  long ha = a->hit < 0 ? 0x7fffffffL : a->hit, hb = b->hit < 0 ? 0x7fffffffL : b->hit;
  return ha < hb ? -1 : (ha > hb ? 1 : 0);
}

/*
 * The next layer of a candidate on layer `cur` (section 4.1's cylinder with
 * lids): the first layer after `cur`, in index order, whose average surface
 * the helix crosses ahead of it with the crossing inside the layer's extent
 * (barrel: z in [lo, hi]; disk: r in [lo, hi]) and, on a disk, within less
 * than half a turn and while still moving outwards (x px + y py > 0; a
 * barrel crossing from inside always is).  On success the
 * state and covariance on that surface (propagated without material) are
 * returned; -1 when the candidate leaves the detector.  Every crossing
 * test is recorded in *mgeo (crossing discriminant, side of a plane), every
 * extent test in *mwin (distance in cm of the extent coordinate from the
 * nearer edge: a position decision like a window edge).
 */
static int next_layer(const orc_detector* d, int cur, const double X[6], int q, const double P[36], double Xa[6],
                      double Pa[36], double* mgeo, double* mwin) {
  for (int j = cur + 1; j < d->n_layers; ++j) {
    double disc = INFINITY;
    int rc = orc_step_surf(d, d->kind[j], (double)d->pos[j], 0, 0, X, q, P, Xa, Pa, &disc);
    if (isfinite(disc)) *mgeo = minf(*mgeo, disc);
    if (d->kind[j] == ORC_DISK && X[5] != 0.0) /* which side of the plane the track is on */
      *mgeo = minf(*mgeo, fabs((double)d->pos[j] - X[2]) / fabs((double)d->pos[j]));
    if (rc) continue;
    if (d->kind[j] == ORC_DISK) {
      /* met on the way out, within less than half a turn (a looper that comes
         back is not followed) */
      double pt0 = sqrt(X[3] * X[3] + X[4] * X[4]);
      double turn = fabs(KAPPA * (double)d->bz / pt0 * ((double)d->pos[j] - X[2]) * pt0 / X[5]);
      double pr = Xa[0] * Xa[3] + Xa[1] * Xa[4];
      double ptr = sqrt(Xa[0] * Xa[0] + Xa[1] * Xa[1]) * sqrt(Xa[3] * Xa[3] + Xa[4] * Xa[4]);
      *mgeo = minf(*mgeo, minf(fabs(pr) / ptr, fabs(PI - turn) / PI));
      if (!(pr > 0.0) || !(turn < PI)) continue;
    }
    double w = extent_coord(d->kind[j], Xa), lo = (double)d->lo[j], hi = (double)d->hi[j];
    *mwin = minf(*mwin, minf(fabs(w - lo), fabs(hi - w)));
    if (w >= lo && w <= hi) return j;
  }
  return -1;
}

/*
 * Combinatorial build over a general detector (sections 2, 4.1, 4.3), with
 * the rules of orc_build (window, chi2 cut, children, ranking, cap,
 * best-finished record) and these differences:
 *   - each candidate moves to its own next layer (next_layer): a track that
 *     leaves the barrel through its end continues on the disks; a candidate
 *     with no next layer has left the detector and finishes (status 0);
 *   - two-step propagation: step 1 to the layer's average surface (no
 *     material), where the window is formed; step 2, for every hit in the
 *     window, from there to the hit's own surface (nearest crossing),
 *     scattering of the layer at the hit, then the update (tangent plane at
 *     the hit's radius on a barrel layer, the disk's plane on a disk) and its
 *     chi2; a hole child takes the layer's scattering at the average surface;
 *   - window: barrel (phi, z), disk (phi, r), each half-width nsigma *
 *     sqrt(S) of the predicted covariance with the nominal resolution
 *     (win_sig_rphi along the arc, win_sig_z along z or r), widened by the
 *     module offset dmod times the track's slope (|dz/dr| and |dphi/dr| on a
 *     barrel layer, |dr/dz| and |dphi/dz| on a disk) so hits of displaced
 *     modules stay inside; a hit is in the window iff |wrap(phi_h - phi_p)|
 *     <= dphi and |w_h - w_p| <= dw (w = z or r).
 * Outputs: out_hits[L - F][ld] per layer (original index, -1 for a hole or a
 * layer not visited), out_visit[ld] the layers the chosen candidate visited,
 * the rest as orc_build; out_margin rows as orc_build, the extent tests
 * counted with the window edges (cm) and the side of a disk's plane with the
 * geometry (gate and learned rows stay infinite).  Cartesian state, plain
 * window.
 */
int orc_build_det(const orc_detector* d, const orc_build_params* bp, int n_hits, const int32_t* layer,
                  const float* xyz, const float* cov, int n_seeds, int ld, const float* seed_par,
                  const float* seed_cov, const int8_t* q, int n_list, const int32_t* seed_list, int32_t* out_hits,
                  uint32_t* out_visit, double* out_par, double* out_cov, double* out_chi2, int32_t* out_nhits,
                  int32_t* out_status, double* out_margin) {
  const int L = d->n_layers, F = bp->first_layer;
  if (!det_ok(d) || n_seeds < 0 || ld < n_seeds || F < 1 || F >= L || bp->cand_cap < 1 || n_list < 0 ||
      n_list > ld || bp->window_mode != 0 || bp->state != 0)
    return 1;
  int* lay_cnt = (int*)calloc((size_t)L, sizeof(int));
  int* lay_off = (int*)calloc((size_t)L + 1, sizeof(int));
  int* lay_idx = (int*)malloc(sizeof(int) * (size_t)(n_hits > 0 ? n_hits : 1));
  for (int i = 0; i < n_hits; ++i) if (layer[i] >= 0 && layer[i] < L) lay_cnt[layer[i]]++;
  for (int l = 0; l < L; ++l) lay_off[l + 1] = lay_off[l] + lay_cnt[l];
  for (int l = 0; l < L; ++l) lay_cnt[l] = 0;
  for (int i = 0; i < n_hits; ++i)
    if (layer[i] >= 0 && layer[i] < L) lay_idx[lay_off[layer[i]] + lay_cnt[layer[i]]++] = i;

  const int cap = bp->cand_cap;
  dcand_t* act = (dcand_t*)malloc(sizeof(dcand_t) * (size_t)cap);
  dcand_t* nxt = (dcand_t*)malloc(sizeof(dcand_t) * (size_t)cap);
  int* stopped = (int*)malloc(sizeof(int) * (size_t)cap);
  size_t ch_cap = 64;
  dchild_t* ch = (dchild_t*)malloc(sizeof(dchild_t) * ch_cap);
  const size_t N = (size_t)n_hits;
  const double ns = (double)bp->nsigma, sr = (double)bp->win_sig_rphi, sw = (double)bp->win_sig_z;

  for (int li = 0; li < n_list; ++li) {
    int i = seed_list ? seed_list[li] : li;
    double mc2 = INFINITY, mwin = INFINITY, mgeo = INFINITY;
    int seed_status = 0, have_fin = 0, qi = q[i], n_act = 1;
    dcand_t fin;
    memset(&act[0], 0, sizeof(dcand_t));
    double u[21];
    for (int c = 0; c < 6; ++c) act[0].X[c] = (double)seed_par[(size_t)c * ld + i];
    for (int c = 0; c < 21; ++c) u[c] = (double)seed_cov[(size_t)c * ld + i];
    sym_from_upper(u, act[0].P);
    for (int l = 0; l < 32; ++l) act[0].hits[l] = -1;
    act[0].layer = F - 1;
    if (!all_finite(act[0].X, 6) || !all_finite(act[0].P, 36)) {
      act[0].status = ORC_TRK_NONFINITE;
      n_act = 0;
      fin = act[0];
      have_fin = 1;
    }
    while (n_act > 0) {
      size_t nch = 0;
      int n_stop = 0;
      for (int a = 0; a < n_act; ++a) {
        dcand_t* c = &act[a];
        double Xa[6], Pa[36];
        const int l = next_layer(d, c->layer, c->X, qi, c->P, Xa, Pa, &mgeo, &mwin);
        if (l < 0) { stopped[n_stop++] = a; continue; }
        const int kind = d->kind[l];
        const double dm = (double)d->dmod[l];
        /* window on the average surface */
        double ra = sqrt(Xa[0] * Xa[0] + Xa[1] * Xa[1]);
        double tx = -Xa[1] / ra, ty = Xa[0] / ra, nx = Xa[0] / ra, ny = Xa[1] / ra;
        double Stt = tx * tx * Pa[0] + 2.0 * tx * ty * Pa[1] + ty * ty * Pa[7] + sr * sr;
        double Sww, slope_w, slope_phi;
        double pr = nx * Xa[3] + ny * Xa[4], pphi = tx * Xa[3] + ty * Xa[4]; /* radial, azimuthal momentum */
        if (kind == ORC_DISK) {
          Sww = nx * nx * Pa[0] + 2.0 * nx * ny * Pa[1] + ny * ny * Pa[7] + sw * sw;
          slope_w = pr / Xa[5];           /* dr/dz */
          slope_phi = pphi / (ra * Xa[5]); /* dphi/dz */
        } else {
          Sww = Pa[14] + sw * sw;
          slope_w = Xa[5] / pr;           /* dz/dr */
          slope_phi = pphi / (ra * pr);   /* dphi/dr */
        }
        double dphi_w = ns * sqrt(Stt) / ra, dw_w = ns * sqrt(Sww);
        if (dm > 0.0) { dphi_w += dm * fabs(slope_phi); dw_w += dm * fabs(slope_w); }
        double php = atan2(Xa[1], Xa[0]), wp = kind == ORC_DISK ? ra : Xa[2];
        int n_own = 0;
        for (int k = lay_off[l]; k < lay_off[l + 1]; ++k) {
          int hi = lay_idx[k];
          double hit[9] = {(double)xyz[hi], (double)xyz[N + hi], (double)xyz[2 * N + hi]};
          for (int cc = 0; cc < 6; ++cc) hit[3 + cc] = (double)cov[(size_t)cc * N + hi];
          double dph = wrap_pi(atan2(hit[1], hit[0]) - php);
          double dw = (kind == ORC_DISK ? sqrt(hit[0] * hit[0] + hit[1] * hit[1]) : hit[2]) - wp;
          double aph = fabs(dph), aw = fabs(dw);
          int pph = aph <= dphi_w, pw = aw <= dw_w;
          double mph = ra * fabs(aph - dphi_w), mw = fabs(aw - dw_w);
          double dmrg = (pph && pw) ? minf(mph, mw) : (!pph && !pw) ? (mph > mw ? mph : mw) : (!pph ? mph : mw);
          mwin = minf(mwin, dmrg);
          if (!(pph && pw)) continue;
          /* step 2: to the hit's surface, scattering there, update */
          double Xh[6], Ph[36], Xu[6], Pu[36], c2, disc = INFINITY;
          int rc = orc_step_surf(d, kind, hit_surface(kind, hit), 1, 1, Xa, qi, Pa, Xh, Ph, &disc);
          if (isfinite(disc)) mgeo = minf(mgeo, disc);
          if (rc) continue;
          if (update_kind(kind, Xh, Ph, hit, Xu, Pu, &c2)) continue;
          mc2 = minf(mc2, fabs(c2 - (double)bp->chi2_cut));
          if (!(c2 < (double)bp->chi2_cut)) continue;
          if (nch == ch_cap) { ch_cap *= 2; ch = (dchild_t*)realloc(ch, sizeof(dchild_t) * ch_cap); }
          dchild_t* e = &ch[nch++];
          e->nhits = c->nhits + 1; e->parent = a; e->hit = hi; e->holes = c->holes; e->layer = l;
          e->chi2 = c->chi2 + c2;
          memcpy(e->X, Xu, sizeof(Xu)); memcpy(e->P, Pu, sizeof(Pu));
          ++n_own;
        }
        if (c->holes < bp->max_holes) {
          /* hole: the layer's scattering at the average surface */
          double Q[36];
          if (nch == ch_cap) { ch_cap *= 2; ch = (dchild_t*)realloc(ch, sizeof(dchild_t) * ch_cap); }
          dchild_t* e = &ch[nch++];
          e->nhits = c->nhits; e->parent = a; e->hit = -1; e->holes = c->holes + 1; e->layer = l;
          e->chi2 = c->chi2;
          orc_ms_cov_surf(Xa, kind, (double)d->x_over_x0, (double)d->mass, Q);
          memcpy(e->X, Xa, sizeof(Xa));
          for (int m = 0; m < 36; ++m) e->P[m] = Pa[m] + Q[m];
          ++n_own;
        }
        if (n_own == 0) stopped[n_stop++] = a;
      }
      for (int s = 0; s < n_stop; ++s) {
        dcand_t* c = &act[stopped[s]];
        if (!have_fin) { fin = *c; have_fin = 1; continue; }
        if (c->nhits == fin.nhits) mc2 = minf(mc2, fabs(c->chi2 - fin.chi2));
        if (better(c->nhits, c->chi2, fin.nhits, fin.chi2)) fin = *c;
      }
      qsort(ch, nch, sizeof(dchild_t), dchild_cmp);
      size_t keep = nch < (size_t)cap ? nch : (size_t)cap;
      if (nch > (size_t)cap) {
        seed_status |= ORC_TRK_CAP_TRUNC;
        if (ch[cap - 1].nhits == ch[cap].nhits) mc2 = minf(mc2, fabs(ch[cap].chi2 - ch[cap - 1].chi2));
      }
      for (size_t k = 0; k < keep; ++k) {
        dcand_t* e = &nxt[k];
        const dcand_t* p = &act[ch[k].parent];
        memcpy(e->hits, p->hits, sizeof(e->hits));
        e->hits[ch[k].layer] = ch[k].hit;
        e->visit = p->visit | (1u << ch[k].layer);
        e->layer = ch[k].layer;
        memcpy(e->X, ch[k].X, sizeof(e->X)); memcpy(e->P, ch[k].P, sizeof(e->P));
        e->nhits = ch[k].nhits; e->holes = ch[k].holes; e->chi2 = ch[k].chi2; e->status = 0;
      }
      dcand_t* t = act; act = nxt; nxt = t;
      n_act = (int)keep;
    }
    /* every candidate has finished: the result is the record */
    const dcand_t* best = have_fin ? &fin : NULL;
    double ub[21];
    for (int l = F; l < L; ++l) out_hits[(size_t)(l - F) * ld + li] = best ? best->hits[l] : -1;
    if (best) {
      upper_from_sym(best->P, ub);
      for (int c = 0; c < 6; ++c) out_par[(size_t)c * ld + li] = best->X[c];
      for (int c = 0; c < 21; ++c) out_cov[(size_t)c * ld + li] = ub[c];
    }
    out_visit[li] = best ? best->visit : 0u;
    out_chi2[li] = best ? best->chi2 : 0.0;
    out_nhits[li] = best ? best->nhits : 0;
    out_status[li] = (best ? best->status : 0) | seed_status;
    if (out_margin) {
      out_margin[li] = mc2;
      out_margin[(size_t)ld + li] = mwin;
      out_margin[2 * (size_t)ld + li] = mgeo;
      out_margin[3 * (size_t)ld + li] = INFINITY;
      out_margin[4 * (size_t)ld + li] = INFINITY;
    }
  }
  free(act); free(nxt); free(ch); free(stopped); free(lay_cnt); free(lay_off); free(lay_idx);
  return 0;
}
