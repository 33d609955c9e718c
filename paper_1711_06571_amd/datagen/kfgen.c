/*
 * kfgen — seeded synthetic events for barrel Kalman-filter tracking.
 *
 * This is the detector simulation that stands in for the paper's toy
 * particle gun (section 3: ideal barrel, uniform longitudinal field,
 * Gaussian-smeared hits, flat pT in [0.5, 10] GeV, no correlations or
 * decays) and for its realistic events (section 4.2).  It is input
 * generation only: it holds none of the reconstruction arithmetic (no
 * Jacobian, no covariance transport, no Kalman update) and shares no code
 * with the oracle or with the GPU library.  Both consume its output.
 *
 * Physics of the simulation (FP64 throughout):
 *   - a charged particle moves on a helix in B = bz * zhat; the crossing
 *     with each barrel cylinder is found from the circle phase angle;
 *   - at every crossing the hit is recorded first, then the momentum
 *     direction receives a multiple-scattering kick (PDG Highland width,
 *     two independent projected angles, |p| kept);
 *   - the hit lies exactly on the cylinder; it is smeared in r*phi and z.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) keyed by
 * SplitMix64(seed ^ event); the counter names the draw (track or hit,
 * purpose, attempt, block), so generation is deterministic and can run in
 * parallel over tracks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KFG_KAPPA 0.299792458e-2 /* GeV / (T cm): pT = KFG_KAPPA * B * rho */
#define KFG_TWO_PI 6.283185307179586476925286766559

typedef struct {
  int32_t n_layers;
  int32_t smear;   /* 0: hits exactly at the crossing */
  double r[32];    /* layer radii, cm */
  double z_half;   /* barrel half length, cm */
  double bz;       /* tesla */
  double x_over_x0;/* material per layer at normal incidence */
  double mass;     /* GeV, used for beta in the Highland width */
  double sig_rphi; /* cm */
  double sig_z;    /* cm */
  double pt_min, pt_max; /* GeV */
  double eta_max;
  double vtx_sxy, vtx_sz; /* cm */
  double noise_lo, noise_hi; /* noise fraction per layer: U[lo,hi] (lo==hi: fixed) */
  uint64_t seed;
} kfg_config;

/* ---------------------------------------------------------------- RNG */

uint64_t kfg_splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

void kfg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct { uint32_t key[2]; } kfg_key;

static kfg_key make_key(uint64_t seed, uint64_t event) {
  uint64_t k = kfg_splitmix64(seed ^ kfg_splitmix64(event));
  kfg_key r; r.key[0] = (uint32_t)k; r.key[1] = (uint32_t)(k >> 32);
  return r;
}

/* two uniforms in [0,1) from one Philox block */
static void uniform2(const kfg_key* k, uint32_t a, uint32_t b, uint32_t c, uint32_t d, double u[2]) {
  uint32_t ctr[4] = {a, b, c, d}, o[4];
  kfg_philox4x32_10(ctr, k->key, o);
  uint64_t w0 = ((uint64_t)o[0] << 32 | o[1]) >> 11;
  uint64_t w1 = ((uint64_t)o[2] << 32 | o[3]) >> 11;
  u[0] = (double)w0 * (1.0 / 9007199254740992.0);
  u[1] = (double)w1 * (1.0 / 9007199254740992.0);
}

/* two independent standard normals (Box-Muller) */
static void normal2(const kfg_key* k, uint32_t a, uint32_t b, uint32_t c, uint32_t d, double g[2]) {
  double u[2];
  uniform2(k, a, b, c, d, u);
  double rad = sqrt(-2.0 * log(1.0 - u[0])); /* 1-u in (0,1] */
  g[0] = rad * cos(KFG_TWO_PI * u[1]);
  g[1] = rad * sin(KFG_TWO_PI * u[1]);
}

/* purpose codes in counter word 1 */
#define P_KIN     0x00000001u
#define P_LAYER   0x00000100u /* + layer */
#define P_NOISE   0x00010000u /* + layer */
#define P_SHUFFLE 0x00020000u /* + layer */
#define P_NFRAC   0x00030000u /* + layer */
#define P_NTRK    0x00040000u

/* ------------------------------------------------------- simulation */

typedef struct { double x, y, z, px, py, pz; } particle;

/* Helix crossing with the cylinder of radius R, via the phase angle of the
 * point on the transverse circle.  Returns 0 and moves the particle on
 * success; returns 1 if the circle never reaches R.  The start is strictly
 * inside R, so the first crossing along the motion is the exit. */
static int move_to_radius(particle* pa, int q, double bz, double R) {
  double pt = hypot(pa->px, pa->py);
  double omega = -(double)q * KFG_KAPPA * bz / pt; /* d(phase)/d(transverse path) */
  double rho = 1.0 / fabs(omega);
  /* centre: to the left of the motion for omega > 0 */
  double cx = pa->x - pa->py / (pt * omega);
  double cy = pa->y + pa->px / (pt * omega);
  double dc = hypot(cx, cy);
  double c = (R * R - dc * dc - rho * rho) / (2.0 * rho * dc);
  if (!(c >= -1.0 && c <= 1.0)) return 1;
  double gam = atan2(cy, cx);
  double th0 = atan2(pa->y - cy, pa->x - cx);
  double acs = acos(c);
  double best = INFINITY;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    double th = gam + sgn * acs;
    double dth = remainder(th - th0, KFG_TWO_PI); /* (-pi, pi] */
    if (omega > 0 && dth <= 0) dth += KFG_TWO_PI;
    if (omega < 0 && dth >= 0) dth -= KFG_TWO_PI;
    double s = dth / omega;
    if (s < best) best = s;
  }
  double th = th0 + omega * best;
  double a = omega * best; /* rotation of the momentum */
  double ca = cos(a), sa = sin(a);
  double npx = pa->px * ca - pa->py * sa;
  double npy = pa->py * ca + pa->px * sa;
  pa->x = cx + rho * cos(th);
  pa->y = cy + rho * sin(th);
  pa->z = pa->z + pa->pz * best / pt;
  pa->px = npx;
  pa->py = npy;
  return 0;
}

/* Highland projected-angle width for a unit-charge particle crossing a thin
 * cylinder with material x/X0 at normal incidence. */
static double highland_theta0(const particle* pa, double x0, double mass) {
  double p2 = pa->px * pa->px + pa->py * pa->py + pa->pz * pa->pz;
  double p = sqrt(p2);
  double r = hypot(pa->x, pa->y);
  double cospsi = fabs((pa->x * pa->px + pa->y * pa->py) / (r * p));
  double xe = x0 / cospsi;
  double beta = p / sqrt(p2 + mass * mass);
  return 0.0136 / (beta * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / (beta * beta)));
}

static void scatter(particle* pa, double th1, double th2) {
  double p = sqrt(pa->px * pa->px + pa->py * pa->py + pa->pz * pa->pz);
  double ux = pa->px / p, uy = pa->py / p, uz = pa->pz / p;
  /* e1 = zhat x u (normalised), e2 = u x e1 */
  double e1x = -uy, e1y = ux, e1z = 0.0;
  double n1 = hypot(e1x, e1y);
  e1x /= n1; e1y /= n1;
  double e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
  double t1 = tan(th1), t2 = tan(th2);
  double vx = ux + t1 * e1x + t2 * e2x, vy = uy + t1 * e1y + t2 * e2y, vz = uz + t1 * e1z + t2 * e2z;
  double nv = sqrt(vx * vx + vy * vy + vz * vz);
  pa->px = p * vx / nv;
  pa->py = p * vy / nv;
  pa->pz = p * vz / nv;
}

static void hit_cov(double phi, double srphi, double sz, double cov[6]) {
  double tx = -sin(phi), ty = cos(phi);
  double a = srphi * srphi, b = sz * sz;
  cov[0] = a * tx * tx; /* xx */
  cov[1] = a * tx * ty; /* xy */
  cov[2] = 0.0;         /* xz */
  cov[3] = a * ty * ty; /* yy */
  cov[4] = 0.0;         /* yz */
  cov[5] = b;           /* zz */
}

/* ------------------------------------------------------------ API */

/* Tracks per event drawn log-uniformly in [lo, hi] (floor), keyed by event. */
int32_t kfg_event_tracks(uint64_t seed, uint64_t event, int32_t lo, int32_t hi) {
  kfg_key k = make_key(seed, 0xA5A5A5A5ull ^ event);
  double u[2];
  uniform2(&k, 0, P_NTRK, 0, 0, u);
  double v = exp(log((double)lo) + u[0] * (log((double)hi) - log((double)lo)));
  int32_t n = (int32_t)floor(v);
  if (n < lo) n = lo;
  if (n > hi) n = hi;
  return n;
}

static double noise_fraction(const kfg_config* cfg, const kfg_key* k, int layer) {
  if (!(cfg->noise_hi > cfg->noise_lo)) return cfg->noise_lo;
  double u[2];
  uniform2(k, 0, P_NFRAC + (uint32_t)layer, 0, 0, u);
  return cfg->noise_lo + u[0] * (cfg->noise_hi - cfg->noise_lo);
}

/* Hits on each layer: n_tracks true hits plus round(f * n_tracks) noise. */
int kfg_layer_counts(const kfg_config* cfg, uint64_t event, int32_t n_tracks, int64_t* counts) {
  if (cfg->n_layers < 1 || cfg->n_layers > 32 || n_tracks < 0) return 1;
  kfg_key k = make_key(cfg->seed, event);
  for (int l = 0; l < cfg->n_layers; ++l) {
    double f = noise_fraction(cfg, &k, l);
    counts[l] = (int64_t)n_tracks + (int64_t)llround(f * (double)n_tracks);
  }
  return 0;
}

/*
 * Generate one event.  Hits are stored layer by layer (all hits of layer 0,
 * then layer 1, ...), shuffled within each layer; a hit's position in these
 * arrays is its event-local original index.
 *   hx, hy, hz [n_hits], hcov [6][n_hits] (xx,xy,xz,yy,yz,zz),
 *   hlayer [n_hits], htrack [n_hits] (-1 for noise),
 *   trk_hits [L][n_tracks] original index of track t's hit on layer l,
 *   trk_q [n_tracks], truth [L][6][n_tracks] state leaving each layer
 *   (after the scattering kick) or NULL, vtx [6][n_tracks] production
 *   state or NULL, attempts [n_tracks] or NULL.
 * Tracks that fail to reach a layer or leave |z| < z_half are regenerated.
 */
int kfg_event(const kfg_config* cfg, uint64_t event, int32_t n_tracks,
              double* hx, double* hy, double* hz, double* hcov, int32_t* hlayer, int32_t* htrack,
              int32_t* trk_hits, int8_t* trk_q, double* truth, double* vtx, int32_t* attempts,
              int64_t n_hits_cap) {
  const int L = cfg->n_layers;
  if (L < 1 || L > 32 || n_tracks < 0) return 1;
  int64_t counts[32], base[33];
  kfg_layer_counts(cfg, event, n_tracks, counts);
  base[0] = 0;
  for (int l = 0; l < L; ++l) base[l + 1] = base[l] + counts[l];
  if (base[L] > n_hits_cap) return 2;
  const int64_t nh = base[L];
  kfg_key key = make_key(cfg->seed, event);
  int failed = 0;

  /* true tracks: pre-shuffle slot of track t on layer l is base[l] + t */
#pragma omp parallel for schedule(dynamic, 256) reduction(+:failed)
  for (int32_t t = 0; t < n_tracks; ++t) {
    int ok = 0;
    for (uint32_t att = 0; att < 1000 && !ok; ++att) {
      double u[2], v[2], g[2], g2[2];
      uniform2(&key, (uint32_t)t, P_KIN, att, 0, u);
      uniform2(&key, (uint32_t)t, P_KIN, att, 1, v);
      normal2(&key, (uint32_t)t, P_KIN, att, 2, g);
      normal2(&key, (uint32_t)t, P_KIN, att, 3, g2);
      int q = u[0] < 0.5 ? 1 : -1;
      double pt = cfg->pt_min + u[1] * (cfg->pt_max - cfg->pt_min);
      double phi0 = KFG_TWO_PI * v[0];
      double eta = -cfg->eta_max + 2.0 * cfg->eta_max * v[1];
      particle pa;
      pa.x = cfg->vtx_sxy * g[0];
      pa.y = cfg->vtx_sxy * g[1];
      pa.z = cfg->vtx_sz * g2[0];
      pa.px = pt * cos(phi0);
      pa.py = pt * sin(phi0);
      pa.pz = pt * sinh(eta);
      particle start = pa;
      int good = 1;
      for (int l = 0; l < L && good; ++l) {
        if (move_to_radius(&pa, q, cfg->bz, cfg->r[l]) || fabs(pa.z) > cfg->z_half) { good = 0; break; }
        double R = cfg->r[l];
        double phit = atan2(pa.y, pa.x);
        double gs[2], gm[2];
        normal2(&key, (uint32_t)t, P_LAYER + (uint32_t)l, att, 0, gs);
        normal2(&key, (uint32_t)t, P_LAYER + (uint32_t)l, att, 1, gm);
        double phih = cfg->smear ? phit + cfg->sig_rphi * gs[0] / R : phit;
        double zh = cfg->smear ? pa.z + cfg->sig_z * gs[1] : pa.z;
        int64_t slot = base[l] + t;
        hx[slot] = cfg->smear ? R * cos(phih) : pa.x;
        hy[slot] = cfg->smear ? R * sin(phih) : pa.y;
        hz[slot] = zh;
        double cv[6];
        hit_cov(phih, cfg->sig_rphi, cfg->sig_z, cv);
        for (int c = 0; c < 6; ++c) hcov[(int64_t)c * n_hits_cap + slot] = cv[c];
        hlayer[slot] = l;
        htrack[slot] = t;
        if (cfg->x_over_x0 > 0) {
          double th0 = highland_theta0(&pa, cfg->x_over_x0, cfg->mass);
          scatter(&pa, th0 * gm[0], th0 * gm[1]);
        }
        if (truth) {
          double st[6] = {pa.x, pa.y, pa.z, pa.px, pa.py, pa.pz};
          for (int c = 0; c < 6; ++c) truth[((int64_t)l * 6 + c) * n_tracks + t] = st[c];
        }
      }
      if (good) {
        ok = 1;
        trk_q[t] = (int8_t)q;
        if (vtx) {
          double st[6] = {start.x, start.y, start.z, start.px, start.py, start.pz};
          for (int c = 0; c < 6; ++c) vtx[(int64_t)c * n_tracks + t] = st[c];
        }
        if (attempts) attempts[t] = (int32_t)att + 1;
      }
    }
    if (!ok) failed += 1;
  }
  if (failed) return 3;

  /* noise hits: uniform in phi and z, same covariance model */
  for (int l = 0; l < L; ++l) {
    int64_t nn = counts[l] - n_tracks;
    double R = cfg->r[l];
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nn; ++j) {
      double u[2];
      uniform2(&key, (uint32_t)j, P_NOISE + (uint32_t)l, (uint32_t)(j >> 32), 0, u);
      double phi = KFG_TWO_PI * u[0];
      double z = -cfg->z_half + 2.0 * cfg->z_half * u[1];
      int64_t slot = base[l] + n_tracks + j;
      hx[slot] = R * cos(phi);
      hy[slot] = R * sin(phi);
      hz[slot] = z;
      double cv[6];
      hit_cov(phi, cfg->sig_rphi, cfg->sig_z, cv);
      for (int c = 0; c < 6; ++c) hcov[(int64_t)c * n_hits_cap + slot] = cv[c];
      hlayer[slot] = l;
      htrack[slot] = -1;
    }
  }

  /* keyed Fisher-Yates shuffle within each layer; perm maps new -> old */
  int64_t maxc = 0;
  for (int l = 0; l < L; ++l) if (counts[l] > maxc) maxc = counts[l];
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxc > 0 ? maxc : 1));
  int64_t* inv = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxc > 0 ? maxc : 1));
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(maxc > 0 ? maxc : 1));
  int32_t* itmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxc > 0 ? maxc : 1));
  if (!perm || !inv || !tmp || !itmp) { free(perm); free(inv); free(tmp); free(itmp); return 4; }
  for (int l = 0; l < L; ++l) {
    int64_t n = counts[l], b = base[l];
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = n - 1; i > 0; --i) {
      double u[2];
      uniform2(&key, (uint32_t)i, P_SHUFFLE + (uint32_t)l, (uint32_t)(i >> 32), 0, u);
      int64_t j = (int64_t)floor(u[0] * (double)(i + 1));
      if (j > i) j = i;
      int64_t s = perm[i]; perm[i] = perm[j]; perm[j] = s;
    }
    for (int64_t i = 0; i < n; ++i) inv[perm[i]] = i;
    double* darr[3] = {hx, hy, hz};
    for (int a = 0; a < 3; ++a) {
      for (int64_t i = 0; i < n; ++i) tmp[i] = darr[a][b + perm[i]];
      memcpy(darr[a] + b, tmp, sizeof(double) * (size_t)n);
    }
    for (int c = 0; c < 6; ++c) {
      double* col = hcov + (int64_t)c * n_hits_cap + b;
      for (int64_t i = 0; i < n; ++i) tmp[i] = col[perm[i]];
      memcpy(col, tmp, sizeof(double) * (size_t)n);
    }
    for (int64_t i = 0; i < n; ++i) itmp[i] = htrack[b + perm[i]];
    memcpy(htrack + b, itmp, sizeof(int32_t) * (size_t)n);
    for (int32_t t = 0; t < n_tracks; ++t) trk_hits[(int64_t)l * n_tracks + t] = (int32_t)(b + inv[t]);
  }
  free(perm); free(inv); free(tmp); free(itmp);
  return 0;
}

/* ===================================================================
 * General detector (section 4.1's "cylinder with lids"): barrel cylinders
 * and endcap disks, listed in the order a track from the origin meets them
 * (barrel layers outwards, then the disks of each side outwards).  Each
 * layer is divided into n_mod phi sectors (modules); module k sits at the
 * layer's average surface + dmod (k even) or - dmod (k odd): radius on a
 * barrel layer, z on a disk.  A track crosses, in index order, every layer
 * whose average surface it reaches ahead of it inside the layer's extent
 * (barrel: z in [lo, hi]; disk: r in [lo, hi], reached within half a turn
 * while still moving outwards); its hit lies on the module at the phi of
 * that crossing.  Barrel hits are smeared
 * along the arc and in z, disk hits along the arc and in r.
 * =================================================================== */

#define KFG_BARREL 0
#define KFG_DISK 1

typedef struct {
  int32_t n_layers;
  int32_t smear;
  int32_t kind[32];
  double pos[32];  /* average radius (barrel) or z of the average plane (disk) */
  double lo[32];   /* extent: z range (barrel), r range (disk) */
  double hi[32];
  double dmod[32]; /* module offset from the average surface */
  int32_t n_mod;   /* modules (phi sectors) per layer */
  int32_t n_seed_layers; /* a track must cross layers 0 .. n_seed_layers - 1 */
  double bz, x_over_x0, mass;
  double sig_rphi; /* along the arc, cm */
  double sig_w;    /* along z (barrel) or r (disk), cm */
  double pt_min, pt_max, eta_max, vtx_sxy, vtx_sz;
  double noise_lo, noise_hi; /* noise hits per layer: U[lo,hi] times the layer's true hits */
  uint64_t seed;
} kfg_det_config;

/* Helix to the plane z = Z ahead of the particle; 1 if it lies behind or
 * the motion is parallel to it. */
static int move_to_z(particle* pa, int q, double bz, double Z) {
  double pt = hypot(pa->px, pa->py);
  if (pa->pz == 0.0) return 1;
  double s = (Z - pa->z) * pt / pa->pz;
  if (!(s > 0.0)) return 1;
  double omega = -(double)q * KFG_KAPPA * bz / pt;
  double cx = pa->x - pa->py / (pt * omega);
  double cy = pa->y + pa->px / (pt * omega);
  double a = omega * s;
  double th0 = atan2(pa->y - cy, pa->x - cx);
  double rho = 1.0 / fabs(omega);
  double ca = cos(a), sa = sin(a);
  double npx = pa->px * ca - pa->py * sa;
  double npy = pa->py * ca + pa->px * sa;
  pa->x = cx + rho * cos(th0 + a);
  pa->y = cy + rho * sin(th0 + a);
  pa->z = Z;
  pa->px = npx;
  pa->py = npy;
  return 0;
}

/* Highland width with the incidence measured from the layer's normal. */
static double highland_theta0_kind(const particle* pa, int kind, double x0, double mass) {
  double p2 = pa->px * pa->px + pa->py * pa->py + pa->pz * pa->pz;
  double p = sqrt(p2);
  double cospsi;
  if (kind == KFG_DISK) cospsi = fabs(pa->pz / p);
  else cospsi = fabs((pa->x * pa->px + pa->y * pa->py) / (hypot(pa->x, pa->y) * p));
  double xe = x0 / cospsi;
  double beta = p / sqrt(p2 + mass * mass);
  return 0.0136 / (beta * p) * sqrt(xe) * (1.0 + 0.038 * log(xe / (beta * beta)));
}

static double module_surface(const kfg_det_config* cfg, int l, double phi) {
  double ph = phi < 0.0 ? phi + KFG_TWO_PI : phi;
  int k = (int)floor(ph * (double)cfg->n_mod / KFG_TWO_PI);
  if (k >= cfg->n_mod) k = cfg->n_mod - 1;
  if (k < 0) k = 0;
  return cfg->pos[l] + ((k & 1) ? -cfg->dmod[l] : cfg->dmod[l]);
}

/* covariance of a disk hit: sig_rphi along the arc, sig_r along r, exact z */
static void disk_hit_cov(double phi, double srphi, double sr, double cov[6]) {
  double tx = -sin(phi), ty = cos(phi), rx = cos(phi), ry = sin(phi);
  double a = srphi * srphi, b = sr * sr;
  cov[0] = a * tx * tx + b * rx * rx;
  cov[1] = a * tx * ty + b * rx * ry;
  cov[2] = 0.0;
  cov[3] = a * ty * ty + b * ry * ry;
  cov[4] = 0.0;
  cov[5] = 0.0;
}

/* One track through the detector: returns 1 if it misses a seed layer.
 * hit[l][9] and crossed[l] per layer, truth[l][6] after the kick. */
static int det_track(const kfg_det_config* cfg, const kfg_key* key, int32_t t, uint32_t att, int* q_out,
                     particle* start, double hit[][9], int crossed[], double truthl[][6]) {
  const int L = cfg->n_layers;
  double u[2], v[2], g[2], g2[2];
  uniform2(key, (uint32_t)t, P_KIN, att, 0, u);
  uniform2(key, (uint32_t)t, P_KIN, att, 1, v);
  normal2(key, (uint32_t)t, P_KIN, att, 2, g);
  normal2(key, (uint32_t)t, P_KIN, att, 3, g2);
  int q = u[0] < 0.5 ? 1 : -1;
  double pt = cfg->pt_min + u[1] * (cfg->pt_max - cfg->pt_min);
  double phi0 = KFG_TWO_PI * v[0];
  double eta = -cfg->eta_max + 2.0 * cfg->eta_max * v[1];
  particle pa;
  pa.x = cfg->vtx_sxy * g[0];
  pa.y = cfg->vtx_sxy * g[1];
  pa.z = cfg->vtx_sz * g2[0];
  pa.px = pt * cos(phi0);
  pa.py = pt * sin(phi0);
  pa.pz = pt * sinh(eta);
  *start = pa;
  *q_out = q;
  for (int l = 0; l < L; ++l) {
    crossed[l] = 0;
    const int kind = cfg->kind[l];
    particle av = pa, pm = pa;
    /* the layer is crossed where the average surface is: inside the extent
       and, on a disk, within half a turn while still moving outwards (a
       looper coming back is not followed) */
    int miss = kind == KFG_DISK ? move_to_z(&av, q, cfg->bz, cfg->pos[l])
                                : move_to_radius(&av, q, cfg->bz, cfg->pos[l]);
    if (!miss) {
      double w = kind == KFG_DISK ? hypot(av.x, av.y) : av.z;
      miss = !(w >= cfg->lo[l] && w <= cfg->hi[l]);
      if (kind == KFG_DISK) {
        double turn = fabs(KFG_KAPPA * cfg->bz * (av.z - pa.z) / pa.pz);
        if (!(av.x * av.px + av.y * av.py > 0.0) || !(turn < 3.14159265358979323846)) miss = 1;
      }
    }
    /* the hit: on the module at the phi of that crossing */
    if (!miss) {
      double surf = module_surface(cfg, l, atan2(av.y, av.x));
      miss = kind == KFG_DISK ? move_to_z(&pm, q, cfg->bz, surf) : move_to_radius(&pm, q, cfg->bz, surf);
    }
    if (miss) {
      if (l < cfg->n_seed_layers) return 1;
      continue;
    }
    pa = pm;
    double gs[2], gm[2];
    normal2(key, (uint32_t)t, P_LAYER + (uint32_t)l, att, 0, gs);
    normal2(key, (uint32_t)t, P_LAYER + (uint32_t)l, att, 1, gm);
    double phit = atan2(pa.y, pa.x), r = hypot(pa.x, pa.y);
    double cv[6];
    if (kind == KFG_DISK) {
      double rh = cfg->smear ? r + cfg->sig_w * gs[1] : r;
      double phih = cfg->smear ? phit + cfg->sig_rphi * gs[0] / r : phit;
      hit[l][0] = cfg->smear ? rh * cos(phih) : pa.x;
      hit[l][1] = cfg->smear ? rh * sin(phih) : pa.y;
      hit[l][2] = pa.z;
      disk_hit_cov(phih, cfg->sig_rphi, cfg->sig_w, cv);
    } else {
      double phih = cfg->smear ? phit + cfg->sig_rphi * gs[0] / r : phit;
      hit[l][0] = cfg->smear ? r * cos(phih) : pa.x;
      hit[l][1] = cfg->smear ? r * sin(phih) : pa.y;
      hit[l][2] = cfg->smear ? pa.z + cfg->sig_w * gs[1] : pa.z;
      hit_cov(phih, cfg->sig_rphi, cfg->sig_w, cv);
    }
    for (int c = 0; c < 6; ++c) hit[l][3 + c] = cv[c];
    crossed[l] = 1;
    if (cfg->x_over_x0 > 0) {
      double th0 = highland_theta0_kind(&pa, kind, cfg->x_over_x0, cfg->mass);
      scatter(&pa, th0 * gm[0], th0 * gm[1]);
    }
    truthl[l][0] = pa.x; truthl[l][1] = pa.y; truthl[l][2] = pa.z;
    truthl[l][3] = pa.px; truthl[l][4] = pa.py; truthl[l][5] = pa.pz;
  }
  return 0;
}

/*
 * Generate one event over a general detector.  Hits are grouped by layer and
 * shuffled within each layer; a hit's position is its original index.
 * Arrays are sized by the caller for n_hits_cap hits; *n_hits receives the
 * count.  trk_hits [L][n_tracks] (-1 where the track does not cross the
 * layer), truth [L][6][n_tracks] (NaN where not crossed) or NULL, vtx
 * [6][n_tracks] or NULL.  Returns 2 if the capacity is too small, 3 if a
 * track could not be generated.
 */
int kfg_det_event(const kfg_det_config* cfg, uint64_t event, int32_t n_tracks, double* hx, double* hy, double* hz,
                  double* hcov, int32_t* hlayer, int32_t* htrack, int32_t* trk_hits, int8_t* trk_q, double* truth,
                  double* vtx, int64_t n_hits_cap, int64_t* n_hits) {
  const int L = cfg->n_layers;
  if (L < 1 || L > 32 || n_tracks < 0 || cfg->n_mod < 1 || cfg->n_seed_layers > L) return 1;
  kfg_key key = make_key(cfg->seed, event);
  double* th = (double*)malloc(sizeof(double) * 9 * (size_t)L * (size_t)(n_tracks > 0 ? n_tracks : 1));
  int* cr = (int*)malloc(sizeof(int) * (size_t)L * (size_t)(n_tracks > 0 ? n_tracks : 1));
  if (!th || !cr) { free(th); free(cr); return 4; }
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+:failed)
  for (int32_t t = 0; t < n_tracks; ++t) {
    double hit[32][9], tr[32][6];
    int crossed[32], q = 1, ok = 0;
    particle st;
    for (uint32_t att = 0; att < 1000 && !ok; ++att) ok = !det_track(cfg, &key, t, att, &q, &st, hit, crossed, tr);
    if (!ok) { failed += 1; continue; }
    trk_q[t] = (int8_t)q;
    for (int l = 0; l < L; ++l) {
      cr[(size_t)l * n_tracks + t] = crossed[l];
      for (int c = 0; c < 9; ++c) th[((size_t)l * n_tracks + t) * 9 + c] = hit[l][c];
      if (truth)
        for (int c = 0; c < 6; ++c) truth[((int64_t)l * 6 + c) * n_tracks + t] = crossed[l] ? tr[l][c] : NAN;
    }
    if (vtx) {
      double s6[6] = {st.x, st.y, st.z, st.px, st.py, st.pz};
      for (int c = 0; c < 6; ++c) vtx[(int64_t)c * n_tracks + t] = s6[c];
    }
  }
  if (failed) { free(th); free(cr); return 3; }
  int64_t ntrue[32], counts[32], base[33];
  base[0] = 0;
  for (int l = 0; l < L; ++l) {
    ntrue[l] = 0;
    for (int32_t t = 0; t < n_tracks; ++t) ntrue[l] += cr[(size_t)l * n_tracks + t];
    double fr = cfg->noise_lo;
    if (cfg->noise_hi > cfg->noise_lo) {
      double uu[2];
      uniform2(&key, 0, P_NFRAC + (uint32_t)l, 0, 0, uu);
      fr = cfg->noise_lo + uu[0] * (cfg->noise_hi - cfg->noise_lo);
    }
    counts[l] = ntrue[l] + (int64_t)llround(fr * (double)ntrue[l]);
    base[l + 1] = base[l] + counts[l];
  }
  *n_hits = base[L];
  if (base[L] > n_hits_cap) { free(th); free(cr); return 2; }
  /* true hits in track order, then noise, per layer */
  for (int l = 0; l < L; ++l) {
    int64_t slot = base[l];
    for (int32_t t = 0; t < n_tracks; ++t) {
      trk_hits[(int64_t)l * n_tracks + t] = -1;
      if (!cr[(size_t)l * n_tracks + t]) continue;
      const double* h = th + ((size_t)l * n_tracks + t) * 9;
      hx[slot] = h[0]; hy[slot] = h[1]; hz[slot] = h[2];
      for (int c = 0; c < 6; ++c) hcov[(int64_t)c * n_hits_cap + slot] = h[3 + c];
      hlayer[slot] = l;
      htrack[slot] = t;
      trk_hits[(int64_t)l * n_tracks + t] = (int32_t)(slot - base[l]); /* pre-shuffle position */
      ++slot;
    }
    for (int64_t j = 0; j < counts[l] - ntrue[l]; ++j, ++slot) {
      double uu[2];
      uniform2(&key, (uint32_t)j, P_NOISE + (uint32_t)l, (uint32_t)(j >> 32), 0, uu);
      double phi = KFG_TWO_PI * uu[0];
      double w = cfg->lo[l] + (cfg->hi[l] - cfg->lo[l]) * uu[1];
      double surf = module_surface(cfg, l, phi);
      double cv[6];
      if (cfg->kind[l] == KFG_DISK) {
        hx[slot] = w * cos(phi); hy[slot] = w * sin(phi); hz[slot] = surf;
        disk_hit_cov(phi, cfg->sig_rphi, cfg->sig_w, cv);
      } else {
        hx[slot] = surf * cos(phi); hy[slot] = surf * sin(phi); hz[slot] = w;
        hit_cov(phi, cfg->sig_rphi, cfg->sig_w, cv);
      }
      for (int c = 0; c < 6; ++c) hcov[(int64_t)c * n_hits_cap + slot] = cv[c];
      hlayer[slot] = l;
      htrack[slot] = -1;
    }
  }
  free(th);
  free(cr);
  /* keyed shuffle within each layer (as kfg_event); perm maps new -> old */
  int64_t maxc = 1;
  for (int l = 0; l < L; ++l) if (counts[l] > maxc) maxc = counts[l];
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)maxc);
  int64_t* inv = (int64_t*)malloc(sizeof(int64_t) * (size_t)maxc);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)maxc);
  int32_t* itmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)maxc);
  if (!perm || !inv || !tmp || !itmp) { free(perm); free(inv); free(tmp); free(itmp); return 4; }
  for (int l = 0; l < L; ++l) {
    int64_t n = counts[l], b = base[l];
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = n - 1; i > 0; --i) {
      double uu[2];
      uniform2(&key, (uint32_t)i, P_SHUFFLE + (uint32_t)l, (uint32_t)(i >> 32), 0, uu);
      int64_t j = (int64_t)floor(uu[0] * (double)(i + 1));
      if (j > i) j = i;
      int64_t sw = perm[i]; perm[i] = perm[j]; perm[j] = sw;
    }
    for (int64_t i = 0; i < n; ++i) inv[perm[i]] = i;
    double* darr[3] = {hx, hy, hz};
    for (int a = 0; a < 3; ++a) {
      for (int64_t i = 0; i < n; ++i) tmp[i] = darr[a][b + perm[i]];
      memcpy(darr[a] + b, tmp, sizeof(double) * (size_t)n);
    }
    for (int c = 0; c < 6; ++c) {
      double* col = hcov + (int64_t)c * n_hits_cap + b;
      for (int64_t i = 0; i < n; ++i) tmp[i] = col[perm[i]];
      memcpy(col, tmp, sizeof(double) * (size_t)n);
    }
    for (int64_t i = 0; i < n; ++i) itmp[i] = htrack[b + perm[i]];
    memcpy(htrack + b, itmp, sizeof(int32_t) * (size_t)n);
    for (int32_t t = 0; t < n_tracks; ++t) {
      int32_t* th_l = trk_hits + (int64_t)l * n_tracks + t;
      if (*th_l >= 0) *th_l = (int32_t)(b + inv[*th_l]);
    }
  }
  free(perm); free(inv); free(tmp); free(itmp);
  return 0;
}
