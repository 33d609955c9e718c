/*
 * kforacle — plain FP64 CPU oracle for Kalman-filter track fitting and
 * combinatorial track building in a barrel of concentric cylinders.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference that the GPU
 * path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Method (Cerati et al., "Parallelized Kalman-Filter-Based Reconstruction
 * of Particle Tracks on Many-Core Architectures"):
 *   - section 2: track building projects a candidate outward layer by layer,
 *     uses the Kalman filter to judge which hits continue it, and branches
 *     into several candidates per seed; fitting reapplies the Kalman filter
 *     over a fixed hit list without branching;
 *   - section 3: ideal barrel, uniform longitudinal field;
 *   - section 4.1: Kalman updates on the plane tangent to the hit radius;
 *   - section 4.3: a fixed number of candidate slots per seed, ranked so the
 *     best candidates are found quickly.
 * Where the paper is silent the readings are recorded beside each function.
 *
 * Conventions: state X = (x, y, z, px, py, pz) in cm and GeV; covariance
 * P is a full 6x6 row-major matrix internally, exchanged as the 21 upper
 * triangle entries in row order (00,01,..,05,11,..,15,22,..,55).  Inputs
 * arrive in FP32 (the values the GPU sees) and are promoted to FP64.
 * Layers are 0-based; layer l has radius geometry.r[l].
 */
#ifndef KFORACLE_H
#define KFORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-track status bits */
#define ORC_TRK_NO_CROSSING 1
#define ORC_TRK_OUT_OF_Z 2
#define ORC_TRK_NONFINITE 4
#define ORC_TRK_S_NOT_PD 8
#define ORC_TRK_CAP_TRUNC 16

typedef struct {
  int32_t n_layers;
  float r[32];
  float z_half;
  float bz;
  float x_over_x0;
  float mass;
} orc_geometry;

typedef struct {
  float chi2_cut;     /* accept a hit iff chi2 < chi2_cut */
  int32_t max_holes;  /* a hole child is added while holes < max_holes */
  int32_t cand_cap;   /* candidates kept per seed */
  float nsigma;       /* window half-width in units of sqrt(S) */
  float win_sig_rphi; /* nominal hit resolution used for the window, cm */
  float win_sig_z;
  int32_t first_layer;/* first layer searched */
  int32_t window_mode;/* 0 plain, 1 learned */
  const double* mlp;  /* learned-window parameters (oracle layout), or NULL */
  int32_t state;      /* 0 Cartesian; 1 hybrid (x, y, z, q/pT, phi, theta) */
} orc_build_params;

/* General detector (section 4.1): barrel cylinders and endcap disks, listed
 * in the order a track from the origin meets them (barrel layers outwards,
 * then the disks of each side outwards).  Modules may sit off a layer's
 * average surface by up to dmod (barrel: radius, disk: z). */
#define ORC_BARREL 0
#define ORC_DISK 1
typedef struct {
  int32_t n_layers;
  int32_t kind[32]; /* ORC_BARREL or ORC_DISK */
  float pos[32];    /* average radius (barrel) or z of the average plane (disk), cm */
  float lo[32];     /* active extent: z range (barrel) or r range (disk), cm */
  float hi[32];
  float dmod[32];   /* largest module offset from the average surface, cm */
  float bz;
  float x_over_x0;
  float mass;
} orc_detector;

/* --- primitives (exposed for the pins) --- */
int orc_propagate(const double X[6], int q, double R, double bz, double Xo[6], double* s_out, double* disc);
void orc_state_at(const double X[6], int q, double bz, double s, double Xo[6]);
void orc_jacobian(const double X[6], int q, double bz, double s, double J[36]);
void orc_ms_cov(const double X[6], double x_over_x0, double mass, double Q[36]);
int orc_update(const double X[6], const double P[36], const double hit[9], double Xo[6], double Po[36],
               double* chi2);
int orc_predict(const orc_geometry* g, int layer, const double X[6], int q, const double P[36], double Xo[6],
                double Po[36], double* disc);
int orc_beam_d0(const double X[6], int q, double bz, double* f, double H[6]);

/* --- batch entry points, SoA layouts with leading dimension ld --- */
int orc_seed(const orc_geometry* g, int n, int ld, const float* hits, double beam_sigma, int8_t* q_out,
             float* seed_par, float* seed_cov, double* seed_par64, double* seed_cov64, int32_t* status);
int orc_seed64(const orc_geometry* g, int n, int ld, const double* hits, double beam_sigma, int8_t* q_out,
               double* seed_par64, double* seed_cov64, int32_t* status);
int orc_fit(const orc_geometry* g, int n, int ld, int first_layer, const float* hits, const uint32_t* hole_mask,
            const float* seed_par, const float* seed_cov, const int8_t* q, double* out_par, double* out_cov,
            double* out_chi2, int32_t* out_ndof, int32_t* out_status);
int orc_fit64(const orc_geometry* g, int n, int ld, int first_layer, const double* hits,
              const double* seed_par, const double* seed_cov, const int8_t* q, double* out_par, double* out_cov,
              double* out_chi2, int32_t* out_ndof, int32_t* out_status);
void orc_hyb_from_cart(const double X[6], int q, double Y[6]);
int orc_cart_from_hyb(const double Y[6], double X[6]);
void orc_hyb_jac_cart_from_hyb(const double Y[6], double A[36]);
void orc_hyb_jac_hyb_from_cart(const double X[6], int q, double B[36]);
int orc_predict_hyb(const orc_geometry* g, int layer, const double Y[6], const double P[36], double Yo[6],
                    double Po[36], double* disc);
int orc_fit_hybrid(const orc_geometry* g, int n, int ld, int first_layer, const float* hits,
                   const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                   double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status);
int orc_fit_hybrid64(const orc_geometry* g, int n, int ld, int first_layer, const double* hits,
                     const double* seed_par, const double* seed_cov, const int8_t* q, double* out_par,
                     double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status);
int orc_hit_bin(const orc_geometry* g, int n_phi, int n_z, int n_hits, const int32_t* layer, const float* xyz,
                int32_t* offsets, int32_t* order, float* phi_sorted);
int orc_build(const orc_geometry* g, const orc_build_params* bp, int n_hits, const int32_t* layer,
              const float* xyz, const float* cov, int n_seeds, int ld, const float* seed_par,
              const float* seed_cov, const int8_t* q, int n_list, const int32_t* seed_list,
              int32_t* out_hits, double* out_par, double* out_cov, double* out_chi2, int32_t* out_nhits,
              int32_t* out_status, double* out_margin);
int orc_mlp_forward(const double* mlp, const double x[27], double w[2]);

/* --- general detector --- */
int orc_cyl_path(const double X[6], int q, double R, double bz, int nearest, double* s_out, double* disc);
int orc_plane_path(const double X[6], double Z, int nearest, double* s_out);
void orc_jacobian_surf(const double X[6], int q, double bz, double s, int kind, double J[36]);
void orc_ms_cov_surf(const double X[6], int kind, double x_over_x0, double mass, double Q[36]);
int orc_step_surf(const orc_detector* d, int kind, double value, int nearest, int material, const double X[6],
                  int q, const double P[36], double Xo[6], double Po[36], double* disc);
int orc_update_disk(const double X[6], const double P[36], const double hit[9], double Xo[6], double Po[36],
                    double* chi2);
int orc_fit_det(const orc_detector* d, int n, int ld, int first_layer, const float* hits, const uint32_t* visit_mask,
                const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status);
int orc_fit_det64(const orc_detector* d, int n, int ld, int first_layer, const double* hits,
                  const uint32_t* visit_mask, const double* seed_par, const double* seed_cov, const int8_t* q,
                  double* out_par, double* out_cov, double* out_chi2, int32_t* out_ndof, int32_t* out_status);
int orc_hit_bin_det(const orc_detector* d, int n_phi, int n_w, int n_hits, const int32_t* layer, const float* xyz,
                    int32_t* offsets, int32_t* order, float* phi_sorted);
int orc_build_det(const orc_detector* d, const orc_build_params* bp, int n_hits, const int32_t* layer,
                  const float* xyz, const float* cov, int n_seeds, int ld, const float* seed_par,
                  const float* seed_cov, const int8_t* q, int n_list, const int32_t* seed_list, int32_t* out_hits,
                  uint32_t* out_visit, double* out_par, double* out_cov, double* out_chi2, int32_t* out_nhits,
                  int32_t* out_status, double* out_margin);
int orc_mlp_blob_size(void);

#ifdef __cplusplus
}
#endif
#endif
