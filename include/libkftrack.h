/*
 * libkftrack — Kalman-filter track fitting and combinatorial track building
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Cerati et al., "Parallelized Kalman-Filter-Based
 * Reconstruction of Particle Tracks on Many-Core Architectures":
 *   - section 2: seeding, building and fitting.  Seeds are given (seeding is
 *     outside the method); building projects each candidate outward layer by
 *     layer, uses the Kalman filter to select compatible hits and branches
 *     into several candidates per seed; fitting reapplies the filter over the
 *     fixed hit list without branching.
 *   - section 2.1 and 4.3: data are matrix-major (structure of arrays), so
 *     consecutive lanes read consecutive addresses.
 *   - section 3: ideal barrel of concentric cylinders, uniform field along z.
 *   - section 3.1: hit selection uses a binned hit structure.
 *   - section 4.1: Kalman updates on the plane tangent to the hit radius.
 *   - section 4.3: a fixed number of candidate slots per seed, ranked so the
 *     best candidates are identified quickly; several events in flight.
 *
 * Conventions (all entry points):
 *   - State X = (x, y, z, px, py, pz) in cm and GeV; charge q = +1 or -1.
 *   - A symmetric 6x6 covariance is stored as its 21 upper-triangle entries
 *     in row order (00,01,02,03,04,05,11,12,...,15,22,...,55).
 *   - A hit is (x, y, z) plus its 3x3 covariance as (xx, xy, xz, yy, yz, zz).
 *   - Arrays are structure of arrays: component c of item i is at
 *     [c * ld + i]; ld >= n.  Arrays per layer: [layer][component][ld].
 *   - Layers are 0-based; layer l is the cylinder of radius geometry.r[l].
 *   - Every pointer argument is a DEVICE pointer, except the descriptor
 *     structs (kf_geometry, kf_build_params, kf_hits, kf_build_extra), which
 *     live in host memory and whose pointer fields are device pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     Every call only enqueues work and returns; outputs are valid once the
 *     stream is synchronised.  The library allocates no device memory: the
 *     caller owns every buffer, including workspaces sized with the
 *     *_workspace_bytes queries.  No caller pointer is kept after return.
 *   - Return value: a kf_status.  On KF_E_HIP, kf_last_error() gives the
 *     HIP message (thread-local).  The library never aborts or throws.
 */
#ifndef LIBKFTRACK_H
#define LIBKFTRACK_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call status */
#define KF_OK 0
#define KF_E_INVALID_ARG 1 /* null pointer with n > 0, n < 0, ld < n, bad layer range, bad sizes */
#define KF_E_WORKSPACE 2   /* workspace missing, smaller than the query returned, or misaligned */
#define KF_E_HIP 3         /* a HIP launch or runtime error; see kf_last_error */
#define KF_E_UNSUPPORTED 4 /* a parameter outside what the kernels implement */

/* per-track status bits (outputs); a flagged track keeps its last good state */
#define KF_TRK_NO_CROSSING 1 /* the helix does not reach the next cylinder */
#define KF_TRK_OUT_OF_Z 2    /* the crossing lies beyond |z| = z_half */
#define KF_TRK_NONFINITE 4   /* a non-finite input or intermediate */
#define KF_TRK_S_NOT_PD 8    /* the 2x2 innovation covariance is not positive definite */
#define KF_TRK_CAP_TRUNC 16  /* build: children were dropped by the candidate cap */
#define KF_TRK_EVENT_TOO_LARGE 32 /* build: the seed's event holds more than 2^24 - 1 binned hits (hit
                                     indices are event-local and 24 bits wide); the seed is not built */

/* arithmetic of the fit and build kernels (storage is always FP32) */
#define KF_ARITH_F32 0 /* FP32 arithmetic */
#define KF_ARITH_F64 1 /* FP64 arithmetic on FP32 data */

typedef struct {
  int32_t n_layers; /* 1..32 */
  float r[32];      /* layer radii, cm, increasing */
  float z_half;     /* barrel half length, cm */
  float bz;         /* field, tesla (non-zero) */
  float x_over_x0;  /* material per layer at normal incidence (0: no scattering) */
  float mass;       /* GeV, sets beta in the scattering width */
} kf_geometry;

const char* kf_status_string(int status);
/* Copies the last HIP error message of this thread into buf (NUL-terminated,
 * truncated to n bytes); returns its full length. */
int kf_last_error(char* buf, size_t n);

/*
 * kf_seed — starting state from the hits on layers 0, 1, 2 (a convention of
 * this library; the paper treats seeding as given, section 2).
 * With a beam spot (beam_sigma > 0, cm: tracks leave the z axis within that
 * transverse distance): the circle through the axis point and the
 * transverse points of hits 0 and 2 gives pT, charge and direction at hit 0;
 * tan(lambda) from the z change over the arc from hit 0 to hit 2; from a
 * broad prior at hit 0 (1 cm tangential, 10 cm in z, |p| per momentum
 * component) one Kalman update with "transverse impact parameter = 0"
 * (variance beam_sigma^2), then the layer-0 scattering and an FP64 Kalman
 * filter over the three hits.  With beam_sigma = 0 the circle passes through
 * the three hits and the impact-parameter update is skipped.  Output: state
 * and covariance at layer 2, rounded to FP32; a failed seed gets a zero state
 * and covariance, q = +1 and its status bit.
 *   hits     [n_layers][9][ld] FP32 (only layers 0..2 are read)
 *   q_out    [ld] int8, seed_par [6][ld], seed_cov [21][ld], status [ld]
 * KF_E_INVALID_ARG for a negative or NaN beam_sigma.
 */
int kf_seed(const kf_geometry* g, int32_t n, int32_t ld, const float* hits, float beam_sigma, int8_t* q_out,
            float* seed_par, float* seed_cov, int32_t* status, void* stream);

/*
 * kf_fit — Kalman-filter fit over a fixed hit list (section 2), one lane per
 * track, FP32.  From the seed, for every layer l in [first_layer, n_layers):
 * propagate along the helix to r[l] (first crossing), transport the
 * covariance with the surface-constrained Jacobian, add Highland scattering
 * noise, then update on the tangent plane with the track's hit on l unless
 * bit l of hole_mask[i] is set (hole_mask may be NULL).
 *   hits     [n_layers][9][ld] FP32
 *   seed_par [6][ld], seed_cov [21][ld], q [ld]
 *   out_par [6][ld], out_cov [21][ld], out_chi2 [ld] (sum over hits),
 *   out_ndof [ld] (2 per hit used), out_status [ld]
 *   arith: KF_ARITH_F32 or KF_ARITH_F64 (inputs and outputs stay FP32)
 * In-place use (out_par == seed_par, out_cov == seed_cov) is allowed.
 */
int kf_fit(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
           const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
           float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof, int32_t* out_status, int32_t arith,
           void* stream);

/*
 * kf_fit_hybrid — the same fit in the hybrid state of section 3: global
 * Cartesian position, polar momentum, Y = (x, y, z, k = q/pT, phi, theta).
 * The seeds are Cartesian as for kf_fit (state, covariance, q) and are
 * converted on entry; each prediction is the Cartesian one at the same point
 * with the covariance carried through the changes of variables, and the
 * update acts on Y, so k may change sign (the charge is not fixed by the
 * seed).  Outputs are hybrid: out_par [6][ld] = Y, out_cov [21][ld] its
 * covariance (upper triangle, row order); chi2, ndof, status as kf_fit.  A
 * state with k = 0 stops with KF_NONFINITE.  Arguments, errors and
 * arithmetic as kf_fit.
 */
int kf_fit_hybrid(const kf_geometry* g, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
                  const uint32_t* hole_mask, const float* seed_par, const float* seed_cov, const int8_t* q,
                  float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof, int32_t* out_status,
                  int32_t arith, void* stream);

/*
 * Binned hits (section 3.1): per event and layer, n_z x n_phi bins,
 * bin = iz * n_phi + iphi with phi = atan2(y, x) in [0, 2 pi) computed in
 * FP64 and rounded to FP32, iphi = min(n_phi-1, floor(phi * n_phi / 2pi)),
 * iz = clamp(floor((z + z_half) * n_z / (2 z_half)), 0, n_z-1).  Hits are
 * ordered by (event, layer, bin, phi, original index).
 */
typedef struct {
  int32_t n_events;
  int32_t n_layers;
  int32_t n_phi, n_z;
  int32_t n_hits;         /* total over events */
  const int32_t* offsets; /* [n_events][n_layers][n_phi*n_z + 1]: first sorted position of each bin; the
                             last entry closes the layer */
  const float* x;         /* [n_hits] sorted */
  const float* y;
  const float* z;
  const float* phi;
  const float* cov;       /* [6][n_hits] sorted */
  const int32_t* orig;    /* [n_hits] event-local original index of each sorted hit */
} kf_hits;

/* Workspace bytes for hit_bin (bin counts and starts, each hit's bin and
   arrival index, one 48-byte record per hit in its bin's slot, and a path
   flag); the workspace must be 256-byte aligned (device allocations are). */
size_t hit_bin_workspace_bytes(int32_t n_events, int32_t n_layers, int32_t n_phi, int32_t n_z, int32_t n_hits);

/*
 * hit_bin — counting sort of the hits of n_events events into the binned
 * layout above (section 3.1).  Events are concatenated: event e owns input
 * hits [event_offsets[e], event_offsets[e+1]) (event_offsets may be NULL
 * when n_events == 1); a hit's original index is its position minus the
 * event's first position.
 *   layer [n_hits] int32, xyz [3][n_hits], cov [6][n_hits]
 *   outputs: offsets [E][L][nb+1], sorted x,y,z,phi [4][n_hits] (x block,
 *   then y, z, phi), sorted cov [6][n_hits], orig [n_hits]
 * A hit on a layer outside [0, n_layers) or with a non-finite coordinate is
 * left out of every bin and counted in *out_bad (int32, may be NULL); the
 * sorted arrays then hold n_hits - bad hits and their tail is unspecified.
 * Any input order is accepted.  When every event's hits come grouped by
 * layer in ascending order, all valid, n_phi * n_z <= 4096 and there are at
 * least six (event, layer) ranges per compute unit, one block per (event,
 * layer) sorts the call; otherwise the general kernels do, with the same
 * result.  The environment variable KFTRACK_HIT_BIN_PATH=grouped (try the
 * grouped path whatever the number of ranges) or =general overrides the
 * choice.  Diagnostic: after the call, the int32 at byte offset
 * hit_bin_workspace_bytes(...) - 256 of ws is 0 when the grouped path
 * sorted the call and 1 otherwise.
 */
int hit_bin(const kf_geometry* g, int32_t n_events, const int32_t* event_offsets, int32_t n_phi, int32_t n_z,
            int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov, int32_t* offsets,
            float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig, int32_t* out_bad, void* ws,
            size_t ws_bytes, void* stream);

typedef struct {
  float chi2_cut;      /* accept a hit iff chi2 < chi2_cut (2 degrees of freedom) */
  int32_t max_holes;   /* a hole child is added while holes < max_holes */
  int32_t cand_cap;    /* candidates kept per seed, 1..8 (one lane per candidate slot) */
  float nsigma;        /* plain window: nsigma * sqrt(S) per coordinate */
  float win_sig_rphi;  /* nominal hit resolution used in the window's S, cm */
  float win_sig_z;
  int32_t first_layer; /* first layer searched; seeds sit on first_layer - 1 */
  int32_t window_mode; /* 0 plain; 1 learned (mlp must point to a network block) */
  const void* mlp;     /* device pointer to the window network block (kf_mlp_block_bytes) */
  int32_t lanes_per_block; /* 64, 128, 256 (0: the widest whose LDS fits) */
  int32_t persistent_blocks; /* blocks of the persistent grid (0: CUs x resident blocks per CU) */
  int32_t arith;       /* KF_ARITH_F32 or KF_ARITH_F64 */
  int32_t phi_refine;  /* sub-bins per phi bin of the fine index the hit search uses, 1..64 (0: 64) */
  int32_t state;       /* 0 Cartesian; 1 hybrid (x, y, z, q/pT, phi, theta; section 3): seeds are
                          converted on entry, the charge follows the sign of q/pT, out_par/out_cov
                          are hybrid; the learned window still reads the Cartesian prediction */
} kf_build_params;

/* Optional build inputs and outputs (all fields may be NULL / 0). */
typedef struct {
  const int32_t* seed_event;  /* [n_seeds] event of each seed (NULL: all event 0) */
  const int32_t* seed_order;  /* [n_seeds] order in which seeds are taken (NULL: 0..n-1) */
  const int32_t* event_n_seeds; /* [n_events] seeds per event, needed for event_done_ticks */
  int64_t* event_done_ticks;  /* [n_events] wall-clock tick when the event's last seed finished (not
                                 written for an event with no seeds) */
  int64_t* start_tick;        /* [1] earliest wall-clock tick seen by any wave of the launch */
  /* training-data dump: for every candidate whose hits so far are all true
     (or holes) and whose seed has a true hit on the layer, one row of 32
     words: the 27 features (predicted state and covariance, Cartesian in
     either state: what the learned window reads), the 2 labels (|arc| and
     |dz| to the true hit), the plain arc and z half-widths of the
     candidate's window, and the int32 (seed << 8) | (layer << 3) | slot
     (seed indices below 2^24 identify the seed) */
  const int32_t* true_hits;   /* [n_layers][ld] true original hit index per seed and layer */
  const float* true_xyz;      /* [n_layers][3][ld] position of that true hit */
  float* dump;                /* [dump_capacity][32] */
  int32_t* dump_count;        /* [1] rows written (rows beyond capacity are counted, not written) */
  int32_t dump_capacity;
  /* work counters, added to (not cleared): candidate-layers predicted, hits
     window-tested, hits given a chi2, Kalman updates applied */
  uint64_t* counters;         /* [4] */
} kf_build_extra;

/*
 * Workspace bytes for kf_build: a queue head, per-event counters, the fine
 * phi index of every (event, layer, z row), n_phi * phi_refine + 1 int32
 * each, a packed copy of the binned hits (48 bytes per hit: phi, x, y, z,
 * cov, orig, which the hit search reads in one pass) and the per-wave
 * history tables; the index and the packed hits are rebuilt by every
 * kf_build call from the binned hits.  The workspace must be 256-byte
 * aligned (device allocations are).  Returns 0 for a NULL or malformed
 * descriptor.
 */
size_t kf_build_workspace_bytes(const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds);

/*
 * kf_build — combinatorial Kalman-filter building (sections 2, 3.1, 4.3),
 * one lane per candidate slot, cand_cap slots per seed, one persistent launch
 * over all seeds of all events (an atomic queue hands out groups of seeds).
 * For each seed, from its state on layer first_layer-1, layer by layer:
 *   1. predict every candidate (a failed crossing or |z| > z_half stops it);
 *   2. window: plain = nsigma*sqrt(S) per coordinate with S = H P H^T +
 *      diag(win_sig_rphi^2, win_sig_z^2) (dphi = w_rphi / r, dz = w_z); in
 *      learned mode, where the plain arc or z half-width exceeds its gate,
 *      the learned widths replace them where not below their floors;
 *   3. every hit of the layer with |wrap(phi_h - phi_p)| <= dphi and
 *      |z_h - z_p| <= dz is tested; accepted iff its update chi2 < chi2_cut;
 *   4. children: one updated child per accepted hit plus a hole child
 *      (predicted state) while holes < max_holes;
 *   5. the seed's children are ranked (nhits desc, chi2 asc, parent slot asc,
 *      hit index asc, hole last) and the first cand_cap kept;
 *   6. a candidate with no child competes for the seed's best-finished
 *      record (nhits desc, chi2 asc; replaces only when strictly better).
 * Result per seed: the best of the active candidates (slot order) then the
 * finished record.  nhits counts hits on the searched layers.
 *   seed_par [6][ld], seed_cov [21][ld], q [ld]: states on layer first_layer-1
 *   out_hits [n_layers - first_layer][ld]: event-local original hit index per
 *     searched layer, -1 for a hole or a layer not reached
 *   out_par [6][ld], out_cov [21][ld], out_chi2, out_nhits, out_status [ld]
 * Results do not depend on lanes_per_block, persistent_blocks or the order of
 * the seeds.
 */
int kf_build(const kf_geometry* g, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds, int32_t ld,
             const float* seed_par, const float* seed_cov, const int8_t* q, int32_t* out_hits, float* out_par,
             float* out_cov, float* out_chi2, int32_t* out_nhits, int32_t* out_status,
             const kf_build_extra* extra, void* ws, size_t ws_bytes, void* stream);

/*
 * kf_build_noalloc — kf_build for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same build, arguments, outputs and errors as kf_build
 * without the workspace, which lives in a static device array of the library
 * holding kf_build_noalloc_max_bytes() = 64 MiB on every GPU the library
 * runs on, until the process ends (enough for one event of 20 000 tracks
 * plus 20 % noise on 17 layers, about 39 MB).  A call whose
 * kf_build_workspace_bytes exceeds it returns KF_E_WORKSPACE (message in
 * kf_last_error) without launching anything.  The call allocates nothing.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (two streams, two host threads) race and must be serialised by the caller.
 */
int kf_build_noalloc(const kf_geometry* g, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds, int32_t ld,
                     const float* seed_par, const float* seed_cov, const int8_t* q, int32_t* out_hits,
                     float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits, int32_t* out_status,
                     const kf_build_extra* extra, void* stream);
size_t kf_build_noalloc_max_bytes(void);

/* Launch shape chosen by the last kf_build call of the calling host thread
 * (zeros before the first): lanes per block, blocks of the persistent grid,
 * dynamic LDS bytes per block, blocks per CU the occupancy calculator allows,
 * the device's LDS limit per block. */
typedef struct {
  int32_t lanes_per_block;
  int32_t blocks;
  int32_t lds_bytes;
  int32_t resident_blocks_per_cu;
  int32_t max_lds_per_block;
} kf_build_launch_info;
int kf_build_last_launch(kf_build_launch_info* info);

/*
 * Learned search window (an addition to the method: the paper sizes the hit
 * search from the covariance).  A device block of kf_mlp_block_bytes() bytes
 * holds the network: standardisation (mean, 1/std of the 27 features), FP32
 * biases, output scales, kappa, the two floors and the two gates (arc, z;
 * 0 consults the network for every candidate), then BF16 weights
 * (layout: the library's kfmlp.h).  Rows of data are 32 floats: the 27
 * features (predicted state, 21 covariance entries), the 2 labels (|arc| at
 * the layer radius and |dz| to the true hit), then 3 words not read here.
 */
size_t kf_mlp_block_bytes(void);
/* widths [n_rows][2] (kappa applied) and, if out_logits is not NULL, the
 * head's pre-softplus outputs [n_rows][2] */
int kf_mlp_forward(const void* block, int32_t n_rows, const float* rows, float* out, float* out_logits,
                   void* stream);
size_t kf_mlp_grad_workspace_bytes(int32_t n_rows);
/* grad [n_params + 1]: gradient of the mean loss over rows and both outputs
 * (order: W1 [64][27], b1, W2 [64][64], b2, W3 [2][64], b3), then the loss
 * 20 * max(0, d - w) + max(0, w - d) averaged the same way */
int kf_mlp_grad(const void* block, int32_t n_rows, const float* rows, float* grad, void* ws, size_t ws_bytes,
                void* stream);
/* one Adam step (step counts from 1) on the FP32 master vector [n_params]
 * with moments m, v; refreshes the block's BF16 weights and FP32 biases */
int kf_mlp_adam(void* block, float* master, float* m, float* v, const float* grad, int32_t step, float lr,
                float beta1, float beta2, float eps, void* stream);

/*
 * kf_gather_hits — the hit rows of built tracks in the fit layout (the final
 * fit after building, section 2).  For seed i and layer l >= first_layer:
 * built_hits[(l - first_layer) * ld + i] is an event-local original index
 * (or -1); the row is copied from the unsorted event hits xyz [3][n_hits],
 * cov [6][n_hits] at event_offsets[seed_event[i]] + index; a missing hit
 * sets bit l of hole_mask[i] and zeroes the row.  seed_event and
 * event_offsets may be NULL for a single event.  Rows of layers below
 * first_layer are not written.
 *   fit_hits [n_layers][9][ld], hole_mask [ld]
 */
int kf_gather_hits(int32_t n_layers, int32_t first_layer, int32_t n_seeds, int32_t ld, const int32_t* built_hits,
                   const int32_t* seed_event, int32_t n_events, const int32_t* event_offsets, int32_t n_hits,
                   const float* xyz, const float* cov, float* fit_hits, uint32_t* hole_mask, void* stream);

/*
 * Batched building as one replayable HIP graph (several events in flight,
 * sections 4.2 and 4.3): kf_batch_plan_create captures hit_bin of all events
 * and the persistent kf_build from `stream` (not the null stream) into a
 * graph and instantiates it; every pointer and size is fixed at creation
 * (contents may change between launches).  The captured work clears its own
 * counters with kernels, so each launch is independent of the previous one.
 * The arguments are those of hit_bin and kf_build; `binned` describes the
 * sorted arrays that hit_bin writes (binned_offsets .. sorted_orig).
 * kf_batch_plan_launch replays the graph on `stream`; kf_batch_plan_destroy
 * frees the host-side graph objects.
 */
typedef struct kf_batch_plan kf_batch_plan;
int kf_batch_plan_create(const kf_geometry* g, const kf_build_params* bp, int32_t n_events,
                         const int32_t* event_offsets, int32_t n_hits, const int32_t* layer, const float* xyz,
                         const float* cov, const kf_hits* binned, int32_t* binned_offsets, float* sorted_xyzphi,
                         float* sorted_cov, int32_t* sorted_orig, void* bin_ws, size_t bin_ws_bytes,
                         int32_t n_seeds, int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q,
                         int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits,
                         int32_t* out_status, const kf_build_extra* extra, void* build_ws, size_t build_ws_bytes,
                         void* stream, kf_batch_plan** plan);
/*
 * The whole step as one graph (section 2: building, then the final fit of
 * the built tracks): what kf_batch_plan_create captures, then
 * kf_gather_hits of the built lists (xyz, cov and event_offsets as given to
 * hit_bin, seed_event from `extra`, first_layer from `bp`) into
 * fit->fit_hits / fit->hole_mask, then kf_fit (kf_fit_hybrid when
 * bp->state is 1) from the same seeds in fit->arith.  fit must not be NULL; every pointer in it is a device pointer
 * the caller owns.  Launch and destroy as a batch plan.
 */
typedef struct {
  int32_t arith;        /* KF_ARITH_F32 or KF_ARITH_F64 for the fit */
  float* fit_hits;      /* [n_layers][9][ld], written by the gather */
  uint32_t* hole_mask;  /* [ld], written by the gather */
  float* out_par;       /* [6][ld] */
  float* out_cov;       /* [21][ld] */
  float* out_chi2;      /* [ld] */
  int32_t* out_ndof;    /* [ld] */
  int32_t* out_status;  /* [ld] */
} kf_fit_stage;
int kf_step_plan_create(const kf_geometry* g, const kf_build_params* bp, int32_t n_events,
                        const int32_t* event_offsets, int32_t n_hits, const int32_t* layer, const float* xyz,
                        const float* cov, const kf_hits* binned, int32_t* binned_offsets, float* sorted_xyzphi,
                        float* sorted_cov, int32_t* sorted_orig, void* bin_ws, size_t bin_ws_bytes,
                        int32_t n_seeds, int32_t ld, const float* seed_par, const float* seed_cov, const int8_t* q,
                        int32_t* out_hits, float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits,
                        int32_t* out_status, const kf_build_extra* extra, void* build_ws, size_t build_ws_bytes,
                        const kf_fit_stage* fit, void* stream, kf_batch_plan** plan);
int kf_batch_plan_launch(kf_batch_plan* plan, void* stream);
int kf_batch_plan_destroy(kf_batch_plan* plan);
/* frequency of the device wall clock read by the build's completion ticks */
int kf_wall_clock_khz(int32_t* khz);

/* Practical vector peak (measurement support, not the method): `blocks`
 * blocks of 256 lanes each run `iters` rounds of 8 independent fused
 * multiply-adds in the arithmetic `arith` (2 flops each) and write one value
 * per lane to out [blocks * 256] (float or double).  The caller times the
 * launch. */
int kf_peak_fma(int32_t arith, int32_t blocks, int32_t iters, void* out, void* stream);

/*
 * General detector (section 4.1: the barrel of concentric cylinders closed
 * by endcap disks, "a cylinder with lids", and modules that sit off a
 * layer's average surface).  Layers are listed in the order a track from
 * the origin meets them: barrel layers outwards, then the disks of each
 * side outwards.  Layer l is a cylinder of average radius pos[l] active over
 * lo[l] <= z <= hi[l] (kind KF_LAYER_BARREL), or a plane z = pos[l] active
 * over lo[l] <= r <= hi[l] (kind KF_LAYER_DISK).  Its modules may sit up to
 * dmod[l] cm off that average surface (in radius on a barrel layer, in z on a
 * disk): a hit lies on its module's surface, which the hit itself gives
 * (barrel: its radius sqrt(x^2 + y^2); disk: its z).  x_over_x0 is the
 * material of every layer at normal incidence.
 */
#define KF_LAYER_BARREL 0
#define KF_LAYER_DISK 1
typedef struct {
  int32_t n_layers; /* 1..32 */
  int32_t kind[32]; /* KF_LAYER_BARREL or KF_LAYER_DISK */
  float pos[32];    /* average radius (barrel, > 0) or z of the average plane (disk), cm */
  float lo[32];     /* active extent: z range (barrel) or r range (disk), cm; lo < hi */
  float hi[32];
  float dmod[32];   /* largest module offset from the average surface, cm (>= 0) */
  float bz;         /* field, tesla (non-zero) */
  float x_over_x0;
  float mass;
} kf_detector;

/*
 * hit_bin_det — hit_bin over a general detector: per event and layer n_w x
 * n_phi bins, bin = iw * n_phi + iphi, phi as hit_bin, and the row
 * coordinate w = z on a barrel layer or w = r = sqrt(x^2 + y^2) (FP64 from
 * the FP32 inputs) on a disk, iw = clamp(floor((w - lo) * n_w / (hi - lo)),
 * 0, n_w - 1).  The output descriptor (kf_hits) has n_z = n_w.  Arguments,
 * workspace (hit_bin_workspace_bytes with n_z = n_w) and errors as hit_bin;
 * a hit with a non-finite coordinate is rejected like one on a bad layer.
 */
int hit_bin_det(const kf_detector* d, int32_t n_events, const int32_t* event_offsets, int32_t n_phi, int32_t n_w,
                int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov, int32_t* offsets,
                float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig, int32_t* out_bad, void* ws,
                size_t ws_bytes, void* stream);

/*
 * kf_fit_det — the Kalman-filter fit (section 2) over a general detector,
 * one lane per track.  For every layer l >= first_layer (in index order)
 * with bit l set in visit_mask[i] (the layers the track crossed): with a hit
 * (bit l clear in hole_mask[i], which may be NULL) the state moves along the
 * helix in one step to the hit's own surface (barrel: the cylinder of the
 * hit's radius; disk: the plane of the hit's z; the first crossing along the
 * motion), the covariance follows with the surface Jacobian, the layer's
 * Highland scattering is added there (incidence from the surface normal),
 * and the state is updated with the hit (barrel: on the plane tangent to the
 * cylinder at the predicted point, coordinates along the arc and z; disk:
 * in the disk's plane, coordinates x and y).  On a hole the step goes to the
 * layer's average surface and takes its scattering.  Extents are not
 * checked: the visit mask says which layers the track crossed.
 *   hits [n_layers][9][ld] FP32 (rows of layers not visited are not read),
 *   visit_mask [ld], hole_mask [ld] or NULL; seeds, outputs, statuses
 *   (KF_TRK_NO_CROSSING: no crossing with a surface) and arith as kf_fit.
 */
int kf_fit_det(const kf_detector* d, int32_t n, int32_t ld, int32_t first_layer, const float* hits,
               const uint32_t* visit_mask, const uint32_t* hole_mask, const float* seed_par, const float* seed_cov,
               const int8_t* q, float* out_par, float* out_cov, float* out_chi2, int32_t* out_ndof,
               int32_t* out_status, int32_t arith, void* stream);

/*
 * kf_build_det — combinatorial building (sections 2, 4.1, 4.3) over a
 * general detector with two-step propagation.  The rules of kf_build (chi2
 * cut, one hole child while holes < max_holes, ranking of the children,
 * cand_cap, best-finished record) with these differences:
 *   - each candidate moves to its own next layer: the first layer after its
 *     current one (index order) whose average surface the helix meets ahead
 *     within the layer's extent, on a disk also moving outwards
 *     (x px + y py > 0) within less than half a turn; a track leaving the
 *     barrel through its end continues on the disks; a candidate with no
 *     next layer has left the detector and finishes (status 0);
 *   - step 1 goes to that layer's average surface (no material), where the
 *     window is formed: (phi, w) with w = z (barrel) or r (disk), half-widths
 *     nsigma * sqrt(S) with the nominal resolution (win_sig_rphi along the
 *     arc, win_sig_z along w), widened by dmod times the track's slope
 *     (|dw/dr| and |dphi/dr| on a barrel layer, |dr/dz| and |dphi/dz| on a
 *     disk); a hit is in the window iff |wrap(phi_h - phi_p)| <= dphi and
 *     |w_h - w_p| <= dw;
 *   - step 2, for every hit in the window: from the average surface to the
 *     hit's own surface (the nearest crossing, forwards or backwards), the
 *     layer's scattering there, then the update and its chi2 (tangent plane
 *     on a barrel layer, the disk's plane on a disk); a hole child takes the
 *     layer's scattering on the average surface;
 *   - every candidate ends in the best-finished record, which is the result.
 * Plain window and Cartesian state only (window_mode and state must be 0,
 * else KF_E_UNSUPPORTED).  hits: from hit_bin_det (n_z = n_w rows).  extra:
 * seed_event, seed_order and counters are honoured; the training dump and
 * the completion ticks are not available (KF_E_UNSUPPORTED if set).
 * Workspace: kf_build_workspace_bytes(bp, hits, n_seeds).
 *   out_hits [n_layers - first_layer][ld]: event-local original hit index
 *     per layer, -1 for a hole or a layer not visited
 *   out_visit [ld]: bit l set for every layer the chosen candidate visited
 *     (with a hit or a hole)
 *   out_par, out_cov, out_chi2, out_nhits, out_status [ld] as kf_build
 * Results do not depend on lanes_per_block, persistent_blocks or the order
 * of the seeds.
 */
int kf_build_det(const kf_detector* d, const kf_build_params* bp, const kf_hits* hits, int32_t n_seeds, int32_t ld,
                 const float* seed_par, const float* seed_cov, const int8_t* q, int32_t* out_hits,
                 uint32_t* out_visit, float* out_par, float* out_cov, float* out_chi2, int32_t* out_nhits,
                 int32_t* out_status, const kf_build_extra* extra, void* ws, size_t ws_bytes, void* stream);
/* Launch shape chosen by the last kf_build_det call of the calling host thread
 * (as kf_build_last_launch). */
int kf_build_det_last_launch(kf_build_launch_info* info);

#ifdef __cplusplus
}
#endif
#endif
