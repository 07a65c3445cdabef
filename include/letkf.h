/*
 * letkf.h -- C ABI of the MI355X (gfx950) local ensemble transform Kalman
 * filter frame for zonal adaptive-optics control (Gray et al., "Local ensemble
 * transform Kalman filter, a fast non-stationary control law for adaptive
 * optics on ELTs", arXiv:1408.7069).
 *
 * One frame k is
 *   forecast  X_b = a X_a + V                      (Sec. 3.1.2, member prediction;
 *                                                    App. B.2 with A_tur = a Id)
 *   analysis  per domain l, independently          (Sec. 4.2)
 *               Y_l  = observation-region rows of D (X_b - x_b 1^T), scaled by
 *                      sqrt(g), g = f^2 / (s r) (taper f on Sigma_w^{-1/2}, Sec. 4.1)
 *               A~   = (m-1)/rho I + Y_l^T Y_l      (m x m, Sec. 3.1.1 EVD matrix)
 *               w    = A~^{-1} Y_l^T sqrt(g) d_l,   W = sqrt((m-1)/rho) A~^{-1/2}
 *                      (Sec. 3.1.1 via A~ = Q Lambda Q^T); A~^{-1/2} from an
 *                      FP64 Newton-Schulz iteration by default, or from the
 *                      FP64 Jacobi eigendecomposition (see `transform`)
 *               X_a,l = (x_b,l + X_l' w) 1^T + sqrt(rho) X_l' W   (owned rows)
 *   gather    the owned rows of all domains form X_a (Sec. 4.2, concatenation)
 * with D the Fried-geometry Shack-Hartmann slope operator (App. B).
 *
 * Layouts at this boundary
 *   nodes     valid actuator nodes of the (N+1)^2 grid, row-major; a node is
 *             valid when it is a corner of a valid subaperture.
 *   slopes    [x-slopes of the valid subapertures, row-major; y-slopes, same
 *             order]; p = 2 * (valid subapertures).
 *   ensemble  [node][member] (member index fastest), one block per instance,
 *             instances concatenated in creation order.
 *   element type: float for LETKF_FP32, double for LETKF_FP64.
 * Device pointers are HIP device addresses on the handle's device; `stream`
 * is a hipStream_t (NULL = the default stream).  The caller keeps every
 * buffer it passes valid until the work on `stream` completes.
 *
 * Ownership: the handle owns all device memory it allocates; getters copy
 * out.  A handle is used from one host thread and one stream at a time.
 *
 * Errors: every int-returning call returns LETKF_OK (0) or a negative code;
 * letkf_strerror() gives a message, letkf_last_error() the detail of the
 * most recent failure on the calling thread.
 */
#ifndef LETKF_H
#define LETKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LETKF_OK 0
#define LETKF_E_INVAL (-1)      /* bad configuration, size or argument        */
#define LETKF_E_NOMEM (-2)      /* device or host allocation failed           */
#define LETKF_E_DEVICE (-3)     /* HIP runtime error                          */
#define LETKF_E_NONFINITE (-4)  /* NaN/Inf met in the slopes or the update     */
#define LETKF_E_NOCONV (-5)     /* transform hit max_sweeps in >= 1 domain   */
#define LETKF_E_STATE (-6)      /* call out of order (e.g. analyse before forecast) */

#define LETKF_FP32 0            /* FP32 state and MFMA contractions, FP64 transform */
#define LETKF_FP64 1            /* FP64 everywhere                                   */

/* Transform of the local analyses (letkf_config.transform): how W and w are
 * obtained from A~ (Sec. 3.1.1).
 *   NS64  A~^{-1/2} by the scaled coupled Newton-Schulz iteration in FP64 on
 *         the FP64 matrix cores (Higham 1997), w = A~^{-1} b from the same
 *         iterate; stops when the predicted residual ||a Z Y - I||_F^2 after
 *         a step is <= jacobi_tol / 100.  With FP32 state its symmetric
 *         products are formed on the upper tiles and mirrored while the
 *         spectrum's lower bound (m-1)/rho / ||A~||_F is at least 1e-4, in
 *         full below (mirrored iterates drift apart past condition numbers
 *         of about 2e4).  Default.
 *   NS32  the same iteration with FP32 iterates on the FP32 matrix cores
 *         (W within ~2e-5 relative), w refined once in FP64 against A~.
 *         FP32 handles only; an FP64 handle runs NS64.  Its FP32 iterates
 *         lose accuracy sooner than the others as A~ grows ill-conditioned
 *         (3.6 times the FP64 transforms' distance from the oracle at a
 *         condition number of 8e6).
 *   EVD   A~ = Q Lambda Q^T by the FP64 one-sided Jacobi on the Cholesky
 *         factor (stop: jacobi_tol on the relative inner products), then
 *         W = sqrt(c) Q Lambda^{-1/2} Q^T and w from the Cholesky factor. */
#define LETKF_TRANSFORM_NS64 0
#define LETKF_TRANSFORM_NS32 1
#define LETKF_TRANSFORM_EVD 2
/*   NSP        the same iteration written on P = Z Y alone (P <- a P T^2,
 *              T = (3 I - a P) / 2: two products of P with its own powers a
 *              step, on the ten upper 16 x 16 tiles), in FP64, carrying only
 *              what the update needs: Z X'^T for the owned rows and Z b.
 *              Same stopping rule as NS64, and a second-order last step
 *              once the residual is below sqrt(tol) (FP32 state) or
 *              tol^(2/3) (FP64): sqrt(a)(I - E/2 + 3/8 E^2), E = a P - I,
 *              in place of one more step.
 *   NSP_MIXED  NSP with the P updates in FP64 while the spectrum's lower
 *              bound l is below 0.01 (the steps whose rounding the small
 *              eigenvalues amplify) and in FP32 after; X' Z in FP32.  The
 *              FP32 steps add a few percent to the error the FP32 Gram
 *              itself carries (its rounding times the condition number of
 *              A~).  FP32 handles; an FP64 handle runs NSP.
 * A handle with the blend-mode gather runs NS64 when NSP or NSP_MIXED is
 * asked for (the P forms carry the owned rows only). */
#define LETKF_TRANSFORM_NSP 3
#define LETKF_TRANSFORM_NSP_MIXED 4

/* State model of an instance (letkf_config.model).
 *   PHASE        delay-free: x_k = phi_k, y_k = D phi_k + w_k.
 *   CLOSED_LOOP  the AO loop of Sec. 2.2: x_k = [phi_k; phi_{k-1}; u_{k-1};
 *                u_{k-2}], y_k = D phi_{k-1} - D N u_{k-2} + w_k, command
 *                u_k = P phi^_{k+1/k}, with a zonal DM whose actuators are the
 *                valid phase nodes (N = P = I).  The library keeps u_{k-1},
 *                u_{k-2} (zero at create).  Each frame analyses phi_{k-1} on
 *                y_k with y_bar = D x_b - D u_{k-2}; phi_k follows the model
 *                (its gain is a times that of phi_{k-1}, the model noise being
 *                independent of the slopes), so the ensemble carried to the
 *                next frame is a X_a + V, which the next frame's forecast
 *                forms; the command is u_k = a^2 x_a.  The piston fit (Sec.
 *                4.4) works on x_a - u_{k-2}.  No adjoint. */
#define LETKF_MODEL_PHASE 0
#define LETKF_MODEL_CLOSED_LOOP 1
/* letkf_config.gather_mode */
#define LETKF_GATHER_CONCAT 0
#define LETKF_GATHER_BLEND 1
/* letkf_config.localisation */
#define LETKF_LOCALISATION_DOMAIN 0
#define LETKF_LOCALISATION_COVARIANCE 1

/* Per-domain status bits (letkf_status); bits 8-15 hold the steps the
 * transform took (Newton-Schulz steps, or Jacobi sweeps begun). */
#define LETKF_FLAG_NONFINITE 1
#define LETKF_FLAG_NOCONV 2
#define LETKF_FLAG_STEPS_SHIFT 8

typedef struct letkf_handle letkf_handle;

/* One adaptive-optics instance.  Host pointers are read during letkf_create
 * only. */
typedef struct letkf_config {
  int32_t n_sub;               /* N: N x N subapertures (Sec. 5 set-up)            */
  const uint8_t *subap_mask;   /* N*N row-major, 1 = valid; NULL = annulus rule:
                                  valid when > 50 % of the subaperture lies in
                                  eps*N/2 <= r <= N/2 (Sec. 5), 64x64 sampling    */
  double obscuration;          /* eps, used when subap_mask == NULL                */
  int32_t m;                   /* ensemble size, 2 <= m <= 128 (past 64: the wide
                                  analysis, see letkf_create)                      */
  int32_t domain_size;         /* b: domains are b x b subaperture blocks (Sec. 4.1) */
  int32_t halo;                /* h >= 0: observation region = block grown by h    */
  double rho;                  /* multiplicative inflation > 0                     */
  const double *r_diag;        /* p noise variances (Sigma_w diagonal, Sec. 3.1.1);
                                  NULL = r_sigma2 for every slope                  */
  double r_sigma2;             /* used when r_diag == NULL                         */
  double r_scale;              /* s > 0: Sigma_w = s diag(r)                       */
  double ar_coeff;             /* a: AR(1) turbulence model (App. B)               */
  double taper_c;              /* Gaspari-Cohn half width in pitches (Sec. 4.1
                                  smooth localisation); 0 = no taper               */
  const float *noise_bank;     /* optional model-noise bank, bank_screens periodic
                                  bank_side x bank_side screens (row-major); used
                                  when a forecast is given no explicit V          */
  int32_t bank_screens;
  int32_t bank_side;           /* power of two, >= N + 1                           */
  uint64_t seed;               /* Philox4x32-10 key for the bank draws             */
  int32_t precision;           /* LETKF_FP32 or LETKF_FP64 (same for all instances) */
  double jacobi_tol;           /* accuracy of the transform: EVD stops when 63
                                  rounds pass with no relative inner product
                                  above tol; NS64/NS32 stop when the predicted
                                  residual is <= tol / 100.  0 = 1e-4 (FP32: W
                                  within ~5e-6 relative with EVD, ~1e-9 with
                                  NS64), 1e-10 (FP64).  The adjoint's Jacobi
                                  uses min(tol, 1e-6) in FP32.                     */
  int32_t max_sweeps;          /* 0 = 30: Jacobi sweeps, or Newton-Schulz steps    */
  int32_t piston_removal;      /* 1: after the gather, remove one piston per domain
                                  fitted by least squares to the slopes of the
                                  subapertures that straddle domains (Sec. 4.4:
                                  local estimates are blind to their own piston);
                                  every member of the domain is shifted. Needs at
                                  most 4096 domains in the instance.              */
  int32_t transform;           /* LETKF_TRANSFORM_* (same for all instances);
                                  0 = NS64                                         */
  int32_t model;               /* LETKF_MODEL_PHASE (0) or LETKF_MODEL_CLOSED_LOOP  */
  double ar2_coeff;            /* a2 of an AR(2) turbulence model (Sec. 6 names it
                                  as the extension of the AR(1) model):
                                  X_b = a X_a(k) + a2 X_a(k-1) + V, each member
                                  forecast from its own last two analyses (the
                                  lagged phase is not re-analysed); |a2| < 1;
                                  0 = AR(1).  Delay-free model only; no adjoint.
                                  letkf_set_ensemble sets both frames.            */
  double refit_forgetting;     /* online refit of the AR(1) model (Sec. 4.2: the
                                  model may be re-identified during the
                                  prediction step); 0 = off, else the forgetting
                                  factor f in (0, 1].  After every frame k the
                                  piston-removed analysis means x_k, x_{k-1}
                                  (means over members, then the mean over the
                                  nodes taken out) update
                                    s01 = f s01 + x_k . x_{k-1}
                                    s11 = f s11 + x_{k-1} . x_{k-1}
                                  and, once s11 > 0, the model of the next
                                  frames: a = clip(s01 / s11, 0, 0.9999) and the
                                  model noise V (drawn for a_0 = ar_coeff, given
                                  or from the bank) scaled by
                                  sqrt((1 - a^2) / (1 - a_0^2)).  Needs
                                  0 <= ar_coeff < 1 and the AR(1) model; no
                                  adjoint.  See letkf_get_model.                  */
  int32_t gather_mode;         /* how X_a is formed from the local analyses:
                                  LETKF_GATHER_CONCAT (0): the owned rows of each
                                  domain, concatenated (Sec. 4.2).
                                  LETKF_GATHER_BLEND (1), a variant: every domain
                                  updates all nodes of its patch (owned nodes and
                                  the corners of its observation subapertures);
                                  the patches are put on a common piston (least
                                  squares over the nodes two patches share, the
                                  minimum-norm solution), then each node takes
                                  the weighted mean of its patch rows with
                                  weights t(d_i) t(d_j), t(d) = 1 - d/(h+2), d_i,
                                  d_j its distance in node pitches from the
                                  domain's block, normalised over the patches.
                                  Needs piston_removal off (the alignment takes
                                  its place); no adjoint.                         */
  int32_t localisation;        /* LETKF_LOCALISATION_DOMAIN (0): the local
                                  analysis of Sec. 4.2 (ensemble transform per
                                  domain).  LETKF_LOCALISATION_COVARIANCE (1):
                                  covariance localisation (Sec. 4 names it):
                                  per domain, over its node patch, the prior
                                  covariance rho_xx o (rho X'X'^T / (m-1)) with
                                  rho_xx the Gaspari-Cohn function of the node
                                  distance over taper_c (0: no taper; the
                                  observation weights are then not tapered),
                                  the gain K = P D^T (D P D^T + R)^{-1} of the
                                  owned rows from an FP64 Cholesky of the p_l x
                                  p_l matrix, x_a = x_b + K d and the anomalies
                                  sqrt(rho) (X' - K D X' / 2) (deterministic
                                  EnKF); the transform field is ignored.  Same
                                  for all instances of a handle; delay-free
                                  model only, no blend-mode gather, no adjoint.  Needs LDS for the patch
                                  rows and three FP64 arrays of about p_l^2,
                                  patch x p_l and n_own x p_l doubles:
                                  letkf_create fails with LETKF_E_INVAL when
                                  the device has too little (b = 4, h = 1 fits
                                  in both precisions).                            */
} letkf_config;

/* Sizes of one instance (or totals when instance = -1). */
typedef struct letkf_sizes {
  int64_t n_nodes;             /* valid nodes                                      */
  int64_t n_slopes;            /* p                                                */
  int64_t n_domains;
  int64_t ensemble_elems;      /* sum of n_nodes * m                               */
  int64_t obs_total;           /* sum over domains of local slopes                 */
  int32_t m;                   /* ensemble size (instance) or max m (totals)       */
  int32_t max_owned;           /* largest number of owned nodes in a domain        */
  int32_t max_obs;             /* largest local slope count p_l                    */
  int32_t max_patch;           /* largest node patch (owned + stencil corners)     */
  int32_t n_sub;               /* N of the instance (0 for totals)                 */
  int32_t n_instances;
} letkf_sizes;

/* Build the geometry of every instance on the host (pupil mask, node and slope
 * numbering, b x b domains with halo h, taper distances, a work list in
 * instance-major, row-major domain order) and allocate the device state on `device`.  The ensemble starts at
 * zero (Sec. 3.1: X_{1/0} = 0).  Returns LETKF_E_INVAL for m < 2 or m > 128,
 * rho <= 0, r_scale <= 0, any r <= 0, b < 1, h < 0, b + 2h > 10,
 * an instance with no valid subaperture, or a bank that is not a power of two
 * wide or is narrower than N + 1.
 *
 * Wide analysis.  A handle in which some instance has m > 64, a node patch of
 * more than 64 nodes or more than 64 observation subapertures (for instance
 * the paper's timing shape, Sec. 5.3 Tables 1-2: m = 101, b = 4, h = 2: 9 x 9
 * patch nodes, 128 local slopes) runs every local analysis on the wide kernel:
 * 8 wavefronts a domain, the Gram in FP64, the P-form iteration in FP64
 * (NS64, NSP and NSP_MIXED are accepted; with FP32 state and NSP_MIXED its P
 * updates run in FP32 once the spectrum's lower bound passes 0.05).  Such a
 * handle has the delay-free AR(1) phase model with the concatenating gather
 * only: the closed loop, AR(2), the online refit, the blend gather, covariance
 * localisation and the EVD/NS32 transforms give LETKF_E_INVAL, and so does
 * letkf_adjoint.  LETKF_E_INVAL also when the layout of the largest domain
 * does not fit the LDS of one workgroup (FP64 with more than about 96 owned
 * nodes, e.g. 10 x 10 domains without a halo). */
int letkf_create(const letkf_config *cfgs, int32_t n_instances, int32_t device,
                 letkf_handle **out);
void letkf_destroy(letkf_handle *h);
const char *letkf_strerror(int code);
const char *letkf_last_error(void);

int letkf_query(letkf_handle *h, int32_t instance, letkf_sizes *out);

/* Host-only planning of one configuration (no device work): the sizes and
 * integer maps letkf_create would build, for checks and for callers that size
 * their buffers first.  Array arguments as in letkf_geometry; pass NULL for
 * every array to get the sizes only. */
int letkf_plan(const letkf_config *cfg, letkf_sizes *sizes, int32_t *node_ij, int32_t *owner,
               int32_t *obs_off, int32_t *obs_idx, int32_t *own_off, int32_t *own_idx);

/* Integer maps of one instance (host buffers, any may be NULL), following the
 * partition of Sec. 4.1 (the pupil cut into local domains, each with the
 * observation region that surrounds it) on the Fried geometry of App. B:
 * node_ij[2n] grid (row, column) of each node; owner[n] domain of each node;
 * obs_off[nd+1] / obs_idx[obs_total] the local slope list of each domain
 * (global slope numbers, the rows of the local observation operator of
 * Sec. 4.2); own_off[nd+1] / own_idx[n] its owned nodes.  Bit-exact with
 * letkf_plan.  LETKF_E_INVAL for a bad handle or instance. */
int letkf_geometry(letkf_handle *h, int32_t instance, int32_t *node_ij, int32_t *owner,
                   int32_t *obs_off, int32_t *obs_idx, int32_t *own_off, int32_t *own_idx);

/* Forecast X_b = a X_a + V (Sec. 3.1.2).  V_dev: ensemble layout, or NULL to
 * draw V from each instance's noise bank (LETKF_E_INVAL if it has none).
 * Advances the frame counter. */
int letkf_forecast(letkf_handle *h, const void *V_dev, void *stream);

/* Analysis of X_b with the slopes y_dev (all instances concatenated), all
 * domains of all instances in one launch; the owned rows form X_a.  Per
 * domain this is the local update of Sec. 4.2 (the ensemble-transform form of
 * Sec. 3.1.1 restricted to the domain's observation region: A~, w, W as in
 * the preamble), then the concatenation of the owned rows and, when enabled,
 * the differential-piston step of Sec. 4.4.  y_dev: device slopes, element
 * type of the handle.  LETKF_E_STATE before a letkf_forecast; per-domain
 * failures (non-finite slopes, no convergence) keep that domain's forecast
 * and are reported by letkf_status, not by the return code. */
int letkf_analyse(letkf_handle *h, const void *y_dev, void *stream);

/* One whole frame: the member prediction of Sec. 3.1.2 (X_b = a X_a + V)
 * fused into the local analyses of Sec. 4.2 (each domain forms its own node
 * patch of X_b), the concatenation and the Sec. 4.4 piston step, replayed
 * from a HIP graph built on the first call (or launched directly, per
 * letkf_set_schedule).  V_dev: device ensemble-layout noise, or NULL to draw
 * it from the noise bank; y_dev: device slopes.  Advances the frame counter.
 * Errors as letkf_analyse. */
int letkf_step(letkf_handle *h, const void *V_dev, const void *y_dev, void *stream);

/* The same frame without batching: one launch per domain, no graph. */
int letkf_step_plain(letkf_handle *h, const void *V_dev, const void *y_dev, void *stream);

/* Copy the analysis ensemble / its member mean ([node] per instance) out, or
 * set the ensemble (restart, tests).  The member mean is the analysis estimate
 * x^ of Sec. 3.1 (with the symmetric square-root transform the members
 * average to it exactly).  on_device != 0: dst/src are device pointers on the
 * handle's device; else host pointers.  Synchronous.  LETKF_E_INVAL for NULL
 * pointers, LETKF_E_DEVICE when a copy fails. */
int letkf_get_ensemble(letkf_handle *h, void *dst, int on_device);
int letkf_set_ensemble(letkf_handle *h, const void *src, int on_device);
int letkf_get_forecast(letkf_handle *h, void *dst, int on_device);
int letkf_get_mean(letkf_handle *h, void *dst, int on_device);

/* Closed loop (LETKF_MODEL_CLOSED_LOOP, Sec. 2.2 control part): the latest
 * command u_k per node of every instance ([sum of n_nodes], element type of
 * the handle; zero for delay-free instances), written by each analysis after
 * the pistons; and the command history (u_{k-1}, u_{k-2}) for exact restarts.
 * Synchronous.  LETKF_E_STATE when no instance runs the closed loop. */
int letkf_get_command(letkf_handle *h, void *dst, int on_device);
int letkf_set_command(letkf_handle *h, const void *u_prev1, const void *u_prev2, int on_device);

/* Frame counter (drives the bank draws): get / set, for exact restarts. */
/* The model each instance's next forecast uses: a[i] (ar_coeff, or the
 * refitted coefficient) and noise_scale[i] (the factor on V; 1 without the
 * refit).  Host arrays of n_instances entries; either may be NULL.  Waits
 * for the device. */
int letkf_get_model(letkf_handle *h, double *a, double *noise_scale);

/* Restart the online refit: sums cleared, a = ar_coeff, noise scale 1.
 * LETKF_E_STATE when no instance refits. */
int letkf_reset_refit(letkf_handle *h);

int letkf_get_frame(letkf_handle *h, uint32_t *frame);
int letkf_set_frame(letkf_handle *h, uint32_t frame);

/* Per-domain status bits of the last analysis, in work-list order mapped back
 * to (instance, domain): flags[sum of domains].  Synchronous.  Returns
 * LETKF_E_NONFINITE / LETKF_E_NOCONV when a domain has that bit set, else
 * LETKF_OK. */
int letkf_status(letkf_handle *h, int32_t *flags);

/* Change rho, r_scale and taper_c of one instance (tuning runs). */
int letkf_set_params(letkf_handle *h, int32_t instance, double rho, double r_scale,
                     double taper_c);

/* Apply the Fried slope operator D (App. B) to one phase vector per
 * instance: phase_dev [node] -> slopes_dev [slope], instances concatenated. */
int letkf_slopes(letkf_handle *h, const void *phase_dev, void *slopes_dev, void *stream);

/* Order in which the workgroups of the analysis launch take the (instance,
 * domain) work items (Sec. 4.1: the domains are independent, so any order
 * gives the same result, bit for bit; only the time changes).
 *   ROW         item = workgroup index.
 *   XCD         the eight XCDs each take a contiguous run of items (the
 *               dispatcher deals workgroups to the XCDs round-robin), so the
 *               overlapping observation regions of neighbouring domains are
 *               read through one L2.
 *   XCD_PAIRED  as XCD, and within each run the items of the second dispatch
 *               round (the workgroups that share a CU with one of the first
 *               round) are the cheapest ones, each paired with the costliest
 *               of them; the items that run alone on a CU are the costliest.
 *               Cost of an item: its transform (m^3), Gram (m^2 p_l) and
 *               staging (m x node patch) work. */
#define LETKF_ORDER_ROW 0
#define LETKF_ORDER_XCD 1
#define LETKF_ORDER_XCD_PAIRED 2

/* Timing knobs picked by letkf_autotune (or set by hand): use_graph (0/1)
 * for letkf_step, and the item order (LETKF_ORDER_*).  No knob changes a
 * result: every work item computes the same values under any schedule.
 * LETKF_E_INVAL for an unknown order. */
int letkf_set_schedule(letkf_handle *h, int32_t use_graph, int32_t order);
int letkf_get_schedule(letkf_handle *h, int32_t *use_graph, int32_t *order);

/* Time letkf_step under every schedule (graph or direct launches x the three
 * item orders) on `stream`, `frames` frames each after one warm-up frame,
 * using the caller's V/y buffers (V_dev NULL: the noise bank), and keep the
 * fastest.  With cache_path != NULL the choice is read from, or appended to,
 * a text file with one line per configuration key (device, precision, work
 * items, m, node patch, observation count, transform, localisation, model,
 * gather mode, AR(2) and refit flags).  The filter state (ensemble, frame
 * counter, AR(2) and command histories, refitted model and its sums) is
 * restored afterwards, on error paths too.  LETKF_E_INVAL for frames < 1 or
 * a NULL y_dev. */
int letkf_autotune(letkf_handle *h, const void *V_dev, const void *y_dev, int32_t frames,
                   const char *cache_path, void *stream);

/* Symmetric positive definite eigensolve by the same FP64 wave-level Jacobi
 * the analysis uses (Cholesky A = L L^T, then one-sided Jacobi rotations of
 * the columns of L until they are orthogonal; their squared norms are the
 * eigenvalues and the normalised columns the eigenvectors).  A_dev: batch
 * row-major m x m FP64 matrices (m <= 64); Q_dev: batch m x m (column k =
 * eigenvector k); lam_dev: batch x m; sweeps_dev: batch int32 sweeps used
 * (NULL allowed).  Eigenvalues are not sorted.  Stateless. */
int letkf_eigh_spd(const double *A_dev, int32_t m, int32_t batch, double tol,
                   int32_t max_sweeps, double *Q_dev, double *lam_dev, int32_t *sweeps_dev,
                   void *stream);

/* Timing of the analysis kernel: with enable != 0, every letkf_step that
 * launches directly (schedule without the graph) records a HIP event pair
 * around its analysis launch on its stream.  letkf_analysis_times waits for
 * them, writes up to `max` durations (ms) in launch order, sets *count to the
 * number recorded and clears the record. */
int letkf_set_timing(letkf_handle *h, int32_t enable);
int letkf_analysis_times(letkf_handle *h, float *ms, int32_t max, int32_t *count);

/* ---------------------------------------------------------------- adjoint
 * Gradient of a loss of the analysis ensembles with respect to each
 * instance's (rho, r_scale, taper_c): the inflation, the noise scale s of
 * Sigma_w = s diag(r) (Sec. 3.1.1) and the Gaspari-Cohn half width of the
 * localisation taper (Sec. 4.1).  The loss provided here is the residual-phase
 * variance of the analysis mean behind the coherent energy of Sec. 5:
 *   var_i = mean over nodes of (e - mean(e))^2,  e = X_a 1 / m - phi,
 * phi the true phase at the nodes ([node] per instance, instances
 * concatenated, element type of the handle).  A caller runs the frames
 * forward, keeps the analysis ensembles it needs (or checkpoints and
 * recomputes them), then walks back one frame at a time.  All pointers are
 * device pointers; all calls are asynchronous on `stream`. */

/* acc_dev[i] += weights_dev[i] * var_i for the analysis ensemble xa_dev
 * (NULL: the handle's current one); weights_dev NULL = 1 for every
 * instance.  acc_dev: n_instances doubles. */
int letkf_residual_variance(letkf_handle *h, const void *xa_dev, const void *truth_dev,
                            const double *weights_dev, double *acc_dev, void *stream);

/* xbar_dev += weights_dev[i] * d var_i / d X_a (ensemble layout). */
int letkf_residual_variance_adjoint(letkf_handle *h, const void *xa_dev, const void *truth_dev,
                                    const double *weights_dev, void *xbar_dev, void *stream);

/* Reverse of the frame that turned xa_prev_dev into the analysis ensemble
 * whose adjoint is in xbar_dev: the forecast a X_prev + V (V_dev, or the
 * instance's noise bank drawn at frame number `frame` when V_dev is NULL) and
 * the analysis with the slopes y_dev are recomputed, then
 *   xbar_dev      <- adjoint of xa_prev_dev (overwritten in place),
 *   theta_bar_dev[3 i + {0, 1, 2}] += d loss / d (rho, r_scale, taper_c) of
 *                    instance i through this frame.
 * Deterministic: slope adjoints of overlapping observation regions are summed
 * in a fixed order.  A domain whose analysis kept its forecast (non-finite
 * input or no convergence) is differentiated as the identity.  The adjoint
 * passes through the eigenvectors themselves, so in FP32 mode its recompute
 * runs the Jacobi to min(jacobi_tol, 1e-6) (the forward's transform W only
 * needs the looser default).  Returns LETKF_E_INVAL when the device cannot
 * give the adjoint kernel its LDS, and for handles with a closed-loop
 * instance, an AR(2) model, the online refit, the blend-mode gather,
 * covariance localisation or the wide analysis (the frame it reverses is the
 * delay-free AR(1) one with the 64-member local analysis and the
 * concatenation). */
int letkf_adjoint(letkf_handle *h, const void *xa_prev_dev, const void *V_dev, uint32_t frame,
                  const void *y_dev, void *xbar_dev, double *theta_bar_dev, void *stream);

/* letkf_adjoint for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, arguments, results (bit for bit) and errors, but the
 * adjoint's per-call buffers (node and slope adjoint slots, per-item partials,
 * which letkf_adjoint allocates on its first call) are taken from a fixed
 * device scratch array of the library, 16 MiB on each device it runs on,
 * held until the process ends.  It calls no hipMalloc or hipFree.  The
 * handle's own buffers (allocated by letkf_create) are used as by
 * letkf_adjoint.  LETKF_E_INVAL, with a message naming the size, when the
 * handle needs more scratch than that (an 80x80, m = 64 instance needs
 * 6.7 MB in FP32 and 13.3 MB in FP64).  Every call on a device shares that
 * device's scratch and leaves its last contents there (every entry a call
 * reads is written by the same call first): calls that overlap on one
 * device, from any handle, stream or thread, race; order them. */
int letkf_adjoint_noalloc(letkf_handle *h, const void *xa_prev_dev, const void *V_dev, uint32_t frame,
                          const void *y_dev, void *xbar_dev, double *theta_bar_dev, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LETKF_H */
