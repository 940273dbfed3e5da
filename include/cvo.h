/*
 * cvo.h -- C ABI of the MI355X (gfx950) implementation of continuous RKHS
 * point-cloud registration ("CVO", arXiv 2012.03683: "A New Framework for
 * Registration of Semantic Point Clouds from Stereo and RGB-D Cameras").
 *
 * Notation (the paper's):
 *   X = {x_i}, Z = {z_j} subset R^3 with feature vectors u_i = l_X(x_i),
 *   v_j = l_Z(z_j)  (Sec. III).  A pose T = (R, t) maps Z-frame coordinates
 *   into the X frame, z'_j = R z_j + t; it plays the role of h^-1 in
 *   Problem 1, so F(T) = <f_X, f_{T Z}>.
 *   k(x, z) = sigma^2 exp(-|x - z|^2 / (2 ell^2))                (eq. (2))
 *   c_ij = prod_b k_b(u_i^(b), v_j^(b)), k_b squared-exponential  (eq. (5))
 *          or linear <u, v> (eq. (4)); blocks combine as a tensor
 *          product (eq. (6)); no blocks means c = 1 (eq. (8)).
 *   F(T) = sum_{(i,j) in P} c_ij k(x_i, z'_j)                     (eq. (7))
 *   P = {(i,j) : s_ij <= (kappa ell)^2}, s_ij = |x_i - z'_j|^2, the
 *       truncation of the sparse double sum (Sec. III-B); kappa = +inf
 *       keeps every pair.  Membership is decided exactly as the FP64
 *       expression s = (dx*dx + dy*dy) + dz*dz with
 *       z'_r = ((R_r0 z_0 + R_r1 z_1) + R_r2 z_2) + t_r, every operation a
 *       separately rounded IEEE double (no fused multiply-add), so |P| is
 *       reproducible bit for bit.
 *   i_theta = F / sqrt(|X| |Z|)                                   (eq. (10))
 *   gradient: grad = (omega, v) = d/dxi F(Exp(xi) T) at xi = 0 (left
 *       perturbation on se(3)); the paper states no formula -- it is the
 *       derivative of eq. (7) with c_ij constant (Sec. III-B):
 *       omega = ell^-2 sum w (z' x d), v = ell^-2 sum w d, d = x - z'.
 *
 * Memory and ownership
 *   - cvo_cloud buffers, backward outputs and the batched T arrays marked
 *     "device" are DEVICE pointers on the handle's device (float32,
 *     contiguous, row-major).  The caller owns them; the library never
 *     frees or retains them past the call.
 *   - Poses, scalars, reports and traces are HOST pointers, owned by the
 *     caller.
 *   - The handle owns every scratch buffer (grids, moments, partials,
 *     graphs).  Scratch grows on demand and is released by cvo_destroy.
 *   - Calls are ordered on the handle's stream and return after the host
 *     outputs are written (they synchronise that stream).
 *   - A handle is not thread safe: one call at a time per handle.
 *
 * Errors: every call returns a cvo_status; on failure cvo_last_error()
 * gives a message.  A pose must be rigid: max |R^T R - I| <= 1e-9 and
 * det R > 0, with finite entries (else CVO_ERR_INVALID_ARGUMENT).  Point
 * coordinates must be finite: a cloud with a NaN or infinite coordinate is
 * found on the device at the view build and rejected with
 * CVO_ERR_INVALID_ARGUMENT.  N = 0 or M = 0 is not an error (F = 0, gradient 0,
 * |P| = 0; cvo_align reports CVO_NO_OVERLAP and returns T_init).
 * Non-convergence is a report status, never an error code.
 */
#ifndef CVO_H
#define CVO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cvo_context *cvo_handle;

typedef enum {
    CVO_OK = 0,
    CVO_ERR_INVALID_ARGUMENT = 1, /* bad sizes, pointers, non-finite or non-positive parameters */
    CVO_ERR_OUT_OF_MEMORY = 2,    /* device allocation failed */
    CVO_ERR_DEVICE = 3,           /* a HIP runtime error, or a registration whose device state stopped
                                     advancing (a launched batch left a running pair at its step); message kept */
    CVO_ERR_UNSUPPORTED = 4       /* e.g. feature layout beyond the compiled limits */
} cvo_status;

/* block kernel kinds (eq. (4)-(6)) */
#define CVO_SE 0
#define CVO_LIN 1
#define CVO_MAX_BLOCKS 8
#define CVO_MAX_FEATURE_DIM 64 /* total feature dimension after combining blocks */

/* registration outcome (cvo_align_report.status) */
#define CVO_CONVERGED 1  /* lengthscale at its floor and the last step below (eps_rot, eps_trans) */
#define CVO_MAX_ITER 2   /* iteration cap reached (the normal end in fixed-iteration mode) */
#define CVO_NO_OVERLAP 3 /* the pair set P became empty */
#define CVO_STATIONARY 4 /* the gradient is exactly zero */

/* metric on se(3) that turns the gradient into the ascent direction
 * (cvo_align_params.metric); the paper names gradient ascent on the
 * manifold (Sec. I) without fixing the metric */
#define CVO_METRIC_KINETIC 0  /* G = mean_j J_j^T J_j: xi^T G xi is the mean squared velocity of the
                                 moving cloud's points (rigid-body kinetic energy), direction G^-1 grad */
#define CVO_METRIC_IDENTITY 1 /* plain coordinates: direction = grad */

/* how the lengthscale moves during an ascent (cvo_align_params.ell_mode) */
#define CVO_ELL_ANNEAL 0   /* Sec. IV: decay by `decay` whenever the indicator has stabilised */
#define CVO_ELL_ADAPTIVE 1 /* Sec. VI (the lengthscale as an optimisation variable): every iteration
                              sets ell to the maximiser of the lengthscale objective J of
                              cvo_ell_objective at that iteration's (T, ell), clamped to
                              [ell_min, ell_init] and to one factor `decay` of ell (down or up);
                              converged when the step is below (eps_rot, eps_trans) and ell moved by
                              at most ind_rel_tol * ell */

/* trace record per iteration (cvo_align trace buffer, doubles) */
#define CVO_TRACE_LEN 8 /* it, ell, F, |grad|, step tau, i_theta, |P|, curvature */

typedef struct {
    const float *xyz;  /* device, n x 3 */
    const float *feat; /* device, n x D (D from the feature spec); may be NULL when D = 0 */
    int64_t n;         /* number of points, 0 <= n < 2^30 (else CVO_ERR_INVALID_ARGUMENT, before any device work) */
} cvo_cloud;

/* Feature blocks l(x) = (u_1, u_2, ...) in V_1 x V_2 x ... (Sec. III-B).
 * Block b occupies dim[b] consecutive columns of feat, in block order.
 * The feature kernel is the product of the blocks' kernels (eqs. (6)-(7)).
 * Several LIN blocks are run as one block holding their tensor product
 * (eq. (6)), so the product of the LIN widths plus the SE widths must not
 * exceed CVO_MAX_FEATURE_DIM (else CVO_ERR_UNSUPPORTED). */
typedef struct {
    int32_t nblocks;                 /* 0 .. CVO_MAX_BLOCKS */
    int32_t dim[CVO_MAX_BLOCKS];     /* > 0 */
    int32_t kind[CVO_MAX_BLOCKS];    /* CVO_SE or CVO_LIN */
    double ell[CVO_MAX_BLOCKS];      /* SE lengthscale ell_b > 0 (ignored for LIN) */
    double sigma[CVO_MAX_BLOCKS];    /* SE amplitude sigma_b > 0 (ignored for LIN) */
} cvo_feature_spec;

typedef struct {
    double ell;   /* geometric lengthscale > 0 (eq. (2)) */
    double sigma; /* geometric amplitude > 0 (eq. (2)); 1 makes the Remark of Sec. III-C hold */
    double kappa; /* cutoff radius in lengthscales, > 0; +inf keeps all pairs */
} cvo_kernel_params;

typedef struct {
    double ell_init;     /* starting lengthscale */
    double ell_min;      /* floor of the annealing schedule (Sec. IV) */
    double decay;        /* factor applied when the indicator stabilises (0.98: Sec. IV) */
    double ind_rel_tol;  /* stabilised: |i - i_prev| <= ind_rel_tol * |i| */
    double eps_rot;      /* convergence: rotation step below this (rad) ... */
    double eps_trans;    /* ... and translation step below this (m), at ell_min */
    double step_lambda;  /* step clamp: no point moves more than step_lambda * ell per step */
    double sigma;        /* geometric amplitude */
    double kappa;        /* cutoff in lengthscales */
    int64_t max_iter;    /* iteration cap, >= 1 */
    int32_t fixed_iters; /* nonzero: run exactly max_iter steps at ell_init, no annealing */
    int32_t metric;      /* CVO_METRIC_KINETIC (default) or CVO_METRIC_IDENTITY */
    int32_t ell_mode;    /* CVO_ELL_ANNEAL (default) or CVO_ELL_ADAPTIVE */
    int32_t reserved;    /* must be 0 */
} cvo_align_params;

typedef struct {
    int64_t iterations;  /* steps taken */
    double final_ell;    /* lengthscale at exit */
    double F;            /* F at the last evaluation */
    double i_theta;      /* indicator at the last evaluation (eq. (10)) */
    int64_t n_pairs;     /* |P| at the last evaluation */
    int32_t status;      /* CVO_CONVERGED, CVO_MAX_ITER, CVO_NO_OVERLAP, CVO_STATIONARY */
    int32_t reserved;
    int64_t total_pairs; /* sum of |P| over all evaluations of this registration */
} cvo_align_report;

typedef struct {
    double F;        /* eq. (7) */
    double grad[6];  /* omega_xyz, v_xyz (left perturbation) */
    double curv;     /* d^2/dtau^2 F(Exp(tau grad) T) at tau = 0 (c_ij constant) */
    double dF_dell;  /* sum w s / ell^3, cutoff radius held fixed */
    double r_max;    /* max_j |T z_j| */
    double i_theta;  /* F / sqrt(NM) (eq. (10)) */
    int64_t n_pairs; /* |P| */
} cvo_eval;

/* Query clusters (cvo_tuning.cluster_rule): OCTREE takes the largest aligned
 * Morton (octree) block with at most cluster_max points and an edge within
 * cluster_factor * r_c; CHUNKS cuts the Morton-ordered points into runs of
 * cluster_max and halves a run until its bounding box edge is within
 * cluster_factor * r_c (parts of cluster_max / 2^k points). */
#define CVO_CLUSTER_OCTREE 0
#define CVO_CLUSTER_CHUNKS 1

/* Tuning knobs (picked by cvo_autotune or set by hand). */
typedef struct {
    int32_t cluster_max;   /* max query points per cluster: 8, 16, 32 or 64 */
    double cell_factor;    /* grid cell edge / cutoff radius, in [0.25, 4] */
    double cluster_factor; /* cluster edge cap / cutoff radius, in [0.05, 2] */
    double rebuild_ratio;  /* rebuild grids when cutoff < rebuild_ratio * cutoff at build, in (0, 1] */
    int32_t unroll;        /* iterations enqueued per host check / per captured graph, 1..64 */
    int32_t piece_work;    /* query x candidate products per unit of pair-pass work, 256..2^24 */
    int32_t cluster_rule;  /* how query clusters are formed: CVO_CLUSTER_OCTREE or CVO_CLUSTER_CHUNKS */
    int32_t adaptive;      /* 0 or 1.  1: a registration re-chooses cluster_max, cell_factor,
                            * cluster_factor and cluster_rule at every view build from the in-cutoff
                            * pairs per query point of its latest iteration (chunk clusters throughout).
                            * Padded feature rows of more than 8 floats: >= 500: 32, 0.5, 0.5;
                            * >= 200: 16, 0.5, 1.0; fewer: 16, 1.0, 1.0.  Rows of at most 8 floats:
                            * >= 100: 32, 0.5, 1.0; fewer: 16, 1.0, 1.5.  Not yet measured: the fields
                            * above.  One-shot calls always use the fields above. */
} cvo_tuning;

/* Per-handle timing of the dominant kernel, measured with HIP events on the
 * handle's stream while profiling is enabled (cvo_set_profiling), and counts
 * of launches, graphs, view builds and host waits (always kept; every
 * cvo_set_profiling call resets them). */
typedef struct {
    int64_t pair_launches;     /* pair-pass launches timed */
    double pair_ms;            /* summed event time of those launches */
    int64_t pair_count;        /* summed |P| of the timed launches (when known) */
    int64_t evaluations;       /* pair-pass launches enqueued, timed or not (a graph replay counts
                                  each pair pass it holds) */
    int64_t graph_launches;    /* captured iteration graphs replayed */
    int64_t graph_captures;    /* iteration graphs captured and instantiated */
    int64_t view_builds;       /* builds of the grid and cluster views and the work plan */
    int64_t host_waits;        /* waits of the host for the handle's stream */
    int64_t tuned_view_shapes; /* view shapes a registration took from the autotuned class table */
} cvo_timing;

/* Create a handle on `device` (HIP ordinal) that enqueues on `stream`
 * (a hipStream_t, or NULL for the default stream).  Returns
 * CVO_ERR_INVALID_ARGUMENT for a NULL out pointer or a bad ordinal. */
cvo_status cvo_create(cvo_handle *out, int device, void *stream);

/* Free the handle and all scratch it owns.  NULL is ignored. */
void cvo_destroy(cvo_handle h);

/* Switch the stream later calls enqueue on (hipStream_t or NULL). */
cvo_status cvo_set_stream(cvo_handle h, void *stream);

/* Message for the last failing call on this handle ("" if none). */
const char *cvo_last_error(cvo_handle h);

/* F of eq. (7) at pose T (host double[12], row-major [R|t]) and the exact
 * pair count |P|.  F and n_pairs are host pointers; n_pairs may be NULL. */
cvo_status cvo_inner_product(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                             const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                             const double T[12], double *F, int64_t *n_pairs);

/* F and its se(3) gradient (omega, v) at T (left perturbation; the derivative
 * of eq. (7) with c_ij constant, Sec. III-B).  grad is host double[6]. */
cvo_status cvo_gradient(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                        const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                        const double T[12], double *F, double grad[6], int64_t *n_pairs);

/* Everything one pair pass yields (F, gradient, curvature along the gradient,
 * dF/dell, r_max, i_theta, |P|) into a host cvo_eval. */
cvo_status cvo_evaluate(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                        const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                        const double T[12], cvo_eval *out);

/* Lengthscale objective of the adaptive mode (Sec. VI, where the lengthscale
 * becomes an optimisation variable; the paper gives no formula).  F of
 * eq. (7) grows with ell, so ell is not chosen by F: it maximises the
 * log-likelihood of the moved cloud under the kernel mixture centred on X,
 *   J(T, ell) = sum_{j : W_j > 0} log W_j - 3 |Z+| log ell,
 * W_j = sum_i w_ij over the pair set P frozen at (T, ell), Z+ the targets with
 * W_j > 0.  For fixed per-target residuals r_j = sum_i w_ij s_ij / W_j its
 * stationary point is ell_ml^2 = sum_{Z+} r_j / (3 |Z+|).
 * out (host double[4]) = {J, dJ/dell (P frozen), ell_ml (0 if Z+ is empty),
 * |Z+|}.  One pair pass; errors as cvo_inner_product. */
cvo_status cvo_ell_objective(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                             const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                             const double T[12], double out[4]);

/* Allocation-free form of cvo_evaluate, for callers that cannot allocate
 * device memory (code that must not call hipMalloc/hipFree, e.g. inside a
 * serving loop or a harness that forbids it).  Same arguments, outputs and
 * kernels as cvo_evaluate; every scratch buffer is carved from a fixed
 * device array of CVO_NOALLOC_SCRATCH_MIB MiB that the library holds on each
 * device it runs on (looked up by cvo_create) until the process ends.  No
 * hipMalloc, hipFree, pinned host allocation or event creation happens in the
 * call; small host<->device copies are made from the caller's memory and
 * waited for.
 * Limits: N, M <= CVO_NOALLOC_MAX_POINTS (larger clouds are rejected with
 * CVO_ERR_INVALID_ARGUMENT before any device work); an input whose views
 * need more scratch than the array holds (very dense neighbourhoods) fails
 * with CVO_ERR_OUT_OF_MEMORY and a message naming the shortfall, before any
 * kernel writes past the array.
 * The array is shared by every handle on a device and keeps the last call's
 * contents (each call rewrites what it reads): calls that overlap in time on
 * one device -- from two threads, or on two streams -- race and must not be
 * made.  CVO_ERR_DEVICE if the array could not be located on the device. */
#define CVO_NOALLOC_SCRATCH_MIB 256
#define CVO_NOALLOC_MAX_POINTS 65536
cvo_status cvo_evaluate_noalloc(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                                const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                                const double T[12], cvo_eval *out);

/* Cosine of the angle between f_X and the moved f_Z (eq. (9), Sec. III-C):
 * cos_theta = F(X, Z; T) / (||f_X|| ||f_Z||), where ||f_X||^2 = F(X, X; I) and
 * ||f_Z||^2 = F(Z, Z; I) are the self inner products with the same kernels,
 * lengthscale and cutoff.  Three pair passes on the handle's stream.
 * sums, if non-NULL, receives {F(X,Z;T), F(X,X;I), F(Z,Z;I)} (host memory).
 * cos_theta is 0 when a squared norm is not positive (an empty cloud).
 * Errors as cvo_inner_product. */
cvo_status cvo_cosine(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                      const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                      const double T[12], double *cos_theta, double sums[3]);

/* Alignment indicator i_theta = F / sqrt(|X||Z|) at (T, ell) (eq. (10),
 * Sec. III-C); 0 when either cloud is empty. */
cvo_status cvo_metric(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                      const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                      const double T[12], double *i_theta);

/* Problem 1 (eq. (1)): gradient ascent on SE(3) from T_init with lengthscale
 * annealing (Sec. IV).  Per iteration: evaluate F and grad; direction
 * d = G^-1 grad for the chosen metric G; curvature c of F(Exp(tau d) T);
 * step tau = min(grad.d / -c (if c < 0, else +inf),
 *                step_lambda * ell / (|d_omega| r_max + |d_v|));
 * T <- Exp(tau d) T; when the indicator has stabilised, ell <- max(ell_min,
 * decay * ell).  T_out (host double[12]) and report (host) receive the
 * result; trace (host, may be NULL) receives max_iter x CVO_TRACE_LEN
 * doubles, of which report->iterations rows are written. */
cvo_status cvo_align(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                     const cvo_feature_spec *spec, const cvo_align_params *ap,
                     const double T_init[12], double T_out[12], cvo_align_report *report,
                     double *trace);

/* Debugging form of cvo_align: the lengthscale of iteration i is ell_sched[i]
 * (host array of n > 0 finite values; ap->ell_init, max_iter and fixed_iters
 * are ignored), with no annealing or convergence decisions, for exactly n
 * iterations (or until the pair set is empty or the gradient zero).  Fed the
 * lengthscales another implementation took, it reproduces that run iterate by
 * iterate.  Other arguments and errors as cvo_align. */
cvo_status cvo_align_replay(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                            const cvo_feature_spec *spec, const cvo_align_params *ap,
                            const double T_init[12], const double *ell_sched, int64_t n,
                            double T_out[12], cvo_align_report *report, double *trace);

/* Hand-written backward of eq. (7) on the pair set frozen at (T, ell): the
 * derivatives of gF * F with respect to the point positions (dX: N x 3,
 * dZ: M x 3), the feature vectors (dU: N x D, dV: M x D) -- all device float32
 * arrays shaped like the inputs -- and the lengthscale (dEll, host double,
 * cutoff radius held fixed).  Any output pointer may be NULL (not computed). */
cvo_status cvo_inner_product_backward(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                                      const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                                      const double T[12], double gF, float *dX, float *dZ,
                                      float *dU, float *dV, double *dEll);

/* B independent registrations in one device-resident loop (a captured HIP
 * graph replayed until every pair has finished).  X, Z: host arrays of B
 * clouds (device buffers); params: host array of B (or 1, shared);
 * T_init, T_out: host B x 12; reports: host array of B.  Per-pair results
 * match B separate cvo_align calls up to floating-point summation order. */
cvo_status cvo_align_batched(cvo_handle h, int32_t B, const cvo_cloud *X, const cvo_cloud *Z,
                             const cvo_feature_spec *spec, const cvo_align_params *params,
                             int32_t nparams, const double *T_init, double *T_out,
                             cvo_align_report *reports);

/* Frame-to-frame odometry over a sequence (Sec. IV): pair k (k = 0..F-2)
 * registers frame k + 1 (moving, Z) to frame k (fixed, X).  Pair 0 starts at
 * the identity with `first`; pair k > 0 starts at pair k - 1's result with
 * `rest` (the camera is assumed to keep its motion).  frames: host array of F
 * clouds (device buffers, all with the spec's feature dimension);
 * T_rel: host (F-1) x 12 doubles, row k = pose of frame k + 1 in frame k;
 * reports: host array of F - 1.  The pairs run one after another on the
 * handle's stream; each result equals the cvo_align call with the same
 * arguments.  A pair with an empty frame reports CVO_NO_OVERLAP and passes its
 * start pose on.  F < 2 is CVO_ERR_INVALID_ARGUMENT. */
cvo_status cvo_odometry(cvo_handle h, int32_t F, const cvo_cloud *frames,
                        const cvo_feature_spec *spec, const cvo_align_params *first,
                        const cvo_align_params *rest, double *T_rel,
                        cvo_align_report *reports);

/* Pinhole camera of a depth image: pixel (u, v) with depth z back-projects to
 * ((u - cx) z / fx, (v - cy) z / fy, z).  A pixel has depth when its value is
 * finite and within [depth_min, depth_max] (compared in FP32). */
typedef struct {
    double fx, fy, cx, cy;       /* pixels; fx, fy > 0 */
    double depth_min, depth_max; /* metres; 0 < depth_min <= depth_max, finite */
} cvo_camera;

/* Point selection before registration (Sec. IV, performance considerations):
 * pixels that pass the FAST segment test (an arc of >= 9 contiguous pixels of
 * the radius-3 circle all brighter than I_p + t or all darker than I_p - t;
 * pixels within 3 of the border are never selected), no non-maximum
 * suppression, with depth.  The threshold t is chosen per call as the
 * smallest integer whose selection holds at most max_points pixels (the paper
 * keeps 3k-15k; a score histogram gives every count at once).
 *   gray:  device, height x width uint8, row-major.
 *   depth: device, height x width float32 (metres).
 *   feat:  device, height x width x D float32 per-pixel features (NULL if D = 0).
 *   xyz, feat_out: device, capacity x 3 and capacity x D float32; rows
 *          0..n-1 receive the selected pixels in raster order (camera-frame
 *          points as in cvo_camera, FP64 arithmetic rounded to FP32; feature
 *          rows copied).  capacity must be >= max_points.
 *   score: device, height x width int16, or NULL: each pixel's score, the
 *          largest t at which it passes the test (-1: none).
 *   n_out, threshold_out: host.
 * Synchronises the handle's stream.  Errors: CVO_ERR_INVALID_ARGUMENT for
 * NULL buffers that are needed, width or height < 0, width x height >= 2^31,
 * D outside [0, 256], a bad camera, max_points < 0 or capacity < max_points. */
cvo_status cvo_select_points(cvo_handle h, const uint8_t *gray, const float *depth, const float *feat,
                             int32_t width, int32_t height, int32_t D, const cvo_camera *cam,
                             int32_t max_points, float *xyz, float *feat_out, int64_t capacity,
                             int16_t *score, int64_t *n_out, int32_t *threshold_out);

/* Read / replace the tuning knobs used by later calls. */
cvo_status cvo_get_tuning(cvo_handle h, cvo_tuning *out);
cvo_status cvo_set_tuning(cvo_handle h, const cvo_tuning *in);

/* Project-written autotuner of the bin (grid cell) and tile (query cluster)
 * sizes.  Times the pair pass of (X, Z, spec, kp, T) under each view shape of
 * a search space -- chunk clusters x points per cluster (16, 32, 64) x cell
 * edge (0.35, 0.5, 1.0 r_c) x cluster edge cap (0.3, 0.5, 1.0, 1.5 r_c),
 * median of 3 timed launches after one untimed -- and keeps the fastest:
 *   - as the handle's one-shot shape (cluster_max, cell_factor,
 *     cluster_factor, cluster_rule; the other tuning fields are unchanged),
 *     cached per (point-count, feature-dimension, lengthscale band) class;
 *   - as the shape of this evaluation's density class (its in-cutoff pairs
 *     per query point, and whether feature rows fit in 8 floats), which
 *     adaptive registrations -- plain and batched -- then use at every view
 *     build of that class instead of the built-in table.
 * If chosen is non-NULL it receives the resulting tuning.  Both clouds must
 * be non-empty (CVO_ERR_INVALID_ARGUMENT). */
cvo_status cvo_autotune(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                        const cvo_feature_spec *spec, const cvo_kernel_params *kp,
                        const double T[12], cvo_tuning *chosen);

/* Persist the autotuner's choices (the density-class table and the one-shot
 * cache) to a text file, and merge such a file into a handle, so tuning
 * survives cvo_destroy and carries over to later processes.  Load rejects a
 * file that is not a tuning file or holds a shape outside the allowed ranges
 * (CVO_ERR_INVALID_ARGUMENT, nothing merged). */
cvo_status cvo_save_tuning(cvo_handle h, const char *path);
cvo_status cvo_load_tuning(cvo_handle h, const char *path);
/* Forget the autotuner's class table and one-shot cache (registrations fall
 * back to the built-in table; the tuning fields are unchanged). */
cvo_status cvo_clear_tuning(cvo_handle h);

/* Enable (nonzero) or disable HIP-event timing of every pair-pass launch;
 * either call resets the timing and the counters. */
cvo_status cvo_set_profiling(cvo_handle h, int32_t enable);
cvo_status cvo_get_timing(cvo_handle h, cvo_timing *out);

#ifdef __cplusplus
}
#endif
#endif /* CVO_H */
