/*
 * purse.h -- C ABI of the MI355X (gfx950) PURSE boundary sampler and MEGB.
 *
 * The operation is the inner approximation of the minimum enclosing geodesic
 * ball (MEGB) of a pose uncertainty set (PURSE) from "CLOSURE: Fast
 * Quantification of Pose Uncertainty Sets" (arXiv 2403.09990):
 *
 *   S = { x = (R, t) in SE(3) : ||g(x, y_i)||_{Lambda_i} <= beta_i, i = 1..N }
 *
 * (eq. PURSE; the 2D-3D form eq. PURSE2D3D with g = z_i - Pi(R Z_i + t), the
 * 3D-3D form eq. PURSE3D3D with g = b_i - (R a_i + t)).  purse_sample draws
 * boundary samples of S with independent randomly started trajectories;
 * purse_megb returns the centre pose and the rotation / translation radii of
 * the geodesic balls enclosing the samples (Section "Minimum Enclosing
 * Geodesic Ball", eqs. megb-rot and megb-tran, Proposition 1); purse_megb_backward
 * returns the gradient of those outputs with respect to the measurements.
 *
 * Conventions for every entry point:
 *  - Pointers named in purse_batch and the array arguments are DEVICE
 *    pointers owned by the caller; the library never frees or keeps them.
 *  - Scalars (n_inst, totals, params) are read on the host during the call.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) and performs no host synchronisation and no device allocation:
 *    scratch comes from the caller's workspace `ws` of at least
 *    purse_workspace_size() bytes, 256-byte aligned.
 *  - Return values: PURSE_OK, or a negative PURSE_E_* code for API misuse
 *    detected synchronously on the host (nothing is launched).  Data-dependent
 *    per-instance outcomes are written asynchronously to inst_status.
 *  - Concurrent calls sharing one workspace race; give each in-flight call
 *    its own workspace.
 *  - purse_megb_backward runs part of its work (the frame tangents, then the
 *    3D-3D reverse sweeps) on an auxiliary stream of the current device, and
 *    purse_sample two of its three trajectory launch groups on two others
 *    (default priority; created with their events on the first call and kept
 *    until the process ends), forked from and joined back to `stream` by
 *    events, so every call stays ordered on `stream` and can be captured in a
 *    graph once that first call has happened outside capture.
 */
#ifndef PURSE_H
#define PURSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t purse_status;

#define PURSE_OK 0
#define PURSE_E_NULL (-1)      /* a required pointer is NULL */
#define PURSE_E_BAD_ARG (-2)   /* a host scalar or parameter is out of range */
#define PURSE_E_WORKSPACE (-3) /* workspace too small or misaligned */
#define PURSE_E_NO_DEVICE (-4) /* no usable HIP device */
#define PURSE_E_HIP (-5)       /* a HIP runtime call failed; see purse_last_error */

/* Per-instance status (low byte) and flags. */
#define PURSE_INST_OK 0
#define PURSE_INST_EMPTY 1          /* no feasible sample: MEGB radii are NaN */
#define PURSE_INST_BAD_SHAPE 2      /* Lambda not SPD, beta < 0, non-finite data, fx or fy <= 0 */
#define PURSE_INST_FIT_FAILED 3     /* centre fit failed (depth <= z_min or singular normal matrix) */
#define PURSE_INST_BAD_SIZE 4       /* N < 3 (3D-3D), N < 6 (2D-3D), N > PURSE_MAX_KP, or M < 1 */
#define PURSE_INST_NO_ANCHOR (1 << 8)        /* no feasible anchor: infeasible ends are dropped */
#define PURSE_INST_ANCHOR_ITERATED (1 << 9)  /* the centre was not inside; the anchor was iterated */

/* Per-sample mask bits (uint8). */
#define PURSE_MASK_FEASIBLE 1  /* the sample is in S and feeds the MEGB */
#define PURSE_MASK_PULLED_IN 2 /* the trajectory ended outside S and was pulled back by bisection */
#define PURSE_MASK_FAILED 4    /* a 2D-3D Gauss-Newton step failed; the sample is dropped */

#define PURSE_KIND_3D3D 0 /* balls around target points b_i (eq. PURSE3D3D, Lambda_i = I) */
#define PURSE_KIND_2D3D 1 /* ellipses around image points z_i (eq. PURSE2D3D) */
#define PURSE_KIND_REG 2  /* pose regression (eq. PURSEregression): keypoint i is pose hypothesis i,
                             with centres[i] = t_i (m), shapes[i] = R_i as a unit quaternion
                             (w, x, y, z), model_pts[i][0] = beta_i^R (bound on ||R - R_i||_F),
                             bounds[i] = beta_i^t (bound on ||t - t_i||, m).  Accepted by purse_init,
                             purse_walk and purse_megb (which takes any poses); purse_sample reports
                             it as PURSE_INST_BAD_SIZE */

#define PURSE_MAX_KP 64

/* Flags (purse_params.flags): debugging and schedule choices. */
#define PURSE_FLAG_FORCE_FP64_POLAR 1 /* always take the float64 3x3 polar step */
#define PURSE_FLAG_NO_PRUNING 2       /* MEGB: scan every feasible sample at every step */
#define PURSE_FLAG_REUSE_PROLOGUE 4   /* purse_sample: keep the per-instance centre fit and anchor that a
                                         previous purse_sample call with the same batch and params left
                                         in this workspace (draws more trajectories without refitting;
                                         inst_status is left as that call wrote it) */
#define PURSE_FLAG_INSTANCE_ORDER 8   /* purse_sample: run the tiles in instance order instead of the
                                         default heaviest-first order (results are identical; this only
                                         changes the schedule, for tuning) */
#define PURSE_FLAG_GENERIC_LOOP 16    /* purse_sample: use the general keypoint loop even when every
                                         instance has at most 16 keypoints (for tuning) */
#define PURSE_FLAG_PAIR_LANES 32      /* purse_sample: 2D-3D instances of at most 16 keypoints run each
                                         trajectory on two lanes (twice the wavefronts, for batches too
                                         small to fill the GPU); results agree with one lane per
                                         trajectory to float32 rounding */
#define PURSE_FLAG_QUAD_LANES 128     /* purse_sample: as PURSE_FLAG_PAIR_LANES with four lanes per
                                         trajectory (takes precedence over it) */
#define PURSE_FLAG_REPLAY_DESCENT 64  /* purse_megb_backward: replay the MEGB descent from the trace even
                                         when purse_megb left its checkpoints for this trace in the
                                         workspace (same results; for testing) */
#define PURSE_FLAG_EXACT_MEB 512      /* purse_megb: after the descent, replace its centre by the exact
                                         minimum enclosing ball (Step III): translations in R^3 and rotations
                                         as hemisphere-aligned unit quaternions in R^4, float64; the radii are
                                         then taken about that centre.  purse_megb_backward differentiates
                                         the descent, so it rejects this flag */
#define PURSE_FLAG_MATRIX_COTANGENT 256 /* purse_megb_backward: g_centre is [n_inst][12], the cotangent of the
                                           centre's entries as purse_megb returns them (R* row-major, then
                                           t*); its rotation part is taken along SO(3) at R* */
#define PURSE_FLAG_WORK_QUEUE 2048 /* purse_sample: persistent trajectory kernels, about eight
                                     wavefronts per SIMD, each workgroup taking its next tile of the
                                     heaviest-first schedule from an atomic counter until none is left
                                     (the same samples; speed only) */
#define PURSE_FLAG_FORWARD_TANGENTS 1024 /* purse_megb_backward: differentiate the trajectories in
                                           forward mode, one float32 re-run per input direction (6N or 4N
                                           per active sample), instead of one reverse sweep per active
                                           sample (the default while the sweep's tape and decisions fit
                                           64 KB of LDS: 2D-3D up to about 280 Gauss-Newton passes, 3D-3D
                                           up to 256 iterations); the reverse sweep takes its decisions
                                           from a float64 recomputation, the forward mode from float32
                                           ones, so the two differ where a decision sits within float32
                                           rounding of its threshold */
#define PURSE_FLAG_SERIAL_GROUPS 4096 /* purse_sample: launch the three trajectory launch groups (3D-3D;
                                        2D-3D with the unrolled or lane-group loop; 2D-3D with the
                                        general loop) one after the other on the caller's stream instead
                                        of concurrently on it and two auxiliary streams (the same
                                        samples; speed only) */

/*
 * A ragged batch of PURSE instances.  Instance j owns keypoints
 * [kp_off[j], kp_off[j+1]) and samples [sample_off[j], sample_off[j+1]).
 */
typedef struct purse_batch {
  int32_t n_inst;         /* host: number of instances, >= 1 */
  int32_t max_kp;         /* host: max over instances of N_j, 3..PURSE_MAX_KP */
  int64_t total_kp;       /* host: sum of N_j */
  int64_t total_samples;  /* host: sum of M_j */
  int64_t max_samples;    /* host: max over instances of M_j */
  const int32_t *kind;        /* [n_inst] PURSE_KIND_* */
  const int32_t *n_kp;        /* [n_inst] N_j */
  const int64_t *kp_off;      /* [n_inst+1] prefix sums of N_j */
  const int64_t *sample_off;  /* [n_inst+1] prefix sums of M_j */
  const float *model_pts;     /* [total_kp][3] a_i or Z_i, metres, model frame */
  const float *centres;       /* [total_kp][3] b_i (m) | (z_i.x, z_i.y, unused) (px) */
  const float *shapes;        /* [total_kp][4] Lambda_i row-major (2D-3D, px^-2); ignored for 3D-3D */
  const float *bounds;        /* [total_kp] beta_i >= 0 (m for 3D-3D, Lambda-units for 2D-3D) */
  const float *intrinsics;    /* [n_inst][4] fx, fy, cx, cy (2D-3D; ignored for 3D-3D) */
  const uint64_t *seed;       /* [n_inst] Philox key word of each instance */
} purse_batch;

/* Method parameters (see purse_default_params for the defaults). */
typedef struct purse_params {
  int32_t n_iters;     /* alternating iterations per trajectory (>= 0) */
  int32_t n_gn;        /* Gauss-Newton steps per 2D-3D refit (>= 1) */
  int32_t n_bis;       /* bisection steps of the pull-in (0..30) */
  int32_t megb_iters;  /* geodesic descent steps T (>= 1) */
  int32_t megb_avg;    /* iterates averaged for the centre (1..T) */
  float omega0;        /* initial angular offset (rad) of rotation-seeking trajectories */
  float v0;            /* initial centre offset (m) of translation-seeking trajectories */
  float kappa;         /* projection shrink factor in (0, 1] */
  float tau_abs_3d;    /* feasibility tolerance, metres */
  float tau_abs_2d;    /* feasibility tolerance, Lambda-units */
  float z_min;         /* minimum valid depth for 2D-3D (m) */
  int32_t ckpt_every;  /* checkpoint spacing of the backward recompute (>= 1) */
  int32_t centre_gn;   /* cap on the Gauss-Newton steps of the 2D-3D centre fit, which
                          stops once the step is below 1e-13 (rotation, rad) and
                          1e-13 (1 + |t|_inf) (translation, m) */
  int32_t tile;        /* samples per workgroup: 64, 128 or 256; 0 = library choice (256) */
  int32_t flags;       /* PURSE_FLAG_* */
  int32_t waves_per_simd; /* purse_sample: cap on the trajectory kernels' resident wavefronts per SIMD
                             (1..8, by padding each workgroup's LDS within the per-workgroup limit; the
                             allocation granularity can leave a workgroup fewer); 0 = no cap.  Speed only */
} purse_params;

/* Fill *p with the defaults: n_iters 50, n_gn 2, n_bis 16, megb_iters 4096,
 * megb_avg 10, omega0 0.5, v0 0.2, kappa 0.999, tau 1e-5 / 1e-4, z_min 1e-3,
 * ckpt_every 5, centre_gn 50, tile 0, flags 0.  Returns PURSE_E_NULL if p is NULL. */
purse_status purse_default_params(purse_params *p);

/* Bytes of workspace every call below needs for this batch and params. */
purse_status purse_workspace_size(const purse_batch *b, const purse_params *p, size_t *bytes);

/*
 * Boundary samples of every instance (the alternating projection sampler
 * built from Section "Geometric Structures" and Step I / Step II of
 * Section "The CLOSURE Algorithm").  Per instance: centre fit (Arun's method
 * for 3D-3D; DLT and weak-perspective starts, Gauss-Newton to convergence, for
 * 2D-3D), pivot and
 * feasible anchor; per trajectory s: a Philox4x64-10 draw (key (seed, 0),
 * counter (s, 0, 0, 0)) picks an outward rotation (even s) or shift (odd s),
 * then n_iters iterations each project every predicted keypoint onto its
 * ball / ellipse shrunk by kappa and refit the pose, and a final in_purse test
 * keeps the pose or pulls it back to the boundary by bisection towards the
 * anchor.
 *
 * Outputs (device, caller-owned):
 *   poses       [total_samples][12] float: R row-major (9), then t (3); the pose
 *               maps model points into the camera / target frame.
 *   mask        [total_samples] uint8: PURSE_MASK_* bits.
 *   inst_status [n_inst] int32: PURSE_INST_* code | flags.
 */
purse_status purse_sample(const purse_batch *b, const purse_params *p, float *poses,
                          uint8_t *mask, int32_t *inst_status, void *ws, size_t ws_bytes,
                          void *stream);

/*
 * purse_sample without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation): the same prologue and trajectory kernels, with their
 * scratch (instance records, keypoint records, tile schedule) in a static
 * device array of the library (3.4 MB per device, held until the process
 * ends).  Outputs and errors as purse_sample; PURSE_E_BAD_ARG for a batch of
 * more than 1024 instances or 65536 keypoints in all.  Every call on a
 * device shares that device's array: calls that overlap on one device race,
 * and PURSE_FLAG_REUSE_PROLOGUE reuses whatever the last call on the device
 * left there.  The array's device address is looked up on the first call on
 * each device (make that first call outside graph capture).  No device
 * memory is allocated or freed.
 */
purse_status purse_sample_noalloc(const purse_batch *b, const purse_params *p, float *poses,
                                  uint8_t *mask, int32_t *inst_status, void *stream);

/*
 * Minimum enclosing geodesic balls of the feasible samples of each instance
 * by geodesic gradient descent (Section "Minimum Enclosing Geodesic Ball",
 * paragraph "Geodesic Gradient Descent"; appendix "Geodesic Gradient
 * Descent": the step fraction 1/i, the average of the last iterates, the
 * Frobenius argmax of the Riemannian Danskin theorem's takeaway).  From the
 * first feasible sample, megb_iters steps each move the rotation centre
 * along the geodesic towards the farthest sample by 1/i (the translation
 * centre likewise in R^3); ties go to the lowest sample index.  The centre is
 * proj_SO3 of the sum (rotation) and the mean (translation) of the last
 * megb_avg iterates; the radii are the largest geodesic angle and distance
 * from it, reduced in float64.
 *
 * Inputs: poses and mask as written by purse_sample (same batch layout).
 * Outputs:
 *   centre      [n_inst][12] float (R row-major, t); NaN for an empty instance.
 *   radii       [n_inst][2] double: D_hat (rad), d_hat (m); NaN if empty.
 *   n_feasible  [n_inst] int64.
 *   trace       [n_inst][megb_iters][2] int32: argmax sample (instance-local
 *               index) of each step, rotation then translation; -1 if empty.
 *   inst_status [n_inst] int32: PURSE_INST_EMPTY is OR-ed in for empty instances.
 */
/* The workspace keeps, for purse_megb_backward, every min(ckpt_every, 16)-th
 * rotation iterate of each descent with a signature of its trace. */
purse_status purse_megb(const purse_batch *b, const purse_params *p, const float *poses,
                        const uint8_t *mask, float *centre, double *radii,
                        int64_t *n_feasible, int32_t *trace, int32_t *inst_status,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * Reverse-mode derivative of the map (measurements) -> (radii, centre) as
 * computed by purse_sample + purse_megb, with every discrete decision held
 * fixed (clamp sets, masks, bisection bits, argmax trace).  Only the samples
 * the trace touches (and the first feasible one) carry cotangent; their
 * trajectories are recomputed from their Philox counters with checkpoints
 * every ckpt_every iterations and swept backwards, then through the centre
 * fit.
 *
 * Workspace contract: `ws` must be the workspace that purse_sample used to
 * produce `poses` and `mask` for this batch (its per-instance records: the
 * centre fit, anchor and keypoint records the trajectories are re-run from).
 * Each instance record is checked against the batch (kind, keypoint and
 * sample ranges, Philox key) and against a fingerprint of the instance's
 * inputs (model points, centres, shapes, bounds, intrinsics); an instance
 * whose record does not match gets NaN gradients instead of being re-run
 * from another batch's records.  The descent's iterates come from the
 * checkpoints purse_megb left in the workspace when their signature (the
 * steps, the winners and the bits of the start's and the winners'
 * rotations) matches `trace` and `poses`; otherwise the descent is replayed
 * from `trace` and the checkpoints are rewritten.
 *
 * Per-instance outcomes (no host synchronisation): an instance without
 * feasible samples gets zero gradients; NaN gradients mark a record of
 * another batch or data, a trace entry that is not a feasible sample, a
 * descent touching more than 256 distinct samples, or a non-finite centre.
 *
 * Inputs: poses, mask, trace as produced by the forward calls;
 *   g_radii  [n_inst][2] double: cotangents of D_hat and d_hat;
 *   g_centre [n_inst][6] float: cotangent of the centre as a left so(3)
 *            3-vector at R* followed by the R^3 cotangent of t*
 *            ([n_inst][12] with PURSE_FLAG_MATRIX_COTANGENT).
 * Outputs (overwritten):
 *   g_centres  [total_kp][3] float: d/d centres (b_i, or z_i in x, y; third unused = 0)
 *   g_shapes   [total_kp][4] float: d/d Lambda_i, symmetrised (zeros for 3D-3D)
 *   g_bounds   [total_kp]    float: d/d beta_i
 *   bwd_status [n_inst] int32 (may be NULL): the instance's outcome in the low
 *              byte (PURSE_BWD_*), and in the bits above it the number of
 *              distinct samples its descent touched (the active set).
 */
#define PURSE_BWD_OK 0
#define PURSE_BWD_EMPTY 1        /* no feasible sample: zero gradients */
#define PURSE_BWD_OVERFLOW 2     /* the descent touched more samples than the active set holds: NaN */
#define PURSE_BWD_BAD_TRACE 3    /* a trace entry is not a feasible sample of the instance: NaN */
#define PURSE_BWD_STALE 4        /* workspace records of another batch or data: NaN */
#define PURSE_BWD_NON_FINITE 5   /* non-finite centre: NaN */
purse_status purse_megb_backward(const purse_batch *b, const purse_params *p,
                                 const float *poses, const uint8_t *mask,
                                 const int32_t *trace, const double *g_radii,
                                 const float *g_centre, float *g_centres, float *g_shapes,
                                 float *g_bounds, int32_t *bwd_status, void *ws, size_t ws_bytes,
                                 void *stream);

/*
 * Step I of the paper (Section "The CLOSURE Algorithm"): candidate start poses
 * for the strategic random walk, each kept when it lies in S.  Instance j runs
 * M_j trials (its sample count in the batch), written to its sample range:
 *  - 3D-3D (random sample averaging with Arun's method): three distinct
 *    correspondences, a random point inside each of their balls, the rigid fit
 *    of the three pairs;
 *  - 2D-3D (random sample averaging with P3P): three distinct correspondences, a
 *    random point inside each of their ellipses, the perspective-3-point
 *    solutions for the three bearing rays in increasing order of the ratio of
 *    the third and first depths; the first in S is kept;
 *  - pose regression (PURSE_KIND_REG): a random convex combination of the
 *    hypotheses, R = proj_SO3(sum w_i R_i), t = sum w_i t_i, weights uniform on
 *    the simplex.
 * in_purse is the sampler's test (tolerance tau, depth > z_min), in float64.
 * Random numbers: Philox4x64-10; pose regression key (seed, 3), counter
 * (trial, i, 0, 0), weight w_i = -ln(1 - U) from the top 24 bits of word 0;
 * keypoint sets key (seed, 4), counter (trial, k, 0, 0): k = 0 picks the
 * correspondences (i_q = floor(U_q (N - q)), skipping those taken), k = 1..3
 * the point in the k-th constraint (ball: direction z = 1 - 2 U1,
 * phi = 2 pi U2, radius beta U3^(1/3); ellipse: z + beta sqrt(U3) U^-1
 * (cos 2 pi U2, sin 2 pi U2), U^T U = Lambda).
 * Outputs (device): poses [total_samples][12] (the identity where no
 * candidate was found), mask [total_samples] (PURSE_MASK_FEASIBLE for a pose in
 * S).  No workspace.
 */
purse_status purse_init(const purse_batch *b, const purse_params *p, float *poses, uint8_t *mask,
                        void *stream);

/*
 * The paper's own Step II, the strategic random walk (Section "The CLOSURE
 * Algorithm", Step II; Alg. "d S_R parallel sampler" and, in the appendix
 * "Boundary Sampler Algorithms", Alg. "d S_t parallel sampler"), as a second
 * sampler mode that starts from given poses of S (S0; e.g. samples of
 * purse_sample).
 *
 * From each start, n_walks walks per mode run n_iters iterations.  Rotation
 * mode: the angular velocity w = omega0 (u + u~) (u: axis of the start's
 * rotation relative to the average rotation of the instance's starts, u~: a
 * random unit vector); each iteration draws n_perturb translation
 * perturbations of the walk's pose (random direction, magnitude uniform in
 * [0, t_pert)), keeps the n_keep of largest boundary distance
 * min_i (beta_i - ||g_i||_Lambda_i) (eq. partial-s-dist; ties to the lower
 * draw index), and moves to the candidate (Exp(w gamma^(m-1)) R, t_k) in S
 * with the largest step (smallest m = 1..n_scales), then the best rank k; no
 * move when none is in S.  Translation mode: v = v0 ((t0 - t_bar)/|.| + v~),
 * rotation perturbations Exp(theta e) R (theta uniform in [0, r_pert)), and
 * candidates (R_k, t + v gamma^(m-1)).  in_purse is the sampler's test
 * (r_i <= beta_i + tau, depth > z_min), with tau and z_min from p.
 * Random numbers: Philox4x64-10, key (seed[j], 1 + mode), counter
 * (instance-local walk index, iteration, perturbation index, 0)
 * (iteration 2^32 - 1 for the initial velocity); the top 24 bits of output
 * words 0..2 give the direction (z = 1 - 2 U1, phi = 2 pi U2) and the
 * magnitude fraction U3.  Instance-local walk index of start s (s-th start of
 * the instance) and walk n: s * n_walks + n.
 *
 * Inputs (device): start_off [n_inst+1] int64 prefix sums of the instances'
 * start counts; starts [total_starts][12] float poses (R row-major, t).
 * Outputs (device, caller-owned):
 *   poses     [2][total_starts * n_walks][12] float: end poses, rotation-mode
 *             walks first, then translation-mode walks;
 *   mask      [2][total_starts * n_walks] uint8: PURSE_MASK_FEASIBLE if the end
 *             pose is in S;
 *   decisions [2][total_starts * n_walks][n_iters] int32 or NULL: per
 *             iteration k * n_scales + (m - 1) of the move taken, -1 for none.
 * Workspace: purse_walk_workspace_size bytes (the average pose of each
 * instance's starts), 256-byte aligned.
 */
typedef struct purse_walk_params {
  int32_t n_walks;    /* N_W: walks per start and mode */
  int32_t n_iters;    /* N_I */
  int32_t n_perturb;  /* N_P <= 256 */
  int32_t n_keep;     /* N_P* <= min(16, N_P) */
  int32_t n_scales;   /* N_T <= 32 */
  float gamma;        /* step decay in (0, 1] */
  float omega0;       /* angular velocity magnitude (rad per unit step) */
  float v0;           /* centre velocity magnitude (m per unit step) */
  float t_pert;       /* translation perturbation scale (m), rotation mode */
  float r_pert;       /* rotation perturbation scale (rad), translation mode */
} purse_walk_params;

/* Defaults: N_W 2, N_I 5, N_P 150, N_P* 10, N_T 15, gamma 0.5, omega0 0.5,
 * v0 0.05, t_pert 0.005, r_pert 0.02. */
purse_status purse_walk_default_params(purse_walk_params *w);
purse_status purse_walk_workspace_size(const purse_batch *b, size_t *bytes);
purse_status purse_walk(const purse_batch *b, const purse_params *p, const purse_walk_params *w,
                        const int64_t *start_off, const float *starts, int64_t total_starts,
                        float *poses, uint8_t *mask, int32_t *decisions, void *ws, size_t ws_bytes,
                        void *stream);

/* Static description of a status code. */
const char *purse_status_string(purse_status s);

/* Message of the last PURSE_E_HIP / PURSE_E_BAD_ARG on this thread ("" if none). */
const char *purse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PURSE_H */
