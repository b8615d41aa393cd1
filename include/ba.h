/*
 * Holistic bundle adjustment on one MI355X (gfx950): the C ABI of libba.so.
 *
 * One call of ba_lm_step runs one Levenberg-Marquardt iteration of the
 * unified bundle adjustment of "Stable and Scalable Bundle Adjustment of
 * Holistic 3D Structures": residuals and Jacobians of every point, line,
 * group-induced and cross-feature reprojection term, Schur elimination of
 * the block-diagonal feature Hessian into the reduced camera + group system
 * (Sec. 3.1 Eq. 3, Sec. 3.2 Eq. 5) and an implicit-Schur preconditioned
 * conjugate-gradient solve of that system, followed by back-substitution,
 * the FP64 cost of the candidate and the gain-ratio test.
 *
 * Conventions shared by every entry point
 *  - Ownership: every pointer argument is borrowed for the duration of the
 *    call; the library copies what it keeps.  Output arrays are allocated
 *    by the caller; a NULL output is skipped.  The handle owns all device
 *    memory and releases it in ba_destroy.
 *  - Errors: every call returns a ba_status; nothing else crosses the ABI.
 *    ba_last_error returns a handle-owned message, valid until the next
 *    call on that handle.
 *  - Threads: one handle per host thread.  Calls are synchronous with the
 *    host: when a call returns, its device work has finished.
 *  - Device: the handle runs on desc->device; hip_stream (a hipStream_t)
 *    may name a caller stream, NULL makes the library create its own.
 *
 * Parameter formats (all double)
 *  - camera  (10): qw qx qy qz tx ty tz f k1 k2.  X_cam = R(q) X + t;
 *    pixel = f s (u, v) + (cx, cy), (u, v) = X_cam,xy / X_cam,z,
 *    s = 1 + k1 r^2 + k2 r^4 (distorted); lines live in undistorted pixels.
 *  - point    (3): X.
 *  - line     (6): two distinct 3D points on the line (input);
 *    output of ba_get_parameters: unit direction d and moment m / |d|
 *    with m = p x d for p on the line (normalised Pluecker coordinates).
 *  - plane    (4): nx ny nz w with |n| = 1 and n . x + w = 0 (App. B).
 *  - vp       (3): unit direction (App. B).
 *  - shape   (16): a surface group of App. B, see ba_add_shapes.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_handle ba_handle; /* opaque; owns all device memory */

typedef enum {
  BA_OK = 0,
  BA_E_INVALID = 1,        /* bad argument: index out of range, NaN/inf, duplicate, ... */
  BA_E_STATE = 2,          /* call not legal in the handle's current state */
  BA_E_OOM = 3,            /* host or device allocation failed */
  BA_E_DEVICE = 4,         /* a HIP runtime call failed */
  BA_E_NUMERIC = 5,        /* non-finite cost; parameters rolled back */
  BA_E_NOT_CONVERGED = 6   /* ba_solve reached max_iters; results are valid */
} ba_status;

typedef enum { BA_PREC_FP64 = 0, BA_PREC_MIXED = 1 } ba_precision;
/* PCG preconditioner of the reduced system.  BLOCK_JACOBI: the inverses of
 * the diagonal blocks of S (the paper's choice).  GAUGE: two-level, block-
 * Jacobi plus the coarse space of the 7 similarity-gauge directions (world
 * rotation, translation, scale of every camera / plane / VP).  LEARNED: the
 * same plus 8 directions predicted by the network (needs ba_set_gnn_weights;
 * block-Jacobi alone without weights or graph). */
typedef enum { BA_PC_BLOCK_JACOBI = 0, BA_PC_LEARNED = 1, BA_PC_GAUGE = 2 } ba_precond;

/* Observation / association kinds accepted by ba_add_observations, and the
 * residual families each creates (expanded at the first step):
 *  - BA_OBS_POINT: the measurement x_ij of Sec. 3.1 Eq. 1 (point
 *    reprojection, R1); its undistorted copy is the observed point of the
 *    line-to-point distance of Sec. 3.4 Eq. 12 (R7).
 *  - BA_OBS_LINE: the endpoints of the observed segment l_ik, for the
 *    perpendicular endpoint vectors of Sec. 3.2 Eq. 4 (R2); their joining
 *    line is the observed line of Sec. 3.4 Eq. 11 (R6).
 *  - BA_ASSOC_PLANE_POINT / _PLANE_LINE: coplanarity groups, one record per
 *    view of the member (Sec. 3.3 Eq. 7, R3; Eq. 8 with the App. B
 *    plane-line projection, R4).
 *  - BA_ASSOC_VP_LINE: parallelism group (Sec. 3.3 Eq. 6, R5).
 *  - BA_ASSOC_JUNCTION: point-line incidence, one record per view that sees
 *    exactly one of the two (Sec. 3.4 Eqs. 11 and 12, R6 / R7). */
typedef enum {
  BA_OBS_POINT = 0,         /* a = camera, b = point; meas[4] = x y (distorted px), xu yu (undistorted px) */
  BA_OBS_LINE = 1,          /* a = camera, b = line;  meas[4] = e1x e1y e2x e2y (undistorted px)            */
  BA_ASSOC_PLANE_POINT = 2, /* a = plane,  b = point; meas = NULL */
  BA_ASSOC_PLANE_LINE = 3,  /* a = plane,  b = line;  meas = NULL */
  BA_ASSOC_VP_LINE = 4,     /* a = vp,     b = line;  meas = NULL */
  BA_ASSOC_JUNCTION = 5,    /* a = point,  b = line;  meas = NULL (the point lies on the line) */
  /* inter-group relations (Sec. 3.2: orthogonality and parallelism between VP pairs and
   * between plane-normal pairs, which touch only the group blocks of the reduced
   * system): a, b = two distinct VPs or planes; meas = NULL.  Residual of the unit
   * directions: orthogonal u_a . u_b (1 row), parallel u_a x u_b (3 rows; opposite
   * directions count as parallel).  Default loss: Cauchy 0.2, weight 5e3, as the VP-line
   * term; left out of E_pix like it.  Residual families 8 (VP orthogonal), 9 (VP
   * parallel), 10 (plane orthogonal), 11 (plane parallel). */
  BA_REL_VP_ORTHO = 6,      /* a = vp,     b = vp */
  BA_REL_VP_PARALLEL = 7,   /* a = vp,     b = vp */
  BA_REL_PLANE_ORTHO = 8,   /* a = plane,  b = plane */
  BA_REL_PLANE_PARALLEL = 9, /* a = plane,  b = plane */
  /* The 3D formulation the paper compares its pixel-space group residuals against
   * (Sec. 3.3's discussion of 3D regularisation; the 2D-vs-3D ablation of Sec. 4): the
   * signed metric distance n . X + w of a point to a plane, one record per association,
   * no camera.  Default loss: trivial, weight 100 (the paper sweeps 1 .. 1000); left out
   * of E_pix (metric, not pixels).  Residual family 12.  A point may carry it for several
   * planes; it may carry a BA_ASSOC_PLANE_POINT association too. */
  BA_ASSOC_PLANE_POINT_3D = 10, /* a = plane, b = point; meas = NULL */
  /* Surface groups beyond planes and VPs (App. B; added with ba_add_shapes): the
   * group-induced reprojection error of Sec. 3.3 with the shape's projection operator,
   * one record per view of the member, like the plane associations.  A point may be on
   * at most one shape, a line on at most one cuboid (the other types constrain points
   * only).  Default loss: that of the plane associations (Cauchy 1 px, weight 0.5).
   * Residual families 13 (point, 2 rows) and 14 (line, 4 rows). */
  BA_ASSOC_SHAPE_POINT = 11, /* a = shape, b = point; meas = NULL */
  BA_ASSOC_SHAPE_LINE = 12   /* a = shape (a cuboid), b = line; meas = NULL */
} ba_kind;

/* Surface group types (App. B, the table of group types; positive quantities are
 * optimised in log space) and their 16-double parameter records (unused entries zero):
 *  - SPHERE    (4 dof): centre c (3), radius r.  A point X goes to c + r (X - c)/|X - c|.
 *  - CYLINDER  (5 dof): axis direction (3, any length), a point on the axis (3), radius r;
 *    the axis is optimised in the orthonormal Pluecker form of the lines.  A point keeps
 *    its position along the axis and goes radially to distance r from it.  Output: the
 *    unit direction and the foot of the perpendicular from the origin.
 *  - CONE      (6 dof): apex A (3), axis direction (3), half-angle alpha in (0, pi/2).  A
 *    point goes to its foot on the generatrix in the half-plane through the axis and
 *    the point (along the normal of the generatrix).
 *  - ELLIPSOID (9 dof): rotation R (row-major 9, local to world, orthonormal), centre c
 *    (3), semi-axes s (3).  A point goes to c + R (s * z / |z|), z = R^T (X - c) / s
 *    (the scaled-radial projection).
 *  - CUBOID    (9 dof): rotation R (row-major 9), face offsets e_0 .. e_5: face i is the
 *    plane n_i . x + e_i = 0 with outward normal n_i = (-1)^i R e_{floor(i/2)}.  A point
 *    goes to the face of smallest |n_i . X + e_i|; a line to the face nearest to its
 *    point closest to the cuboid's centre, by the plane-line projection (App. B).
 * Every shape takes 9 entries of the reduced system (after the VPs); a type with fewer
 * degrees of freedom leaves the rest at zero step. */
typedef enum { BA_SHAPE_SPHERE = 0, BA_SHAPE_CYLINDER = 1, BA_SHAPE_CONE = 2, BA_SHAPE_ELLIPSOID = 3,
               BA_SHAPE_CUBOID = 4 } ba_shape_type;

typedef enum { BA_LOSS_TRIVIAL = 0, BA_LOSS_HUBER = 1, BA_LOSS_CAUCHY = 2 } ba_loss_kind;

/* Robust loss of one residual family: cost = weight * rho(|r|^2) / 2 with
 * rho(s) = s (trivial), Huber: s <= scale^2 ? s : 2 scale sqrt(s) - scale^2,
 * Cauchy: scale^2 log(1 + s / scale^2). */
typedef struct {
  int32_t kind;  /* ba_loss_kind */
  double scale;
  double weight;
} ba_loss;

typedef struct {
  int32_t n_cameras, n_points, n_lines, n_planes, n_vps;
  int32_t camera_dof;     /* 9 = rotation, translation, f, k1, k2; 6 = pose only */
  double cx, cy;          /* fixed principal point */
  const double *cameras;  /* n_cameras x 10 */
  const double *points;   /* n_points x 3 */
  const double *lines;    /* n_lines x 6 (two points) */
  const double *planes;   /* n_planes x 4 */
  const double *vps;      /* n_vps x 3 */
  int32_t precision;      /* ba_precision */
  int32_t precond;        /* ba_precond */
  void *hip_stream;       /* hipStream_t or NULL */
  int32_t device;
} ba_problem_desc;

/* ba_step_report.pcg_flags */
#define BA_PCG_BREAKDOWN 1         /* p.Sp <= 0 or not finite: the solve stopped early */
#define BA_PCG_COARSE_FALLBACK 2   /* the two-level solve broke down and was repeated with block-Jacobi */
#define BA_PCG_NONFINITE_RHS 4     /* the reduced right-hand side was not finite: step rejected, relinearised next */
#define BA_SOLVE_NOT_SPD 8         /* dense solver: a pivot of the Cholesky factorisation of S was not positive
                                      (S not positive definite in FP64): no step formed, rejected (E_after NaN) */

/* Solver of the reduced camera / group system S h_a = b (Sec. 3.1 Eq. 3).  The paper
 * solves it with a sparse or a dense Schur-complement method chosen by image count
 * (Sec. 4.1).  BA_SOLVER_PCG: implicit-Schur preconditioned conjugate gradients
 * (S never formed).  BA_SOLVER_DENSE: S formed explicitly in FP64 from the record
 * Jacobians (both precisions' Jacobians; FP64 arithmetic), factored by Cholesky on the
 * device and solved exactly; for reduced systems of at most 8192 rows (n_A^2 doubles of
 * device memory). */
typedef enum { BA_SOLVER_PCG = 0, BA_SOLVER_DENSE = 1 } ba_linear_solver;

typedef struct {
  int32_t max_iters;      /* ba_solve: attempts (accepted or rejected); default 100 */
  double func_tol;        /* stop after an accepted step with |dE_pix| / E_pix < func_tol; 1e-6 */
  double grad_tol;        /* ba_solve: stop, before solving, when a fresh linearisation has
                             |g|_inf < grad_tol, g = J^T W r over all parameters (0: off); 1e-10 */
  double pcg_tol;         /* PCG stops at |r_k| <= pcg_tol |b|; 1e-6 */
  int32_t pcg_max_iters;  /* 1000 */
  double lambda0;         /* initial Marquardt lambda (used on the first step only); 1e-4 */
  double nu0;             /* 2 */
  double kappa_max;       /* FP32 feature blocks with estimated condition above it are redone in FP64; 1e4 */
  int32_t time_kernels;   /* 1: time every implicit-Schur product launch with HIP events
                             (ba_step_report.matvec_ms / matvec_count); 0 */
  int32_t deterministic;  /* 1: every sum of the step is taken in a fixed order, so that the
                             same inputs give bit-identical results run after run: the
                             implicit-Schur product forms s_f per feature and then each
                             camera / group row of S x over its records in a fixed order
                             (instead of FP64 LDS atomics), and the PCG dot products are
                             summed per workgroup and then in workgroup order (instead of
                             one FP64 atomic per workgroup).  Slower; 0 (the default)
                             keeps the atomics.  The network's message aggregation of the
                             learned preconditioner still sums with FP32 atomics. */
  int32_t linear_solver;  /* ba_linear_solver; BA_SOLVER_PCG.  With BA_SOLVER_DENSE the PCG
                             and preconditioner options are unused, pcg_iters is 0,
                             pcg_rel_residual is |S h_a - b| / |b| with S h_a from the
                             implicit product, and the step's ms[BA_PHASE_PCG] is the
                             assembly, factorisation and solve; deterministic by
                             construction */
  int32_t fix_a_side;     /* 1: cameras, planes and VPs are held fixed and only the features
                             move (h_a = 0, h_f = -(V_f + lambda D_f)^-1 g_f; the
                             fixed-pose stage of the reliability-aware refinement); the
                             linear solver is then unused; 0 */
} ba_solve_options;

enum {
  BA_PHASE_LINEARIZE = 0, BA_PHASE_FEATURE = 1, BA_PHASE_SCHUR = 2, BA_PHASE_PRECOND = 3,
  BA_PHASE_PCG = 4, BA_PHASE_BACKSUB = 5, BA_PHASE_COST = 6, BA_PHASE_COUNT = 8
};

typedef struct {
  double E_before, E_after;      /* 1/2 sum w rho, FP64 (E_after = candidate cost) */
  double Epix_before, Epix_after;/* same without the angular VP family (Sec. 3.5) */
  double model_decrease;         /* L(0) - L(h) */
  double gain_ratio;
  double lambda;                 /* lambda used by this step */
  int32_t accepted;
  int32_t pcg_iters;
  double pcg_rel_residual;       /* |r_k| / |b| (recursive residual) */
  int32_t n_fp64_blocks;         /* feature blocks inverted in FP64 */
  int32_t relinearized;          /* 1 if this step evaluated Jacobians */
  double ms[BA_PHASE_COUNT];     /* device time per phase */
  double matvec_ms;              /* with time_kernels: summed duration of the PCG products */
  int32_t matvec_count;          /* number of those products */
  int32_t coarse;                /* columns of the coarse space used by this step's PCG (0: block-Jacobi) */
  int32_t pcg_flags;             /* BA_PCG_* bits */
  int32_t n_degenerate;          /* line-projection records (R2, R4, R7) of this step's
                                    linearisation at a nearly degenerate image line: normal
                                    |(l1, l2)| = rel (|m| + |t| |d|) with rel < 1e-3 (the line
                                    passes close to the camera centre or lies near its principal
                                    plane; Eqs. 4, 8 and 12 stay differentiable, with derivatives
                                    growing like 1 / rel).  The FP64 path keeps their exact
                                    Jacobian; the FP32 path evaluates it in FP64 and scales it by
                                    rel / 1e-3 before storing it in FP32.  Also counted: records
                                    whose working-precision Jacobian is not finite (dropped).
                                    Residuals stay in the cost. */
  double grad_inf;               /* |g|_inf of the linearisation this step used: g = J^T W r, the
                                    gradient of E in the local coordinates of every camera,
                                    point, line, plane and VP (FP64 for the A side, the working
                                    precision for the features) */
  int32_t n_fp64_failed;         /* of n_fp64_blocks, feature blocks whose FP64 Cholesky failed too:
                                    their inverse is zero, so the feature does not move this step */
} ba_step_report;

typedef struct {
  int32_t iters, accepted;
  double E_initial, E_final, Epix_final;
  int32_t termination;           /* 0 func_tol, 1 grad_tol, 2 max_iters, 3 lambda_max, 4 numeric */
  double total_ms;
  int32_t pcg_iters_total;
} ba_summary;

/* Reliability-aware two-stage refinement (App. A.2).  The paper classifies feature
 * tracks as reliable or not from their active observations and their estimated
 * uncertainty, refines cameras, reliable features, groups and wireframe records
 * first, then the unreliable features with the poses fixed, and leaves groups with
 * too little support out of the first stage.  It gives no formulas or thresholds;
 * this library's readings:
 *   active observation: an observation record (point: Eq. 1, line: Eq. 4) whose
 *     residual lies in the quadratic part of its loss, |r|^2 <= scale^2 (every record
 *     under the trivial loss);
 *   sigma = lambda_min(V_f)^-1/2, V_f the undamped feature block (sum of J~^T J~ over
 *     the feature's records, Eq. 3) at the current parameters; for a point divided by
 *     its mean distance to the cameras observing it; for a line in the tangent
 *     coordinates of its orthonormal representation;
 *   reliable: n_active >= min_active_obs and sigma <= max_sigma_point (points) or
 *     max_sigma_line (lines);
 *   group support: distinct reliable features associated with the group (planes:
 *     points and lines; VPs: lines); below min_group_support the group and its
 *     relations are left out of stage 1. */
typedef struct {
  int32_t min_active_obs;     /* 3 */
  double max_sigma_point;     /* 0.01 (relative to the viewing distance) */
  double max_sigma_line;      /* 0.1 (tangent coordinates) */
  int32_t min_group_support;  /* 3 */
} ba_reliability_options;

typedef struct {
  int32_t n_points_unreliable, n_lines_unreliable;  /* refined in stage 2 */
  int32_t n_planes_out, n_vps_out;                  /* left out of stage 1 */
  ba_summary stage1, stage2;
} ba_two_stage_summary;

/* Fill *opt with the defaults listed in ba_solve_options. */
void ba_default_options(ba_solve_options *opt);

/* Create a problem (Sec. 3.1: cameras C_i = (K, R_i, t_i); Sec. 3.2:
 * features (points, lines) and groups (planes, VPs) placed with the
 * cameras in the non-eliminated set A).  Copies the initial parameters to
 * the device (FP64 master copy).  Errors: BA_E_INVALID for negative
 * counts, camera_dof other than 6 or 9, non-finite values, non-unit plane
 * normals or VPs (| |n| - 1 | > 1e-6), degenerate lines; BA_E_DEVICE /
 * BA_E_OOM on device failure.  On error *out is NULL. */
ba_status ba_create(const ba_problem_desc *desc, ba_handle **out);

/* Append n observations or associations of one kind (ba_kind; layouts
 * above).  a, b: int32 arrays of length n; meas: n x 4 doubles for the
 * two observation kinds, NULL otherwise.  loss: the robust loss of the
 * residual family the kind creates (NULL keeps the default: trivial for
 * points and lines; Cauchy 1 px, weight 0.5 for plane associations;
 * Cauchy 0.2, weight 5e3 for VP-line; Cauchy 1 px, weight 0.1 for
 * junctions - weights from the paper's supplementary Sec. C).  Legal only
 * before the first ba_lm_step / ba_solve (else BA_E_STATE).  Errors:
 * BA_E_INVALID for out-of-range indices or non-finite measurements.
 * Duplicate observations, a feature in two planes or a line in two VPs
 * are reported by the first ba_lm_step. */
ba_status ba_add_observations(ba_handle *h, int32_t kind, int64_t n, const int32_t *a, const int32_t *b,
                              const double *meas, const ba_loss *loss);

/* Exactly one LM iteration (one solve attempt, accepted or rejected).
 * The first call expands associations into residual records with the
 * visibility rules of Sec. 3.3-3.4 (the analogue of the symbolic phase of
 * Sec. 4.1).  opt NULL = defaults; lambda0 applies to the first call only,
 * later calls continue the handle's lambda / nu.  rep may be NULL.
 * Errors: BA_E_INVALID for inconsistent observations (reported here);
 * BA_E_NUMERIC when the cost is not finite (parameters unchanged). */
ba_status ba_lm_step(ba_handle *h, const ba_solve_options *opt, ba_step_report *rep);

/* ba_lm_step until termination (Sec. 3.5: relative change of the pixel
 * cost on accepted steps; see ba_solve_options).  Returns BA_OK or
 * BA_E_NOT_CONVERGED (parameters and summary still valid). */
ba_status ba_solve(ba_handle *h, const ba_solve_options *opt, ba_summary *sum);

/* Add n surface groups (App. B; types and 16-double records above) before the first
 * step; shapes are numbered in the order added, from 0.  BA_E_INVALID for an unknown
 * type, a non-positive radius, half-angle or semi-axis, a half-angle of pi/2 or more, a
 * zero axis direction, a rotation that is not orthonormal to 1e-6, or a non-finite
 * value; BA_E_STATE after the first step. */
ba_status ba_add_shapes(ba_handle *h, int64_t n, const int32_t *types, const double *params);

/* Current shape parameters (n_shapes x 16, the format of ba_add_shapes). */
ba_status ba_get_shapes(const ba_handle *h, double *params);

/* Current parameters (formats above; lines as unit d and m / |d|). */
ba_status ba_get_parameters(const ba_handle *h, double *cameras, double *points, double *lines,
                            double *planes, double *vps);

/* Replace the parameters (input formats of ba_create).  Any array may be
 * NULL (kept).  Resets the linearisation; lambda / nu are kept. */
ba_status ba_set_parameters(ba_handle *h, const double *cameras, const double *points, const double *lines,
                            const double *planes, const double *vps);

/* LM damping state (for resume): get and set lambda and nu. */
ba_status ba_get_lm_state(const ba_handle *h, double *lambda, double *nu);
ba_status ba_set_lm_state(ba_handle *h, double lambda, double nu);

/* Inspection entry points used by parity checks.
 *
 * ba_linearize: evaluate residuals, Jacobians, the feature blocks V_f,
 * the reduced right-hand side b and the diagonal blocks of S at the
 * current parameters and damping lambda (Sec. 3.1 Eq. 3), without
 * stepping.  Requires the records to exist (calls the expansion if
 * needed). */
ba_status ba_linearize(ba_handle *h, double lambda);

/* Number of residual records of a family (1 point, 2 line, 3 plane-point,
 * 4 plane-line, 5 vp-line, 6 point-to-line, 7 line-to-point; inter-group
 * relations 8 VP orthogonal, 9 VP parallel, 10 plane orthogonal, 11 plane
 * parallel; 12 3D point-to-plane; 13 point on a shape, 14 line on a cuboid). */
ba_status ba_record_count(const ba_handle *h, int32_t family, int64_t *count);

/* Export the last linearisation of a family, in the handle's internal record
 * order.  keys: count x 3 int64 (camera or -1, feature, group / partner
 * feature or -1, in the caller's indices); r: count x rows (IRLS-weighted,
 * as used by the solver); J: count x rows x (camera_dof + feature dof +
 * group dof) in that column order (weighted).  Relation families 8-11: keys
 * (-1, group a, group b), rows 1 (orthogonal) or 3 (parallel), J columns
 * [group a | group b] with 2 per VP and 3 per plane (the offset column is
 * zero).  Family 12: keys (-1, point, plane), 1 row, J columns [point (3) |
 * plane (3)] (no camera, as family 5).  Families 13 / 14: keys (camera, point / line,
 * shape), 2 / 4 rows, J columns [camera | feature | shape (9)].  Any output may be NULL. */
ba_status ba_export_records(const ba_handle *h, int32_t family, int64_t *keys, double *r, double *J);

/* Feature blocks of the last linearisation: V_f = sum J~_f^T J~_f (undamped)
 * and g_f, points (n_points x 9 and x 3) and lines (n_lines x 16 and x 4),
 * caller's feature order. */
ba_status ba_export_feature_blocks(const ba_handle *h, double *Vp, double *gp, double *Vl, double *gl);

/* Reduced system at the damping of the last ba_linearize: b (n_A) and the
 * diagonal blocks of S (cameras n_cameras x cd x cd, planes x 3 x 3,
 * vps x 2 x 2), A ordered cameras, planes, vps. */
ba_status ba_export_reduced(const ba_handle *h, double *b, double *S_cam, double *S_plane, double *S_vp);

/* Diagonal blocks of S of the shapes at the damping of the last ba_linearize
 * (n_shapes x 9 x 9; their rows of b are the last 9 n_shapes entries of b). */
ba_status ba_export_shape_blocks(const ba_handle *h, double *S_shape);

/* y = S x with the implicit Schur product at the last linearisation
 * (x, y: n_A doubles on the host). */
ba_status ba_schur_matvec(ba_handle *h, const double *x, double *y);

/* Solve S x = b of the last ba_linearize with the handle's PCG
 * (preconditioner of desc->precond; a two-level solve that breaks down is
 * repeated with block-Jacobi, as in ba_lm_step, and iters counts both);
 * x: n_A doubles; iters, rel_res out. */
ba_status ba_pcg_solve(ba_handle *h, double tol, int32_t max_iters, double *x, int32_t *iters, double *rel_res);

/* Sizes: n_A (reduced dimension) and camera_dof. */
ba_status ba_reduced_dim(const ba_handle *h, int64_t *n_A, int32_t *camera_dof);

/* ---------------------------------------------------------------------------
 * Learned coarse-space correction (this project's addition to the method:
 * the paper preconditions the reduced-system CG with the inverses of its
 * diagonal blocks, which leaves the slow global modes of BA, e.g. the
 * similarity gauge, to CG).  A message-passing network predicts K = 8
 * vectors per block; together with the 7 similarity-gauge directions they
 * span the coarse space Z (n_A x 15).  With E = Z^T S Z, Q = Z E^-1 Z^T and
 * M = blockdiag(S_ii)^-1, PCG starts from x0 = Q b and uses
 *     P r = (I - Q S) M r + Q r
 * (M alone when E is not positive definite).  The coarse space is used for
 * lambda <= 0.1 only (above, block-Jacobi PCG needs fewer iterations than the
 * coarse set-up costs in products) and, with FP32 records, lambda >= 1e-6
 * (below, the FP32 product does not resolve S on the near-null gauge
 * directions); otherwise M is used alone.
 * Graph: one node per camera / plane / VP block of the reduced system, in
 * that order; directed edges both ways between blocks that share a feature,
 * sorted by destination, then source.
 * Node input (64 floats): log diag(S_ii) minus its mean [0, n); strictly
 * lower correlations S_pq / sqrt(S_pp S_qq), row by row, from 9;
 * log(lambda) at 45; log(1 + records touching the block) at 46;
 * log(1 + in-degree) at 47; type one-hot at 48..50; geometry from 51:
 * camera R row-major then t / s0, plane n, w / s0, b1, b2, VP v, b1, b2
 * ((b1, b2) the sphere tangent basis, s0 the RMS distance of the input
 * camera centres from their mean, 1 if zero); zeros elsewhere.  Edge input
 * (8 floats): log(1 + shared features), then one-hot camera-camera,
 * camera-plane, camera-VP, group-group; zeros.
 * Network, width 64, gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))):
 *   h = gelu(x W_in + b_in);  3 times: m_i = mean over edges j->i of
 *   gelu([h_j, e_ji] W_e + b_e), h = gelu(h W_s + b_s + m) + h;
 *   Y_i = h_i W_t + b_t for the node's type, read as n_t x 8 (row-major).
 * Z_i = diag(u_i) Y_i with row scales u: camera (1,1,1, s0,s0,s0, 1,1,1),
 * plane (1, 1, s0), VP (1, 1).  Training loss per system:
 * tr((Z^T D Z)^-1 Z^T S Z) with Z = [gauge (7 columns), network (8)],
 * D = blockdiag(S_ii); a batch takes the mean.
 * Parameters: float32 blob in the order W_in (64x64) b_in, (W_e (72x64)
 * b_e W_s (64x64) b_s) x3, (W_t (64 x 8 n_t) b_t) for cameras, planes,
 * VPs; matrices row-major.
 * ------------------------------------------------------------------------- */

/* Load network weights into a problem handle (used by BA_PC_LEARNED).  The
 * solver uses block-Jacobi alone when no weights are loaded, when the
 * problem has more than 6000 blocks (the graph is not built) or when E is
 * not positive definite.  bytes must be 4 * ba_gnn_param_count(camera_dof),
 * else BA_E_INVALID; non-finite weights give BA_E_INVALID.  The blob is
 * copied. */
ba_status ba_set_gnn_weights(ba_handle *h, const void *blob, size_t bytes);

/* Number of float32 parameters of the network for a camera block size. */
size_t ba_gnn_param_count(int32_t camera_dof);

/* Graph of the reduced system at the last ba_linearize, for building
 * training data.  Sizes first (NULL outputs skipped).  node_x: n x 64 at the
 * last lambda and parameters; node_off: each block's offset in the reduced
 * vector; node_unit: n x 9 row scales u_i (zero-padded); edge_rev[e]: index
 * of the reverse edge; edge_x: m x 8.  BA_E_STATE before the first
 * linearisation or when the graph is not built (more than 6000 blocks). */
ba_status ba_export_gnn_graph(ba_handle *h, int32_t *n_nodes, int32_t *n_edges, float *node_x, int32_t *node_type,
                              int32_t *node_off, float *node_unit, int32_t *edge_src, int32_t *edge_dst,
                              int32_t *edge_rev, float *edge_x);

/* The damped reduced matrix S of the last ba_linearize, dense (n_A x n_A
 * doubles, row-major, caller-allocated), formed column by column with the
 * implicit-Schur product (n_A products: meant for small systems, e.g.
 * training data and tests).  Temporary device memory: 8 n_A^2 bytes. */
ba_status ba_export_schur_dense(ba_handle *h, double *S);

void ba_default_reliability_options(ba_reliability_options *o);

/* Leave records out of the problem: every record whose parameters include a flagged
 * point, line, plane or VP (arrays of n_points, n_lines, n_planes, n_vps bytes in the
 * caller's order, nonzero = left out; NULL = none; all NULL clears the mask) has zero
 * weight in the linearisation and no cost, so the flagged parameters do not move.  A
 * junction record (Eqs. 11, 12) belongs to the feature it adjusts; its partner only
 * supplies the measurement.  Relations are left out with either of their groups.
 * Takes effect at the next linearisation; the cost is re-evaluated. */
ba_status ba_set_record_mask(ba_handle *h, const uint8_t *points_out, const uint8_t *lines_out,
                             const uint8_t *planes_out, const uint8_t *vps_out);

/* Per-feature statistics of the reliability test at the current parameters (see
 * ba_reliability_options), in the caller's order: active observations, observations
 * and sigma (infinite when V_f is singular or the feature has no observation) per point
 * and per line; NULL outputs are skipped.  Linearises first (with the current record
 * mask).  Sigma is computed from V_f in the working precision. */
ba_status ba_feature_reliability(ba_handle *h, int32_t *pt_active, int32_t *pt_obs, double *pt_sigma,
                                 int32_t *ln_active, int32_t *ln_obs, double *ln_sigma);

/* The two-stage refinement from the current parameters: classify (without a mask),
 * then ba_solve with the unreliable features and the unsupported groups left out,
 * then ba_solve with fix_a_side over the unreliable features alone (the reliable
 * features left out), each stage starting from lambda0; the mask is cleared at the
 * end.  opt's fix_a_side is ignored.  Returns BA_OK unless an error occurred (a stage
 * that ends on max_iters is reported in its summary). */
ba_status ba_solve_two_stage(ba_handle *h, const ba_solve_options *opt, const ba_reliability_options *ro,
                             ba_two_stage_summary *out);

/* The damped reduced matrix S of the last ba_linearize (Sec. 3.1 Eq. 3), dense
 * (n_A x n_A doubles, row-major, caller-allocated), as the dense solver forms it:
 * block pair by block pair from the records' Jacobians and the feature blocks'
 * inverses, in FP64 (BA_SOLVER_DENSE).  BA_E_STATE before the first linearisation;
 * BA_E_INVALID when n_A exceeds 8192.  Allocates the dense solver's device storage
 * on first use (kept with the handle). */
ba_status ba_export_schur_assembled(ba_handle *h, double *S);

/* Dense symmetric positive definite solve on the device (the factorisation and
 * triangular solves of BA_SOLVER_DENSE): A (n x n doubles, row-major, device memory;
 * the lower triangle is read) is overwritten by its lower Cholesky factor L, A = L
 * L^T, with the strict upper triangle zeroed, and b (n doubles, device memory) by
 * x = A^-1 b.  FP64 throughout: right-looking blocked Cholesky on 64 x 64 tiles,
 * tile products on the matrix cores.  Runs on hip_stream (NULL: the default stream)
 * of the given device and returns when it is done.  *info = 0 on success, else
 * 1 + the first column whose pivot was not positive or not finite (A not positive
 * definite in FP64); A and b are then unspecified and the status is BA_E_NUMERIC.
 * Temporary device memory: about 8 (n + 63)^2 bytes.  n = 0 is a no-op. */
ba_status ba_dense_spd_solve(int32_t device, int64_t n, double *A, double *b, void *hip_stream, int32_t *info);

/* ba_export_schur_dense for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same S, formed by the same products, but staged through a
 * fixed per-GPU scratch panel of 2^19 doubles (4 MiB, held until the process
 * ends) in column panels of floor(2^19 / n_A) columns, each copied to S before
 * the next.  Calls no hipMalloc / hipFree.  BA_E_INVALID when n_A > 2^19;
 * BA_E_STATE before the first linearisation.  Every handle on one GPU shares
 * that GPU's panel: calls that overlap on one GPU (from different threads)
 * race and must be serialised by the caller. */
ba_status ba_export_schur_dense_noalloc(ba_handle *h, double *S);

/* The 7 similarity-gauge directions of the reduced parameters at the current
 * parameters (world rotation about x, y, z; translation along x, y, z;
 * scale), n_A x 7 doubles row-major (caller-allocated).  Cameras: rotation w
 * gives dtheta = -R w, dt = (R w) x t; translation u gives dt = -R u; scale s
 * gives dt = s t.  Planes: (b1, b2) . (w x n), dw = -n . u, dw = s w.  VPs:
 * (b1, b2) . (w x v). */
ba_status ba_export_gauge_basis(ba_handle *h, double *G);

/* The coarse space of the last assembly (BA_PC_GAUGE / BA_PC_LEARNED): its
 * column count k (0 for block-Jacobi), Z and S Z (n_A x k doubles each,
 * row-major, caller-allocated, NULL skipped; size them with k from a first
 * call with both NULL). */
ba_status ba_export_coarse_space(ba_handle *h, int32_t *k, double *Z, double *SZ);

/* y = L^-1 S L^-T x with S_ii = L_i L_i^T (the block-normalised reduced
 * system of the last ba_linearize); x, y: n_A doubles (host). */
ba_status ba_normalized_matvec(ba_handle *h, const double *x, double *y);

/* A batch of systems for training or evaluation.  Nodes sorted by type
 * within the batch (cameras, planes, VPs); node_graph: each node's system,
 * 0 .. n_graphs-1; node_unit: n x 9 row scales.  Edges join nodes of one
 * system, sorted by destination, with edge_rev[e] the index of the reverse
 * edge.  For the loss: the gauge block of every node (ba_export_gauge_basis
 * rows of the node's entries) and the S blocks (FP64, row-major): the damped
 * diagonal block of node i (n_i x n_i) at s_node + s_node_off[i], the block
 * S_{dst,src} of edge e (n_dst x n_src) at s_edge + s_edge_off[e]; the
 * offsets must stay inside s_node_len / s_edge_len. */
typedef struct {
  int32_t n_nodes, n_edges, n_graphs;
  const float *node_x;
  const int32_t *node_type, *node_graph;
  const float *node_unit;
  const double *node_gauge;   /* n x 9 x 7: the gauge rows of each node (row-major, zero-padded); loss only */
  const int32_t *edge_src, *edge_dst, *edge_rev;
  const float *edge_x;
  const double *s_node, *s_edge;
  const int64_t *s_node_off, *s_edge_off;
  int64_t s_node_len, s_edge_len;
} ba_gnn_batch;

typedef struct ba_gnn ba_gnn; /* network parameters, Adam state and work buffers on one device */

/* precision: 0 = FP32 throughout (debug / gradient checks), 1 = BF16 MFMA
 * products with FP32 accumulation (training and inference).  Parameters
 * start at zero: set them before use. */
ba_status ba_gnn_create(int32_t camera_dof, int32_t precision, int32_t device, ba_gnn **out);
ba_status ba_gnn_set_params(ba_gnn *g, const float *params, size_t count);
ba_status ba_gnn_get_params(const ba_gnn *g, float *params, size_t count);
/* Forward pass: heads (n_nodes x 72 floats: Y_i row-major n_i x 8, rows
 * zero-padded to 9) and, when loss is not NULL, the batch loss (needs the S
 * blocks).  A system whose Z^T D Z is not positive definite adds zero. */
ba_status ba_gnn_forward(ba_gnn *g, const ba_gnn_batch *b, float *heads, double *loss);
/* Forward + backward: loss, gradient (param count floats, NULL skipped);
 * with lr > 0 also one Adam step (beta1 0.9, beta2 0.999, eps 1e-8). */
ba_status ba_gnn_train_step(ba_gnn *g, const ba_gnn_batch *b, double lr, double *loss, float *grad);
const char *ba_gnn_last_error(const ba_gnn *g);
void ba_gnn_destroy(ba_gnn *g);

const char *ba_last_error(const ba_handle *h);
void ba_destroy(ba_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
