// Device-side layout of one holistic BA problem and the kernel launchers.
//
// Records of each residual family are stored feature-major (sorted by the
// internal feature id, then camera): one array-of-structures slot per record
// with its IRLS-weighted Jacobian blocks, and its weighted residual in a
// separate array (the Schur product reads only the Jacobians).
// Camera-side reductions walk camera-major index lists into those arrays;
// feature-side reductions walk the feature CSR offsets.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ba_math.h"

namespace ba {

// families 1..7 of Sec. 3; 8, the 3D point-to-plane distance of the 3D formulation
// (exported as family 12, after the four relation families); 9, a point on a surface
// group (exported 13) and 10, a line on a cuboid (exported 14); index 0 unused
constexpr int NFAM = 11;

// compile-time shape of a family's record slot
template <int FAM, int CD> struct Fam;
template <int CD> struct Fam<1, CD> { static constexpr int ROWS = 2, NC = CamCols<CD>::PT, NG = 0, NF = 3, MEAS = 2, GT = 0, FT = 0; };
template <int CD> struct Fam<2, CD> { static constexpr int ROWS = 4, NC = CamCols<CD>::LN, NG = 0, NF = 4, MEAS = 4, GT = 0, FT = 1; };
template <int CD> struct Fam<3, CD> { static constexpr int ROWS = 2, NC = CamCols<CD>::PT, NG = 3, NF = 3, MEAS = 0, GT = 1, FT = 0; };
template <int CD> struct Fam<4, CD> { static constexpr int ROWS = 4, NC = CamCols<CD>::LN, NG = 3, NF = 4, MEAS = 4, GT = 1, FT = 1; };
template <int CD> struct Fam<5, CD> { static constexpr int ROWS = 3, NC = 0, NG = 2, NF = 4, MEAS = 0, GT = 2, FT = 1; };
template <int CD> struct Fam<6, CD> { static constexpr int ROWS = 1, NC = CamCols<CD>::PT, NG = 0, NF = 3, MEAS = 3, GT = 0, FT = 0; };
template <int CD> struct Fam<7, CD> { static constexpr int ROWS = 1, NC = CamCols<CD>::LN, NG = 0, NF = 4, MEAS = 2, GT = 0, FT = 1; };
template <int CD> struct Fam<8, CD> { static constexpr int ROWS = 1, NC = 0, NG = 3, NF = 3, MEAS = 0, GT = 1, FT = 0; };
template <int CD> struct Fam<9, CD> { static constexpr int ROWS = 2, NC = CamCols<CD>::PT, NG = SH_DOF, NF = 3, MEAS = 0, GT = 3, FT = 0; };
template <int CD> struct Fam<10, CD> { static constexpr int ROWS = 4, NC = CamCols<CD>::LN, NG = SH_DOF, NF = 4, MEAS = 4, GT = 3, FT = 1; };

// Jacobian slot of one record: [ J_cam (ROWS x NC) | J_group (ROWS x NG) | J_feature (ROWS x NF) | pad ];
// the weighted residual lives in a separate ROWS-wide array
template <int FAM, int CD> struct Slot {
  using F = Fam<FAM, CD>;
  static constexpr int ROWS = F::ROWS, NC = F::NC, NG = F::NG, NF = F::NF;
  static constexpr int OC = 0, OG = OC + ROWS * NC, OF = OG + ROWS * NG;
  static constexpr int USED = OF + ROWS * NF;
  static constexpr int STRIDE = (USED + 3) / 4 * 4;
};

inline int meas_width(int fam) { return fam == 1 ? 2 : fam == 2 ? 4 : fam == 3 ? 0 : fam == 4 ? 4 : fam == 5 ? 0 : fam == 6 ? 3 : fam == 7 ? 2 : fam == 10 ? 4 : 0; }
inline int fam_rows(int fam) { return fam == 1 ? 2 : fam == 2 ? 4 : fam == 3 ? 2 : fam == 4 ? 4 : fam == 5 ? 3 : fam == 9 ? 2 : fam == 10 ? 4 : 1; }
inline bool fam_is_line(int fam) { return fam == 2 || fam == 4 || fam == 5 || fam == 7 || fam == 10; }
int slot_stride(int fam, int cd);
int slot_nc(int fam, int cd);
int slot_ng(int fam);
int slot_nf(int fam);

// All device pointers of a problem.  Passed by value to kernels.
struct Dev {
  int CD = 9;
  int nc = 0, np = 0, nl = 0, ng = 0, nv = 0, ns = 0;
  int nA = 0, offPl = 0, offVp = 0, offSh = 0;
  int fp64 = 0;  // 1: T = double, 0: T = float
  // parameters: FP64 master (current and candidate) and work copy in T; shapes
  // (surface groups, SH_STRIDE doubles each, see ba_shape.h) in FP64 only
  double *cam64 = nullptr, *pt64 = nullptr, *ln64 = nullptr, *pl64 = nullptr, *vp64 = nullptr, *sh64 = nullptr;
  double *cam64n = nullptr, *pt64n = nullptr, *ln64n = nullptr, *pl64n = nullptr, *vp64n = nullptr, *sh64n = nullptr;
  void *camT = nullptr, *ptT = nullptr, *lnT = nullptr, *plT = nullptr, *vpT = nullptr;
  // residual families
  int64_t fn[NFAM] = {0};
  int32_t *fcam[NFAM] = {nullptr}, *fgrp[NFAM] = {nullptr}, *ffeat[NFAM] = {nullptr}, *foff[NFAM] = {nullptr};
  double *fmeas[NFAM] = {nullptr};
  void *frec[NFAM] = {nullptr};   // Jacobian slots (T)
  void *fres[NFAM] = {nullptr};   // weighted residuals (T), n x ROWS
  int lkind[NFAM] = {0};
  double lscale[NFAM] = {0}, lweight[NFAM] = {0};
  // camera-major lists
  int32_t *po_off = nullptr, *lo_off = nullptr;  // per camera: range of its R1 / R2 positions
  int32_t *px_start = nullptr, *px_cnt = nullptr, *px_off = nullptr;
  int32_t *lx_start = nullptr, *lx_cnt = nullptr, *lx_off = nullptr;
  // camera-major copies, written by the linearisation, of the R1 / R2 slots (cameras in
  // order, each camera's records in record order) and of their aligned R3 / R4 slots
  // (compact, in the same order): cmpos[fam][i] is record i's position, cmfeat[fam][j] the
  // feature at position j, cmal[fam][j] (fam 1, 2) the position of the aligned plane
  // record or -1, cmgrp[fam][k] (fam 3, 4) the plane of a plane-record position
  void *cmrec[NFAM] = {nullptr}, *cmres[NFAM] = {nullptr};  // slots and weighted residuals (T)
  int32_t *cmpos[NFAM] = {nullptr}, *cmfeat[NFAM] = {nullptr}, *cmal[NFAM] = {nullptr}, *cmgrp[NFAM] = {nullptr};
  // group member lists
  int32_t *plp_off = nullptr, *plp = nullptr, *pll_off = nullptr, *pll = nullptr;
  // camera of each workgroup of the per-camera passes: consecutive workgroups go to
  // different XCDs, so each XCD is given a run of spatially close cameras (which share
  // features, whose data its L2 then serves)
  int32_t* cam_order = nullptr;
  int32_t *vpm_off = nullptr, *vpm = nullptr;
  // surface groups: per shape its points (family 9) and lines (family 10) in feature order;
  // per observation record (camera-major position of R1 / R2) the index of the family 9 /
  // 10 record of the same camera and feature, or -1.  A point or line is on at most one
  // shape; a line on a cuboid is one of the product's big features.
  int32_t *shp_off = nullptr, *shp = nullptr, *shl_off = nullptr, *shl = nullptr;
  int32_t *shal_p = nullptr, *shal_l = nullptr;
  // per camera (offsets shc_off[k], nc + 1), its point-on-shape (k = 0) or line-on-cuboid
  // (k = 1) records in camera-major order and their features: the camera sweeps that add
  // each record on its own take them in a loop of their own
  int32_t *shc_off[2] = {nullptr, nullptr}, *shc_rec[2] = {nullptr, nullptr}, *shc_feat[2] = {nullptr, nullptr};
  // the shape passes take chunks of at most SH_CHUNK members of one shape, a workgroup
  // each: int4 (shape, first member, members, 0 points / 1 lines); FP64 accumulators
  // summed over a shape's chunks: U (packed) and g, or the S-block terms and b
  // (SH_ACC per shape), and the shape rows of S Z (SH_DOF x SZ_COLS x SZ_PANELS)
  int n_shch = 0;
  int4* shch = nullptr;
  double *shacc = nullptr, *shsz = nullptr;
  // feature blocks (T unless noted)
  void *Vp = nullptr, *gp = nullptr, *Vl = nullptr, *gl = nullptr;
  void *Vip = nullptr, *Vil = nullptr, *sp = nullptr, *sl = nullptr;
  double *Vip64 = nullptr, *Vil64 = nullptr;
  uint8_t *flp = nullptr, *fll = nullptr;
  double *Dp = nullptr, *Dl = nullptr;
  double *hp = nullptr, *hl = nullptr;
  // A side (double)
  double *Ucam = nullptr, *Upl = nullptr, *Uvp = nullptr, *Ush = nullptr;  // full blocks
  double *gA = nullptr, *DA = nullptr, *bA = nullptr;
  double *Scam = nullptr, *Spl = nullptr, *Svp = nullptr, *Ssh = nullptr;  // damped diagonal blocks of S
  double *Mcam = nullptr, *Mpl = nullptr, *Mvp = nullptr, *Msh = nullptr;  // preconditioner blocks
  // two-level preconditioner: Z (coarse_k columns of length nA, column-major; the
  // gauge columns first), S Z, E^-1 = (Z^T S Z)^-1 (COARSE_K x COARSE_K storage),
  // Z^T b; PCG starts from x0 = Z E^-1 Z^T b and applies (I - Q S) M + Q, Q = Z E^-1 Z^T
  int coarse_k = 0;            // active columns (0: block-Jacobi; SC_COARSE decides on the device)
  double *Zc = nullptr, *SZc = nullptr, *Einv = nullptr, *Ztb = nullptr;
  void *szr = nullptr, *szfp = nullptr, *szfl = nullptr;  // S Z sweeps: Z rows, s_f of points / lines (T)
  // PCG (double vectors of length nA) and matvec partials (T)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  void *xT = nullptr;       // matvec input in T
  double *mv_part = nullptr;  // n_mv_wg x nA partial sums (LDS mode) or nA accumulator (global mode)
  double *scal = nullptr;   // device scalars, see PcgScal
  double *red = nullptr;    // reduction partials
  int64_t n_red_max = 0;    // pairs of partials red holds
  int n_mv_wg = 0;          // matvec workgroups (partials rows)
  int mv_lds = 0;           // 1: accumulate in LDS
  int mv_stage = 0;         // 1: FP32 with point-on-shape records (LDS staging of their rows)
  // wavefront tiles of the product: int4 (first slot, slots, first feature, 0), point tiles
  // first, then line tiles; one slot per record in feature order, int4 ((family << 28) |
  // record, camera, group, feature - first feature of the tile)
  int n_tiles = 0, n_ptiles = 0;
  int4* tiles = nullptr;
  int4* wrec = nullptr;
  // features too large for one tile (and lines on a shape): one wavefront each in the
  // product, S Z and back-substitution, one lane each in the deterministic pass
  int n_bigp = 0, n_bigl = 0;
  int32_t *bigp = nullptr, *bigl = nullptr;
  // inter-group relations (A-side records, FP64): group indices (planes or VPs), kind
  // 0 VP orthogonal, 1 VP parallel, 2 plane orthogonal, 3 plane parallel; weighted
  // residual (3 rows, unused rows zero) and Jacobian (3 rows x [J_a (3) | J_b (3)],
  // a VP's third column zero); per group block (planes, then VPs) a CSR of its
  // entries 2 * record + side; rel_y: the relations' part of S x (group rows)
  int n_rel = 0;
  int32_t *rel_ga = nullptr, *rel_gb = nullptr, *rel_kind = nullptr;
  int32_t *rel_goff = nullptr, *rel_gent = nullptr;
  double *rel_r = nullptr, *rel_J = nullptr, *rel_y = nullptr;
  int rel_lkind[4] = {0, 0, 0, 0};
  double rel_lscale[4] = {0, 0, 0, 0}, rel_lweight[4] = {0, 0, 0, 0};
  // dense Schur solver (reduced systems of at most DENSE_MAX_NA rows; the tables exist
  // when dense_n > 0).  A blocks are numbered cameras, planes, VPs.  fent: one entry per
  // (feature, distinct block of its records), feature = point index or np + line index;
  // dY: per entry Y = W_fa G_f (DENSE_Y doubles, element (i, k) at k * 9 + i: i < 9 rows
  // of the block, k < 4 feature coordinates, zero beyond the block's and the feature's
  // sizes), with W_fa = sum over the feature's records touching block a of J_a^T J_f and
  // G_f G_f^T = V_f^-1, so that W_fa V_f^-1 W_fb^T = Y_fa Y_fb^T.  Pairs (a <= b) of
  // blocks that S couples, every diagonal pair included, sorted by (a, b); per pair the
  // entries (e_a, e_b) of its shared features (in feature order) and its U entries
  // (code, index): code 3 / 4 a family-3 / 4 record touching (camera a, plane b), code 8
  // a relation with block(ga) = a, 9 one with block(gb) = a.  dS: S (dense_npad squared,
  // row-major; the padding rows are the identity), overwritten by its lower Cholesky
  // factor; dLinv: the inverse of each 64 x 64 diagonal factor tile; dv, dw: solve vectors
  // Pairs with more than DENSE_CHUNK shared features are split into chunks of at most
  // DENSE_CHUNK entries (chunk: entry range), summed per chunk into dpart (3 x 64 doubles)
  // and then per pair in chunk order; pair_choff: per pair, its range of chunks.
  int dense_n = 0, dense_npad = 0, n_fent = 0, n_pair = 0, n_chunk = 0;
  int2 *fent = nullptr, *pair_ab = nullptr, *pair_ent = nullptr, *pair_u = nullptr, *chunk = nullptr;
  int32_t *pair_off = nullptr, *pair_uoff = nullptr, *pair_choff = nullptr;
  double *dY = nullptr, *dS = nullptr, *dLinv = nullptr, *dv = nullptr, *dw = nullptr, *dpart = nullptr;
  int* dinfo = nullptr;
  // records left out (the reliability-aware refinement): with has_mask, a record whose
  // parameters include a point, line, plane or VP flagged here (internal order) has
  // zero weight in the linearisation and no cost; the flagged parameters do not move
  int has_mask = 0;
  uint8_t *mpt = nullptr, *mln = nullptr, *mpl = nullptr, *mvp = nullptr;
  // deterministic mode: the product's s_f per feature (T; points x 3, lines x 4) and the
  // per-workgroup partials of the PCG dot products (det_stride workgroups per accumulator:
  // the SC_COUNT scalars, then the COARSE_K entries of Z^T b)
  int det = 0, det_stride = 0;
  void *sdp = nullptr, *sdl = nullptr;
  double* detp = nullptr;
  unsigned int *cnt = nullptr;  // grid-wide "last workgroup" counters (zeroed, self-resetting)
  double *part2 = nullptr;      // per-workgroup partial dot products of the PCG kernels
};

// record i of family FAM (feature f) left out by the record mask: its point or line
// (a junction record's partner feature only supplies the measurement), its plane or VP
template <int FAM> __device__ __forceinline__ bool record_masked(const Dev& d, int64_t i, int f) {
  if (!d.has_mask) return false;
  const bool line = FAM == 2 || FAM == 4 || FAM == 5 || FAM == 7 || FAM == 10;
  if ((line ? d.mln : d.mpt)[f]) return true;
  if constexpr (FAM == 3 || FAM == 4 || FAM == 8) return d.mpl[d.fgrp[FAM][i]] != 0;
  if constexpr (FAM == 5) return d.mvp[d.fgrp[FAM][i]] != 0;
  return false;  // shapes are not left out
}

// first entry of group g of type gt (1 plane, 2 VP, 3 shape) in the reduced vector
__host__ __device__ __forceinline__ int a_grp(const Dev& d, int gt, int g) {
  return gt == 1 ? d.offPl + 3 * g : gt == 2 ? d.offVp + 2 * g : d.offSh + SH_DOF * g;
}

// product: 1024-thread workgroups sharing one FP64 copy of y in LDS (FP32 LDS atomics
// measured 2x slower on gfx950); each wavefront takes tiles of at most MV_TILE records
constexpr int MV_THREADS = 1024, MV_TILE = 64;
// the product's large features (k_mv_big): 8 wavefronts per workgroup, each one feature,
// with the shape rows summed in LDS when at most MV_BIG_SH_MAX of them
constexpr int MV_BIG_THREADS = 512, MV_BIG_SH_MAX = 4096;
// LDS staging of the FP32 product on scenes with point-on-shape records, after y: the
// shape rows of each wavefront's lanes (SH_DOF x 64 floats) and each lane's shape offset
constexpr int MV_STAGE_BYTES = MV_THREADS / 64 * SH_DOF * 64 * 4 + MV_THREADS * 4;

// indices into Dev::scal
enum PcgScal {
  SC_RZ = 0, SC_BB, SC_RR, SC_PQ, SC_ALPHA, SC_BETA, SC_DONE, SC_ITER, SC_TOL2, SC_LAMBDA,
  SC_GH, SC_JH2, SC_E, SC_EPIX, SC_NFLAG, SC_MAXIT, SC_BREAK,
  SC_COARSE,  // 1: the coarse correction of the preconditioner is active for this solve
  SC_NDEG,    // records of the current linearisation with a scaled or dropped Jacobian
  SC_GINF,    // |g|_inf of the current linearisation
  SC_NFAIL,   // feature blocks whose FP64 Cholesky failed too (zero inverse)
  // PCG accumulators, three sets rotated by iteration (k mod 3): p.q, r.r, r.(M r),
  // Z^T r, (S Z)^T (M r)
  SC_ACC = 24, SC_COUNT = 128
};
static_assert(SC_NFAIL < SC_ACC, "single scalars overlap the PCG accumulators");
// coarse space of the two-level preconditioner: 7 similarity-gauge columns, then the
// network's columns
constexpr int COARSE_GAUGE = 7, COARSE_NET = 8, COARSE_K = COARSE_GAUGE + COARSE_NET;
// the coarse columns in the S Z sweeps (Z rows, s_f) are stored in panels of SZ_COLS
// columns, row-major within a panel
constexpr int SZ_COLS = 8, SZ_PANELS = 2;
constexpr int SH_CHUNK = 128, SH_ACC = SH_DOF * (SH_DOF + 1) / 2 + SH_DOF;
static_assert(COARSE_K <= SZ_COLS * SZ_PANELS, "coarse columns per S Z panel set");
// With FP32 records the product resolves S Z only to ~1e-7 |S| |Z|, while on the
// near-null (gauge) directions S Z ~ lambda D_A Z: below this damping the coarse
// matrix E is not resolved, and the FP32 path preconditions with block-Jacobi alone.
constexpr double COARSE_MIN_DAMPING_FP32 = 1e-6;
// Above this damping S is dominated by its damped diagonal blocks and block-Jacobi
// PCG needs a handful of iterations: fewer than the coarse set-up costs in products.
constexpr double COARSE_MAX_DAMPING = 0.1;
constexpr int ACC_PQ = 0, ACC_RR = 1, ACC_RZ = 2, ACC_ZR = 4, ACC_W = ACC_ZR + COARSE_K, ACC_STRIDE = ACC_W + COARSE_K;
static_assert(SC_ACC + 3 * ACC_STRIDE <= SC_COUNT, "PCG scalar area too small");

// runs the statement with T (the working precision) and CD (camera dof) bound
#define BA_DISPATCH_T_CD(d, ...)                                      \
  do {                                                                \
    if ((d).fp64) {                                                   \
      using T = double;                                               \
      if ((d).CD == 9) { constexpr int CD = 9; __VA_ARGS__; }         \
      else { constexpr int CD = 6; __VA_ARGS__; }                     \
    } else {                                                          \
      using T = float;                                                \
      if ((d).CD == 9) { constexpr int CD = 9; __VA_ARGS__; }         \
      else { constexpr int CD = 6; __VA_ARGS__; }                     \
    }                                                                 \
  } while (0)

// ---- launchers (ba_kernels.hip) --------------------------------------------
void launch_cast_params(const Dev& d, bool candidate, hipStream_t s);
void launch_linearize(const Dev& d, hipStream_t s);
void launch_cost(const Dev& d, bool candidate, hipStream_t s);           // -> scal[SC_E], scal[SC_EPIX]
void launch_feature_accum(const Dev& d, hipStream_t s);                  // V_f, g_f, D_f
void launch_grad_inf(const Dev& d, hipStream_t s);                       // -> scal[SC_GINF]
void launch_camera_pass_a(const Dev& d, hipStream_t s);                  // U_a, g_a, D_a
void launch_feature_invert(const Dev& d, double lambda, double kappa_max, hipStream_t s);  // V^-1, s_f, flags
void launch_camera_pass_b(const Dev& d, double lambda, hipStream_t s);   // S diag blocks, b
void launch_precond_blockjacobi(const Dev& d, hipStream_t s);           // M = blockdiag(S)^-1
void launch_pcg_init(const Dev& d, double tol, int max_iters, hipStream_t s);
void launch_pcg_product(const Dev& d, hipStream_t s);                  // q' = partial J_a^T(...) products
void launch_pcg_update(const Dev& d, double lambda, int iter, hipStream_t s);  // q = S p, then the CG update
void launch_schur_matvec(const Dev& d, const double* xin, double* yout, double lambda, hipStream_t s);
// S (nA x nA, device; column c = S e_c) by nA products
void launch_dense_schur(const Dev& d, double lambda, double* S, hipStream_t s);
// dense Schur solver (ba_dense.hip), after the feature inverses and b of the current
// lambda: launch_dense_assemble forms S in d.dS; launch_dense_solve forms, factors and
// solves S h_a = b into d.x, leaving *d.dinfo = 1 + the first column with a
// non-positive pivot (then d.x is unchanged), else 0; launch_dense_residual puts
// |S x - b|^2 and |b|^2 (S x from the implicit product) into the PCG scalars
constexpr int DENSE_MAX_NA = 8192, DENSE_Y = 36, DENSE_NB = 64, DENSE_CHUNK = 64;
void launch_dense_assemble(const Dev& d, double lambda, hipStream_t s);
void launch_dense_solve(const Dev& d, double lambda, hipStream_t s);
void launch_dense_residual(const Dev& d, double lambda, hipStream_t s);
// Cholesky factorisation of the SPD matrix A (npad x npad, row-major, npad a multiple of
// DENSE_NB, lower triangle read and overwritten by L) and the solve A x = v (v
// overwritten by x), with Linv (npad / DENSE_NB tiles of DENSE_NB^2) and w (npad) as
// work space; *info (device, zero on entry) is set to 1 + the first column with a
// non-positive pivot
void launch_dense_factor_solve(double* A, int npad, double* Linv, double* v, double* w, int* info, hipStream_t s);
// A (npad x npad) = 0 except the identity on rows n .. npad - 1
void launch_dense_pad_identity(double* A, int n, int npad, hipStream_t s);
// zero the strict upper triangle of A (npad x npad)
void launch_dense_zero_upper(double* A, int npad, hipStream_t s);
// inter-group relations (ba_rel.hip)
void launch_rel_linearize(const Dev& d, hipStream_t s);
void launch_rel_a(const Dev& d, hipStream_t s);          // after the group pass A: U_gg, g_g, D_g
void launch_rel_matvec(const Dev& d, const double* done, hipStream_t s);  // d.rel_y from d.xT
void launch_rel_sz(const Dev& d, hipStream_t s);         // S Z += U_rel Z on the active columns
void launch_rel_cost(const Dev& d, bool candidate, double* part, hipStream_t s);  // one partial
void launch_rel_md(const Dev& d, hipStream_t s);  // after the model decrease: + sum |J~ h_a|^2
// columns c0 .. c0 + ncols - 1 of the damped reduced matrix into S (ncols x n_A)
void launch_dense_schur_columns(const Dev& d, double lambda, int c0, int ncols, double* S, hipStream_t s);
// gauge columns of d.Zc from the current parameters
void launch_gauge_basis(const Dev& d, hipStream_t s);
// S Z and E = Z^T S Z for the first d.coarse_k columns of d.Zc, E^-1 and SC_COARSE
void launch_coarse_setup(const Dev& d, double lambda, hipStream_t s);
void launch_backsub(const Dev& d, hipStream_t s);                        // h_f, model decrease terms
// surface groups (ba_shape.hip): U, g, D of the shape blocks (after the camera pass A);
// their damped S blocks and b (after the camera pass B); their gauge rows
void launch_shape_pass_a(const Dev& d, hipStream_t s);
void launch_shape_pass_b(const Dev& d, double lambda, hipStream_t s);
void launch_shape_gauge(const Dev& d, hipStream_t s);
void launch_retract(const Dev& d, hipStream_t s);                        // candidate = current [+] h
void launch_zero(void* p, size_t bytes, hipStream_t s);
// per point (NF 3, observation records R1) or line (NF 4, R2): active observations
// (residual in the quadratic part of the loss), observations, and sigma =
// lambda_min(V_f)^-1/2 (points: over the mean distance to the observing cameras)
void launch_feature_stats(const Dev& d, int32_t* n_active, int32_t* n_obs, double* sigma, int nf, hipStream_t s);
// the product's dynamic LDS: the most a workgroup may take, and what it takes for d (y
// when accumulated in LDS, then the staging)
int matvec_max_lds_bytes();
size_t matvec_lds_bytes(const Dev& d);

}  // namespace ba
