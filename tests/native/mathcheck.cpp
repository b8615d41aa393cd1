// Test helper: evaluates one residual record with the library's device math
// templates compiled for the host, so that the analytic Jacobians can be
// compared with the oracle on the CPU.  Not part of the product library.
#include "../../paper_2609_04026_amd/csrc/ba_math.h"

using namespace ba;

namespace {
template <typename S, int CD>
int eval(int fam, const double* cam, const double* pt, const double* ln, const double* pl, const double* vp,
         const double* meas, double* r, double* Jc, double* Jg, double* Jf) {
  S rr[4] = {0, 0, 0, 0}, jc[4 * 9] = {0}, jg[4 * 3] = {0}, jf[4 * 4] = {0}, m[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) m[k] = (S)meas[k];
  Cam<S> C = load_cam<S>(cam);
  S X[3] = {(S)pt[0], (S)pt[1], (S)pt[2]};
  Line<S> L = load_line<S>(ln);
  Plane<S> P = load_plane<S>(pl);
  Vp<S> V = load_vp<S>(vp);
  int rows = 0, nc = 0, ng = 0, nf = 0;
  switch (fam) {
    case 1: jac_R1<S, CD>(C, X, m, rr, jc, jf); rows = 2; nc = CamCols<CD>::PT; nf = 3; break;
    case 2: jac_R2<S, CD>(C, L, m, rr, jc, jf); rows = 4; nc = CamCols<CD>::LN; nf = 4; break;
    case 3: jac_R3<S, CD>(C, X, P, rr, jc, jg, jf); rows = 2; nc = CamCols<CD>::PT; ng = 3; nf = 3; break;
    case 4: jac_R4<S, CD>(C, L, P, m, rr, jc, jg, jf); rows = 4; nc = CamCols<CD>::LN; ng = 3; nf = 4; break;
    case 5: jac_R5<S>(L, V, rr, jg, jf); rows = 3; ng = 2; nf = 4; break;
    case 6: jac_R6<S, CD>(C, X, m, rr, jc, jf); rows = 1; nc = CamCols<CD>::PT; nf = 3; break;
    case 7: jac_R7<S, CD>(C, L, m, rr, jc, jf); rows = 1; nc = CamCols<CD>::LN; nf = 4; break;
    case 12: jac_R12<S>(X, P, rr, jg, jf); rows = 1; ng = 3; nf = 3; break;
    default: return -1;
  }
  for (int i = 0; i < rows; ++i) {
    r[i] = rr[i];
    for (int k = 0; k < CD; ++k) Jc[i * 9 + k] = k < nc ? (double)jc[i * nc + k] : 0.0;
    for (int k = 0; k < ng; ++k) Jg[i * 3 + k] = jg[i * ng + k];
    for (int k = 0; k < nf; ++k) Jf[i * 4 + k] = jf[i * nf + k];
  }
  return rows;
}

template <typename S>
void res(int fam, const double* cam, const double* pt, const double* ln, const double* pl, const double* vp,
         const double* meas, double* r) {
  S rr[4] = {0, 0, 0, 0}, m[4];
  for (int k = 0; k < 4; ++k) m[k] = (S)meas[k];
  Cam<S> C = load_cam<S>(cam);
  S X[3] = {(S)pt[0], (S)pt[1], (S)pt[2]};
  Line<S> L = load_line<S>(ln);
  Plane<S> P = load_plane<S>(pl);
  Vp<S> V = load_vp<S>(vp);
  switch (fam) {
    case 1: res_R1<S>(C, X, m, rr); break;
    case 2: res_R2<S>(C, L, m, rr); break;
    case 3: res_R3<S>(C, X, P, rr); break;
    case 4: res_R4<S>(C, L, P, m, rr); break;
    case 5: res_R5<S>(L, V, rr); break;
    case 6: res_R6<S>(C, X, m, rr); break;
    case 7: res_R7<S>(C, L, m, rr); break;
    case 12: res_R12<S>(X, P, rr); break;
  }
  for (int k = 0; k < 4; ++k) r[k] = rr[k];
}
}  // namespace

extern "C" int mc_eval(int fam, int cd, int fp64, const double* cam, const double* pt, const double* ln,
                       const double* pl, const double* vp, const double* meas, double* r, double* Jc, double* Jg,
                       double* Jf) {
  if (fam == 3 || fam == 4) fp64 = 1;  // the library evaluates these families in FP64
  if (fp64) return cd == 9 ? eval<double, 9>(fam, cam, pt, ln, pl, vp, meas, r, Jc, Jg, Jf)
                           : eval<double, 6>(fam, cam, pt, ln, pl, vp, meas, r, Jc, Jg, Jf);
  return cd == 9 ? eval<float, 9>(fam, cam, pt, ln, pl, vp, meas, r, Jc, Jg, Jf)
                 : eval<float, 6>(fam, cam, pt, ln, pl, vp, meas, r, Jc, Jg, Jf);
}

extern "C" void mc_residual(int fam, int fp64, const double* cam, const double* pt, const double* ln, const double* pl,
                            const double* vp, const double* meas, double* r) {
  if (fp64) res<double>(fam, cam, pt, ln, pl, vp, meas, r);
  else res<float>(fam, cam, pt, ln, pl, vp, meas, r);
}

// R13 / R14: one record against a shape in its device layout (SH_STRIDE doubles);
// the cuboid face is chosen in FP64, as the library does.  Jg is 4 x SH_DOF.
namespace {
template <typename S, int CD>
int eval_shape(int fam, const double* cam, const double* pt, const double* ln, const double* sh, const double* meas,
               double* r, double* Jc, double* Jg, double* Jf) {
  S rr[4] = {0, 0, 0, 0}, jc[4 * 9] = {0}, jg[4 * SH_DOF] = {0}, jf[4 * 4] = {0}, m[4];
  S shp[SH_STRIDE];
  for (int k = 0; k < 4; ++k) m[k] = (S)meas[k];
  for (int k = 0; k < SH_STRIDE; ++k) shp[k] = (S)sh[k];
  Cam<S> C = load_cam<S>(cam);
  int rows = 0, nc = 0, nf = 0, face = 0;
  if (fam == 13) {
    S X[3] = {(S)pt[0], (S)pt[1], (S)pt[2]};
    if (shape_type(sh) == SH_CUBOID) face = cuboid_face<double>(sh, pt);
    jac_R13<S, CD>(C, X, shp, face, rr, jc, jg, jf);
    rows = 2; nc = CamCols<CD>::PT; nf = 3;
  } else if (fam == 14) {
    Line<S> L = load_line<S>(ln);
    const Line<double> L64 = load_line<double>(ln);
    double d[3], mm[3];
    line_dm(L64, d, mm);
    face = cuboid_face_line<double>(sh, d, mm);
    jac_R14<S, CD>(C, L, shp, face, m, rr, jc, jg, jf);
    rows = 4; nc = CamCols<CD>::LN; nf = 4;
  } else {
    return -1;
  }
  for (int i = 0; i < rows; ++i) {
    r[i] = rr[i];
    for (int k = 0; k < CD; ++k) Jc[i * 9 + k] = k < nc ? (double)jc[i * nc + k] : 0.0;
    for (int k = 0; k < SH_DOF; ++k) Jg[i * SH_DOF + k] = jg[i * SH_DOF + k];
    for (int k = 0; k < nf; ++k) Jf[i * 4 + k] = jf[i * nf + k];
  }
  return rows;
}
}  // namespace

extern "C" int mc_eval_shape(int fam, int cd, int fp64, const double* cam, const double* pt, const double* ln,
                             const double* sh, const double* meas, double* r, double* Jc, double* Jg, double* Jf) {
  fp64 = 1;  // the library evaluates these families in FP64 and stores them in the working precision
  if (fp64) return cd == 9 ? eval_shape<double, 9>(fam, cam, pt, ln, sh, meas, r, Jc, Jg, Jf)
                           : eval_shape<double, 6>(fam, cam, pt, ln, sh, meas, r, Jc, Jg, Jf);
  return cd == 9 ? eval_shape<float, 9>(fam, cam, pt, ln, sh, meas, r, Jc, Jg, Jf)
                 : eval_shape<float, 6>(fam, cam, pt, ln, sh, meas, r, Jc, Jg, Jf);
}
