// Residuals and analytic Jacobians of the seven residual families of the
// holistic bundle adjustment, templated on the scalar type (float for the
// mixed-precision path, double for the FP64 path and for every cost).
//
// Families (Sec. 3.1 - 3.4 of the paper):
//   R1 point reprojection pi_p(C, X) - x                          (Eq. 1)
//   R2 line reprojection rho(pi_l(C, L), l) in R^4                 (Eq. 4)
//   R3 plane-induced point  pi_p(C, X) - pi_p(C, Proj_G(X))        (Eq. 7)
//   R4 plane-induced line   rho(l(L)) - rho(l(Proj_G(L)))          (Eq. 8, App. B)
//   R5 VP-line  (d/|d|) x v, norm = |sin theta|                    (Eq. 6, App. B)
//   R6 point -> observed line distance (undistorted)              (Eq. 11)
//   R7 observed point -> projected line distance (undistorted)    (Eq. 12)
//   R12 point -> plane metric distance n . X + w (3D formulation baseline)
//
// Conventions: X_c = R X + t; pose tangent (dtheta, dt) acts on the camera
// frame, X_c <- Exp(dtheta) X_c + dt, so dX_c/dtheta_k = e_k x X_c and
// dX_c/dt = I; intrinsics f, k1, k2 follow (camera_dof 9) or are fixed (6).
// Lines: d = w1 u1, m = w2 u2 (m = p x d), tangent U <- U Exp(dtheta_L),
// (w1, w2) rotated by dphi.  Planes n . x + w = 0, tangent (B_n dn, dw);
// VPs v, tangent B_v dv.  Image measurements are stored shifted by the
// principal point, so the image line of (d_c, m_c) is (m_c,x, m_c,y, f m_c,z).
#pragma once
#include <hip/hip_runtime.h>

#define BA_HD __host__ __device__ __forceinline__

namespace ba {

// parameter strides (elements) in the device arrays
constexpr int CAM_STRIDE = 16;    // R (row-major 9), t (3), f, k1, k2, pad
constexpr int PT_STRIDE = 4;      // X (3), pad
constexpr int LN_STRIDE = 12;     // u1 (3), u2 (3), u3 (3), w1, w2, pad
constexpr int PL_STRIDE = 12;     // n (3), w, b1 (3), b2 (3), pad (2)
constexpr int VP_STRIDE = 12;     // v (3), pad, b1 (3), b2 (3), pad (2)

template <typename S> struct Cam { S R[9]; S t[3]; S f, k1, k2; };
template <typename S> struct Line { S u1[3], u2[3], u3[3]; S w1, w2; };
template <typename S> struct Plane { S n[3]; S w; S b1[3], b2[3]; };
template <typename S> struct Vp { S v[3]; S b1[3], b2[3]; };

template <typename S, typename P> BA_HD Cam<S> load_cam(const P* p) {
  Cam<S> c;
#pragma unroll
  for (int i = 0; i < 9; ++i) c.R[i] = (S)p[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) c.t[i] = (S)p[9 + i];
  c.f = (S)p[12]; c.k1 = (S)p[13]; c.k2 = (S)p[14];
  return c;
}
template <typename S, typename P> BA_HD Line<S> load_line(const P* p) {
  Line<S> l;
#pragma unroll
  for (int i = 0; i < 3; ++i) { l.u1[i] = (S)p[i]; l.u2[i] = (S)p[3 + i]; l.u3[i] = (S)p[6 + i]; }
  l.w1 = (S)p[9]; l.w2 = (S)p[10];
  return l;
}
template <typename S, typename P> BA_HD Plane<S> load_plane(const P* p) {
  Plane<S> g;
#pragma unroll
  for (int i = 0; i < 3; ++i) { g.n[i] = (S)p[i]; g.b1[i] = (S)p[4 + i]; g.b2[i] = (S)p[7 + i]; }
  g.w = (S)p[3];
  return g;
}
template <typename S, typename P> BA_HD Vp<S> load_vp(const P* p) {
  Vp<S> v;
#pragma unroll
  for (int i = 0; i < 3; ++i) { v.v[i] = (S)p[i]; v.b1[i] = (S)p[4 + i]; v.b2[i] = (S)p[7 + i]; }
  return v;
}

template <typename S> BA_HD S dot3(const S* a, const S* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <typename S> BA_HD void cross3(const S* a, const S* b, S* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
template <typename S> BA_HD void rot(const S* R, const S* x, S* o) {
  o[0] = R[0] * x[0] + R[1] * x[1] + R[2] * x[2];
  o[1] = R[3] * x[0] + R[4] * x[1] + R[5] * x[2];
  o[2] = R[6] * x[0] + R[7] * x[1] + R[8] * x[2];
}
// e_k x p
template <typename S> BA_HD void ekx(int k, const S* p, S* o) {
  if (k == 0) { o[0] = 0; o[1] = -p[2]; o[2] = p[1]; }
  else if (k == 1) { o[0] = p[2]; o[1] = 0; o[2] = -p[0]; }
  else { o[0] = -p[1]; o[1] = p[0]; o[2] = 0; }
}

// --------------------------------------------------------------------------
// number of camera columns stored for point-type and line-type records
template <int CD> struct CamCols { static constexpr int PT = CD; static constexpr int LN = (CD == 9 ? 7 : 6); };

// --------------------------------------------------------------------------
// point projection
// --------------------------------------------------------------------------
template <typename S> struct PProj {
  S p[3];       // camera coordinates
  S u, v, s;    // normalised coordinates, radial factor
  S r2;
  S x, y;       // pixel minus principal point
  S B[2][3];    // d(x, y) / d p
};

template <typename S, bool DIST> BA_HD void pproject(const Cam<S>& c, const S* X, PProj<S>& o, bool jac) {
  S q[3];
  rot(c.R, X, q);
  o.p[0] = q[0] + c.t[0]; o.p[1] = q[1] + c.t[1]; o.p[2] = q[2] + c.t[2];
  S iz = S(1) / o.p[2];
  o.u = o.p[0] * iz; o.v = o.p[1] * iz;
  o.r2 = o.u * o.u + o.v * o.v;
  o.s = DIST ? S(1) + o.r2 * (c.k1 + c.k2 * o.r2) : S(1);
  o.x = c.f * o.s * o.u;
  o.y = c.f * o.s * o.v;
  if (!jac) return;
  S ds = DIST ? S(2) * (c.k1 + S(2) * c.k2 * o.r2) : S(0);
  S a00 = c.f * (o.s + ds * o.u * o.u), a01 = c.f * ds * o.u * o.v, a11 = c.f * (o.s + ds * o.v * o.v);
  o.B[0][0] = iz * a00; o.B[0][1] = iz * a01; o.B[0][2] = -iz * (a00 * o.u + a01 * o.v);
  o.B[1][0] = iz * a01; o.B[1][1] = iz * a11; o.B[1][2] = -iz * (a01 * o.u + a11 * o.v);
}

// camera columns of d(x,y)/d(camera) for rows `row` given B (1x3 row), p, and intrinsic partials
template <typename S, int NC> BA_HD void cam_cols_point(const S* Brow, const S* p, S df, S dk1, S dk2, S* Jrow) {
  S e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { ekx(k, p, e); Jrow[k] = dot3(Brow, e); }
  Jrow[3] = Brow[0]; Jrow[4] = Brow[1]; Jrow[5] = Brow[2];
  if (NC >= 7) Jrow[6] = df;
  if (NC >= 9) { Jrow[7] = dk1; Jrow[8] = dk2; }
}

template <typename S> BA_HD void feat_cols_point(const S* Brow, const S* R, S* Jrow) {
  // Brow * R
  Jrow[0] = Brow[0] * R[0] + Brow[1] * R[3] + Brow[2] * R[6];
  Jrow[1] = Brow[0] * R[1] + Brow[1] * R[4] + Brow[2] * R[7];
  Jrow[2] = Brow[0] * R[2] + Brow[1] * R[5] + Brow[2] * R[8];
}

// ---- R1 -------------------------------------------------------------------
// meas: observed distorted pixel minus principal point
template <typename S> BA_HD void res_R1(const Cam<S>& c, const S* X, const S* meas, S* r) {
  PProj<S> o;
  pproject<S, true>(c, X, o, false);
  r[0] = o.x - meas[0];
  r[1] = o.y - meas[1];
}

template <typename S, int CD> BA_HD void jac_R1(const Cam<S>& c, const S* X, const S* meas, S* r, S* Jc, S* Jf) {
  constexpr int NC = CamCols<CD>::PT;
  PProj<S> o;
  pproject<S, true>(c, X, o, true);
  r[0] = o.x - meas[0];
  r[1] = o.y - meas[1];
  S su = o.s * o.u, sv = o.s * o.v, r4 = o.r2 * o.r2;
  cam_cols_point<S, NC>(o.B[0], o.p, su, c.f * o.r2 * o.u, c.f * r4 * o.u, Jc);
  cam_cols_point<S, NC>(o.B[1], o.p, sv, c.f * o.r2 * o.v, c.f * r4 * o.v, Jc + NC);
  feat_cols_point(o.B[0], c.R, Jf);
  feat_cols_point(o.B[1], c.R, Jf + 3);
}

// ---- R3 -------------------------------------------------------------------
template <typename S> BA_HD void plane_proj_point(const Plane<S>& g, const S* X, S* Xp, S& cdist) {
  S nn = dot3(g.n, g.n);
  cdist = (dot3(g.n, X) + g.w) / nn;
  Xp[0] = X[0] - cdist * g.n[0]; Xp[1] = X[1] - cdist * g.n[1]; Xp[2] = X[2] - cdist * g.n[2];
}

template <typename S> BA_HD void res_R3(const Cam<S>& c, const S* X, const Plane<S>& g, S* r) {
  S Xp[3], cd;
  plane_proj_point(g, X, Xp, cd);
  PProj<S> a, b;
  pproject<S, true>(c, X, a, false);
  pproject<S, true>(c, Xp, b, false);
  r[0] = a.x - b.x;
  r[1] = a.y - b.y;
}

template <typename S, int CD>
BA_HD void jac_R3(const Cam<S>& c, const S* X, const Plane<S>& g, S* r, S* Jc, S* Jg, S* Jf) {
  constexpr int NC = CamCols<CD>::PT;
  S Xp[3], cd;
  plane_proj_point(g, X, Xp, cd);
  PProj<S> a, b;
  pproject<S, true>(c, X, a, true);
  pproject<S, true>(c, Xp, b, true);
  r[0] = a.x - b.x;
  r[1] = a.y - b.y;
  // camera: difference of the two point Jacobians
  S ja[NC], jb[NC];
  S ra4 = a.r2 * a.r2, rb4 = b.r2 * b.r2;
#pragma unroll
  for (int row = 0; row < 2; ++row) {
    S ua = row == 0 ? a.u : a.v, ub = row == 0 ? b.u : b.v;
    cam_cols_point<S, NC>(a.B[row], a.p, a.s * ua, c.f * a.r2 * ua, c.f * ra4 * ua, ja);
    cam_cols_point<S, NC>(b.B[row], b.p, b.s * ub, c.f * b.r2 * ub, c.f * rb4 * ub, jb);
#pragma unroll
    for (int k = 0; k < NC; ++k) Jc[row * NC + k] = ja[k] - jb[k];
  }
  // point: Ba R - Bb R (I - n n^T / |n|^2)
  S nn = dot3(g.n, g.n);
#pragma unroll
  for (int row = 0; row < 2; ++row) {
    S fa[3], fb[3];
    feat_cols_point(a.B[row], c.R, fa);
    feat_cols_point(b.B[row], c.R, fb);
    S fbn = dot3(fb, g.n) / nn;
#pragma unroll
    for (int k = 0; k < 3; ++k) Jf[row * 3 + k] = fa[k] - (fb[k] - fbn * g.n[k]);
  }
  // plane: dXp/dn = -(n X^T + c I) (tangent part, B ⟂ n), dXp/dw = -n; r = pi(X) - pi(Xp)
  S xb1 = dot3(X, g.b1), xb2 = dot3(X, g.b2);
  S d0[3], d1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d0[k] = g.n[k] * xb1 + cd * g.b1[k];
    d1[k] = g.n[k] * xb2 + cd * g.b2[k];
  }
#pragma unroll
  for (int row = 0; row < 2; ++row) {
    S fb[3];
    feat_cols_point(b.B[row], c.R, fb);  // dpi(Xp)/dXp
    Jg[row * 3 + 0] = dot3(fb, d0);
    Jg[row * 3 + 1] = dot3(fb, d1);
    Jg[row * 3 + 2] = dot3(fb, g.n);
  }
}

// ---- R6 -------------------------------------------------------------------
// meas: normalised observed line (l1, l2, l3) in shifted pixels, l1^2 + l2^2 = 1
template <typename S> BA_HD void res_R6(const Cam<S>& c, const S* X, const S* meas, S* r) {
  PProj<S> o;
  pproject<S, false>(c, X, o, false);
  r[0] = meas[0] * o.x + meas[1] * o.y + meas[2];
}

template <typename S, int CD> BA_HD void jac_R6(const Cam<S>& c, const S* X, const S* meas, S* r, S* Jc, S* Jf) {
  constexpr int NC = CamCols<CD>::PT;
  PProj<S> o;
  pproject<S, false>(c, X, o, true);
  r[0] = meas[0] * o.x + meas[1] * o.y + meas[2];
  S b[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) b[k] = meas[0] * o.B[0][k] + meas[1] * o.B[1][k];
  cam_cols_point<S, NC>(b, o.p, meas[0] * o.u + meas[1] * o.v, S(0), S(0), Jc);
  feat_cols_point(b, c.R, Jf);
}

// --------------------------------------------------------------------------
// lines
// --------------------------------------------------------------------------
template <typename S> struct LProj {
  S dc[3], mc[3];  // camera-frame Pluecker coordinates
  S l[3];          // image line in shifted pixels: (mc0, mc1, f mc2)
};

template <typename S> BA_HD void lproject(const Cam<S>& c, const S* d, const S* m, LProj<S>& o) {
  S rm[3], txd[3];
  rot(c.R, d, o.dc);
  rot(c.R, m, rm);
  cross3(c.t, o.dc, txd);
#pragma unroll
  for (int k = 0; k < 3; ++k) o.mc[k] = rm[k] + txd[k];
  o.l[0] = o.mc[0]; o.l[1] = o.mc[1]; o.l[2] = c.f * o.mc[2];
}

// Normal (l_1, l_2) of the image line of (d, m) in camera c, relative to
// |m| + |t| |d|, a bound on |m_c|.  It vanishes for a line through the camera
// centre or in the camera's principal plane: there the image line has no
// direction and the line-projection residuals are not differentiable.
template <typename S> BA_HD S image_line_normal(const Cam<S>& c, const S* d, const S* m) {
  LProj<S> o;
  lproject(c, d, m, o);
  const S den = sqrt(dot3(m, m)) + sqrt(dot3(c.t, c.t)) * sqrt(dot3(d, d));
  return den > S(0) ? sqrt(o.mc[0] * o.mc[0] + o.mc[1] * o.mc[1]) / den : S(0);
}
// Line-projection records (R2, R4, R7) whose image line is closer to degenerate
// than DEGENERATE_IMAGE_LINE keep their residual, and their Jacobian is scaled by
// (normal / DEGENERATE_IMAGE_LINE): same direction, the magnitude it has at the
// threshold.  Below FP64_IMAGE_LINE the working-precision path evaluates their
// Jacobian in FP64 (the image line is a difference of nearly equal terms there).
constexpr double DEGENERATE_IMAGE_LINE = 1e-3, FP64_IMAGE_LINE = 1e-2;

// endpoint vector and its derivative w.r.t. the image line (2 x 3)
template <typename S> BA_HD void endpoint(const S* l, const S* e, S* rho, S G[2][3], bool jac) {
  S h = l[0] * e[0] + l[1] * e[1] + l[2];
  S iq = S(1) / (l[0] * l[0] + l[1] * l[1]);
  S a = h * iq;
  rho[0] = a * l[0];
  rho[1] = a * l[1];
  if (!jac) return;
  S da[3] = {e[0] * iq - S(2) * a * l[0] * iq, e[1] * iq - S(2) * a * l[1] * iq, iq};
#pragma unroll
  for (int k = 0; k < 3; ++k) { G[0][k] = l[0] * da[k]; G[1][k] = l[1] * da[k]; }
  G[0][0] += a;
  G[1][1] += a;
}

// camera columns of a line-type row with d r / d l = G (1x3), line (dc, mc), focal f
template <typename S, int NC> BA_HD void cam_cols_line(const S* G, const LProj<S>& o, S f, S* Jrow) {
  S gm[3] = {G[0], G[1], G[2] * f};  // d r / d m_c
  S e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { ekx(k, o.mc, e); Jrow[k] = dot3(gm, e); }
#pragma unroll
  for (int k = 0; k < 3; ++k) { ekx(k, o.dc, e); Jrow[3 + k] = dot3(gm, e); }
  if (NC >= 7) Jrow[6] = G[2] * o.mc[2];
}

// d m_c / d xi_L (3 x 4, column-major dmc[k][0..2]) for the line tangent
template <typename S> BA_HD void line_tangent_mc(const Cam<S>& c, const Line<S>& L, S dmc[4][3]) {
  S a1[3], a2[3], a3[3];
  rot(c.R, L.u1, a1); rot(c.R, L.u2, a2); rot(c.R, L.u3, a3);
  // d(dc)/dxi = [0, -w1 a3, w1 a2, -w2 a1];  d(R m)/dxi = [w2 a3, 0, -w2 a1, w1 a2]
  S ddc[4][3], drm[4][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ddc[0][i] = 0; ddc[1][i] = -L.w1 * a3[i]; ddc[2][i] = L.w1 * a2[i]; ddc[3][i] = -L.w2 * a1[i];
    drm[0][i] = L.w2 * a3[i]; drm[1][i] = 0; drm[2][i] = -L.w2 * a1[i]; drm[3][i] = L.w1 * a2[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    S tx[3];
    cross3(c.t, ddc[k], tx);
    dmc[k][0] = drm[k][0] + tx[0]; dmc[k][1] = drm[k][1] + tx[1]; dmc[k][2] = drm[k][2] + tx[2];
  }
}

template <typename S> BA_HD void line_dm(const Line<S>& L, S* d, S* m) {
#pragma unroll
  for (int i = 0; i < 3; ++i) { d[i] = L.w1 * L.u1[i]; m[i] = L.w2 * L.u2[i]; }
}

// ---- R2 -------------------------------------------------------------------
// meas: e1x e1y e2x e2y minus principal point
template <typename S> BA_HD void res_R2(const Cam<S>& c, const Line<S>& L, const S* meas, S* r) {
  S d[3], m[3];
  line_dm(L, d, m);
  LProj<S> o;
  lproject(c, d, m, o);
  S G[2][3];
  endpoint(o.l, meas, r, G, false);
  endpoint(o.l, meas + 2, r + 2, G, false);
}

template <typename S, int CD>
BA_HD void jac_R2(const Cam<S>& c, const Line<S>& L, const S* meas, S* r, S* Jc, S* Jf) {
  constexpr int NC = CamCols<CD>::LN;
  S d[3], m[3];
  line_dm(L, d, m);
  LProj<S> o;
  lproject(c, d, m, o);
  S G[4][3];
  endpoint(o.l, meas, r, (S(*)[3])G[0], true);
  endpoint(o.l, meas + 2, r + 2, (S(*)[3])G[2], true);
  S dmc[4][3];
  line_tangent_mc(c, L, dmc);
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    cam_cols_line<S, NC>(G[row], o, c.f, Jc + row * NC);
    S gm[3] = {G[row][0], G[row][1], G[row][2] * c.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) Jf[row * 4 + k] = dot3(gm, dmc[k]);
  }
}

// ---- R7 -------------------------------------------------------------------
// meas: observed undistorted point minus principal point
template <typename S> BA_HD void res_R7(const Cam<S>& c, const Line<S>& L, const S* meas, S* r) {
  S d[3], m[3];
  line_dm(L, d, m);
  LProj<S> o;
  lproject(c, d, m, o);
  S h = o.l[0] * meas[0] + o.l[1] * meas[1] + o.l[2];
  r[0] = h / sqrt(o.l[0] * o.l[0] + o.l[1] * o.l[1]);
}

template <typename S, int CD>
BA_HD void jac_R7(const Cam<S>& c, const Line<S>& L, const S* meas, S* r, S* Jc, S* Jf) {
  constexpr int NC = CamCols<CD>::LN;
  S d[3], m[3];
  line_dm(L, d, m);
  LProj<S> o;
  lproject(c, d, m, o);
  S h = o.l[0] * meas[0] + o.l[1] * meas[1] + o.l[2];
  S q = o.l[0] * o.l[0] + o.l[1] * o.l[1];
  S iN = S(1) / sqrt(q);
  r[0] = h * iN;
  S iN3 = iN * iN * iN;
  S G[3] = {meas[0] * iN - h * o.l[0] * iN3, meas[1] * iN - h * o.l[1] * iN3, iN};
  cam_cols_line<S, NC>(G, o, c.f, Jc);
  S dmc[4][3];
  line_tangent_mc(c, L, dmc);
  S gm[3] = {G[0], G[1], G[2] * c.f};
#pragma unroll
  for (int k = 0; k < 4; ++k) Jf[k] = dot3(gm, dmc[k]);
}

// ---- R5 -------------------------------------------------------------------
template <typename S> BA_HD void res_R5(const Line<S>& L, const Vp<S>& V, S* r) {
  S iu = S(1) / sqrt(dot3(L.u1, L.u1));
  S u[3] = {L.u1[0] * iu, L.u1[1] * iu, L.u1[2] * iu};
  cross3(u, V.v, r);
}

template <typename S> BA_HD void jac_R5(const Line<S>& L, const Vp<S>& V, S* r, S* Jg, S* Jf) {
  S iu = S(1) / sqrt(dot3(L.u1, L.u1));
  S u[3] = {L.u1[0] * iu, L.u1[1] * iu, L.u1[2] * iu};
  cross3(u, V.v, r);
  // d u / d xi = [0, -u3, u2, 0]; d r = du x v
  S c1[3], c2[3], m3[3] = {-L.u3[0], -L.u3[1], -L.u3[2]};
  cross3(m3, V.v, c1);
  cross3(L.u2, V.v, c2);
  S g1[3], g2[3];
  cross3(u, V.b1, g1);
  cross3(u, V.b2, g2);
#pragma unroll
  for (int row = 0; row < 3; ++row) {
    Jf[row * 4 + 0] = 0; Jf[row * 4 + 1] = c1[row]; Jf[row * 4 + 2] = c2[row]; Jf[row * 4 + 3] = 0;
    Jg[row * 2 + 0] = g1[row]; Jg[row * 2 + 1] = g2[row];
  }
}

// ---- R4 -------------------------------------------------------------------
// plane projection of a Pluecker line (App. B) and its partial derivatives
// R12: the signed metric distance n . X + w of a point to a plane (the 3D
// formulation the paper compares against); plane tangent (b1, b2 of the normal, w)
template <typename S> BA_HD void res_R12(const S* X, const Plane<S>& g, S* r) { r[0] = dot3(g.n, X) + g.w; }

template <typename S> BA_HD void jac_R12(const S* X, const Plane<S>& g, S* r, S* Jg, S* Jf) {
  r[0] = dot3(g.n, X) + g.w;
  Jg[0] = dot3(g.b1, X);
  Jg[1] = dot3(g.b2, X);
  Jg[2] = S(1);
#pragma unroll
  for (int k = 0; k < 3; ++k) Jf[k] = g.n[k];
}

template <typename S> struct PlaneLine {
  S d2[3], m2[3];
  S Ddd[3][3];      // d d' / d d
  S Ddn[3][3];      // d d' / d n
  S Dmd[3][3];      // d m' / d d
  S Dmm[3][3];      // d m' / d m
  S Dmn[3][3];      // d m' / d n
  S Dmw[3];         // d m' / d w
  bool degenerate;
};

template <typename S> BA_HD void plane_line(const S* d, const S* m, const Plane<S>& g, PlaneLine<S>& o, bool jac) {
  const S* n = g.n;
  S al = dot3(d, n), ga = dot3(m, n);
  S dxn[3];
  cross3(d, n, dxn);
  S e = dot3(dxn, m);
  S D = dot3(d, d), iD = S(1) / D;
  S a = S(1) - al * al * iD, b = al * ga * iD, cc = g.w - e * iD;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o.d2[k] = d[k] - al * n[k];
    o.m2[k] = a * m[k] + b * d[k] + cc * dxn[k];
  }
  o.degenerate = dot3(o.d2, o.d2) < S(1e-12) * D;
  if (!jac) return;
  S nxm[3], mxd[3];
  cross3(n, m, nxm);
  cross3(m, d, mxd);
  S ga_d[3], ga_n[3], gb_d[3], gb_m[3], gb_n[3], gc_d[3], gc_m[3], gc_n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ga_d[k] = -S(2) * al * iD * n[k] + S(2) * al * al * iD * iD * d[k];
    ga_n[k] = -S(2) * al * iD * d[k];
    gb_d[k] = ga * iD * n[k] - S(2) * al * ga * iD * iD * d[k];
    gb_m[k] = al * iD * n[k];
    gb_n[k] = iD * (ga * d[k] + al * m[k]);
    gc_d[k] = -iD * nxm[k] + S(2) * e * iD * iD * d[k];
    gc_m[k] = -iD * dxn[k];
    gc_n[k] = -iD * mxd[k];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S id = (i == j) ? S(1) : S(0);
      o.Ddd[i][j] = id - n[i] * n[j];
      o.Ddn[i][j] = -(n[i] * d[j] + al * id);
      o.Dmd[i][j] = m[i] * ga_d[j] + b * id + d[i] * gb_d[j] + dxn[i] * gc_d[j];
      o.Dmm[i][j] = a * id + d[i] * gb_m[j] + dxn[i] * gc_m[j];
      o.Dmn[i][j] = m[i] * ga_n[j] + d[i] * gb_n[j] + dxn[i] * gc_n[j];
    }
    o.Dmw[i] = dxn[i];
  }
  // - c [n]x  (d(d x n)/dd = -[n]x)   and  + c [d]x  (d(d x n)/dn = [d]x)
  o.Dmd[0][1] += cc * n[2]; o.Dmd[0][2] -= cc * n[1];
  o.Dmd[1][0] -= cc * n[2]; o.Dmd[1][2] += cc * n[0];
  o.Dmd[2][0] += cc * n[1]; o.Dmd[2][1] -= cc * n[0];
  o.Dmn[0][1] -= cc * d[2]; o.Dmn[0][2] += cc * d[1];
  o.Dmn[1][0] += cc * d[2]; o.Dmn[1][2] -= cc * d[0];
  o.Dmn[2][0] -= cc * d[1]; o.Dmn[2][1] += cc * d[0];
}

template <typename S> BA_HD void res_R4(const Cam<S>& c, const Line<S>& L, const Plane<S>& g, const S* meas, S* r) {
  S d[3], m[3];
  line_dm(L, d, m);
  PlaneLine<S> P;
  plane_line(d, m, g, P, false);
  if (P.degenerate) { r[0] = r[1] = r[2] = r[3] = 0; return; }
  LProj<S> o1, o2;
  lproject(c, d, m, o1);
  lproject(c, P.d2, P.m2, o2);
  S G[2][3], r2[4];
  endpoint(o1.l, meas, r, G, false);
  endpoint(o1.l, meas + 2, r + 2, G, false);
  endpoint(o2.l, meas, r2, G, false);
  endpoint(o2.l, meas + 2, r2 + 2, G, false);
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] -= r2[k];
}

template <typename S, int CD>
BA_HD void jac_R4(const Cam<S>& c, const Line<S>& L, const Plane<S>& g, const S* meas, S* r, S* Jc, S* Jg, S* Jf) {
  constexpr int NC = CamCols<CD>::LN;
  S d[3], m[3];
  line_dm(L, d, m);
  PlaneLine<S> P;
  plane_line(d, m, g, P, true);
  if (P.degenerate) {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = 0;
#pragma unroll
    for (int k = 0; k < 4 * NC; ++k) Jc[k] = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) Jg[k] = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) Jf[k] = 0;
    return;
  }
  LProj<S> o1, o2;
  lproject(c, d, m, o1);
  lproject(c, P.d2, P.m2, o2);
  S G1[4][3], G2[4][3], r2[4];
  endpoint(o1.l, meas, r, (S(*)[3])G1[0], true);
  endpoint(o1.l, meas + 2, r + 2, (S(*)[3])G1[2], true);
  endpoint(o2.l, meas, r2, (S(*)[3])G2[0], true);
  endpoint(o2.l, meas + 2, r2 + 2, (S(*)[3])G2[2], true);
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] -= r2[k];

  // tangent derivatives of (d, m) in the world frame: dd[k], dm[k], k over xi_L
  S dd[4][3], dm[4][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dd[0][i] = 0; dd[1][i] = -L.w1 * L.u3[i]; dd[2][i] = L.w1 * L.u2[i]; dd[3][i] = -L.w2 * L.u1[i];
    dm[0][i] = L.w2 * L.u3[i]; dm[1][i] = 0; dm[2][i] = -L.w2 * L.u1[i]; dm[3][i] = L.w1 * L.u2[i];
  }
  // projected line tangent derivatives: dd2 = Ddd dd, dm2 = Dmd dd + Dmm dm
  S dmc1[4][3], dmc2[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    S dd2[3], dm2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dd2[i] = P.Ddd[i][0] * dd[k][0] + P.Ddd[i][1] * dd[k][1] + P.Ddd[i][2] * dd[k][2];
      dm2[i] = P.Dmd[i][0] * dd[k][0] + P.Dmd[i][1] * dd[k][1] + P.Dmd[i][2] * dd[k][2] +
               P.Dmm[i][0] * dm[k][0] + P.Dmm[i][1] * dm[k][1] + P.Dmm[i][2] * dm[k][2];
    }
    S a[3], b[3], tx[3];
    rot(c.R, dd[k], a); rot(c.R, dm[k], b); cross3(c.t, a, tx);
#pragma unroll
    for (int i = 0; i < 3; ++i) dmc1[k][i] = b[i] + tx[i];
    rot(c.R, dd2, a); rot(c.R, dm2, b); cross3(c.t, a, tx);
#pragma unroll
    for (int i = 0; i < 3; ++i) dmc2[k][i] = b[i] + tx[i];
  }
  // plane tangent derivatives of the projected line: (B_n dn, dw)
  S dmcg[3][3];
  {
    const S* bb[2] = {g.b1, g.b2};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      S dd2[3], dm2[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        dd2[i] = P.Ddn[i][0] * bb[k][0] + P.Ddn[i][1] * bb[k][1] + P.Ddn[i][2] * bb[k][2];
        dm2[i] = P.Dmn[i][0] * bb[k][0] + P.Dmn[i][1] * bb[k][1] + P.Dmn[i][2] * bb[k][2];
      }
      S a[3], b[3], tx[3];
      rot(c.R, dd2, a); rot(c.R, dm2, b); cross3(c.t, a, tx);
#pragma unroll
      for (int i = 0; i < 3; ++i) dmcg[k][i] = b[i] + tx[i];
    }
    S b[3];
    rot(c.R, P.Dmw, b);
#pragma unroll
    for (int i = 0; i < 3; ++i) dmcg[2][i] = b[i];
  }
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    S ja[NC], jb[NC];
    cam_cols_line<S, NC>(G1[row], o1, c.f, ja);
    cam_cols_line<S, NC>(G2[row], o2, c.f, jb);
#pragma unroll
    for (int k = 0; k < NC; ++k) Jc[row * NC + k] = ja[k] - jb[k];
    S g1[3] = {G1[row][0], G1[row][1], G1[row][2] * c.f};
    S g2[3] = {G2[row][0], G2[row][1], G2[row][2] * c.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) Jf[row * 4 + k] = dot3(g1, dmc1[k]) - dot3(g2, dmc2[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) Jg[row * 3 + k] = -dot3(g2, dmcg[k]);
  }
}

// --------------------------------------------------------------------------
// robust losses: rho(s) and rho'(s)
// --------------------------------------------------------------------------
template <typename S> BA_HD void loss_eval(int kind, S scale, S s, S& rho, S& drho) {
  if (kind == 1) {  // Huber
    S d2 = scale * scale;
    if (s > d2) { S ss = sqrt(s); rho = S(2) * scale * ss - d2; drho = scale / ss; }
    else { rho = s; drho = S(1); }
  } else if (kind == 2) {  // Cauchy
    S c2 = scale * scale;
    rho = c2 * log1p(s / c2);
    drho = S(1) / (S(1) + s / c2);
  } else {
    rho = s; drho = S(1);
  }
}

}  // namespace ba

#include "ba_shape.h"
