// Surface groups beyond planes and vanishing directions (App. B, the table of
// group types and the projections after it): sphere, cylinder, cone, ellipsoid,
// cuboid.  The projection of a point onto each surface with its analytic
// derivatives, the cuboid face choice, and the two residual families built on
// them:
//   R13 point on a shape   pi_p(C, X) - pi_p(C, Proj_G(X))             (Eq. 7 form)
//   R14 line on a cuboid   rho(l(L)) - rho(l(Proj_face(L)))            (Eq. 8 form)
//
// Device storage of one shape: SH_STRIDE doubles, the type at [15]:
//   sphere     c (3), log r
//   cylinder   u1 u2 u3 (the axis' orthonormal Pluecker frame U, columns), w1, w2, log r
//   cone       apex A (3), unit axis d (3), b1 (3), b2 (3) (tangent basis of d), log alpha
//   ellipsoid  R (row-major 9, local to world), c (3), log s (3)
//   cuboid     R (row-major 9), e_0 .. e_5 (face i: n_i . x + e_i = 0,
//              n_i = (-1)^i R e_{i/2}, outward)
// Every shape has SH_DOF = 9 tangent coordinates in the reduced system; a type
// uses the first 4 (sphere: dc, d log r), 5 (cylinder: dtheta with
// U <- U Exp(dtheta), dphi rotating (w1, w2), d log r), 6 (cone: dA, the two
// basis coordinates of dd, d log alpha) or all 9 (ellipsoid: dtheta with
// R <- R Exp(dtheta), dc, d log s; cuboid: dtheta, de).  Unused columns are zero.
#pragma once

namespace ba {

constexpr int SH_STRIDE = 16, SH_DOF = 9;
enum ShapeType { SH_SPHERE = 0, SH_CYLINDER = 1, SH_CONE = 2, SH_ELLIPSOID = 3, SH_CUBOID = 4 };

template <typename S> BA_HD int shape_type(const S* p) { return (int)p[15]; }

// outward normal of cuboid face i
template <typename S> BA_HD void cuboid_normal(const S* p, int i, S* n) {
  const int k = i >> 1;
  const S sg = (i & 1) ? S(-1) : S(1);
  n[0] = sg * p[k]; n[1] = sg * p[3 + k]; n[2] = sg * p[6 + k];
}

// face of smallest |n_i . X + e_i|, lowest index on ties
template <typename S> BA_HD int cuboid_face(const S* p, const S* X) {
  int best = 0;
  S bv = S(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    S n[3];
    cuboid_normal(p, i, n);
    const S a = fabs(dot3(n, X) + p[9 + i]);
    if (i == 0 || a < bv) { bv = a; best = i; }
  }
  return best;
}

// face chosen for the line (d, m): the one nearest to the line's point closest to
// the cuboid centre c = R mc, mc_k = (e_{2k+1} - e_{2k}) / 2
template <typename S> BA_HD int cuboid_face_line(const S* p, const S* d, const S* m) {
  const S iD = S(1) / dot3(d, d);
  S p0[3], c[3], mc[3] = {S(0.5) * (p[10] - p[9]), S(0.5) * (p[12] - p[11]), S(0.5) * (p[14] - p[13])};
  cross3(d, m, p0);
  rot(p, mc, c);
#pragma unroll
  for (int k = 0; k < 3; ++k) p0[k] *= iD;
  S dc[3] = {c[0] - p0[0], c[1] - p0[1], c[2] - p0[2]};
  const S t = dot3(dc, d) * iD;
  S q[3] = {p0[0] + t * d[0], p0[1] + t * d[1], p0[2] + t * d[2]};
  return cuboid_face(p, q);
}

// P = Proj_G(X); with jac: dPdX[i][j] = dP_i / dX_j and dPdg[k][i] = dP_i / dg_k
// (k < SH_DOF, zero beyond the type's own coordinates).  `face` is the cuboid
// face (ignored for the other types).
template <typename S>
BA_HD void shape_project(const S* p, int face, const S* X, S* P, S (*dPdX)[3], S (*dPdg)[3], bool jac) {
  const int type = shape_type(p);
  if (jac) {
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) dPdg[k][0] = dPdg[k][1] = dPdg[k][2] = S(0);
  }
  if (type == SH_SPHERE) {
    const S* c = p;
    const S r = exp(p[3]);
    S u[3] = {X[0] - c[0], X[1] - c[1], X[2] - c[2]};
    const S in = S(1) / sqrt(dot3(u, u));
    S uh[3] = {u[0] * in, u[1] * in, u[2] * in};
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = c[i] + r * uh[i];
    if (!jac) return;
    const S a = r * in;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) dPdX[i][j] = a * ((i == j ? S(1) : S(0)) - uh[i] * uh[j]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 3; ++i) dPdg[k][i] = (i == k ? S(1) : S(0)) - dPdX[i][k];
#pragma unroll
    for (int i = 0; i < 3; ++i) dPdg[3][i] = r * uh[i];
  } else if (type == SH_CYLINDER) {
    const S *u1 = p, *u2 = p + 3, *u3 = p + 6;
    const S w1 = p[9], w2 = p[10], r = exp(p[11]);
    const S kap = w2 / w1;
    S p0[3] = {kap * u3[0], kap * u3[1], kap * u3[2]};
    S v[3] = {X[0] - p0[0], X[1] - p0[1], X[2] - p0[2]};
    const S h = dot3(v, u1);
    S qv[3] = {v[0] - h * u1[0], v[1] - h * u1[1], v[2] - h * u1[2]};
    const S iq = S(1) / sqrt(dot3(qv, qv));
    S qh[3] = {qv[0] * iq, qv[1] * iq, qv[2] * iq};
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = p0[i] + h * u1[i] + r * qh[i];
    if (!jac) return;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dPdX[i][j] = u1[i] * u1[j] + r * iq * ((i == j ? S(1) : S(0)) - u1[i] * u1[j] - qh[i] * qh[j]);
    // derivative along an axis motion (da: direction, dp: foot of the perpendicular)
    auto axis_dir = [&](const S* da, const S* dp, S* dP) {
      const S dh = -dot3(dp, u1) + dot3(v, da);
      S dq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dq[i] = -dp[i] - dh * u1[i] - h * da[i];
      const S qd = dot3(qh, dq);
#pragma unroll
      for (int i = 0; i < 3; ++i) dP[i] = dp[i] + dh * u1[i] + h * da[i] + r * iq * (dq[i] - qd * qh[i]);
    };
    const S zero[3] = {S(0), S(0), S(0)};
    const S m_ku2[3] = {-kap * u2[0], -kap * u2[1], -kap * u2[2]};
    const S ku1[3] = {kap * u1[0], kap * u1[1], kap * u1[2]};
    const S mu3[3] = {-u3[0], -u3[1], -u3[2]};
    const S dk = (w1 * w1 + w2 * w2) / (w1 * w1);
    const S dku3[3] = {dk * u3[0], dk * u3[1], dk * u3[2]};
    axis_dir(zero, m_ku2, dPdg[0]);   // dtheta_1: u3 -> -u2
    axis_dir(mu3, ku1, dPdg[1]);      // dtheta_2: u1 -> -u3, u3 -> u1
    axis_dir(u2, zero, dPdg[2]);      // dtheta_3: u1 -> u2
    axis_dir(zero, dku3, dPdg[3]);    // dphi: w2 / w1 -> + (w1^2 + w2^2) / w1^2
#pragma unroll
    for (int i = 0; i < 3; ++i) dPdg[4][i] = r * qh[i];
  } else if (type == SH_CONE) {
    const S *A = p, *ax = p + 3, *b1 = p + 6, *b2 = p + 9;
    const S al = exp(p[12]), ca = cos(al), sa = sin(al);
    S v[3] = {X[0] - A[0], X[1] - A[1], X[2] - A[2]};
    const S h = dot3(v, ax);
    S qv[3] = {v[0] - h * ax[0], v[1] - h * ax[1], v[2] - h * ax[2]};
    const S iq = S(1) / sqrt(dot3(qv, qv));
    S e[3] = {qv[0] * iq, qv[1] * iq, qv[2] * iq};
    S g[3] = {ca * ax[0] + sa * e[0], ca * ax[1] + sa * e[1], ca * ax[2] + sa * e[2]};
    const S t = dot3(v, g);
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = A[i] + t * g[i];
    if (!jac) return;
    // derivative of P - A for a change (dv, dd, dal) of v = X - A, the axis and alpha
    auto dir = [&](const S* dv, const S* dd, S dal, S* dP) {
      const S dh = dot3(dv, ax) + dot3(v, dd);
      S dq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dq[i] = dv[i] - dh * ax[i] - h * dd[i];
      const S ed = dot3(e, dq);
      S dg[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dg[i] = -sa * dal * ax[i] + ca * dd[i] + ca * dal * e[i] + sa * iq * (dq[i] - ed * e[i]);
      const S dt = dot3(dv, g) + dot3(v, dg);
#pragma unroll
      for (int i = 0; i < 3; ++i) dP[i] = dt * g[i] + t * dg[i];
    };
    const S zero[3] = {S(0), S(0), S(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const S ej[3] = {S(j == 0), S(j == 1), S(j == 2)};
      S col[3];
      dir(ej, zero, S(0), col);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        dPdX[i][j] = col[i];
        dPdg[j][i] = ej[i] - col[i];  // dA = e_j moves v by -e_j
      }
    }
    dir(zero, b1, S(0), dPdg[3]);
    dir(zero, b2, S(0), dPdg[4]);
    dir(zero, zero, al, dPdg[5]);
  } else if (type == SH_ELLIPSOID) {
    const S *R = p, *c = p + 9;
    const S s[3] = {S(exp(p[12])), S(exp(p[13])), S(exp(p[14]))};
    S u[3] = {X[0] - c[0], X[1] - c[1], X[2] - c[2]};
    S y[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = R[i] * u[0] + R[3 + i] * u[1] + R[6 + i] * u[2];  // R^T u
    S z[3] = {y[0] / s[0], y[1] / s[1], y[2] / s[2]};
    const S iz = S(1) / sqrt(dot3(z, z));
    S zh[3] = {z[0] * iz, z[1] * iz, z[2] * iz};
    S w[3] = {s[0] * zh[0], s[1] * zh[1], s[2] * zh[2]};
    S Rw[3];
    rot(R, w, Rw);
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = c[i] + Rw[i];
    if (!jac) return;
    // derivative of P - c for a change dy of y (in the local frame), a local
    // rotation dth and a change dsig of log s
    auto dir = [&](const S* dy, const S* dth, const S* dsig, S* dP) {
      S dz[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) dz[i] = dy[i] / s[i] - z[i] * dsig[i];
      const S zd = dot3(zh, dz);
      S loc[3], tx[3];
      cross3(dth, w, tx);
#pragma unroll
      for (int i = 0; i < 3; ++i) loc[i] = tx[i] + s[i] * dsig[i] * zh[i] + s[i] * iz * (dz[i] - zd * zh[i]);
      rot(R, loc, dP);
    };
    const S zero[3] = {S(0), S(0), S(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const S rj[3] = {R[3 * j], R[3 * j + 1], R[3 * j + 2]};  // R^T e_j
      S col[3];
      dir(rj, zero, zero, col);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        dPdX[i][j] = col[i];
        dPdg[3 + j][i] = (i == j ? S(1) : S(0)) - col[i];
      }
      const S ej[3] = {S(j == 0), S(j == 1), S(j == 2)};
      S dy[3];
      cross3(y, ej, dy);  // -dth x y with dth = e_j
      dir(dy, ej, zero, dPdg[j]);
      dir(zero, zero, ej, dPdg[6 + j]);
    }
  } else {  // cuboid
    S n[3];
    cuboid_normal(p, face, n);
    const S sd = dot3(n, X) + p[9 + face];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = X[i] - sd * n[i];
    if (!jac) return;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) dPdX[i][j] = (i == j ? S(1) : S(0)) - n[i] * n[j];
    const int k = face >> 1;
    const S sg = (face & 1) ? S(-1) : S(1);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S ej[3] = {S(j == 0), S(j == 1), S(j == 2)}, ek[3] = {S(k == 0), S(k == 1), S(k == 2)}, ex[3], dn[3];
      cross3(ej, ek, ex);
      rot(p, ex, dn);
#pragma unroll
      for (int i = 0; i < 3; ++i) dn[i] *= sg;
      const S dsd = dot3(dn, X);
#pragma unroll
      for (int i = 0; i < 3; ++i) dPdg[j][i] = -dsd * n[i] - sd * dn[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) dPdg[3 + face][i] = -n[i];
  }
}

// ---- R13 ------------------------------------------------------------------
template <typename S> BA_HD void res_R13(const Cam<S>& c, const S* X, const S* sh, int face, S* r) {
  S P[3];
  shape_project<S>(sh, face, X, P, nullptr, nullptr, false);
  PProj<S> a, b;
  pproject<S, true>(c, X, a, false);
  pproject<S, true>(c, P, b, false);
  r[0] = a.x - b.x;
  r[1] = a.y - b.y;
}

// Jg: 2 x SH_DOF
template <typename S, int CD>
BA_HD void jac_R13(const Cam<S>& c, const S* X, const S* sh, int face, S* r, S* Jc, S* Jg, S* Jf) {
  constexpr int NC = CamCols<CD>::PT;
  S P[3], dX[3][3], dg[SH_DOF][3];
  shape_project<S>(sh, face, X, P, dX, dg, true);
  PProj<S> a, b;
  pproject<S, true>(c, X, a, true);
  pproject<S, true>(c, P, b, true);
  r[0] = a.x - b.x;
  r[1] = a.y - b.y;
  S ja[NC], jb[NC];
  S ra4 = a.r2 * a.r2, rb4 = b.r2 * b.r2;
#pragma unroll
  for (int row = 0; row < 2; ++row) {
    S ua = row == 0 ? a.u : a.v, ub = row == 0 ? b.u : b.v;
    cam_cols_point<S, NC>(a.B[row], a.p, a.s * ua, c.f * a.r2 * ua, c.f * ra4 * ua, ja);
    cam_cols_point<S, NC>(b.B[row], b.p, b.s * ub, c.f * b.r2 * ub, c.f * rb4 * ub, jb);
#pragma unroll
    for (int k = 0; k < NC; ++k) Jc[row * NC + k] = ja[k] - jb[k];
    S fa[3], fb[3];
    feat_cols_point(a.B[row], c.R, fa);
    feat_cols_point(b.B[row], c.R, fb);  // d pi(P) / d P
#pragma unroll
    for (int k = 0; k < 3; ++k) Jf[row * 3 + k] = fa[k] - (fb[0] * dX[0][k] + fb[1] * dX[1][k] + fb[2] * dX[2][k]);
#pragma unroll
    for (int k = 0; k < SH_DOF; ++k) Jg[row * SH_DOF + k] = -dot3(fb, dg[k]);
  }
}

// ---- R14 ------------------------------------------------------------------
template <typename S> BA_HD Plane<S> cuboid_face_plane(const S* sh, int face) {
  Plane<S> g;
  cuboid_normal(sh, face, g.n);
  g.w = sh[9 + face];
#pragma unroll
  for (int k = 0; k < 3; ++k) g.b1[k] = g.b2[k] = S(0);
  return g;
}

template <typename S> BA_HD void res_R14(const Cam<S>& c, const Line<S>& L, const S* sh, int face, const S* meas, S* r) {
  res_R4<S>(c, L, cuboid_face_plane<S>(sh, face), meas, r);
}

// Jg: 4 x SH_DOF; the face plane moves with the rotation (dn = (-1)^i R (e_j x e_k))
// and with its own offset
template <typename S, int CD>
BA_HD void jac_R14(const Cam<S>& c, const Line<S>& L, const S* sh, int face, const S* meas, S* r, S* Jc, S* Jg,
                   S* Jf) {
  constexpr int NC = CamCols<CD>::LN;
  const Plane<S> g = cuboid_face_plane<S>(sh, face);
  S d[3], m[3];
  line_dm(L, d, m);
  PlaneLine<S> P;
  plane_line(d, m, g, P, true);
#pragma unroll
  for (int k = 0; k < 4 * SH_DOF; ++k) Jg[k] = S(0);
  if (P.degenerate) {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = 0;
#pragma unroll
    for (int k = 0; k < 4 * NC; ++k) Jc[k] = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) Jf[k] = 0;
    return;
  }
  S jg4[12];
  jac_R4<S, CD>(c, L, g, meas, r, Jc, jg4, Jf);  // camera and line columns, the residual
  LProj<S> o2;
  lproject(c, P.d2, P.m2, o2);
  S G2[4][3], r2[4];
  endpoint(o2.l, meas, r2, (S(*)[3])G2[0], true);
  endpoint(o2.l, meas + 2, r2 + 2, (S(*)[3])G2[2], true);
  // group directions: rotation (3) and the face's own offset
  const int k = face >> 1;
  const S sg = (face & 1) ? S(-1) : S(1);
  S dmcg[4][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    S ej[3] = {S(j == 0), S(j == 1), S(j == 2)}, ek[3] = {S(k == 0), S(k == 1), S(k == 2)}, ex[3], dn[3];
    cross3(ej, ek, ex);
    rot(sh, ex, dn);
#pragma unroll
    for (int i = 0; i < 3; ++i) dn[i] *= sg;
    S dd2[3], dm2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dd2[i] = P.Ddn[i][0] * dn[0] + P.Ddn[i][1] * dn[1] + P.Ddn[i][2] * dn[2];
      dm2[i] = P.Dmn[i][0] * dn[0] + P.Dmn[i][1] * dn[1] + P.Dmn[i][2] * dn[2];
    }
    S a[3], b[3], tx[3];
    rot(c.R, dd2, a); rot(c.R, dm2, b); cross3(c.t, a, tx);
#pragma unroll
    for (int i = 0; i < 3; ++i) dmcg[j][i] = b[i] + tx[i];
  }
  rot(c.R, P.Dmw, dmcg[3]);
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    S g2[3] = {G2[row][0], G2[row][1], G2[row][2] * c.f};
#pragma unroll
    for (int j = 0; j < 3; ++j) Jg[row * SH_DOF + j] = -dot3(g2, dmcg[j]);
    Jg[row * SH_DOF + 3 + face] = -dot3(g2, dmcg[3]);
  }
}

}  // namespace ba
