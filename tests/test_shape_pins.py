"""Pins of the oracle's surface groups (App. B: sphere, cylinder, cone, ellipsoid,
cuboid) against facts fixed by geometry, not by the oracle's formulas:

* surface points (sampled by the scene generator from each shape's own
  construction) project onto themselves, and their group residuals vanish;
* a projection lies on the surface: |P - c| = r, distance r from the cylinder's
  axis, angle alpha to the cone's axis, the ellipsoid's quadric equals 1, the
  chosen cuboid face's plane equation is zero;
* brute force: for the sphere, cylinder, cone and cuboid the projection is the
  nearest point of a dense sampling of the surface; an ellipsoid with equal
  semi-axes projects like the sphere of that radius (its special case);
* Sec. 3.3 Eq. 9: for a point displaced by a small delta off the surface the
  group residual is J_i delta to first order (J_i by finite differences of the
  camera projection alone);
* the complex-step Jacobians of R13 / R14 equal central differences of the
  residual through the retraction (two independent routes to the tangent
  space), and the unused tangent columns of the smaller types are zero;
* a similarity of the whole scene (cameras, points, lines, shapes) leaves the
  R13 / R14 residuals unchanged;
* a line on a cuboid projects into the chosen face's plane, and a line lying in
  a face projects onto itself;
* the 9-column shape blocks: the LM step of the padded system equals the step
  of the compact system with the unused columns deleted, and is zero on them;
* from exact measurements and perturbed shapes, LM returns every shape to its
  ground truth.
"""
import copy

import numpy as np
import pytest

from scenegen import (shape_scene, add_shapes, make_scene, small_config, SHAPE_SPHERE, SHAPE_CYLINDER, SHAPE_CONE,
                      SHAPE_ELLIPSOID, SHAPE_CUBOID)
from scenegen.shapes import _sample_surface, _layout, _orthonormal, _cuboid_segments
from oracle import lm, model, shapes as S


def _gt_shapes(seed=5):
    rng = np.random.default_rng(seed)
    return _layout(rng)


def _project(types, params, idx, X):
    sh = S.Shapes.from_abi(types, params)
    g = S.GatheredShapes(sh, np.asarray(idx))
    return np.real(S.project_point(g, X.astype(np.complex128)))


def test_surface_points_project_onto_themselves():
    types, params = _gt_shapes()
    rng = np.random.default_rng(1)
    for s, (t, p) in enumerate(zip(types, params)):
        X = _sample_surface(rng, t, p, 50)
        P = _project(types, params, np.full(50, s), X)
        assert np.abs(P - X).max() <= 1e-12 * max(1.0, np.abs(X).max()), t


def _near_points(rng, t, p, n, spread=0.3):
    X = _sample_surface(rng, t, p, n)
    return X + rng.normal(scale=spread, size=X.shape)


def test_projection_lies_on_the_surface():
    types, params = _gt_shapes()
    rng = np.random.default_rng(2)
    for s, (t, p) in enumerate(zip(types, params)):
        X = _near_points(rng, t, p, 200)
        P = _project(types, params, np.full(len(X), s), X)
        if t == SHAPE_SPHERE:
            err = np.abs(np.linalg.norm(P - p[0:3], axis=1) - p[3])
        elif t == SHAPE_CYLINDER:
            a = p[0:3] / np.linalg.norm(p[0:3])
            v = P - p[3:6]
            err = np.abs(np.linalg.norm(v - (v @ a)[:, None] * a, axis=1) - p[6])
            # and at X's height along the axis
            err = np.maximum(err, np.abs((P - X) @ a))
        elif t == SHAPE_CONE:
            v = P - p[0:3]
            ang = np.arccos(np.clip((v @ p[3:6]) / np.linalg.norm(v, axis=1), -1, 1))
            err = np.abs(ang - p[6])
        elif t == SHAPE_ELLIPSOID:
            R = p[0:9].reshape(3, 3)
            y = (P - p[9:12]) @ R
            err = np.abs(np.sum((y / p[12:15]) ** 2, axis=1) - 1.0)
        else:
            sh = S.Shapes.from_abi(types[s:s + 1], params[s:s + 1])
            n, e = S.cuboid_faces(sh.R, sh.q)
            face = S.cuboid_face_of_point(np.repeat(sh.R, len(X), 0), np.repeat(sh.q, len(X), 0), X)
            err = np.abs(np.einsum("ij,ij->i", n[0][face], P) + e[0][face])
        assert err.max() <= 1e-12, (t, err.max())


def _dense_surface(t, p):
    """A dense grid on the surface, built from each shape's own description."""
    if t == SHAPE_SPHERE:
        th, ph = np.meshgrid(np.linspace(0, np.pi, 721), np.linspace(0, 2 * np.pi, 1441), indexing="ij")
        u = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1).reshape(-1, 3)
        return p[0:3] + p[3] * u
    if t == SHAPE_CYLINDER:
        a, b1, b2 = _orthonormal(p[0:3])
        h, ph = np.meshgrid(np.linspace(-3, 3, 1201), np.linspace(0, 2 * np.pi, 1441), indexing="ij")
        h, ph = h.reshape(-1, 1), ph.reshape(-1, 1)
        return p[3:6] + h * a + p[6] * (np.cos(ph) * b1 + np.sin(ph) * b2)
    if t == SHAPE_CONE:
        a, b1, b2 = _orthonormal(p[3:6])
        h, ph = np.meshgrid(np.linspace(0, 3, 1201), np.linspace(0, 2 * np.pi, 1441), indexing="ij")
        h, ph = h.reshape(-1, 1), ph.reshape(-1, 1)
        return p[0:3] + h * a + h * np.tan(p[6]) * (np.cos(ph) * b1 + np.sin(ph) * b2)
    # cuboid: the six faces as fine grids in the local frame
    R = p[0:9].reshape(3, 3)
    lo, hi = -p[9:15][0::2], p[9:15][1::2]
    out = []
    for k in range(3):
        o = [j for j in range(3) if j != k]
        u, v = np.meshgrid(np.linspace(lo[o[0]], hi[o[0]], 601), np.linspace(lo[o[1]], hi[o[1]], 601))
        for val in (lo[k], hi[k]):
            L = np.zeros((u.size, 3))
            L[:, o[0]], L[:, o[1]], L[:, k] = u.ravel(), v.ravel(), val
            out.append(L @ R.T)
    return np.concatenate(out)


@pytest.mark.parametrize("t", [SHAPE_SPHERE, SHAPE_CYLINDER, SHAPE_CONE, SHAPE_CUBOID])
def test_projection_is_the_nearest_surface_point(t):
    types, params = _gt_shapes()
    s = int(np.nonzero(types == t)[0][0])
    p = params[s]
    rng = np.random.default_rng(3)
    X = _near_points(rng, t, p, 12, spread=0.15)
    P = _project(types, params, np.full(len(X), s), X)
    if t == SHAPE_CUBOID:
        # the nearest face plane's foot is the nearest surface point when it lies on the
        # face itself (a point beside an edge, outside, is the case the rule leaves open)
        L = P @ p[0:9].reshape(3, 3)
        inside = np.all((L >= -p[9:15][0::2] - 1e-9) & (L <= p[9:15][1::2] + 1e-9), axis=1)
        assert inside.sum() >= 6
        X, P = X[inside], P[inside]
    Y = _dense_surface(t, p)
    for x, q in zip(X, P):
        dmin = np.sqrt(np.min(np.sum((Y - x) ** 2, axis=1)))
        assert abs(np.linalg.norm(x - q) - dmin) <= 5e-3, (t, np.linalg.norm(x - q), dmin)


def test_ellipsoid_with_equal_axes_is_a_sphere():
    rng = np.random.default_rng(4)
    R = S.so3_exp(rng.normal(size=3))
    c = np.array([0.3, -0.2, 0.5])
    types = np.array([SHAPE_ELLIPSOID, SHAPE_SPHERE])
    params = np.zeros((2, 16))
    params[0, 0:9], params[0, 9:12], params[0, 12:15] = R.ravel(), c, 0.7
    params[1, 0:3], params[1, 3] = c, 0.7
    X = c + rng.normal(size=(40, 3))
    Pe = _project(types, params, np.zeros(40, int), X)
    Ps = _project(types, params, np.ones(40, int), X)
    assert np.abs(Pe - Ps).max() <= 1e-13


def _scene():
    return shape_scene(seed=301)


def _project_pixels(st, cam, X, cx, cy):
    return model.project_distorted(st.cam_R[cam], st.cam_t[cam], st.cam_f[cam], st.cam_k1[cam], st.cam_k2[cam],
                                   X, cx, cy)


def test_group_residual_is_projection_jacobian_times_offset():
    s = _scene()
    prob = lm.Problem(s)
    st = model.State.from_scene(s, gt=True)
    rec = prob.recs["R13"]
    rng = np.random.default_rng(6)
    delta = rng.normal(size=(len(rec["pt"]), 3))
    delta /= np.linalg.norm(delta, axis=1, keepdims=True)
    for eps in (1e-3, 5e-4):
        st2 = st.copy()
        # move each record's point off its surface along delta (one record per point here)
        first = np.unique(rec["pt"], return_index=True)[1]
        r0 = rec["pt"][first]
        st2.pts[r0] = st.pts[r0] + eps * delta[first]
        r = model.residuals(st2, rec, "R13", prob.cx, prob.cy)
        P = np.real(S.project_point(S.GatheredShapes(st2.sh, rec["sh"]), st2.pts[rec["pt"]].astype(complex)))
        d = st2.pts[rec["pt"]] - P
        # J_i by central differences of the camera projection at X
        J = np.zeros((len(d), 2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, :, k] = (_project_pixels(st2, rec["cam"], st2.pts[rec["pt"]] + e, prob.cx, prob.cy)
                          - _project_pixels(st2, rec["cam"], st2.pts[rec["pt"]] - e, prob.cx, prob.cy)) / (2 * h)
        lin = np.einsum("nij,nj->ni", J, d)
        err = np.abs(r - lin).max() / np.abs(lin).max()
        assert err <= 20 * eps, (eps, err)


def _fd_jacobian(prob, st, fam, block, k, eps=1e-6):
    """Central difference of a family's residuals through State.retract."""
    rec = prob.recs[fam]
    n = len(rec[block])
    J = np.zeros((n, model.FAMILIES[fam][1]))
    # perturb every parameter of this block type at once: records touch one of each
    for sign in (+1, -1):
        z = {b: np.zeros(prob.n[b] * prob.dof[b]) for b in ("cam", "pt", "ln", "pl", "vp", "sh")}
        dof = prob.dof[block] if block != "cam" else prob.camera_dof
        z[block].reshape(-1, dof)[:, k] = sign * eps
        st2 = st.retract(z["cam"], z["pt"], z["ln"], z["pl"], z["vp"], camera_dof=prob.camera_dof, dsh=z["sh"])
        J += sign * model.residuals(st2, rec, fam, prob.cx, prob.cy)
    return J / (2 * eps)


@pytest.mark.parametrize("fam", ["R13", "R14"])
def test_jacobians_match_differences_through_the_retraction(fam):
    s = _scene()
    prob = lm.Problem(s)
    st = prob.state0()
    Jc = model.jacobians(st, prob.recs[fam], fam, prob.cx, prob.cy, camera_dof=9)
    key = "pt" if fam == "R13" else "ln"
    types = st.sh.type[prob.recs[fam]["sh"]]
    for block, dof in (("sh", 9), (key, 3 if key == "pt" else 4)):
        for k in range(dof):
            Jf = _fd_jacobian(prob, st, fam, block, k)
            scale = np.abs(Jc[block][:, :, k]).max() + 1e-3
            err = np.abs(Jf - Jc[block][:, :, k]).max() / scale
            assert err <= 1e-6, (fam, block, k, err)
    # the unused tangent columns of the smaller types are exactly zero
    for t, used in S.TYPE_DOF.items():
        m = types == t
        if m.any() and used < 9:
            assert np.all(Jc["sh"][m][:, :, used:] == 0), t


def _random_similarity(rng):
    return 1.7, S.so3_exp(rng.normal(size=3)), rng.normal(size=3)


def test_similarity_leaves_group_residuals_unchanged():
    s = _scene()
    prob = lm.Problem(s)
    st = prob.state0()
    sc, Q, tau = _random_similarity(np.random.default_rng(7))
    st2 = st.copy()
    st2.pts = sc * st.pts @ Q.T + tau
    d, m = st.plucker()
    p0 = np.cross(d, m) / np.sum(d * d, axis=1, keepdims=True)
    dq = d @ Q.T
    q0 = sc * p0 @ Q.T + tau
    st2.line_U, st2.line_w = model.line_from_points(q0, q0 + dq)
    st2.cam_R = st.cam_R @ Q.T
    st2.cam_t = sc * st.cam_t - np.einsum("nij,j->ni", st2.cam_R, tau)
    st2.sh = S.similarity(st.sh, sc, Q, tau)
    for fam in ("R13", "R14", "R1", "R2"):
        r1 = model.residuals(st, prob.recs[fam], fam, prob.cx, prob.cy)
        r2 = model.residuals(st2, prob.recs[fam], fam, prob.cx, prob.cy)
        assert np.abs(r1 - r2).max() <= 1e-8 * max(1.0, np.abs(r1).max()), fam


def test_cuboid_line_projection_lies_in_the_face():
    types, params = _gt_shapes()
    s = int(np.nonzero(types == SHAPE_CUBOID)[0][0])
    rng = np.random.default_rng(8)
    A, B = _cuboid_segments(rng, params[s], 20)
    sh = S.Shapes.from_abi(types, params)
    g = S.GatheredShapes(sh, np.full(20, s))
    U, w = model.line_from_points(A, B)
    d, m = model.line_plucker(U, w)
    # exact: a line lying in a face projects onto itself
    n, e = S.cuboid_line_plane(g, d, m)
    d2, m2 = model.plane_project_line(d, m, n, e)
    assert np.abs(d2 - d).max() <= 1e-12 and np.abs(m2 - m).max() <= 1e-12
    # displaced lines: two points of the projected line satisfy the face's plane equation
    A2 = A + rng.normal(scale=0.2, size=A.shape)
    B2 = B + rng.normal(scale=0.2, size=B.shape)
    U, w = model.line_from_points(A2, B2)
    d, m = model.line_plucker(U, w)
    n, e = S.cuboid_line_plane(g, d, m)
    n, e = np.real(n), np.real(e)
    d2, m2 = model.plane_project_line(d, m, n, e)
    p = np.cross(d2, m2) / np.sum(d2 * d2, axis=1, keepdims=True)
    for x in (p, p + d2):
        assert np.abs(np.sum(n * x, axis=1) + e).max() <= 1e-12


def test_padded_shape_columns_are_inert():
    s = _scene()
    prob = lm.Problem(s)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    lam = 1e-3
    h, _ = lm.solve_schur(prob, lin, lam)
    # compact system: delete the unused columns of each shape, solve the damped normal equations
    unused = []
    for i, t in enumerate(st.sh.type):
        o = prob.off["sh"] + 9 * i
        unused += list(range(o + S.TYPE_DOF[t], o + 9))
    keep = np.setdiff1d(np.arange(prob.N), unused)
    J = lin.J.toarray()[:, keep]
    H = J.T @ J + lam * np.diag(lin.D[keep])
    hc = np.linalg.solve(H, -lin.g[keep])
    assert np.all(h[unused] == 0.0) or np.abs(h[unused]).max() <= 1e-300
    assert np.abs(h[keep] - hc).max() <= 1e-8 * np.abs(hc).max()


def test_lm_returns_perturbed_shapes_to_ground_truth():
    s = copy.deepcopy(shape_scene(seed=311, noise=False))
    rng = np.random.default_rng(9)
    from scenegen.shapes import _perturb_shapes
    s["shapes"] = dict(type=s["shapes_gt"]["type"], params=_perturb_shapes(rng, s["shapes_gt"]["type"],
                                                                           s["shapes_gt"]["params"]))
    prob = lm.Problem(s)
    E0 = lm.cost(prob, prob.state0())[0]
    out = lm.lm_solve(prob, func_tol=1e-14, max_iters=80)
    assert out["E"] <= 1e-14 * E0, (out["E"], E0)
    gt = S.Shapes.from_abi(s["shapes_gt"]["type"], s["shapes_gt"]["params"])
    # the solution is unique up to a similarity of the whole scene: map it onto the
    # ground truth with the similarity that best aligns the points (Umeyama)
    A, B = out["state"].pts, np.asarray(s["points_gt"])
    ma, mb = A.mean(0), B.mean(0)
    U_, D, Vt = np.linalg.svd((B - mb).T @ (A - ma) / len(A))
    E_ = np.diag([1.0, 1.0, np.sign(np.linalg.det(U_ @ Vt))])
    Q = U_ @ E_ @ Vt
    sc = np.trace(np.diag(D) @ E_) / np.mean(np.sum((A - ma) ** 2, axis=1))
    tau = mb - sc * Q @ ma
    assert np.abs(sc * A @ Q.T + tau - B).max() <= 1e-6
    got = S.similarity(out["state"].sh, sc, Q, tau)
    # compare geometry: every ground-truth surface point projects onto itself
    rng = np.random.default_rng(10)
    for i, (t, p) in enumerate(zip(s["shapes_gt"]["type"], s["shapes_gt"]["params"])):
        X = _sample_surface(rng, t, p, 20)
        P = np.real(S.project_point(S.GatheredShapes(got, np.full(20, i)), X.astype(complex)))
        assert np.abs(P - X).max() <= 1e-6, t
    assert len(gt) == len(got)


def test_cuboid_centre_is_the_mean_of_its_corners():
    """The centre used for a line's face choice is the cuboid's centroid: the mean
    of its 8 corners, each the intersection of three face planes."""
    types, params = _gt_shapes()
    s = int(np.nonzero(types == SHAPE_CUBOID)[0][0])
    sh = S.Shapes.from_abi(types[s:s + 1], params[s:s + 1])
    n, e = S.cuboid_faces(sh.R, sh.q)
    corners = []
    for i in (0, 1):
        for j in (2, 3):
            for k in (4, 5):
                corners.append(np.linalg.solve(n[0][[i, j, k]], -e[0][[i, j, k]]))
    c = S.cuboid_centre(sh.R, sh.q)[0]
    assert np.abs(c - np.mean(corners, axis=0)).max() <= 1e-12


def test_similarity_gauge_is_a_null_vector_of_the_jacobian():
    """The world rotations, translations and scale, moving every camera, point, line,
    plane and shape (the shapes' rows by numerical differentiation of their similarity
    through the retraction), leave every residual of a scene without VP records
    unchanged to first order: J [G; G_f] = 0 (Sec. 3.1's gauge freedom)."""
    from oracle import gnn
    base = make_scene(small_config(n_cams=9, n_points=40, n_lines=12, n_vps=0, vp_lines=0), seed=41)
    s = add_shapes(base, seed=42)
    prob = lm.Problem(s)
    st = prob.state0()
    rows, worst = S.gauge_rows(st.sh)
    assert worst <= 1e-8, worst
    lin = lm.linearize(prob, st)
    Z = np.concatenate([gnn.gauge_basis(prob, st), gnn.gauge_basis_features(prob, st)])
    JZ = lin.J @ Z
    scale = np.abs(lin.J).max() * np.abs(Z).max()
    assert np.abs(JZ).max() <= 1e-6 * scale, np.abs(JZ).max() / scale
    # and a wrong shape row is seen: zeroing the shapes' rows breaks it
    Z2 = Z.copy()
    o = prob.off["sh"]
    Z2[o:o + 9 * prob.n["sh"]] = 0
    assert np.abs(lin.J @ Z2).max() > 1e-3 * scale


def test_shapes_without_cuboid_lines():
    """The generator adds point-on-shape associations only when asked for no lines on the
    cuboid (an empty line set keeps boolean masks), and the oracle's problem then has R13
    records and no R14 records."""
    from scenegen.scene import ASSOC_SHAPE_POINT, ASSOC_SHAPE_LINE
    base = make_scene(small_config(n_cams=9, n_points=40, n_lines=12, n_vps=0, vp_lines=0), seed=41)
    s = add_shapes(base, seed=3, points_per_shape=50, lines_per_cuboid=0)
    assert len(s["obs"][ASSOC_SHAPE_LINE][0]) == 0 and len(s["obs"][ASSOC_SHAPE_POINT][0]) > 0
    assert len(s["lines"]) == len(base["lines"])
    prob = lm.Problem(s)
    assert prob.record_count("R13") > 0 and prob.record_count("R14") == 0
