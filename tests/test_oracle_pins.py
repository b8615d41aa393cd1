"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it follows.  None of them re-types an oracle
formula: they use finite differences, ground-truth geometry, invariances,
direct geometric constructions, a dense non-Schur solve, a statistical
identity and an independent library optimiser.
"""
import json
import os

import numpy as np
import pytest

from scenegen import (make_scene, small_config, manhattan_config, scene_counts, ASSOC_JUNCTION, OBS_POINT, OBS_LINE,
                      plane_3d_scene, add_shapes)
from oracle import lm, model
from oracle.records import expand

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _zero_steps(prob):
    n = prob.n
    return dict(cam=np.zeros((n["cam"], 9)), pt=np.zeros((n["pt"], 3)), ln=np.zeros((n["ln"], 4)),
                pl=np.zeros((n["pl"], 3)), vp=np.zeros((n["vp"], 2)), sh=np.zeros((n["sh"], 9)))


def _retract_block(st, prob, block, k, h):
    d = _zero_steps(prob)
    d[block][:, k] = h
    return st.retract(d["cam"], d["pt"], d["ln"], d["pl"], d["vp"], dsh=d["sh"])


def _retract_one(st, prob, block, i, k, h):
    """Move only entity i of `block` along tangent coordinate k."""
    d = _zero_steps(prob)
    d[block][i, k] = h
    return st.retract(d["cam"], d["pt"], d["ln"], d["pl"], d["vp"], dsh=d["sh"])


@pytest.fixture(scope="module")
def tiny():
    """Every family of Sec. 3 plus the 3D point-to-plane records of the 3D formulation
    and the surface groups of App. B."""
    s = add_shapes(plane_3d_scene(make_scene(small_config(), seed=11), keep_2d=True), seed=12)
    prob = lm.Problem(s)
    return s, prob


@pytest.fixture(scope="module")
def manhattan():
    """A tiny Manhattan scene with all four inter-group relation families."""
    s = make_scene(manhattan_config(), seed=12)
    prob = lm.Problem(s)
    assert all(prob.record_count(f) > 0 for f in ("R8", "R10", "R11"))
    return s, prob


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("fam", model.FAMILY_ORDER)
def test_jacobian_matches_central_differences(tiny, manhattan, fam):
    """Complex-step Jacobians vs central differences through the exact
    retraction, with non-zero distortion (Sec. 3.1-3.4 residuals; the
    inter-group relations on the Manhattan scene; a VP-VP parallel pair is
    made there by relating two Manhattan VPs that are then set parallel)."""
    s, prob = manhattan if fam in model.RELATION_FAMILIES else tiny
    st = prob.state0()
    if fam == "R9":
        prob = lm.Problem(s)
        prob.recs["R9"] = dict(ga=np.array([0, 1]), gb=np.array([3, 2]))
        st.vp[3] = st.vp[0] + np.array([0.0, 0.05, -0.03])
        st.vp[3] /= np.linalg.norm(st.vp[3])
    st.cam_k1 = st.cam_k1 + 0.08
    st.cam_k2 = st.cam_k2 - 0.05
    rec = prob.recs[fam]
    assert prob.record_count(fam) > 0
    J = model.jacobians(st, rec, fam, prob.cx, prob.cy)
    for b, key, dof in model.FAMILIES[fam][2]:
        scale = max(np.abs(J[key]).max(), 1.0)
        for k in range(dof):
            # Richardson-extrapolated central difference: error O(h^4); a relation's
            # group is moved through the retraction of its own index only
            def cd(h):
                if key in ("ga", "gb"):
                    rp = np.stack([model.residuals(_retract_one(st, prob, b, int(rec[key][i]), k, h),
                                                   {kk: v[i:i + 1] for kk, v in rec.items()}, fam, prob.cx, prob.cy)[0]
                                   for i in range(len(rec[key]))])
                    rm = np.stack([model.residuals(_retract_one(st, prob, b, int(rec[key][i]), k, -h),
                                                   {kk: v[i:i + 1] for kk, v in rec.items()}, fam, prob.cx, prob.cy)[0]
                                   for i in range(len(rec[key]))])
                else:
                    rp = model.residuals(_retract_block(st, prob, b, k, h), rec, fam, prob.cx, prob.cy)
                    rm = model.residuals(_retract_block(st, prob, b, k, -h), rec, fam, prob.cx, prob.cy)
                return (rp - rm) / (2 * h)
            fd = (4 * cd(1e-5) - cd(2e-5)) / 3
            err = np.abs(fd - J[key][:, :, k]).max()
            assert err <= 1e-6 * scale, (fam, b, k, err, scale)


def test_jacobian_near_degenerate_geometry():
    """Lines through the origin (m = 0) and lines almost normal to their
    plane keep finite, FD-consistent Jacobians."""
    s = make_scene(small_config(), seed=2)
    prob = lm.Problem(s)
    st = prob.state0()
    # move line 0 so that it passes through the origin
    d, m = st.plucker()
    U, w = model.line_from_points(np.zeros(3)[None], d[0][None] / np.linalg.norm(d[0]))
    st.line_U[0], st.line_w[0] = U[0], w[0]
    for fam in ("R2", "R5", "R7"):
        rec = prob.recs[fam]
        sel = np.nonzero(rec["ln"] == 0)[0]
        if sel.size == 0:
            continue
        sub = {k: v[sel] for k, v in rec.items()}
        J = model.jacobians(st, sub, fam, prob.cx, prob.cy)
        assert all(np.all(np.isfinite(v)) for v in J.values())
        for k in range(4):
            rp = model.residuals(_retract_block(st, prob, "ln", k, 1e-6), sub, fam, prob.cx, prob.cy)
            rm = model.residuals(_retract_block(st, prob, "ln", k, -1e-6), sub, fam, prob.cx, prob.cy)
            fd = (rp - rm) / 2e-6
            assert np.abs(fd - J["ln"][:, :, k]).max() <= 1e-5 * max(np.abs(J["ln"]).max(), 1.0)


def test_image_line_normal_closed_forms():
    """Degenerate image lines (a reading; the paper leaves the case open):
    with the camera at the world frame, the line through (0, y0, Z) along e_x
    has moment (0, Z, -y0) and image-line normal (0, Z), so the relative
    normal is Z / sqrt(Z^2 + y0^2).  It is zero for a line through the camera
    centre and for a line in the principal plane, and invariant to a scaling
    of the scene."""
    I, t0 = np.eye(3)[None], np.zeros((1, 3))
    for y0, Z in ((0.5, 3.0), (-2.0, 0.1), (4.0, 7.5)):
        P = np.array([[0.0, y0, Z]])
        U, w = model.line_from_points(P, P + np.array([[1.0, 0.0, 0.0]]))
        d, m = model.line_plucker(U, w)
        assert abs(model.image_line_normal(I, t0, d, m)[0] - Z / np.hypot(Z, y0)) < 1e-14
    rng = np.random.default_rng(4)
    for _ in range(5):
        R = model.so3_exp(rng.normal(size=(1, 3)))
        t = rng.normal(size=(1, 3)) * 3
        C = -(R[0].T @ t[0])
        u = rng.normal(size=3)
        U, w = model.line_from_points(C[None], (C + u)[None])
        d, m = model.line_plucker(U, w)
        assert model.image_line_normal(R, t, d, m)[0] < 1e-12
        # principal plane: the camera-frame line through (0, 2, 0) along e_x
        P = C + R[0].T @ np.array([0.0, 2.0, 0.0])
        U, w = model.line_from_points(P[None], (P + R[0].T @ np.array([1.0, 0.0, 0.0]))[None])
        d, m = model.line_plucker(U, w)
        assert model.image_line_normal(R, t, d, m)[0] < 1e-12
        # a generic line, and the same scene scaled by 7
        P, Q = rng.normal(size=(1, 3)), rng.normal(size=(1, 3))
        U, w = model.line_from_points(P, Q)
        d, m = model.line_plucker(U, w)
        U7, w7 = model.line_from_points(7 * P, 7 * Q)
        d7, m7 = model.line_plucker(U7, w7)
        v, v7 = model.image_line_normal(R, t, d, m)[0], model.image_line_normal(R, 7 * t, d7, m7)[0]
        assert v > 1e-6 and abs(v - v7) < 1e-12 * max(v, 1.0)


def _line_near_camera(st, c, u, target):
    """Line along u placed beside camera c's centre so that its relative
    image-line normal in camera c is `target` (fixed-point on the offset)."""
    R, t = st.cam_R[c], st.cam_t[c]
    C = -(R.T @ t)
    off = np.cross(u, [0.3, -0.5, 0.8])
    off /= np.linalg.norm(off)
    delta = 1.0
    for _ in range(60):
        U, w = model.line_from_points((C + delta * off)[None], (C + delta * off + u)[None])
        d, m = model.line_plucker(U, w)
        rel = model.image_line_normal(R[None], t[None], d, m)[0]
        delta *= target / rel
    return U[0], w[0], rel


def test_degenerate_line_record_jacobian_is_exact():
    """A line moved next to the centre of a camera that observes it (relative
    image-line normal 4e-4, then 1e-4).  Every line-projection Jacobian of
    the line (Eqs. 4, 8 and 12), in that camera and in the others, equals
    unscaled central differences of the residual with a step of 1e-3 of the
    distance to the degeneracy (Richardson-extrapolated; the residual itself
    loses about 1/rel of its precision to cancellation there, which bounds
    how small the step may be).  Closer in (1e-6) the derivative in the near
    camera keeps growing: there is no cap."""
    s = make_scene(small_config(), seed=2)
    prob = lm.Problem(s)
    st0 = prob.state0()
    rec = prob.recs["R2"]
    j, c = int(rec["ln"][0]), int(rec["cam"][0])
    d, _ = st0.plucker()
    u = d[j] / np.linalg.norm(d[j])
    norms = {}
    for target in (4e-4, 1e-4, 1e-6):
        st = st0.copy()
        U, w, rel = _line_near_camera(st, c, u, target)
        assert abs(rel / target - 1) < 1e-6
        st.line_U[j], st.line_w[j] = U, w
        for fam in ("R2", "R4", "R7"):
            rf = prob.recs[fam]
            sel = np.nonzero(rf["ln"] == j)[0]
            if sel.size == 0:
                continue
            sub = {k: v[sel] for k, v in rf.items()}
            deg = model.degenerate_line_records(st, sub, fam)
            assert np.array_equal(deg, sub["cam"] == c), fam
            J = model.jacobians(st, sub, fam, prob.cx, prob.cy)
            assert all(np.all(np.isfinite(v)) for v in J.values())
            norms[(target, fam)] = max(np.abs(v[deg]).max(initial=0.0) for v in J.values())
            if target < 1e-4:
                continue
            near = sub["cam"] == c
            for b, dof in (("ln", 4), ("cam", 9)):
                for k in range(dof):
                    # step 1e-3 rel, and at most a 5 % change of the near camera's normal
                    hh0 = 1e-3 * target
                    for _ in range(40):
                        moved = [model.line_record_normal(_retract_block(st, prob, b, k, sg * hh0), sub, fam)[near]
                                 for sg in (1, -1, 2, -2)]
                        if all(np.all(np.abs(mv / target - 1) <= 0.05) for mv in moved):
                            break
                        hh0 *= 0.5

                    def cd(hh):
                        rp = model.residuals(_retract_block(st, prob, b, k, hh), sub, fam, prob.cx, prob.cy)
                        rm = model.residuals(_retract_block(st, prob, b, k, -hh), sub, fam, prob.cx, prob.cy)
                        return (rp - rm) / (2 * hh)
                    fd = (4 * cd(hh0) - cd(2 * hh0)) / 3
                    for row in range(sel.size):
                        Jk = J[b][row, :, k]
                        scale = max(np.abs(J[b][row]).max(), 1.0)
                        assert np.abs(fd[row] - Jk).max() <= 1e-5 * scale, (target, fam, b, k, row)
    assert norms[(4e-4, "R2")] > 0
    for fam in ("R2", "R4", "R7"):
        if norms.get((4e-4, fam), 0.0) > 0:
            assert norms[(1e-4, fam)] > 3 * norms[(4e-4, fam)], fam
            assert norms[(1e-6, fam)] > 30 * norms[(1e-4, fam)], fam
    lin = lm.linearize(prob, st)
    assert np.all(np.isfinite(lin.g))


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("cfg,seed,families", [(small_config(), 5, 7), (2, 2000, 7), (manhattan_config(), 6, 10)])
def test_zero_residual_at_ground_truth(cfg, seed, families):
    """Noise-free scene at ground truth: every residual vanishes (members lie
    exactly on their planes, junction points on their lines, VP lines are
    parallel to their VP, related Manhattan VPs and plane normals are exactly
    perpendicular or parallel) - Eqs. 1, 4, 6, 7, 8, 11, 12 and the
    inter-group relations of Sec. 3.2."""
    s = make_scene(cfg, seed=seed, noise=False)
    prob = lm.Problem(s)
    st = prob.state0()
    present = 0
    for fam in model.FAMILY_ORDER:
        if prob.record_count(fam) == 0:
            continue
        present += 1
        r = model.residuals(st, prob.recs[fam], fam, prob.cx, prob.cy)
        tol = 1e-12 if fam == "R5" or fam in model.RELATION_FAMILIES else 1e-9
        assert np.abs(r).max() <= tol, fam
    assert present == families


def test_relation_residual_closed_forms():
    """The relation residuals of two unit directions at angle theta: the
    orthogonality residual is cos(theta), the parallelism residual has norm
    |sin(theta)| and is normal to both directions; opposite directions are
    parallel (a plane's normal is defined up to sign)."""
    rng = np.random.default_rng(8)
    for theta in (0.0, 0.3, np.pi / 2, 2.0, np.pi):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        p = np.cross(a, rng.normal(size=3))
        p /= np.linalg.norm(p)
        b = np.cos(theta) * a + np.sin(theta) * p
        st = model.State(np.zeros((0, 3, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0),
                         np.zeros((0, 3)), np.zeros((0, 3, 3)), np.zeros((0, 2)), np.zeros((0, 3)), np.zeros(0),
                         np.stack([a, b]))
        rec = dict(ga=np.array([0]), gb=np.array([1]))
        ro = model.residuals(st, rec, "R8", 0.0, 0.0)[0]
        rp = model.residuals(st, rec, "R9", 0.0, 0.0)[0]
        assert abs(ro[0] - np.cos(theta)) < 1e-14
        assert abs(np.linalg.norm(rp) - abs(np.sin(theta))) < 1e-14
        assert abs(rp @ a) < 1e-14 and abs(rp @ b) < 1e-14


# ---------------------------------------------------------------- P3
def _similarity(s, scale, Q, tr):
    """Apply X -> scale Q X + tr to every entity of a scene (its initial values)."""
    from scenegen import quaternion_to_matrix, matrix_to_quaternion
    out = dict(s)
    cams = s["cameras"].copy()
    R = quaternion_to_matrix(cams[:, 0:4])
    t = cams[:, 4:7]
    R2 = R @ Q.T
    t2 = scale * t - np.einsum("nij,j->ni", R2, tr)
    cams[:, 0:4] = matrix_to_quaternion(R2)
    cams[:, 4:7] = t2
    out["cameras"] = cams
    out["points"] = scale * s["points"] @ Q.T + tr
    L = s["lines"].reshape(-1, 2, 3)
    out["lines"] = (scale * L @ Q.T + tr).reshape(-1, 6)
    n = s["planes"][:, 0:3] @ Q.T
    w = scale * s["planes"][:, 3] - n @ tr
    out["planes"] = np.concatenate([n, w[:, None]], 1)
    out["vps"] = s["vps"] @ Q.T
    return out


@pytest.mark.parametrize("cfg", [small_config(), manhattan_config()])
def test_cost_invariant_under_similarity(cfg):
    """Pixel residuals, the angular VP residual and the inter-group relations
    are invariant to a global similarity (the scale-gauge of Sec. 3.3; intro
    and Sec. 3.3 discussion)."""
    s = make_scene(cfg, seed=7)
    prob = lm.Problem(s)
    E0, Ep0 = lm.cost(prob, prob.state0())
    rng = np.random.default_rng(0)
    Q = model.so3_exp(rng.normal(size=3))
    s2 = _similarity(s, 2.7, Q, np.array([0.3, -1.2, 4.0]))
    prob2 = lm.Problem(s2)
    E1, Ep1 = lm.cost(prob2, prob2.state0())
    assert abs(E1 - E0) <= 1e-10 * E0
    assert abs(Ep1 - Ep0) <= 1e-10 * Ep0


# ---------------------------------------------------------------- P4
def test_plane_line_projection_matches_direct_construction():
    """App. B formula for the projected moment equals p' x d' where p' is the
    orthogonal projection of a point of the line onto the plane."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = rng.normal(size=3) * 3
        d = rng.normal(size=3)
        d *= rng.uniform(0.1, 3.0) / np.linalg.norm(d)
        m = np.cross(p, d)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        w = rng.normal() * 2
        d2, m2 = model.plane_project_line(d[None], m[None], n[None], np.array([w]))
        q = p + rng.normal() * d              # any point of the line
        q2 = q - (n @ q + w) * n              # its projection onto the plane
        dd = d - (d @ n) * n
        np.testing.assert_allclose(d2[0], dd, atol=1e-12)
        np.testing.assert_allclose(m2[0], np.cross(q2, dd), rtol=1e-10, atol=1e-10)
        # the projected line lies in the plane: every point has n.x + w = 0
        x0 = np.cross(d2[0], m2[0]) / (d2[0] @ d2[0])
        assert abs(n @ x0 + w) < 1e-9
        assert abs(n @ d2[0]) < 1e-12


def test_plane_line_projection_golden():
    rows = [l.split("|") for l in open(os.path.join(GOLDEN, "plane_line_example.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for lhs, rhs in rows:
        a = np.array(lhs.split(), dtype=float)
        want = np.array(rhs.split(), dtype=float)
        d2, m2 = model.plane_project_line(a[0:3][None], a[3:6][None], a[6:9][None], a[9:10])
        got = np.concatenate([d2[0], m2[0]])
        # Pluecker coordinates are homogeneous: compare up to a common scale
        sc = (got @ want) / (want @ want)
        np.testing.assert_allclose(got, sc * want, atol=1e-12)
        np.testing.assert_allclose(d2[0], want[0:3], atol=1e-12)


def test_plane_point_projection_in_plane():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(50, 3))
    n = rng.normal(size=(50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = rng.normal(size=50)
    Xp = model.plane_project_point(X, n, w)
    assert np.abs(np.sum(n * Xp, 1) + w).max() < 1e-12
    # the displacement is along the normal
    assert np.abs(np.cross(X - Xp, n)).max() < 1e-12


# ---------------------------------------------------------------- P5
def test_vp_residual_is_sine_of_angle():
    """|d x v| = |v - (v.d) d| = sin(theta) (App. B, VP)."""
    s = make_scene(small_config(), seed=4)
    prob = lm.Problem(s)
    st = prob.state0()
    rec = prob.recs["R5"]
    r = model.residuals(st, rec, "R5", prob.cx, prob.cy)
    d, _ = st.plucker()
    u = d[rec["ln"]] / np.linalg.norm(d[rec["ln"]], axis=1, keepdims=True)
    v = st.vp[rec["vp"]]
    theta = np.arccos(np.clip(np.sum(u * v, 1), -1, 1))
    np.testing.assert_allclose(np.linalg.norm(r, axis=1), np.abs(np.sin(theta)), atol=1e-12)
    perp = v - np.sum(u * v, 1)[:, None] * u
    np.testing.assert_allclose(np.linalg.norm(r, axis=1), np.linalg.norm(perp, axis=1), atol=1e-12)


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("lam", [1e-6, 1e-3, 1.0])
@pytest.mark.parametrize("scene", ["tiny", "manhattan"])
def test_schur_step_equals_full_step(tiny, manhattan, scene, lam):
    """Eq. 3 (Schur complement) gives the same step as the full damped normal
    equations of Eq. 2 / Eq. 5, also with the inter-group relations, whose
    rows touch only groups in A."""
    s, prob = tiny if scene == "tiny" else manhattan
    st = prob.state0()
    lin = lm.linearize(prob, st)
    h1, _ = lm.solve_schur(prob, lin, lam)
    h2 = lm.solve_full(prob, lin, lam)
    assert np.abs(h1 - h2).max() <= 1e-9 * np.abs(h2).max()


# ---------------------------------------------------------------- P7
def test_chi_square_at_convergence():
    """Point-only workload (10 cameras, 1000 points, sigma = 1 px, trivial
    loss): at the minimum 2E ~ chi^2 with N_res - N_par + 7 degrees of freedom
    (7 = similarity gauge of the pixel objective)."""
    s = make_scene(1)
    prob = lm.Problem(s)
    res = lm.lm_solve(prob, func_tol=1e-10)
    n_res = 2 * prob.record_count("R1")
    n_par = 9 * prob.n["cam"] + 3 * prob.n["pt"]
    dof = n_res - n_par + 7
    assert abs(2 * res["E"] - dof) <= 5 * np.sqrt(2 * dof)
    assert res["reason"] == "func_tol"


# ---------------------------------------------------------------- P8
def test_group_residual_linearises_as_J_delta():
    """Sec. 3.3 Eq. 9: r_g^(p) ~ J_i delta with delta = X - Proj_G(X); the
    error is second order in the off-plane displacement."""
    s = make_scene(small_config(), seed=6, noise=False)
    prob = lm.Problem(s)
    st = prob.state0()
    rec = prob.recs["R3"]
    errs = []
    for eps in (1e-2, 5e-3):
        st2 = st.copy()
        n = st.pl_n[rec["pl"]]
        moved = np.unique(rec["pt"])
        # push every member along its plane normal by eps
        for j in moved:
            g = rec["pl"][rec["pt"] == j][0]
            st2.pts[j] = st.pts[j] + eps * st.pl_n[g]
        r = model.residuals(st2, rec, "R3", prob.cx, prob.cy)
        delta = st2.pts[rec["pt"]] - model.plane_project_point(st2.pts[rec["pt"]], n, st.pl_w[rec["pl"]])
        # projection Jacobian d pi_p / d X at X (from the point family)
        sub = {"cam": rec["cam"], "pt": rec["pt"], "meas": np.zeros((len(rec["pt"]), 2))}
        Jx = model.jacobians(st2, sub, "R1", prob.cx, prob.cy)["pt"]
        lin = np.einsum("nij,nj->ni", Jx, delta)
        errs.append(np.abs(r - lin).max())
        assert np.abs(lin).max() > 0
    # second order: halving eps divides the error by about 4
    assert errs[1] < errs[0] / 3.0


# ---------------------------------------------------------------- P9
def test_feature_hessian_block_diagonal_and_Hcg_pattern():
    """H_ff is block-diagonal with all families on (Sec. 3.2, 3.3, 3.4) and a
    camera-group block is non-zero iff the camera sees a feature of the group
    (Sec. 3.3, sparsity of H_cg)."""
    s = make_scene(small_config(n_cams=8), seed=9)
    prob = lm.Problem(s)
    lin = lm.linearize(prob, prob.state0())
    _, _, n_off = lm.feature_blocks(prob, lin)
    assert n_off == 0
    sys_ = lm.schur(prob, lin, 1e-3)
    S = sys_["S"]
    cd = prob.camera_dof
    recs = prob.recs
    # cameras that see each feature (any record with a camera touching it)
    from collections import defaultdict
    sees_pt, sees_ln = defaultdict(set), defaultdict(set)
    for fam in ("R1", "R3", "R6"):
        for c, j in zip(recs[fam]["cam"], recs[fam]["pt"]):
            sees_pt[j].add(c)
    for fam in ("R2", "R4", "R7"):
        for c, k in zip(recs[fam]["cam"], recs[fam]["ln"]):
            sees_ln[k].add(c)
    for g in range(prob.n["pl"]):
        cams = set()
        for j in recs["R3"]["pt"][recs["R3"]["pl"] == g]:
            cams |= sees_pt[j]
        for k in recs["R4"]["ln"][recs["R4"]["pl"] == g]:
            cams |= sees_ln[k]
        o = prob.off["pl"] + 3 * g
        for c in range(prob.n["cam"]):
            blk = S[c * cd:(c + 1) * cd, o:o + 3]
            assert (np.abs(blk).max() > 0) == (c in cams), (g, c)


def test_relations_touch_only_group_blocks(manhattan):
    """Sec. 3.2, inter-group relations: they add to H_gg only.  With them on,
    H_ff stays block-diagonal, no relation record has a camera or feature
    column, and the group-group block of H between two distinct groups is
    non-zero exactly when they are related (no feature couples two VPs or
    two planes in this scene)."""
    s, prob = manhattan
    lin = lm.linearize(prob, prob.state0())
    _, _, n_off = lm.feature_blocks(prob, lin)
    assert n_off == 0
    H = (lin.J.T @ lin.J).toarray()
    related = set()
    for fam in model.RELATION_FAMILIES:
        b = model.FAMILIES[fam][2][0][0]
        for a, c in zip(prob.recs[fam]["ga"], prob.recs[fam]["gb"]):
            related.add((b, int(a), int(c)))
            related.add((b, int(c), int(a)))
    # rows of the relation records
    row0 = sum(prob.record_count(f) * model.FAMILIES[f][1] for f in model.FAMILY_ORDER if f not in model.RELATION_FAMILIES)
    Jrel = lin.J[row0:].toarray()
    assert Jrel.shape[0] == sum(prob.record_count(f) * model.FAMILIES[f][1] for f in model.RELATION_FAMILIES) > 0
    assert np.all(Jrel[:, :prob.off["pl"]] == 0) and np.all(Jrel[:, prob.nA:] == 0)
    for b in ("pl", "vp"):
        d, o, n = prob.dof[b], prob.off[b], prob.n[b]
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                blk = H[o + i * d:o + (i + 1) * d, o + j * d:o + (j + 1) * d]
                assert (np.abs(blk).max() > 0) == ((b, i, j) in related), (b, i, j)


# ---------------------------------------------------------------- P10
def test_wireframe_adds_camera_blocks_only_without_shared_features():
    """Supplementary Sec. C: a camera pair block of S that only the cross-
    feature records create belongs to cameras that share no co-observed
    feature, with the junction's point seen in one and its line in the other."""
    s = make_scene(small_config(n_cams=10, n_points=30, n_lines=10), seed=12)
    s_nowf = dict(s)
    obs = dict(s["obs"])
    e = np.zeros(0, dtype=np.int32)
    obs[ASSOC_JUNCTION] = (e, e, None)
    s_nowf["obs"] = obs
    pa, pb = lm.Problem(s), lm.Problem(s_nowf)
    Sa = lm.schur(pa, lm.linearize(pa, pa.state0()), 1e-3)["S"]
    Sb = lm.schur(pb, lm.linearize(pb, pb.state0()), 1e-3)["S"]
    cd, nc = pa.camera_dof, pa.n["cam"]
    pc, pp, _ = s["obs"][OBS_POINT]
    lc, ll, _ = s["obs"][OBS_LINE]
    vis_p = {(int(c), int(j)) for c, j in zip(pc, pp)}
    vis_l = {(int(c), int(k)) for c, k in zip(lc, ll)}
    feats = {}
    for c, j in vis_p:
        feats.setdefault(c, set()).add(("p", j))
    for c, k in vis_l:
        feats.setdefault(c, set()).add(("l", k))
    jp, jl, _ = s["obs"][ASSOC_JUNCTION]
    new = 0
    for i in range(nc):
        for j in range(i + 1, nc):
            a = np.abs(Sa[i * cd:(i + 1) * cd, j * cd:(j + 1) * cd]).max() > 0
            b = np.abs(Sb[i * cd:(i + 1) * cd, j * cd:(j + 1) * cd]).max() > 0
            if a and not b:
                new += 1
                assert not (feats.get(i, set()) & feats.get(j, set()))
                ok = False
                for p, l in zip(jp, jl):
                    pi, pj = (i, p) in vis_p, (j, p) in vis_p
                    li, lj = (i, l) in vis_l, (j, l) in vis_l
                    if (pi and lj and not pj and not li) or (pj and li and not pi and not lj):
                        ok = True
                assert ok
            assert b <= a  # wireframe records never remove a block
    # density D as in the supplementary Table 6 (fraction of non-zero camera pairs)
    def density(S):
        nz = sum(np.abs(S[i * cd:(i + 1) * cd, j * cd:(j + 1) * cd]).max() > 0
                 for i in range(nc) for j in range(nc) if i != j)
        return nz / (nc * (nc - 1))
    assert density(Sa) >= density(Sb)


# ---------------------------------------------------------------- P11
def test_matches_scipy_least_squares():
    """Independent optimiser: scipy's MINPACK LM on the same (trivially
    weighted) objective reaches the oracle's converged cost."""
    from scipy.optimize import least_squares
    from scenegen import LOSS_TRIVIAL
    s = make_scene(small_config(n_cams=5, n_points=20, n_lines=6, grids=1, grid=2, plane_points=6,
                                plane_lines=2, vp_lines=2), seed=21)
    s["loss"] = {k: (LOSS_TRIVIAL, 1.0, w) for k, (_, _, w) in s["loss"].items()}
    prob = lm.Problem(s)
    st0 = prob.state0()
    res = lm.lm_solve(prob, func_tol=1e-14, max_iters=200)

    def f(x):
        st = prob.retract(st0, x)
        out = []
        for fam in model.FAMILY_ORDER:
            if prob.record_count(fam) == 0:
                continue
            r = model.residuals(st, prob.recs[fam], fam, prob.cx, prob.cy)
            out.append(np.sqrt(prob.loss[fam][2]) * r.ravel())
        return np.concatenate(out)

    sol = least_squares(f, np.zeros(prob.N), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=200000)
    E_scipy = 0.5 * float(sol.fun @ sol.fun)
    assert abs(E_scipy - res["E"]) <= 1e-8 * res["E"]


@pytest.mark.parametrize("kind,scipy_loss,scale", [(1, "huber", 2.0), (2, "cauchy", 1.0), (2, "cauchy", 0.2)])
def test_robust_cost_matches_scipy(kind, scipy_loss, scale):
    """Robust loss values (O4: E = 1/2 sum rho(|r|^2) per record) against an
    independent implementation: scipy's least_squares evaluates its own
    Huber / Cauchy cost, 1/2 sum C^2 rho(f^2 / C^2), at the starting point
    when given one scalar residual |r_i| per record and no evaluation budget
    beyond it.  Every family of a holistic scene with 10 % outliers, weight 1,
    at the initial and at a perturbed state, with records on both sides of
    the Huber threshold.  Together with the exact-gradient test below this
    pins rho and its derivative."""
    from scipy.optimize import least_squares
    cfg = small_config()
    cfg["outlier_frac"] = 0.1
    s = make_scene(cfg, seed=23)
    s["loss"] = {k: (kind, scale, 1.0) for k in s["loss"]}
    prob = lm.Problem(s)
    st0 = prob.state0()
    fams = [f for f in model.FAMILY_ORDER if prob.record_count(f)]
    assert len(fams) == 7
    rng = np.random.default_rng(3)
    for st in (st0, prob.retract(st0, rng.normal(size=prob.N) * 1e-3)):
        norms = np.concatenate([np.sqrt(np.sum(model.residuals(st, prob.recs[f], f, prob.cx, prob.cy) ** 2, 1))
                                for f in fams])
        assert np.sum(norms > scale) >= 10 and np.sum(norms < scale) >= 10
        sol = least_squares(lambda x: norms + 0.0 * x[0], np.zeros(1), loss=scipy_loss, f_scale=scale, max_nfev=1)
        assert sol.nfev == 1 and sol.x[0] == 0.0
        E = lm.cost(prob, st)[0]
        assert abs(sol.cost - E) <= 1e-12 * E, (sol.cost, E)


# ---------------------------------------------------------------- expansion
def test_record_expansion_by_brute_force():
    """Visibility rules of Sec. 3.3 and 3.4, re-derived with plain loops."""
    s = make_scene(small_config(n_cams=9), seed=13)
    recs = expand(s)
    obs = s["obs"]
    pc, pp, pm = obs[OBS_POINT]
    lc, ll, lm_ = obs[OBS_LINE]
    P = {(int(c), int(j)) for c, j in zip(pc, pp)}
    L = {(int(c), int(k)) for c, k in zip(lc, ll)}
    from scenegen import ASSOC_PLANE_POINT, ASSOC_PLANE_LINE
    want3 = {(c, int(j), int(g)) for g, j in zip(*obs[ASSOC_PLANE_POINT][:2]) for (c, jj) in P if jj == j}
    got3 = set(zip(recs["R3"]["cam"].tolist(), recs["R3"]["pt"].tolist(), recs["R3"]["pl"].tolist()))
    assert want3 == got3
    want4 = {(c, int(k), int(g)) for g, k in zip(*obs[ASSOC_PLANE_LINE][:2]) for (c, kk) in L if kk == k}
    got4 = set(zip(recs["R4"]["cam"].tolist(), recs["R4"]["ln"].tolist(), recs["R4"]["pl"].tolist()))
    assert want4 == got4
    want6, want7 = set(), set()
    for j, k in zip(*obs[ASSOC_JUNCTION][:2]):
        for c in range(len(s["cameras"])):
            if (c, k) in L and (c, j) not in P:
                want6.add((c, int(j), int(k)))
            if (c, j) in P and (c, k) not in L:
                want7.add((c, int(k), int(j)))
    got6 = set(zip(recs["R6"]["cam"].tolist(), recs["R6"]["pt"].tolist(), recs["R6"]["ln"].tolist()))
    got7 = set(zip(recs["R7"]["cam"].tolist(), recs["R7"]["ln"].tolist(), recs["R7"]["pt"].tolist()))
    assert want6 == got6 and want7 == got7
    assert len(want6) > 0 and len(want7) > 0
    # R6 measurement is that view's observed line; R7 that view's undistorted point
    lmeas = {(int(c), int(k)): m for c, k, m in zip(lc, ll, lm_)}
    for c, j, k, m in zip(recs["R6"]["cam"], recs["R6"]["pt"], recs["R6"]["ln"], recs["R6"]["meas"]):
        np.testing.assert_array_equal(m, lmeas[(int(c), int(k))])
    pmeas = {(int(c), int(j)): m for c, j, m in zip(pc, pp, pm)}
    for c, k, j, m in zip(recs["R7"]["cam"], recs["R7"]["ln"], recs["R7"]["pt"], recs["R7"]["meas"]):
        np.testing.assert_array_equal(m, pmeas[(int(c), int(j))][2:4])


# ---------------------------------------------------------------- losses / golden constants
def test_loss_derivatives():
    s = np.linspace(0.01, 30.0, 101)
    for kind, scale in ((0, 1.0), (1, 2.0), (2, 1.0), (2, 0.2)):
        rho, drho = model.loss_rho(kind, scale, s)
        h = 1e-6
        fd = (model.loss_rho(kind, scale, s + h)[0] - model.loss_rho(kind, scale, s - h)[0]) / (2 * h)
        np.testing.assert_allclose(drho, fd, rtol=1e-6)
        r0, d0 = model.loss_rho(kind, scale, np.array([0.0]))
        assert r0[0] == 0.0 and abs(d0[0] - 1.0) < 1e-12


def test_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    from scenegen import DEFAULT_LOSS, ASSOC_VP_LINE, ASSOC_PLANE_POINT, ASSOC_PLANE_LINE
    assert model.VP_DOF == g["group_dof"]["vp"] and model.PLANE_DOF == g["group_dof"]["plane"]
    assert model.LINE_DOF == g["line_dof"] and model.POINT_DOF == g["point_dof"]
    assert DEFAULT_LOSS[ASSOC_VP_LINE][2] == g["weights"]["vp_line"]
    assert DEFAULT_LOSS[ASSOC_VP_LINE][1] == g["weights"]["vp_cauchy_scale"]
    assert DEFAULT_LOSS[ASSOC_PLANE_POINT][2] == g["weights"]["plane_point"]
    assert DEFAULT_LOSS[ASSOC_PLANE_LINE][2] == g["weights"]["plane_line"]
    assert DEFAULT_LOSS[ASSOC_JUNCTION][2] == g["weights"]["junction"]
    assert DEFAULT_LOSS[OBS_POINT][2] == g["weights"]["point"] == DEFAULT_LOSS[OBS_LINE][2]
    assert model.FAMILIES["R2"][1] == g["rho_dim"] == model.FAMILIES["R4"][1]
    assert model.FAMILIES["R3"][1] == g["group_point_dim"]


def test_gradient_is_exact_with_robust_loss():
    """IRLS reading: g = J~^T r~ equals the gradient of E = 1/2 sum w rho."""
    s = make_scene(small_config(), seed=17)
    prob = lm.Problem(s)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    rng = np.random.default_rng(0)
    for _ in range(5):
        dirn = rng.normal(size=prob.N) * 1e-3
        h = 1e-4
        Ep = lm.cost(prob, prob.retract(st, h * dirn))[0]
        Em = lm.cost(prob, prob.retract(st, -h * dirn))[0]
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - lin.g @ dirn) <= 1e-5 * max(abs(fd), 1e-3)


def test_lm_decreases_cost_holistic():
    s = make_scene(2)
    prob = lm.Problem(s)
    res = lm.lm_solve(prob, max_iters=3)
    E = [h["E"] for h in res["history"]]
    assert all(b <= a for a, b in zip(E, E[1:]))
    assert E[-1] < 0.5 * E[0]
