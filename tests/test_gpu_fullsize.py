"""Parity at the full size of the 1M-point scene (1500 cameras, 1M points,
200k lines, 2000 planes, 12.0M records), in the configuration bench.py times
(mixed precision, learned two-level preconditioner), on outputs the oracle can
compute one by one:

- records: every record of every 2000th point and 400th line (all families),
  against the oracle's records of the same features: residual and each
  Jacobian block within 1e-4 relative, as for the small scenes (and the FP64
  path's records within 1e-9);
- two cameras' rows of the reduced system: b_c, the diagonal block S_cc and
  (S x)_c for a random x, against the oracle's sparse Schur terms of the
  sub-problem that holds exactly the features camera c observes (those rows
  of S and b depend on no other feature), within 1e-3 relative (the bar of
  the small-scene reduced-system test: FP32 sums of thousands of records,
  and S is a difference of two such sums; the FP64 path within 1e-8);
- S Z of the 15 coarse columns in two cameras' and two planes' rows, against
  the oracle's Schur terms of the sub-problem holding every feature those rows
  depend on, entry by entry;
- properties of the whole product: symmetry y.(S x) = x.(S y) and x.(S x) > 0.
"""
import os

import numpy as np
import pytest

from scenegen import make_scene, OBS_POINT, OBS_LINE, ASSOC_PLANE_POINT, ASSOC_PLANE_LINE, ASSOC_VP_LINE, ASSOC_JUNCTION
from oracle import lm
from oracle.records import record_keys

pytestmark = pytest.mark.gpu

LAM = 1e-3
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_04026_amd",
                       "weights", "gnn_precond.bin")


def subset(scene, keep_pt, keep_ln):
    """The scene restricted to the kept points and lines, with all their
    observations and associations; cameras, planes and VPs unchanged.
    Returns (sub-scene, old index of each kept point, of each kept line)."""
    newp = np.cumsum(keep_pt) - 1
    newl = np.cumsum(keep_ln) - 1
    out = dict(scene)
    out["points"] = scene["points"][keep_pt]
    out["lines"] = scene["lines"][keep_ln]
    for k in ("points_gt", "lines_gt"):
        if k in scene:
            out[k] = scene[k][keep_pt if k == "points_gt" else keep_ln]
    obs = {}
    for kind, (a, b, m) in scene["obs"].items():
        a, b = np.asarray(a), np.asarray(b)
        if kind in (OBS_POINT, ASSOC_PLANE_POINT):
            keep = keep_pt[b]
            obs[kind] = (a[keep], newp[b[keep]].astype(np.int32), None if m is None else m[keep])
        elif kind in (OBS_LINE, ASSOC_PLANE_LINE, ASSOC_VP_LINE):
            keep = keep_ln[b]
            obs[kind] = (a[keep], newl[b[keep]].astype(np.int32), None if m is None else m[keep])
        elif kind == ASSOC_JUNCTION:
            keep = keep_pt[a] & keep_ln[b]
            obs[kind] = (newp[a[keep]].astype(np.int32), newl[b[keep]].astype(np.int32), None)
    out["obs"] = obs
    return out, np.flatnonzero(keep_pt), np.flatnonzero(keep_ln)


def sample_features(scene, every_pt, every_ln):
    npt, nln = len(scene["points"]), len(scene["lines"])
    return subset(scene, np.arange(npt) % every_pt == 0, np.arange(nln) % every_ln == 0)


def features_of_camera(scene, c):
    npt, nln = len(scene["points"]), len(scene["lines"])
    kp = np.zeros(npt, dtype=bool)
    kl = np.zeros(nln, dtype=bool)
    a, b, _ = scene["obs"][OBS_POINT]
    kp[np.asarray(b)[np.asarray(a) == c]] = True
    a, b, _ = scene["obs"][OBS_LINE]
    kl[np.asarray(b)[np.asarray(a) == c]] = True
    return subset(scene, kp, kl)


def _code(keys, nfeat, ngrp):
    """One int64 per (camera or -1, feature, group or -1) key."""
    k = keys.astype(np.int64)
    return ((k[:, 0] + 1) * (nfeat + 1) + k[:, 1]) * (ngrp + 2) + (k[:, 2] + 1)


@pytest.fixture(scope="module")
def full():
    print("[fullsize] generating the 1M-point scene", flush=True)
    scene = make_scene(4)
    from paper_2609_04026_amd.binding import BA
    ba = BA.from_scene(scene, precision="mixed", precond="learned")
    if os.path.exists(WEIGHTS):
        ba.set_gnn_weights(open(WEIGHTS, "rb").read())
    ba.linearize(LAM)
    yield scene, ba
    ba.close()


@pytest.fixture(scope="module")
def full_fp64(full):
    """The same scene on the FP64 path (block-Jacobi), linearised at the same lambda."""
    scene, _ = full
    from paper_2609_04026_amd.binding import BA
    ba = BA.from_scene(scene, precision="fp64", precond="jacobi")
    ba.linearize(LAM)
    yield scene, ba
    ba.close()


def test_fullsize_records_match_oracle(full):
    _check_records(*full, tol=1e-4)


def test_fullsize_fp64_records_match_oracle(full_fp64):
    """The FP64 path's records at full size, within 1e-9 relative."""
    _check_records(*full_fp64, tol=1e-9)


def _check_records(scene, ba, tol):
    sub, pts, lns = sample_features(scene, 2000, 400)
    prob = lm.Problem(sub)
    lin = lm.linearize(prob, prob.state0())
    keys_or = record_keys(prob.recs)
    npt, nln = len(scene["points"]), len(scene["lines"])
    ngrp = max(len(scene["planes"]), len(scene["vps"]))
    checked = 0
    for fam in range(1, 8):
        name = f"R{fam}"
        if prob.record_count(name) == 0:
            continue
        ko = keys_or[name][:, 1:].copy()
        # sub-scene feature indices back to the full scene's
        if fam in (1, 3):
            ko[:, 1] = pts[ko[:, 1]]
        elif fam in (2, 4, 5):
            ko[:, 1] = lns[ko[:, 1]]
        elif fam == 6:
            ko[:, 1], ko[:, 2] = pts[ko[:, 1]], lns[ko[:, 2]]
        else:
            ko[:, 1], ko[:, 2] = lns[ko[:, 1]], pts[ko[:, 2]]
        nfeat = max(npt, nln)
        keys, r, J = ba.export_records(fam)
        cg, co = _code(keys, nfeat, max(ngrp, npt)), _code(ko, nfeat, max(ngrp, npt))
        order = np.argsort(cg)
        pos = np.searchsorted(cg[order], co)
        assert np.all(pos < len(cg)) and np.array_equal(cg[order][pos], co), name
        idx = order[pos]
        L = lin.fam[name]
        rt, rg = L["rt"], r[idx]
        floor = 1e-3 if fam == 5 else 1.0
        err = np.linalg.norm(rg - rt, axis=1) / np.maximum(np.linalg.norm(rt, axis=1), floor)
        assert err.max() <= tol, (name, err.max())
        cd = prob.camera_dof
        nf = 4 if fam in (2, 4, 5, 7) else 3
        ng = 3 if fam in (3, 4) else 2 if fam == 5 else 0
        c = 0 if fam == 5 else cd
        cols = {}
        if c:
            cols["cam"] = slice(0, c)
        cols["pt" if nf == 3 else "ln"] = slice(c, c + nf)
        if ng:
            cols["pl" if ng == 3 else "vp"] = slice(c + nf, c + nf + ng)
        for b, sl in cols.items():
            Jo, Jg = L["J"][b], J[idx][:, :, sl]
            nrm = np.linalg.norm(Jo, axis=(1, 2))
            e = np.linalg.norm(Jg - Jo, axis=(1, 2))
            assert np.all(e <= tol * nrm + 1e-9 * (tol / 1e-4)), (name, b, float((e / np.maximum(nrm, 1e-30)).max()))
        checked += len(idx)
    print(f"[fullsize] {checked} records of {len(pts)} points and {len(lns)} lines match within {tol:g}", flush=True)
    assert checked > 5000


@pytest.mark.parametrize("cam", [17, 903])
def test_fullsize_camera_rows_match_oracle(full, cam):
    _check_camera_rows(*full, cam, tol=1e-3)


@pytest.mark.parametrize("cam", [17, 903])
def test_fullsize_fp64_camera_rows_match_oracle(full_fp64, cam):
    """The same rows on the FP64 path, within 1e-8 relative."""
    _check_camera_rows(*full_fp64, cam, tol=1e-8)


def _check_camera_rows(scene, ba, cam, tol):
    sub, pts, lns = features_of_camera(scene, cam)
    prob = lm.Problem(sub)
    lin = lm.linearize(prob, prob.state0())
    t = lm.schur_terms(prob, lin, LAM)
    nA, cd = ba.reduced_dim()
    assert nA == prob.nA and cd == prob.camera_dof
    rows = slice(cd * cam, cd * (cam + 1))
    # b_c and the damped diagonal block S_cc
    b, Sc, _, _ = ba.export_reduced()
    b_or = t["b"][rows]
    assert np.linalg.norm(b[rows] - b_or) <= tol * np.linalg.norm(b_or), (cam, np.linalg.norm(b[rows] - b_or) / np.linalg.norm(b_or))
    U = t["U"][rows][:, rows].toarray() + LAM * np.diag(lin.D[rows])
    S_cc = U - t["WVW"][rows][:, rows].toarray()
    assert np.linalg.norm(Sc[cam] - S_cc) <= tol * np.linalg.norm(S_cc), (cam, np.linalg.norm(Sc[cam] - S_cc) / np.linalg.norm(S_cc))
    # (S x)_c for a random x over all of A, entry by entry against the size of its terms
    x = np.random.default_rng(cam).normal(size=nA)
    y = ba.schur_matvec(x)[rows]
    _check_rows(y[:, None], x[:, None], t, lin, rows, tol, f"camera {cam} S x")
    print(f"[fullsize] camera {cam}: {len(pts)} points, {len(lns)} lines, rows of b, S and S x match within {tol:g}", flush=True)


def _check_rows(got, X, t, lin, rows, tol, what):
    """Rows `rows` of S X (columns of X) from the oracle's sparse Schur terms,
    S = U + lambda D - W V^-1 W^T, entry by entry: each |got - ref| against
    (|U| |X| + lambda D |X| + |W V^-1 W^T| |X|), the size of the terms summed."""
    U, WVW = t["U"][rows], t["WVW"][rows]
    ref = U @ X + (LAM * lin.D[rows])[:, None] * X[rows] - WVW @ X
    mag = abs(U) @ np.abs(X) + (LAM * lin.D[rows])[:, None] * np.abs(X[rows]) + abs(WVW) @ np.abs(X)
    err = np.abs(got - ref) / np.maximum(mag, 1e-300)
    assert err.max() <= tol, (what, float(err.max()))


def test_fullsize_product_is_symmetric_positive(full):
    _, ba = full
    nA, _ = ba.reduced_dim()
    rng = np.random.default_rng(5)
    x, y = rng.normal(size=nA), rng.normal(size=nA)
    Sx, Sy = ba.schur_matvec(x), ba.schur_matvec(y)
    a, c = y @ Sx, x @ Sy
    assert abs(a - c) <= 1e-5 * np.sqrt((x @ Sx) * (y @ Sy)), (a, c)
    assert x @ Sx > 0 and y @ Sy > 0


def features_of_plane(scene, g):
    """The sub-problem of the features associated with plane g: the rows of
    plane g in S and b depend on no other feature."""
    npt, nln = len(scene["points"]), len(scene["lines"])
    kp = np.zeros(npt, dtype=bool)
    kl = np.zeros(nln, dtype=bool)
    a, b, _ = scene["obs"][ASSOC_PLANE_POINT]
    kp[np.asarray(b)[np.asarray(a) == g]] = True
    a, b, _ = scene["obs"][ASSOC_PLANE_LINE]
    kl[np.asarray(b)[np.asarray(a) == g]] = True
    return subset(scene, kp, kl)


@pytest.mark.parametrize("block", [("cam", 17), ("cam", 903), ("plane", 5), ("plane", 1377)])
def test_fullsize_coarse_columns_of_s_z(full, block):
    """S Z of all 15 coarse columns at full size (the gauge columns from the
    features' gauge motion in closed form, as this scene has no VP records;
    the network columns from the record sweeps), in the rows of one camera or
    one plane, against the oracle's exact Schur terms of the sub-problem that
    holds every feature those rows depend on (the camera's observed features,
    or the plane's member features), entry by entry within 1e-3 of the size
    of the summed terms (FP32 records, as for the camera rows of S x)."""
    scene, ba = full
    kind, i = block
    sub, pts, lns = features_of_camera(scene, i) if kind == "cam" else features_of_plane(scene, i)
    prob = lm.Problem(sub)
    lin = lm.linearize(prob, prob.state0())
    t = lm.schur_terms(prob, lin, LAM)
    Z, SZ = ba.export_coarse_space()
    assert Z.shape[1] == 15
    cd = prob.camera_dof
    rows = slice(cd * i, cd * (i + 1)) if kind == "cam" else slice(prob.off["pl"] + 3 * i, prob.off["pl"] + 3 * i + 3)
    _check_rows(SZ[rows], Z, t, lin, rows, 1e-3, f"{kind} {i} S Z")
    print(f"[fullsize] S Z of {Z.shape[1]} coarse columns in the rows of {kind} {i} ({len(pts)} points, "
          f"{len(lns)} lines) matches the oracle", flush=True)
