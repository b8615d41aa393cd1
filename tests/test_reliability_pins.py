"""Pins of the oracle's reliability-aware two-stage refinement (App. A.2,
Reliability-Aware Refinement) against facts fixed by construction.

* active observations: a noise-free scene at its ground truth has every residual
  zero, so every observation is active; planting k gross outliers in one feature's
  observations lowers its count by exactly k and no other feature's;
* uncertainty: a point seen by one camera only has a singular V_f (depth is not
  observed), so its sigma is unbounded; multiplying every loss weight by 4
  multiplies every V_f by 4 and halves every sigma;
* left-out records: the masked problem's cost is the full cost minus exactly the
  dropped records' costs, with the dropped set derived from the record keys;
* fixed-pose stage: from a noise-free scene with one point displaced, LM with the
  A side fixed returns that point to its ground truth and moves nothing else;
* two stages with every feature reliable: stage 1 is the plain LM solve.
"""
import copy

import numpy as np
import pytest

from scenegen import make_scene, small_config, OBS_POINT, ASSOC_PLANE_POINT, ASSOC_JUNCTION
from oracle import lm, reliability as R
from tests.two_stage_scenes import outlier_scene


def _tiny(noise=True):
    return make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101, noise=noise)


def test_active_counts_by_construction():
    s = copy.deepcopy(_tiny(noise=False))
    s["loss"][OBS_POINT] = (1, 2.0, 1.0)
    prob = lm.Problem(s)
    st = prob.state0()
    base = R.feature_stats(prob, st)
    assert np.array_equal(base["pt"]["n_active"], base["pt"]["n_obs"])
    assert np.array_equal(base["ln"]["n_active"], base["ln"]["n_obs"])
    cam, pt, meas = (np.array(a) for a in s["obs"][OBS_POINT])
    meas = meas.reshape(-1, 4).copy()
    j = int(np.argmax(np.bincount(pt)))
    rows = np.nonzero(pt == j)[0][:2]
    meas[rows, 0:2] += 30.0
    s["obs"][OBS_POINT] = (cam, pt, meas)
    prob2 = lm.Problem(s)
    got = R.feature_stats(prob2, prob2.state0())["pt"]["n_active"]
    want = base["pt"]["n_obs"].copy()
    want[j] -= 2
    assert np.array_equal(got, want)


def test_single_view_point_has_unbounded_sigma():
    s = copy.deepcopy(_tiny(noise=False))
    assoc = set(np.asarray(s["obs"][ASSOC_PLANE_POINT][1]).tolist())
    assoc |= set(np.asarray(s["obs"][ASSOC_JUNCTION][0]).tolist())
    cam, pt, meas = (np.array(a) for a in s["obs"][OBS_POINT])
    j = next(p for p in np.unique(pt) if p not in assoc)
    rows = np.nonzero(pt == j)[0]
    keep = np.ones(len(pt), dtype=bool)
    keep[rows[1:]] = False
    s["obs"][OBS_POINT] = (cam[keep], pt[keep], meas.reshape(-1, 4)[keep])
    prob = lm.Problem(s)
    stats = R.feature_stats(prob, prob.state0())["pt"]
    assert stats["n_obs"][j] == 1
    assert stats["sigma"][j] > 1e3, stats["sigma"][j]
    others = np.delete(stats["sigma"], j)
    assert np.all(others < 0.1)


def test_sigma_halves_when_weights_quadruple():
    s = _tiny()
    prob = lm.Problem(s)
    st = prob.state0()
    a = R.feature_stats(prob, st)
    s4 = copy.deepcopy(s)
    s4["loss"] = {k: (v[0], v[1], 4.0 * v[2]) for k, v in s["loss"].items()}
    prob4 = lm.Problem(s4)
    b = R.feature_stats(prob4, st)
    for k in ("pt", "ln"):
        np.testing.assert_allclose(b[k]["sigma"], 0.5 * a[k]["sigma"], rtol=1e-10)


def test_masked_problem_drops_exactly_the_records_of_left_out_parameters():
    s = _tiny()
    prob = lm.Problem(s)
    st = prob.state0()
    rng = np.random.default_rng(4)
    pt_out = rng.random(prob.n["pt"]) < 0.3
    ln_out = rng.random(prob.n["ln"]) < 0.3
    pl_out = np.zeros(prob.n["pl"], bool)
    pl_out[0] = True
    vp_out = np.zeros(prob.n["vp"], bool)
    vp_out[-1] = True
    pm = R.masked_problem(prob, pt_out, ln_out, pl_out, vp_out)
    E_full = E_drop = 0.0
    for fam, rec in prob.recs.items():
        n = prob.record_count(fam)
        if n == 0:
            continue
        c = lm.family_cost(prob, st, fam)
        # parameters of each record: the adjusted feature and the group, not a junction's partner
        drop = np.zeros(n, bool)
        if "pt" in rec and fam != "R7":
            drop |= pt_out[rec["pt"]]
        if "ln" in rec and fam != "R6":
            drop |= ln_out[rec["ln"]]
        if "pl" in rec:
            drop |= pl_out[rec["pl"]]
        if "vp" in rec:
            drop |= vp_out[rec["vp"]]
        if fam in ("R8", "R9"):
            drop |= vp_out[rec["ga"]] | vp_out[rec["gb"]]
        if fam in ("R10", "R11"):
            drop |= pl_out[rec["ga"]] | pl_out[rec["gb"]]
        assert pm.record_count(fam) == n - drop.sum(), fam
        E_full += 0.5 * c.sum()
        E_drop += 0.5 * c[drop].sum()
    assert E_drop > 0
    assert abs(lm.cost(pm, st)[0] - (E_full - E_drop)) <= 1e-12 * E_full


def test_fixed_pose_stage_returns_a_displaced_point():
    s = copy.deepcopy(_tiny(noise=False))
    assoc = set(np.asarray(s["obs"][ASSOC_PLANE_POINT][1]).tolist())
    assoc |= set(np.asarray(s["obs"][ASSOC_JUNCTION][0]).tolist())
    pt = np.asarray(s["obs"][OBS_POINT][1])
    j = next(p for p in np.unique(pt) if p not in assoc)
    gt = np.array(s["points"][j], dtype=float)
    pts = np.array(s["points"], dtype=float)
    pts[j] += np.array([0.05, -0.03, 0.04])
    s["points"] = pts
    prob = lm.Problem(s)
    st0 = prob.state0()
    others = np.ones(prob.n["pt"], bool)
    others[j] = False
    pm = R.masked_problem(prob, pt_out=others, ln_out=np.ones(prob.n["ln"], bool))
    res = lm.lm_solve(pm, st0, func_tol=1e-14, max_iters=50, fixed_a=True)
    st = res["state"]
    assert np.abs(st.pts[j] - gt).max() <= 1e-9
    assert np.array_equal(np.delete(st.pts, j, 0), np.delete(st0.pts, j, 0))
    assert np.array_equal(st.cam_t, st0.cam_t) and np.array_equal(st.cam_R, st0.cam_R)
    assert np.array_equal(st.pl_n, st0.pl_n) and np.array_equal(st.vp, st0.vp)


def test_two_stages_with_every_feature_reliable_is_plain_lm():
    s = _tiny()
    prob = lm.Problem(s)
    out = R.two_stage(prob, min_active=0, max_sigma_point=np.inf, max_sigma_line=np.inf, min_group_support=0,
                      func_tol=1e-10, max_iters=100)
    ref = lm.lm_solve(prob, func_tol=1e-10, max_iters=100)
    assert out["reliable"]["pt"].all() and out["reliable"]["ln"].all()
    assert out["stage1"]["E"] == ref["E"]
    assert out["stage2"]["E"] == 0.0


def test_outlier_scene_flags_the_planted_features():
    """After a full solve of the outlier scene, exactly the features with planted
    outliers fail the active-observation test."""
    s, bad_pts, bad_lns = outlier_scene()
    prob = lm.Problem(s)
    st = lm.lm_solve(prob, func_tol=1e-10, max_iters=100)["state"]
    stats = R.feature_stats(prob, st)
    rel = R.classify(stats, 3, np.inf, np.inf)
    assert np.array_equal(np.nonzero(~rel["pt"])[0], bad_pts)
    assert np.array_equal(np.nonzero(~rel["ln"])[0], bad_lns)
