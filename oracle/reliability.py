"""Reliability-aware two-stage refinement (App. A.2, Reliability-Aware Refinement).

Test infrastructure: the FP64 reference the GPU path is checked against.

The paper classifies feature tracks as reliable or unreliable from their number of
active observations and their estimated uncertainty, then refines in two stages: a
full optimisation over cameras, reliable features, groups and wireframe records,
followed by a refinement of the unreliable features with the poses fixed.  Groups
with too little active support are left out of the first stage.  It gives no
thresholds and no formula for the uncertainty; the readings used here:

* active observation: an observation record (R1 for a point, R2 for a line) whose
  residual lies in the quadratic part of its robust loss, |r|^2 <= scale^2 (every
  record under the trivial loss);
* uncertainty: sigma_f = lambda_min(V_f)^(-1/2), V_f = sum over the feature's records
  of J~^T J~ (the undamped feature block of H at the current parameters, poses and
  groups fixed), in the feature's tangent coordinates; for a point divided by its
  mean distance to the cameras that observe it (an angle), for a line taken as is
  (the tangent of the orthonormal representation is a rotation and an angle);
* reliable: at least min_active active observations and sigma_f at most
  max_sigma_point (points, relative) or max_sigma_line (lines, tangent units);
* group support: the number of distinct reliable features associated with the group
  (planes: points and lines; VPs: lines); groups below min_group_support, and the
  relations that involve them, are left out of stage 1;
* leaving a feature or group out drops every record whose parameters include it
  from the cost and from the system (a junction record's partner feature only
  supplies its measurement); its parameters do not move;
* stage 1: LM over the problem without the unreliable features and the unsupported
  groups; stage 2: LM with cameras, planes and VPs fixed, over the unreliable
  features alone (records of the reliable features dropped), starting from stage 1's
  parameters.  Classification is done once, at the parameters the refinement starts
  from.
"""
from __future__ import annotations

import copy

import numpy as np

from . import lm, model

POINT_FAMILIES = ("R1", "R3", "R6")
LINE_FAMILIES = ("R2", "R4", "R5", "R7")


def masked_problem(prob, pt_out=None, ln_out=None, pl_out=None, vp_out=None):
    """The same problem with every record that involves a left-out point, line,
    plane or VP removed (boolean arrays over the features / groups, None: none)."""
    out = copy.copy(prob)
    out.recs = {}
    masks = dict(pt=pt_out, ln=ln_out, pl=pl_out, vp=vp_out)
    # a junction record's partner feature only supplies the measurement
    partner = {"R6": "ln", "R7": "pt"}
    for fam, rec in prob.recs.items():
        n = len(next(iter(rec.values())))
        drop = np.zeros(n, dtype=bool)
        for key, m in masks.items():
            if m is not None and key in rec and partner.get(fam) != key:
                drop |= np.asarray(m, dtype=bool)[rec[key]]
        if fam in ("R8", "R9"):
            for side in ("ga", "gb"):
                if vp_out is not None:
                    drop |= np.asarray(vp_out, dtype=bool)[rec[side]]
        if fam in ("R10", "R11"):
            for side in ("ga", "gb"):
                if pl_out is not None:
                    drop |= np.asarray(pl_out, dtype=bool)[rec[side]]
        out.recs[fam] = {k: v[~drop] for k, v in rec.items()}
    return out


def _camera_centres(state):
    return -np.einsum("nji,nj->ni", state.cam_R, state.cam_t)


def feature_stats(prob, state):
    """Per point and per line: active observations, observations, and the
    uncertainty sigma (points: relative to the mean viewing distance)."""
    lin = lm.linearize(prob, state)
    Vp, Vl, _ = lm.feature_blocks(prob, lin)
    out = {}
    for kind, fam, V, key in (("pt", "R1", Vp, "pt"), ("ln", "R2", Vl, "ln")):
        n = prob.n[kind]
        rec = prob.recs[fam]
        r = model.residuals(state, rec, fam, prob.cx, prob.cy)
        s = np.sum(r * r, axis=1)
        lkind, scale, _ = prob.loss[fam]
        active = np.ones(len(s), dtype=bool) if lkind == 0 else s <= scale * scale
        n_active = np.bincount(rec[key], weights=active.astype(float), minlength=n).astype(np.int64)
        n_obs = np.bincount(rec[key], minlength=n).astype(np.int64)
        lam_min = np.linalg.eigvalsh(V)[:, 0] if n else np.zeros(0)
        with np.errstate(divide="ignore", invalid="ignore"):
            sigma = np.where(lam_min > 0, 1.0 / np.sqrt(np.where(lam_min > 0, lam_min, 1.0)), np.inf)
        if kind == "pt":
            C = _camera_centres(state)
            dist = np.linalg.norm(state.pts[rec["pt"]] - C[rec["cam"]], axis=1)
            dsum = np.bincount(rec["pt"], weights=dist, minlength=n)
            with np.errstate(divide="ignore", invalid="ignore"):
                dmean = np.where(n_obs > 0, dsum / np.maximum(n_obs, 1), np.nan)
                sigma = np.where(n_obs > 0, sigma / dmean, np.inf)
        out[kind] = dict(n_active=n_active, n_obs=n_obs, sigma=sigma)
    return out


def classify(stats, min_active=3, max_sigma_point=0.01, max_sigma_line=0.1):
    """Reliable flags per point and per line."""
    smax = dict(pt=max_sigma_point, ln=max_sigma_line)
    return {k: (v["n_active"] >= min_active) & (v["sigma"] <= smax[k]) for k, v in stats.items()}


def group_support(prob, reliable):
    """Distinct reliable features associated with each plane and each VP."""
    sc = prob.scene["obs"]
    from scenegen import ASSOC_PLANE_POINT, ASSOC_PLANE_LINE, ASSOC_VP_LINE
    out = {}
    pl = np.zeros(prob.n["pl"], dtype=np.int64)
    for kind, feat in ((ASSOC_PLANE_POINT, "pt"), (ASSOC_PLANE_LINE, "ln")):
        g, f, _ = sc[kind]
        g, f = np.asarray(g, np.int64), np.asarray(f, np.int64)
        pairs = np.unique(np.stack([g, f], 1), axis=0) if len(g) else np.zeros((0, 2), np.int64)
        keep = reliable[feat][pairs[:, 1]] if len(pairs) else np.zeros(0, bool)
        pl += np.bincount(pairs[keep, 0], minlength=prob.n["pl"]) if len(pairs) else 0
    out["pl"] = pl
    v, f, _ = sc[ASSOC_VP_LINE]
    v, f = np.asarray(v, np.int64), np.asarray(f, np.int64)
    pairs = np.unique(np.stack([v, f], 1), axis=0) if len(v) else np.zeros((0, 2), np.int64)
    keep = reliable["ln"][pairs[:, 1]] if len(pairs) else np.zeros(0, bool)
    out["vp"] = np.bincount(pairs[keep, 0], minlength=prob.n["vp"]) if len(pairs) else np.zeros(prob.n["vp"], np.int64)
    return out


def two_stage(prob, state=None, min_active=3, max_sigma_point=0.01, max_sigma_line=0.1, min_group_support=3,
              **lm_kw):
    """Stage 1 over cameras, reliable features and supported groups; stage 2 over
    the unreliable features with cameras and groups fixed.  Returns the statistics,
    the flags, both LM results and the final state."""
    state = prob.state0() if state is None else state
    stats = feature_stats(prob, state)
    rel = classify(stats, min_active, max_sigma_point, max_sigma_line)
    sup = group_support(prob, rel)
    grp_out = {k: v < min_group_support for k, v in sup.items()}
    p1 = masked_problem(prob, pt_out=~rel["pt"], ln_out=~rel["ln"], pl_out=grp_out["pl"], vp_out=grp_out["vp"])
    r1 = lm.lm_solve(p1, state, **lm_kw)
    p2 = masked_problem(prob, pt_out=rel["pt"], ln_out=rel["ln"])
    r2 = lm.lm_solve(p2, r1["state"], fixed_a=True, **lm_kw)
    return dict(stats=stats, reliable=rel, support=sup, group_out=grp_out, stage1=r1, stage2=r2,
                state=r2["state"])
