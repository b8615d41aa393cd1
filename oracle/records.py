"""Expansion of observations and associations into residual records.

The visibility rules are the paper's:

* R1 one record per point observation (i, j) in O_p (Sec. 3.1 Eq. 1);
* R2 one record per line observation (i, k) in O_l (Sec. 3.2 Eq. 4);
* R3 one record per plane-point association (g, j) and per view i that
  observes the point (Sec. 3.3 Eq. 7, residual in camera C_i);
* R4 one record per plane-line association (g, k) and per view i that
  observes the line, with that view's observed endpoints (Sec. 3.3 Eq. 8);
* R5 one record per VP-line association (v, k) (Sec. 3.3 Eq. 6);
* R6 one record per junction (j, k) and per view i in which the line is
  observed and the point is not, measured against that view's observed
  line (Sec. 3.4 Eq. 11);
* R7 one record per junction (j, k) and per view i in which the point is
  observed and the line is not, measured at that view's observed point
  (undistorted pixels) (Sec. 3.4 Eq. 12);
* views that observe both features of a junction get no cross-feature
  record (Sec. 3.4, after Eq. 12);
* R8-R11 one record per inter-group relation: VP-VP orthogonal, VP-VP
  parallel, plane-plane orthogonal, plane-plane parallel (Sec. 3.2, the
  inter-group relations between VP pairs and plane-normal pairs);
* R12 one record per 3D point-to-plane association (g, j): the metric
  distance of the 3D formulation the paper compares against;
* R13 one record per shape-point association (s, j) and per view i that
  observes the point, like R3 with the shape's projection (Sec. 3.3 after
  Eq. 8, App. B);
* R14 one record per shape-line association (s, k) (a cuboid) and per view i
  that observes the line, with that view's observed endpoints, like R4.

Each family is a dict of equally long arrays; ``key`` gives a record's
identity for matching against another implementation:
(family id, camera or -1, feature, group or partner or -1).
"""
from __future__ import annotations

import numpy as np

from scenegen import (OBS_POINT, OBS_LINE, ASSOC_PLANE_POINT, ASSOC_PLANE_LINE, ASSOC_VP_LINE,
                      ASSOC_JUNCTION, REL_VP_ORTHO, REL_VP_PARALLEL, REL_PLANE_ORTHO, REL_PLANE_PARALLEL,
                      ASSOC_PLANE_POINT_3D, ASSOC_SHAPE_POINT, ASSOC_SHAPE_LINE)

FAMILY_KIND = {"R1": OBS_POINT, "R2": OBS_LINE, "R3": ASSOC_PLANE_POINT, "R4": ASSOC_PLANE_LINE,
               "R5": ASSOC_VP_LINE, "R6": ASSOC_JUNCTION, "R7": ASSOC_JUNCTION,
               "R8": REL_VP_ORTHO, "R9": REL_VP_PARALLEL, "R10": REL_PLANE_ORTHO, "R11": REL_PLANE_PARALLEL,
               "R12": ASSOC_PLANE_POINT_3D, "R13": ASSOC_SHAPE_POINT, "R14": ASSOC_SHAPE_LINE}
FAMILY_ID = {"R1": 1, "R2": 2, "R3": 3, "R4": 4, "R5": 5, "R6": 6, "R7": 7, "R8": 8, "R9": 9, "R10": 10, "R11": 11,
             "R12": 12, "R13": 13, "R14": 14}


def _views_of(feat_of_obs, n_feat):
    """CSR (offsets, order) of observations grouped by feature, cameras ascending."""
    order = np.argsort(feat_of_obs, kind="stable")
    counts = np.bincount(feat_of_obs, minlength=n_feat)
    off = np.zeros(n_feat + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off, order


def _expand(assoc_feat, off, order):
    """For each association, the observation rows of its feature."""
    cnt = off[assoc_feat + 1] - off[assoc_feat]
    a_idx = np.repeat(np.arange(len(assoc_feat)), cnt)
    start = np.repeat(off[assoc_feat], cnt)
    pos = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    return a_idx, order[start + pos]


def expand(scene) -> dict:
    obs = scene["obs"]
    npt, nln = len(scene["points"]), len(scene["lines"])
    pc, pp, pm = (np.asarray(a) for a in obs[OBS_POINT])
    lc, ll, lm = (np.asarray(a) for a in obs[OBS_LINE])
    pc, pp, lc, ll = (a.astype(np.int64) for a in (pc, pp, lc, ll))
    pm = pm.reshape(-1, 4)
    lm = lm.reshape(-1, 4)
    recs = {}
    recs["R1"] = dict(cam=pc, pt=pp, meas=pm[:, 0:2])
    recs["R2"] = dict(cam=lc, ln=ll, meas=lm)

    poff, pord = _views_of(pp, npt)
    loff, lord = _views_of(ll, nln)

    g, j, _ = obs[ASSOC_PLANE_POINT]
    g, j = np.asarray(g, np.int64), np.asarray(j, np.int64)
    a, o = _expand(j, poff, pord)
    recs["R3"] = dict(cam=pc[o], pt=j[a], pl=g[a])

    g, k, _ = obs[ASSOC_PLANE_LINE]
    g, k = np.asarray(g, np.int64), np.asarray(k, np.int64)
    a, o = _expand(k, loff, lord)
    recs["R4"] = dict(cam=lc[o], ln=k[a], pl=g[a], meas=lm[o])

    v, k, _ = obs[ASSOC_VP_LINE]
    recs["R5"] = dict(ln=np.asarray(k, np.int64), vp=np.asarray(v, np.int64))

    jp, jl, _ = obs[ASSOC_JUNCTION]
    jp, jl = np.asarray(jp, np.int64), np.asarray(jl, np.int64)
    ncam = max(len(scene["cameras"]), 1)
    pkeys = np.sort(pp * ncam + pc)
    lkeys = np.sort(ll * ncam + lc)
    # R6: views of the line where the point is not observed
    a, o = _expand(jl, loff, lord)
    cam = lc[o]
    seen = np.isin(jp[a] * ncam + cam, pkeys)
    recs["R6"] = dict(cam=cam[~seen], pt=jp[a][~seen], ln=jl[a][~seen], meas=lm[o][~seen])
    # R7: views of the point where the line is not observed
    a, o = _expand(jp, poff, pord)
    cam = pc[o]
    seen = np.isin(jl[a] * ncam + cam, lkeys)
    recs["R7"] = dict(cam=cam[~seen], ln=jl[a][~seen], pt=jp[a][~seen], meas=pm[o][~seen][:, 2:4])
    # inter-group relations (Sec. 3.2): one record per related pair of groups
    for fam in ("R8", "R9", "R10", "R11"):
        a, b, _ = obs.get(FAMILY_KIND[fam], (np.zeros(0), np.zeros(0), None))
        recs[fam] = dict(ga=np.asarray(a, np.int64), gb=np.asarray(b, np.int64))
    # R12: one record per 3D point-to-plane association (g, j), no camera
    g, j, _ = obs.get(ASSOC_PLANE_POINT_3D, (np.zeros(0), np.zeros(0), None))
    recs["R12"] = dict(pt=np.asarray(j, np.int64), pl=np.asarray(g, np.int64))
    # R13 / R14: surface groups, one record per association and view of the feature
    g, j, _ = obs.get(ASSOC_SHAPE_POINT, (np.zeros(0), np.zeros(0), None))
    g, j = np.asarray(g, np.int64), np.asarray(j, np.int64)
    a, o = _expand(j, poff, pord)
    recs["R13"] = dict(cam=pc[o], pt=j[a], sh=g[a])
    g, k, _ = obs.get(ASSOC_SHAPE_LINE, (np.zeros(0), np.zeros(0), None))
    g, k = np.asarray(g, np.int64), np.asarray(k, np.int64)
    a, o = _expand(k, loff, lord)
    recs["R14"] = dict(cam=lc[o], ln=k[a], sh=g[a], meas=lm[o])
    return recs


def record_keys(recs) -> dict:
    """(n, 4) int64 identity per record: family id, camera, feature, group/partner."""
    out = {}
    for fam, r in recs.items():
        n = len(next(iter(r.values())))
        neg = np.full(n, -1, dtype=np.int64)
        if fam == "R1":
            k = (r["cam"], r["pt"], neg)
        elif fam == "R2":
            k = (r["cam"], r["ln"], neg)
        elif fam == "R3":
            k = (r["cam"], r["pt"], r["pl"])
        elif fam == "R4":
            k = (r["cam"], r["ln"], r["pl"])
        elif fam == "R5":
            k = (neg, r["ln"], r["vp"])
        elif fam == "R6":
            k = (r["cam"], r["pt"], r["ln"])
        elif fam == "R7":
            k = (r["cam"], r["ln"], r["pt"])
        elif fam == "R12":
            k = (neg, r["pt"], r["pl"])
        elif fam == "R13":
            k = (r["cam"], r["pt"], r["sh"])
        elif fam == "R14":
            k = (r["cam"], r["ln"], r["sh"])
        else:  # relations: (-1, group a, group b)
            k = (neg, r["ga"], r["gb"])
        out[fam] = np.stack([np.full(n, FAMILY_ID[fam], dtype=np.int64), *k], axis=1)
    return out


def loss_of(scene, fam):
    from scenegen import DEFAULT_LOSS
    return scene["loss"].get(FAMILY_KIND[fam], DEFAULT_LOSS[FAMILY_KIND[fam]])
