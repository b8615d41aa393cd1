"""Seeded surface groups added to a synthetic scene: one sphere, cylinder, cone,
ellipsoid and cuboid (the group types of the paper's App. B) inside the scene's
cube, points sampled on each surface, line segments lying in the cuboid's faces,
their observations rendered with the scene's own cameras, and noisy initial
values.  Inputs only, like ``scenegen.scene``: no residual or projection-operator
arithmetic.

Shapes are stored in the C-ABI format, a ``dict(type=(n,) int32, params=(n, 16)
float64)``:

* sphere: centre (3), radius
* cylinder: axis direction (3), a point on the axis (3), radius
* cone: apex (3), unit axis direction (3), half-angle (rad)
* ellipsoid: rotation R (row-major 9, local to world), centre (3), semi-axes (3)
* cuboid: rotation R (row-major 9), face offsets e_0 .. e_5: face i is the plane
  n_i . x + e_i = 0 with outward normal n_i = (-1)^i R e_{floor(i/2)}
"""
from __future__ import annotations

import numpy as np

from .scene import (_RenderCams, _sample_tracks, _axis_angle_to_matrix, quaternion_to_matrix, make_scene,
                    small_config, OBS_POINT, OBS_LINE, SHAPE_SPHERE, SHAPE_CYLINDER, SHAPE_CONE, SHAPE_ELLIPSOID,
                    SHAPE_CUBOID, ASSOC_SHAPE_POINT, ASSOC_SHAPE_LINE, DEFAULT_LOSS)


def _orthonormal(a):
    a = a / np.linalg.norm(a)
    e = np.zeros(3)
    e[np.argmin(np.abs(a))] = 1.0
    b1 = e - (e @ a) * a
    b1 /= np.linalg.norm(b1)
    return a, b1, np.cross(a, b1)


def _rot(rng, deg):
    return _axis_angle_to_matrix(rng.normal(scale=np.deg2rad(deg), size=(1, 3)))[0]


def _layout(rng):
    """Ground-truth shapes (type, params) at fixed places in the cube of half-extent 3."""
    j = lambda s: rng.normal(scale=s, size=3)
    types, params = [], []

    def add(t, vals):
        p = np.zeros(16)
        p[:len(vals)] = vals
        types.append(t)
        params.append(p)

    add(SHAPE_SPHERE, [*(np.array([-1.5, -1.5, 0.6]) + j(0.1)), 0.8])
    add(SHAPE_CYLINDER, [*(np.array([0.15, 0.1, 1.0]) + j(0.05)), *(np.array([1.6, -1.3, 0.0]) + j(0.1)), 0.6])
    d = np.array([0.1, -0.1, -1.0]) + j(0.05)
    add(SHAPE_CONE, [*(np.array([-1.3, 1.5, 1.8]) + j(0.1)), *(d / np.linalg.norm(d)), 0.45])
    R = _rot(rng, 25.0)
    add(SHAPE_ELLIPSOID, [*R.ravel(), *(np.array([1.5, 1.4, -0.7]) + j(0.1)), 0.9, 0.6, 0.45])
    R = _rot(rng, 20.0)
    c = np.array([0.0, 0.0, -1.6]) + j(0.1)
    m = R.T @ c
    h = np.array([0.9, 0.75, 0.6])
    e = np.zeros(6)
    e[0::2] = h - m
    e[1::2] = m + h
    add(SHAPE_CUBOID, [*R.ravel(), *e])
    return np.array(types, np.int32), np.array(params)


def _cuboid_frame(p):
    R = p[0:9].reshape(3, 3)
    e = p[9:15]
    lo, hi = -e[0::2], e[1::2]   # R_k . x ranges over [lo_k, hi_k]
    return R, lo, hi


def _sample_surface(rng, t, p, n):
    """n points on the surface of one ground-truth shape."""
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    phi = rng.uniform(0, 2 * np.pi, size=n)
    if t == SHAPE_SPHERE:
        return p[0:3] + p[3] * u
    if t == SHAPE_CYLINDER:
        a, b1, b2 = _orthonormal(p[0:3])
        h = rng.uniform(-1.0, 1.0, size=n)
        return p[3:6] + h[:, None] * a + p[6] * (np.cos(phi)[:, None] * b1 + np.sin(phi)[:, None] * b2)
    if t == SHAPE_CONE:
        a, b1, b2 = _orthonormal(p[3:6])
        h = rng.uniform(0.5, 1.6, size=n)
        rad = h * np.tan(p[6])
        return p[0:3] + h[:, None] * a + rad[:, None] * (np.cos(phi)[:, None] * b1 + np.sin(phi)[:, None] * b2)
    if t == SHAPE_ELLIPSOID:
        R = p[0:9].reshape(3, 3)
        return p[9:12] + (u * p[12:15]) @ R.T
    R, lo, hi = _cuboid_frame(p)
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    face = rng.integers(0, 6, size=n)
    loc = mid + rng.uniform(-0.6, 0.6, size=(n, 3)) * half   # away from the edges
    k = face // 2
    loc[np.arange(n), k] = np.where(face % 2 == 0, lo[k], hi[k])
    return loc @ R.T


def _cuboid_segments(rng, p, n):
    """n segments lying in the cuboid's faces, along one in-face axis."""
    R, lo, hi = _cuboid_frame(p)
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    A, B = np.zeros((n, 3)), np.zeros((n, 3))
    for i in range(n):
        f = int(rng.integers(0, 6))
        k = f // 2
        ax = [a for a in range(3) if a != k]
        along, across = (ax[0], ax[1]) if rng.random() < 0.5 else (ax[1], ax[0])
        loc = mid.copy()
        loc[k] = lo[k] if f % 2 == 0 else hi[k]
        loc[across] = mid[across] + rng.uniform(-0.5, 0.5) * half[across]
        a, b = loc.copy(), loc.copy()
        a[along] = mid[along] - 0.7 * half[along]
        b[along] = mid[along] + 0.7 * half[along]
        A[i], B[i] = R @ a, R @ b
    return A, B


def _perturb_shapes(rng, types, params):
    out = params.copy()
    for i, t in enumerate(types):
        p = out[i]
        if t == SHAPE_SPHERE:
            p[0:3] += rng.normal(scale=0.05, size=3)
            p[3] *= np.exp(rng.normal(scale=0.05))
        elif t == SHAPE_CYLINDER:
            p[0:3] = _rot(rng, 2.0) @ p[0:3]
            p[3:6] += rng.normal(scale=0.05, size=3)
            p[6] *= np.exp(rng.normal(scale=0.05))
        elif t == SHAPE_CONE:
            p[0:3] += rng.normal(scale=0.05, size=3)
            p[3:6] = _rot(rng, 2.0) @ p[3:6]
            p[6] *= np.exp(rng.normal(scale=0.03))
        elif t == SHAPE_ELLIPSOID:
            p[0:9] = (p[0:9].reshape(3, 3) @ _rot(rng, 2.0)).ravel()
            p[9:12] += rng.normal(scale=0.05, size=3)
            p[12:15] *= np.exp(rng.normal(scale=0.05, size=3))
        else:
            p[0:9] = (p[0:9].reshape(3, 3) @ _rot(rng, 2.0)).ravel()
            p[9:15] += rng.normal(scale=0.05, size=6)
    return out


def add_shapes(scene, seed, noise=True, points_per_shape=14, lines_per_cuboid=6):
    """A copy of `scene` with the five shapes, their surface points and the
    cuboid's face lines, observed by the scene's cameras (at least 3 views each)."""
    import copy
    rng = np.random.default_rng(seed)
    cfg = scene["config"]
    out = copy.copy(scene)
    out["obs"] = dict(scene["obs"])
    out["loss"] = dict(scene["loss"])
    cg = np.asarray(scene["cameras_gt"])
    cams = _RenderCams(quaternion_to_matrix(cg[:, 0:4]), cg[:, 4:7], cg[:, 7], cg[:, 8], cg[:, 9])
    C = -np.einsum("nji,nj->ni", cams.R, cams.t)
    dist = np.linalg.norm(C[:, None, :] - C[None, :, :], axis=2)
    nbrs = np.argsort(dist, axis=1, kind="stable")[:, :min(cfg["K"] + 1, len(C))]

    types, params = _layout(rng)
    pts, sh_of_pt = [], []
    for s, (t, p) in enumerate(zip(types, params)):
        pts.append(_sample_surface(rng, t, p, points_per_shape))
        sh_of_pt += [s] * points_per_shape
    pts = np.concatenate(pts)
    sh_of_pt = np.array(sh_of_pt)
    cub = int(np.nonzero(types == SHAPE_CUBOID)[0][0])
    seg_a, seg_b = _cuboid_segments(rng, params[cub], lines_per_cuboid)

    tr_pt = _sample_tracks(cams, nbrs, pts, None, 3, rng)
    tr_ln = _sample_tracks(cams, nbrs, seg_a, seg_b, 3, rng, min_len=30.0)
    kp = np.array([len(x) > 0 for x in tr_pt], dtype=bool)
    kl = np.array([len(x) > 0 for x in tr_ln], dtype=bool)
    pts, sh_of_pt, tr_pt = pts[kp], sh_of_pt[kp], [x for x, k in zip(tr_pt, kp) if k]
    seg_a, seg_b, tr_ln = seg_a[kl], seg_b[kl], [x for x, k in zip(tr_ln, kl) if k]
    pix = cfg["pix"] if noise else 0.0
    np0, nl0 = len(scene["points"]), len(scene["lines"])

    op_cam = np.concatenate(tr_pt).astype(np.int32)
    op_pt = np.repeat(np.arange(len(pts)), [len(x) for x in tr_pt])
    xd, _ = cams.pixels(op_cam, pts[op_pt], distort=True)
    xu, _ = cams.pixels(op_cam, pts[op_pt], distort=False)
    nz = rng.normal(size=xd.shape) * pix
    op_meas = np.concatenate([xd + nz, xu + nz], axis=1)
    ol_cam = np.concatenate(tr_ln).astype(np.int32) if len(tr_ln) else np.zeros(0, np.int32)
    ol_ln = np.repeat(np.arange(len(seg_a)), [len(x) for x in tr_ln])
    sa = rng.uniform(0.0, 0.3, size=ol_cam.size)
    sb = rng.uniform(0.7, 1.0, size=ol_cam.size)
    A, B = seg_a[ol_ln], seg_b[ol_ln]
    e1, _ = cams.pixels(ol_cam, A + sa[:, None] * (B - A), distort=False)
    e2, _ = cams.pixels(ol_cam, A + sb[:, None] * (B - A), distort=False)
    ol_meas = np.concatenate([e1, e2], axis=1) + rng.normal(size=(ol_cam.size, 4)) * pix

    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    c0, p0, m0 = scene["obs"][OBS_POINT]
    out["obs"][OBS_POINT] = (i32(np.concatenate([c0, op_cam])), i32(np.concatenate([p0, np0 + op_pt])),
                             f64(np.concatenate([np.asarray(m0).reshape(-1, 4), op_meas])))
    c0, l0, m0 = scene["obs"][OBS_LINE]
    out["obs"][OBS_LINE] = (i32(np.concatenate([c0, ol_cam])), i32(np.concatenate([l0, nl0 + ol_ln])),
                            f64(np.concatenate([np.asarray(m0).reshape(-1, 4), ol_meas])))
    out["obs"][ASSOC_SHAPE_POINT] = (i32(sh_of_pt), i32(np0 + np.arange(len(pts))), None)
    out["obs"][ASSOC_SHAPE_LINE] = (i32(np.full(len(seg_a), cub)), i32(nl0 + np.arange(len(seg_a))), None)
    out["loss"][ASSOC_SHAPE_POINT] = DEFAULT_LOSS[ASSOC_SHAPE_POINT]
    out["loss"][ASSOC_SHAPE_LINE] = DEFAULT_LOSS[ASSOC_SHAPE_LINE]

    if noise:
        pts0 = pts + rng.normal(scale=cfg["struct"], size=pts.shape)
        a0 = seg_a + rng.normal(scale=cfg["struct"], size=seg_a.shape)
        b0 = seg_b + rng.normal(scale=cfg["struct"], size=seg_b.shape)
        params0 = _perturb_shapes(rng, types, params)
    else:
        pts0, a0, b0, params0 = pts, seg_a, seg_b, params
    out["points"] = f64(np.concatenate([scene["points"], pts0]))
    out["points_gt"] = f64(np.concatenate([scene["points_gt"], pts]))
    out["lines"] = f64(np.concatenate([scene["lines"], np.concatenate([a0, b0], axis=1)]))
    out["lines_gt"] = f64(np.concatenate([scene["lines_gt"], np.concatenate([seg_a, seg_b], axis=1)]))
    out["shapes"] = dict(type=i32(types), params=f64(params0))
    out["shapes_gt"] = dict(type=i32(types), params=f64(params))
    return out


def shape_scene(seed=301, noise=True, n_cams=10):
    """A tiny holistic scene (every residual family) with the five shapes added."""
    base = make_scene(small_config(n_cams=n_cams, n_points=40, n_lines=12), seed=seed, noise=noise)
    return add_shapes(base, seed + 1, noise=noise)
