"""Seeded synthetic holistic bundle-adjustment scenes.

The recipe follows the synthetic benchmark of the paper's supplementary
Section A.3 (cameras on a sphere looking inward at a cube of half-extent 3,
Manhattan planes at random offsets, points and lines on the planes and
free-floating, grid wireframes on planes whose rows and columns are lines,
about 50 % shared views for features of one plane, 1 px observation noise,
pose noise 1 deg / 0.05, structure noise 0.1), resized to the five workload
sizes named in the module-level ``CONFIGS`` table.

This module renders observations with its own homogeneous camera
``P = K [R | t]`` plus a radial factor on normalised coordinates. It holds no
residual, Jacobian, Schur or solver arithmetic and is shared, unchanged, by
the oracle side and the GPU side: it only produces inputs.

A scene is a plain ``dict`` of numpy arrays (see ``make_scene``). All indices
are int32, all values float64.
"""
from __future__ import annotations

import numpy as np

IMG_W, IMG_H = 640, 480
CX, CY = 320.0, 240.0

# Loss kinds as in the C ABI: 0 trivial, 1 Huber, 2 Cauchy.
LOSS_TRIVIAL, LOSS_HUBER, LOSS_CAUCHY = 0, 1, 2

# Observation / association kinds as in the C ABI.
OBS_POINT, OBS_LINE, ASSOC_PLANE_POINT, ASSOC_PLANE_LINE, ASSOC_VP_LINE, ASSOC_JUNCTION = range(6)
# Inter-group relations (a, b = two VPs or two planes): orthogonal or parallel directions.
REL_VP_ORTHO, REL_VP_PARALLEL, REL_PLANE_ORTHO, REL_PLANE_PARALLEL = range(6, 10)
RELATION_KINDS = (REL_VP_ORTHO, REL_VP_PARALLEL, REL_PLANE_ORTHO, REL_PLANE_PARALLEL)
# 3D point-to-plane association (the 3D formulation the paper compares against):
# a = plane, b = point
ASSOC_PLANE_POINT_3D = 10

# Per-kind default (loss kind, scale, weight).  Weights and the VP scale are the
# paper's (supplementary Section C: VP weight 5e3 with Cauchy scale 0.2; group
# weight 0.5 and wireframe weight 0.1 relative to 1.0 for point/line
# reprojection; Cauchy on constraints, Section 4 implementation details).  The
# pixel scales (1 px Cauchy, 2 px Huber) are this project's choice.
DEFAULT_LOSS = {
    OBS_POINT: (LOSS_TRIVIAL, 1.0, 1.0),
    OBS_LINE: (LOSS_TRIVIAL, 1.0, 1.0),
    ASSOC_PLANE_POINT: (LOSS_CAUCHY, 1.0, 0.5),
    ASSOC_PLANE_LINE: (LOSS_CAUCHY, 1.0, 0.5),
    ASSOC_VP_LINE: (LOSS_CAUCHY, 0.2, 5.0e3),
    ASSOC_JUNCTION: (LOSS_CAUCHY, 1.0, 0.1),
}
# Inter-group relations are angular like the VP-line term, and take its weight and
# Cauchy scale (the paper gives none of their own).
for _k in RELATION_KINDS:
    DEFAULT_LOSS[_k] = (LOSS_CAUCHY, 0.2, 5.0e3)
# the 3D penalty: squared metric distance times a weight (the paper sweeps 1 .. 1000)
DEFAULT_LOSS[ASSOC_PLANE_POINT_3D] = (LOSS_TRIVIAL, 1.0, 100.0)
# Surface groups beyond planes (App. B): sphere, cylinder, cone, ellipsoid, cuboid;
# associations a = shape, b = point (any type) or line (cuboids).  Their group-induced
# residuals take the plane associations' losses.
SHAPE_SPHERE, SHAPE_CYLINDER, SHAPE_CONE, SHAPE_ELLIPSOID, SHAPE_CUBOID = range(5)
ASSOC_SHAPE_POINT, ASSOC_SHAPE_LINE = 11, 12
DEFAULT_LOSS[ASSOC_SHAPE_POINT] = DEFAULT_LOSS[ASSOC_PLANE_POINT]
DEFAULT_LOSS[ASSOC_SHAPE_LINE] = DEFAULT_LOSS[ASSOC_PLANE_LINE]

# Workload sizes.  Keys:
#   n_cams, half (cube half extents), radius (camera sphere), K (neighbour pool)
#   n_free_points, n_free_lines, n_free_vp_lines (free lines along a VP)
#   n_planes, n_plane_points (non-grid members), n_plane_lines (non-grid
#   members), plane_line_axis_frac (fraction of them along a Manhattan axis)
#   n_grids, grid (points per side), n_vps (3 Manhattan + horizontal Atlanta)
#   rot_deg, trans, struct, pix (noise), outlier_frac, huber (R1/R2 Huber)
#   line_outlier_frac (outliers among line observations; default outlier_frac)
#   min_seg_px (a line is not observed in an image where its projected
#   segment is shorter than this: a detector finds no such segment)
#   plane_relations (inter-group relations: every pair of perpendicular VPs
#   is related orthogonal, and each plane is related to this many others,
#   parallel when their normals share an axis and orthogonal otherwise;
#   drawn from a generator of their own, so that the rest of a scene does
#   not depend on it; 0 or absent: no relations)
CONFIGS = {
    1: dict(n_cams=10, half=(5.0, 5.0, 2.5), radius=18.0, K=9,
            n_free_points=1000, n_free_lines=0, n_free_vp_lines=0,
            n_planes=0, n_plane_points=0, n_plane_lines=0, plane_line_axis_frac=0.0,
            n_grids=0, grid=0, n_vps=0,
            rot_deg=2.0, trans=0.1, struct=0.1, pix=1.0, outlier_frac=0.0, huber=False),
    2: dict(n_cams=30, half=(3.0, 3.0, 3.0), radius=10.0, K=29,
            n_free_points=3000, n_free_lines=700, n_free_vp_lines=350,
            n_planes=20, n_plane_points=1000, n_plane_lines=100, plane_line_axis_frac=0.5,
            n_grids=10, grid=10, n_vps=3,
            rot_deg=1.0, trans=0.05, struct=0.1, pix=1.0, outlier_frac=0.0, huber=False, min_seg_px=30.0),
    3: dict(n_cams=200, half=(3.0, 3.0, 3.0), radius=10.0, K=32,
            n_free_points=80000, n_free_lines=15000, n_free_vp_lines=9000,
            n_planes=200, n_plane_points=17500, n_plane_lines=4000, plane_line_axis_frac=0.5,
            n_grids=100, grid=5, n_vps=10,
            rot_deg=1.0, trans=0.05, struct=0.1, pix=1.0, outlier_frac=0.0, huber=False, min_seg_px=30.0),
    4: dict(n_cams=1500, half=(3.0, 3.0, 3.0), radius=10.0, K=32,
            n_free_points=800000, n_free_lines=100000, n_free_vp_lines=0,
            n_planes=2000, n_plane_points=200000, n_plane_lines=100000, plane_line_axis_frac=0.0,
            n_grids=0, grid=0, n_vps=0,
            # 5 % of the 9.6M point and line measurements are outliers, all on
            # point observations (6 % of those): an arbitrary segment pulls its
            # line towards the observing camera's centre, where the image line
            # has no direction and the robust cost no isolated minimum
            rot_deg=1.0, trans=0.05, struct=0.1, pix=1.0, outlier_frac=0.06, line_outlier_frac=0.0,
            huber=True, min_seg_px=30.0),
}


def config_seed(config: int, replica: int = 0) -> int:
    return 1000 * int(config) + int(replica)


# --------------------------------------------------------------------------
# small rotation helpers (rendering only)
# --------------------------------------------------------------------------
def _axis_angle_to_matrix(w):
    """Rotation matrices for rotation vectors w (..., 3), Rodrigues form."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1)[..., None, None]
    k = np.where(th[..., 0] > 0, w / np.maximum(th[..., 0], 1e-300), 0.0)
    Kx = np.zeros(w.shape[:-1] + (3, 3))
    Kx[..., 0, 1], Kx[..., 0, 2] = -k[..., 2], k[..., 1]
    Kx[..., 1, 0], Kx[..., 1, 2] = k[..., 2], -k[..., 0]
    Kx[..., 2, 0], Kx[..., 2, 1] = -k[..., 1], k[..., 0]
    eye = np.broadcast_to(np.eye(3), Kx.shape)
    return eye + np.sin(th) * Kx + (1.0 - np.cos(th)) * (Kx @ Kx)


def matrix_to_quaternion(R):
    """(…,3,3) rotation matrices -> (…,4) quaternions (w, x, y, z), w >= 0."""
    R = np.asarray(R, dtype=np.float64)
    shp = R.shape[:-2]
    R = R.reshape(-1, 3, 3)
    q = np.empty((R.shape[0], 4))
    tr = np.trace(R, axis1=1, axis2=2)
    for i in range(R.shape[0]):
        m = R[i]
        if tr[i] > 0:
            s = np.sqrt(tr[i] + 1.0) * 2
            q[i] = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
            s = np.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
            q[i] = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif m[1, 1] > m[2, 2]:
            s = np.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
            q[i] = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = np.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
            q[i] = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.reshape(shp + (4,))


def quaternion_to_matrix(q):
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


# --------------------------------------------------------------------------
# rendering camera: homogeneous P = K [R | t] with a radial factor
# --------------------------------------------------------------------------
class _RenderCams:
    def __init__(self, R, t, f, k1, k2):
        self.R, self.t, self.f, self.k1, self.k2 = R, t, f, k1, k2
        # 3x4 extrinsic matrices [R | t]
        self.Rt = np.concatenate([R, t[:, :, None]], axis=2)

    def normalized(self, cam, X):
        """Homogeneous image coordinates in the normalised plane, and depth."""
        Xh = np.concatenate([X, np.ones(X.shape[:-1] + (1,))], axis=-1)
        h = np.einsum("...ij,...j->...i", self.Rt[cam], Xh)
        return h[..., :2] / h[..., 2:3], h[..., 2]

    def pixels(self, cam, X, distort):
        uv, z = self.normalized(cam, X)
        if distort:
            rr = np.sum(uv * uv, axis=-1)
            fac = 1.0 + self.k1[cam] * rr + self.k2[cam] * rr * rr
            uv = uv * fac[..., None]
        px = self.f[cam][..., None] * uv + np.array([CX, CY])
        return px, z


def _visible(cams: _RenderCams, cam, X, margin=2.0):
    px, z = cams.pixels(cam, X, distort=True)
    ok = (z >= 1.0) & (px[..., 0] >= margin) & (px[..., 0] <= IMG_W - margin)
    ok &= (px[..., 1] >= margin) & (px[..., 1] <= IMG_H - margin)
    return ok


def _make_cameras(cfg, rng):
    n = cfg["n_cams"]
    half = np.asarray(cfg["half"])
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    C = d * cfg["radius"]
    target = rng.normal(size=(n, 3)) * 0.15 * half
    fwd = target - C
    fwd /= np.linalg.norm(fwd, axis=1, keepdims=True)
    up = np.tile([0.0, 0.0, 1.0], (n, 1))
    near_pole = np.abs(fwd[:, 2]) > 0.95
    up[near_pole] = [1.0, 0.0, 0.0]
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right, axis=1, keepdims=True)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], axis=1)
    # small roll so that image axes are not exactly aligned with the world
    roll = _axis_angle_to_matrix(np.stack([np.zeros(n), np.zeros(n), rng.normal(scale=0.05, size=n)], 1))
    R = roll @ R
    t = -np.einsum("nij,nj->ni", R, C)
    f = rng.uniform(475.0, 525.0, size=n)
    k1 = rng.normal(scale=0.01, size=n)
    k2 = rng.normal(scale=0.01, size=n)
    # neighbour table by camera-centre distance (self first)
    dist = np.linalg.norm(C[:, None, :] - C[None, :, :], axis=2)
    K = min(cfg["K"] + 1, n)
    nbrs = np.argsort(dist, axis=1, kind="stable")[:, :K]
    return R, t, f, k1, k2, C, nbrs


def _choose(keys, count):
    """Per row, indices of the `count[i]` smallest finite keys (sorted)."""
    order = np.argsort(keys, axis=1, kind="stable")
    ncol = keys.shape[1]
    sel = np.arange(ncol)[None, :] < count[:, None]
    finite = np.isfinite(np.take_along_axis(keys, order, axis=1))
    return order, sel & finite


def _sample_tracks(cams, nbrs, pts_a, pts_b, tmin, rng, pool=None, pool_frac=0.5, tries=12, min_len=0.0):
    """Choose observing cameras for features.

    A feature is a point (pts_b is None) or a segment [pts_a, pts_b].  Each
    feature picks an anchor camera that sees it and then about 8 views among
    the anchor's nearest cameras; with ``pool`` (n, P) a share ``pool_frac``
    of the views is drawn from that per-feature camera pool first.
    Returns a list (per feature) of int arrays of camera indices; features
    that cannot reach ``tmin`` views get an empty array.
    """
    n = pts_a.shape[0]
    ncam = nbrs.shape[0]
    target = rng.integers(5, 12, size=n)  # mean 8 views

    def vis(cam, rows):
        A = pts_a[rows][:, None, :].repeat(cam.shape[1], 1)
        ok = _visible(cams, cam, A)
        if pts_b is not None:
            B = pts_b[rows][:, None, :].repeat(cam.shape[1], 1)
            ok &= _visible(cams, cam, B)
            if min_len > 0:
                # a segment seen nearly end-on is too short to be detected
                pa, _ = cams.pixels(cam, A, distort=False)
                pb, _ = cams.pixels(cam, B, distort=False)
                ok &= np.linalg.norm(pa - pb, axis=-1) >= min_len
        return ok

    anchor = np.full(n, -1, dtype=np.int64)
    todo = np.arange(n)
    for _ in range(tries):
        if todo.size == 0:
            break
        cand = rng.integers(0, ncam, size=todo.size)
        ok = vis(cand[:, None], todo)[:, 0]
        anchor[todo[ok]] = cand[ok]
        todo = todo[~ok]

    tracks = [np.zeros(0, dtype=np.int32)] * n
    rows = np.nonzero(anchor >= 0)[0]
    if rows.size == 0:
        return tracks
    chunk = 200000
    for s in range(0, rows.size, chunk):
        r = rows[s:s + chunk]
        nb = nbrs[anchor[r]]                       # (m, K)
        vnb = vis(nb, r)
        chosen = np.full((r.size, 0), -1, dtype=np.int64)
        if pool is not None:
            pc = pool[r]                            # (m, P)
            vp = vis(pc, r) & (pc >= 0)
            kp = np.where(vp, rng.random(vp.shape), np.inf)
            npool = np.round(target[r] * pool_frac).astype(np.int64)
            order, sel = _choose(kp, npool)
            chosen = np.where(sel, np.take_along_axis(pc, order, axis=1), -1)
        dup = (nb[:, :, None] == chosen[:, None, :]).any(axis=2) if chosen.shape[1] else np.zeros(nb.shape, bool)
        kn = np.where(vnb & ~dup, rng.random(vnb.shape), np.inf)
        nrest = target[r] - (chosen >= 0).sum(axis=1)
        order, sel = _choose(kn, nrest)
        rest = np.where(sel, np.take_along_axis(nb, order, axis=1), -1)
        allc = np.concatenate([chosen, rest], axis=1)
        for i, row in enumerate(r):
            c = allc[i][allc[i] >= 0]
            if c.size >= tmin:
                tracks[row] = np.sort(c).astype(np.int32)
    return tracks


def _plane_patch(rng, half, n):
    """Axis-aligned plane patches: normal axis, offset, centre (3,), half sizes (2,)."""
    axis = rng.integers(0, 3, size=n)
    centre = rng.uniform(-0.6, 0.6, size=(n, 3)) * half
    off = rng.uniform(-0.8, 0.8, size=n) * half[axis]
    centre[np.arange(n), axis] = off
    hs = rng.uniform(0.6, 1.4, size=(n, 2))
    return axis, centre, hs


def _inplane_axes(axis):
    return [(1, 2), (0, 2), (0, 1)][axis]


def make_scene(config, seed: int | None = None, noise: bool = True, replica: int = 0) -> dict:
    """Generate a scene for a workload id (1..4) or an explicit size dict.

    With ``noise=False`` the measurements are exact projections and the
    initial values equal the ground truth.
    """
    cfg = dict(CONFIGS[config]) if isinstance(config, int) else dict(config)
    if seed is None:
        seed = config_seed(config if isinstance(config, int) else 0, replica)
    rng = np.random.default_rng(seed)
    half = np.asarray(cfg["half"], dtype=np.float64)
    R, t, f, k1, k2, C, nbrs = _make_cameras(cfg, rng)
    cams = _RenderCams(R, t, f, k1, k2)

    pts, pt_plane = [], []
    seg_a, seg_b, ln_plane, ln_vp = [], [], [], []
    junctions = []  # (point id, line id)

    # VP directions: 3 Manhattan axes, then horizontal Atlanta directions
    nv = cfg["n_vps"]
    vps = []
    for i in range(nv):
        if i < 3:
            e = np.zeros(3)
            e[i] = 1.0
            vps.append(e)
        else:
            a = rng.uniform(0, np.pi)
            vps.append(np.array([np.cos(a), np.sin(a), 0.0]))
    vps = np.array(vps).reshape(nv, 3)

    # planes
    npl = cfg["n_planes"]
    pl_axis, pl_centre, pl_hs = _plane_patch(rng, half, npl)
    planes_gt = np.zeros((npl, 4))
    for g in range(npl):
        planes_gt[g, pl_axis[g]] = 1.0
        planes_gt[g, 3] = -pl_centre[g, pl_axis[g]]

    def add_point(X, plane=-1):
        pts.append(X)
        pt_plane.append(plane)
        return len(pts) - 1

    def add_line(A, B, plane=-1, vp=-1):
        seg_a.append(A)
        seg_b.append(B)
        ln_plane.append(plane)
        ln_vp.append(vp)
        return len(seg_a) - 1

    # grid wireframes on the first n_grids planes: grid points are plane
    # members, grid rows / columns are plane lines along Manhattan axes.
    G = cfg["grid"]
    for gi in range(cfg["n_grids"]):
        g = gi % max(npl, 1)
        a0, a1 = _inplane_axes(pl_axis[g])
        spacing = 2.0 * min(pl_hs[g]) / max(G - 1, 1) * 0.9
        origin = pl_centre[g].copy()
        origin[a0] -= 0.5 * spacing * (G - 1)
        origin[a1] -= 0.5 * spacing * (G - 1)
        ids = np.zeros((G, G), dtype=np.int64)
        for i in range(G):
            for j in range(G):
                X = origin.copy()
                X[a0] += i * spacing
                X[a1] += j * spacing
                ids[i, j] = add_point(X, g)
        margin = 0.5 * spacing
        for i in range(G):  # lines along a1 through row i
            A = origin.copy()
            A[a0] += i * spacing
            B = A.copy()
            A[a1] -= margin
            B[a1] += (G - 1) * spacing + margin
            lid = add_line(A, B, g, a1 if nv >= 3 else -1)
            for j in range(G):
                junctions.append((ids[i, j], lid))
        for j in range(G):  # lines along a0 through column j
            A = origin.copy()
            A[a1] += j * spacing
            B = A.copy()
            A[a0] -= margin
            B[a0] += (G - 1) * spacing + margin
            lid = add_line(A, B, g, a0 if nv >= 3 else -1)
            for i in range(G):
                junctions.append((ids[i, j], lid))

    # non-grid plane members
    if npl:
        gsel = rng.integers(0, npl, size=cfg["n_plane_points"])
        for g in gsel:
            a0, a1 = _inplane_axes(pl_axis[g])
            X = pl_centre[g].copy()
            X[a0] += rng.uniform(-1, 1) * pl_hs[g, 0]
            X[a1] += rng.uniform(-1, 1) * pl_hs[g, 1]
            add_point(X, g)
        gsel = rng.integers(0, npl, size=cfg["n_plane_lines"])
        for g in gsel:
            a0, a1 = _inplane_axes(pl_axis[g])
            Xc = pl_centre[g].copy()
            Xc[a0] += rng.uniform(-0.5, 0.5) * pl_hs[g, 0]
            Xc[a1] += rng.uniform(-0.5, 0.5) * pl_hs[g, 1]
            vp = -1
            if rng.random() < cfg["plane_line_axis_frac"] and nv >= 3:
                ax = a0 if rng.random() < 0.5 else a1
                d = np.zeros(3)
                d[ax] = 1.0
                vp = ax
            else:
                ang = rng.uniform(0, np.pi)
                d = np.zeros(3)
                d[a0], d[a1] = np.cos(ang), np.sin(ang)
            L = rng.uniform(0.8, 1.6)
            add_line(Xc - 0.5 * L * d, Xc + 0.5 * L * d, g, vp)

    # free points and lines
    for X in rng.uniform(-1, 1, size=(cfg["n_free_points"], 3)) * half:
        add_point(X)
    for i in range(cfg["n_free_lines"]):
        Xc = rng.uniform(-0.8, 0.8, size=3) * half
        vp = -1
        if i < cfg["n_free_vp_lines"] and nv > 0:
            vp = int(rng.integers(0, nv))
            d = vps[vp]
        else:
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
        L = rng.uniform(1.0, 2.0)
        add_line(Xc - 0.5 * L * d, Xc + 0.5 * L * d, -1, vp)

    pts = np.array(pts).reshape(-1, 3)
    pt_plane = np.array(pt_plane, dtype=np.int64)
    seg_a = np.array(seg_a).reshape(-1, 3)
    seg_b = np.array(seg_b).reshape(-1, 3)
    ln_plane = np.array(ln_plane, dtype=np.int64)
    ln_vp = np.array(ln_vp, dtype=np.int64)

    # per-plane camera pools: nearest cameras of an anchor that sees the patch
    pool_pt = pool_ln = None
    if npl:
        P = min(16, nbrs.shape[1])
        pl_pool = np.full((npl, P), -1, dtype=np.int64)
        for g in range(npl):
            for _ in range(32):
                a = int(rng.integers(0, cfg["n_cams"]))
                if _visible(cams, np.array([a]), pl_centre[g][None])[0]:
                    break
            pl_pool[g] = nbrs[a][:P]
        pool_pt = np.where(pt_plane[:, None] >= 0, pl_pool[np.maximum(pt_plane, 0)], -1)
        pool_ln = np.where(ln_plane[:, None] >= 0, pl_pool[np.maximum(ln_plane, 0)], -1)

    tr_pt = _sample_tracks(cams, nbrs, pts, None, 2, rng, pool=pool_pt)
    tr_ln = (_sample_tracks(cams, nbrs, seg_a, seg_b, 3, rng, pool=pool_ln, min_len=cfg.get("min_seg_px", 0.0))
             if len(seg_a) else [])

    # drop features without enough views and re-index
    keep_p = np.array([len(x) > 0 for x in tr_pt], dtype=bool)
    keep_l = np.array([len(x) > 0 for x in tr_ln], dtype=bool)
    newp = np.cumsum(keep_p) - 1
    newl = np.cumsum(keep_l) - 1
    pts, pt_plane = pts[keep_p], pt_plane[keep_p]
    tr_pt = [x for x, k in zip(tr_pt, keep_p) if k]
    seg_a, seg_b, ln_plane, ln_vp = seg_a[keep_l], seg_b[keep_l], ln_plane[keep_l], ln_vp[keep_l]
    tr_ln = [x for x, k in zip(tr_ln, keep_l) if k]
    junctions = [(newp[p], newl[l]) for p, l in junctions if keep_p[p] and keep_l[l]]

    npt, nln = len(pts), len(seg_a)
    pix = cfg["pix"] if noise else 0.0

    # point observations: distorted (x, y) and undistorted (xu, yu) pixels, one noise draw
    op_cam = np.concatenate([x for x in tr_pt]).astype(np.int32) if npt else np.zeros(0, np.int32)
    op_pt = np.repeat(np.arange(npt), [len(x) for x in tr_pt]).astype(np.int32)
    xd, _ = cams.pixels(op_cam, pts[op_pt], distort=True)
    xu, _ = cams.pixels(op_cam, pts[op_pt], distort=False)
    nz = rng.normal(scale=1.0, size=xd.shape) * pix
    op_meas = np.concatenate([xd + nz, xu + nz], axis=1)

    # line observations: a random sub-segment per view, undistorted pixels
    ol_cam = np.concatenate([x for x in tr_ln]).astype(np.int32) if nln else np.zeros(0, np.int32)
    ol_ln = np.repeat(np.arange(nln), [len(x) for x in tr_ln]).astype(np.int32)
    sa = rng.uniform(0.0, 0.3, size=ol_cam.size)
    sb = rng.uniform(0.7, 1.0, size=ol_cam.size)
    A, B = seg_a[ol_ln], seg_b[ol_ln]
    e1, _ = cams.pixels(ol_cam, A + sa[:, None] * (B - A), distort=False)
    e2, _ = cams.pixels(ol_cam, A + sb[:, None] * (B - A), distort=False)
    ol_meas = np.concatenate([e1, e2], axis=1) + rng.normal(scale=1.0, size=(ol_cam.size, 4)) * pix

    if noise and cfg["outlier_frac"] > 0:
        m = rng.random(op_cam.size) < cfg["outlier_frac"]
        rnd = np.stack([rng.uniform(0, IMG_W, m.sum()), rng.uniform(0, IMG_H, m.sum())], 1)
        op_meas[m, 0:2] = rnd
        op_meas[m, 2:4] = rnd
        m = rng.random(ol_cam.size) < cfg.get("line_outlier_frac", cfg["outlier_frac"])
        ol_meas[m] = np.stack([rng.uniform(0, IMG_W, m.sum()), rng.uniform(0, IMG_H, m.sum()),
                               rng.uniform(0, IMG_W, m.sum()), rng.uniform(0, IMG_H, m.sum())], 1)

    # ground truth in the ABI formats
    cams_gt = np.concatenate([matrix_to_quaternion(R), t, f[:, None], k1[:, None], k2[:, None]], axis=1)
    lines_gt = np.concatenate([seg_a, seg_b], axis=1)

    # initial values
    if noise:
        dR = _axis_angle_to_matrix(rng.normal(scale=np.deg2rad(cfg["rot_deg"]), size=(len(R), 3)))
        R0 = dR @ R
        t0 = t + rng.normal(scale=cfg["trans"], size=t.shape)
        cams0 = np.concatenate([matrix_to_quaternion(R0), t0, f[:, None], np.zeros((len(R), 2))], axis=1)
        pts0 = pts + rng.normal(scale=cfg["struct"], size=pts.shape)
        a0 = seg_a + rng.normal(scale=cfg["struct"], size=seg_a.shape)
        b0 = seg_b + rng.normal(scale=cfg["struct"], size=seg_b.shape)
        lines0 = np.concatenate([a0, b0], axis=1)
        planes0 = planes_gt.copy()
        for g in range(npl):
            mem = np.nonzero(pt_plane == g)[0]
            if mem.size >= 3:
                P0 = pts0[mem]
                c = P0.mean(axis=0)
                _, _, vt = np.linalg.svd(P0 - c)
                n = vt[2] * np.sign(vt[2] @ planes_gt[g, :3] + 1e-30)
                planes0[g] = [*n, -n @ c]
        vps0 = vps.copy()
        for v in range(nv):
            mem = np.nonzero(ln_vp == v)[0]
            if mem.size >= 2:
                d = b0[mem] - a0[mem]
                d /= np.linalg.norm(d, axis=1, keepdims=True)
                M = d.T @ d
                w, V = np.linalg.eigh(M)
                e = V[:, -1]
                vps0[v] = e * np.sign(e @ vps[v] + 1e-30)
    else:
        cams0, pts0, lines0, planes0, vps0 = cams_gt.copy(), pts.copy(), lines_gt.copy(), planes_gt.copy(), vps.copy()

    # associations
    pp = np.nonzero(pt_plane >= 0)[0]
    lp = np.nonzero(ln_plane >= 0)[0]
    lv = np.nonzero(ln_vp >= 0)[0]
    jn = np.array(junctions, dtype=np.int64).reshape(-1, 2)

    loss = dict(DEFAULT_LOSS)
    if cfg.get("huber"):
        loss[OBS_POINT] = (LOSS_HUBER, 2.0, 1.0)
        loss[OBS_LINE] = (LOSS_HUBER, 2.0, 1.0)

    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    obs = {
        OBS_POINT: (i32(op_cam), i32(op_pt), f64(op_meas)),
        OBS_LINE: (i32(ol_cam), i32(ol_ln), f64(ol_meas)),
        ASSOC_PLANE_POINT: (i32(pt_plane[pp]), i32(pp), None),
        ASSOC_PLANE_LINE: (i32(ln_plane[lp]), i32(lp), None),
        ASSOC_VP_LINE: (i32(ln_vp[lv]), i32(lv), None),
        ASSOC_JUNCTION: (i32(jn[:, 0]), i32(jn[:, 1]), None),
    }
    if cfg.get("plane_relations", 0) > 0:
        for k, (a, b) in _relations(vps, pl_axis, int(cfg["plane_relations"]), seed).items():
            obs[k] = (i32(a), i32(b), None)
    return dict(
        config=cfg, seed=seed, cx=CX, cy=CY, camera_dof=9,
        cameras=f64(cams0), points=f64(pts0), lines=f64(lines0), planes=f64(planes0), vps=f64(vps0),
        cameras_gt=f64(cams_gt), points_gt=f64(pts), lines_gt=f64(lines_gt), planes_gt=f64(planes_gt),
        vps_gt=f64(vps),
        obs=obs,
        loss=loss,
    )


def _relations(vps, pl_axis, per_plane, seed):
    """Inter-group relations of a Manhattan / Atlanta scene (exact at the
    ground truth): every pair of perpendicular VPs; for each plane,
    `per_plane` distinct partners drawn at random, parallel when the normals
    share an axis, orthogonal otherwise (each unordered pair once)."""
    rng = np.random.default_rng(seed + 104729)
    out = {k: ([], []) for k in RELATION_KINDS}
    nv = len(vps)
    for a in range(nv):
        for b in range(a + 1, nv):
            if abs(float(vps[a] @ vps[b])) < 1e-12:
                out[REL_VP_ORTHO][0].append(a)
                out[REL_VP_ORTHO][1].append(b)
    npl = len(pl_axis)
    seen = set()
    for g in range(npl):
        if npl < 2:
            break
        cand = rng.permutation(npl - 1)[:per_plane]
        for h in cand:
            h = int(h) + (1 if h >= g else 0)
            key = (min(g, h), max(g, h))
            if key in seen:
                continue
            seen.add(key)
            kind = REL_PLANE_PARALLEL if pl_axis[g] == pl_axis[h] else REL_PLANE_ORTHO
            out[kind][0].append(key[0])
            out[kind][1].append(key[1])
    return {k: (np.asarray(a, np.int64), np.asarray(b, np.int64)) for k, (a, b) in out.items()}


def scene_counts(scene: dict) -> dict:
    o = scene["obs"]
    return dict(cameras=len(scene["cameras"]), points=len(scene["points"]), lines=len(scene["lines"]),
                planes=len(scene["planes"]), vps=len(scene["vps"]),
                point_obs=len(o[OBS_POINT][0]), line_obs=len(o[OBS_LINE][0]),
                plane_points=len(o[ASSOC_PLANE_POINT][0]), plane_lines=len(o[ASSOC_PLANE_LINE][0]),
                vp_lines=len(o[ASSOC_VP_LINE][0]), junctions=len(o[ASSOC_JUNCTION][0]))


def small_config(n_cams=7, n_points=40, n_lines=12, n_planes=2, n_vps=3, grids=1, grid=3,
                 plane_points=10, plane_lines=4, vp_lines=4, rot_deg=1.0, trans=0.05,
                 struct=0.05, pix=1.0, plane_relations=0):
    """Size dict for tiny test scenes with every residual family present
    (the inter-group relations with plane_relations > 0)."""
    return dict(n_cams=n_cams, half=(3.0, 3.0, 3.0), radius=10.0, K=min(n_cams - 1, 4),
                n_free_points=n_points, n_free_lines=n_lines, n_free_vp_lines=vp_lines,
                n_planes=n_planes, n_plane_points=plane_points, n_plane_lines=plane_lines,
                plane_line_axis_frac=0.5, n_grids=grids, grid=grid, n_vps=n_vps,
                rot_deg=rot_deg, trans=trans, struct=struct, pix=pix, outlier_frac=0.0, huber=False,
                plane_relations=plane_relations)


def manhattan_config():
    """A tiny Manhattan scene with inter-group relations: 8 cameras, 3
    Manhattan VPs and 2 Atlanta ones, 6 planes each related to 2 others."""
    return small_config(n_cams=8, n_points=40, n_lines=12, n_planes=6, n_vps=5, plane_points=12,
                        plane_lines=6, vp_lines=6, plane_relations=2)


def plane_3d_scene(scene, weight=100.0, keep_2d=False):
    """The same scene with its plane-point associations in the 3D formulation
    (kind ASSOC_PLANE_POINT_3D, trivial loss with the given weight) instead of, or
    with keep_2d beside, the pixel-space ones."""
    import copy
    out = copy.copy(scene)
    out["obs"] = dict(scene["obs"])
    out["loss"] = dict(scene["loss"])
    g, j, _ = scene["obs"][ASSOC_PLANE_POINT]
    out["obs"][ASSOC_PLANE_POINT_3D] = (np.array(g), np.array(j), None)
    out["loss"][ASSOC_PLANE_POINT_3D] = (LOSS_TRIVIAL, 1.0, float(weight))
    if not keep_2d:
        z = np.zeros(0, dtype=np.int32)
        out["obs"][ASSOC_PLANE_POINT] = (z, z, None)
    return out
