"""Parameters, manifolds, projections and residual families in plain FP64.

Every function is vectorised over records and written with complex-analytic
operations only (no abs, no conjugates), so the same code evaluates the
residual at real parameters and, with an imaginary tangent step, its
derivative by complex-step differentiation.

Conventions (readings of the paper, stated once here):

* camera i: rotation R, translation t, focal f, radial k1, k2; X_c = R X + t;
  principal point (cx, cy) fixed.  Tangent (dtheta, dt, df, dk1, dk2):
  R <- Exp(dtheta) R, t <- Exp(dtheta) t + dt (a left perturbation of the
  camera frame).  camera_dof 6 drops (df, dk1, dk2).  Sec. 3.1 names
  C_i = (K, R, t) and leaves the intrinsic model open.
* distorted projection pi_p: u = X_c,x / X_c,z, v likewise, s = 1 + k1 r^2 +
  k2 r^4, pixel = (f s u + cx, f s v + cy); the pinhole pi-bar drops s.
* line: orthonormal Pluecker form (Sec. 2, Sec. 3.2; 4 DOF).  U in SO(3),
  (w1, w2) on the unit circle, direction d = w1 U e1, moment m = w2 U e2 with
  m = p x d for any point p on the line.  Tangent (dtheta_L, dphi):
  U <- U Exp(dtheta_L), (w1, w2) <- rotation of (w1, w2) by dphi.
* plane (n, w), n unit, n . x + w = 0 (App. B); tangent (dn in R^2, dw) with
  the basis B_n = [b1, b2], b1 = normalise(e_k - (e_k . n) n) for the index
  k of the smallest |n_k| (lowest index on ties), b2 = n x b1, and
  n <- cos|v| n + sin|v| v/|v|, v = B_n dn.
* vanishing direction v unit, 2 DOF, same sphere chart as the plane normal.
* lines in the image are in undistorted pixels: the image line of (d, m) in
  camera i is l = (m_c,x, m_c,y, f m_c,z - cx m_c,x - cy m_c,y) with
  d_c = R d and m_c = R m + t x d_c, i.e. K^-T m_c up to the factor f.
"""
from __future__ import annotations

import numpy as np

CAM_DOF_MAX = 9
POINT_DOF, LINE_DOF, PLANE_DOF, VP_DOF = 3, 4, 3, 2
SHAPE_DOF = 9  # tangent coordinates of every surface group (oracle.shapes)


# ---------------------------------------------------------------------------
# complex-safe small vector helpers
# ---------------------------------------------------------------------------
def dot(a, b):
    return np.sum(a * b, axis=-1)


def cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def skew(v):
    z = np.zeros_like(v[..., 0])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], axis=-2)


def matvec(M, v):
    return np.einsum("...ij,...j->...i", M, v)


def so3_exp(w):
    """Rodrigues exponential of rotation vectors (real arrays)."""
    w = np.asarray(w, dtype=np.float64)
    th = np.sqrt(dot(w, w))[..., None, None]
    W = skew(w)
    small = th < 1e-8
    ths = np.where(small, 1.0, th)
    a = np.where(small, 1.0 - th ** 2 / 6.0, np.sin(ths) / ths)
    b = np.where(small, 0.5 - th ** 2 / 24.0, (1.0 - np.cos(ths)) / ths ** 2)
    return np.eye(3) + a * W + b * (W @ W)


def s2_basis(n):
    """Tangent basis B_n (..., 3, 2) of the unit sphere at n (real)."""
    n = np.asarray(n, dtype=np.float64)
    k = np.argmin(np.abs(n), axis=-1)
    e = np.zeros_like(n)
    np.put_along_axis(e, k[..., None], 1.0, axis=-1)
    b1 = e - dot(e, n)[..., None] * n
    b1 = b1 / np.sqrt(dot(b1, b1))[..., None]
    b2 = cross(n, b1)
    return np.stack([b1, b2], axis=-1)


def s2_retract(n, dn):
    v = matvec(s2_basis(n), dn)
    th = np.sqrt(dot(v, v))[..., None]
    ths = np.where(th < 1e-12, 1.0, th)
    out = np.cos(th) * n + np.where(th < 1e-12, v, np.sin(th) * v / ths)
    return out / np.sqrt(dot(out, out))[..., None]


# ---------------------------------------------------------------------------
# lines: orthonormal representation
# ---------------------------------------------------------------------------
def line_from_points(P, Q):
    """Orthonormal representation (U, w) of the line through P and Q."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    d = Q - P
    m = cross(P, d)
    nd = np.sqrt(dot(d, d))
    nm = np.sqrt(dot(m, m))
    u1 = d / nd[..., None]
    deg = nm < 1e-12 * nd
    # m = 0 (line through the origin): any unit vector orthogonal to u1
    k = np.argmin(np.abs(u1), axis=-1)
    e = np.zeros_like(u1)
    np.put_along_axis(e, k[..., None], 1.0, axis=-1)
    alt = e - dot(e, u1)[..., None] * u1
    alt = alt / np.sqrt(dot(alt, alt))[..., None]
    u2 = np.where(deg[..., None], alt, m / np.where(deg, 1.0, nm)[..., None])
    u3 = cross(u1, u2)
    U = np.stack([u1, u2, u3], axis=-1)
    nm = np.where(deg, 0.0, nm)
    s = np.sqrt(nd ** 2 + nm ** 2)
    w = np.stack([nd / s, nm / s], axis=-1)
    return U, w


def line_plucker(U, w):
    """(d, m) = (w1 U e1, w2 U e2)."""
    return w[..., 0:1] * U[..., :, 0], w[..., 1:2] * U[..., :, 1]


def plane_project_point(X, n, w):
    """Proj_G(X) = X - (n.X + w) / |n|^2 n  (Sec. 3.3 Eq. 7, App. B)."""
    return X - ((dot(n, X) + w) / dot(n, n))[..., None] * n


def plane_project_line(d, m, n, w):
    """Pluecker line (d, m) projected onto the plane n.x + w = 0 (App. B).

    d' = d - (d.n) n and
    m' = (1 - a^2/|d|^2) m + (a g/|d|^2) d + (w - e/|d|^2) (d x n)
    with a = d.n, g = m.n, e = (d x n).m.
    """
    a = dot(d, n)
    g = dot(m, n)
    dxn = cross(d, n)
    e = dot(dxn, m)
    dd = dot(d, d)
    d2 = d - a[..., None] * n
    m2 = ((1.0 - a * a / dd)[..., None] * m + (a * g / dd)[..., None] * d
          + (w - e / dd)[..., None] * dxn)
    return d2, m2


# ---------------------------------------------------------------------------
# camera model
# ---------------------------------------------------------------------------
def to_camera(R, t, X):
    return matvec(R, X) + t


def project_distorted(R, t, f, k1, k2, X, cx, cy):
    Xc = to_camera(R, t, X)
    u = Xc[..., 0] / Xc[..., 2]
    v = Xc[..., 1] / Xc[..., 2]
    r2 = u * u + v * v
    s = 1.0 + k1 * r2 + k2 * r2 * r2
    return np.stack([f * s * u + cx, f * s * v + cy], axis=-1)


def project_pinhole(R, t, f, X, cx, cy):
    Xc = to_camera(R, t, X)
    return np.stack([f * Xc[..., 0] / Xc[..., 2] + cx, f * Xc[..., 1] / Xc[..., 2] + cy], axis=-1)


def image_line(R, t, f, d, m, cx, cy):
    """Image line (undistorted pixels) of the 3D line (d, m) in camera (R, t, f)."""
    dc = matvec(R, d)
    mc = matvec(R, m) + cross(t, dc)
    return np.stack([mc[..., 0], mc[..., 1], f * mc[..., 2] - cx * mc[..., 0] - cy * mc[..., 1]], axis=-1)


def endpoint_vectors(l, e):
    """Perpendicular vector from the foot of endpoint e on line l to e.

    l (..., 3) homogeneous, e (..., 2).  Returns (h/q) (l1, l2) with
    h = l . (e, 1), q = l1^2 + l2^2; its norm is the point-line distance,
    invariant to the scale and sign of l.
    """
    h = l[..., 0] * e[..., 0] + l[..., 1] * e[..., 1] + l[..., 2]
    q = l[..., 0] ** 2 + l[..., 1] ** 2
    return (h / q)[..., None] * l[..., :2]


def rho4(l, meas4):
    """The 4-vector rho of Sec. 3.2 Eq. 4 for observed endpoints meas4 = (e1, e2)."""
    return np.concatenate([endpoint_vectors(l, meas4[..., 0:2]), endpoint_vectors(l, meas4[..., 2:4])], axis=-1)


def signed_distance(x, l):
    """l . (x, 1) / sqrt(l1^2 + l2^2): perpendicular point-line distance."""
    return (l[..., 0] * x[..., 0] + l[..., 1] * x[..., 1] + l[..., 2]) / np.sqrt(l[..., 0] ** 2 + l[..., 1] ** 2)


def observed_line(meas4):
    """Homogeneous line through the two observed endpoints, (e1, 1) x (e2, 1)."""
    one = np.ones_like(meas4[..., 0])
    a = np.stack([meas4[..., 0], meas4[..., 1], one], -1)
    b = np.stack([meas4[..., 2], meas4[..., 3], one], -1)
    return cross(a, b)


# ---------------------------------------------------------------------------
# parameter state
# ---------------------------------------------------------------------------
class State:
    """FP64 parameters of a holistic BA problem."""

    def __init__(self, cam_R, cam_t, cam_f, cam_k1, cam_k2, pts, line_U, line_w, pl_n, pl_w, vp, sh=None):
        from .shapes import Shapes
        self.cam_R, self.cam_t = cam_R, cam_t
        self.cam_f, self.cam_k1, self.cam_k2 = cam_f, cam_k1, cam_k2
        self.pts = pts
        self.line_U, self.line_w = line_U, line_w
        self.pl_n, self.pl_w = pl_n, pl_w
        self.vp = vp
        self.sh = Shapes.empty() if sh is None else sh  # surface groups (oracle.shapes)

    @staticmethod
    def from_arrays(cameras, points, lines, planes, vps, shapes=None):
        from scenegen import quaternion_to_matrix  # input format conversion only
        cameras = np.asarray(cameras, dtype=np.float64).reshape(-1, 10)
        R = quaternion_to_matrix(cameras[:, 0:4]) if len(cameras) else np.zeros((0, 3, 3))
        lines = np.asarray(lines, dtype=np.float64).reshape(-1, 6)
        U, w = line_from_points(lines[:, 0:3], lines[:, 3:6])
        planes = np.asarray(planes, dtype=np.float64).reshape(-1, 4)
        vps = np.asarray(vps, dtype=np.float64).reshape(-1, 3)
        from .shapes import Shapes
        sh = None if shapes is None else Shapes.from_abi(shapes["type"], shapes["params"])
        return State(R, cameras[:, 4:7].copy(), cameras[:, 7].copy(), cameras[:, 8].copy(),
                     cameras[:, 9].copy(), np.asarray(points, dtype=np.float64).reshape(-1, 3).copy(),
                     U, w, planes[:, 0:3].copy(), planes[:, 3].copy(), vps.copy(), sh)

    @staticmethod
    def from_scene(scene, gt=False):
        sfx = "_gt" if gt else ""
        return State.from_arrays(scene["cameras" + sfx], scene["points" + sfx], scene["lines" + sfx],
                                 scene["planes" + sfx], scene["vps" + sfx], scene.get("shapes" + sfx))

    def copy(self):
        return State(*(a.copy() for a in (self.cam_R, self.cam_t, self.cam_f, self.cam_k1, self.cam_k2,
                                          self.pts, self.line_U, self.line_w, self.pl_n, self.pl_w, self.vp)),
                     self.sh.copy())

    @property
    def counts(self):
        return dict(cameras=len(self.cam_R), points=len(self.pts), lines=len(self.line_U),
                    planes=len(self.pl_n), vps=len(self.vp), shapes=len(self.sh))

    def plucker(self):
        return line_plucker(self.line_U, self.line_w)

    def retract(self, dcam, dpt, dln, dpl, dvp, camera_dof=9, dsh=None):
        """x [+] h with the exact manifold updates listed in the module docstring
        (shapes: oracle.shapes)."""
        s = self.copy()
        if len(s.sh) and dsh is not None:
            s.sh = self.sh.retract(dsh)
        if len(s.cam_R):
            dcam = np.asarray(dcam).reshape(len(s.cam_R), camera_dof)
            E = so3_exp(dcam[:, 0:3])
            s.cam_R = E @ self.cam_R
            s.cam_t = matvec(E, self.cam_t) + dcam[:, 3:6]
            if camera_dof == 9:
                s.cam_f = self.cam_f + dcam[:, 6]
                s.cam_k1 = self.cam_k1 + dcam[:, 7]
                s.cam_k2 = self.cam_k2 + dcam[:, 8]
        if len(s.pts):
            s.pts = self.pts + np.asarray(dpt).reshape(-1, 3)
        if len(s.line_U):
            dln = np.asarray(dln).reshape(-1, 4)
            s.line_U = self.line_U @ so3_exp(dln[:, 0:3])
            c, sn = np.cos(dln[:, 3]), np.sin(dln[:, 3])
            w1, w2 = self.line_w[:, 0], self.line_w[:, 1]
            s.line_w = np.stack([w1 * c - w2 * sn, w1 * sn + w2 * c], axis=-1)
        if len(s.pl_n):
            dpl = np.asarray(dpl).reshape(-1, 3)
            s.pl_n = s2_retract(self.pl_n, dpl[:, 0:2])
            s.pl_w = self.pl_w + dpl[:, 2]
        if len(s.vp):
            s.vp = s2_retract(self.vp, np.asarray(dvp).reshape(-1, 2))
        return s

    def to_abi(self):
        """Parameters in the C-ABI output formats (cameras as quaternions,
        lines as unit direction and moment over |d|, planes (n, w), vps)."""
        from scenegen import matrix_to_quaternion
        cams = np.concatenate([matrix_to_quaternion(self.cam_R) if len(self.cam_R) else np.zeros((0, 4)),
                               self.cam_t, self.cam_f[:, None], self.cam_k1[:, None], self.cam_k2[:, None]], 1)
        d, m = self.plucker()
        nd = np.sqrt(dot(d, d))[..., None]
        lines = np.concatenate([d / nd, m / nd], axis=1)
        planes = np.concatenate([self.pl_n, self.pl_w[:, None]], axis=1)
        return cams, self.pts.copy(), lines, planes, self.vp.copy()


# ---------------------------------------------------------------------------
# per-record parameter gathering and first-order tangent perturbation
# ---------------------------------------------------------------------------
class Gathered:
    """Per-record complex copies of the parameter blocks a family touches.

    An inter-group relation record touches two groups of one kind (`rel` =
    (kind "vp" or "pl", index a, index b)): their directions (the VP, or the
    plane normal) and sphere tangent bases are gathered as ua, Ba, ub, Bb."""

    def __init__(self, state: State, cam=None, pt=None, ln=None, pl=None, vp=None, rel=None, sh=None):
        c = np.complex128
        if sh is not None:
            from .shapes import GatheredShapes
            self.sh = GatheredShapes(state.sh, sh)
        if rel is not None:
            kind, ia, ib = rel
            src = state.vp if kind == "vp" else state.pl_n
            self.ua, self.ub = src[ia].astype(c), src[ib].astype(c)
            self.Ba, self.Bb = s2_basis(src[ia]), s2_basis(src[ib])
            return
        self.R = state.cam_R[cam].astype(c) if cam is not None else None
        self.t = state.cam_t[cam].astype(c) if cam is not None else None
        self.f = state.cam_f[cam].astype(c) if cam is not None else None
        self.k1 = state.cam_k1[cam].astype(c) if cam is not None else None
        self.k2 = state.cam_k2[cam].astype(c) if cam is not None else None
        self.X = state.pts[pt].astype(c) if pt is not None else None
        self.U = state.line_U[ln].astype(c) if ln is not None else None
        self.w = state.line_w[ln].astype(c) if ln is not None else None
        self.n = state.pl_n[pl].astype(c) if pl is not None else None
        self.wp = state.pl_w[pl].astype(c) if pl is not None else None
        self.Bn = s2_basis(state.pl_n[pl]) if pl is not None else None
        self.v = state.vp[vp].astype(c) if vp is not None else None
        self.Bv = s2_basis(state.vp[vp]) if vp is not None else None

    def plucker(self):
        return line_plucker(self.U, self.w)

    def perturb(self, block, k, h):
        """First-order tangent step h along coordinate k of `block` (in place)."""
        if block == "cam":
            if k < 3:
                e = np.zeros(3, dtype=np.complex128)
                e[k] = h
                Sk = np.eye(3) + skew(e)
                self.R = Sk @ self.R
                self.t = matvec(Sk, self.t)
            elif k < 6:
                self.t = self.t.copy()
                self.t[:, k - 3] += h
            elif k == 6:
                self.f = self.f + h
            elif k == 7:
                self.k1 = self.k1 + h
            else:
                self.k2 = self.k2 + h
        elif block == "pt":
            self.X = self.X.copy()
            self.X[:, k] += h
        elif block == "ln":
            if k < 3:
                e = np.zeros(3, dtype=np.complex128)
                e[k] = h
                self.U = self.U @ (np.eye(3) + skew(e))
            else:
                w1, w2 = self.w[:, 0], self.w[:, 1]
                self.w = np.stack([w1 - h * w2, w2 + h * w1], axis=-1)
        elif block == "pl":
            if k < 2:
                self.n = self.n + h * self.Bn[:, :, k]
            else:
                self.wp = self.wp + h
        elif block == "vp":
            self.v = self.v + h * self.Bv[:, :, k]
        elif block == "sh":
            self.sh.perturb(k, h)
        elif block in ("ga", "gb"):
            # a relation's group: the direction moves with the first two tangent
            # coordinates; a plane's third (the offset w) leaves it unchanged
            if k < 2:
                if block == "ga":
                    self.ua = self.ua + h * self.Ba[:, :, k]
                else:
                    self.ub = self.ub + h * self.Bb[:, :, k]
        else:
            raise ValueError(block)


# ---------------------------------------------------------------------------
# residual families
# ---------------------------------------------------------------------------
def res_point(g: Gathered, rec, cx, cy):
    """R1, Sec. 3.1 Eq. 1: pi_p(C_i, X_j) - x_ij (distorted pixels)."""
    return project_distorted(g.R, g.t, g.f, g.k1, g.k2, g.X, cx, cy) - rec["meas"]


def res_line(g: Gathered, rec, cx, cy):
    """R2, Sec. 3.2 Eq. 4: rho(pi_l(C_i, L_k), l_ik) in R^4."""
    d, m = g.plucker()
    return rho4(image_line(g.R, g.t, g.f, d, m, cx, cy), rec["meas"])


def res_plane_point(g: Gathered, rec, cx, cy):
    """R3, Sec. 3.3 Eq. 7: pi_p(C_i, X_j) - pi_p(C_i, Proj_G(X_j))."""
    Xp = plane_project_point(g.X, g.n, g.wp)
    return (project_distorted(g.R, g.t, g.f, g.k1, g.k2, g.X, cx, cy)
            - project_distorted(g.R, g.t, g.f, g.k1, g.k2, Xp, cx, cy))


def res_plane_line(g: Gathered, rec, cx, cy):
    """R4, Sec. 3.3 Eq. 8 with the plane-line projection of App. B.

    A line nearly orthogonal to the plane (|d'|^2 < 1e-12 |d|^2) has no
    defined projection; such a record contributes zero (a reading: the
    paper does not treat the case)."""
    d, m = g.plucker()
    d2, m2 = plane_project_line(d, m, g.n, g.wp)
    l1 = image_line(g.R, g.t, g.f, d, m, cx, cy)
    l2 = image_line(g.R, g.t, g.f, d2, m2, cx, cy)
    r = rho4(l1, rec["meas"]) - rho4(l2, rec["meas"])
    deg = np.real(dot(d2, d2)) < 1e-12 * np.real(dot(d, d))
    return np.where(deg[:, None], 0.0, r)


def res_vp_line(g: Gathered, rec, cx, cy):
    """R5, Sec. 3.3 Eq. 6 / App. B: the 3-vector (d/|d|) x v.

    Its norm is |sin theta|, the paper's scalar residual; the vector form
    has the same squared cost and is smooth at zero (a reading)."""
    d, _ = g.plucker()
    u = d / np.sqrt(dot(d, d))[..., None]
    return cross(u, g.v)


def res_plane_point_3d(g: Gathered, rec, cx, cy):
    """R12, the 3D formulation the paper compares against (Sec. 3.3 discussion,
    Sec. 4 ablation): the signed metric distance n . X + w of the point to the
    plane, in scene units (the weight of the sweep enters through the loss)."""
    return (dot(g.n, g.X) + g.wp)[..., None]


def res_shape_point(g: Gathered, rec, cx, cy):
    """R13, Sec. 3.3 after Eq. 8 (any group with a projection operator) with the
    projections of App. B: pi_p(C_i, X_j) - pi_p(C_i, Proj_G(X_j)) for a sphere,
    cylinder, cone, ellipsoid or cuboid (oracle.shapes)."""
    from .shapes import project_point
    Xp = project_point(g.sh, g.X)
    return (project_distorted(g.R, g.t, g.f, g.k1, g.k2, g.X, cx, cy)
            - project_distorted(g.R, g.t, g.f, g.k1, g.k2, Xp, cx, cy))


def res_shape_line(g: Gathered, rec, cx, cy):
    """R14: Eq. 8 for a line on a cuboid (App. B): the line is projected onto the
    plane of the face chosen for it (oracle.shapes) with the plane-line
    projection; a line nearly orthogonal to that face contributes zero, as in R4."""
    from .shapes import cuboid_line_plane
    d, m = g.plucker()
    n, w = cuboid_line_plane(g.sh, d, m)
    d2, m2 = plane_project_line(d, m, n, w)
    l1 = image_line(g.R, g.t, g.f, d, m, cx, cy)
    l2 = image_line(g.R, g.t, g.f, d2, m2, cx, cy)
    r = rho4(l1, rec["meas"]) - rho4(l2, rec["meas"])
    deg = np.real(dot(d2, d2)) < 1e-12 * np.real(dot(d, d))
    return np.where(deg[:, None], 0.0, r)


def res_point_to_line(g: Gathered, rec, cx, cy):
    """R6, Sec. 3.4 Eq. 11: d(pi-bar(C_i, X_j), l_ik), observed line l_ik."""
    x = project_pinhole(g.R, g.t, g.f, g.X, cx, cy)
    return signed_distance(x, observed_line(rec["meas"]))[..., None]


def res_line_to_point(g: Gathered, rec, cx, cy):
    """R7, Sec. 3.4 Eq. 12: d(x-bar_ij, pi_l(C_i, L_k)), observed point x-bar_ij."""
    d, m = g.plucker()
    l = image_line(g.R, g.t, g.f, d, m, cx, cy)
    return signed_distance(rec["meas"], l)[..., None]


def res_rel_ortho(g: Gathered, rec, cx, cy):
    """Inter-group orthogonality (Sec. 3.2, inter-group relations): the cosine
    u_a . u_b of two VP directions or two plane normals, zero when they are
    perpendicular; angular and scale-free like Eq. 6 (a reading: the paper
    names the relation, not its residual)."""
    return dot(g.ua, g.ub)[..., None]


def res_rel_parallel(g: Gathered, rec, cx, cy):
    """Inter-group parallelism (Sec. 3.2): the 3-vector u_a x u_b, whose norm
    is |sin| of the angle; zero for parallel or opposite directions (a plane's
    (n, w) and (-n, -w) are one plane), the same vector form as R5."""
    return cross(g.ua, g.ub)


# family name -> (residual fn, rows, [(block type, index key, dof)]); the key also names
# the block in jacobians() and Gathered.perturb
FAMILIES = {
    "R1": (res_point, 2, [("cam", "cam", 9), ("pt", "pt", 3)]),
    "R2": (res_line, 4, [("cam", "cam", 9), ("ln", "ln", 4)]),
    "R3": (res_plane_point, 2, [("cam", "cam", 9), ("pt", "pt", 3), ("pl", "pl", 3)]),
    "R4": (res_plane_line, 4, [("cam", "cam", 9), ("ln", "ln", 4), ("pl", "pl", 3)]),
    "R5": (res_vp_line, 3, [("ln", "ln", 4), ("vp", "vp", 2)]),
    "R6": (res_point_to_line, 1, [("cam", "cam", 9), ("pt", "pt", 3)]),
    "R7": (res_line_to_point, 1, [("cam", "cam", 9), ("ln", "ln", 4)]),
    "R8": (res_rel_ortho, 1, [("vp", "ga", 2), ("vp", "gb", 2)]),        # VP _|_ VP
    "R9": (res_rel_parallel, 3, [("vp", "ga", 2), ("vp", "gb", 2)]),     # VP || VP
    "R10": (res_rel_ortho, 1, [("pl", "ga", 3), ("pl", "gb", 3)]),       # plane _|_ plane
    "R11": (res_rel_parallel, 3, [("pl", "ga", 3), ("pl", "gb", 3)]),    # plane || plane
    "R12": (res_plane_point_3d, 1, [("pt", "pt", 3), ("pl", "pl", 3)]),  # 3D point-to-plane
    "R13": (res_shape_point, 2, [("cam", "cam", 9), ("pt", "pt", 3), ("sh", "sh", 9)]),  # point on a shape
    "R14": (res_shape_line, 4, [("cam", "cam", 9), ("ln", "ln", 4), ("sh", "sh", 9)]),  # line on a cuboid
}
FAMILY_ORDER = ["R1", "R2", "R3", "R4", "R5", "R6", "R7", "R8", "R9", "R10", "R11", "R12", "R13", "R14"]
RELATION_FAMILIES = ("R8", "R9", "R10", "R11")
PIXEL_FAMILIES = ("R1", "R2", "R3", "R4", "R6", "R7", "R13", "R14")  # R5 and the relations are angular (Sec. 3.5)


def gather(state, rec, fam):
    blocks = FAMILIES[fam][2]
    if fam in RELATION_FAMILIES:
        return Gathered(state, rel=(blocks[0][0], rec["ga"], rec["gb"]))
    kw = {b: rec[key] for b, key, _ in blocks}
    return Gathered(state, **kw)


def residuals(state, rec, fam, cx, cy):
    fn = FAMILIES[fam][0]
    if len(next(iter(rec.values()))) == 0:
        return np.zeros((0, FAMILIES[fam][1]))
    return np.real(fn(gather(state, rec, fam), rec, cx, cy))


# Nearly degenerate image lines.  At a line through a camera's centre, or one
# lying in its principal plane, the image line has no direction: rho of Eq. 4
# and the distances of Eqs. 8 and 12 stay bounded there, and their derivatives
# grow like the inverse of the image-line normal.  The oracle differentiates
# the residuals exactly at every configuration; the functions below only
# measure how close a record is to that case (a diagnostic the solver reports).
DEGENERATE_IMAGE_LINE = 1e-3


def image_line_normal(R, t, d, m):
    """|(m_c,x, m_c,y)| / (|m| + |t| |d|), the normal of the image line of
    (d, m) relative to a bound on |m_c|; zero for a line through the camera
    centre or in its principal plane.  Real inputs."""
    dc = matvec(R, d)
    mc = matvec(R, m) + cross(t, dc)
    den = np.sqrt(dot(m, m)) + np.sqrt(dot(t, t)) * np.sqrt(dot(d, d))
    return np.sqrt(mc[..., 0] ** 2 + mc[..., 1] ** 2) / den


def line_record_normal(state, rec, fam):
    """Relative image-line normal of each record of a line-projection family
    (R2, R4, R7; +inf for the others).  For R4 the smaller of the line's and
    of its plane projection's (a record whose projection is undefined is zero
    already and keeps +inf for the projection)."""
    n = len(next(iter(rec.values())))
    if fam not in ("R2", "R4", "R7") or n == 0:
        return np.full(n, np.inf)
    R, t = state.cam_R[rec["cam"]], state.cam_t[rec["cam"]]
    d, m = line_plucker(state.line_U[rec["ln"]], state.line_w[rec["ln"]])
    rel = image_line_normal(R, t, d, m)
    if fam == "R4":
        n_, w_ = state.pl_n[rec["pl"]], state.pl_w[rec["pl"]]
        d2, m2 = plane_project_line(d, m, n_, w_)
        ok = dot(d2, d2) >= 1e-12 * dot(d, d)
        d2 = np.where(ok[:, None], d2, d)
        m2 = np.where(ok[:, None], m2, m)
        rel = np.minimum(rel, np.where(ok, image_line_normal(R, t, d2, m2), np.inf))
    return rel


def degenerate_line_records(state, rec, fam):
    """Mask of the line-projection records whose relative image-line normal
    is below DEGENERATE_IMAGE_LINE (diagnostic only)."""
    return line_record_normal(state, rec, fam) < DEGENERATE_IMAGE_LINE


def jacobians(state, rec, fam, cx, cy, camera_dof=9, h=1e-30):
    """Complex-step Jacobians of a family w.r.t. each of its parameter blocks.

    Returns {block: (n, rows, dof)}.  The tangent step is first order, which
    is all a derivative at zero sees; the result is the exact derivative of
    the residual up to rounding, at every configuration."""
    fn, rows, blocks = FAMILIES[fam]
    n = len(next(iter(rec.values())))
    out = {}
    for b, key, dof in blocks:
        if b == "cam":
            dof = camera_dof
        J = np.zeros((n, rows, dof))
        for k in range(dof):
            g = gather(state, rec, fam)
            g.perturb(key, k, 1j * h)
            J[:, :, k] = np.imag(fn(g, rec, cx, cy)) / h
        out[key] = J
    return out


# ---------------------------------------------------------------------------
# robust losses (w rho(s), s = |r|^2) and their derivatives
# ---------------------------------------------------------------------------
def loss_rho(kind, scale, s):
    if kind == 0:
        return s, np.ones_like(s)
    if kind == 1:  # Huber
        d2 = scale * scale
        big = s > d2
        ss = np.sqrt(np.maximum(s, 1e-300))
        return np.where(big, 2.0 * scale * ss - d2, s), np.where(big, scale / ss, 1.0)
    if kind == 2:  # Cauchy
        c2 = scale * scale
        return c2 * np.log1p(s / c2), 1.0 / (1.0 + s / c2)
    raise ValueError(kind)
