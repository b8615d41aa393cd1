"""Surface groups beyond planes and vanishing directions (App. B, the table of
supported group types and the paragraphs after it): sphere, cylinder, cone,
ellipsoid and cuboid.  Their parameters, tangent updates, and the projection of
a 3D point (every type) and of a 3D line (cuboid) onto the surface, in plain
FP64 numpy.  Test infrastructure: the definition the GPU path is checked
against; nothing of the product path imports it.

Every function that takes gathered (per-record) parameters is written with
complex-analytic operations only, like ``oracle.model``, so complex-step
differentiation gives its exact derivative.  The cuboid's face choice is a
discrete decision taken on the real parts (the current parameters) and held
fixed by the derivative.

Readings (the paper states each projection in words; where it leaves a detail
open, the choice made here):

* Each shape is one block of SHAPE_DOF = 9 tangent coordinates on the A side
  (cameras + groups).  A type with fewer degrees of freedom (sphere 4,
  cylinder 5, cone 6; ellipsoid and cuboid 9) leaves the rest unused: their
  Jacobian columns are zero, their damped diagonal is lambda * 1e-6 (the clip of
  an all-zero diagonal entry) and their step is zero.
* Positive quantities live in log space (the table's caption): radius of sphere
  and cylinder, the cone's half-angle, the ellipsoid's semi-axes.
* sphere (c, log r), tangent (dc, d log r): P = c + r (X - c) / |X - c|.
* cylinder: the axis in the orthonormal Pluecker form of the lines (U in
  SO(3), (w1, w2) on the unit circle; axis direction u1, foot of the
  perpendicular from the origin (w2 / w1) u3) and log r; tangent (dtheta with
  U <- U Exp(dtheta), dphi rotating (w1, w2), d log r).  P keeps X's position
  along the axis and puts it at distance r from the axis, radially.
* cone (apex A, unit axis d, log alpha), tangent (dA, dd in the sphere chart of
  the plane normals, d log alpha): with v = X - A and e the unit direction of
  v's part orthogonal to d, the generatrix in the half-plane through the axis
  and X has direction g = cos(alpha) d + sin(alpha) e, and P = A + (v . g) g,
  the foot of X on that (infinite) generatrix line.
* ellipsoid (R, c, log s), local frame y = R^T (X - c), tangent (dtheta with
  R <- R Exp(dtheta), dc, d log s): P = c + R (s * z / |z|), z = y / s
  (elementwise; the scaled-radial projection).
* cuboid (R, e_0 .. e_5), tangent (dtheta, de): face i has the outward normal
  n_i = (-1)^i R e_{floor(i/2)} and is the plane n_i . x + e_i = 0 (the plane
  convention of the planes).  A point goes to the face of smallest
  |n_i . X + e_i| (lowest index on ties): P = X - (n_i . X + e_i) n_i.  A line
  goes through the point p of the line closest to the cuboid's centre
  c = R m, m_k = (e_{2k+1} - e_{2k}) / 2: the face of smallest |n_i . p + e_i|
  is chosen and the line is projected onto that face's plane with the plane-line
  projection of the planes.
"""
from __future__ import annotations

import numpy as np

from .model import cross, dot, matvec, skew, so3_exp, s2_basis, s2_retract, line_from_points, line_plucker

SPHERE, CYLINDER, CONE, ELLIPSOID, CUBOID = range(5)
SHAPE_DOF = 9
# degrees of freedom per type (App. B, the table of group types)
TYPE_DOF = {SPHERE: 4, CYLINDER: 5, CONE: 6, ELLIPSOID: 9, CUBOID: 9}
ABI_PARAMS = 16


class Shapes:
    """FP64 parameters of the shapes of a scene, one row per shape.

    type (n,); R (n, 3, 3): U of the cylinder's axis, the ellipsoid's and the
    cuboid's rotation, identity otherwise; w (n, 2): the cylinder's (w1, w2);
    c (n, 3): sphere centre, cone apex, ellipsoid centre; d (n, 3): cone axis
    (e_z for the other types); q (n, 6): log r (sphere, cylinder), log alpha
    (cone), log s (ellipsoid, 3), e (cuboid, 6)."""

    def __init__(self, type_, R, w, c, d, q):
        self.type, self.R, self.w, self.c, self.d, self.q = type_, R, w, c, d, q

    @staticmethod
    def empty():
        return Shapes(np.zeros(0, np.int64), np.zeros((0, 3, 3)), np.zeros((0, 2)), np.zeros((0, 3)),
                      np.zeros((0, 3)), np.zeros((0, 6)))

    def __len__(self):
        return len(self.type)

    def copy(self):
        return Shapes(*(a.copy() for a in (self.type, self.R, self.w, self.c, self.d, self.q)))

    @staticmethod
    def from_abi(types, params):
        """From the C-ABI input format (16 doubles per shape):
        sphere (c, r); cylinder (axis direction, a point on the axis, r); cone
        (apex, axis direction, alpha); ellipsoid (R row-major, c, s); cuboid
        (R row-major, e_0 .. e_5)."""
        t = np.asarray(types, np.int64).reshape(-1)
        p = np.asarray(params, np.float64).reshape(-1, ABI_PARAMS)
        n = len(t)
        s = Shapes(t.copy(), np.tile(np.eye(3), (n, 1, 1)), np.tile([1.0, 0.0], (n, 1)), np.zeros((n, 3)),
                   np.tile([0.0, 0.0, 1.0], (n, 1)), np.zeros((n, 6)))
        for i in range(n):
            k = t[i]
            if k == SPHERE:
                s.c[i] = p[i, 0:3]
                s.q[i, 0] = np.log(p[i, 3])
            elif k == CYLINDER:
                d = p[i, 0:3] / np.linalg.norm(p[i, 0:3])
                U, w = line_from_points(p[i, 3:6], p[i, 3:6] + d)
                s.R[i], s.w[i] = U, w
                s.q[i, 0] = np.log(p[i, 6])
            elif k == CONE:
                s.c[i] = p[i, 0:3]
                s.d[i] = p[i, 3:6] / np.linalg.norm(p[i, 3:6])
                s.q[i, 0] = np.log(p[i, 6])
            elif k == ELLIPSOID:
                s.R[i] = p[i, 0:9].reshape(3, 3)
                s.c[i] = p[i, 9:12]
                s.q[i, 0:3] = np.log(p[i, 12:15])
            elif k == CUBOID:
                s.R[i] = p[i, 0:9].reshape(3, 3)
                s.q[i, 0:6] = p[i, 9:15]
            else:
                raise ValueError(f"shape type {k}")
        return s

    def to_abi(self):
        """(types, params (n, 16)) in the input format; a cylinder's axis is given
        by its unit direction and the foot of the perpendicular from the origin."""
        n = len(self)
        p = np.zeros((n, ABI_PARAMS))
        for i in range(n):
            k = self.type[i]
            if k == SPHERE:
                p[i, 0:3], p[i, 3] = self.c[i], np.exp(self.q[i, 0])
            elif k == CYLINDER:
                u1, u3 = self.R[i][:, 0], self.R[i][:, 2]
                p[i, 0:3] = u1
                p[i, 3:6] = (self.w[i, 1] / self.w[i, 0]) * u3
                p[i, 6] = np.exp(self.q[i, 0])
            elif k == CONE:
                p[i, 0:3], p[i, 3:6], p[i, 6] = self.c[i], self.d[i], np.exp(self.q[i, 0])
            elif k == ELLIPSOID:
                p[i, 0:9], p[i, 9:12], p[i, 12:15] = self.R[i].ravel(), self.c[i], np.exp(self.q[i, 0:3])
            else:
                p[i, 0:9], p[i, 9:15] = self.R[i].ravel(), self.q[i, 0:6]
        return self.type.copy(), p

    def retract(self, dsh):
        """x [+] h for every shape (the tangent updates of the module docstring)."""
        out = self.copy()
        if not len(self):
            return out
        h = np.asarray(dsh, np.float64).reshape(-1, SHAPE_DOF)
        for i in range(len(self)):
            k = self.type[i]
            if k == SPHERE:
                out.c[i] = self.c[i] + h[i, 0:3]
                out.q[i, 0] = self.q[i, 0] + h[i, 3]
            elif k == CYLINDER:
                out.R[i] = self.R[i] @ so3_exp(h[i, 0:3])
                c, s = np.cos(h[i, 3]), np.sin(h[i, 3])
                w1, w2 = self.w[i]
                out.w[i] = [w1 * c - w2 * s, w1 * s + w2 * c]
                out.q[i, 0] = self.q[i, 0] + h[i, 4]
            elif k == CONE:
                out.c[i] = self.c[i] + h[i, 0:3]
                out.d[i] = s2_retract(self.d[i][None], h[i, 3:5][None])[0]
                out.q[i, 0] = self.q[i, 0] + h[i, 5]
            elif k == ELLIPSOID:
                out.R[i] = self.R[i] @ so3_exp(h[i, 0:3])
                out.c[i] = self.c[i] + h[i, 3:6]
                out.q[i, 0:3] = self.q[i, 0:3] + h[i, 6:9]
            else:
                out.R[i] = self.R[i] @ so3_exp(h[i, 0:3])
                out.q[i, 0:6] = self.q[i, 0:6] + h[i, 3:9]
        return out


class GatheredShapes:
    """Per-record complex copies of the shape parameters, with first-order tangent
    perturbation."""

    def __init__(self, sh: Shapes, idx):
        c = np.complex128
        self.type = sh.type[idx]
        self.R, self.w, self.c = sh.R[idx].astype(c), sh.w[idx].astype(c), sh.c[idx].astype(c)
        self.d, self.q = sh.d[idx].astype(c), sh.q[idx].astype(c)
        self.Bd = s2_basis(sh.d[idx])

    def perturb(self, k, h):
        """Step h along tangent coordinate k of each record's shape (in place)."""
        t = self.type
        n = len(t)
        e = np.zeros(3, dtype=np.complex128)
        if k < 3:
            e[k] = h
        rot = np.where(np.isin(t, (CYLINDER, ELLIPSOID, CUBOID)), k < 3, False)
        Sk = np.eye(3) + skew(e)
        self.R = np.where(rot[:, None, None], self.R @ Sk, self.R)
        dc = np.zeros((n, 3), dtype=np.complex128)
        dq = np.zeros((n, 6), dtype=np.complex128)
        dd = np.zeros((n, 3), dtype=np.complex128)
        sph, cyl, con, ell, cub = (t == s for s in (SPHERE, CYLINDER, CONE, ELLIPSOID, CUBOID))
        if k < 3:
            dc[sph | con, k] = h
        if k == 3:
            dq[sph, 0] = h
        if k in (3, 4):
            dd[con] = h * self.Bd[con][:, :, k - 3]
        if k == 5:
            dq[con, 0] = h
        if 3 <= k < 6:
            dc[ell, k - 3] = h
        if k >= 6:
            dq[ell, k - 6] = h
        if k >= 3:
            dq[cub, k - 3] = h
        if k == 4:
            dq[cyl, 0] = h
        if k == 3:
            w1, w2 = self.w[:, 0], self.w[:, 1]
            self.w = np.where(cyl[:, None], np.stack([w1 - h * w2, w2 + h * w1], axis=-1), self.w)
        self.c = self.c + dc
        self.q = self.q + dq
        self.d = self.d + dd


def _proj_sphere(X, c, q):
    u = X - c
    n = np.sqrt(dot(u, u))[..., None]
    return c + np.exp(q[..., 0:1]) * u / n


def _proj_cylinder(X, U, w, q):
    a = U[..., :, 0]
    p0 = (w[..., 1] / w[..., 0])[..., None] * U[..., :, 2]
    v = X - p0
    h = dot(v, a)[..., None]
    qv = v - h * a
    rho = np.sqrt(dot(qv, qv))[..., None]
    return p0 + h * a + np.exp(q[..., 0:1]) * qv / rho


def _proj_cone(X, A, d, q):
    v = X - A
    h = dot(v, d)[..., None]
    qv = v - h * d
    e = qv / np.sqrt(dot(qv, qv))[..., None]
    al = np.exp(q[..., 0:1])
    g = np.cos(al) * d + np.sin(al) * e
    return A + dot(v, g)[..., None] * g


def _proj_ellipsoid(X, R, c, q):
    s = np.exp(q[..., 0:3])
    y = np.einsum("...ji,...j->...i", R, X - c)   # R^T (X - c)
    z = y / s
    zn = z / np.sqrt(dot(z, z))[..., None]
    return c + matvec(R, s * zn)


def cuboid_faces(R, q):
    """Face normals n (..., 6, 3) and offsets e (..., 6)."""
    sign = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    axis = np.array([0, 0, 1, 1, 2, 2])
    n = sign[None, :, None] * np.swapaxes(R[..., :, axis], -1, -2)
    return n, q[..., 0:6]


def cuboid_centre(R, q):
    m = 0.5 * (q[..., [1, 3, 5]] - q[..., [0, 2, 4]])
    return matvec(R, m)


def cuboid_face_of_point(R, q, X):
    """Index of the face of smallest |n_i . X + e_i| (real inputs; lowest index on ties)."""
    n, e = cuboid_faces(np.real(R), np.real(q))
    s = np.einsum("...ij,...j->...i", n, np.real(X)) + e
    return np.argmin(np.abs(s), axis=-1)


def _proj_cuboid(X, R, q):
    i = cuboid_face_of_point(R, q, X)
    n, e = cuboid_faces(R, q)
    r = np.arange(len(i))
    ni, ei = n[r, i], e[r, i]
    return X - (dot(ni, X) + ei)[..., None] * ni


def project_point(g: GatheredShapes, X):
    """Proj_G(X) for each record's shape (App. B)."""
    P = np.zeros_like(X, dtype=np.complex128)
    t = g.type
    for k, fn in ((SPHERE, lambda m: _proj_sphere(X[m], g.c[m], g.q[m])),
                  (CYLINDER, lambda m: _proj_cylinder(X[m], g.R[m], g.w[m], g.q[m])),
                  (CONE, lambda m: _proj_cone(X[m], g.c[m], g.d[m], g.q[m])),
                  (ELLIPSOID, lambda m: _proj_ellipsoid(X[m], g.R[m], g.c[m], g.q[m])),
                  (CUBOID, lambda m: _proj_cuboid(X[m], g.R[m], g.q[m]))):
        m = t == k
        if m.any():
            P[m] = fn(m)
    return P


def cuboid_face_of_line(R, q, d, m):
    """Face chosen for a line (d, m) (real inputs): the one nearest to the point of
    the line closest to the cuboid's centre."""
    R, q, d, m = (np.real(a) for a in (R, q, d, m))
    dd = dot(d, d)[..., None]
    p0 = cross(d, m) / dd
    c = cuboid_centre(R, q)
    p = p0 + (dot(c - p0, d)[..., None] / dd) * d
    return cuboid_face_of_point(R, q, p)


def cuboid_line_plane(g: GatheredShapes, d, m):
    """(n, w) of the face plane each record's line is projected onto."""
    i = cuboid_face_of_line(g.R, g.q, d, m)
    n, e = cuboid_faces(g.R, g.q)
    r = np.arange(len(i))
    return n[r, i], e[r, i]


def similarity(sh: Shapes, s, Q, tau):
    """The shapes moved by x -> s Q x + tau (a similarity of the whole scene)."""
    out = sh.copy()
    for i in range(len(sh)):
        k = sh.type[i]
        if k in (SPHERE, CONE, ELLIPSOID):
            out.c[i] = s * Q @ sh.c[i] + tau
        if k == CONE:
            out.d[i] = Q @ sh.d[i]
        if k in (SPHERE, CYLINDER):
            out.q[i, 0] = sh.q[i, 0] + np.log(s)
        if k == ELLIPSOID:
            out.R[i] = Q @ sh.R[i]
            out.q[i, 0:3] = sh.q[i, 0:3] + np.log(s)
        if k == CYLINDER:
            U = sh.R[i]
            d, m = line_plucker(U[None], sh.w[i][None])
            p0 = (cross(d, m) / dot(d, d)[..., None])[0]
            a = Q @ U[:, 0]
            U2, w2 = line_from_points(s * Q @ p0 + tau, s * Q @ p0 + tau + a)
            out.R[i], out.w[i] = U2, w2
        if k == CUBOID:
            out.R[i] = Q @ sh.R[i]
            n, e = cuboid_faces(out.R[i][None], sh.q[i][None])
            out.q[i, 0:6] = s * sh.q[i, 0:6] - (n[0] @ tau)
    return out


def _ambient(sh: Shapes):
    """Every stored parameter of each shape, flattened (n, 23)."""
    n = len(sh)
    return np.concatenate([sh.R.reshape(n, 9), sh.w, sh.c, sh.d, sh.q], axis=1)


def gauge_rows(sh: Shapes, eps=1e-6):
    """(n, 9, 7): the tangent-coordinate motion of each shape under the world's
    rotations about e_0..e_2, translations along e_0..e_2 and scale (the similarity
    gauge of the reduced system), computed numerically: central differences of
    `similarity` in the stored parameters, solved for the tangent step in the
    differential of `Shapes.retract` (least squares over the type's own coordinates).
    Also returns the largest relative residual of those solves (zero when the motion
    lies in the shape's tangent space)."""
    n = len(sh)
    out = np.zeros((n, SHAPE_DOF, 7))
    if n == 0:
        return out, 0.0
    A = np.zeros((n, _ambient(sh).shape[1], SHAPE_DOF))
    for k in range(SHAPE_DOF):
        h = np.zeros((n, SHAPE_DOF))
        h[:, k] = eps
        A[:, :, k] = (_ambient(sh.retract(h)) - _ambient(sh.retract(-h))) / (2 * eps)
    E3 = np.eye(3)

    def moved(c, e):
        if c < 3:
            return similarity(sh, 1.0, so3_exp(e * E3[c]), np.zeros(3))
        if c < 6:
            return similarity(sh, 1.0, np.eye(3), e * E3[c - 3])
        return similarity(sh, np.exp(e), np.eye(3), np.zeros(3))

    worst = 0.0
    for c in range(7):
        b = (_ambient(moved(c, eps)) - _ambient(moved(c, -eps))) / (2 * eps)
        for i in range(n):
            used = TYPE_DOF[int(sh.type[i])]
            x, *_ = np.linalg.lstsq(A[i][:, :used], b[i], rcond=None)
            out[i, :used, c] = x
            worst = max(worst, np.linalg.norm(A[i][:, :used] @ x - b[i]) / max(np.linalg.norm(b[i]), 1e-12))
    return out, worst
