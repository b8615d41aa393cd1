"""Linearisation, Schur elimination and the Levenberg-Marquardt iteration in FP64.

Written from the paper's Section 3.1 (normal equations Eq. 2 and Schur
complement Eq. 3), Section 3.2 (augmented set A = cameras + groups, block-
diagonal feature Hessian H_ff, Eq. 5) and Section 3.5 (termination on the
relative change of the pixel-space cost only).  The damping, gain-ratio and
lambda schedule are not given in the paper (Ceres is named as the solver);
the readings used are:

* cost E = 1/2 sum_r w_r rho_r(|r_r|^2); E_pix is the same sum without the
  angular VP family;
* robust loss by iteratively reweighted least squares: r~ = sqrt(w rho') r
  and J~ = sqrt(w rho') J, so that g = J~^T r~ is the exact gradient and the
  Gauss-Newton matrix is H = J~^T J~;
* Marquardt damping H + lambda diag(D), D = clip(diag H, 1e-6, 1e32);
* model decrease L(0) - L(h) = -h.g - 1/2 |J~ h|^2, gain ratio
  rho = (E(x) - E(x [+] h)) / (L(0) - L(h)); accept when rho > 0 with
  lambda <- lambda max(1/3, 1 - (2 rho - 1)^3), nu <- 2, else
  lambda <- lambda nu, nu <- 2 nu (Nielsen's rule); lambda0 = 1e-4,
  lambda >= 1e-10;
* stop after an accepted step with |dE_pix| / E_pix < func_tol, or when
  |g|_inf < grad_tol, lambda > 1e16, or max_iters attempts.

The Schur complement S = U - W V^-1 W^T is formed densely with sparse
library products and solved with a dense Cholesky factorisation.  Nothing
here is blocked, fused or reordered beyond the block-diagonal structure of
V that the paper states.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import model
from .model import FAMILIES, FAMILY_ORDER, PIXEL_FAMILIES
from .records import expand, loss_of


class Problem:
    """Records, losses and the parameter layout of one scene."""

    def __init__(self, scene, camera_dof=None):
        self.scene = scene
        self.cx, self.cy = float(scene["cx"]), float(scene["cy"])
        self.camera_dof = int(camera_dof if camera_dof is not None else scene.get("camera_dof", 9))
        self.recs = expand(scene)
        self.loss = {f: loss_of(scene, f) for f in FAMILY_ORDER}
        nc, npt, nln = len(scene["cameras"]), len(scene["points"]), len(scene["lines"])
        npl, nvp = len(scene["planes"]), len(scene["vps"])
        nsh = len(scene["shapes"]["type"]) if scene.get("shapes") is not None else 0
        self.n = dict(cam=nc, pt=npt, ln=nln, pl=npl, vp=nvp, sh=nsh)
        cd = self.camera_dof
        self.dof = dict(cam=cd, pt=3, ln=4, pl=3, vp=2, sh=model.SHAPE_DOF)
        # parameter ordering: A = cameras, planes, vps, shapes ; F = points, lines
        self.off = {}
        o = 0
        for b in ("cam", "pl", "vp", "sh"):
            self.off[b] = o
            o += self.n[b] * self.dof[b]
        self.nA = o
        for b in ("pt", "ln"):
            self.off[b] = o
            o += self.n[b] * self.dof[b]
        self.nF = o - self.nA
        self.N = o

    def record_count(self, fam):
        return len(next(iter(self.recs[fam].values())))

    def state0(self):
        return model.State.from_scene(self.scene)

    def split(self, h):
        """Full step vector -> per-block arrays for State.retract."""
        out = {}
        for b in ("cam", "pl", "vp", "sh", "pt", "ln"):
            o = self.off[b]
            out[b] = h[o:o + self.n[b] * self.dof[b]]
        return out

    def retract(self, state, h):
        p = self.split(h)
        return state.retract(p["cam"], p["pt"], p["ln"], p["pl"], p["vp"], camera_dof=self.camera_dof,
                             dsh=p["sh"])


# ---------------------------------------------------------------------------
# cost
# ---------------------------------------------------------------------------
def family_cost(prob, state, fam, recs=None):
    """Per-record w rho(|r|^2) (without the factor 1/2)."""
    rec = prob.recs[fam] if recs is None else recs
    r = model.residuals(state, rec, fam, prob.cx, prob.cy)
    kind, scale, weight = prob.loss[fam]
    rho, _ = model.loss_rho(kind, scale, np.sum(r * r, axis=1))
    return weight * rho


def cost(prob, state):
    """(E, E_pix): E = 1/2 sum w rho(|r|^2), E_pix without the angular families (VP-line, relations)."""
    E = Epix = 0.0
    for fam in FAMILY_ORDER:
        if prob.record_count(fam) == 0:
            continue
        c = 0.5 * float(np.sum(family_cost(prob, state, fam)))
        E += c
        if fam in PIXEL_FAMILIES:
            Epix += c
    return E, Epix


# ---------------------------------------------------------------------------
# linearisation
# ---------------------------------------------------------------------------
class Linearization:
    pass


def linearize_family(prob, state, fam, recs=None):
    """Residuals r, IRLS scale sqrt(w rho'), weighted r~ and J~ for one family."""
    rec = prob.recs[fam] if recs is None else recs
    r = model.residuals(state, rec, fam, prob.cx, prob.cy)
    J = model.jacobians(state, rec, fam, prob.cx, prob.cy, camera_dof=prob.camera_dof)
    kind, scale, weight = prob.loss[fam]
    s = np.sum(r * r, axis=1)
    _, drho = model.loss_rho(kind, scale, s)
    ws = np.sqrt(weight * drho)
    return dict(r=r, ws=ws, rt=ws[:, None] * r, J={b: ws[:, None, None] * Jb for b, Jb in J.items()})


def linearize(prob, state):
    lin = Linearization()
    lin.fam = {}
    rows, cols, vals, rts = [], [], [], []
    row0 = 0
    for fam in FAMILY_ORDER:
        n = prob.record_count(fam)
        if n == 0:
            continue
        L = linearize_family(prob, state, fam)
        lin.fam[fam] = L
        m = FAMILIES[fam][1]
        rid = row0 + np.arange(n)[:, None] * m + np.arange(m)[None, :]  # (n, m)
        for b, key, _ in FAMILIES[fam][2]:
            dof = prob.dof[b]
            c0 = prob.off[b] + dof * prob.recs[fam][key]               # (n,)
            cc = c0[:, None, None] + np.arange(dof)[None, None, :]      # (n,1,dof)
            rr = np.broadcast_to(rid[:, :, None], (n, m, dof))
            cc = np.broadcast_to(cc, (n, m, dof))
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(L["J"][key].ravel())
        rts.append(L["rt"].ravel())
        row0 += n * m
    lin.nrows = row0
    if row0:
        lin.J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(row0, prob.N))
        lin.rt = np.concatenate(rts)
    else:
        lin.J = sp.csr_matrix((0, prob.N))
        lin.rt = np.zeros(0)
    lin.g = lin.J.T @ lin.rt
    lin.Hdiag = np.asarray(lin.J.multiply(lin.J).sum(axis=0)).ravel()
    lin.D = np.clip(lin.Hdiag, 1e-6, 1e32)
    return lin


# ---------------------------------------------------------------------------
# feature blocks and the Schur complement
# ---------------------------------------------------------------------------
def _feature_block_index(prob):
    """Per feature-column (0..nF): block id, local index, block size."""
    npt, nln = prob.n["pt"], prob.n["ln"]
    c = np.arange(prob.nF)
    is_pt = c < 3 * npt
    blk = np.where(is_pt, c // 3, npt + (c - 3 * npt) // 4)
    loc = np.where(is_pt, c % 3, (c - 3 * npt) % 4)
    return blk, loc


def feature_blocks(prob, lin):
    """V_f = sum_r J~_rf^T J~_rf per feature (the diagonal blocks of H_ff).

    Returns (Vp (npt,3,3), Vl (nln,4,4), n_offblock) where n_offblock counts
    nonzeros of H_ff outside the feature blocks (zero by Sec. 3.2)."""
    Jf = lin.J[:, prob.nA:]
    Hff = (Jf.T @ Jf).tocoo()
    blk, loc = _feature_block_index(prob)
    bi, bj = blk[Hff.row], blk[Hff.col]
    inside = bi == bj
    n_off = int(np.count_nonzero(Hff.data[~inside]))
    npt, nln = prob.n["pt"], prob.n["ln"]
    Vp = np.zeros((npt, 3, 3))
    Vl = np.zeros((nln, 4, 4))
    r, c, v, b = Hff.row[inside], Hff.col[inside], Hff.data[inside], bi[inside]
    isp = b < npt
    np.add.at(Vp, (b[isp], loc[r[isp]], loc[c[isp]]), v[isp])
    np.add.at(Vl, (b[~isp] - npt, loc[r[~isp]], loc[c[~isp]]), v[~isp])
    return Vp, Vl, n_off


def damped_feature_inverse(prob, lin, lam):
    """(V_f + lam diag(D_f))^-1 per block, assembled as a sparse matrix."""
    Vp, Vl, _ = feature_blocks(prob, lin)
    Df = lin.D[prob.nA:]
    npt, nln = prob.n["pt"], prob.n["ln"]
    Vp = Vp + lam * np.einsum("ni,ij->nij", Df[:3 * npt].reshape(npt, 3), np.eye(3))
    Vl = Vl + lam * np.einsum("ni,ij->nij", Df[3 * npt:].reshape(nln, 4), np.eye(4))
    Ip = np.linalg.inv(Vp) if npt else Vp
    Il = np.linalg.inv(Vl) if nln else Vl
    rows, cols, vals = [], [], []
    if npt:
        base = 3 * np.arange(npt)
        rows.append(np.repeat(base, 9) + np.tile(np.repeat(np.arange(3), 3), npt))
        cols.append(np.repeat(base, 9) + np.tile(np.tile(np.arange(3), 3), npt))
        vals.append(Ip.ravel())
    if nln:
        base = 3 * npt + 4 * np.arange(nln)
        rows.append(np.repeat(base, 16) + np.tile(np.repeat(np.arange(4), 4), nln))
        cols.append(np.repeat(base, 16) + np.tile(np.tile(np.arange(4), 4), nln))
        vals.append(Il.ravel())
    if rows:
        Vinv = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(prob.nF, prob.nF))
    else:
        Vinv = sp.csr_matrix((prob.nF, prob.nF))
    return Vinv, (Vp, Vl)


def schur_terms(prob, lin, lam):
    """Sparse terms of the reduced system of Sec. 3.1 Eq. 3 over A = cameras
    + groups: U = J_a^T J_a, W = J_a^T J_f, (V + lam D_f)^-1, the elimination
    term W V^-1 W^T and b = -g_a + W V^-1 g_f."""
    nA = prob.nA
    Ja = lin.J[:, :nA]
    Jf = lin.J[:, nA:]
    U = (Ja.T @ Ja).tocsr()
    W = (Ja.T @ Jf).tocsr()
    Vinv, _ = damped_feature_inverse(prob, lin, lam)
    WV = W @ Vinv
    WVW = (WV @ W.T).tocsr()
    ga, gf = lin.g[:nA], lin.g[nA:]
    b = -ga + WV @ gf
    return dict(U=U, W=W, Vinv=Vinv, WVW=WVW, b=b)


def schur(prob, lin, lam):
    """Reduced system S = U + lam diag(D_a) - W V_lam^-1 W^T (dense) and b."""
    t = schur_terms(prob, lin, lam)
    U = t["U"].toarray() + lam * np.diag(lin.D[:prob.nA])
    S = U - t["WVW"].toarray()
    return dict(S=S, b=t["b"], W=t["W"], Vinv=t["Vinv"], U=U)


def cholesky_solve(S, b):
    """x = S^-1 b for symmetric positive definite S by a dense Cholesky
    factorisation and two triangular solves; None when S is not positive
    definite."""
    import scipy.linalg
    try:
        c = scipy.linalg.cho_factor(S, lower=True, check_finite=False)
    except np.linalg.LinAlgError:
        return None
    return scipy.linalg.cho_solve(c, b, check_finite=False)


def solve_schur(prob, lin, lam):
    """Step h = (h_a, h_f) by dense Cholesky of S and back-substitution
    h_f = V^-1 (-g_f - W^T h_a).  Returns None when S is not positive definite."""
    sys_ = schur(prob, lin, lam)
    ha = cholesky_solve(sys_["S"], sys_["b"])
    if ha is None:
        return None, sys_
    gf = lin.g[prob.nA:]
    hf = sys_["Vinv"] @ (-gf - sys_["W"].T @ ha)
    return np.concatenate([ha, hf]), sys_


def solve_features(prob, lin, lam):
    """Step with the A side held fixed (h_a = 0): each feature alone,
    h_f = -(V_f + lam diag(D_f))^-1 g_f (the fixed-pose refinement of App. A.2)."""
    Vinv, _ = damped_feature_inverse(prob, lin, lam)
    hf = Vinv @ (-lin.g[prob.nA:])
    return np.concatenate([np.zeros(prob.nA), hf])


def solve_full(prob, lin, lam):
    """Step from the full damped normal equations (H + lam diag D) h = -g, dense."""
    H = (lin.J.T @ lin.J).toarray() + lam * np.diag(lin.D)
    return np.linalg.solve(H, -lin.g)


def model_decrease(lin, h):
    Jh = lin.J @ h
    return float(-h @ lin.g - 0.5 * Jh @ Jh)


def diag_blocks(prob, M):
    """Diagonal blocks of an A x A matrix: cameras, planes, vps, shapes."""
    out = {}
    for b in ("cam", "pl", "vp", "sh"):
        d, o, n = prob.dof[b], prob.off[b], prob.n[b]
        out[b] = np.stack([M[o + i * d:o + (i + 1) * d, o + i * d:o + (i + 1) * d] for i in range(n)]) \
            if n else np.zeros((0, d, d))
    return out


# ---------------------------------------------------------------------------
# Levenberg-Marquardt
# ---------------------------------------------------------------------------
def lm_solve(prob, state=None, max_iters=100, func_tol=1e-6, grad_tol=1e-10, lambda0=1e-4, nu0=2.0,
             lambda_min=1e-10, lambda_max=1e16, verbose=False, fixed_a=False):
    """LM as above; with fixed_a the cameras and groups are held fixed and only the
    features move (solve_features instead of the Schur step)."""
    state = prob.state0() if state is None else state
    E, Epix = cost(prob, state)
    lam, nu = lambda0, nu0
    lin = linearize(prob, state)
    hist = [dict(iter=0, E=E, Epix=Epix, lam=lam, accepted=True)]
    reason = "max_iters"
    n_acc = 0
    for it in range(1, max_iters + 1):
        if np.max(np.abs(lin.g)) < grad_tol:
            reason = "grad_tol"
            break
        h = solve_features(prob, lin, lam) if fixed_a else solve_schur(prob, lin, lam)[0]
        accepted = False
        rel = None
        if h is not None:
            new = prob.retract(state, h)
            En, Epn = cost(prob, new)
            dL = model_decrease(lin, h)
            rho = (E - En) / dL if dL > 0 else -np.inf
            if np.isfinite(En) and rho > 0:
                accepted = True
                n_acc += 1
                rel = abs(Epix - Epn) / max(Epix, 1e-300)
                state, E, Epix = new, En, Epn
                lam = max(lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3), lambda_min)
                nu = nu0
        if not accepted:
            lam, nu = lam * nu, nu * 2.0
        hist.append(dict(iter=it, E=E, Epix=Epix, lam=lam, accepted=accepted))
        if verbose:
            print(it, E, Epix, lam, accepted)
        if accepted:
            if rel < func_tol:
                reason = "func_tol"
                break
            lin = linearize(prob, state)
        if lam > lambda_max:
            reason = "lambda_max"
            break
    return dict(state=state, E=E, Epix=Epix, iters=len(hist) - 1, accepted=n_acc, reason=reason,
                history=hist, lam=lam, nu=nu)
