"""FP64 reference of the learned coarse-space correction (test infrastructure).

The paper solves the reduced camera + group system by CG preconditioned
with the inverses of its diagonal blocks.  The coarse-space correction is
this project's addition to that method.  Its coarse basis has two parts:

* G (n_A x 7): the similarity gauge of the reduced parameters - the first-
  order change of every camera, plane and VP under a world rotation (3),
  translation (3) and scale (1), in the solver's tangent coordinates.  The
  cost is invariant under these motions, so J [G; G_features] = 0 and the
  undamped reduced matrix annihilates G: these are the slowest modes of the
  damped system (eigenvalues of order lambda after block normalisation).
* Z_net (n_A x 8): vectors predicted by a small message-passing network
  over the block graph, trained to span the next slowest modes.

With Z = [G, Z_net], E = Z^T S Z, Q = Z E^-1 Z^T and M = blockdiag(S_ii)^-1,
PCG starts from x0 = Q b and uses the two-level preconditioner
    P r = (I - Q S) M r + Q r
(the "A-DEF2" form: deflation of span(Z) applied after block-Jacobi), with
M alone when E is not positive definite.

This module is a plain PyTorch-CPU float64 implementation of every
definition below; gradients come from autograd and are checked against
central differences in the tests.  It is used only by the tests, the
smoke check and the CPU baseline.

Definitions (written independently by the HIP kernels):

* gauge: camera (left perturbation R <- Exp(dtheta) R, t <- Exp(dtheta) t
  + dt): rotation w: dtheta = -R w, dt = (R w) x t; translation u: dt = -R u;
  scale s: dt = s t.  Plane (n, w), tangent (b1, b2, w): rotation w:
  (b1, b2) . (w x n); translation u: dw = -n . u; scale s: dw = s w.  VP v:
  rotation w: (b1, b2) . (w x v).  Columns: rotation about x, y, z,
  translation along x, y, z, scale;
* graph: one node per block of the reduced system, cameras first, then
  planes, then VPs (the order of the reduced vector); a directed edge j -> i
  for every ordered pair of distinct blocks that share a feature (a point or
  line with records touching both); edges sorted by destination, then source;
* scene scale s0: RMS distance of the input camera centres -R^T t from
  their mean (1 when that is zero or there are no cameras);
* node input x_i (64): [0, n) log(u_p^2 S_pp) - mean_p log(u_p^2 S_pp) of the
  damped block S_ii (u_i the unit scales below, so that the inputs do not
  change when the whole scene is scaled); from 9, the strictly lower
  correlations S_pq / sqrt(S_pp S_qq) row by row; 45 log(lambda);
  46 log(1 + records touching the block); 47 log(1 + in-degree);
  48 + type: 1; geometry from 51: camera R row-major (9) then t / s0 (3);
  plane n (3), w / s0, b1 (3), b2 (3); VP v (3), b1 (3), b2 (3), with
  (b1, b2) the tangent basis of the parameter's sphere;
* edge input e_ji (8): log(1 + shared features), then one-hot
  camera-camera / camera-plane / camera-VP / group-group, then zeros;
* network, hidden width H = 64,
  gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))):
    h = gelu(x W_in + b_in)
    3 times:  m_i = mean over edges j -> i of gelu([h_j, e_ji] W_e + b_e)
              h = gelu(h W_s + b_s + m) + h
    Y_i = h_i W_t + b_t for the node's type t, read as an n_t x K matrix
    (row-major);
* Z_net,i = diag(u_i) Y_i with unit scales u: camera (1,1,1, s0,s0,s0,
  1,1,1) (rotation, translation, intrinsics), plane (1, 1, s0), VP (1, 1);
* training loss, per system: tr((Z^T D Z)^-1 Z^T S Z) with Z = [G, Z_net]
  and D = blockdiag(S_ii) (the sum of the Ritz values of the block-
  normalised S on span(Z), smallest when Z spans its 15 slowest
  directions); a batch takes the mean over its systems.
"""
from __future__ import annotations

import math

import numpy as np
import torch

H = 64
NODE_IN = 64
EDGE_IN = 8
LAYERS = 3
K = 8          # network columns
K_GAUGE = 7    # analytic gauge columns
TYPE_CAM, TYPE_PLANE, TYPE_VP = 0, 1, 2


def block_sizes(camera_dof):
    return {TYPE_CAM: camera_dof, TYPE_PLANE: 3, TYPE_VP: 2}


def param_shapes(camera_dof=9):
    """Ordered (name, shape) list of the parameter blob (float32, row-major)."""
    shapes = [("W_in", (NODE_IN, H)), ("b_in", (H,))]
    for l in range(LAYERS):
        shapes += [(f"W_e{l}", (H + EDGE_IN, H)), (f"b_e{l}", (H,)), (f"W_s{l}", (H, H)), (f"b_s{l}", (H,))]
    for t, n in block_sizes(camera_dof).items():
        shapes += [(f"W_t{t}", (H, n * K)), (f"b_t{t}", (n * K,))]
    return shapes


def param_count(camera_dof=9):
    return int(sum(np.prod(s) for _, s in param_shapes(camera_dof)))


def init_params(camera_dof=9, seed=0):
    """Gaussian weights with variance 1 / fan-in, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes(camera_dof):
        p[name] = np.zeros(shp) if name.startswith("b") else rng.normal(size=shp) * math.sqrt(1.0 / shp[0])
    return p


def pack(params, camera_dof=9):
    return np.concatenate([np.asarray(params[name], dtype=np.float32).ravel()
                           for name, _ in param_shapes(camera_dof)])


def unpack(blob, camera_dof=9):
    v = np.frombuffer(blob, dtype=np.float32) if isinstance(blob, (bytes, bytearray)) else np.asarray(blob)
    out, o = {}, 0
    for name, shp in param_shapes(camera_dof):
        n = int(np.prod(shp))
        out[name] = v[o:o + n].astype(np.float64).reshape(shp)
        o += n
    assert o == len(v)
    return out


# ---------------------------------------------------------------------------
# graph and inputs
# ---------------------------------------------------------------------------
def scene_scale(cameras):
    """RMS distance of the camera centres -R^T t from their mean (1 if zero)."""
    from scenegen import quaternion_to_matrix  # input format conversion only
    cams = np.asarray(cameras, dtype=np.float64).reshape(-1, 10)
    if len(cams) == 0:
        return 1.0
    R = quaternion_to_matrix(cams[:, 0:4])
    c = -np.einsum("nji,nj->ni", R, cams[:, 4:7])
    s = math.sqrt(float(np.mean(np.sum((c - c.mean(axis=0)) ** 2, axis=1))))
    return s if s > 0 and math.isfinite(s) else 1.0


def gauge_basis(prob, state):
    """G (n_A x 7): first-order motion of the reduced parameters under a world
    rotation (3), translation (3) and scale (1)."""
    from oracle.model import s2_basis
    cd = prob.camera_dof
    nc, npl, nvp = prob.n["cam"], prob.n["pl"], prob.n["vp"]
    G = np.zeros((prob.nA, K_GAUGE))
    E3 = np.eye(3)
    for i in range(nc):
        R, t = state.cam_R[i], state.cam_t[i]
        o = prob.off["cam"] + cd * i
        for k in range(3):
            Rw = R @ E3[k]
            G[o:o + 3, k] = -Rw
            G[o + 3:o + 6, k] = np.cross(Rw, t)
            G[o + 3:o + 6, 3 + k] = -Rw
        G[o + 3:o + 6, 6] = t
    for g in range(npl):
        n, w = state.pl_n[g], state.pl_w[g]
        B = s2_basis(n)
        o = prob.off["pl"] + 3 * g
        for k in range(3):
            G[o:o + 2, k] = B.T @ np.cross(E3[k], n)
            G[o + 2, 3 + k] = -n[k]
        G[o + 2, 6] = w
    for v in range(nvp):
        d = state.vp[v]
        B = s2_basis(d)
        o = prob.off["vp"] + 2 * v
        for k in range(3):
            G[o:o + 2, k] = B.T @ np.cross(E3[k], d)
    if prob.n.get("sh", 0):
        from oracle.shapes import gauge_rows
        rows, _ = gauge_rows(state.sh)
        o = prob.off["sh"]
        G[o:o + rows.size // 7] = rows.reshape(-1, 7)
    return G


def gauge_basis_features(prob, state):
    """G_f ((3 n_pt + 4 n_ln) x 7): the same world rotation, translation and
    scale as gauge_basis, as first-order motions of the points and lines in
    their tangent coordinates, so that [G; G_f] is the motion of every
    parameter.  Points move additively: e_k x X, e_k, X.  A line (d, m) =
    (w1 U e1, w2 U e2) with m = p x d moves to (d + w x d, m + w x m) under a
    rotation w, (d, m + t x d) under a translation t and (d, (1 + s) m) under a
    scale s, each up to the common scale of (d, m); in the tangent
    (dtheta, dphi) of U <- U Exp(dtheta) and the rotation of (w1, w2) by dphi
    that is dtheta = U^T e_k for rotation k, dtheta = (-w1 (u2 . e_k) / w2, 0, 0)
    and dphi = w1^2 (u3 . e_k) for translation k, and dphi = w1 w2 for the scale."""
    npt, nln = prob.n["pt"], prob.n["ln"]
    G = np.zeros((3 * npt + 4 * nln, K_GAUGE))
    E3 = np.eye(3)
    for j in range(npt):
        X = state.pts[j]
        for k in range(3):
            G[3 * j:3 * j + 3, k] = np.cross(E3[k], X)
            G[3 * j:3 * j + 3, 3 + k] = E3[k]
        G[3 * j:3 * j + 3, 6] = X
    o = 3 * npt
    for j in range(nln):
        U, (w1, w2) = state.line_U[j], state.line_w[j]
        u2, u3 = U[:, 1], U[:, 2]
        r = o + 4 * j
        for k in range(3):
            G[r:r + 3, k] = U.T @ E3[k]
            G[r, 3 + k] = -w1 * u2[k] / w2
            G[r + 3, 3 + k] = w1 * w1 * u3[k]
        G[r + 3, 6] = w1 * w2
    return G


def block_graph(prob):
    """Block graph of the reduced system of an oracle Problem."""
    nc, npl, nvp = prob.n["cam"], prob.n["pl"], prob.n["vp"]
    n = nc + npl + nvp
    cd = prob.camera_dof
    ntype = np.array([TYPE_CAM] * nc + [TYPE_PLANE] * npl + [TYPE_VP] * nvp, dtype=np.int64)
    sizes = np.array([cd] * nc + [3] * npl + [2] * nvp, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if n else np.zeros(0, np.int64)
    # (feature id, block) incidences of every record; points first, then lines
    npt = prob.n["pt"]
    feats, blocks = [], []
    for fam, r in prob.recs.items():
        if fam not in ("R1", "R2", "R3", "R4", "R5", "R6", "R7", "R12"):
            continue  # inter-group relations share no feature
        f = r["ln"] + npt if fam in ("R2", "R4", "R5", "R7") else r["pt"]
        if "cam" in r:
            feats.append(f)
            blocks.append(r["cam"])
        if "pl" in r:
            feats.append(f)
            blocks.append(nc + r["pl"])
        if "vp" in r:
            feats.append(f)
            blocks.append(nc + npl + r["vp"])
    feats = np.concatenate(feats) if feats else np.zeros(0, np.int64)
    blocks = np.concatenate(blocks) if blocks else np.zeros(0, np.int64)
    records = np.bincount(blocks, minlength=n)
    pairs = np.unique(np.stack([feats, blocks], axis=1), axis=0) if len(feats) else np.zeros((0, 2), np.int64)
    shared = {}
    starts = np.flatnonzero(np.r_[True, pairs[1:, 0] != pairs[:-1, 0]]) if len(pairs) else []
    for bs in np.split(pairs[:, 1], starts[1:]) if len(pairs) else []:
        for a in bs:
            for b in bs:
                if a != b:
                    shared[(int(b), int(a))] = shared.get((int(b), int(a)), 0) + 1  # edge a -> b
    keys = sorted(shared, key=lambda k: (k[0], k[1]))  # (dst, src)
    dst = np.array([k[0] for k in keys], dtype=np.int64)
    src = np.array([k[1] for k in keys], dtype=np.int64)
    cnt = np.array([shared[k] for k in keys], dtype=np.float64)
    ex = np.zeros((len(keys), EDGE_IN))
    ex[:, 0] = np.log1p(cnt)
    ts, td = ntype[src], ntype[dst]
    cc = (ts == TYPE_CAM) & (td == TYPE_CAM)
    cp = ((ts == TYPE_CAM) & (td == TYPE_PLANE)) | ((ts == TYPE_PLANE) & (td == TYPE_CAM))
    cv = ((ts == TYPE_CAM) & (td == TYPE_VP)) | ((ts == TYPE_VP) & (td == TYPE_CAM))
    ex[:, 1], ex[:, 2], ex[:, 3] = cc, cp, cv
    ex[:, 4] = ~(cc | cp | cv)
    degree = np.bincount(dst, minlength=n)
    return dict(n=n, node_type=ntype, sizes=sizes, offsets=offsets, edge_src=src, edge_dst=dst,
                edge_x=ex, shared=cnt, records=records, degree=degree)


def unit_scales(graph, s0, camera_dof):
    """Per node the row scales u_i (padded to 9)."""
    cam = [1, 1, 1, s0, s0, s0, 1, 1, 1][:camera_dof]
    rows = {TYPE_CAM: cam, TYPE_PLANE: [1, 1, s0], TYPE_VP: [1, 1]}
    out = np.zeros((graph["n"], 9))
    for i, t in enumerate(graph["node_type"]):
        u = rows[int(t)]
        out[i, :len(u)] = u
    return out


def node_inputs(graph, S_blocks, lam, state, s0):
    """x (n x 64) from the damped diagonal blocks S_ii, lambda, structure and geometry."""
    from oracle.model import s2_basis
    n = graph["n"]
    units = unit_scales(graph, s0, int(max(graph["sizes"])) if n else 9)
    x = np.zeros((n, NODE_IN))
    nc = int(np.sum(graph["node_type"] == TYPE_CAM))
    npl = int(np.sum(graph["node_type"] == TYPE_PLANE))
    for i in range(n):
        S = np.asarray(S_blocks[i], dtype=np.float64)
        nb = S.shape[0]
        ld = np.log(np.diag(S) * units[i, :nb] ** 2)
        x[i, :nb] = ld - ld.mean()
        c = 9
        for p in range(1, nb):
            for q in range(p):
                x[i, c] = S[p, q] / math.sqrt(S[p, p] * S[q, q])
                c += 1
        x[i, 45] = math.log(lam)
        x[i, 46] = math.log1p(graph["records"][i])
        x[i, 47] = math.log1p(graph["degree"][i])
        t = int(graph["node_type"][i])
        x[i, 48 + t] = 1.0
        if t == TYPE_CAM:
            x[i, 51:60] = state.cam_R[i].ravel()
            x[i, 60:63] = state.cam_t[i] / s0
        elif t == TYPE_PLANE:
            g = i - nc
            nv = state.pl_n[g]
            B = s2_basis(nv)
            x[i, 51:54] = nv
            x[i, 54] = state.pl_w[g] / s0
            x[i, 55:58] = B[:, 0]
            x[i, 58:61] = B[:, 1]
        else:
            v = state.vp[i - nc - npl]
            B = s2_basis(v)
            x[i, 51:54] = v
            x[i, 54:57] = B[:, 0]
            x[i, 57:60] = B[:, 1]
    return x


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def gelu(x):
    return 0.5 * x * (1.0 + torch.tanh(math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3)))


def _t(v):
    return v if torch.is_tensor(v) else torch.as_tensor(np.asarray(v), dtype=torch.float64)


def _bf(x):
    """x rounded to bfloat16 (to nearest, ties to even) through FP32, back in float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _Bf16Matmul(torch.autograd.Function):
    """A @ W on BF16-rounded operands; both backward products (dA = dC W^T,
    dW = A^T dC) on BF16-rounded operands too.  The network's dense layers in BF16
    precision: every GEMM operand is rounded, accumulation is wide."""

    @staticmethod
    def forward(ctx, A, W):
        ctx.save_for_backward(A, W)
        return _bf(A) @ _bf(W)

    @staticmethod
    def backward(ctx, g):
        A, W = ctx.saved_tensors
        gb = _bf(g)
        return gb @ _bf(W).T, _bf(A).T @ gb


class _Bf16WeightGrad(torch.autograd.Function):
    """A @ W unrounded (a product formed inside the edge kernel), whose weight gradient
    A^T dC is a BF16 GEMM (rounded operands); A takes no gradient."""

    @staticmethod
    def forward(ctx, A, W):
        ctx.save_for_backward(A)
        return A @ W

    @staticmethod
    def backward(ctx, g):
        (A,) = ctx.saved_tensors
        return None, _bf(A).T @ _bf(g)


def forward(params, node_x, node_type, edge_src, edge_dst, edge_x, camera_dof=9, bf16=False):
    """Y_i (n_i x K tensors) per node.  With bf16 the dense products round their
    operands to BF16 as the BF16 network does (the message layer split into its
    per-node h-part, a GEMM, and its per-edge input part, formed in full precision)."""
    P = {k: _t(v) for k, v in params.items()}
    x = _t(node_x)
    ex = _t(edge_x).reshape(-1, EDGE_IN)
    src = torch.as_tensor(np.asarray(edge_src), dtype=torch.long)
    dst = torch.as_tensor(np.asarray(edge_dst), dtype=torch.long)
    n = x.shape[0]
    deg = torch.zeros(n, dtype=torch.float64).index_add_(0, dst, torch.ones(len(dst), dtype=torch.float64))
    mm = _Bf16Matmul.apply if bf16 else (lambda a, b: a @ b)
    h = gelu(mm(x, P["W_in"]) + P["b_in"])
    for l in range(LAYERS):
        W = P[f"W_e{l}"]
        if bf16:
            pre = mm(h, W[:H])[src] + _Bf16WeightGrad.apply(ex, W[H:]) + P[f"b_e{l}"]
        else:
            pre = torch.cat([h[src], ex], dim=1) @ W + P[f"b_e{l}"]
        msg = gelu(pre)
        m = torch.zeros(n, H, dtype=torch.float64).index_add_(0, dst, msg)
        m = m / torch.clamp(deg, min=1.0)[:, None]
        h = gelu(mm(h, P[f"W_s{l}"]) + P[f"b_s{l}"] + m) + h
    sizes = block_sizes(camera_dof)
    out = []
    for i, t in enumerate(np.asarray(node_type)):
        y = mm(h[i:i + 1], P[f"W_t{int(t)}"])[0] + P[f"b_t{int(t)}"]
        out.append(y.reshape(sizes[int(t)], K))
    return out


def coarse_basis(Y, units):
    """Z (n_A x K): Z_i = diag(u_i) Y_i stacked in node order."""
    rows = [torch.as_tensor(units[i][:y.shape[0]], dtype=torch.float64)[:, None] * y for i, y in enumerate(Y)]
    return torch.cat(rows, dim=0)


def block_diagonal(S, sizes):
    D = torch.zeros_like(S)
    o = 0
    for nb in sizes:
        nb = int(nb)
        D[o:o + nb, o:o + nb] = S[o:o + nb, o:o + nb]
        o += nb
    return D


def coarse_loss(Z, S, sizes):
    """tr((Z^T D Z)^-1 Z^T S Z), D = blockdiag(S)."""
    S = _t(S)
    D = block_diagonal(S, sizes)
    A = Z.T @ S @ Z
    G = Z.T @ D @ Z
    return torch.trace(torch.linalg.solve(G, A))


def full_basis(G, Y, units):
    """Z = [G, Z_net] (n_A x 15)."""
    return torch.cat([_t(G), coarse_basis(Y, units)], dim=1)


def batch_loss(params, systems, camera_dof=9, bf16=False):
    """Mean coarse loss over systems; each a dict with node_x, graph, S (dense), units, gauge."""
    total = torch.zeros((), dtype=torch.float64)
    for s in systems:
        g = s["graph"]
        Y = forward(params, s["node_x"], g["node_type"], g["edge_src"], g["edge_dst"], g["edge_x"], camera_dof, bf16)
        total = total + coarse_loss(full_basis(s["gauge"], Y, s["units"]), s["S"], g["sizes"])
    return total / len(systems)


def loss_and_grads(params, systems, camera_dof=9, bf16=False):
    P = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in params.items()}
    L = batch_loss(P, systems, camera_dof, bf16)
    L.backward()
    return float(L.detach()), {k: v.grad.numpy().copy() for k, v in P.items()}


# ---------------------------------------------------------------------------
# preconditioner and PCG
# ---------------------------------------------------------------------------
def block_jacobi(S, sizes):
    """M = blockdiag(S_ii)^-1 (numpy)."""
    M = np.zeros_like(S)
    o = 0
    for nb in sizes:
        nb = int(nb)
        M[o:o + nb, o:o + nb] = np.linalg.inv(S[o:o + nb, o:o + nb])
        o += nb
    return M


def two_level(S, sizes, Z):
    """Dense A-DEF2 preconditioner (I - Q S) M + Q with Q = Z (Z^T S Z)^-1 Z^T,
    and the start vector's map Q (None, None for M alone, also when Z^T S Z is
    not positive definite)."""
    M = block_jacobi(S, sizes)
    if Z is None:
        return M, None
    E = Z.T @ S @ Z
    try:
        np.linalg.cholesky(E)
    except np.linalg.LinAlgError:
        return M, None
    Q = Z @ np.linalg.solve(E, Z.T)
    return (np.eye(len(S)) - Q @ S) @ M + Q, Q


def pcg(S, b, P, tol=1e-6, max_iters=10000, x0=None):
    """Textbook preconditioned CG from x0 (0 if None); stops when
    |b - S x| <= tol |b|.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - S @ x
    bb = b @ b
    if bb == 0:
        return x, 0
    if r @ r <= tol * tol * bb:
        return x, 0
    z = P @ r
    p = z.copy()
    rz = r @ z
    for k in range(max_iters):
        q = S @ p
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        if r @ r <= tol * tol * bb:
            return x, k + 1
        z = P @ r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iters
