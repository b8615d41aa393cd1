"""Pins of the learned coarse-space oracle (oracle/gnn.py) on the CPU.

The network, the loss and the two-level preconditioner are this project's
addition to the method, so the pins are mathematical: central differences
for the autograd gradient, the Ky Fan bound for the loss (its minimum over
K-dimensional subspaces is the sum of the K smallest eigenvalues of the
block-normalised matrix), invariance of the loss under a change of basis of
span(Z), node-permutation equivariance of the network, known values of the
tanh form of GELU, brute-force shared-feature counts of the block graph,
and the effect of an exact slow-mode basis on textbook PCG.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gnn, lm
from scenegen import make_scene, small_config


@pytest.fixture(scope="module")
def tiny():
    sc = make_scene(small_config(n_cams=6, n_points=30, n_lines=10, n_planes=2, n_vps=2), seed=7)
    prob = lm.Problem(sc)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    lam = 1e-3
    S = lm.schur(prob, lin, lam)["S"]
    S = 0.5 * (S + S.T)
    g = gnn.block_graph(prob)
    blocks = [S[o:o + n, o:o + n] for o, n in zip(g["offsets"], g["sizes"])]
    s0 = gnn.scene_scale(sc["cameras"])
    x = gnn.node_inputs(g, blocks, lam, st, s0)
    u = gnn.unit_scales(g, s0, prob.camera_dof)
    return dict(sc=sc, prob=prob, st=st, S=S, graph=g, x=x, units=u, s0=s0, lam=lam)


def _normalised(S, sizes):
    Linv = np.zeros_like(S)
    o = 0
    for n in sizes:
        Linv[o:o + n, o:o + n] = np.linalg.inv(np.linalg.cholesky(S[o:o + n, o:o + n]))
        o += n
    return Linv, Linv @ S @ Linv.T


def test_gelu_tanh_form_values():
    """x/2 (1 + tanh(sqrt(2/pi)(x + 0.044715 x^3))) at x = 0, +-1, 3."""
    def ref(x):
        return 0.5 * x * (1 + math.tanh(math.sqrt(2 / math.pi) * (x + 0.044715 * x ** 3)))
    xs = torch.tensor([0.0, 1.0, -1.0, 3.0], dtype=torch.float64)
    got = gnn.gelu(xs).numpy()
    assert got[0] == 0.0
    assert abs(got[1] - 0.8411919906082768) < 1e-12
    assert abs(got[2] + 0.15880800939172324) < 1e-12
    assert abs(got[3] - ref(3.0)) < 1e-12


def test_block_graph_against_brute_force(tiny):
    prob, g = tiny["prob"], tiny["graph"]
    nc, npl, nvp = prob.n["cam"], prob.n["pl"], prob.n["vp"]
    # brute force: the set of blocks every feature touches, from the records one by one
    touch = {}
    for fam, r in prob.recs.items():
        nrec = len(next(iter(r.values())))
        for k in range(nrec):
            f = ("ln", int(r["ln"][k])) if fam in ("R2", "R4", "R5", "R7") else ("pt", int(r["pt"][k]))
            bl = touch.setdefault(f, set())
            if "cam" in r:
                bl.add(int(r["cam"][k]))
            if "pl" in r:
                bl.add(nc + int(r["pl"][k]))
            if "vp" in r:
                bl.add(nc + npl + int(r["vp"][k]))
    n = nc + npl + nvp
    cnt = np.zeros((n, n), dtype=int)
    for bl in touch.values():
        for a in bl:
            for b in bl:
                if a != b:
                    cnt[b, a] += 1
    dst, src = np.nonzero(cnt)
    order = np.lexsort((src, dst))
    assert np.array_equal(g["edge_dst"], dst[order]) and np.array_equal(g["edge_src"], src[order])
    assert np.array_equal(g["shared"], cnt[dst[order], src[order]])
    # both directions present, with equal counts
    assert np.array_equal(cnt, cnt.T)
    assert np.array_equal(g["degree"], (cnt > 0).sum(axis=1))
    # the reduced matrix has a nonzero off-diagonal block exactly on the edges
    S = tiny["S"]
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            oi, ni = g["offsets"][i], g["sizes"][i]
            oj, nj = g["offsets"][j], g["sizes"][j]
            nz = np.abs(S[oi:oi + ni, oj:oj + nj]).max() > 0
            assert nz == (cnt[i, j] > 0), (i, j)


def test_node_inputs_structure(tiny):
    x, g = tiny["x"], tiny["graph"]
    for i, t in enumerate(g["node_type"]):
        n = g["sizes"][i]
        assert abs(x[i, :n].sum()) < 1e-9          # log-diagonal is centred
        assert np.all(x[i, n:9] == 0)
        assert np.all(np.abs(x[i, 9:45]) <= 1 + 1e-12)  # correlations
        assert x[i, 48 + t] == 1 and x[i, 48:51].sum() == 1
        assert x[i, 45] == pytest.approx(math.log(tiny["lam"]))
    cams = g["node_type"] == 0
    R = x[cams, 51:60].reshape(-1, 3, 3)
    assert np.allclose(np.einsum("nij,nkj->nik", R, R), np.eye(3), atol=1e-9)


def test_loss_gradient_matches_central_differences(tiny):
    cd = tiny["prob"].camera_dof
    p = gnn.init_params(cd, seed=3)
    sysd = [dict(node_x=tiny["x"], graph=tiny["graph"], S=tiny["S"], units=tiny["units"])]
    L, grads = gnn.loss_and_grads(p, sysd, cd)
    assert np.isfinite(L)
    rng = np.random.default_rng(0)
    for name, _ in gnn.param_shapes(cd):
        idx = [tuple(rng.integers(0, s) for s in p[name].shape) for _ in range(2)]
        for ix in idx:
            h = 1e-5 * max(1.0, abs(p[name][ix]))
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][ix] += h
            pm[name][ix] -= h
            fd = (float(gnn.batch_loss(pp, sysd, cd)) - float(gnn.batch_loss(pm, sysd, cd))) / (2 * h)
            assert abs(fd - grads[name][ix]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (name, ix, fd, grads[name][ix])


def test_loss_ky_fan_bound_and_basis_invariance(tiny):
    S, g = tiny["S"], tiny["graph"]
    Linv, Sh = _normalised(S, g["sizes"])
    w, V = np.linalg.eigh(Sh)
    K = gnn.K
    # exact slow modes: Z = L^-T V_K gives the sum of the K smallest eigenvalues
    Z = torch.as_tensor(Linv.T @ V[:, :K])
    assert float(gnn.coarse_loss(Z, S, g["sizes"])) == pytest.approx(w[:K].sum(), rel=1e-9)
    rng = np.random.default_rng(1)
    for _ in range(5):
        Zr = rng.normal(size=(S.shape[0], K))
        Lr = float(gnn.coarse_loss(torch.as_tensor(Zr), S, g["sizes"]))
        assert Lr >= w[:K].sum() - 1e-9
        assert Lr <= w[-K:].sum() + 1e-9
        Q = rng.normal(size=(K, K)) + 3 * np.eye(K)
        assert float(gnn.coarse_loss(torch.as_tensor(Zr @ Q), S, g["sizes"])) == pytest.approx(Lr, rel=1e-9)


def test_network_is_equivariant_to_camera_relabelling(tiny):
    g, x = tiny["graph"], tiny["x"]
    cd = tiny["prob"].camera_dof
    p = gnn.init_params(cd, seed=5)
    Y = gnn.forward(p, x, g["node_type"], g["edge_src"], g["edge_dst"], g["edge_x"], cd)
    nc = int(np.sum(g["node_type"] == 0))
    perm = np.arange(g["n"])
    perm[:nc] = np.random.default_rng(2).permutation(nc)  # new node k is old node perm[k]
    inv = np.argsort(perm)
    Y2 = gnn.forward(p, x[perm], g["node_type"][perm], inv[g["edge_src"]], inv[g["edge_dst"]], g["edge_x"], cd)
    for k in range(g["n"]):
        assert torch.allclose(Y2[k], Y[perm[k]], atol=1e-12)


def test_exact_slow_modes_cut_pcg_iterations(tiny):
    """Textbook PCG with P = M + Z (Z^T S Z)^-1 Z^T and Z the exact slowest
    block-normalised modes needs fewer iterations than block-Jacobi alone,
    and both reach the same solution."""
    S, g = tiny["S"], tiny["graph"]
    b = np.random.default_rng(4).normal(size=S.shape[0])
    Linv, Sh = _normalised(S, g["sizes"])
    w, V = np.linalg.eigh(Sh)
    Z = Linv.T @ V[:, :gnn.K]
    P0 = gnn.two_level(S, g["sizes"], None)
    P1 = gnn.two_level(S, g["sizes"], Z)
    assert np.allclose(P1, P1.T, atol=1e-8 * np.abs(P1).max())
    assert np.linalg.eigvalsh(0.5 * (P1 + P1.T)).min() > 0
    x0, it0 = gnn.pcg(S, b, P0, tol=1e-10)
    x1, it1 = gnn.pcg(S, b, P1, tol=1e-10)
    xs = np.linalg.solve(S, b)
    assert np.linalg.norm(x0 - xs) <= 1e-6 * np.linalg.norm(xs)
    assert np.linalg.norm(x1 - xs) <= 1e-6 * np.linalg.norm(xs)
    assert it1 < it0, (it0, it1)


def test_pack_unpack_round_trip():
    p = gnn.init_params(9, seed=0)
    blob = gnn.pack(p).tobytes()
    q = gnn.unpack(blob)
    assert len(blob) == 4 * gnn.param_count(9)
    for k in p:
        assert np.allclose(p[k], q[k], atol=1e-6)


def test_inputs_and_loss_do_not_change_when_the_scene_is_scaled(tiny):
    """Scaling every length of the scene by a (camera t, points, lines, plane
    offsets) leaves the images unchanged; with the unit scales u the node
    inputs and the loss of a fixed network must not change."""
    a = 3.7
    sc = dict(tiny["sc"])
    cams = np.array(sc["cameras"], dtype=np.float64).copy()
    cams[:, 4:7] *= a
    pl = np.array(sc["planes"], dtype=np.float64).copy()
    pl[:, 3] *= a
    sc.update(cameras=cams, points=np.asarray(sc["points"]) * a, lines=np.asarray(sc["lines"]) * a, planes=pl)
    prob = lm.Problem(sc)
    st = prob.state0()
    lam = tiny["lam"]
    S = lm.schur(prob, lm.linearize(prob, st), lam)["S"]
    S = 0.5 * (S + S.T)
    g = gnn.block_graph(prob)
    s0 = gnn.scene_scale(sc["cameras"])
    assert s0 == pytest.approx(a * tiny["s0"], rel=1e-12)
    x = gnn.node_inputs(g, [S[o:o + n, o:o + n] for o, n in zip(g["offsets"], g["sizes"])], lam, st, s0)
    assert np.allclose(x, tiny["x"], atol=1e-8)
    cd = prob.camera_dof
    p = gnn.init_params(cd, seed=9)
    L1 = float(gnn.batch_loss(p, [dict(node_x=tiny["x"], graph=tiny["graph"], S=tiny["S"], units=tiny["units"])], cd))
    L2 = float(gnn.batch_loss(p, [dict(node_x=x, graph=g, S=S, units=gnn.unit_scales(g, s0, cd))], cd))
    assert L2 == pytest.approx(L1, rel=1e-7)
