"""Pins of the learned coarse-space oracle (oracle/gnn.py) on the CPU.

The network, the loss and the two-level preconditioner are this project's
addition to the method, so the pins are mathematical: central differences
for the autograd gradient, the Ky Fan bound for the loss (its minimum over
K-dimensional subspaces is the sum of the K smallest eigenvalues of the
block-normalised matrix), invariance of the loss under a change of basis of
span(Z), node-permutation equivariance of the network, known values of the
tanh form of GELU, brute-force shared-feature counts of the block graph,
the annihilation of the gauge basis by the undamped reduced matrix, and the
effect of exact slow-mode bases on textbook PCG.
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
    G = gnn.gauge_basis(prob, st)
    return dict(sc=sc, prob=prob, st=st, S=S, graph=g, x=x, units=u, s0=s0, lam=lam, gauge=G, lin=lin)


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
    sysd = [dict(node_x=tiny["x"], graph=tiny["graph"], S=tiny["S"], units=tiny["units"], gauge=tiny["gauge"])]
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
    K = gnn.K + gnn.K_GAUGE
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


def test_gauge_basis_is_annihilated_by_the_undamped_reduced_matrix(tiny):
    """Every residual except the VP 3-vector is invariant under a world
    similarity, so J [G; G_f] = 0 and the reduced matrix maps the gauge basis
    to O(lambda).  The VP residual (d/|d|) x v rotates with the world (its norm
    does not), which leaves O(|r_VP|) in the rotation columns: exact at a
    noise-free state, checked there with VPs present."""
    def rel_residual(sc, lam):
        prob = lm.Problem(sc)
        st = prob.state0()
        S = lm.schur(prob, lm.linearize(prob, st), lam)["S"]
        G = gnn.gauge_basis(prob, st)
        assert np.linalg.matrix_rank(G) == gnn.K_GAUGE
        return np.linalg.norm(S @ G, axis=0) / (np.linalg.norm(S) * np.linalg.norm(G, axis=0)), S
    no_vp = small_config(n_cams=6, n_points=30, n_lines=10, n_planes=2, n_vps=0, vp_lines=0)
    for lam in (1e-10, 1e-6):
        rel, S = rel_residual(make_scene(no_vp, seed=7), lam)
        assert rel.max() < 50 * lam + 1e-11, (lam, rel)
    with_vp = small_config(n_cams=6, n_points=30, n_lines=10, n_planes=2, n_vps=2)
    rel, S = rel_residual(make_scene(with_vp, seed=7, noise=False), 1e-10)
    assert rel.max() < 1e-9, rel
    # a generic direction is not annihilated
    v = np.random.default_rng(3).normal(size=(S.shape[0], 1))
    assert np.linalg.norm(S @ v) / (np.linalg.norm(S) * np.linalg.norm(v)) > 1e-4


def test_feature_gauge_motion_is_annihilated_by_the_jacobian():
    """With the features' motion G_f beside G, the whole similarity [G; G_f]
    is a null direction of the weighted Jacobian of every family but the VP
    3-vector (points, lines, planes, junctions; noisy state, robust weights):
    J [G; G_f] = 0 to rounding.  A wrong sign, index or factor in any of the
    13 point / line formulas leaves an O(|J| |z|) residual."""
    sc = make_scene(small_config(n_cams=6, n_points=40, n_lines=14, n_planes=2, n_vps=0, vp_lines=0), seed=9)
    prob = lm.Problem(sc)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    assert prob.n["ln"] > 0 and prob.record_count("R4") > 0 and prob.record_count("R6") > 0
    Z = np.vstack([gnn.gauge_basis(prob, st), gnn.gauge_basis_features(prob, st)])
    J = lin.J.toarray()
    rel = np.linalg.norm(J @ Z, axis=0) / (np.linalg.norm(J) * np.linalg.norm(Z, axis=0))
    assert rel.max() < 1e-12, rel
    # the feature part is needed: the A side alone is not annihilated
    Za = np.vstack([gnn.gauge_basis(prob, st), np.zeros((prob.nF, gnn.K_GAUGE))])
    rel_a = np.linalg.norm(J @ Za, axis=0) / (np.linalg.norm(J) * np.linalg.norm(Za, axis=0))
    assert rel_a.min() > 1e-4, rel_a


def test_exact_slow_modes_cut_pcg_iterations(tiny):
    """Textbook PCG with the A-DEF2 two-level preconditioner started from
    x0 = Q b: the gauge basis alone, and the gauge plus the exact next slowest
    modes, need fewer iterations than block-Jacobi; all reach the same x."""
    S, g, G = tiny["S"], tiny["graph"], tiny["gauge"]
    b = np.random.default_rng(4).normal(size=S.shape[0])
    Linv, Sh = _normalised(S, g["sizes"])
    # the next slowest block-normalised modes after removing span(L^T G)
    Q0, _ = np.linalg.qr(np.linalg.solve(Linv.T, G))  # span of the gauge in block-normalised coordinates
    Pp = np.eye(len(b)) - Q0 @ Q0.T
    w, V = np.linalg.eigh(Pp @ Sh @ Pp)
    keep = [k for k in np.argsort(w) if w[k] > 1e-10][:gnn.K]
    Zn = Linv.T @ V[:, keep]
    xs = np.linalg.solve(S, b)
    its = {}
    for name, Z in (("bj", None), ("gauge", G), ("gauge+next", np.hstack([G, Zn]))):
        P, Q = gnn.two_level(S, g["sizes"], Z)
        x, it = gnn.pcg(S, b, P, tol=1e-10, x0=None if Q is None else Q @ b)
        assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs), name
        its[name] = it
    assert its["gauge"] < its["bj"] and its["gauge+next"] <= its["gauge"], its
    # the coarse-space start already solves the problem restricted to span(Z)
    P, Q = gnn.two_level(S, g["sizes"], G)
    r0 = b - S @ (Q @ b)
    assert np.abs(G.T @ r0).max() <= 1e-8 * np.abs(G.T @ b).max()


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
    L1 = float(gnn.batch_loss(p, [dict(node_x=tiny["x"], graph=tiny["graph"], S=tiny["S"], units=tiny["units"],
                                       gauge=tiny["gauge"])], cd))
    L2 = float(gnn.batch_loss(p, [dict(node_x=x, graph=g, S=S, units=gnn.unit_scales(g, s0, cd),
                                       gauge=gnn.gauge_basis(prob, st))], cd))
    assert L2 == pytest.approx(L1, rel=1e-7)


def test_bf16_mode_with_exact_rounding_is_the_network(tiny, monkeypatch):
    """The BF16 emulation (operands of every dense product rounded, the message layer
    split into its per-node h-part and its per-edge input part, custom backward
    products) reduces to the plain network when rounding is the identity: same heads,
    loss and gradients to 1e-10 (summation order).  And with true BF16 rounding it stays within BF16's
    reach of it (heads 5e-2, gradients 0.2)."""
    cd = tiny["prob"].camera_dof
    p = gnn.init_params(cd, seed=4)
    sysd = [dict(node_x=tiny["x"], graph=tiny["graph"], S=tiny["S"], units=tiny["units"], gauge=tiny["gauge"])]
    g = tiny["graph"]
    args = (tiny["x"], g["node_type"], g["edge_src"], g["edge_dst"], g["edge_x"], cd)
    L0, G0 = gnn.loss_and_grads(p, sysd, cd)
    Y0 = torch.cat([y.reshape(-1) for y in gnn.forward(p, *args)])
    Lb, Gb = gnn.loss_and_grads(p, sysd, cd, bf16=True)
    Yb = torch.cat([y.reshape(-1) for y in gnn.forward(p, *args, bf16=True)])
    assert float(torch.linalg.norm(Yb - Y0) / torch.linalg.norm(Y0)) <= 5e-2
    for k in G0:
        assert np.linalg.norm(Gb[k] - G0[k]) <= 0.2 * np.linalg.norm(G0[k]), k
    assert 0 < float(torch.linalg.norm(Yb - Y0)), "rounding had no effect"
    monkeypatch.setattr(gnn, "_bf", lambda x: x)
    L1, G1 = gnn.loss_and_grads(p, sysd, cd, bf16=True)
    Y1 = torch.cat([y.reshape(-1) for y in gnn.forward(p, *args, bf16=True)])
    assert float(torch.abs(Y1 - Y0).max()) <= 1e-10 * float(torch.abs(Y0).max())
    assert abs(L1 - L0) <= 1e-10 * abs(L0)
    for k in G0:
        assert np.abs(G1[k] - G0[k]).max() <= 1e-10 * max(np.abs(G0[k]).max(), 1e-30), k
