"""Dense Schur solver (the dense-Schur variant of the solver, Sec. 4.1) through
the C ABI.

The device SPD solve against numpy / scipy on seeded matrices (ragged and
exact tile counts, one row, ill-conditioned, not positive definite); S as the
dense solver assembles it against the oracle's S of Sec. 3.1 Eq. 3 entry by
entry (scaled by sqrt(S_ii S_jj)); one LM step against the oracle's exact
Schur step; the converged cost against the oracle's; bitwise repeatability.
Tolerances: FP64 path 1e-10 (S, step), mixed path 1e-4 as for the implicit
path; converged cost 1e-9 (FP64) / 1e-6 (mixed) relative.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from scenegen import make_scene, small_config, manhattan_config
from oracle import lm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_converged.json")

SCENES = {
    "tiny_holistic": lambda: make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101),
    "points_10cam": lambda: make_scene(1),
    "holistic_30cam": lambda: make_scene(2),
    "manhattan_relations": lambda: make_scene(manhattan_config(), seed=12),
}


def _binding():
    from paper_2609_04026_amd import binding
    return binding


@pytest.fixture(scope="module", params=list(SCENES))
def case(request):
    print(f"[case] {request.param}", flush=True)
    s = SCENES[request.param]()
    prob = lm.Problem(s)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    return request.param, s, prob, st, lin


def _spd_solve(A, b):
    import torch
    B = _binding()
    At = torch.tensor(A, dtype=torch.float64, device="cuda")
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    st, info = B.dense_spd_solve(At, bt, stream=torch.cuda.current_stream().cuda_stream)
    return st, info, At.cpu().numpy(), bt.cpu().numpy()


@pytest.mark.parametrize("n", [1, 7, 64, 65, 200, 333])
def test_spd_solve_matches_lapack(n):
    rng = np.random.default_rng(n)
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    b = rng.normal(size=n)
    print(f"[spd] n={n}", flush=True)
    st, info, L, x = _spd_solve(A, b)
    assert st == 0 and info == 0
    Lref = np.linalg.cholesky(A)
    assert np.all(np.triu(L, 1) == 0.0)
    assert np.abs(L - Lref).max() <= 1e-12 * np.sqrt(np.abs(A).max())
    xref = scipy.linalg.cho_solve((Lref, True), b)
    assert np.abs(x - xref).max() <= 1e-12 * np.abs(xref).max()


def test_spd_solve_ill_conditioned():
    """Condition 1e10: the backward error |A x - b| stays at FP64 rounding."""
    n = 150
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = (Q * np.logspace(0, -10, n)) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.normal(size=n)
    st, info, L, x = _spd_solve(A, b)
    assert st == 0 and info == 0
    res = np.abs(A @ x - b).max() / (np.abs(A).max() * np.abs(x).max())
    assert res <= 1e-13, res


@pytest.mark.parametrize("n,col", [(100, 70), (100, 0), (130, 129)])
def test_spd_solve_not_positive_definite(n, col):
    """A non-positive pivot is reported as 1 + its column, with BA_E_NUMERIC."""
    A = np.eye(n) * 2.0
    A[col, col] = -1.0
    st, info, _, _ = _spd_solve(A, np.ones(n))
    assert st == _binding().BA_E_NUMERIC and info == col + 1, (st, info)


def test_spd_solve_nan_pivot_and_empty():
    n = 80
    A = np.eye(n)
    A[30, 30] = np.nan
    st, info, _, _ = _spd_solve(A, np.ones(n))
    assert st == _binding().BA_E_NUMERIC and info == 31
    import torch
    e = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    st, info = _binding().dense_spd_solve(e, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert st == 0 and info == 0


def _scaled_err(S, Sref):
    d = np.sqrt(np.abs(np.diag(Sref)))
    return np.abs(S - Sref) / np.maximum(np.outer(d, d), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_assembled_schur_matches_oracle(case, precision):
    name, s, prob, st, lin = case
    lam = 1e-3
    ba = _binding().BA.from_scene(s, precision=precision)
    ba.linearize(lam)
    S = ba.export_schur_assembled()
    Sref = lm.schur(prob, lin, lam)["S"]
    assert np.array_equal(S, S.T)
    err = _scaled_err(S, Sref).max()
    print(f"[assembled] {name} {precision}: {err:.3e}", flush=True)
    assert err <= (1e-10 if precision == "fp64" else 1e-4), err
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dense_step_matches_exact_schur_step(case, precision):
    name, s, prob, st, lin = case
    lam = 1e-3
    ba = _binding().BA.from_scene(s, precision=precision)
    rep = ba.lm_step(lambda0=lam, solver="dense")
    h, _ = lm.solve_schur(prob, lin, lam)
    st1 = prob.retract(st, h)
    E1 = lm.cost(prob, st1)[0]
    tol = 1e-10 if precision == "fp64" else 1e-4
    print(f"[dense step] {name} {precision}: {rep['E_after']} vs {E1}, residual {rep['pcg_rel_residual']:.2e}",
          flush=True)
    assert rep["accepted"] == 1 and rep["pcg_iters"] == 0 and rep["pcg_flags"] == 0
    assert abs(rep["E_after"] - E1) <= tol * E1, (rep, E1)
    dL = lm.model_decrease(lin, h)
    assert abs(rep["model_decrease"] - dL) <= 10 * tol * abs(dL)
    assert rep["pcg_rel_residual"] <= (1e-9 if precision == "fp64" else 1e-4)
    if precision == "fp64":
        # the accepted step moved the points as the oracle's step does
        p = ba.get_parameters()["points"]
        assert np.abs(p - st1.pts).max() <= 1e-9 * max(1.0, np.abs(st1.pts).max())
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dense_converged_cost_matches_oracle(case, precision):
    name, s, prob, st, lin = case
    ref = json.load(open(GOLDEN))[name]
    ba = _binding().BA.from_scene(s, precision=precision)
    out = ba.solve(func_tol=1e-12, max_iters=200, solver="dense")
    print(f"[dense solve] {name} {precision}: {out} vs {ref['E']}", flush=True)
    tol = 1e-9 if precision == "fp64" else 1e-6
    assert abs(out["E_final"] - ref["E"]) <= tol * ref["E"], (out["E_final"], ref["E"])
    assert out["pcg_iters_total"] == 0
    ba.close()


def test_dense_solver_repeats_bitwise():
    s = SCENES["holistic_30cam"]()
    runs = []
    for _ in range(2):
        ba = _binding().BA.from_scene(s, precision="mixed")
        reps = [ba.lm_step(lambda0=1e-3, solver="dense") for _ in range(3)]
        runs.append(([r["E_after"] for r in reps], ba.get_parameters()["points"].copy()))
        ba.close()
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])


def test_dense_solver_size_limit():
    """More than 8192 reduced rows: the dense solver refuses with BA_E_INVALID and
    says why."""
    s = make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101)
    cams = np.repeat(np.asarray(s["cameras"])[:1], 911, axis=0)
    B = _binding()
    ba = B.BA(cams, np.zeros((0, 3)), np.zeros((0, 6)), np.zeros((0, 4)), np.zeros((0, 3)), s["cx"], s["cy"],
              precision="fp64")
    with pytest.raises(B.BAError) as e:
        ba.lm_step(solver="dense")
    assert "8192" in str(e.value)
    ba.close()
