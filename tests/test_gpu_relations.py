"""Inter-group relations on the GPU (Sec. 3.2: orthogonality and parallelism
between VP pairs and between plane-normal pairs), through the C ABI, on a
small Manhattan scene, against the oracle:

- the relation records (residual and both group blocks of the Jacobian;
  FP64 in both precisions: they are few and A-side only), and every other
  family as usual;
- the reduced system: b, the diagonal blocks of S and the implicit-Schur
  product entry by entry (the relations add U_gh blocks between groups);
- one LM step against the oracle's exact Schur step, and the converged cost
  against the oracle's (golden file written by the oracle);
- S Z of the gauge coarse space against the oracle's dense S (the relation
  rows are added to the closed-form gauge columns);
- a deterministic-mode repeat, bit for bit.
"""
import json
import os

import numpy as np
import pytest

from scenegen import make_scene, manhattan_config, REL_VP_PARALLEL
from oracle import lm, model
from oracle.records import record_keys

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_converged.json")
LAM = 1e-3


def _ba():
    from paper_2609_04026_amd.binding import BA
    return BA


def _scene(extra_parallel=False):
    s = make_scene(manhattan_config(), seed=12)
    if extra_parallel:
        # two Atlanta VPs related parallel (they are not: a violated relation, for
        # the VP-parallel family's records)
        s = dict(s)
        s["obs"] = dict(s["obs"])
        s["obs"][REL_VP_PARALLEL] = (np.array([3], np.int32), np.array([4], np.int32), None)
    return s


@pytest.fixture(scope="module")
def manh():
    s = _scene()
    prob = lm.Problem(s)
    st = prob.state0()
    return s, prob, st, lm.linearize(prob, st)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_relation_records_match_oracle(precision):
    s = _scene(extra_parallel=True)
    prob = lm.Problem(s)
    lin = lm.linearize(prob, prob.state0())
    ba = _ba().from_scene(s, precision=precision)
    ba.linearize(LAM)
    keys_or = record_keys(prob.recs)
    for fam in (8, 9, 10, 11):
        name = f"R{fam}"
        n = prob.record_count(name)
        assert n > 0 and ba.record_count(fam) == n, name
        keys, r, J = ba.export_records(fam)
        og = np.lexsort(keys.T[::-1])
        oo = np.lexsort(keys_or[name][:, 1:].T[::-1])
        assert np.array_equal(keys[og], keys_or[name][:, 1:][oo]), name
        L = lin.fam[name]
        assert np.abs(r[og] - L["rt"][oo]).max() <= 1e-9 * max(np.abs(L["rt"]).max(), 1.0), name
        gd = L["J"]["ga"].shape[2]
        Jref = np.concatenate([L["J"]["ga"][oo], L["J"]["gb"][oo]], axis=2)
        assert J.shape[2] == 2 * gd
        assert np.abs(J[og] - Jref).max() <= 1e-9 * np.abs(Jref).max(), name
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_relations_reduced_system_and_step_match_oracle(manh, precision):
    s, prob, st, lin = manh
    assert all(prob.record_count(f) > 0 for f in ("R8", "R10", "R11"))
    ba = _ba().from_scene(s, precision=precision)
    ba.linearize(LAM)
    tol = 1e-9 if precision == "fp64" else 1e-4
    sys_ = lm.schur(prob, lin, LAM)
    b, Sc, Sp, Sv = ba.export_reduced()
    assert np.abs(b - sys_["b"]).max() <= 10 * tol * np.abs(sys_["b"]).max()
    blocks = lm.diag_blocks(prob, sys_["S"])
    for got, key in ((Sc, "cam"), (Sp, "pl"), (Sv, "vp")):
        ref = blocks[key]
        err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
        assert err.max() <= 10 * tol, (key, err.max())
    S = sys_["S"]
    rng = np.random.default_rng(4)
    for _ in range(3):
        x = rng.normal(size=prob.nA)
        y = ba.schur_matvec(x)
        err = np.abs(y - S @ x) / np.maximum(np.abs(S) @ np.abs(x), 1e-300)
        assert err.max() <= 10 * tol, err.max()
    ba.close()
    ba = _ba().from_scene(s, precision=precision)
    rep = ba.lm_step(lambda0=LAM, pcg_tol=1e-12 if precision == "fp64" else 1e-7, pcg_max_iters=2000)
    h, _ = lm.solve_schur(prob, lin, LAM)
    E0 = lm.cost(prob, st)
    E1 = lm.cost(prob, prob.retract(st, h))
    assert abs(rep["E_before"] - E0[0]) <= 1e-12 * E0[0] and abs(rep["Epix_before"] - E0[1]) <= 1e-12 * E0[1]
    stol = 1e-8 if precision == "fp64" else 1e-4
    assert rep["accepted"] == 1 and abs(rep["E_after"] - E1[0]) <= stol * E1[0], (rep, E1)
    dL = lm.model_decrease(lin, h)
    assert abs(rep["model_decrease"] - dL) <= 10 * stol * abs(dL)
    g = np.max(np.abs(lin.g))
    assert abs(rep["grad_inf"] - g) <= (1e-9 if precision == "fp64" else 1e-4) * g
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_relations_converged_cost_matches_oracle(precision):
    ref = json.load(open(GOLDEN))["manhattan_relations"]
    ba = _ba().from_scene(_scene(), precision=precision)
    out = ba.solve(func_tol=1e-12, max_iters=200, pcg_tol=1e-10 if precision == "fp64" else 1e-8,
                   pcg_max_iters=2000)
    print("[relations]", precision, out, ref["E"], flush=True)
    assert abs(out["E_final"] - ref["E"]) <= 1e-6 * ref["E"], (out["E_final"], ref["E"])
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_relations_gauge_coarse_space_matches_oracle(manh, precision):
    s, prob, st, lin = manh
    S = lm.schur(prob, lin, LAM)["S"]
    ba = _ba().from_scene(s, precision=precision, precond="gauge")
    ba.linearize(LAM)
    Z, SZ = ba.export_coarse_space()
    assert Z.shape == (prob.nA, 7)
    ref = S @ Z
    tol = 1e-9 if precision == "fp64" else 1e-4
    col_err = np.linalg.norm(SZ - ref, axis=0) / np.linalg.norm(np.abs(S) @ np.abs(Z), axis=0)
    assert col_err.max() <= tol, col_err
    ba.close()


def test_relations_deterministic_repeat():
    s = _scene()
    runs = []
    for _ in range(2):
        ba = _ba().from_scene(s, precision="mixed", precond="gauge")
        reps = [ba.lm_step(deterministic=1) for _ in range(4)]
        runs.append(([r["E_after"] for r in reps], ba.get_parameters()))
        ba.close()
    assert runs[0][0] == runs[1][0]
    for k in runs[0][1]:
        assert np.array_equal(runs[0][1][k], runs[1][1][k]), k
