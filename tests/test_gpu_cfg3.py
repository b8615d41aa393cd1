"""Parity on the 200-camera holistic scene (100k points, 20k lines, 200
planes, 10 VPs, 5k junctions, about 1.24M records), through the C ABI.

Every record of all seven families against the oracle (residual and each
Jacobian block; FP64 path 1e-9, mixed 1e-4 relative, as for the small
scenes); the reduced right-hand side b, the diagonal blocks of S and the
implicit-Schur product entry by entry against the oracle's dense S; and the
converged cost of both paths against the oracle's converged cost
(tests/golden/oracle_converged.json, written by the oracle alone), within
1e-6 relative.
"""
import json
import os

import numpy as np
import pytest

from scenegen import make_scene
from oracle import lm
from oracle.records import record_keys

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_converged.json")
LAM = 1e-3


def _ba():
    from paper_2609_04026_amd.binding import BA
    return BA


@pytest.fixture(scope="module")
def scene3():
    print("[cfg3] generating the 200-camera scene and its oracle linearisation", flush=True)
    s = make_scene(3)
    prob = lm.Problem(s)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    return s, prob, st, lin


@pytest.fixture(scope="module")
def schur3(scene3):
    s, prob, st, lin = scene3
    print("[cfg3] oracle reduced system", flush=True)
    return lm.schur(prob, lin, LAM)


def _block_cols(fam, cd):
    nf = 4 if fam in (2, 4, 5, 7) else 3
    ng = 3 if fam in (3, 4) else 2 if fam == 5 else 0
    c = 0 if fam == 5 else cd
    out = {}
    if c:
        out["cam"] = slice(0, c)
    out["pt" if nf == 3 else "ln"] = slice(c, c + nf)
    if ng:
        out["pl" if ng == 3 else "vp"] = slice(c + nf, c + nf + ng)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg3_records_match_oracle(scene3, precision):
    s, prob, st, lin = scene3
    ba = _ba().from_scene(s, precision=precision)
    ba.linearize(LAM)
    keys_or = record_keys(prob.recs)
    tol = 1e-9 if precision == "fp64" else 1e-4
    for fam in range(1, 8):
        name = f"R{fam}"
        n = prob.record_count(name)
        assert n > 0 and ba.record_count(fam) == n, name
        keys, r, J = ba.export_records(fam)
        og = np.lexsort(keys.T[::-1])
        oo = np.lexsort(keys_or[name][:, 1:].T[::-1])
        assert np.array_equal(keys[og], keys_or[name][:, 1:][oo]), name
        rt, rg = lin.fam[name]["rt"][oo], r[og]
        floor = 1e-3 if fam == 5 else 1.0
        err = np.linalg.norm(rg - rt, axis=1) / np.maximum(np.linalg.norm(rt, axis=1), floor)
        assert err.max() <= tol, (name, err.max())
        for b, sl in _block_cols(fam, prob.camera_dof).items():
            Jo, Jg = lin.fam[name]["J"][b][oo], J[og][:, :, sl]
            nrm = np.linalg.norm(Jo, axis=(1, 2))
            e = np.linalg.norm(Jg - Jo, axis=(1, 2))
            assert np.all(e <= tol * nrm + 1e-9 * (tol / 1e-4)), (name, b, float((e / np.maximum(nrm, 1e-30)).max()))
        print(f"[cfg3] {precision} {name}: {n} records within {tol:g}", flush=True)
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg3_reduced_system_matches_oracle(scene3, schur3, precision):
    s, prob, st, lin = scene3
    ba = _ba().from_scene(s, precision=precision)
    ba.linearize(LAM)
    tol = 1e-8 if precision == "fp64" else 1e-3
    b, Sc, Sp, Sv = ba.export_reduced()
    b_or = schur3["b"]
    assert np.abs(b - b_or).max() <= tol * np.abs(b_or).max()
    blocks = lm.diag_blocks(prob, schur3["S"])
    for got, key in ((Sc, "cam"), (Sp, "pl"), (Sv, "vp")):
        ref = blocks[key]
        assert len(ref)
        err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
        assert err.max() <= tol, (key, err.max())
    S = schur3["S"]
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = rng.normal(size=prob.nA)
        y = ba.schur_matvec(x)
        err = np.abs(y - S @ x) / np.maximum(np.abs(S) @ np.abs(x), 1e-300)
        assert err.max() <= tol, err.max()
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg3_converged_cost_matches_oracle(precision):
    ref = json.load(open(GOLDEN))["holistic_200cam"]
    s = make_scene(3)
    ba = _ba().from_scene(s, precision=precision)
    out = ba.solve(func_tol=1e-12, max_iters=300, pcg_tol=1e-10 if precision == "fp64" else 1e-8,
                   pcg_max_iters=3000)
    print("[cfg3]", precision, out, ref["E"], flush=True)
    assert abs(out["E_final"] - ref["E"]) <= 1e-6 * ref["E"], (out["E_final"], ref["E"])
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg3_dense_solver(scene3, schur3, precision):
    """The dense solver on the 200-camera scene (2,420 reduced rows): its S
    against the oracle's entry by entry (scaled by sqrt(S_ii S_jj)), then the
    converged cost against the oracle's; the solve's time per LM step beside the
    implicit path's is printed."""
    s, prob, st, lin = scene3
    ba = _ba().from_scene(s, precision=precision)
    ba.linearize(LAM)
    S = ba.export_schur_assembled()
    Sref = schur3["S"]
    d = np.sqrt(np.abs(np.diag(Sref)))
    err = (np.abs(S - Sref) / np.maximum(np.outer(d, d), 1e-300)).max()
    print(f"[cfg3] dense {precision}: assembled S within {err:.2e}", flush=True)
    assert err <= (1e-10 if precision == "fp64" else 1e-4), err
    ba.close()
    ref = json.load(open(GOLDEN))["holistic_200cam"]
    ba = _ba().from_scene(s, precision=precision)
    out = ba.solve(func_tol=1e-12, max_iters=300, solver="dense")
    ms = ba.lm_step(solver="dense")["ms"]
    print("[cfg3] dense", precision, out, ref["E"], "last step ms", ms, flush=True)
    tol = 1e-9 if precision == "fp64" else 1e-6
    assert abs(out["E_final"] - ref["E"]) <= tol * ref["E"], (out["E_final"], ref["E"])
    ba.close()
