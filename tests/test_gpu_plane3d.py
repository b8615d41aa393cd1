"""The 3D point-to-plane distance of the 3D formulation (family 12) on the GPU
against the oracle, through the C ABI.

Two scenes: the tiny holistic scene with its plane-point associations in the 3D
formulation only (weight 100), and with both formulations (weight 1000).  Per-record
residuals and Jacobians (FP64 1e-9, mixed 1e-4), the feature blocks, b, the diagonal
blocks of S and the product entry by entry against the oracle's S, the dense
solver's S, one LM step against the exact Schur step, and ten LM steps of the dense
solver against ten oracle steps.  The formulation has no scale-invariant minimum
(the metric penalty shrinks with the scene while the reprojection terms do not), so
there is no converged cost to compare: LM keeps shrinking the scene on both sides.
"""
import numpy as np
import pytest

from scenegen import make_scene, small_config, plane_3d_scene
from oracle import lm
from oracle.records import record_keys

pytestmark = pytest.mark.gpu

SCENES = {
    "3d_w100": lambda: plane_3d_scene(make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101), 100.0),
    "both_w1000": lambda: plane_3d_scene(make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101),
                                         1000.0, keep_2d=True),
}


def _BA():
    from paper_2609_04026_amd.binding import BA
    return BA


@pytest.fixture(scope="module", params=list(SCENES))
def case(request):
    print(f"[case] {request.param}", flush=True)
    s = SCENES[request.param]()
    prob = lm.Problem(s)
    st = prob.state0()
    lin = lm.linearize(prob, st)
    assert prob.record_count("R12") > 0
    return request.param, s, prob, st, lin


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plane3d_records_match_oracle(case, precision):
    name, s, prob, st, lin = case
    ba = _BA().from_scene(s, precision=precision)
    ba.linearize(1e-3)
    n = prob.record_count("R12")
    assert ba.record_count(12) == n
    keys, r, J = ba.export_records(12)
    ko = record_keys(prob.recs)["R12"][:, 1:]
    og, oo = np.lexsort(keys.T[::-1]), np.lexsort(ko.T[::-1])
    assert np.array_equal(keys[og], ko[oo])
    tol = 1e-9 if precision == "fp64" else 1e-4
    rt = lin.fam["R12"]["rt"][oo]
    err = np.abs(r[og] - rt).max() / max(np.abs(rt).max(), 1e-3)
    assert err <= tol, err
    for b, sl in (("pt", slice(0, 3)), ("pl", slice(3, 6))):
        Jo, Jg = lin.fam["R12"]["J"][b][oo], J[og][:, :, sl]
        e = np.linalg.norm(Jg - Jo, axis=(1, 2)) / np.maximum(np.linalg.norm(Jo, axis=(1, 2)), 1e-30)
        assert e.max() <= tol, (b, e.max())
    ba.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plane3d_reduced_system_matches_oracle(case, precision):
    name, s, prob, st, lin = case
    lam = 1e-3
    ba = _BA().from_scene(s, precision=precision)
    ba.linearize(lam)
    tol = 1e-9 if precision == "fp64" else 1e-4
    Vp, gp, Vl, gl = ba.export_feature_blocks()
    Vp_o, Vl_o, _ = lm.feature_blocks(prob, lin)
    err = np.linalg.norm(Vp - Vp_o, axis=(1, 2)) / np.maximum(np.linalg.norm(Vp_o, axis=(1, 2)), 1e-30)
    assert err.max() <= tol, err.max()
    sys_ = lm.schur(prob, lin, lam)
    S = sys_["S"]
    b, Sc, Sp, Sv = ba.export_reduced()
    assert np.abs(b - sys_["b"]).max() <= 10 * tol * np.abs(sys_["b"]).max()
    blocks = lm.diag_blocks(prob, S)
    e = np.linalg.norm(Sp - blocks["pl"], axis=(1, 2)) / np.linalg.norm(blocks["pl"], axis=(1, 2))
    assert e.max() <= 10 * tol, e.max()
    rng = np.random.default_rng(2)
    for _ in range(3):
        x = rng.normal(size=S.shape[0])
        y = ba.schur_matvec(x)
        err = np.abs(y - S @ x) / np.maximum(np.abs(S) @ np.abs(x), 1e-300)
        assert err.max() <= 10 * tol, err.max()
    Sd = ba.export_schur_assembled()
    d = np.sqrt(np.abs(np.diag(S)))
    assert (np.abs(Sd - S) / np.outer(d, d)).max() <= (1e-10 if precision == "fp64" else 1e-4)
    ba.close()


@pytest.mark.parametrize("precision,solver", [("fp64", "pcg"), ("fp64", "dense"), ("mixed", "pcg")])
def test_plane3d_step_matches_exact_schur_step(case, precision, solver):
    name, s, prob, st, lin = case
    lam = 1e-3
    ba = _BA().from_scene(s, precision=precision)
    rep = ba.lm_step(lambda0=lam, pcg_tol=1e-12 if precision == "fp64" else 1e-7, pcg_max_iters=3000,
                     solver=solver)
    h, _ = lm.solve_schur(prob, lin, lam)
    E0, _ = lm.cost(prob, st)
    E1, Epix1 = lm.cost(prob, prob.retract(st, h))
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert abs(rep["E_before"] - E0) <= 1e-12 * E0
    assert abs(rep["E_after"] - E1) <= tol * E1, (rep["E_after"], E1)
    assert abs(rep["Epix_after"] - Epix1) <= tol * Epix1, (rep["Epix_after"], Epix1)
    ba.close()


def test_plane3d_ten_dense_steps_match_oracle(case):
    name, s, prob, st, lin = case
    ref = lm.lm_solve(prob, max_iters=10, func_tol=0.0, grad_tol=0.0)
    ba = _BA().from_scene(s, precision="fp64")
    out = ba.solve(max_iters=10, func_tol=0.0, grad_tol=0.0, solver="dense")
    print(f"[plane3d] {name}: {out['E_final']} vs {ref['E']} after {out['iters']} / {ref['iters']} attempts",
          flush=True)
    assert out["iters"] == ref["iters"] == 10
    assert abs(out["E_final"] - ref["E"]) <= 1e-9 * ref["E"]
    p = ba.get_parameters()
    assert np.abs(p["points"] - ref["state"].pts).max() <= 1e-7 * np.abs(ref["state"].pts).max()
    ba.close()
