"""The no-allocation dense export against the allocating one, through the C ABI.

Two calls in a row on one GPU share its scratch panel: first the 200-camera
scene (n_A = 2,420: twelve column panels, the last one partial), then a tiny
scene (one panel), each against ba_export_schur_dense of the same handle.
Both exports form every column with the same implicit-Schur product, whose
FP64 sums run in a run-dependent order, so they agree to rounding (1e-12 of
the largest entry) rather than bit for bit.
"""
import numpy as np
import pytest

from scenegen import make_scene, small_config

pytestmark = pytest.mark.gpu


def _compare(scene, precision):
    from paper_2609_04026_amd.binding import BA
    ba = BA.from_scene(scene, precision=precision)
    ba.linearize(1e-3)
    nA, _ = ba.reduced_dim()
    print(f"[no-alloc] n_A={nA} precision={precision}", flush=True)
    S_ref = ba.export_schur_dense()
    S = ba.export_schur_dense_noalloc()
    ba.close()
    scale = np.abs(S_ref).max()
    assert scale > 0 and np.all(np.isfinite(S))
    assert np.abs(S - S_ref).max() <= 1e-12 * scale, np.abs(S - S_ref).max() / scale
    return nA


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_dense_export_matches_allocating_export(precision):
    n1 = _compare(make_scene(3), precision)
    n2 = _compare(make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101), precision)
    assert n1 == 2420 and n2 < n1


def test_noalloc_dense_export_rejects_oversize_and_early_calls():
    from paper_2609_04026_amd import binding
    from paper_2609_04026_amd.binding import BA
    n_cams = (1 << 19) // 9 + 1  # n_A = 9 n_cams > 2^19
    cams = np.zeros((n_cams, 10))
    cams[:, 0] = 1.0
    cams[:, 6] = 10.0
    cams[:, 7] = 500.0
    ba = BA(cams, np.zeros((0, 3)), np.zeros((0, 6)), np.zeros((0, 4)), np.zeros((0, 3)), 320.0, 240.0,
            precision="fp64")
    # the C entry point directly: both errors are raised before anything is written,
    # so a one-element output buffer is enough
    out = np.zeros(1)
    st = binding._lib.ba_export_schur_dense_noalloc(ba._h, binding._dp(out))
    assert st == 2  # BA_E_STATE: no linearisation yet
    ba.linearize(1e-3)
    st = binding._lib.ba_export_schur_dense_noalloc(ba._h, binding._dp(out))
    assert st == 1 and b"no-allocation limit" in binding._lib.ba_last_error(ba._h)
    assert out[0] == 0.0
    ba.close()
