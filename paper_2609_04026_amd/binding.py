"""Thin ctypes binding of libba (include/ba.h): argument marshalling only.

Every step of the bundle-adjustment path runs in the HIP library; this module
converts numpy arrays to pointers and C structs to dicts.  Importing it
without a built libba.so raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# BA_LIB_PATH selects another build of the same library (e.g. a debug build)
LIB_PATH = os.environ.get("BA_LIB_PATH") or os.path.join(_PKG, "libba.so")

BA_OK, BA_E_INVALID, BA_E_STATE, BA_E_OOM, BA_E_DEVICE, BA_E_NUMERIC, BA_E_NOT_CONVERGED = range(7)
STATUS_NAMES = ["BA_OK", "BA_E_INVALID", "BA_E_STATE", "BA_E_OOM", "BA_E_DEVICE", "BA_E_NUMERIC",
                "BA_E_NOT_CONVERGED"]
PREC = {"fp64": 0, "mixed": 1}
PRECOND = {"jacobi": 0, "learned": 1}
PHASES = ["linearize", "feature", "schur", "precond", "pcg", "backsub", "cost"]
FAMILY_ROWS = {1: 2, 2: 4, 3: 2, 4: 4, 5: 3, 6: 1, 7: 1}


class BAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


class Loss(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("scale", c_double), ("weight", c_double)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_cameras", c_int32), ("n_points", c_int32), ("n_lines", c_int32), ("n_planes", c_int32),
                ("n_vps", c_int32), ("camera_dof", c_int32), ("cx", c_double), ("cy", c_double),
                ("cameras", POINTER(c_double)), ("points", POINTER(c_double)), ("lines", POINTER(c_double)),
                ("planes", POINTER(c_double)), ("vps", POINTER(c_double)), ("precision", c_int32),
                ("precond", c_int32), ("hip_stream", c_void_p), ("device", c_int32)]


class SolveOptions(ctypes.Structure):
    _fields_ = [("max_iters", c_int32), ("func_tol", c_double), ("grad_tol", c_double), ("pcg_tol", c_double),
                ("pcg_max_iters", c_int32), ("lambda0", c_double), ("nu0", c_double), ("kappa_max", c_double),
                ("time_kernels", c_int32)]


class StepReport(ctypes.Structure):
    _fields_ = [("E_before", c_double), ("E_after", c_double), ("Epix_before", c_double), ("Epix_after", c_double),
                ("model_decrease", c_double), ("gain_ratio", c_double), ("lambda_", c_double),
                ("accepted", c_int32), ("pcg_iters", c_int32), ("pcg_rel_residual", c_double),
                ("n_fp64_blocks", c_int32), ("relinearized", c_int32), ("ms", c_double * 8),
                ("matvec_ms", c_double), ("matvec_count", c_int32)]


class Summary(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("accepted", c_int32), ("E_initial", c_double), ("E_final", c_double),
                ("Epix_final", c_double), ("termination", c_int32), ("total_ms", c_double),
                ("pcg_iters_total", c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libba.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          "python -m paper_2609_04026_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    D = POINTER(c_double)
    I32 = POINTER(c_int32)
    I64 = POINTER(c_int64)
    sig = {
        "ba_default_options": (None, [POINTER(SolveOptions)]),
        "ba_create": (c_int32, [POINTER(ProblemDesc), POINTER(c_void_p)]),
        "ba_add_observations": (c_int32, [H, c_int32, c_int64, I32, I32, D, POINTER(Loss)]),
        "ba_lm_step": (c_int32, [H, POINTER(SolveOptions), POINTER(StepReport)]),
        "ba_solve": (c_int32, [H, POINTER(SolveOptions), POINTER(Summary)]),
        "ba_get_parameters": (c_int32, [H, D, D, D, D, D]),
        "ba_set_parameters": (c_int32, [H, D, D, D, D, D]),
        "ba_get_lm_state": (c_int32, [H, D, D]),
        "ba_set_lm_state": (c_int32, [H, c_double, c_double]),
        "ba_linearize": (c_int32, [H, c_double]),
        "ba_record_count": (c_int32, [H, c_int32, I64]),
        "ba_export_records": (c_int32, [H, c_int32, I64, D, D]),
        "ba_export_feature_blocks": (c_int32, [H, D, D, D, D]),
        "ba_export_reduced": (c_int32, [H, D, D, D, D]),
        "ba_schur_matvec": (c_int32, [H, D, D]),
        "ba_pcg_solve": (c_int32, [H, c_double, c_int32, D, I32, D]),
        "ba_reduced_dim": (c_int32, [H, I64, I32]),
        "ba_set_gnn_weights": (c_int32, [H, c_void_p, c_size_t]),
        "ba_last_error": (ctypes.c_char_p, [H]),
        "ba_destroy": (None, [H]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def exported_symbols():
    return [n for n in dir(_lib) if n.startswith("ba_")]


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(POINTER(c_double))


def _f64(a, shape_last=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def default_options(**kw) -> SolveOptions:
    o = SolveOptions()
    _lib.ba_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class BA:
    """One holistic BA problem on the GPU (see include/ba.h)."""

    def __init__(self, cameras, points, lines, planes, vps, cx, cy, camera_dof=9, precision="mixed",
                 precond="jacobi", device=0, stream=None):
        self._keep = [_f64(cameras).reshape(-1, 10), _f64(points).reshape(-1, 3), _f64(lines).reshape(-1, 6),
                      _f64(planes).reshape(-1, 4), _f64(vps).reshape(-1, 3)]
        c, p, l, g, v = self._keep
        d = ProblemDesc(len(c), len(p), len(l), len(g), len(v), int(camera_dof), float(cx), float(cy),
                        _dp(c), _dp(p), _dp(l), _dp(g), _dp(v), PREC[precision], PRECOND[precond],
                        c_void_p(stream) if stream else None, int(device))
        h = c_void_p()
        st = _lib.ba_create(ctypes.byref(d), ctypes.byref(h))
        if st != BA_OK:
            raise BAError(st, "ba_create failed")
        self._h = h
        self.n = dict(cam=len(c), pt=len(p), ln=len(l), pl=len(g), vp=len(v))
        self.camera_dof = int(camera_dof)
        self.precision = precision

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            _lib.ba_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st not in (BA_OK,):
            raise BAError(st, (_lib.ba_last_error(self._h) or b"").decode())
        return st

    @classmethod
    def from_scene(cls, scene, precision="mixed", precond="jacobi", device=0, stream=None, losses=True):
        ba = cls(scene["cameras"], scene["points"], scene["lines"], scene["planes"], scene["vps"], scene["cx"],
                 scene["cy"], camera_dof=scene.get("camera_dof", 9), precision=precision, precond=precond,
                 device=device, stream=stream)
        for kind, (a, b, meas) in scene["obs"].items():
            loss = scene["loss"][kind] if losses else None
            ba.add_observations(kind, a, b, meas, loss)
        return ba

    def add_observations(self, kind, a, b, meas=None, loss=None):
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
        m = None if meas is None else np.ascontiguousarray(meas, dtype=np.float64).reshape(-1, 4)
        lo = None if loss is None else ctypes.byref(Loss(int(loss[0]), float(loss[1]), float(loss[2])))
        self._check(_lib.ba_add_observations(self._h, int(kind), len(a), a.ctypes.data_as(POINTER(c_int32)),
                                             b.ctypes.data_as(POINTER(c_int32)), _dp(m), lo))

    # -- solver
    def lm_step(self, **opts):
        o = default_options(**opts)
        r = StepReport()
        self._check(_lib.ba_lm_step(self._h, ctypes.byref(o), ctypes.byref(r)))
        out = {k: getattr(r, k) for k, _ in StepReport._fields_ if k != "ms"}
        out["lambda"] = out.pop("lambda_")
        out["ms"] = {PHASES[i]: r.ms[i] for i in range(len(PHASES))}
        return out

    def solve(self, **opts):
        o = default_options(**opts)
        s = Summary()
        st = _lib.ba_solve(self._h, ctypes.byref(o), ctypes.byref(s))
        if st not in (BA_OK, BA_E_NOT_CONVERGED):
            self._check(st)
        out = {k: getattr(s, k) for k, _ in Summary._fields_}
        out["converged"] = st == BA_OK
        return out

    def get_parameters(self):
        n = self.n
        out = dict(cameras=np.zeros((n["cam"], 10)), points=np.zeros((n["pt"], 3)), lines=np.zeros((n["ln"], 6)),
                   planes=np.zeros((n["pl"], 4)), vps=np.zeros((n["vp"], 3)))
        self._check(_lib.ba_get_parameters(self._h, *(_dp(out[k]) for k in ("cameras", "points", "lines", "planes",
                                                                           "vps"))))
        return out

    def set_parameters(self, cameras=None, points=None, lines=None, planes=None, vps=None):
        arrs = [_f64(x) for x in (cameras, points, lines, planes, vps)]
        self._check(_lib.ba_set_parameters(self._h, *(_dp(a) for a in arrs)))

    def get_lm_state(self):
        lam, nu = c_double(), c_double()
        self._check(_lib.ba_get_lm_state(self._h, ctypes.byref(lam), ctypes.byref(nu)))
        return lam.value, nu.value

    def set_lm_state(self, lam, nu):
        self._check(_lib.ba_set_lm_state(self._h, float(lam), float(nu)))

    # -- inspection
    def linearize(self, lam):
        self._check(_lib.ba_linearize(self._h, float(lam)))

    def record_count(self, fam):
        n = c_int64()
        self._check(_lib.ba_record_count(self._h, int(fam), ctypes.byref(n)))
        return n.value

    def reduced_dim(self):
        n, cd = c_int64(), c_int32()
        self._check(_lib.ba_reduced_dim(self._h, ctypes.byref(n), ctypes.byref(cd)))
        return n.value, cd.value

    def export_records(self, fam):
        n = self.record_count(fam)
        rows = FAMILY_ROWS[fam]
        cd = 0 if fam == 5 else self.camera_dof
        nf = 4 if fam in (2, 4, 5, 7) else 3
        ng = 3 if fam in (3, 4) else 2 if fam == 5 else 0
        keys = np.zeros((n, 3), dtype=np.int64)
        r = np.zeros((n, rows))
        J = np.zeros((n, rows, cd + nf + ng))
        self._check(_lib.ba_export_records(self._h, int(fam), keys.ctypes.data_as(POINTER(c_int64)), _dp(r),
                                           _dp(J)))
        return keys, r, J

    def export_feature_blocks(self):
        n = self.n
        Vp, gp = np.zeros((n["pt"], 3, 3)), np.zeros((n["pt"], 3))
        Vl, gl = np.zeros((n["ln"], 4, 4)), np.zeros((n["ln"], 4))
        self._check(_lib.ba_export_feature_blocks(self._h, _dp(Vp), _dp(gp), _dp(Vl), _dp(gl)))
        return Vp, gp, Vl, gl

    def export_reduced(self):
        nA, cd = self.reduced_dim()
        n = self.n
        b = np.zeros(nA)
        Sc, Sp, Sv = np.zeros((n["cam"], cd, cd)), np.zeros((n["pl"], 3, 3)), np.zeros((n["vp"], 2, 2))
        self._check(_lib.ba_export_reduced(self._h, _dp(b), _dp(Sc), _dp(Sp), _dp(Sv)))
        return b, Sc, Sp, Sv

    def schur_matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        self._check(_lib.ba_schur_matvec(self._h, _dp(x), _dp(y)))
        return y

    def pcg_solve(self, tol=1e-6, max_iters=1000):
        nA, _ = self.reduced_dim()
        x = np.zeros(nA)
        it, rel = c_int32(), c_double()
        self._check(_lib.ba_pcg_solve(self._h, float(tol), int(max_iters), _dp(x), ctypes.byref(it),
                                      ctypes.byref(rel)))
        return x, it.value, rel.value

    def set_gnn_weights(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(_lib.ba_set_gnn_weights(self._h, ctypes.cast(buf, c_void_p), len(blob)))
