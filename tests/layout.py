"""Test helpers: oracle parameters and records in the library's device layouts.

Used only by tests that evaluate the library's math templates on the host.
"""
import numpy as np

from oracle import model


def cam_slot(st, i):
    s = np.zeros(16)
    s[0:9] = st.cam_R[i].reshape(9)
    s[9:12] = st.cam_t[i]
    s[12:15] = st.cam_f[i], st.cam_k1[i], st.cam_k2[i]
    return s


def pt_slot(st, j):
    s = np.zeros(4)
    s[0:3] = st.pts[j]
    return s


def ln_slot(st, k):
    s = np.zeros(12)
    U = st.line_U[k]
    s[0:3], s[3:6], s[6:9] = U[:, 0], U[:, 1], U[:, 2]
    s[9:11] = st.line_w[k]
    return s


def pl_slot(st, g):
    s = np.zeros(12)
    s[0:3] = st.pl_n[g]
    s[3] = st.pl_w[g]
    B = model.s2_basis(st.pl_n[g])
    s[4:7], s[7:10] = B[:, 0], B[:, 1]
    return s


def vp_slot(st, v):
    s = np.zeros(12)
    s[0:3] = st.vp[v]
    B = model.s2_basis(st.vp[v])
    s[4:7], s[7:10] = B[:, 0], B[:, 1]
    return s


def sh_slot(st, i):
    """Shape i in the device layout (SH_STRIDE = 16 doubles, the type at [15])."""
    from oracle import shapes as S
    sh = st.sh
    s = np.zeros(16)
    t = int(sh.type[i])
    s[15] = t
    if t == S.SPHERE:
        s[0:3], s[3] = sh.c[i], sh.q[i, 0]
    elif t == S.CYLINDER:
        U = sh.R[i]
        s[0:3], s[3:6], s[6:9] = U[:, 0], U[:, 1], U[:, 2]
        s[9:11], s[11] = sh.w[i], sh.q[i, 0]
    elif t == S.CONE:
        B = model.s2_basis(sh.d[i])
        s[0:3], s[3:6], s[6:9], s[9:12], s[12] = sh.c[i], sh.d[i], B[:, 0], B[:, 1], sh.q[i, 0]
    elif t == S.ELLIPSOID:
        s[0:9], s[9:12], s[12:15] = sh.R[i].reshape(9), sh.c[i], sh.q[i, 0:3]
    else:
        s[0:9], s[9:15] = sh.R[i].reshape(9), sh.q[i, 0:6]
    return s


def shifted_meas(fam, rec, i, cx, cy):
    """Measurement of record i as the library stores it (shifted by the
    principal point; the observed line of R6 normalised)."""
    m = np.zeros(4)
    if fam == "R1":
        m[0:2] = rec["meas"][i] - [cx, cy]
    elif fam in ("R2", "R4", "R14"):
        m[0:4] = rec["meas"][i] - [cx, cy, cx, cy]
    elif fam == "R6":
        e = rec["meas"][i] - [cx, cy, cx, cy]
        l = np.cross([e[0], e[1], 1.0], [e[2], e[3], 1.0])
        m[0:3] = l / np.hypot(l[0], l[1])
    elif fam == "R7":
        m[0:2] = rec["meas"][i] - [cx, cy]
    return m
