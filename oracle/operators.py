"""LAPW+LO operators (oracle; test infrastructure only).

H0 = T + V, S, P_z in the LAPW+LO basis of one k-point (Sec. 2.1, Eq. (9)),
built from the interstitial plane-wave part and per-atom muffin-tin blocks
(Sec. 2.3, Eqs. (17)-(19); App. A, Eqs. (A.1)-(A.7)).  The velocity-gauge
Hamiltonian is H(t) = H0 + (A/c) P_z + (A^2/2c^2) S (Sec. 2, Eq. (2), expanded
as in Eq. (15)).

Three independent ways of applying the operators are provided:

* ``dense_operators`` assembles every matrix element (small systems only);
* ``apply_fft`` is matrix-free, interstitial part by FFT convolution
  (Sec. 2.3, second route);
* ``apply_mm`` is matrix-free, interstitial part as a dense convolution matrix
  times the block (Sec. 2.3, first route).
"""

from __future__ import annotations

import numpy as np
import scipy.fft

_WORKERS = -1


def dft(f: np.ndarray) -> np.ndarray:
    """f~(q) = (1/N) sum_j f_j exp(-2 pi i q.j / N) over the last three axes
    (reading R4 of App. A, Eq. (A.7), on the grid)."""
    n = f.shape[-1] * f.shape[-2] * f.shape[-3]
    return scipy.fft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS) / n


def idft(c: np.ndarray) -> np.ndarray:
    """psi_j = sum_q c_q exp(+2 pi i q.j / N) over the last three axes (no 1/N)."""
    n = c.shape[-1] * c.shape[-2] * c.shape[-3]
    return scipy.fft.ifftn(c, axes=(-3, -2, -1), workers=_WORKERS) * n


def grid_index(g: np.ndarray, grid) -> tuple:
    """Index of each integer G triple in a (N3, N2, N1) array: g mod N."""
    n1, n2, n3 = grid
    return (np.mod(g[:, 2], n3), np.mod(g[:, 1], n2), np.mod(g[:, 0], n1))


def conv_matrix(ft: np.ndarray, g: np.ndarray, grid) -> np.ndarray:
    """M[G, G'] = f~(g - g'), the plane-wave matrix of a multiplicative field
    (App. A, Eq. (A.4) interstitial term with Eq. (A.7))."""
    n1, n2, n3 = grid
    d = g[:, None, :].astype(np.int64) - g[None, :, :].astype(np.int64)
    return ft[np.mod(d[..., 2], n3), np.mod(d[..., 1], n2), np.mod(d[..., 0], n1)]


# ---------------------------------------------------------------------------
# Muffin-tin part: per-atom blocks through the matching coefficients.
# ---------------------------------------------------------------------------

def mt_embedding(sys, ik: int, alpha: int) -> np.ndarray:
    """M_alpha = [[A_alpha, 0], [0, E_alpha]]: maps a basis vector onto atom
    alpha's muffin-tin channels (through its matching coefficients) and its
    local orbitals (Sec. 2.3, Eq. (19), the block matrix around the potential)."""
    kp = sys.kpts[ik]
    at = sys.atoms[alpha]
    a_off, l_off = sys.mt_offsets()
    nb = sys.n_basis(ik)
    m = np.zeros((at.size, nb), dtype=np.complex128)
    m[:at.n_mt, :kp.n_g] = kp.A[a_off[alpha]:a_off[alpha] + at.n_mt, :]
    for i in range(at.n_lo):
        m[at.n_mt + i, kp.n_g + l_off[alpha] + i] = 1.0
    return m


def mt_dense(sys, ik: int, blocks) -> np.ndarray:
    """sum_alpha M_alpha^H x_alpha M_alpha over atoms (Eq. (19); App. A,
    Eqs. (A.4)-(A.6) muffin-tin terms; the LO-LAPW block read with ^H, R3)."""
    nb = sys.n_basis(ik)
    out = np.zeros((nb, nb), dtype=np.complex128)
    for alpha in range(sys.n_atoms):
        m = mt_embedding(sys, ik, alpha)
        out += m.conj().T @ blocks[alpha] @ m
    return out


# ---------------------------------------------------------------------------
# Interstitial part.
# ---------------------------------------------------------------------------

def interstitial_dense(sys, ik: int, vr=None):
    """Dense plane-wave blocks (N_G x N_G) of S, T, V, P_z restricted to the
    interstitial: S = Theta~(g-g'), T = 1/2 (G+k).(G'+k) Theta~(g-g') (R6),
    V = (Theta V)~(g-g') (App. A, Eqs. (A.2), (A.4), (A.7)),
    P_z = 1/2 [(G+k)_z + (G'+k)_z] Theta~(g-g') (R7)."""
    kp = sys.kpts[ik]
    vr = sys.vr if vr is None else vr
    th = dft(sys.theta)
    thv = dft(sys.theta * vr)
    s_i = conv_matrix(th, kp.g_int, sys.grid)
    v_i = conv_matrix(thv, kp.g_int, sys.grid)
    gk = kp.gk
    t_i = 0.5 * (gk @ gk.T) * s_i
    p_i = 0.5 * (gk[:, 2][:, None] + gk[:, 2][None, :]) * s_i
    return dict(S=s_i, T=t_i, V=v_i, P=p_i)


def dense_operators(sys, ik: int, vr=None, h=None):
    """All of T, V, P_z, S and H0 = T + V as dense N_basis x N_basis matrices.

    T is the interstitial kinetic part only; the muffin-tin Hamiltonian block
    h_alpha (kinetic + potential inside the sphere) is carried by V, so that V
    is exactly the part rebuilt each step (Sec. 2.3, text after Eq. (16))."""
    kp = sys.kpts[ik]
    ng, nb = kp.n_g, sys.n_basis(ik)
    ii = interstitial_dense(sys, ik, vr)
    h = sys.h if h is None else h

    def pad(x):
        out = np.zeros((nb, nb), dtype=np.complex128)
        out[:ng, :ng] = x
        return out

    ops = dict(
        T=pad(ii["T"]),
        V=pad(ii["V"]) + mt_dense(sys, ik, h),
        P=pad(ii["P"]) + mt_dense(sys, ik, sys.pz),
        S=pad(ii["S"]) + mt_dense(sys, ik, sys.o),
    )
    ops["H0"] = ops["T"] + ops["V"]
    return ops


def hamiltonian(ops: dict, a_z: float, c_light: float):
    """H(A) = H0 + (A/c) P_z + (A^2/2c^2) S (Eq. (2), expanded as in Eq. (15))."""
    return ops["T"] + ops["V"] + (a_z / c_light) * ops["P"] + (a_z * a_z / (2 * c_light ** 2)) * ops["S"]


# ---------------------------------------------------------------------------
# Matrix-free applies.
# ---------------------------------------------------------------------------

def _mt_apply(sys, ik: int, c: np.ndarray, blocks) -> np.ndarray:
    """sum_alpha M_alpha^H (x_alpha (M_alpha C)) without forming M_alpha^H x M_alpha."""
    kp = sys.kpts[ik]
    ng = kp.n_g
    a_off, l_off = sys.mt_offsets()
    out = np.zeros_like(c)
    for alpha, at in enumerate(sys.atoms):
        a = kp.A[a_off[alpha]:a_off[alpha] + at.n_mt, :]
        lo = slice(ng + l_off[alpha], ng + l_off[alpha] + at.n_lo)
        w = np.vstack([a @ c[:ng], c[lo]])
        y = blocks[alpha] @ w
        out[:ng] += a.conj().T @ y[:at.n_mt]
        out[lo] += y[at.n_mt:]
    return out


def _scatter(sys, ik, cg):
    """Place plane-wave coefficients (N_G x n) on the grid: (n, N3, N2, N1)."""
    n1, n2, n3 = sys.grid
    out = np.zeros((cg.shape[1], n3, n2, n1), dtype=np.complex128)
    i3, i2, i1 = grid_index(sys.kpts[ik].g_int, sys.grid)
    out[:, i3, i2, i1] = cg.T
    return out


def _gather(sys, ik, f):
    i3, i2, i1 = grid_index(sys.kpts[ik].g_int, sys.grid)
    return f[:, i3, i2, i1].T


def interstitial_fft(sys, ik: int, cg: np.ndarray, vr=None, chunk: int = 8):
    """Interstitial T, V, P_z, S applied to plane-wave coefficients by FFT
    convolution (Sec. 2.3, second route): transform to real space, multiply by
    the step function (and potential), transform back, read off at G."""
    kp = sys.kpts[ik]
    vr = sys.vr if vr is None else vr
    gk = kp.gk
    theta = sys.theta
    thv = sys.theta * vr
    res = {k: np.zeros(cg.shape, dtype=np.complex128) for k in ("T", "V", "P", "S")}
    for j0 in range(0, cg.shape[1], chunk):
        c = cg[:, j0:j0 + chunk]
        psi = idft(_scatter(sys, ik, c))
        s_g = _gather(sys, ik, dft(theta * psi))
        v_g = _gather(sys, ik, dft(thv * psi))
        t_g = np.zeros_like(c)
        p_g = 0.5 * gk[:, 2][:, None] * s_g
        for i in range(3):
            pi = idft(_scatter(sys, ik, gk[:, i][:, None] * c))
            f_g = _gather(sys, ik, dft(theta * pi))
            t_g += 0.5 * gk[:, i][:, None] * f_g
            if i == 2:
                p_g += 0.5 * f_g
        res["S"][:, j0:j0 + chunk] = s_g
        res["V"][:, j0:j0 + chunk] = v_g
        res["T"][:, j0:j0 + chunk] = t_g
        res["P"][:, j0:j0 + chunk] = p_g
    return res


def interstitial_mm(sys, ik: int, cg: np.ndarray, vr=None):
    """Same quantities as ``interstitial_fft`` by explicit convolution matrices
    (Sec. 2.3, first route).  O(N_G^2) memory: small systems only."""
    ii = interstitial_dense(sys, ik, vr)
    return {k: ii[k] @ cg for k in ("T", "V", "P", "S")}


def apply_ops(sys, ik: int, c: np.ndarray, route: str = "fft", vr=None, h=None) -> dict:
    """T C, V C, P_z C, S C for a block C (N_basis x n) without assembling any
    N_basis^2 matrix (Sec. 2.3, Eqs. (16)-(19))."""
    kp = sys.kpts[ik]
    ng = kp.n_g
    c = np.asarray(c, dtype=np.complex128)
    if route == "fft":
        ii = interstitial_fft(sys, ik, c[:ng], vr)
    elif route == "mm":
        ii = interstitial_mm(sys, ik, c[:ng], vr)
    else:
        raise ValueError(route)
    h = sys.h if h is None else h
    out = {}
    for key, blocks in (("T", None), ("V", h), ("P", sys.pz), ("S", sys.o)):
        x = np.zeros_like(c)
        x[:ng] = ii[key]
        if blocks is not None:
            x += _mt_apply(sys, ik, c, blocks)
        out[key] = x
    return out


def apply_hs(sys, ik: int, c: np.ndarray, a_z: float, route: str = "fft"):
    """H(A) C and S C (Eq. (10) operators; Eq. (2) expanded as Eq. (15))."""
    o = apply_ops(sys, ik, c, route)
    cl = sys.c_light
    hc = o["T"] + o["V"] + (a_z / cl) * o["P"] + (a_z * a_z / (2 * cl * cl)) * o["S"]
    return hc, o["S"]
