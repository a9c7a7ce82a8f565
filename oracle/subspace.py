"""Auxiliary-subspace quantities (oracle; test infrastructure only).

Sec. 2.2: the initial Kohn-Sham states Phi = C(0) (N_basis x N_aux) span the
auxiliary subspace, C(t) ~ Phi theta(t) (Eq. (12)), and the Hamiltonian is
projected as H_sub = Phi^H H Phi (Eq. (14)).  Sec. 2.3: H_sub splits into
T_sub + (A/c) P_sub + (A^2/2c^2) S_sub + V_sub(t) (Eqs. (15)-(16)) and only
V_sub(t) is rebuilt each step, as the sum of an interstitial term (Eq. (18))
and a muffin-tin term R^H V R with R = A C_L cached (Eq. (19) and the cost
discussion after it).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from . import operators as ops


def herm(x: np.ndarray) -> np.ndarray:
    """(X + X^H)/2."""
    return 0.5 * (x + x.conj().T)


def project(sys, ik: int, phi: np.ndarray, route: str = "fft") -> dict:
    """T_sub, V_sub, P_sub, S_sub = Phi^H X Phi, each Hermitian-symmetrised
    (Eqs. (14), (16)); H0_sub = T_sub + V_sub."""
    o = ops.apply_ops(sys, ik, phi, route)
    sub = {k: herm(phi.conj().T @ o[k]) for k in ("T", "V", "P", "S")}
    sub["H0"] = sub["T"] + sub["V"]
    return sub


def mt_cache(sys, ik: int, phi: np.ndarray):
    """R_alpha = [A_alpha Phi_G; Phi_LO,alpha] per atom (the cached product
    of the matching coefficients with the LAPW part of the auxiliary basis)."""
    kp = sys.kpts[ik]
    ng = kp.n_g
    a_off, l_off = sys.mt_offsets()
    out = []
    for alpha, at in enumerate(sys.atoms):
        a = kp.A[a_off[alpha]:a_off[alpha] + at.n_mt, :]
        lo = slice(ng + l_off[alpha], ng + l_off[alpha] + at.n_lo)
        out.append(np.vstack([a @ phi[:ng], phi[lo]]))
    return out


def rebuild_v_sub(sys, ik: int, phi: np.ndarray, vr=None, h=None, r_cache=None) -> np.ndarray:
    """V_sub(t) = V^I_sub(t) + V^MT_sub(t) (Eq. (17)).

    Interstitial (Eq. (18)): sum_{GG'} Phi*_{G i} (Theta V)~(g-g') Phi_{G' i'},
    evaluated by FFT convolution.  Muffin-tin (Eq. (19)): sum_alpha R_alpha^H
    h_alpha(t) R_alpha."""
    ng = sys.kpts[ik].n_g
    vr = sys.vr if vr is None else vr
    h = sys.h if h is None else h
    phig = phi[:ng]
    psi = ops.idft(ops._scatter(sys, ik, phig))
    vg = ops._gather(sys, ik, ops.dft(sys.theta * vr * psi))
    v = phig.conj().T @ vg
    rs = mt_cache(sys, ik, phi) if r_cache is None else r_cache
    for alpha in range(sys.n_atoms):
        v = v + rs[alpha].conj().T @ h[alpha] @ rs[alpha]
    return herm(v)


def ritz_rotation(sys, ik: int, x: np.ndarray, route: str = "fft"):
    """The rotation W and Ritz values eps of the Rayleigh-Ritz problem of
    (H0, S) over span(X): (X^H H0 X) W = (X^H S X) W diag(eps),
    W^H (X^H S X) W = I, eps ascending."""
    sub = project(sys, ik, x, route)
    eps, w = scipy.linalg.eigh(sub["H0"], sub["S"])
    return w, eps


def ritz(sys, ik: int, x: np.ndarray, route: str = "fft"):
    """Rayleigh-Ritz vectors Phi = X W of (H0, S) over span(X) (``ritz_rotation``)."""
    w, eps = ritz_rotation(sys, ik, x, route)
    return x @ w, eps


def ground_state(sys, ik: int, n_aux: int = None, dense_max: int = 2500):
    """Stand-in for the ground-state orbitals Phi = C(0) (Sec. 2.2, Eq. (11)).

    Small bases: the lowest n_aux generalized eigenvectors of (H0, S) from the
    dense matrices (S-orthonormal).  Large bases: Rayleigh-Ritz vectors of the
    seeded start block (reading R9)."""
    n_aux = sys.n_aux if n_aux is None else n_aux
    nb = sys.n_basis(ik)
    if nb <= dense_max:
        d = ops.dense_operators(sys, ik)
        eps, w = scipy.linalg.eigh(d["H0"], d["S"], subset_by_index=[0, n_aux - 1])
        return w, eps
    x = sys.kpts[ik].start[:, :n_aux]
    return ritz(sys, ik, x)


def map_back(phi: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """C(t) = Phi theta(t) (Eq. (12))."""
    return phi @ theta


def project_states(sub: dict, phi: np.ndarray, sc: np.ndarray) -> np.ndarray:
    """theta = S_sub^{-1} Phi^H S C: the subspace coefficients of states C
    (the S-orthogonal projection; reduces to <psi_i(0)|psi_j> of Eq. (12)'s
    definition when Phi is S-orthonormal).  ``sc`` is S C."""
    return np.linalg.solve(sub["S"], phi.conj().T @ sc)
