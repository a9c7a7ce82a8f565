"""Subspace time propagation and observables (oracle; test infrastructure only).

The subspace equation (Sec. 2.2, Eq. (13)), carried with the subspace overlap
(reading R2): S_sub d(theta)/dt = -i H_sub(t) theta.  Propagator (reading R1):
exponential midpoint rule, the "simplest" exponential propagator of the
coefficient equation (Sec. 2.1, Eq. (10)) evaluated at t_n + dt/2.

Observables: induced current (reading R8), dipole change by time integration of
the induced current (Sec. 2, Eq. (4)), energy, and the critical time step
(Sec. 3.1, Eq. (20)).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def h_sub_at(sub: dict, a_z: float, c_light: float, v_sub=None) -> np.ndarray:
    """H_sub(t) = T_sub + (A/c) P_sub + (A^2/2c^2) S_sub + V_sub(t) (Eq. (15))."""
    v = sub["V"] if v_sub is None else v_sub
    return sub["T"] + v + (a_z / c_light) * sub["P"] + (a_z * a_z / (2 * c_light ** 2)) * sub["S"]


def emr_propagator(h_sub: np.ndarray, s_sub: np.ndarray, dt: float) -> np.ndarray:
    """U = exp(-i dt S_sub^{-1} H_sub) through S_sub = L L^H and the Hermitian
    eigendecomposition of L^{-1} H_sub L^{-H} = W diag(lam) W^H:
    U = L^{-H} W diag(exp(-i lam dt)) W^H L^H."""
    l = np.linalg.cholesky(s_sub)
    linv = scipy.linalg.solve_triangular(l, np.eye(l.shape[0]), lower=True)
    ht = linv @ h_sub @ linv.conj().T
    ht = 0.5 * (ht + ht.conj().T)
    lam, w = np.linalg.eigh(ht)
    return linv.conj().T @ (w * np.exp(-1j * lam * dt)) @ w.conj().T @ l.conj().T


def spectrum_center(sub: dict) -> float:
    """c0 = (eps_min + eps_max)/2 of the generalized eigenvalues of (H0_sub, S_sub)
    at A = 0: the centre of the spectrum the explicit propagator expands about."""
    eps = scipy.linalg.eigh(sub["H0"], sub["S"], eigvals_only=True)
    return 0.5 * (eps[0] + eps[-1])


def taylor_propagator(h_sub: np.ndarray, s_sub: np.ndarray, dt: float, order: int, c0: float) -> np.ndarray:
    """The explicit, conditionally stable step the paper's O(N_aux^2 N_states) cost
    and its divergence limit dt_cr point to (reading of Sec. 2.2 cost statement and
    Sec. 3.1, Eq. (20)): the exponential of -i dt S^{-1} H truncated after `order`
    terms of its Taylor series about the spectral centre c0,
    U = L^{-H} exp(-i dt c0) [sum_{q=0}^{order} (-i dt (H~ - c0))^q / q!] L^H,
    H~ = L^{-1} H_sub L^{-H}.  The phase exp(-i dt c0) is exact, so the condition
    dt <= f / (eps_max - eps_min) bounds |(lambda - c0) dt| <= f / 2."""
    l = np.linalg.cholesky(s_sub)
    linv = scipy.linalg.solve_triangular(l, np.eye(l.shape[0]), lower=True)
    ht = linv @ h_sub @ linv.conj().T
    ht = 0.5 * (ht + ht.conj().T)
    x = -1j * dt * (ht - c0 * np.eye(ht.shape[0]))
    term = np.eye(ht.shape[0], dtype=np.complex128)
    poly = term.copy()
    for q in range(1, order + 1):
        term = term @ x / q
        poly = poly + term
    return linv.conj().T @ (np.exp(-1j * dt * c0) * poly) @ l.conj().T


def current(theta: np.ndarray, sub: dict, a_z: float, occ: float, omega: float, c_light: float) -> float:
    """J = -(f/Omega) sum_j Re theta_j^H (P_sub + (A/c) S_sub) theta_j (reading R8:
    electrons of charge -1, velocity p + A/c in the velocity gauge)."""
    m = sub["P"] + (a_z / c_light) * sub["S"]
    return float(-(occ / omega) * np.real(np.sum(theta.conj() * (m @ theta))))


def excited_electrons(theta: np.ndarray, s_sub: np.ndarray, n_occ: int, occ: float) -> float:
    """N_exc = f sum_j (<psi_j|psi_j> - sum_{i < n_occ} |<psi_i(0)|psi_j(t)>|^2) with
    psi_i(0) the first n_occ auxiliary functions (the occupied ground states) and
    <psi_i(0)|psi_j(t)> = (S_sub theta_j)_i: the occupation that has left the initially
    occupied states (the number of excited electrons of Secs. 3.2-3.3; the norm
    <psi_j|psi_j> = theta_j^H S_sub theta_j in place of 1 keeps N_exc(0) = 0 exactly)."""
    st = s_sub @ theta
    norms = np.real(np.sum(theta.conj() * st, axis=0))
    occ_part = np.sum(np.abs(st[:n_occ, :]) ** 2, axis=0)
    return float(occ * np.sum(norms - occ_part))


def energy(theta: np.ndarray, h_sub: np.ndarray, occ: float) -> float:
    """E = f sum_j Re theta_j^H H_sub theta_j."""
    return float(occ * np.real(np.sum(theta.conj() * (h_sub @ theta))))


def dipole_change(j: np.ndarray, dt: float, omega: float) -> np.ndarray:
    """delta mu(t_n) = Omega int_0^{t_n} J_ind dt' (Eq. (4)), trapezoid rule on
    the uniform grid, J_ind = J - J(0)."""
    ji = np.asarray(j, float) - j[0]
    out = np.zeros_like(ji)
    out[1:] = omega * dt * np.cumsum(0.5 * (ji[1:] + ji[:-1]))
    return out


def initial_theta(n_aux: int, n_states: int) -> np.ndarray:
    """theta(0) = first N_states unit vectors (reading R9): the occupied states
    are the first auxiliary functions (Sec. 2.2, text after Eq. (12))."""
    th = np.zeros((n_aux, n_states), dtype=np.complex128)
    th[np.arange(n_states), np.arange(n_states)] = 1.0
    return th


def propagate(sub: dict, theta0: np.ndarray, a_t: np.ndarray, a_mid: np.ndarray, dt: float,
              occ: float, omega: float, c_light: float, v_sub_fn=None, n_steps=None,
              keep_theta: bool = False, taylor_order: int = 0) -> dict:
    """Advance theta over n_steps with the exponential midpoint rule (taylor_order
    > 0: the exponential truncated after that many Taylor terms about the spectral
    centre, ``taylor_propagator``).

    AFFINE form (v_sub_fn None): H_sub(t) = H0-part fixed, A enters through
    Eq. (15).  REBUILD form: v_sub_fn(n) returns V_sub for step n -> n+1 (the
    potential handed in for that step, Sec. 2.3 text after Eq. (16)); the energy
    at t_{n+1} uses that same V_sub.

    Returns J_n, E_n, delta mu(t_n) and the excited electrons N_exc(t_n) for
    n = 0..N (the first theta0.shape[1] auxiliary functions taken as the occupied
    ground states), theta_N (and all theta_n if asked)."""
    n_steps = len(a_mid) if n_steps is None else n_steps
    theta = np.array(theta0, dtype=np.complex128)
    j = np.zeros(n_steps + 1)
    e = np.zeros(n_steps + 1)
    v_cur = sub["V"]
    nx = np.zeros(n_steps + 1)
    n_occ = theta.shape[1]
    j[0] = current(theta, sub, a_t[0], occ, omega, c_light)
    e[0] = energy(theta, h_sub_at(sub, a_t[0], c_light, v_cur), occ)
    nx[0] = excited_electrons(theta, sub["S"], n_occ, occ)
    thetas = [theta.copy()] if keep_theta else None
    c0 = spectrum_center(sub) if taylor_order > 0 else 0.0
    for n in range(n_steps):
        if v_sub_fn is not None:
            v_cur = v_sub_fn(n)
        h = h_sub_at(sub, a_mid[n], c_light, v_cur)
        if taylor_order > 0:
            u = taylor_propagator(h, sub["S"], dt, taylor_order, c0)
        else:
            u = emr_propagator(h, sub["S"], dt)
        theta = u @ theta
        j[n + 1] = current(theta, sub, a_t[n + 1], occ, omega, c_light)
        e[n + 1] = energy(theta, h_sub_at(sub, a_t[n + 1], c_light, v_cur), occ)
        nx[n + 1] = excited_electrons(theta, sub["S"], n_occ, occ)
        if keep_theta:
            thetas.append(theta.copy())
    out = dict(J=j, E=e, dmu=dipole_change(j, dt, omega), theta=theta, nexc=nx)
    if keep_theta:
        out["thetas"] = thetas
    return out


def critical_timestep(h_sub: np.ndarray, s_sub: np.ndarray, f: float = 0.2) -> float:
    """dt_cr = f / (eps_max - eps_min), eigenvalues of the subspace Hamiltonian
    (Sec. 3.1, Eq. (20)), f = 0.2."""
    eps = scipy.linalg.eigh(h_sub, s_sub, eigvals_only=True)
    return f / (eps[-1] - eps[0])


def speedup_per_au(t_ref: float, dtcr_ref: float, t_new: float, dtcr_new: float) -> float:
    """Overall speedup over a fixed simulated time window (Sec. 3.1): the ratio
    of wall time per simulated a.u., (t_ref/dtcr_ref) / (t_new/dtcr_new)."""
    return (t_ref / dtcr_ref) / (t_new / dtcr_new)


def state_gram(theta: np.ndarray, s_sub: np.ndarray) -> np.ndarray:
    """G = theta^H S_sub theta, the overlap of the propagated states in the
    subspace metric (the exact propagator keeps G = I: Sec. 2.2, the states stay
    S-orthonormal)."""
    return theta.conj().T @ s_sub @ theta


def lowdin(theta: np.ndarray, s_sub: np.ndarray) -> np.ndarray:
    """Loewdin's symmetric orthonormalisation in the S_sub metric, theta G^{-1/2}
    with G = theta^H S_sub theta: the S-orthonormal set spanning the same space
    that is closest to theta (the reorthonormalisation of the mixed-precision
    extension; not in the paper)."""
    g = state_gram(theta, s_sub)
    w, v = np.linalg.eigh(0.5 * (g + g.conj().T))
    return theta @ ((v / np.sqrt(w)) @ v.conj().T)
