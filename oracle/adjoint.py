"""Discrete adjoint of the subspace propagation (oracle; test infrastructure only).

Loss: the time-integrated induced current, L = dt sum_{n=0}^{N} w_n J_ind,n
with trapezoid weights (w_0 = w_N = 1/2, else 1), so that L = delta mu_z(T) /
Omega (Sec. 2, Eq. (4)).  The gradient is that of the discrete propagation
(discretise, then differentiate) with respect to the sampled vector potential:
A at the midpoints t_n + dt/2 (through the step propagators) and A at t_n
(explicitly, through the current).  For a piecewise-linear pulse the chain rule
maps these onto the knot amplitudes.

Everything is stored (no checkpointing): this is the plain reference.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .propagate import current, emr_propagator, h_sub_at, propagate


def trapezoid_weights(n_steps: int) -> np.ndarray:
    w = np.ones(n_steps + 1)
    w[0] = w[-1] = 0.5
    return w


def loss_from_current(j: np.ndarray, dt: float) -> float:
    """L = dt sum_n w_n (J_n - J_0)."""
    w = trapezoid_weights(len(j) - 1)
    return float(dt * np.sum(w * (j - j[0])))


def propagator_derivative(h_sub, s_sub, dh, dt):
    """dU/da for U = exp(-i dt S^{-1} H(a)) with dH/da = dh (Daleckii-Krein):
    with S = L L^H, L^{-1} H L^{-H} = W diag(lam) W^H and D = W^H L^{-1} dh
    L^{-H} W, dU/da = L^{-H} W (F o D) W^H L^H, where the divided differences
    of exp(-i dt x) are F_ij = -i dt exp(-i dt (lam_i+lam_j)/2)
    sinc(dt (lam_i-lam_j)/2)."""
    l = np.linalg.cholesky(s_sub)
    linv = scipy.linalg.solve_triangular(l, np.eye(l.shape[0]), lower=True)
    ht = linv @ h_sub @ linv.conj().T
    ht = 0.5 * (ht + ht.conj().T)
    lam, w = np.linalg.eigh(ht)
    d = w.conj().T @ (linv @ dh @ linv.conj().T) @ w
    x = 0.5 * dt * (lam[:, None] - lam[None, :])
    f = -1j * dt * np.exp(-0.5j * dt * (lam[:, None] + lam[None, :])) * np.sinc(x / np.pi)
    return linv.conj().T @ w @ (f * d) @ w.conj().T @ l.conj().T


def gradients(sub: dict, theta0, a_t, a_mid, dt, occ, omega, c_light, v_sub_fn=None) -> dict:
    """dL/dA(t_n + dt/2) for every step and dL/dA(t_n) for every time point.

    v_sub_fn(n): V_sub of step n -> n+1 when the potential part is rebuilt every
    step (Sec. 2.3, text after Eq. (16)); it enters the step propagators only,
    not dH/dA.

    Adjoint recursion (real loss, gradient convention dL = Re <mu, d theta>):
    mu_N = dt w_N g_N, mu_n = U_n^H mu_{n+1} + dt w_n g_n with the current's
    gradient g_n = -(2f/Omega) (P_sub + (A_n/c) S_sub) theta_n; the midpoint
    sensitivity is Re <mu_{n+1}, (dU_n/da) theta_n>.  The explicit term is
    dJ_n/dA_n = -(f/(Omega c)) sum_j theta_j^H S_sub theta_j, and the J_0 that
    is subtracted in J_ind contributes -T dJ_0/dA_0 (T = N dt)."""
    n_steps = len(a_mid)
    fw = propagate(sub, theta0, a_t, a_mid, dt, occ, omega, c_light, v_sub_fn=v_sub_fn, keep_theta=True)
    th = fw["thetas"]
    w = trapezoid_weights(n_steps)
    p, s = sub["P"], sub["S"]

    def g_j(n):
        return -(2.0 * occ / omega) * (p + (a_t[n] / c_light) * s) @ th[n]

    def dj_da(n):
        return float(-(occ / (omega * c_light)) * np.real(np.sum(th[n].conj() * (s @ th[n]))))

    d_mid = np.zeros(n_steps)
    d_at = np.zeros(n_steps + 1)
    mu = dt * w[n_steps] * g_j(n_steps)
    for n in range(n_steps - 1, -1, -1):
        hm = h_sub_at(sub, a_mid[n], c_light, None if v_sub_fn is None else v_sub_fn(n))
        dh = p / c_light + (a_mid[n] / c_light ** 2) * s
        du = propagator_derivative(hm, s, dh, dt)
        d_mid[n] = float(np.real(np.sum(mu.conj() * (du @ th[n]))))
        if n > 0:
            u = emr_propagator(hm, s, dt)
            mu = u.conj().T @ mu + dt * w[n] * g_j(n)
    for n in range(n_steps + 1):
        d_at[n] = dt * w[n] * dj_da(n)
    d_at[0] -= n_steps * dt * dj_da(0)
    return dict(mid=d_mid, at=d_at, loss=loss_from_current(fw["J"], dt), J=fw["J"])


def hat_matrix(times: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """phi_k(t) = max(0, 1 - |t - tau_k| / h) on uniform knots tau (spacing h)."""
    h = tau[1] - tau[0]
    return np.maximum(0.0, 1.0 - np.abs(times[:, None] - tau[None, :]) / h)


def knot_gradient(grads: dict, tau: np.ndarray, dt: float) -> np.ndarray:
    """dL/dq_k = sum_n dL/dA(t_n+dt/2) phi_k(t_n+dt/2) + sum_n dL/dA(t_n) phi_k(t_n)."""
    n_steps = len(grads["mid"])
    t = np.arange(n_steps + 1) * dt
    tm = (np.arange(n_steps) + 0.5) * dt
    return hat_matrix(tm, tau).T @ grads["mid"] + hat_matrix(t, tau).T @ grads["at"]
