"""Pins for the oracle's explicit (truncated Taylor) subspace propagator, the
scheme that the paper's O(N_aux^2 N_states) cost and its critical time step
(Sec. 3.1, Eq. (20)) point to (CPU only).

* Order 4 equals the classical Runge-Kutta method applied to the shifted linear
  equation d(theta~)/dt = -i (H~ - c0) theta~ (an independent algorithm:
  the four stages written out), times the exact phase exp(-i dt c0).
* Local error against the exact exponential scales as dt^(order+1).
* A high order reproduces the exact exponential (the EMR step) to rounding.
* Stability: at dt <= dt_cr the S-norm of every state does not grow; far beyond
  the stability limit of the order-4 polynomial (|(lambda - c0) dt| > 2 sqrt 2)
  it grows without bound (the divergence dt_cr guards against).
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples


@pytest.fixture(scope="module")
def sub0():
    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    # a non-orthonormal basis (mixes the auxiliary functions) so that S_sub != I
    rng = np.random.default_rng(3)
    mix = np.eye(16) + 0.1 * (rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))
    return sys, ss.project(sys, 0, phi @ mix)


def _h(sys, sub, a):
    return pr.h_sub_at(sub, a, sys.c_light)


def test_order4_equals_classical_rk4(sub0):
    sys, sub = sub0
    c0 = pr.spectrum_center(sub)
    h = _h(sys, sub, 0.7)
    dt = 0.05
    l = np.linalg.cholesky(sub["S"])
    linv = scipy.linalg.solve_triangular(l, np.eye(16), lower=True)
    ht = linv @ h @ linv.conj().T
    ht = 0.5 * (ht + ht.conj().T)
    rng = np.random.default_rng(4)
    th = rng.standard_normal((16, 3)) + 1j * rng.standard_normal((16, 3))
    # RK4 on y' = f(y) = -i (H~ - c0) y, y = L^H theta
    f = lambda y: -1j * (ht - c0 * np.eye(16)) @ y
    y = l.conj().T @ th
    k1 = f(y)
    k2 = f(y + 0.5 * dt * k1)
    k3 = f(y + 0.5 * dt * k2)
    k4 = f(y + dt * k3)
    y1 = y + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    ref = linv.conj().T @ (np.exp(-1j * dt * c0) * y1)
    got = pr.taylor_propagator(h, sub["S"], dt, 4, c0) @ th
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("order", [2, 4])
def test_local_error_order(sub0, order):
    sys, sub = sub0
    c0 = pr.spectrum_center(sub)
    h = _h(sys, sub, 0.3)
    errs = []
    for dt in (0.04, 0.02):
        d = pr.taylor_propagator(h, sub["S"], dt, order, c0) - pr.emr_propagator(h, sub["S"], dt)
        errs.append(np.abs(d).max())
    ratio = errs[0] / errs[1]
    assert abs(np.log2(ratio) - (order + 1)) < 0.25, ratio


def test_high_order_is_exact_exponential(sub0):
    sys, sub = sub0
    c0 = pr.spectrum_center(sub)
    h = _h(sys, sub, -0.4)
    u = pr.taylor_propagator(h, sub["S"], 0.1, 30, c0)
    ue = pr.emr_propagator(h, sub["S"], 0.1)
    assert np.abs(u - ue).max() < 1e-13


def test_stable_below_dt_cr_and_diverges_far_above(sub0):
    sys, sub = sub0
    dtcr = pr.critical_timestep(sub["H0"], sub["S"])
    n = 200
    a_t, a_mid = pulse_samples(sys, n)
    z = np.zeros_like
    th0 = pr.initial_theta(16, 4)
    g = lambda th: np.real(np.diag(pr.state_gram(th, sub["S"])))
    out = pr.propagate(sub, th0, z(a_t), z(a_mid), dtcr, sys.occ, sys.omega, sys.c_light, n_steps=n,
                       taylor_order=4)
    assert np.all(g(out["theta"]) <= g(th0) * (1.0 + 1e-12))
    assert np.all(g(out["theta"]) >= g(th0) * (1.0 - 1e-4))  # damping of the polynomial, not a collapse
    # |(lambda - c0) dt| = 3 > 2 sqrt 2 at the spectrum's edges: amplification per step
    eps = scipy.linalg.eigh(sub["H0"], sub["S"], eigvals_only=True)
    dt_big = 6.0 / (eps[-1] - eps[0])
    th1 = np.zeros((16, 1), complex)
    th1[-1, 0] = 1.0  # the highest state: the largest |lambda - c0|
    out = pr.propagate(sub, th1, z(a_t), z(a_mid), dt_big, sys.occ, sys.omega, sys.c_light, n_steps=40,
                       taylor_order=4)
    assert g(out["theta"])[0] > 1e3 * g(th1)[0]


def test_excited_electrons_rabi_closed_form():
    """Two auxiliary functions, H = [[0, v], [v, D]], one state starting in the
    first: the occupation of the second is (4 v^2 / W^2) sin^2(W t / 2),
    W = sqrt(D^2 + 4 v^2) (Rabi), so N_exc(t) = f times that."""
    v, d = 0.07, 0.3
    sub = dict(T=np.array([[0.0, v], [v, d]], complex), V=np.zeros((2, 2), complex),
               P=np.zeros((2, 2), complex), S=np.eye(2, dtype=complex))
    sub["H0"] = sub["T"] + sub["V"]
    n, dt = 120, 0.25
    z = np.zeros(n + 1)
    out = pr.propagate(sub, np.array([[1.0], [0.0]], complex), z, z[:n], dt, 2.0, 1.0, 137.0)
    t = np.arange(n + 1) * dt
    w = np.sqrt(d * d + 4 * v * v)
    ref = 2.0 * (4 * v * v / (w * w)) * np.sin(w * t / 2) ** 2
    assert np.abs(out["nexc"] - ref).max() < 1e-12


def test_excited_electrons_zero_for_stationary_states(sub0):
    sys, _ = sub0
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    z = np.zeros(41)
    out = pr.propagate(sub, pr.initial_theta(16, 4), z, z[:40], 0.1, sys.occ, sys.omega, sys.c_light)
    assert np.abs(out["nexc"]).max() < 1e-12
