"""Pins for the oracle's propagator and observables (CPU only).

* Full subspace (N_aux = N_basis): one step equals scipy's Pade-based
  ``expm`` of -i dt S^{-1} H(t_n + dt/2) (an independent algorithm).
* A = 0: energy and S_sub-orthonormality conserved, and each stationary state
  acquires exactly the phase exp(-i eps_j t) (closed form).
* Time reversal, second-order convergence, linear response symmetry.
* The current equals -(c/Omega) dE/dA at fixed theta (energy functional
  differentiated by finite differences), pinning sign and factor of J.
* Eq. (20) on a 2x2 closed form; the paper's printed speedup tables.
"""

import os

import numpy as np
import pytest
import scipy.linalg

from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def setup0():
    sys = make_system(0)
    phi, eps = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    return sys, phi, eps, sub


def test_full_subspace_step_equals_expm():
    sys = make_system(0)
    d = op.dense_operators(sys, 0)
    nb = sys.n_basis(0)
    phi, eps = ss.ground_state(sys, 0, n_aux=nb)
    sub = ss.project(sys, 0, phi, route="mm")
    a_t, a_mid = pulse_samples(sys, 30)
    # amplify the pulse so that A actually matters at this tolerance
    a_t, a_mid = 400 * a_t, 400 * a_mid
    th0 = np.eye(nb, 3, dtype=complex)
    out = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, keep_theta=True)
    # the same evolution in the original basis with scipy's Pade expm
    c = phi @ th0
    for n in range(30):
        h = op.hamiltonian(d, a_mid[n], sys.c_light)
        u = scipy.linalg.expm(-1j * sys.dt * np.linalg.solve(d["S"], h))
        c = u @ c
        assert np.abs(phi @ out["thetas"][n + 1] - c).max() < 1e-11


def test_stationary_states_acquire_phase_only(setup0):
    sys, phi, eps, sub = setup0
    n = 200
    zeros = np.zeros(n + 1), np.zeros(n)
    th0 = pr.initial_theta(16, 4)
    out = pr.propagate(sub, th0, zeros[0], zeros[1], sys.dt, sys.occ, sys.omega, sys.c_light)
    t = n * sys.dt
    expect = th0 * np.exp(-1j * eps[:4] * t)[None, :]
    assert np.abs(out["theta"] - expect).max() < 1e-11
    assert np.abs(out["E"] - out["E"][0]).max() < 1e-12
    assert np.abs(out["J"] - out["J"][0]).max() < 1e-15
    # no induced current, so no dipole change (Eq. (4)): delta mu stays at the rounding
    # level of what the static current would integrate to over the run
    assert np.abs(out["dmu"]).max() < 1e-12 * sys.omega * t * np.abs(out["J"]).max()


def test_norm_and_energy_conservation_static(setup0):
    """A = 0, arbitrary (non-stationary) initial states."""
    sys, phi, eps, sub = setup0
    rng = np.random.default_rng(4)
    th0 = rng.standard_normal((16, 4)) + 1j * rng.standard_normal((16, 4))
    th0 = th0 @ np.linalg.inv(np.linalg.cholesky(th0.conj().T @ sub["S"] @ th0)).conj().T
    z = np.zeros(301), np.zeros(300)
    out = pr.propagate(sub, th0, z[0], z[1], sys.dt, sys.occ, sys.omega, sys.c_light)
    th = out["theta"]
    assert np.abs(th.conj().T @ sub["S"] @ th - np.eye(4)).max() < 1e-12
    assert np.abs(out["E"] - out["E"][0]).max() < 1e-12 * abs(out["E"][0]) + 1e-13


def test_time_reversal(setup0):
    sys, phi, eps, sub = setup0
    a_t, a_mid = pulse_samples(sys, 80)
    th0 = pr.initial_theta(16, 4)
    fw = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light)
    bw = pr.propagate(sub, fw["theta"], a_t[::-1], a_mid[::-1], -sys.dt, sys.occ, sys.omega, sys.c_light)
    assert np.abs(bw["theta"] - th0).max() < 1e-12


def test_second_order_convergence(setup0):
    sys, phi, eps, sub = setup0
    big = 300.0  # strong field so that the time dependence dominates the error

    def run(dt):
        n = int(round(4.0 / dt))
        t = np.arange(n + 1) * dt
        tm = (np.arange(n) + 0.5) * dt
        f = lambda x: big * 0.01 * np.sin(0.3 * x) * np.exp(-((x - 2.0) / 1.0) ** 2)
        return pr.propagate(sub, pr.initial_theta(16, 4), f(t), f(tm), dt, sys.occ, sys.omega,
                            sys.c_light)["theta"]

    ref = run(0.0025)
    e1 = np.abs(run(0.08) - ref).max()
    e2 = np.abs(run(0.04) - ref).max()
    assert 3.5 < e1 / e2 < 4.5


def test_current_is_energy_derivative(setup0):
    """J = -(c/Omega) dE/dA at fixed theta (velocity gauge: dH/dA = P/c + A S/c^2)."""
    sys, phi, eps, sub = setup0
    rng = np.random.default_rng(8)
    th = rng.standard_normal((16, 4)) + 1j * rng.standard_normal((16, 4))
    a0, h = 0.7, 0.05  # E is quadratic in A: central differences are exact
    e = lambda a: pr.energy(th, pr.h_sub_at(sub, a, sys.c_light), sys.occ)
    de = (e(a0 + h) - e(a0 - h)) / (2 * h)
    j = pr.current(th, sub, a0, sys.occ, sys.omega, sys.c_light)
    assert abs(j - (-(sys.c_light / sys.omega) * de)) < 1e-10 * abs(j)


def test_induced_dipole_linear_response(setup0):
    sys, phi, eps, sub = setup0
    a_t, a_mid = pulse_samples(sys)
    th0 = pr.initial_theta(16, 4)

    def dmu(s):
        return pr.propagate(sub, th0, s * a_t, s * a_mid, sys.dt, sys.occ, sys.omega,
                            sys.c_light)["dmu"]

    d1, d2, dm = dmu(1.0), dmu(2.0), dmu(-1.0)
    assert d1[0] == 0.0
    scale = np.abs(d1).max()
    assert scale > 0
    # dmu(s) = s a + s^2 b + s^3 c + ...: the odd part dominates (linear
    # response) and the even part is second order: d2 - 2 d1 = 2b + 6c = d1 + dm + O(c)
    assert np.abs((d1 - dm) / 2 - d1).max() < 1e-2 * scale
    assert np.abs(d2 - 2 * d1).max() < 5e-2 * scale
    even = np.abs(d1 + dm).max()
    assert even > 0
    assert np.abs((d2 - 2 * d1) - (d1 + dm)).max() < 1e-2 * even


def test_dipole_trapezoid_exact_for_linear_current():
    j = 3.0 + 0.5 * np.arange(11) * 0.1
    dm = pr.dipole_change(j, 0.1, 2.0)
    t = np.arange(11) * 0.1
    assert np.allclose(dm, 2.0 * 0.5 * 0.5 * t * t, atol=1e-15)


def test_critical_timestep_closed_form():
    h = np.diag([-0.3, 0.2])
    s = np.eye(2)
    assert abs(pr.critical_timestep(h, s) - 0.2 / 0.5) < 1e-15
    # generalized: (H, S) with S = diag(2, 1) scales the first eigenvalue
    assert abs(pr.critical_timestep(np.diag([1.0, 3.0]), np.diag([2.0, 1.0])) - 0.2 / 2.5) < 1e-15


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.split())
    return rows


def test_h2_speedup_table_from_paper():
    rows = _read_table("h2_timing_table.txt")
    conv = rows[0]
    t_conv, dt_conv = float(conv[1]), float(conv[2])
    for r in rows[1:]:
        t_mm, t_fft, dtcr, s_mm, s_fft = map(float, r[1:])
        for t, s in ((t_mm, s_mm), (t_fft, s_fft)):
            v = pr.speedup_per_au(t_conv, dt_conv, t, dtcr)
            assert abs(v - s) < 1.0  # printed to integers (rounded, one truncated)


def test_co_per_step_speedups_from_paper():
    rows = _read_table("co_timing_table.txt")
    r4 = [r for r in rows if r[0] == "4.0"][0]
    t_conv, t_mm, t_fft = float(r4[2]), float(r4[3]), float(r4[4])
    assert round(pr.speedup_per_au(t_conv, 1.0, t_mm, 1.0)) == 98
    assert round(pr.speedup_per_au(t_conv, 1.0, t_fft, 1.0)) == 123


def _perturbed(setup0, eps=0.05, seed=7):
    sys, phi, _, sub = setup0
    rng = np.random.default_rng(seed)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    # S-orthonormal start: the Ritz vectors' coefficients, orthonormalised by the exact Cholesky route
    l = np.linalg.cholesky(sub["S"])
    th0 = scipy.linalg.solve_triangular(l.conj().T, th0, lower=False)
    noise = rng.standard_normal(th0.shape) + 1j * rng.standard_normal(th0.shape)
    return th0 + eps * noise, th0, sub["S"]


def test_lowdin_is_s_orthonormal_same_span_and_idempotent(setup0):
    th, th0, s = _perturbed(setup0)
    assert np.abs(pr.state_gram(th0, s) - np.eye(th0.shape[1])).max() < 1e-13
    q = pr.lowdin(th, s)
    assert np.abs(pr.state_gram(q, s) - np.eye(q.shape[1])).max() < 1e-13
    # q lies in the column space of theta: least-squares coefficients reproduce it
    c, *_ = np.linalg.lstsq(th, q, rcond=None)
    assert np.abs(th @ c - q).max() < 1e-12 * np.abs(q).max()
    # an S-orthonormal input is left unchanged; a second application changes nothing
    assert np.abs(pr.lowdin(th0, s) - th0).max() < 1e-13
    assert np.abs(pr.lowdin(q, s) - q).max() < 1e-13


def test_lowdin_is_the_closest_s_orthonormal_set(setup0):
    """Loewdin's set minimises sum_j ||q_j - theta_j||_S over S-orthonormal sets
    spanning theta's space: Gram-Schmidt and rotations of Loewdin's set are farther."""
    th, _, s = _perturbed(setup0, eps=0.2)
    q = pr.lowdin(th, s)

    def dist(x):
        d = x - th
        return float(np.real(np.trace(d.conj().T @ s @ d)))

    # Gram-Schmidt in the S metric: theta R^{-1} with G = R^H R
    r = np.linalg.cholesky(pr.state_gram(th, s)).conj().T
    gs = scipy.linalg.solve_triangular(r.T, th.T, lower=True).T
    assert np.abs(pr.state_gram(gs, s) - np.eye(gs.shape[1])).max() < 1e-12
    assert dist(q) < dist(gs)
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.standard_normal((q.shape[1],) * 2) + 1j * rng.standard_normal((q.shape[1],) * 2)
        u = scipy.linalg.expm(1e-2 * (a - a.conj().T))  # unitary near I
        assert dist(q) < dist(q @ u)
