"""The pins must fail on plausible mistakes.  Each test plants one mistake in
the oracle (monkeypatched, CPU only) and checks that the corresponding pin's
comparison would no longer pass."""

import numpy as np
import pytest

from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system
from tests.test_oracle_operators import brute_operators, rel, tiny_system


@pytest.fixture(scope="module")
def tiny():
    return tiny_system()


def test_flipped_momentum_sign_is_caught(tiny, monkeypatch):
    orig = op.hamiltonian
    monkeypatch.setattr(op, "hamiltonian", lambda d, a, c: orig(d, -a, c))
    h_ref, _ = brute_operators(tiny, 1, 0.9)
    assert rel(op.hamiltonian(op.dense_operators(tiny, 1), 0.9, tiny.c_light), h_ref) > 1e-6


def test_transposed_convolution_is_caught(tiny, monkeypatch):
    orig = op.conv_matrix
    monkeypatch.setattr(op, "conv_matrix", lambda ft, g, grid: orig(ft, g, grid).T)
    _, s_ref = brute_operators(tiny, 1, 0.0)
    assert rel(op.dense_operators(tiny, 1)["S"], s_ref) > 1e-6


def test_dropped_local_orbitals_are_caught(tiny, monkeypatch):
    orig = op.mt_embedding

    def no_lo(sys, ik, alpha):
        m = orig(sys, ik, alpha)
        m[sys.atoms[alpha].n_mt:, :] = 0.0
        return m

    monkeypatch.setattr(op, "mt_embedding", no_lo)
    h_ref, _ = brute_operators(tiny, 1, 0.0)
    assert rel(op.hamiltonian(op.dense_operators(tiny, 1), 0.0, tiny.c_light), h_ref) > 1e-6


def test_left_endpoint_pulse_is_caught():
    """Evaluating H at t_n instead of t_n + dt/2 drops the order to one."""
    sys = make_system(0)
    phi, eps = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    f = lambda x: 3.0 * np.sin(0.3 * x) * np.exp(-((x - 2.0) / 1.0) ** 2)

    def run(dt, shift):
        n = int(round(4.0 / dt))
        t = np.arange(n + 1) * dt
        tm = (np.arange(n) + shift) * dt
        return pr.propagate(sub, pr.initial_theta(16, 4), f(t), f(tm), dt, sys.occ, sys.omega,
                            sys.c_light)["theta"]

    ref = run(0.0025, 0.5)
    ratio = np.abs(run(0.08, 0.0) - ref).max() / np.abs(run(0.04, 0.0) - ref).max()
    assert not (3.5 < ratio < 4.5)


def test_wrong_current_sign_is_caught(monkeypatch):
    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    orig = pr.current
    monkeypatch.setattr(pr, "current", lambda th, s, a, f, o, c: -orig(th, s, a, f, o, c))
    rng = np.random.default_rng(8)
    th = rng.standard_normal((16, 4)) + 1j * rng.standard_normal((16, 4))
    e = lambda a: pr.energy(th, pr.h_sub_at(sub, a, sys.c_light), sys.occ)
    de = (e(0.75) - e(0.65)) / 0.1
    j = pr.current(th, sub, 0.7, sys.occ, sys.omega, sys.c_light)
    assert abs(j - (-(sys.c_light / sys.omega) * de)) > 1e-3 * abs(j)


@pytest.mark.parametrize("power", [-1.0, 0.5, -0.25])
def test_wrong_lowdin_power_is_caught(power):
    """theta G^p with p != -1/2 fails the S-orthonormality pin."""
    from tests.test_oracle_propagate import _perturbed

    sys = make_system(0)
    phi, eps = ss.ground_state(sys, 0)
    th, _, s = _perturbed((sys, phi, eps, ss.project(sys, 0, phi)))
    g = pr.state_gram(th, s)
    w, v = np.linalg.eigh(0.5 * (g + g.conj().T))
    q = th @ ((v * w**power) @ v.conj().T)
    assert np.abs(pr.state_gram(q, s) - np.eye(q.shape[1])).max() > 1e-6


def test_unconjugated_lowdin_gram_is_caught():
    """G = theta^T S theta (conjugate dropped) fails the same pin."""
    from tests.test_oracle_propagate import _perturbed

    sys = make_system(0)
    phi, eps = ss.ground_state(sys, 0)
    th, _, s = _perturbed((sys, phi, eps, ss.project(sys, 0, phi)))
    g = th.T @ s @ th
    w, v = np.linalg.eig(g)
    q = th @ (v @ np.diag(1.0 / np.sqrt(w)) @ np.linalg.inv(v))
    assert np.abs(pr.state_gram(q, s) - np.eye(q.shape[1])).max() > 1e-6
