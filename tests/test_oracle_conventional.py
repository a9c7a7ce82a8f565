"""Pins for the oracle's conventional (full-basis) propagation (CPU only).

* With the auxiliary basis complete (N_aux = N_basis, the full eigenbasis), one
  full-basis step equals the subspace explicit step mapped back (two
  formulations: dense S^{-1} H against the Cholesky-reduced subspace matrix).
* Local error against scipy's expm of -i dt S^{-1} H scales as dt^(order+1).
* dt_cr of the full basis is far below the subspace one (the high plane waves),
  the S-norm does not grow at dt_cr and diverges far beyond it.
"""

import numpy as np
import scipy.linalg

from oracle import conventional as cv
from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system


def _setup():
    sys = make_system(0)
    d = op.dense_operators(sys, 0)
    return sys, d


def test_full_step_equals_complete_subspace_step():
    sys, d = _setup()
    nb = sys.n_basis(0)
    phi, _ = ss.ground_state(sys, 0, n_aux=nb)
    sub = ss.project(sys, 0, phi, route="mm")
    rng = np.random.default_rng(61)
    th = rng.standard_normal((nb, 3)) + 1j * rng.standard_normal((nb, 3))
    c = phi @ th
    a, dt, c0 = 0.8, 0.01, 0.7
    got = cv.taylor_step_full(d, a, sys.c_light, dt, 4, c0, c)
    ref = phi @ (pr.taylor_propagator(pr.h_sub_at(sub, a, sys.c_light), sub["S"], dt, 4, c0) @ th)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_full_step_order_of_accuracy():
    sys, d = _setup()
    rng = np.random.default_rng(62)
    c = rng.standard_normal((sys.n_basis(0), 2)) + 1j * rng.standard_normal((sys.n_basis(0), 2))
    lo, hi = cv.full_spectrum(d)
    c0 = 0.5 * (lo + hi)
    h = op.hamiltonian(d, 0.3, sys.c_light)
    errs = []
    for dt in (0.04, 0.02):
        u = scipy.linalg.expm(-1j * dt * np.linalg.solve(d["S"], h))
        errs.append(np.abs(cv.taylor_step_full(d, 0.3, sys.c_light, dt, 4, c0, c) - u @ c).max())
    assert abs(np.log2(errs[0] / errs[1]) - 5.0) < 0.3, errs


def test_full_dt_cr_and_stability():
    sys, d = _setup()
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    dt_full = cv.critical_timestep_full(d)
    dt_sub = pr.critical_timestep(sub["H0"], sub["S"])
    assert dt_full < dt_sub
    rng = np.random.default_rng(63)
    c = rng.standard_normal((sys.n_basis(0), 2)) + 1j * rng.standard_normal((sys.n_basis(0), 2))
    norm = lambda x: np.real(np.diag(x.conj().T @ d["S"] @ x))
    z = np.zeros(200)
    out = cv.propagate_full(d, c, z, dt_full, 4, sys.c_light)
    assert np.all(norm(out) <= norm(c) * (1 + 1e-12))
    lo, hi = cv.full_spectrum(d)
    out = cv.propagate_full(d, c, z[:40], 6.0 / (hi - lo), 4, sys.c_light)
    assert np.all(norm(out) > 1e3 * norm(c))
