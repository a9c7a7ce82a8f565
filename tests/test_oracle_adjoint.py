"""Pins for the oracle's discrete adjoint (CPU only).

* The Daleckii-Krein derivative of the step propagator against central
  differences of the propagator itself.
* The knot gradient of the time-integrated induced current against central
  finite differences of the forward loss on every knot.
* L = delta mu_z(T) / Omega (Eq. (4) at the final time).
"""

import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples
from synth.lapw_inputs import knot_times, knot_values


@pytest.fixture(scope="module")
def knot_setup():
    sys = make_system(0, n_steps=60, pulse=dict(kind="knots", n_knots=8, base=dict(
        kind="gauss_sin", amp=0.01, omega=0.3, t0=3.0, width=1.5)))
    phi, eps = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    return sys, sub


def _loss(sys, sub, q):
    a_t, a_mid = pulse_samples(sys, knots=q)
    out = pr.propagate(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                       sys.occ, sys.omega, sys.c_light)
    return ad.loss_from_current(out["J"], sys.dt), out


def test_propagator_derivative_matches_fd(knot_setup):
    sys, sub = knot_setup
    a0, h = 0.3, 1e-4
    dh = sub["P"] / sys.c_light + (a0 / sys.c_light ** 2) * sub["S"]
    du = ad.propagator_derivative(pr.h_sub_at(sub, a0, sys.c_light), sub["S"], dh, 0.7)
    up = pr.emr_propagator(pr.h_sub_at(sub, a0 + h, sys.c_light), sub["S"], 0.7)
    um = pr.emr_propagator(pr.h_sub_at(sub, a0 - h, sys.c_light), sub["S"], 0.7)
    fd = (up - um) / (2 * h)
    assert np.abs(du - fd).max() < 1e-7 * np.abs(du).max()


def test_loss_is_final_dipole_over_volume(knot_setup):
    sys, sub = knot_setup
    t_end = sys.n_steps * sys.dt
    q = knot_values(sys.pulse, t_end)
    loss, out = _loss(sys, sub, q)
    assert abs(loss - out["dmu"][-1] / sys.omega) < 1e-15 + 1e-12 * abs(loss)


def test_knot_gradient_matches_central_fd(knot_setup):
    sys, sub = knot_setup
    t_end = sys.n_steps * sys.dt
    tau = knot_times(sys.pulse["n_knots"], t_end)
    q = knot_values(sys.pulse, t_end)
    a_t, a_mid = pulse_samples(sys, knots=q)
    g = ad.gradients(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                     sys.occ, sys.omega, sys.c_light)
    grad = ad.knot_gradient(g, tau, sys.dt)
    h = 1e-4
    fd = np.zeros_like(q)
    for k in range(len(q)):
        e = np.zeros_like(q)
        e[k] = h
        fd[k] = (_loss(sys, sub, q + e)[0] - _loss(sys, sub, q - e)[0]) / (2 * h)
    assert np.linalg.norm(grad - fd) < 1e-6 * np.linalg.norm(fd)
    # first knot: the J_0 subtraction makes its gradient differ from the bare sum
    assert abs(fd[0]) > 0


def test_directional_derivative(knot_setup):
    """Tangent-linear check: <grad, v> against a directional central difference."""
    sys, sub = knot_setup
    t_end = sys.n_steps * sys.dt
    tau = knot_times(sys.pulse["n_knots"], t_end)
    q = knot_values(sys.pulse, t_end)
    a_t, a_mid = pulse_samples(sys, knots=q)
    g = ad.gradients(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                     sys.occ, sys.omega, sys.c_light)
    grad = ad.knot_gradient(g, tau, sys.dt)
    v = np.random.default_rng(1).standard_normal(q.shape)
    h = 1e-3
    fd = (_loss(sys, sub, q + h * v)[0] - _loss(sys, sub, q - h * v)[0]) / (2 * h)
    assert abs(grad @ v - fd) < 1e-6 * abs(fd)


def test_knot_gradient_with_rebuilt_potential_matches_fd(knot_setup):
    """REBUILD form: a V_sub that changes every step enters each step's propagator;
    the adjoint must use the same V_sub(n) in its backward sweep."""
    sys, sub = knot_setup
    t_end = sys.n_steps * sys.dt
    tau = knot_times(sys.pulse["n_knots"], t_end)
    q = knot_values(sys.pulse, t_end)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(sub["V"].shape) + 1j * rng.standard_normal(sub["V"].shape)
    dv = 0.05 * (x + x.conj().T) * np.abs(sub["V"]).max() / np.abs(x).max()

    def vfn(n):
        return sub["V"] + np.sin(0.2 * n) * dv

    def loss(qq):
        a_t, a_mid = pulse_samples(sys, knots=qq)
        out = pr.propagate(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                           sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
        return ad.loss_from_current(out["J"], sys.dt)

    a_t, a_mid = pulse_samples(sys, knots=q)
    g = ad.gradients(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                     sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    assert abs(g["loss"] - loss(q)) < 1e-14 + 1e-12 * abs(g["loss"])
    grad = ad.knot_gradient(g, tau, sys.dt)
    h = 1e-4
    fd = np.array([(loss(q + h * e) - loss(q - h * e)) / (2 * h) for e in np.eye(len(q))])
    assert np.linalg.norm(grad - fd) < 1e-6 * np.linalg.norm(fd)
    # the static-potential gradient differs: the test sees the per-step V_sub
    g0 = ad.knot_gradient(ad.gradients(sub, pr.initial_theta(sys.n_aux, sys.n_states), a_t, a_mid, sys.dt,
                                       sys.occ, sys.omega, sys.c_light), tau, sys.dt)
    assert np.linalg.norm(g0 - fd) > 1e-4 * np.linalg.norm(fd)
