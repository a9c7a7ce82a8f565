"""Pins for the oracle's subspace setup (CPU only).

* With Phi the generalized eigenvectors of the dense (H0, S) from LAPACK, the
  matrix-free projection must give S_sub = I and H0_sub = diag(eps).
* Rayleigh-Ritz values are upper bounds of the exact eigenvalues, index by
  index (Courant-Fischer), and the Ritz basis is S-orthonormal.
* The per-step potential rebuild equals Phi^H V' Phi built densely for a
  different potential V'.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import operators as op
from oracle import subspace as ss
from synth import make_system


@pytest.fixture(scope="module")
def sys0():
    return make_system(0)


def test_projection_of_exact_eigenvectors(sys0):
    d = op.dense_operators(sys0, 0)
    eps, w = scipy.linalg.eigh(d["H0"], d["S"])
    phi = w[:, :16]
    sub = ss.project(sys0, 0, phi)
    assert np.abs(sub["S"] - np.eye(16)).max() < 1e-12
    assert np.abs(sub["H0"] - np.diag(eps[:16])).max() < 1e-12
    # T and V separately reproduce the dense quadratic forms
    assert np.abs(sub["T"] - phi.conj().T @ d["T"] @ phi).max() < 1e-13
    assert np.abs(sub["P"] - phi.conj().T @ d["P"] @ phi).max() < 1e-13


def test_ground_state_dense_branch(sys0):
    phi, eps = ss.ground_state(sys0, 0)
    d = op.dense_operators(sys0, 0)
    ev = scipy.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(d["S"]), np.linalg.solve(
        np.linalg.cholesky(d["S"]), d["H0"]).conj().T))
    assert np.allclose(eps, np.sort(ev)[:16], atol=1e-12)
    # residual of the generalized eigenproblem
    r = d["H0"] @ phi - d["S"] @ phi * eps
    assert np.abs(r).max() < 1e-12


def test_ritz_bounds_and_orthonormality(sys0):
    rng = np.random.default_rng(11)
    nb = sys0.n_basis(0)
    x = rng.standard_normal((nb, 24)) + 1j * rng.standard_normal((nb, 24))
    phi, theta = ss.ritz(sys0, 0, x)
    d = op.dense_operators(sys0, 0)
    exact = scipy.linalg.eigh(d["H0"], d["S"], eigvals_only=True)
    assert np.all(theta >= exact[:24] - 1e-12)
    assert np.abs(phi.conj().T @ d["S"] @ phi - np.eye(24)).max() < 1e-12
    assert np.abs(phi.conj().T @ d["H0"] @ phi - np.diag(theta)).max() < 1e-11


def test_rebuild_matches_dense_for_new_potential(sys0):
    phi, _ = ss.ground_state(sys0, 0)
    rng = np.random.default_rng(2)
    v2 = sys0.vr * (1.0 + 0.3 * rng.random(sys0.vr.shape))
    h2 = [h + 0.1 * np.eye(h.shape[0]) for h in sys0.h]
    d = op.dense_operators(sys0, 0, vr=v2, h=h2)
    vsub = ss.rebuild_v_sub(sys0, 0, phi, vr=v2, h=h2)
    assert np.abs(vsub - phi.conj().T @ d["V"] @ phi).max() < 1e-13
    # static potential reproduces the setup projection
    sub = ss.project(sys0, 0, phi)
    assert np.abs(ss.rebuild_v_sub(sys0, 0, phi) - sub["V"]).max() < 1e-14


def test_map_back_and_state_projection(sys0):
    phi, _ = ss.ground_state(sys0, 0)
    sub = ss.project(sys0, 0, phi)
    rng = np.random.default_rng(3)
    th = rng.standard_normal((16, 4)) + 1j * rng.standard_normal((16, 4))
    c = ss.map_back(phi, th)
    sc = op.apply_ops(sys0, 0, c)["S"]
    assert np.abs(ss.project_states(sub, phi, sc) - th).max() < 1e-12
