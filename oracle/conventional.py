"""Conventional propagation in the full LAPW+LO basis (oracle; test
infrastructure only): the coefficient equation S dC/dt = -i H(t) C (Sec. 2.1,
Eq. (10)) without the auxiliary subspace, the reference the paper's speedups
are measured against (Sec. 3.1, Table 1; Sec. 3.2).

The step is the explicit one of the subspace propagator (``propagate.
taylor_propagator``) applied to the full basis: the exponential of
-i dt S^{-1} H(t_n + dt/2) truncated after `order` Taylor terms about the
centre c0 of the full spectrum, times the exact phase exp(-i dt c0).  Its
critical time step is f / (eps_max - eps_min) with the extreme eigenvalues of
the full (H0, S): for the full-basis scheme the limit comes from the spectrum of
the full Hamiltonian rather than that of the subspace one (Sec. 3.1, Eq. (20)
and the discussion of Table 1).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from . import operators as ops


def full_spectrum(d: dict):
    """Extreme generalized eigenvalues of the dense (H0, S)."""
    eps = scipy.linalg.eigh(d["H0"], d["S"], eigvals_only=True)
    return float(eps[0]), float(eps[-1])


def critical_timestep_full(d: dict, f: float = 0.2) -> float:
    """dt_cr = f / (eps_max - eps_min) of the full basis (Eq. (20))."""
    lo, hi = full_spectrum(d)
    return f / (hi - lo)


def taylor_step_full(d: dict, a_z: float, c_light: float, dt: float, order: int, c0: float,
                     c: np.ndarray) -> np.ndarray:
    """One explicit step of C: exp(-i dt c0) sum_{q <= order} (-i dt (S^{-1} H(a) - c0))^q / q! C."""
    h = ops.hamiltonian(d, a_z, c_light)
    term = np.array(c, dtype=np.complex128)
    acc = term.copy()
    for q in range(1, order + 1):
        term = (-1j * dt / q) * (np.linalg.solve(d["S"], h @ term) - c0 * term)
        acc = acc + term
    return np.exp(-1j * dt * c0) * acc


def propagate_full(d: dict, c0_states: np.ndarray, a_mid: np.ndarray, dt: float, order: int, c_light: float,
                   n_steps: int = None, c0: float = None) -> np.ndarray:
    """C after n_steps explicit steps at A(t_n + dt/2); c0 defaults to the centre
    of the full spectrum."""
    n_steps = len(a_mid) if n_steps is None else n_steps
    if c0 is None:
        lo, hi = full_spectrum(d)
        c0 = 0.5 * (lo + hi)
    c = np.array(c0_states, dtype=np.complex128)
    for n in range(n_steps):
        c = taylor_step_full(d, a_mid[n], c_light, dt, order, c0, c)
    return c
