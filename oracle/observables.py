"""Pulses and spectra of the real-time propagation (oracle; test infrastructure
only).

* Vector potentials of the paper's two excitations: the impulsive kick of the
  polarizability runs (Sec. 3.1) and the sin^2-envelope laser (Sec. 3.2),
  A(t) = A0 cos(w t) sin^2[pi (t - t0)/T_p] e_z for t0 <= t <= t0 + T_p.
* The dynamical polarizability alpha_zz(w) = (i Omega / w) J(w) / E(w) from the
  induced current and the field, both taken to the frequency domain (Sec. 2,
  Eq. (5)), with E(t) = -(1/c) dA/dt (velocity gauge, Eq. (2)).

Readings where the paper is silent (listed with the others in the design notes):

* the kick: E(t) = E0 delta(t - 0+), so A(t) = -c E0 for t > 0 and A(0) = 0;
* the transforms are sums over the time grid with an exponential damping
  exp(-gamma t) (a broadening the paper's spectra imply but do not state):
  J(w) = dt sum_n w_n J_ind(t_n) exp((i w - gamma) t_n) with trapezoid weights
  (w_0 = w_N = 1/2), and E(w) = sum_n E(t_{n+1/2}) exp((i w - gamma) t_{n+1/2}) dt
  with E(t_{n+1/2}) = -(A(t_{n+1}) - A(t_n)) / (c dt), the field of the sampled A.
"""

from __future__ import annotations

import numpy as np


def pulse_sin2(t: np.ndarray, a0: float, w: float, t0: float, tp: float) -> np.ndarray:
    """A(t) = A0 cos(w t) sin^2[pi (t - t0)/T_p] inside [t0, t0 + T_p], 0 outside (Sec. 3.2)."""
    t = np.asarray(t, float)
    inside = (t >= t0) & (t <= t0 + tp)
    return np.where(inside, a0 * np.cos(w * t) * np.sin(np.pi * (t - t0) / tp) ** 2, 0.0)


def pulse_kick(t: np.ndarray, e0: float, c_light: float) -> np.ndarray:
    """A(t) of an impulsive field E0 delta(t - 0+): -c E0 for t > 0, 0 at t <= 0 (Sec. 3.1)."""
    t = np.asarray(t, float)
    return np.where(t > 0.0, -c_light * e0, 0.0)


def current_spectrum(j: np.ndarray, dt: float, w: np.ndarray, gamma: float) -> np.ndarray:
    """J(w) = dt sum_n w_n (J_n - J_0) exp((i w - gamma) t_n), trapezoid weights."""
    ji = np.asarray(j, float) - j[0]
    n = len(ji) - 1
    t = np.arange(n + 1) * dt
    wt = np.ones(n + 1)
    wt[0] = wt[-1] = 0.5
    ph = np.exp((1j * np.asarray(w, float)[:, None] - gamma) * t[None, :])
    return dt * (ph * (wt * ji)[None, :]).sum(axis=1)


def field_spectrum(a_t: np.ndarray, dt: float, c_light: float, w: np.ndarray, gamma: float) -> np.ndarray:
    """E(w) = sum_n E_{n+1/2} exp((i w - gamma) t_{n+1/2}) dt, E_{n+1/2} = -(A_{n+1} - A_n)/(c dt)."""
    a = np.asarray(a_t, float)
    n = len(a) - 1
    tm = (np.arange(n) + 0.5) * dt
    e = -(a[1:] - a[:-1]) / (c_light * dt)
    ph = np.exp((1j * np.asarray(w, float)[:, None] - gamma) * tm[None, :])
    return dt * (ph * e[None, :]).sum(axis=1)


def polarizability(j: np.ndarray, a_t: np.ndarray, dt: float, omega_cell: float, c_light: float,
                   w: np.ndarray, gamma: float) -> np.ndarray:
    """alpha_zz(w) = (i Omega / w) J(w) / E(w) (Sec. 2, Eq. (5))."""
    w = np.asarray(w, float)
    return 1j * omega_cell / w * current_spectrum(j, dt, w, gamma) / field_spectrum(a_t, dt, c_light, w, gamma)
