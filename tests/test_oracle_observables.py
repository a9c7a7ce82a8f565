"""Pins for the oracle's pulses and spectra (CPU only).

* sin^2 laser: zero outside [t0, t0 + T_p], the closed form at the envelope's
  peak, and E = -(1/c) dA/dt integrating to -(A(end) - A(start))/c = 0.
* Kick: the sampled field has total weight E0 (sum of E dt) and E(w) -> E0 as
  w, gamma -> 0.
* J(w) at the grid frequencies 2 pi k/(N dt) without damping equals numpy's
  inverse FFT of the samples plus the trapezoid end corrections (an independent
  routine).
* alpha(w) is linear in J and scales as 1/E0; a damped oscillator J_ind has its
  spectral peak at its frequency.
"""

import numpy as np

from oracle import observables as ob


def test_sin2_pulse_closed_forms():
    a0, w, t0, tp = 10.0, 0.294, 1.0, 800.0
    t = np.array([0.0, 0.5, t0, t0 + tp / 2, t0 + tp, t0 + tp + 3.0])
    a = ob.pulse_sin2(t, a0, w, t0, tp)
    assert a[0] == 0.0 and a[1] == 0.0 and a[-1] == 0.0
    assert abs(a[2]) < 1e-30 and abs(a[4]) < 1e-12 * a0
    assert abs(a[3] - a0 * np.cos(w * (t0 + tp / 2))) < 1e-12 * a0


def test_kick_field_weight():
    dt, c = 0.1, 137.035999084
    a = ob.pulse_kick(np.arange(101) * dt, 1e-3, c)
    assert a[0] == 0.0 and np.all(a[1:] == -c * 1e-3)
    e = ob.field_spectrum(a, dt, c, np.array([1e-9]), 0.0)
    assert abs(e[0] - 1e-3) < 1e-12


def test_current_spectrum_matches_fft():
    rng = np.random.default_rng(9)
    n, dt = 256, 0.2
    j = rng.standard_normal(n + 1)
    k = np.arange(1, 20)
    w = 2 * np.pi * k / (n * dt)
    ji = j - j[0]
    ref = dt * (n * np.fft.ifft(ji[:n])[k] - 0.5 * ji[0] + 0.5 * ji[n])
    assert np.abs(ob.current_spectrum(j, dt, w, 0.0) - ref).max() < 1e-12 * np.abs(ref).max()


def test_polarizability_linearity_and_peak():
    dt, c, om = 0.1, 137.0, 1000.0
    n = 4000
    t = np.arange(n + 1) * dt
    w0, gam = 0.5, 0.01
    j = 1e-6 * np.sin(w0 * t) * np.exp(-gam * t)
    a = ob.pulse_kick(t, 1e-3, c)
    w = np.linspace(0.2, 0.8, 601)
    al = ob.polarizability(j, a, dt, om, c, w, 0.005)
    al2 = ob.polarizability(2 * j, a, dt, om, c, w, 0.005)
    al3 = ob.polarizability(j, ob.pulse_kick(t, 2e-3, c), dt, om, c, w, 0.005)
    assert np.allclose(al2, 2 * al, rtol=1e-12) and np.allclose(al3, al / 2, rtol=1e-12)
    assert abs(w[np.argmax(np.abs(al))] - w0) < 0.005
