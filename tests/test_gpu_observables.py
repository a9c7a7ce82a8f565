"""GPU parity of the pulses (sin^2 laser, kick, Gaussian-envelope pulse) and of
the polarizability spectrum alpha_zz(w) (Sec. 2, Eq. (5)) against the CPU FP64
oracle, the latter on the current of a kicked propagation of the tiny
workload.  Bar: 1e-10 relative (pulses to rounding)."""

import numpy as np
import pytest

from oracle import observables as ob
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system

pytestmark = pytest.mark.gpu


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


def test_pulse_samples_match_oracle():
    import torch

    from paper_2403_04351_amd import _lib, ltd

    n, dt = 5000, 0.2
    t, tm = np.arange(n + 1) * dt, (np.arange(n) + 0.5) * dt
    c = 137.035999084
    cases = [
        (_lib.LTD_PULSE_SIN2, (10.0, 0.294, 1.0, 800.0), lambda x: ob.pulse_sin2(x, 10.0, 0.294, 1.0, 800.0)),
        (_lib.LTD_PULSE_KICK, (1e-3, c, 0.0, 0.0), lambda x: ob.pulse_kick(x, 1e-3, c)),
        (_lib.LTD_PULSE_GAUSS_SIN, (0.005, 0.2, 5.0, 2.0),
         lambda x: 0.005 * np.sin(0.2 * x) * np.exp(-((x - 5.0) / 2.0) ** 2)),
    ]
    for kind, prm, f in cases:
        a_t, a_mid = ltd.pulse_samples(kind, prm, dt, n)
        torch.cuda.synchronize()
        assert rel_max(a_t.cpu().numpy(), f(t)) < 1e-13
        assert rel_max(a_mid.cpu().numpy(), f(tm)) < 1e-13


def test_polarizability_of_kicked_propagation():
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    lt = ltd.Ltd(sys)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    n, dt, e0 = 600, sys.dt, 1e-3
    a_t, a_mid = ltd.pulse_samples(_lib.LTD_PULSE_KICK, (e0, sys.c_light, 0.0, 0.0), dt, n, lt.device)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(lt.device)
    st = lt.propagate(ltd.LTD_STEP_AFFINE, dt, a_t, a_mid, theta, n)
    w = torch.linspace(0.05, 3.0, 240, dtype=torch.float64, device=lt.device)
    al = ltd.polarizability(st["j"], a_t, dt, sys.omega, sys.c_light, w, 0.02)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    ta, tm = a_t.cpu().numpy(), a_mid.cpu().numpy()
    ref_run = pr.propagate(sub, th0, ta, tm, dt, sys.occ, sys.omega, sys.c_light)
    ref = ob.polarizability(ref_run["J"], ta, dt, sys.omega, sys.c_light, w.cpu().numpy(), 0.02)
    # the spectrum of the GPU's own current against the oracle's transform of it
    own = ob.polarizability(st["j"].cpu().numpy(), ta, dt, sys.omega, sys.c_light, w.cpu().numpy(), 0.02)
    e_own, e_ref = rel_max(al.cpu().numpy(), own), rel_max(al.cpu().numpy(), ref)
    print(f"polarizability: transform {e_own:.2e}, against the oracle run {e_ref:.2e}", flush=True)
    assert e_own < 1e-10
    assert e_ref < 1e-8  # J_ind's own resolution (a difference of large currents)
