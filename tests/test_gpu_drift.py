"""S-orthonormality drift and Loewdin reorthonormalisation of the states on
the GPU (ltd_state_drift) against the oracle (max |theta^H S_sub theta - I| and
theta G^{-1/2}), on the tiny system and the molecule; and the drift of the
FP64 and FP32-residual propagations, which keep the states S-orthonormal."""

import numpy as np
import pytest
import scipy.linalg

from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [0, 1], ids=["tiny", "molecule"])
def test_drift_and_lowdin_match_oracle(cfg):
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(cfg)
    phi = np.ascontiguousarray(sys.kpts[0].start[:, : sys.n_aux])  # not S-orthonormal: S_sub != I
    sub = ss.project(sys, 0, phi)
    lt = ltd.Ltd(sys, max_cols=sys.n_aux)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    s = sub["S"]
    assert np.abs(s - np.eye(sys.n_aux)).max() > 1e-2
    rng = np.random.default_rng(11)
    l = np.linalg.cholesky(s)
    th0 = scipy.linalg.solve_triangular(l.conj().T, pr.initial_theta(sys.n_aux, sys.n_states), lower=False)
    th = th0 + 0.03 * (rng.standard_normal(th0.shape) + 1j * rng.standard_normal(th0.shape))
    dev = torch.from_numpy(np.ascontiguousarray(th.T)[None]).to(lt.device)
    d_ref = float(np.abs(pr.state_gram(th, s) - np.eye(sys.n_states)).max())
    d = lt.state_drift(dev)
    print(f"[drift cfg{cfg}] gpu {d:.6e} oracle {d_ref:.6e}", flush=True)
    assert abs(d - d_ref) < 1e-10 * max(1.0, d_ref)
    d2 = lt.state_drift(dev, reorthonormalize=True)
    assert abs(d2 - d_ref) < 1e-10 * max(1.0, d_ref)
    q = pr.lowdin(th, s)
    got = dev[0].cpu().numpy().T
    err = float(np.abs(got - q).max() / np.abs(q).max())
    after = lt.state_drift(dev)
    print(f"[drift cfg{cfg}] loewdin vs oracle {err:.2e}, drift after {after:.2e}", flush=True)
    assert err < 1e-10
    assert after < 1e-12


@pytest.mark.parametrize("precision", ["LTD_FP64", "LTD_FP32_RESID"])
def test_propagation_keeps_states_s_orthonormal(precision):
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    lt = ltd.Ltd(sys, precision=getattr(_lib, precision))
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    n = 200
    a_t, a_mid = pulse_samples(sys, n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(lt.device)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(lt.device),
                      torch.from_numpy(a_mid).to(lt.device), theta, n)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    d = lt.state_drift(st["theta"])
    print(f"[drift {precision}] after {n} steps: {d:.2e}", flush=True)
    assert d < 1e-12


def test_reorthonormalisation_every_k_steps_keeps_the_result():
    """Loewdin every 25 steps of an FP64 run changes the states by rounding only
    (they stay S-orthonormal to ~1e-14), so J agrees with the plain run."""
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    lt = ltd.Ltd(sys)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    n = 100
    a_t, a_mid = pulse_samples(sys, n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    runs = []
    for every in (None, 25):
        theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(lt.device)
        st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(lt.device),
                          torch.from_numpy(a_mid).to(lt.device), theta, n, reorth_every=every)
        torch.cuda.synchronize()
        runs.append(st)
    drifts = runs[1]["drift"]
    print(f"[reorth] drifts {['%.1e' % d for d in drifts]}", flush=True)
    assert len(drifts) == 4 and max(drifts) < 1e-12
    j0, j1 = runs[0]["j"].cpu().numpy(), runs[1]["j"].cpu().numpy()
    assert np.abs(j1 - j0).max() < 1e-11 * np.abs(j0).max()
