"""GPU parity of the explicit subspace step (the exponential's Taylor series
truncated after 4 terms about the spectral centre, at dt <= dt_cr of Sec. 3.1,
Eq. (20)) and of the excited-electron series, against the CPU FP64 oracle; the
critical-time-step check on the host (LTD_ESTEP).

Bar: 1e-10 relative."""

import numpy as np
import pytest

from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module")
def tiny():
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    lt = ltd.Ltd(sys)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    return dict(sys=sys, phi=phi, sub=sub, lt=lt, ltd=ltd, torch=torch)


def _run(t, mode, dt, n, order, graph=True):
    sys, lt, ltd, torch = t["sys"], t["lt"], t["ltd"], t["torch"]
    a_t, a_mid = pulse_samples(sys, n)
    a_t, a_mid = 20 * a_t, 20 * a_mid  # a pulse strong enough to excite
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(lt.device)
    st = lt.propagate(mode, dt, torch.from_numpy(a_t).to(lt.device), torch.from_numpy(a_mid).to(lt.device),
                      theta, n, graph=graph, taylor_order=order, nexc=True)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    return st, a_t, a_mid, th0


@pytest.mark.parametrize("graph", [False, True])
def test_taylor4_matches_oracle(tiny, graph):
    sys, sub, ltd = tiny["sys"], tiny["sub"], tiny["ltd"]
    _, _, dtcr = tiny["lt"].subspace_info(0)
    dt = 0.9 * dtcr
    n = 80
    st, a_t, a_mid, th0 = _run(tiny, ltd.LTD_STEP_AFFINE, dt, n, 4, graph)
    ref = pr.propagate(sub, th0, a_t, a_mid, dt, sys.occ, sys.omega, sys.c_light, taylor_order=4)
    j, nx = st["j"].cpu().numpy(), st["nexc"].cpu().numpy()
    th = st["theta"][0].cpu().numpy().T
    print(f"taylor-4 dt={dt:.4f}: J {rel_max(j, ref['J']):.2e} theta {rel_max(th, ref['theta']):.2e} "
          f"N_exc {rel_max(nx, ref['nexc']):.2e} (max N_exc {np.abs(ref['nexc']).max():.2e})", flush=True)
    assert rel_max(j, ref["J"]) < TOL
    assert rel_max(th, ref["theta"]) < TOL
    assert rel_max(nx, ref["nexc"]) < 1e-8  # a small difference of norms (see the exponential test)


def test_taylor4_rebuild_matches_oracle(tiny):
    sys, sub, ltd, phi = tiny["sys"], tiny["sub"], tiny["ltd"], tiny["phi"]
    _, _, dtcr = tiny["lt"].subspace_info(0)
    dt = 0.5 * dtcr
    n = 40
    st, a_t, a_mid, th0 = _run(tiny, ltd.LTD_STEP_REBUILD, dt, n, 4)
    vfn = lambda k: ss.rebuild_v_sub(sys, 0, phi)
    ref = pr.propagate(sub, th0, a_t, a_mid, dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn, taylor_order=4)
    assert rel_max(st["j"].cpu().numpy(), ref["J"]) < TOL
    assert rel_max(st["theta"][0].cpu().numpy().T, ref["theta"]) < TOL


def test_excited_electrons_exponential(tiny):
    sys, sub, ltd = tiny["sys"], tiny["sub"], tiny["ltd"]
    n = 100
    st, a_t, a_mid, th0 = _run(tiny, ltd.LTD_STEP_AFFINE, sys.dt, n, 0)
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light)
    nx = st["nexc"].cpu().numpy()
    err = np.abs(nx - ref["nexc"]).max()
    print(f"N_exc (exponential): abs err {err:.2e}, max {np.abs(ref['nexc']).max():.2e}", flush=True)
    # N_exc is a difference of O(f N_states) norms: its absolute error is set by
    # the FP64 rounding of those norms (1e-10 relative to them)
    assert err < 1e-10 * sys.occ * sys.n_states
    assert np.abs(ref["nexc"]).max() > 1e-6  # the pulse excites


def test_step_above_dt_cr_is_rejected(tiny):
    from paper_2403_04351_amd import _lib

    sys, lt, ltd, torch = tiny["sys"], tiny["lt"], tiny["ltd"], tiny["torch"]
    _, _, dtcr = lt.subspace_info(0)
    a_t, a_mid = pulse_samples(sys, 4)
    theta = torch.zeros((1, sys.n_states, sys.n_aux), dtype=torch.complex128, device=lt.device)
    st = lt.make_step_args(ltd.LTD_STEP_AFFINE, 1.01 * dtcr, torch.from_numpy(a_t).to(lt.device),
                           torch.from_numpy(a_mid).to(lt.device), theta, 4, taylor_order=4)
    with pytest.raises(_lib.LtdError) as ei:
        lt.run(st, 4)
    assert ei.value.code == _lib.LTD_ESTEP
    st = lt.make_step_args(ltd.LTD_STEP_AFFINE, 0.1, torch.from_numpy(a_t).to(lt.device),
                           torch.from_numpy(a_mid).to(lt.device), theta, 4, taylor_order=9)
    with pytest.raises(_lib.LtdError) as ei:
        lt.step(st)
    assert ei.value.code == _lib.LTD_EINVAL
