"""Device-detected failures latch into the status word and surface from
ltd_sync_status, with every kernel running to its normal end (no GPU fault):

* a non-finite potential handed in for a step: LTD_ENONFINITE;
* a finite potential whose change moves the subspace spectrum out of the
  interval of the step's Chebyshev series: LTD_ESPECTRUM;
* after either, a step with a good potential runs clean again.
"""

import numpy as np
import pytest

from oracle import subspace as ss
from synth import make_system, pulse_samples, td_potential

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    lt = ltd.Ltd(sys)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    return dict(sys=sys, lt=lt, ltd=ltd, torch=torch)


def _step_with(t, v):
    sys, lt, ltd, torch = t["sys"], t["lt"], t["ltd"], t["torch"]
    a_t, a_mid = pulse_samples(sys, 2)
    th0 = np.zeros((1, sys.n_states, sys.n_aux), dtype=np.complex128)
    th0[0, np.arange(sys.n_states), np.arange(sys.n_states)] = 1.0
    theta = torch.from_numpy(th0).to(lt.device)
    vt = torch.from_numpy(np.ascontiguousarray(v.ravel())).to(lt.device)
    st = lt.make_step_args(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(lt.device),
                           torch.from_numpy(a_mid).to(lt.device), theta, 2, v_r_t=vt)
    lt.step(st)
    torch.cuda.synchronize()
    return lt.sync_status()


def test_nonfinite_potential_latches_enonfinite(tiny):
    from paper_2403_04351_amd import _lib

    v = tiny["sys"].vr.copy()
    v.flat[123] = np.nan
    assert _step_with(tiny, v) == _lib.LTD_ENONFINITE
    assert _step_with(tiny, tiny["sys"].vr) == _lib.LTD_OK


def test_potential_beyond_the_interval_latches_espectrum(tiny):
    from paper_2403_04351_amd import _lib

    sys = tiny["sys"]
    _, wfield, _ = td_potential(sys)
    assert _step_with(tiny, sys.vr + 50.0 * wfield) == _lib.LTD_ESPECTRUM
    assert _step_with(tiny, sys.vr) == _lib.LTD_OK


def test_transverse_vector_potential_is_refused(tiny):
    """Only the z momentum block is part of the system: a nonzero A_x or A_y is
    refused on the host (LTD_EUNSUPPORTED) instead of being dropped."""
    import ctypes as C

    from paper_2403_04351_amd import _lib
    from paper_2403_04351_amd.ltd import _ptr

    sys, lt, ltd, torch = tiny["sys"], tiny["lt"], tiny["ltd"], tiny["torch"]
    nb = sys.n_basis(0)
    c = ltd.colmajor(np.ones((nb, 2), dtype=np.complex128), lt.device)
    hc, sc = torch.empty_like(c), torch.empty_like(c)
    for a in ((0.1, 0.0, 0.0), (0.0, -0.2, 0.3)):
        av = (C.c_double * 3)(*a)
        st = lt.lib.ltd_apply_HS(lt.handle, 0, av, _ptr(c), nb, 2, _ptr(hc), nb, _ptr(sc), nb, lt.stream())
        assert st == _lib.LTD_EUNSUPPORTED
    av = (C.c_double * 3)(0.0, 0.0, 0.3)
    assert lt.lib.ltd_apply_HS(lt.handle, 0, av, _ptr(c), nb, 2, _ptr(hc), nb, _ptr(sc), nb, lt.stream()) == 0
    torch.cuda.synchronize()
