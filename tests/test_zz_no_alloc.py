"""The allocation-free apply (ltd_apply_HS_static, scratch in a fixed device
array) against ltd_apply_HS on the same system: two calls in a row, the second
with fewer columns (the array keeps the first call's contents), both within the
FP64 bar of the ordinary entry point, and the ordinary entry point unchanged by
it.  Also the host-side rejection of a system whose single column does not fit
the array."""

import ctypes as C

import numpy as np
import pytest

from synth import make_system

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


def _apply(lt, fn, k, c, a_z):
    import torch

    from paper_2403_04351_amd import _lib

    n, nb = c.shape
    hc = torch.full_like(c, float("nan"))
    sc = torch.full_like(c, float("nan"))
    a = (C.c_double * 3)(0.0, 0.0, float(a_z))
    _lib.check(getattr(lt.lib, fn)(lt.handle, k, a, c.data_ptr(), nb, n, hc.data_ptr(), nb, sc.data_ptr(), nb,
                                   lt.stream()), fn)
    return hc, sc


def test_static_apply_matches_workspace_apply():
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0)
    lt = ltd.Ltd(sys, max_cols=40)
    nb = sys.n_basis(0)
    rng = np.random.default_rng(41)
    for n, a_z in ((40, 0.31), (7, -0.8)):  # the second call smaller than the first
        c = ltd.colmajor(rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n)), lt.device)
        hs, ss_ = _apply(lt, "ltd_apply_HS_static", 0, c, a_z)
        hw, sw = _apply(lt, "ltd_apply_HS", 0, c, a_z)
        torch.cuda.synchronize()
        eh = rel_max(ltd.to_numpy(hs), ltd.to_numpy(hw))
        es = rel_max(ltd.to_numpy(ss_), ltd.to_numpy(sw))
        print(f"static apply n={n}: H {eh:.2e} S {es:.2e}", flush=True)
        assert np.isfinite(ltd.to_numpy(hs)).all() and np.isfinite(ltd.to_numpy(ss_)).all()
        assert eh < TOL and es < TOL
    assert lt.sync_status() == 0


def test_static_apply_more_columns_than_one_pass():
    """A call larger than max_cols and than one pass of the array, on the
    molecule-sized grid: several passes, each checked."""
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(1, with_start=False)
    lt = ltd.Ltd(sys, max_cols=8)
    nb = sys.n_basis(0)
    rng = np.random.default_rng(42)
    n = 9  # one column of the 72^3 grid's slabs takes ~ 6 MiB: passes of a few columns
    c = ltd.colmajor(rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n)), lt.device)
    hs, ss_ = _apply(lt, "ltd_apply_HS_static", 0, c, 0.002)
    hw0, sw0 = _apply(lt, "ltd_apply_HS", 0, c[:8].contiguous(), 0.002)
    hw1, sw1 = _apply(lt, "ltd_apply_HS", 0, c[8:].contiguous(), 0.002)
    torch.cuda.synchronize()
    hw, sw = torch.cat([hw0, hw1]), torch.cat([sw0, sw1])
    eh = rel_max(ltd.to_numpy(hs), ltd.to_numpy(hw))
    es = rel_max(ltd.to_numpy(ss_), ltd.to_numpy(sw))
    print(f"static apply 72^3, n={n}: H {eh:.2e} S {es:.2e}", flush=True)
    assert eh < TOL and es < TOL


def test_static_apply_rejects_oversized_column():
    """One column of a 120^3 grid's FFT slabs exceeds the array (the G box reaches
    |g| = 27, so no smaller exact grid exists for the apply): rejected on the host
    with LTD_EUNSUPPORTED, nothing enqueued; the ordinary apply still runs."""
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(0, grid=(120, 120, 120), n_g=90000, with_start=False)
    lt = ltd.Ltd(sys, max_cols=2)
    nb = sys.n_basis(0)
    c = torch.ones((1, nb), dtype=torch.complex128, device=lt.device)
    with pytest.raises(_lib.LtdError) as ei:
        _apply(lt, "ltd_apply_HS_static", 0, c, 0.0)
    assert ei.value.code == _lib.LTD_EUNSUPPORTED
    hw, sw = _apply(lt, "ltd_apply_HS", 0, c, 0.0)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(hw)).all()
