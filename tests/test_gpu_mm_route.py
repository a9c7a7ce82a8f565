"""GPU parity of the interstitial matrix-matrix route (dense N_G x N_G blocks of
Fourier coefficients at G - G', applied by GEMM; Sec. 2.3, first route; App. A,
Eq. (A.7)) against the CPU FP64 oracle's own MM route and FFT route, and
against the library's FFT route on the same system: the apply, the projection,
and REBUILD steps with a potential handed in per step (the dense block of the
step's potential built inside the replayed graph).

Bar: 1e-10 relative."""

import numpy as np
import pytest

from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, potential_scale, pulse_samples, td_potential

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module")
def mm0():
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(0)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi, route="mm")
    lt = ltd.Ltd(sys, max_cols=40, route=_lib.LTD_ROUTE_MM)
    lf = ltd.Ltd(sys, max_cols=40)
    return dict(sys=sys, phi=phi, sub=sub, lt=lt, lf=lf, ltd=ltd, torch=torch)


def test_mm_apply_matches_oracle_routes(mm0):
    sys, lt, lf, ltd, torch = mm0["sys"], mm0["lt"], mm0["lf"], mm0["ltd"], mm0["torch"]
    rng = np.random.default_rng(51)
    nb = sys.n_basis(0)
    for n, a_z in ((1, 0.0), (17, 0.42), (40, -1.3)):
        c = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
        cd = ltd.colmajor(c, lt.device)
        hc, sc = lt.apply_hs(0, cd, a_z)
        hf, sf = lf.apply_hs(0, cd, a_z)
        torch.cuda.synchronize()
        hm, sm = op.apply_hs(sys, 0, c, a_z, route="mm")
        e = (rel_max(ltd.to_numpy(hc), hm), rel_max(ltd.to_numpy(sc), sm),
             rel_max(ltd.to_numpy(hc), ltd.to_numpy(hf)), rel_max(ltd.to_numpy(sc), ltd.to_numpy(sf)))
        print(f"MM apply n={n}: H {e[0]:.2e} S {e[1]:.2e}; against the GPU FFT route H {e[2]:.2e} S {e[3]:.2e}",
              flush=True)
        assert max(e) < TOL


def test_mm_projection_matches_oracle(mm0):
    lt, ltd, torch, sub = mm0["lt"], mm0["ltd"], mm0["torch"], mm0["sub"]
    h0, s, _ = lt.project_subspace(0, ltd.colmajor(mm0["phi"], lt.device))
    torch.cuda.synchronize()
    assert rel_max(ltd.to_numpy(h0), sub["H0"]) < TOL
    assert rel_max(ltd.to_numpy(s), sub["S"]) < TOL


def test_mm_rebuild_series_matches_oracle(mm0):
    sys, lt, ltd, torch, sub, phi = mm0["sys"], mm0["lt"], mm0["ltd"], mm0["torch"], mm0["sub"], mm0["phi"]
    n = 50
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    dev = lt.device
    eps_v, wfield, wblk = td_potential(sys)
    s_n = potential_scale(n)
    sd = torch.from_numpy(s_n).to(dev)[:, None]
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
    vs = (v0[None, :] + eps_v * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + eps_v * sd * wb[None, :]).contiguous()
    a_t, a_mid = pulse_samples(sys, n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(dev), torch.from_numpy(a_mid).to(dev),
                      theta, n, v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
    torch.cuda.synchronize()
    assert lt.sync_status() == 0

    def vfn(q):
        return ss.rebuild_v_sub(sys, 0, phi, vr=sys.vr + eps_v * s_n[q] * wfield,
                                h=[h + eps_v * s_n[q] * w for h, w in zip(sys.h, wblk)])

    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    j, th = st["j"].cpu().numpy(), st["theta"][0].cpu().numpy().T
    print(f"MM rebuild {n} steps: J {rel_max(j, ref['J']):.2e} theta {rel_max(th, ref['theta']):.2e}", flush=True)
    assert rel_max(j, ref["J"]) < TOL
    assert rel_max(th, ref["theta"]) < TOL


def test_mm_apply_medium_size_sampled():
    """A 3000-plane-wave system (dense blocks of 144 MB each): sampled columns."""
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(1, n_g=3000, grid=(48, 48, 48), n_aux=16, with_start=False)
    lt = ltd.Ltd(sys, max_cols=4, route=_lib.LTD_ROUTE_MM)
    rng = np.random.default_rng(52)
    nb = sys.n_basis(0)
    c = rng.standard_normal((nb, 3)) + 1j * rng.standard_normal((nb, 3))
    hc, sc = lt.apply_hs(0, ltd.colmajor(c, lt.device), 0.003)
    torch.cuda.synchronize()
    hr, sr = op.apply_hs(sys, 0, c, 0.003)
    print(f"MM apply N_G=3000: H {rel_max(ltd.to_numpy(hc), hr):.2e} S {rel_max(ltd.to_numpy(sc), sr):.2e}",
          flush=True)
    assert rel_max(ltd.to_numpy(hc), hr) < TOL
    assert rel_max(ltd.to_numpy(sc), sr) < TOL
