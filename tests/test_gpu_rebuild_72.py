"""GPU parity of the per-step rebuild on a 72^3 rebuild grid whose box reaches
|g| = 16 and 17 (the molecule's cell and grid with N_G = 18000 and 22000): the
register x/z kernel's 72 x 72 instance with the known-zero inputs and unread
outputs of every line dropped at compile time (valid while 4 b + 1 <= 72), in
FP64 and in the complex64 residual form, against the oracle's per-step rebuild.
The apply on the same grid (the register plane passes, pruned the same way, and
the register z lines) on ragged column counts against the oracle's apply.

Bars: FP64 1e-10 relative (element maxima against the largest reference
element); FP32 residual 1e-6.
"""

import numpy as np
import pytest

from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, potential_scale, pulse_samples, td_potential

pytestmark = pytest.mark.gpu

N_STEPS = 4


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module", params=[18000, 22000])
def box(request):
    sys = make_system(1, n_g=request.param, n_aux=24, n_states=4)
    phi = np.ascontiguousarray(sys.kpts[0].start)
    sub = ss.project(sys, 0, phi)
    eps_v, wfield, wblk = td_potential(sys)
    s_n = potential_scale(N_STEPS)

    def vfn(n):
        return ss.rebuild_v_sub(sys, 0, phi, vr=sys.vr + eps_v * s_n[n] * wfield,
                                h=[h + eps_v * s_n[n] * w for h, w in zip(sys.h, wblk)])

    a_t, a_mid = pulse_samples(sys, N_STEPS)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    return dict(sys=sys, phi=phi, eps_v=eps_v, wfield=wfield, wblk=wblk, s_n=s_n, a_t=a_t, a_mid=a_mid, th0=th0,
                ref=ref)


@pytest.mark.parametrize("precision", ["LTD_FP64", "LTD_FP32_RESID"])
def test_pruned_72_rebuild_matches_oracle(box, precision):
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = box["sys"]
    b = np.abs(sys.kpts[0].g_int).max(0)
    lt = ltd.Ltd(sys, max_cols=sys.n_aux, precision=getattr(_lib, precision))
    assert tuple(lt.rebuild_grid()) == (72, 72, 72) and 16 <= b.max() <= 17
    dev = lt.device
    lt.project_subspace(0, ltd.colmajor(box["phi"], dev))
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(box["wfield"].ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in box["wblk"]])).to(dev)
    sd = torch.from_numpy(box["s_n"]).to(dev)[:, None]
    vs = (v0[None, :] + box["eps_v"] * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + box["eps_v"] * sd * wb[None, :]).contiguous()
    theta = torch.from_numpy(np.ascontiguousarray(box["th0"].T)[None]).to(dev)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(box["a_t"]).to(dev),
                      torch.from_numpy(box["a_mid"]).to(dev), theta, N_STEPS, v_r_t=vs, h_t=hs,
                      v_stride=vs.shape[1], h_stride=hs.shape[1])
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    ref = box["ref"]
    j, th = st["j"].cpu().numpy(), st["theta"][0].cpu().numpy().T
    ej, et = rel_max(j, ref["J"]), rel_max(th, ref["theta"])
    print(f"72^3 rebuild, |g| <= {b.max()}, {precision}: J {ej:.2e} theta {et:.2e}", flush=True)
    bar = 1e-10 if precision == "LTD_FP64" else 1e-6
    assert ej < bar and et < bar
    lt.close()


@pytest.mark.parametrize("n", [1, 9, 29])
def test_apply_on_72_planes(box, n):
    import torch

    from paper_2403_04351_amd import ltd

    sys = box["sys"]
    lt = ltd.Ltd(sys, max_cols=32)
    assert tuple(lt.rebuild_grid()) == (72, 72, 72)
    rng = np.random.default_rng(70 + n)
    c = rng.standard_normal((sys.n_basis(0), n)) + 1j * rng.standard_normal((sys.n_basis(0), n))
    hc, sc = lt.apply_hs(0, ltd.colmajor(c, lt.device), 0.0029)
    torch.cuda.synchronize()
    hr, sr = op.apply_hs(sys, 0, c, 0.0029)
    eh, es = rel_max(ltd.to_numpy(hc), hr), rel_max(ltd.to_numpy(sc), sr)
    b = np.abs(sys.kpts[0].g_int).max(0)
    print(f"72^3 apply, |g| <= {b.max()}, n = {n}: H {eh:.2e} S {es:.2e}", flush=True)
    assert eh < 1e-10 and es < 1e-10
    lt.close()
