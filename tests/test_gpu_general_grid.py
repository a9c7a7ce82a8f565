"""GPU parity on a grid whose lengths have no register transform (20 x 20 x 40:
radix 5 on every axis) with a large subspace (N_aux = 300, so the subspace
Hamiltonian does not fit in LDS and the step kernel streams it from memory):
the general plan-driven transforms of the apply and of the per-step rebuild,
the non-LDS step kernel and the Jacobi/Cholesky set-up at n = 300, all against
the CPU FP64 oracle (dense ground state, FFT-route applies).

Bar: 1e-10 relative (element maxima against the largest reference element).
"""

import numpy as np
import pytest

from oracle import operators as op
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, potential_scale, pulse_samples, td_potential

pytestmark = pytest.mark.gpu

TOL = 1e-10
N_STEPS = 30


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module")
def gen():
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0, cell=(10.0, 10.0, 20.0), grid=(20, 20, 40), n_g=600, n_aux=300, n_states=8)
    phi, eps = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    lt = ltd.Ltd(sys, max_cols=300)
    phid = ltd.colmajor(phi, lt.device)
    return dict(sys=sys, phi=phi, eps=eps, sub=sub, lt=lt, ltd=ltd, torch=torch, phid=phid)


def test_general_grid_is_used(gen):
    lt, sys = gen["lt"], gen["sys"]
    g = np.abs(sys.kpts[0].g_int).max(0)
    print(f"box half-widths {g.tolist()}, rebuild grid {lt.rebuild_grid()}", flush=True)
    assert lt.rebuild_grid() == tuple(sys.grid)  # no smaller register grid exists


def test_apply_general_grid(gen):
    sys, lt, ltd, torch = gen["sys"], gen["lt"], gen["ltd"], gen["torch"]
    rng = np.random.default_rng(21)
    nb = sys.n_basis(0)
    for n, a_z in ((3, 0.21), (37, -0.6)):
        c = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
        hc, sc = lt.apply_hs(0, ltd.colmajor(c, lt.device), a_z)
        torch.cuda.synchronize()
        hr, sr = op.apply_hs(sys, 0, c, a_z)
        print(f"apply n={n}: H {rel_max(ltd.to_numpy(hc), hr):.2e} S {rel_max(ltd.to_numpy(sc), sr):.2e}",
              flush=True)
        assert rel_max(ltd.to_numpy(hc), hr) < TOL
        assert rel_max(ltd.to_numpy(sc), sr) < TOL


def test_projection_n300(gen):
    lt, ltd, torch, sub, eps = gen["lt"], gen["ltd"], gen["torch"], gen["sub"], gen["eps"]
    h0, s, _ = lt.project_subspace(0, gen["phid"])
    torch.cuda.synchronize()
    print(f"projection n=300: H0 {rel_max(ltd.to_numpy(h0), sub['H0']):.2e} "
          f"S {rel_max(ltd.to_numpy(s), sub['S']):.2e}", flush=True)
    assert rel_max(ltd.to_numpy(h0), sub["H0"]) < TOL
    assert rel_max(ltd.to_numpy(s), sub["S"]) < TOL
    emin, emax, _ = lt.subspace_info(0)
    assert abs(emin - eps[0]) < 1e-10 * abs(eps).max() and abs(emax - eps[-1]) < 1e-10 * abs(eps).max()


def test_rebuild_series_n300(gen):
    """REBUILD with a potential handed in per step (general x/z and y rebuild
    kernels, non-LDS step kernel) against the oracle's per-step rebuild."""
    sys, lt, ltd, torch, sub, phi = gen["sys"], gen["lt"], gen["ltd"], gen["torch"], gen["sub"], gen["phi"]
    lt.project_subspace(0, gen["phid"])
    dev = lt.device
    eps_v, wfield, wblk = td_potential(sys)
    s_n = potential_scale(N_STEPS)
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
    sd = torch.from_numpy(s_n).to(dev)[:, None]
    vs = (v0[None, :] + eps_v * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + eps_v * sd * wb[None, :]).contiguous()
    a_t, a_mid = pulse_samples(sys, N_STEPS)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(dev), torch.from_numpy(a_mid).to(dev),
                      theta, N_STEPS, v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
    torch.cuda.synchronize()
    assert lt.sync_status() == 0

    def vfn(n):
        return ss.rebuild_v_sub(sys, 0, phi, vr=sys.vr + eps_v * s_n[n] * wfield,
                                h=[h + eps_v * s_n[n] * w for h, w in zip(sys.h, wblk)])

    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    j, e = st["j"].cpu().numpy(), st["e"].cpu().numpy()
    th = st["theta"][0].cpu().numpy().T
    print(f"rebuild n=300, {N_STEPS} steps: J {rel_max(j, ref['J']):.2e} E {rel_max(e, ref['E']):.2e} "
          f"theta {rel_max(th, ref['theta']):.2e}", flush=True)
    assert rel_max(j, ref["J"]) < TOL
    assert rel_max(e, ref["E"]) < TOL
    assert rel_max(th, ref["theta"]) < TOL


def test_affine_n300_stepwise_equals_graph(gen):
    """AFFINE steps: eager stepwise calls and one graph-replayed call agree bit for
    bit, and both match the oracle."""
    sys, lt, ltd, torch, sub = gen["sys"], gen["lt"], gen["ltd"], gen["torch"], gen["sub"]
    lt.project_subspace(0, gen["phid"])
    dev = lt.device
    a_t, a_mid = pulse_samples(sys, N_STEPS)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    runs = []
    for graph in (False, True):
        theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
        st = lt.propagate(ltd.LTD_STEP_AFFINE, sys.dt, torch.from_numpy(a_t).to(dev),
                          torch.from_numpy(a_mid).to(dev), theta, N_STEPS, graph=graph)
        torch.cuda.synchronize()
        runs.append(st)
    assert lt.sync_status() == 0
    assert torch.equal(runs[0]["j"], runs[1]["j"]) and torch.equal(runs[0]["theta"], runs[1]["theta"])
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light)
    assert rel_max(runs[1]["j"].cpu().numpy(), ref["J"]) < TOL
    assert rel_max(runs[1]["theta"][0].cpu().numpy().T, ref["theta"]) < TOL
