"""GPU parity of the REBUILD step when the potential is handed in per step.

* The potential series (one V(r) and one set of muffin-tin blocks per step,
  indexed by the device step counter inside a replayed hipGraph) against the
  oracle's per-step rebuild of V_sub.
* The same on a grid larger than the rebuild needs: the library then runs the
  per-step transforms on a smaller grid (lengths >= 4 b + 1) with Theta V
  re-expressed on it, which must reproduce the oracle's full-grid convolution.
* The adjoint (pulse gradient) under a per-step potential against the oracle's
  adjoint with the same V_sub(n).
"""

import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples, td_potential
from synth.lapw_inputs import knot_times, knot_values

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


def _setup(grid=None, **over):
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0, **({} if grid is None else dict(grid=grid)), **over)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    lt = ltd.Ltd(sys)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    return sys, phi, sub, lt, ltd, torch


def _series(sys, phi, lt, torch, s_n, eps_v=1e-2):
    """Device series V_n = V + eps s_n W, h_n = h + eps s_n w and the oracle's V_sub(n)."""
    eps, wfield, wblk = td_potential(sys, eps_v)
    dev = lt.device
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
    sd = torch.from_numpy(np.asarray(s_n, dtype=np.float64)).to(dev)[:, None]
    vs = (v0[None, :] + eps * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + eps * sd * wb[None, :]).contiguous()

    def vfn(n):
        return ss.rebuild_v_sub(sys, 0, phi, vr=sys.vr + eps * s_n[n] * wfield,
                                h=[h + eps * s_n[n] * w for h, w in zip(sys.h, wblk)])

    pot = dict(v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
    return pot, vfn


@pytest.mark.parametrize("grid", [None, (64, 64, 64)], ids=["grid16", "grid64_rebuilt_on_16"])
def test_static_rebuild_matches_oracle(grid):
    sys, phi, sub, lt, ltd, torch = _setup(grid)
    n = 30
    a_t, a_mid = pulse_samples(sys, n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(lt.device)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(lt.device),
                      torch.from_numpy(a_mid).to(lt.device), theta, n)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light,
                       v_sub_fn=lambda k: ss.rebuild_v_sub(sys, 0, phi))
    j = st["j"].cpu().numpy()
    print(f"static rebuild {grid}: J {rel_max(j, ref['J']):.2e}", flush=True)
    assert rel_max(j, ref["J"]) < TOL
    assert rel_max(st["e"].cpu().numpy(), ref["E"]) < TOL
    assert rel_max(st["theta"][0].cpu().numpy().T, ref["theta"]) < TOL


@pytest.mark.parametrize("grid", [None, (64, 64, 64)], ids=["grid16", "grid64_rebuilt_on_16"])
def test_potential_series_in_graph_matches_oracle(grid):
    sys, phi, sub, lt, ltd, torch = _setup(grid)
    n = 40
    a_t, a_mid = pulse_samples(sys, n)
    s_n = a_mid / np.abs(a_mid).max()
    pot, vfn = _series(sys, phi, lt, torch, s_n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    dev = lt.device
    theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(dev), torch.from_numpy(a_mid).to(dev),
                      theta, n, **pot)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    j = st["j"].cpu().numpy()
    jr = ref["J"] - ref["J"][0]
    print(f"potential series {grid}: J {rel_max(j, ref['J']):.2e} J_ind {rel_max(j - j[0], jr):.2e}", flush=True)
    assert rel_max(j, ref["J"]) < TOL
    assert rel_max(st["e"].cpu().numpy(), ref["E"]) < TOL
    assert rel_max(st["theta"][0].cpu().numpy().T, ref["theta"]) < TOL
    # the series matters: the static-potential propagation differs
    ref0 = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light)
    assert np.abs(ref0["E"] - ref["E"]).max() > 1e3 * TOL * np.abs(ref["E"]).max()


def test_adjoint_with_potential_series_matches_oracle():
    sys, phi, sub, lt, ltd, torch = _setup(None, n_steps=50, pulse=dict(kind="knots", n_knots=8, base=dict(
        kind="gauss_sin", amp=0.01, omega=0.3, t0=3.0, width=1.5)))
    n_steps, n_knots = 50, 8
    t_end = n_steps * sys.dt
    q = knot_values(sys.pulse, t_end)
    a_t, a_mid = pulse_samples(sys, knots=q)
    s_n = np.sin(0.2 * np.arange(n_steps))
    pot, vfn = _series(sys, phi, lt, torch, s_n)
    th0n = pr.initial_theta(sys.n_aux, sys.n_states)
    g = ad.gradients(sub, th0n, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn)
    gq = ad.knot_gradient(g, knot_times(n_knots, t_end), sys.dt)
    th0 = torch.from_numpy(np.ascontiguousarray(th0n.T)[None]).to(lt.device)
    qd = torch.from_numpy(q).to(lt.device)
    loss, fw = ltd.pulse_forward(lt, ltd.LTD_STEP_REBUILD, sys.dt, qd, t_end, n_steps, th0, checkpoint=9,
                                 potential=pot)
    grad, g_t, g_mid = ltd.pulse_backward(lt, ltd.LTD_STEP_REBUILD, sys.dt, qd, t_end, n_steps, fw)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    print(f"adjoint series: loss {abs(loss.item() - g['loss']) / abs(g['loss']):.2e} "
          f"q {rel_max(grad.cpu().numpy(), gq):.2e}", flush=True)
    assert abs(loss.item() - g["loss"]) < 1e-10 * abs(g["loss"])
    assert rel_max(g_mid.cpu().numpy(), g["mid"]) < 1e-9
    assert rel_max(grad.cpu().numpy(), gq) < 1e-9


@pytest.mark.parametrize("grid", [None, (64, 64, 64)], ids=["grid16", "grid64_rebuilt_on_16"])
@pytest.mark.parametrize("with_c", [True, False])
def test_pipelined_replay_equals_stepwise_with_series(grid, with_c):
    """ltd_propagate rebuilds V~ of step n + 1 beside the exponential of step n,
    and synthesises Theta V of step n + 2 beside the read-out of step n + 1
    (step indices from device counters, clamped to the call's last step); the
    arithmetic is that of the stepwise calls, so the results are bit-identical:
    one call of n steps (graphs of 32, 8 and 1 steps), two calls of n1 + n2
    steps, and n single steps (the series, the states and, with_c, the
    mapped-back coefficients C, which join the streams every step)."""
    sys, phi, sub, lt, ltd, torch = _setup(grid)
    n, n1 = 45, 9
    a_t, a_mid = pulse_samples(sys, n)
    s_n = np.sin(0.4 * np.arange(n))
    pot, _ = _series(sys, phi, lt, torch, s_n)
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)
    dev = lt.device

    def fresh():
        theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
        cout = torch.zeros((sys.n_states, sys.n_basis(0)), dtype=torch.complex128, device=dev) if with_c else None
        return lt.make_step_args(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(dev),
                                 torch.from_numpy(a_mid).to(dev), theta, n, c_out=cout, **pot)

    runs = {}
    st = fresh()
    lt.run(st, n)
    runs["one call"] = st
    st = fresh()
    lt.run(st, n1)
    lt.run(st, n - n1)
    runs["two calls"] = st
    st = fresh()
    for _ in range(n):
        lt.step(st)
    runs["stepwise"] = st
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    ref = runs["stepwise"]
    for name in ("one call", "two calls"):
        for key in ("j", "e", "dmu", "theta") + (("c_out",) if with_c else ()):
            assert np.array_equal(runs[name][key].cpu().numpy(), ref[key].cpu().numpy()), (name, key)
    assert int(runs["two calls"]["step"].item()) == n
