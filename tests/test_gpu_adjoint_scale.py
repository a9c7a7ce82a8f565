"""Pulse gradient at the gradient workload's size: the molecule system (N_G =
12000, 72^3 grid, N_aux = 64, 5 states), 64 piecewise-linear knots over 2000
steps of dt = 0.1, checkpoints every 50 steps.

* The hand-written adjoint (AFFINE and REBUILD) against the oracle's adjoint.
* The knot gradient against central finite differences (h = 1e-6) of the GPU
  forward loss on every one of the 64 knots (128 forward runs of 2000 steps).
"""

import time

import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import subspace as ss
from synth import make_system, pulse_samples
from synth.lapw_inputs import knot_times, knot_values

from tests.bounds import DMU_TOL  # noqa: E402

pytestmark = pytest.mark.gpu


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module")
def w4():
    import torch

    from oracle import propagate as pr
    from paper_2403_04351_amd import ltd

    import time

    t0 = time.perf_counter()
    sys = make_system(4)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    print(f"\n[w4] oracle subspace {time.perf_counter() - t0:.1f} s", flush=True)
    lt = ltd.Ltd(sys, max_cols=64)
    torch.cuda.synchronize()
    print(f"[w4] library bound {time.perf_counter() - t0:.1f} s", flush=True)
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    torch.cuda.synchronize()
    print(f"[w4] subspace projected {time.perf_counter() - t0:.1f} s", flush=True)
    t_end = sys.n_steps * sys.dt
    q = knot_values(sys.pulse, t_end)
    th0n = pr.initial_theta(sys.n_aux, sys.n_states)
    th0 = torch.from_numpy(np.ascontiguousarray(th0n.T)[None]).to(lt.device)
    a_t, a_mid = pulse_samples(sys, knots=q)
    g = ad.gradients(sub, th0n, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light)
    gq = ad.knot_gradient(g, knot_times(len(q), t_end), sys.dt)
    torch.cuda.synchronize()
    print(f"[w4] oracle adjoint over {sys.n_steps} steps done at {time.perf_counter() - t0:.1f} s", flush=True)
    return dict(sys=sys, lt=lt, ltd=ltd, torch=torch, q=q, t_end=t_end, th0=th0, g=g, gq=gq)


@pytest.mark.parametrize("mode", ["affine", "rebuild"])
def test_adjoint_matches_oracle_at_scale(w4, mode):
    lt, ltd, torch, sys = w4["lt"], w4["ltd"], w4["torch"], w4["sys"]
    m = ltd.LTD_STEP_AFFINE if mode == "affine" else ltd.LTD_STEP_REBUILD
    qd = torch.from_numpy(w4["q"]).to(lt.device)
    tf = time.perf_counter()
    loss, fw = ltd.pulse_forward(lt, m, sys.dt, qd, w4["t_end"], sys.n_steps, w4["th0"], checkpoint=50)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    grad, g_t, g_mid = ltd.pulse_backward(lt, m, sys.dt, qd, w4["t_end"], sys.n_steps, fw)
    torch.cuda.synchronize()
    te = time.perf_counter()
    print(f"[{mode}] forward {1e3 * (tb - tf):.1f} ms, checkpointed backward {1e3 * (te - tb):.1f} ms "
          f"({sys.n_steps} steps, segments of 50 recomputed by replayed calls)", flush=True)
    assert lt.sync_status() == 0
    g = w4["g"]
    j = fw["st"]["j"].cpu().numpy()
    ej = rel_max(j, g["J"])
    # L = dt sum_n w_n (J_n - J_0) = delta mu(T)/Omega: the dipole change's bar
    el = abs(loss.item() - g["loss"]) / abs(g["loss"])
    em, et, eq = (rel_max(g_mid.cpu().numpy(), g["mid"]), rel_max(g_t.cpu().numpy(), g["at"]),
                  rel_max(grad.cpu().numpy(), w4["gq"]))
    print(f"adjoint at scale ({mode}): J {ej:.2e} loss {el:.2e} (bar {DMU_TOL:.1e}) mid {em:.2e} "
          f"explicit {et:.2e} q {eq:.2e}", flush=True)
    assert ej < 1e-10
    assert el < DMU_TOL
    assert em < 1e-10 and et < 1e-10 and eq < 1e-10


def test_knot_gradient_matches_central_fd_all_knots(w4):
    lt, ltd, torch, sys = w4["lt"], w4["ltd"], w4["torch"], w4["sys"]
    m = ltd.LTD_STEP_AFFINE
    q = w4["q"]
    qd = torch.from_numpy(q).to(lt.device)
    loss, fw = ltd.pulse_forward(lt, m, sys.dt, qd, w4["t_end"], sys.n_steps, w4["th0"], checkpoint=50)
    grad, _, _ = ltd.pulse_backward(lt, m, sys.dt, qd, w4["t_end"], sys.n_steps, fw)
    grad = grad.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(q)
    for k in range(len(q)):
        e = np.zeros_like(q)
        e[k] = h
        lp, _ = ltd.pulse_forward(lt, m, sys.dt, torch.from_numpy(q + e).to(lt.device), w4["t_end"], sys.n_steps,
                                  w4["th0"], checkpoint=sys.n_steps)
        lm, _ = ltd.pulse_forward(lt, m, sys.dt, torch.from_numpy(q - e).to(lt.device), w4["t_end"], sys.n_steps,
                                  w4["th0"], checkpoint=sys.n_steps)
        fd[k] = (lp.item() - lm.item()) / (2 * h)
        if k % 8 == 7:
            print(f"[fd] {k + 1} knots", flush=True)
    assert lt.sync_status() == 0
    err = np.linalg.norm(grad - fd) / np.linalg.norm(fd)
    print(f"64-knot gradient vs central FD (h = 1e-6): {err:.2e}; max per knot "
          f"{np.abs(grad - fd).max() / np.abs(fd).max():.2e}", flush=True)
    assert err < 1e-6
