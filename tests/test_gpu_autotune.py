"""Tuned launch shapes of the per-step rebuild (batched k-points: tiles chosen
by a tuner).

* The three launch shapes of the two-factor x/z kernel compute the same
  arithmetic in the same order, so the propagated states are bit-identical
  across them, in FP64 and in the FP32 residual mode, on the tiny system (16^3
  transforms) and on the molecule (72^3 grid rebuilt on 64^3).
* The register-resident kernel (FP32 residual, 64-point rebuild grid) takes
  another summation order: its states agree with the two-factor kernel's to
  FP32 rounding and with the oracle to the mixed-precision bound.
* The tuner returns a valid choice, and the steps after it (its projection
  split only reorders a sum) match the oracle to the FP64 bound.
"""

import numpy as np
import pytest

from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, pulse_samples, td_potential

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.mark.parametrize("precision", ["LTD_FP64", "LTD_FP32_RESID"])
@pytest.mark.parametrize("cfg", [0, 1], ids=["tiny16", "molecule64"])
def test_launch_shapes_bit_identical_and_tuned_steps_match_oracle(cfg, precision):
    import torch

    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(cfg)
    phi, _ = ss.ground_state(sys, 0)
    sub = ss.project(sys, 0, phi)
    print(f"[tune cfg{cfg} {precision}] oracle subspace", flush=True)
    lt = ltd.Ltd(sys, max_cols=sys.n_aux, precision=getattr(_lib, precision))
    lt.project_subspace(0, ltd.colmajor(phi, lt.device))
    n = 12
    a_t, a_mid = pulse_samples(sys, n)
    s_n = np.sin(0.3 * np.arange(n))
    eps, wfield, wblk = td_potential(sys, 1e-2)
    dev = lt.device
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
    sd = torch.from_numpy(s_n)[:, None].to(dev)
    vs = (v0[None, :] + eps * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + eps * sd * wb[None, :]).contiguous()
    pot = dict(v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
    th0 = pr.initial_theta(sys.n_aux, sys.n_states)

    def run():
        theta = torch.from_numpy(np.ascontiguousarray(th0.T)[None]).to(dev)
        st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(a_t).to(dev),
                          torch.from_numpy(a_mid).to(dev), theta, n, **pot)
        torch.cuda.synchronize()
        assert lt.sync_status() == 0
        return st["theta"][0].cpu().numpy(), st["j"].cpu().numpy()

    shapes = []
    for v in range(3):
        lt.set_tuning(v, 512)
        shapes.append(run())
    for v in (1, 2):
        assert np.array_equal(shapes[v][0], shapes[0][0]), f"launch shape {v} differs"
        assert np.array_equal(shapes[v][1], shapes[0][1])
    n_shapes = 4 if (precision == "LTD_FP32_RESID" and cfg == 1) else 3
    if n_shapes == 4:
        lt.set_tuning(3, 512)
        th3, j3 = run()
        d = rel_max(th3, shapes[0][0])
        print(f"[tune cfg{cfg} {precision}] register kernel vs two-factor: theta {d:.2e}", flush=True)
        assert d < 1e-6
    else:
        with pytest.raises(Exception):
            lt.set_tuning(3, 512)
    tuned = lt.autotune()
    print(f"[tune cfg{cfg} {precision}] choice {tuned}", flush=True)
    assert tuned["n_shapes"] == n_shapes
    assert 0 <= tuned["xz_shape"] < n_shapes and tuned["projection_blocks"] in (256, 512, 1024, 2048)
    assert len(tuned["times_us"]) == n_shapes + 4 and all(t > 0 for t in tuned["times_us"])
    th, j = run()

    v_ref = ss.rebuild_v_sub(sys, 0, phi)
    d = ss.rebuild_v_sub(sys, 0, phi, vr=sys.vr + eps * wfield,
                         h=[h + eps * w for h, w in zip(sys.h, wblk)]) - v_ref
    ref = pr.propagate(sub, th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light,
                       v_sub_fn=lambda k: v_ref + s_n[k] * d)
    ej, et = rel_max(j, ref["J"]), rel_max(th.T, ref["theta"])
    print(f"[tune cfg{cfg} {precision}] after tuning: J {ej:.2e} theta {et:.2e}", flush=True)
    bound = TOL if precision == "LTD_FP64" else 1e-6
    assert ej < bound and et < bound
