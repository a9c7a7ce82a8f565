"""More k-points than one batched launch takes: 20 k-points (a 5x4x1 set) of the
tiny cell, so the per-step rebuild runs its k-points in two launches of each
FFT stage (16 + 4) and the step and projection tables span all 20.

* Projection of every k against the oracle.
* 12 graph-replayed REBUILD steps with a potential that changes every step
  (V_n = V + eps s_n W and h_n = h + eps s_n w, the same for every k) against
  the oracle's per-step rebuild of V_sub for each k, combined with the k
  weights (J, E, theta of every k).
* The same run in one call and in two calls (4 + 8 steps): the same states.

Bar: 1e-10 relative (element maxima against the largest reference element).
"""

import numpy as np
import pytest

from oracle import propagate as pr
from oracle import subspace as ss
from synth import make_system, potential_scale, pulse_samples, td_potential

pytestmark = pytest.mark.gpu

TOL = 1e-10
N_STEPS = 12


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module")
def many():
    import torch

    from paper_2403_04351_amd import ltd

    sys = make_system(0, kgrid=(5, 4, 1))
    assert len(sys.kpts) == 20
    n = sys.n_aux
    phis = [np.ascontiguousarray(kp.start[:, :n]) for kp in sys.kpts]
    subs = [ss.project(sys, k, phis[k]) for k in range(len(sys.kpts))]
    eps_v, wfield, wblk = td_potential(sys)
    s_n = potential_scale(N_STEPS)
    a_t, a_mid = pulse_samples(sys, N_STEPS)
    th0 = pr.initial_theta(n, sys.n_states)
    refs = []
    for k in range(len(sys.kpts)):
        def vfn(i, k=k):
            return ss.rebuild_v_sub(sys, k, phis[k], vr=sys.vr + eps_v * s_n[i] * wfield,
                                    h=[h + eps_v * s_n[i] * w for h, w in zip(sys.h, wblk)])

        refs.append(pr.propagate(subs[k], th0, a_t, a_mid, sys.dt, sys.occ, sys.omega, sys.c_light, v_sub_fn=vfn))
    lt = ltd.Ltd(sys, max_cols=n)
    yield dict(sys=sys, phis=phis, subs=subs, refs=refs, eps_v=eps_v, wfield=wfield, wblk=wblk, s_n=s_n, a_t=a_t,
               a_mid=a_mid, th0=th0, lt=lt, ltd=ltd, torch=torch)
    lt.close()


def _bind(m):
    lt, ltd = m["lt"], m["ltd"]
    for k in range(len(m["sys"].kpts)):
        lt.project_subspace(k, ltd.colmajor(m["phis"][k], lt.device))


def _series(m):
    torch, lt, sys = m["torch"], m["lt"], m["sys"]
    dev = lt.device
    v0 = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
    w0 = torch.from_numpy(np.ascontiguousarray(m["wfield"].ravel())).to(dev)
    wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in m["wblk"]])).to(dev)
    sd = torch.from_numpy(m["s_n"]).to(dev)[:, None]
    vs = (v0[None, :] + m["eps_v"] * sd * w0[None, :]).contiguous()
    hs = (lt.h[None, :] + m["eps_v"] * sd * wb[None, :]).contiguous()
    return vs, hs


def test_many_k_projection(many):
    lt, ltd, torch = many["lt"], many["ltd"], many["torch"]
    for k in range(len(many["sys"].kpts)):
        h0, s, _ = lt.project_subspace(k, ltd.colmajor(many["phis"][k], lt.device))
        torch.cuda.synchronize()
        assert rel_max(ltd.to_numpy(h0), many["subs"][k]["H0"]) < TOL
        assert rel_max(ltd.to_numpy(s), many["subs"][k]["S"]) < TOL


def test_many_k_rebuild_series(many):
    sys, lt, ltd, torch = many["sys"], many["lt"], many["ltd"], many["torch"]
    _bind(many)
    vs, hs = _series(many)
    dev = lt.device
    nk = len(sys.kpts)
    theta = torch.from_numpy(np.ascontiguousarray(np.stack([many["th0"].T] * nk))).to(dev)
    st = lt.propagate(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(many["a_t"]).to(dev),
                      torch.from_numpy(many["a_mid"]).to(dev), theta, N_STEPS, v_r_t=vs, h_t=hs,
                      v_stride=vs.shape[1], h_stride=hs.shape[1])
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    j = np.zeros(N_STEPS + 1)
    e = np.zeros(N_STEPS + 1)
    th = st["theta"].cpu().numpy()
    worst = 0.0
    for k, kp in enumerate(sys.kpts):
        ref = many["refs"][k]
        j += kp.weight * ref["J"]
        e += kp.weight * ref["E"]
        worst = max(worst, rel_max(th[k].T, ref["theta"]))
    ej, ee = rel_max(st["j"].cpu().numpy(), j), rel_max(st["e"].cpu().numpy(), e)
    print(f"20 k, {N_STEPS} rebuild steps with a per-step potential: J {ej:.2e} E {ee:.2e} theta (worst k) "
          f"{worst:.2e}", flush=True)
    assert ej < TOL and ee < TOL and worst < TOL
    many["theta_one_call"] = th


def test_many_k_two_calls_equal_one(many):
    sys, lt, ltd, torch = many["sys"], many["lt"], many["ltd"], many["torch"]
    if "theta_one_call" not in many:
        pytest.skip("needs the one-call run")
    _bind(many)
    vs, hs = _series(many)
    dev = lt.device
    nk = len(sys.kpts)
    theta = torch.from_numpy(np.ascontiguousarray(np.stack([many["th0"].T] * nk))).to(dev)
    st = lt.make_step_args(ltd.LTD_STEP_REBUILD, sys.dt, torch.from_numpy(many["a_t"]).to(dev),
                           torch.from_numpy(many["a_mid"]).to(dev), theta, N_STEPS, v_r_t=vs, h_t=hs,
                           v_stride=vs.shape[1], h_stride=hs.shape[1])
    lt.run(st, 4)
    lt.run(st, N_STEPS - 4)
    torch.cuda.synchronize()
    assert lt.sync_status() == 0
    th = st["theta"].cpu().numpy()
    diff = float(np.abs(th - many["theta_one_call"]).max())
    print(f"20 k: two calls against one, max |theta difference| {diff:.1e}", flush=True)
    assert diff == 0.0
