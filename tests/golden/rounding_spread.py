"""Writes rounding_spread.json: how far the oracle's own J_ind and delta mu move
when only the rounding of the computation changes, per workload.

J_ind = J - J(0) is a small difference of large currents (the static current
J(0) of the synthetic blocks is hundreds of times the induced one) and delta mu
(Sec. 2, Eq. (4)) integrates it over the whole run, so their relative errors are
amplified by cancellation.  To measure the resolution an FP64 computation can
have, the oracle is run twice on the same system: once as is, once with the
plane-wave basis listed in a random order (G triples, G+k, the columns of the
matching coefficients and the rows of the auxiliary basis permuted together).
The physics is identical; only the order of every sum over G changes.  The
relative differences of J, J_ind (against its own maximum) and delta mu (against
its own maximum) between the two runs are the spread.

The GPU parity bars on J_ind and delta mu are set from this spread (a fixed
multiple of it, never below 1e-10): a bar below the spread would demand more
accuracy than the oracle itself has.

Run: python tests/golden/rounding_spread.py   (about a minute).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "rounding_spread.json")


def _permuted(sysd, ik, perm):
    import copy

    s2 = copy.copy(sysd)
    kp = copy.copy(sysd.kpts[ik])
    kp.g_int = np.ascontiguousarray(kp.g_int[perm])
    kp.gk = np.ascontiguousarray(kp.gk[perm])
    kp.A = np.ascontiguousarray(kp.A[:, perm])
    s2.kpts = list(sysd.kpts)
    s2.kpts[ik] = kp
    return s2


def spread(cfg, n_steps=None, series=False):
    from oracle import propagate as pr
    from oracle import subspace as ss
    from synth import make_system, potential_scale, pulse_samples, td_potential

    sysd = make_system(cfg)
    phi, _ = ss.ground_state(sysd, 0)
    ng = sysd.kpts[0].n_g
    perm = np.random.default_rng(5).permutation(ng)
    rows = np.concatenate([perm, np.arange(ng, sysd.n_basis(0))])
    sys2 = _permuted(sysd, 0, perm)
    phi2 = phi[rows]
    n = sysd.n_steps if n_steps is None else n_steps
    a_t, a_mid = pulse_samples(sysd, n)
    th0 = pr.initial_theta(sysd.n_aux, sysd.n_states)
    runs = []
    for s_, p_ in ((sysd, phi), (sys2, phi2)):
        sub = ss.project(s_, 0, p_)
        vfn = None
        if series:
            eps_v, wfield, wblk = td_potential(s_)
            d = ss.rebuild_v_sub(s_, 0, p_, vr=eps_v * wfield, h=[eps_v * b for b in wblk])
            s_n = potential_scale(n)
            vfn = (lambda sub_, d_: (lambda k: sub_["V"] + s_n[k] * d_))(sub, d)
        runs.append(pr.propagate(sub, th0, a_t, a_mid, sysd.dt, sysd.occ, sysd.omega, sysd.c_light,
                                 v_sub_fn=vfn))
    r0, r1 = runs
    rel = lambda x, y: float(np.abs(x - y).max() / np.abs(y).max())
    ji0, ji1 = r0["J"] - r0["J"][0], r1["J"] - r1["J"][0]
    return dict(steps=n, j=rel(r1["J"], r0["J"]), j_ind=rel(ji1, ji0), dmu=rel(r1["dmu"], r0["dmu"]),
                max_j=float(np.abs(r0["J"]).max()), max_j_ind=float(np.abs(ji0).max()),
                max_dmu=float(np.abs(r0["dmu"]).max()))


def main():
    import threadpoolctl

    from oracle import operators as op

    op._WORKERS = max(1, min(len(os.sched_getaffinity(0)), 16))
    # the propagation's matrices are small: one BLAS thread
    threadpoolctl.threadpool_limits(1, user_api="blas")
    out = {
        "method": "oracle vs the oracle with the plane-wave order permuted (same physics, other rounding)",
        "tiny": spread(0),
        "molecule": spread(1),
        "molecule_series": spread(1, series=True),
    }
    json.dump(out, open(OUT, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
