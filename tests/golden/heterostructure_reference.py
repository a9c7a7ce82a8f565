"""Writes heterostructure_reference.npz: expected values of the heterostructure
workload (1 k-point, N_G = 30000, 26 atoms, 96 x 96 x 160 grid, N_aux = 300,
N_states = 60, dt = 0.2, 500 steps) computed by the CPU FP64 oracle only.

The workload is too large for the oracle to run inside a GPU test, so its
reference values are computed once here and stored:

* ``w``, ``eps``: the Rayleigh-Ritz rotation of the seeded start block X and the
  Ritz values of (H0, S) (oracle ``ritz_rotation``); the auxiliary basis is
  Phi = X w (Sec. 2.2, Eq. (11) stand-in).
* ``t``, ``v``, ``p``, ``s``: T_sub, V_sub, P_sub and S_sub of Phi (oracle
  ``project``; Eqs. (14)-(16)); H0_sub = T_sub + V_sub.
* ``affine_*``: J, E, delta mu and the final theta of the 500-step propagation
  with the reference potential (exponential midpoint rule, Eq. (13); Eq. (4)).
* ``series_*``: the same with a potential handed in per step, V_n = V + eps s_n
  W, h_n = h + eps s_n w (``synth.td_potential``, ``synth.potential_scale``).
  V_sub of step n is V_sub,ref + s_n D with D the oracle's rebuild of the
  perturbation eps (W, w) alone: the potential part of Eqs. (17)-(19) is linear
  in the potential, so this equals the rebuild of V_n itself to rounding.

Run: python tests/golden/heterostructure_reference.py   (a few minutes).
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "heterostructure_reference.npz")
CFG = 2


def main():
    import threadpoolctl

    from oracle import operators as op
    from oracle import propagate as pr
    from oracle import subspace as ss
    from synth import make_system, potential_scale, pulse_samples, td_potential

    cores = len(os.sched_getaffinity(0))
    op._WORKERS = cores
    t0 = time.time()
    with threadpoolctl.threadpool_limits(cores):
        sysd = make_system(CFG)
        x = sysd.kpts[0].start
        w, eps = ss.ritz_rotation(sysd, 0, x)
        phi = x @ w
        print(f"ritz {time.time() - t0:.1f} s", flush=True)
        sub = ss.project(sysd, 0, phi)
        print(f"projection {time.time() - t0:.1f} s", flush=True)
        eps_v, wfield, wblk = td_potential(sysd)
        d = ss.rebuild_v_sub(sysd, 0, phi, vr=eps_v * wfield, h=[eps_v * b for b in wblk])
        n = sysd.n_steps
        a_t, a_mid = pulse_samples(sysd, n)
        th0 = pr.initial_theta(sysd.n_aux, sysd.n_states)
        aff = pr.propagate(sub, th0, a_t, a_mid, sysd.dt, sysd.occ, sysd.omega, sysd.c_light)
        s_n = potential_scale(n)
        ser = pr.propagate(sub, th0, a_t, a_mid, sysd.dt, sysd.occ, sysd.omega, sysd.c_light,
                           v_sub_fn=lambda k: sub["V"] + s_n[k] * d)
        print(f"propagation {time.time() - t0:.1f} s", flush=True)
    np.savez(OUT, w=w, eps=eps, t=sub["T"], v=sub["V"], p=sub["P"], s=sub["S"],
             affine_j=aff["J"], affine_e=aff["E"], affine_dmu=aff["dmu"], affine_theta=aff["theta"],
             series_j=ser["J"], series_e=ser["E"], series_dmu=ser["dmu"], series_theta=ser["theta"],
             n_steps=np.array(n), eps_v=np.array(eps_v))
    print("wrote", OUT, f"{os.path.getsize(OUT) / 1e6:.1f} MB in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
