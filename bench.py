#!/usr/bin/env python3
"""Throughput of the subspace time propagation on one MI355X.

Workload: the molecule-in-large-cell system (1 k-point, N_G = 12000 plane
waves, 2 atoms at lmax = 8 with 2 radial functions and 10 local orbitals each,
FFT grid 72^3, N_aux = 64, N_states = 5, dt = 0.2 a.u.), seeded synthetic
inputs.  One bench "step" is one time step of every state: the per-step
rebuild of the potential part of the subspace Hamiltonian from the potential
handed in for the step (a different V(r) and set of muffin-tin blocks every
step, V_n = V + eps s_n W, h_n = h + eps s_n w, resident in HBM: Theta V_n on
the rebuild grid, interstitial FFT passes, muffin-tin block products,
projection), the FP64 Chebyshev exponential of the midpoint Hamiltonian and
the current/energy/dipole observables, replayed from a hipGraph.

Prints one JSON line: state-steps/s (whole job), the roofline of the dominant
kernel stage from HIP events, the FP64 MFMA rate of the H-apply GEMMs, and the
CPU FP64 oracle on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KS state-steps/s + H-apply MFMA util, FP64 vs mixed/batched at stated dipole err"
WORKLOADS = {
    1: "molecule in large cell: 1 k-point, N_G=12000, 2 atoms lmax 8 (162 MT channels + 10 LO each), "
       "FFT grid 72^3, N_aux=64, N_states=5, dt=0.2",
    2: "heterostructure: 1 k-point, N_G=30000, 26 atoms (6 at lmax 8, 20 at lmax 6; 2 radial functions + 8 LO "
       "each), FFT grid 96x96x160, N_aux=300, N_states=60, dt=0.2",
    3: "batched k-points: 16 k (4x4x1), N_G 8000..9500 per k, 3 atoms lmax 7 (128 MT channels + 6 LO each), "
       "FFT grid 64^3, N_aux=80, N_states=20 per k, dt=0.2, all k in one launch per stage",
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6   # dense FP64 MFMA, and FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFS = 157.3  # FP32 vector (packed); the kernels here issue unpacked FP32
STAGES = ["potential", "xz_planes", "y_lines", "mt_blocks", "v_projection", "subspace_step", "map_back"]


def parse():
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--config", type=int, choices=[1, 2, 3], default=2,
                   help="2: the heterostructure (the largest single-GPU workload, headline); 1: the molecule "
                        "in a large cell; 3: 16 batched k-points")
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--mode", choices=["rebuild", "affine"], default="rebuild")
    p.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                   help="fp32: the per-step rebuild of the potential difference in FP32 (mixed mode)")
    p.add_argument("--potential", choices=["series", "static"], default="series",
                   help="rebuild from a per-step potential series (default) or from one potential")
    p.add_argument("--profile-steps", type=int, default=20)
    p.add_argument("--cpu-steps", type=int, default=None,
                   help="time steps of the CPU oracle sample (default: 50, 2 for the heterostructure)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--compare-full", action="store_true",
                   help="also time the conventional full-basis propagation of the same states at the full "
                        "basis' critical step and report seconds per simulated atomic unit of both")
    p.add_argument("--full-steps", type=int, default=3, help="timed full-basis steps (--compare-full)")
    p.add_argument("--sweep-ng", type=str, default=None, metavar="N1,N2,...",
                   help="only run the N_G sweep: per-step rebuild time of the FFT and the dense-block "
                        "interstitial routes at N_aux = 255 on the molecule system with N_G plane waves")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run 5 plain device-to-device copies of MIB MiB (counter calibration)")
    return p.parse_args()


def stage_bytes(sysd, n, nbx, nbz, rgrid, es=16):
    """Algorithmic bytes of one launch of each step stage (read + write of its own
    inputs and outputs once), summed over the k-points.  The cached grid image of
    one column is the box array c[kz][y][kx]: nbz * N2' * nbx complex values on
    the rebuild grid (N1', N2', N3'); es bytes per complex value of the slabs
    (8 for the FP32 residual, whose Theta V is float)."""
    c16 = 16
    n1, n2, n3 = rgrid
    nk = len(sysd.kpts)
    slab = nbz * n2 * nbx * n * es * nk
    ngrid = n1 * n2 * n3
    ng = sum(kp.n_g for kp in sysd.kpts)
    k_ext = ng + nk * (sysd.n_a + sysd.n_lo)
    return {
        "potential": 2 * sysd.n_grid * 8 + ngrid * es // 2,
        "xz_planes": 2 * slab + ngrid * es // 2,
        "y_lines": slab + ng * n * c16 + ng * 8,
        "v_projection": 2 * k_ext * n * c16 + nk * n * n * c16,
    }


def stage_flops(sysd, n, nbx, nbz, rgrid):
    """Algorithmic floating-point operations of the transform stages (5 L log2 L
    per complex transform of length L, 2 per complex-by-real product), summed
    over the k-points.  x/z planes: per column and rebuild plane y', inverse and
    forward x transforms of the nbz box rows, and per grid column x the inverse
    z transform, the product with Theta V and the forward z transform."""
    n1, n2, n3 = rgrid
    nk = len(sysd.kpts)
    f = lambda L: 5.0 * L * math.log2(L)
    xz = n * n2 * (2 * nbz * f(n1) + n1 * (2 * f(n3) + 2 * n3)) * nk
    y = n * nbz * nbx * f(n2) * nk
    return {"xz_planes": xz, "y_lines": y}


def traffic_from_profiles(kernel_file, stage, precision, config):
    """HBM traffic of the dominant kernel from committed rocprofv3 counter runs,
    valid only for the same workload, stage and precision while the kernel source
    is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        recs = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2403_04351_amd", "csrc", kernel_file), "rb").read()
        sha = hashlib.sha256(src).hexdigest()
        for rec in recs if isinstance(recs, list) else [recs]:
            if (rec.get("source_sha256") == sha and rec.get("stage") == stage
                    and rec.get("precision", "fp64") == precision and rec.get("config") == config):
                return rec.get("bytes_per_launch")
        return None
    except Exception:
        return None


def potential_series(sysd, n_total):
    """s_n, the per-step potential scale of the series V_n = V + eps s_n W."""
    from synth import potential_scale

    return potential_scale(n_total)


def _rel_errors(j, dmu, ref_j, ref_dmu, n_steps, against):
    rel = lambda x, r: float(np.abs(x - r).max() / np.abs(r).max())
    return dict(steps=n_steps, j=rel(j, ref_j), j_ind=rel(j - j[0], ref_j - ref_j[0]), dmu=rel(dmu, ref_dmu),
                against=against, norm="max abs difference / max abs reference, each series against its own maximum")


def dipole_error_stored(st, n_steps):
    """Relative errors of J, J_ind and delta mu of the heterostructure run (first
    n_steps, at most the 500 stored) against the FP64 oracle's values for the same
    per-step potential, stored by tests/golden/heterostructure_reference.py."""
    ref = np.load(os.path.join(ROOT, "tests", "golden", "heterostructure_reference.npz"))
    n = min(n_steps, int(ref["n_steps"]))
    j = st["j"][: n + 1].cpu().numpy()
    dmu = st["dmu"][: n + 1].cpu().numpy()
    return _rel_errors(j, dmu, ref["series_j"][: n + 1], ref["series_dmu"][: n + 1], n,
                       "FP64 oracle (stored), same per-step potential")


def dipole_error_oracle(sysd, st, n_steps):
    """Relative errors of J, J_ind and delta mu of the run (first n_steps) against
    the FP64 oracle with the same per-step potential (the oracle's V_sub is linear
    in the potential: V_ref + s_n D, D its rebuild of the perturbation alone).
    Part of the CPU oracle leg."""
    from oracle import propagate as pr
    from oracle import subspace as ss
    from synth import pulse_samples, td_potential

    phi, _ = ss.ground_state(sysd, 0)
    sub = ss.project(sysd, 0, phi)
    eps, wfield, wblk = td_potential(sysd)
    d = ss.rebuild_v_sub(sysd, 0, phi, vr=eps * wfield, h=[eps * w for w in wblk])
    s_n = potential_series(sysd, n_steps)
    a_t, a_mid = pulse_samples(sysd, n_steps)
    # the GPU run starts from the Ritz basis of the library; the oracle uses its own
    # Ritz basis of the same start block (the same subspace and states to rounding)
    ref = pr.propagate(sub, pr.initial_theta(sysd.n_aux, sysd.n_states), a_t, a_mid, sysd.dt, sysd.occ,
                       sysd.omega, sysd.c_light, v_sub_fn=lambda k: sub["V"] + s_n[k] * d, n_steps=n_steps)
    j = st["j"][: n_steps + 1].cpu().numpy()
    dmu = st["dmu"][: n_steps + 1].cpu().numpy()
    return _rel_errors(j, dmu, ref["J"], ref["dmu"], n_steps, "FP64 oracle, same per-step potential")


def cpu_baseline(sysd, n_steps, mode, series, ks):
    """The FP64 oracle, timed on the host cores over a bounded number of steps of
    the k-points ks (setup excluded)."""
    import threadpoolctl

    from oracle import operators as op
    from oracle import propagate as pr
    from oracle import subspace as ss
    from synth import pulse_samples

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    op._WORKERS = cores
    t = 0.0
    with threadpoolctl.threadpool_limits(cores):
        a_t, a_mid = pulse_samples(sysd, n_steps)
        if mode == "rebuild" and series:
            from synth import td_potential

            eps, wfield, wblk = td_potential(sysd)
            s_n = potential_series(sysd, n_steps)
        for k in ks:
            if sysd.cfg == 2:  # set-up (Ritz basis, projection) from the oracle's stored values
                ref = np.load(os.path.join(ROOT, "tests", "golden", "heterostructure_reference.npz"))
                phi = sysd.kpts[k].start @ ref["w"]
                sub = dict(T=ref["t"], V=ref["v"], P=ref["p"], S=ref["s"], H0=ref["t"] + ref["v"])
            else:
                phi, _ = ss.ground_state(sysd, k)
                sub = ss.project(sysd, k, phi)
            vfn = None
            if mode == "rebuild" and series:
                def vfn(n, k=k, phi=phi):
                    return ss.rebuild_v_sub(sysd, k, phi, vr=sysd.vr + eps * s_n[n] * wfield,
                                            h=[h + eps * s_n[n] * w for h, w in zip(sysd.h, wblk)])
            elif mode == "rebuild":
                def vfn(n, k=k, phi=phi):
                    return ss.rebuild_v_sub(sysd, k, phi)
            t0 = time.perf_counter()
            pr.propagate(sub, pr.initial_theta(sysd.n_aux, sysd.n_states), a_t, a_mid, sysd.dt, sysd.occ,
                         sysd.omega, sysd.c_light, v_sub_fn=vfn, n_steps=n_steps)
            t += time.perf_counter() - t0
    kdesc = "the k-point" if len(sysd.kpts) == 1 else f"{len(ks)} of the {len(sysd.kpts)} k-points"
    return dict(value=len(ks) * sysd.n_states * n_steps / t, unit="state-steps/s", cores=cores, kind="oracle",
                sample=f"first {n_steps} time steps ({mode}, {'per-step potential' if series else 'one potential'}) "
                       f"of {kdesc} of the same workload, setup excluded; {t:.2f} s")


def compare_full(args, torch, lt, sysd, phi, emin, sub_ms_per_step):
    """Seconds per simulated atomic unit of time: the subspace propagation (its
    dt) against the conventional one in the full basis (Sec. 2.1, Eq. (10)) at the
    full basis' critical step 0.2 / (eps_max - eps_min) (Sec. 3.1, Eq. (20)),
    explicit order-4 Taylor steps with conjugate-gradient solves of S."""
    dev = phi.device
    nb = sysd.n_basis(0)
    rng = np.random.default_rng(91)
    x0 = torch.from_numpy(rng.standard_normal(nb) + 1j * rng.standard_normal(nb)).to(dev)
    t0 = time.perf_counter()
    eps_max = lt.full_spectrum(0, x0, iters=30, cg_tol=1e-8)
    t_spec = time.perf_counter() - t0
    dt_full = 0.2 / (eps_max - emin)
    c0 = 0.5 * (eps_max + emin)
    c = phi[: sysd.n_states].clone()
    a_mid = np.full(args.full_steps + 1, 0.005)
    cg_tol = 1e-10
    lt.propagate_full(0, c, dt_full, 4, c0, a_mid[:1], cg_max_iter=5000, cg_tol=cg_tol)  # warm-up step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, its = lt.propagate_full(0, c, dt_full, 4, c0, a_mid[1:], cg_max_iter=5000, cg_tol=cg_tol)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.full_steps
    sub_s_au = sub_ms_per_step * 1e-3 / sysd.dt
    full_s_au = t_step / dt_full
    return dict(states=sysd.n_states, dt_cr_full=dt_full, eps_max_power_iteration=eps_max, eps_min_ritz=emin,
                power_iteration_s=round(t_spec, 3), order=4, cg_tol=cg_tol, cg_iters_max=its, cg_resid_max=res,
                steps_timed=args.full_steps, s_per_step=t_step, s_per_au=full_s_au,
                subspace_dt=sysd.dt, subspace_s_per_au=sub_s_au, speedup=full_s_au / sub_s_au)


def sweep_ng(args, torch, ltd, _lib, dev):
    """Per-step rebuild time of the two interstitial routes as N_G grows (the
    paper's basis-size study, Sec. 3.2): FFT (flat in N_G) against dense N_G x N_G
    blocks (N_G^2 storage and work), N_aux = 255, the molecule system's cell,
    atoms and 72^3 grid, a potential handed in per step."""
    from synth import make_system, pulse_samples, td_potential

    rows = []
    for ng in [int(x) for x in args.sweep_ng.split(",")]:
        sysd = make_system(1, n_g=ng, n_aux=255, n_states=5)
        n_steps = 20
        a_t, a_mid = pulse_samples(sysd, 5 + n_steps)
        eps, wfield, wblk = td_potential(sysd)
        for route, rname in ((_lib.LTD_ROUTE_FFT, "fft"), (_lib.LTD_ROUTE_MM, "mm")):
            t0 = time.perf_counter()
            lt = ltd.Ltd(sysd, device=dev, route=route)
            phi = ltd.colmajor(sysd.kpts[0].start, dev)
            lt.ritz_basis(0, phi)
            lt.project_subspace(0, phi)
            if route == _lib.LTD_ROUTE_FFT:
                lt.autotune()
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            sd = torch.from_numpy(potential_series(sysd, 5 + n_steps)).to(dev)[:, None]
            v0 = torch.from_numpy(np.ascontiguousarray(sysd.vr.ravel())).to(dev)
            w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
            wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
            vs = (v0[None, :] + eps * sd * w0[None, :]).contiguous()
            hs = (lt.h[None, :] + eps * sd * wb[None, :]).contiguous()
            th0 = np.zeros((1, sysd.n_states, sysd.n_aux), dtype=np.complex128)
            for j in range(sysd.n_states):
                th0[0, j, j] = 1.0
            st = lt.make_step_args(ltd.LTD_STEP_REBUILD, sysd.dt, torch.from_numpy(a_t).to(dev),
                                   torch.from_numpy(a_mid).to(dev), torch.from_numpy(th0).to(dev), 5 + n_steps,
                                   v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
            lt.run(st, 5)
            lt.prepare(st, n_steps)
            torch.cuda.synchronize()
            s = torch.cuda.current_stream(dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            lt.run(st, n_steps)
            e1.record(s)
            torch.cuda.synchronize()
            if lt.sync_status() != 0:
                print(f"device status {lt.sync_status()} (N_G {ng}, {rname})", file=sys.stderr)
                return 1
            ms = e0.elapsed_time(e1) / n_steps
            rows.append(dict(n_g=ng, n_basis=sysd.n_basis(0), route=rname, ms_per_step=round(ms, 4),
                             setup_s=round(t_setup, 2), j_last=float(st["j"][5 + n_steps].item())))
            print(f"[sweep] N_G {ng} {rname}: {ms:.3f} ms/step, setup {t_setup:.1f} s", file=sys.stderr, flush=True)
            lt.close()
            del lt, st, vs, hs, phi
            torch.cuda.empty_cache()
    print(json.dumps({"sweep": "per-step rebuild time vs N_G, FFT and dense-block interstitial routes",
                      "n_aux": 255, "n_states": 5, "grid": [72, 72, 72], "steps_timed": 20, "rows": rows}),
          flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the k-point and column "
              "sharding across GPUs is described in the design notes but not run.", file=sys.stderr)
        return 2
    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "reads_plus_writes_per_copy": 2 * nbytes}))
        return 0
    from paper_2403_04351_amd import _lib, ltd
    from synth import make_system, pulse_samples

    dev = torch.device("cuda:0")
    if args.sweep_ng:
        return sweep_ng(args, torch, ltd, _lib, dev)
    sysd = make_system(args.config)
    nk = len(sysd.kpts)

    prec = _lib.LTD_FP64 if args.precision == "fp64" else _lib.LTD_FP32_RESID
    lt = ltd.Ltd(sysd, device=dev, precision=prec)
    # auxiliary basis per k: Rayleigh-Ritz vectors of the seeded start block, on the GPU
    phis = []
    for k in range(nk):
        phi = ltd.colmajor(sysd.kpts[k].start[:, :sysd.n_aux], dev)
        lt.ritz_basis(k, phi)
        lt.project_subspace(k, phi)
        phis.append(phi)
    phi = phis[0]
    emin, emax, dtcr = lt.subspace_info(0)
    tuned = lt.autotune() if args.mode == "rebuild" else None
    mode = ltd.LTD_STEP_REBUILD if args.mode == "rebuild" else ltd.LTD_STEP_AFFINE
    total = args.warmup + args.steps + args.profile_steps
    a_t, a_mid = pulse_samples(sysd, total)
    at = torch.from_numpy(a_t).to(dev)
    am = torch.from_numpy(a_mid).to(dev)
    th0 = np.zeros((nk, sysd.n_states, sysd.n_aux), dtype=np.complex128)
    for j in range(sysd.n_states):
        th0[:, j, j] = 1.0
    theta = torch.from_numpy(th0).to(dev)
    pot = {}
    series = args.mode == "rebuild" and args.potential == "series"
    if series:
        from synth import td_potential

        eps, wfield, wblk = td_potential(sysd)
        sd = torch.from_numpy(potential_series(sysd, total)).to(dev)[:, None]
        v0 = torch.from_numpy(np.ascontiguousarray(sysd.vr.ravel())).to(dev)
        w0 = torch.from_numpy(np.ascontiguousarray(wfield.ravel())).to(dev)
        wb = torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in wblk])).to(dev)
        vs = (v0[None, :] + eps * sd * w0[None, :]).contiguous()
        hs = (lt.h[None, :] + eps * sd * wb[None, :]).contiguous()
        pot = dict(v_r_t=vs, h_t=hs, v_stride=vs.shape[1], h_stride=hs.shape[1])
    st = lt.make_step_args(mode, sysd.dt, at, am, theta, total, **pot)
    s = torch.cuda.current_stream(dev)
    if args.warmup:
        lt.run(st, args.warmup)
    # the graphs the timed call replays are captured here, outside the timed region
    lt.prepare(st, args.steps)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    lt.run(st, args.steps)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    status = lt.sync_status()
    if status != 0:
        print(f"device status {status} after the timed run", file=sys.stderr)
        return 1
    value = nk * sysd.n_states * args.steps / (ms / 1e3)

    # stage profile (HIP events between stages, eager)
    stage_ms = lt.profile_steps(st, max(1, args.profile_steps))
    prof = {STAGES[i]: round(stage_ms[i] * 1e3, 3) for i in range(len(STAGES))}
    rgrid = lt.rebuild_grid()
    nbx = 2 * int(np.abs(sysd.kpts[0].g_int[:, 0]).max()) + 1
    nbz = 2 * int(np.abs(sysd.kpts[0].g_int[:, 2]).max()) + 1
    sb = stage_bytes(sysd, sysd.n_aux, nbx, nbz, rgrid, 16 if args.precision == "fp64" else 8)
    hbm_stages = {k: v for k, v in prof.items() if k in sb}
    dom = max(hbm_stages, key=hbm_stages.get)
    dom_us = hbm_stages[dom]
    affine_only = dom_us <= 0.0  # AFFINE: no rebuild stage ran; the step is the exponential
    if affine_only:
        dom_us = 1.0
    achieved = sb[dom] / (dom_us * 1e-6) / 1e9
    kernel_file = "fft.hip" if dom in ("potential", "xz_planes", "y_lines") else "api.hip"
    traffic = traffic_from_profiles(kernel_file, dom, args.precision, args.config)
    fl = stage_flops(sysd, sysd.n_aux, nbx, nbz, rgrid).get(dom)
    alu_peak = FP64_PEAK_TFS if args.precision == "fp64" else FP32_PEAK_TFS
    # the binding roofline: the resource whose peak needs the longer time for the stage's work
    if fl is not None and fl / (alu_peak * 1e12) > sb[dom] / (HBM_PEAK_GBS * 1e9):
        tf = fl / (dom_us * 1e-6) / 1e12
        roofline = dict(bound="alu", kernel=dom, achieved=round(tf, 2), peak=alu_peak, unit="TFLOP/s",
                        frac=round(tf / alu_peak, 4), traffic=traffic, flops_per_launch=fl,
                        bytes_per_launch=sb[dom], avg_launch_us=dom_us,
                        hbm=dict(achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                                 frac=round(achieved / HBM_PEAK_GBS, 4)))
    else:
        roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, bytes_per_launch=sb[dom],
                        avg_launch_us=dom_us)

    if affine_only:
        roofline = None
    # H-apply MFMA rate: the muffin-tin GEMMs of one apply at n = N_aux
    apms, _, _ = lt.profile_apply(0, phi)
    n = sysd.n_aux
    ng = sysd.kpts[0].n_g
    f_k1 = 8.0 * sysd.n_a * ng * n
    f_k3 = 8.0 * ng * sysd.n_a * 2 * n
    t_k = (apms[3] + apms[5]) * 1e-3
    tfs = (f_k1 + f_k3) / t_k / 1e12
    h_apply = dict(gemm_tflops=round(tfs, 2), peak_tflops=FP64_PEAK_TFS, frac=round(tfs / FP64_PEAK_TFS, 4),
                   k1_us=round(apms[3] * 1e3, 1), k3_us=round(apms[5] * 1e3, 1),
                   apply_total_us=round(sum(apms[:6]) * 1e3, 1))

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "state-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (WORKLOADS[args.config] + f", {args.mode} mode"
                         + (", potential handed in per step" if series else "")
                         + (", FP64" if args.precision == "fp64" else ", FP32 residual rebuild on FP64")),
            "n_k": nk, "n_g": [kp.n_g for kp in sysd.kpts] if nk > 1 else ng, "n_aux": n,
            "n_states": sysd.n_states, "grid": list(sysd.grid),
            "rebuild_grid": list(rgrid), "mode": args.mode, "potential": args.potential if
            args.mode == "rebuild" else None, "precision": args.precision,
        },
        "wall_s": round(wall, 4),
        "stage_us": prof,
        "roofline": roofline,
        "tuning": tuned,
        "h_apply": h_apply,
        "subspace": dict(eps_min=emin, eps_max=emax, dt_cr=dtcr),
        "dmu_final": float(st["dmu"][args.warmup + args.steps].item()),
        "state_drift": lt.state_drift(theta),
    }
    if series and nk == 1 and args.config == 2:
        out["dipole_error"] = dipole_error_stored(st, args.warmup + args.steps)
    elif series and nk == 1 and not args.no_cpu_baseline:
        out["dipole_error"] = dipole_error_oracle(sysd, st, args.warmup + args.steps)
    if args.compare_full and nk == 1:
        out["conventional"] = compare_full(args, torch, lt, sysd, phi, emin, ms / args.steps)
    if not args.no_cpu_baseline:
        ks = [0] if nk == 1 else [0, 1]
        cpu_steps = args.cpu_steps if args.cpu_steps is not None else (3 if nk > 1 else 2 if args.config == 2 else 50)
        out["cpu_baseline"] = cpu_baseline(sysd, cpu_steps, args.mode, series, ks)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
