"""Python binding of the ltd library: argument marshalling between torch
tensors and the C ABI of include/ltd.h.  Every computation runs in the HIP
library; torch only provides device memory and the stream.

Matrix convention: a column-major rows x cols matrix is a contiguous torch
tensor of shape (cols, rows) (``colmajor``/``to_numpy`` convert from/to a
numpy (rows, cols) array).
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import AdjointArgs, StepArgs, SystemDesc, check

LTD_STEP_REBUILD = _lib.LTD_STEP_REBUILD
LTD_STEP_AFFINE = _lib.LTD_STEP_AFFINE


def _torch():
    import torch

    return torch


def colmajor(a: np.ndarray, device) -> "torch.Tensor":
    """numpy (rows, cols) -> device tensor (cols, rows) holding the column-major matrix."""
    t = _torch()
    return t.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(device)


def to_numpy(x) -> np.ndarray:
    """device tensor (cols, rows) -> numpy (rows, cols)."""
    return x.detach().cpu().numpy().T


def _ptr(x) -> int:
    return 0 if x is None else int(x.data_ptr())


class Ltd:
    """One ltd system bound to a device workspace."""

    def __init__(self, sys, device="cuda", max_cols=None, precision=_lib.LTD_FP64, route=_lib.LTD_ROUTE_FFT):
        torch = _torch()
        self.lib = _lib.load()
        self.sysdef = sys
        self.device = torch.device(device)
        dev = self.device
        kp = sys.kpts
        self.n_k = len(kp)
        self.n_aux = sys.n_aux
        self.n_states = sys.n_states
        self.n_basis = [sys.n_basis(k) for k in range(self.n_k)]
        # host arrays (kept alive: the library copies them at create)
        self._n_g = np.array([k.n_g for k in kp], dtype=np.int32)
        self._g_int = np.ascontiguousarray(np.concatenate([k.g_int for k in kp]).astype(np.int32))
        self._gk = np.ascontiguousarray(np.concatenate([k.gk for k in kp]).astype(np.float64))
        self._n_mt = np.array([a.n_mt for a in sys.atoms], dtype=np.int32)
        self._n_lo = np.array([a.n_lo for a in sys.atoms], dtype=np.int32)
        self._kw = np.array([k.weight for k in kp], dtype=np.float64)
        # device arrays (kept alive: the library keeps their pointers)
        self.theta_r = torch.from_numpy(np.ascontiguousarray(sys.theta.ravel())).to(dev)
        self.v_r = torch.from_numpy(np.ascontiguousarray(sys.vr.ravel())).to(dev)
        amats = [np.ascontiguousarray(k.A.T).ravel() for k in kp]
        if sum(a.size for a in amats) == 0:
            amats = [np.zeros(1, dtype=np.complex128)]
        self.amat = torch.from_numpy(np.concatenate(amats)).to(dev)
        def blk(xs):
            if not xs:  # no atoms: a placeholder the library never reads
                return torch.zeros(1, dtype=torch.complex128, device=dev)
            return torch.from_numpy(np.concatenate([np.ascontiguousarray(x.T).ravel() for x in xs])).to(dev)

        self.h = blk(sys.h)
        self.o = blk(sys.o)
        self.pz = blk(sys.pz)
        self.max_cols = max(sys.n_aux, sys.n_states) if max_cols is None else max_cols
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
        self._desc = SystemDesc(
            n_k=self.n_k, n_g=ip(self._n_g), g_int=self._g_int.ctypes.data_as(C.POINTER(C.c_int32)),
            gk_cart=self._gk.ctypes.data_as(C.POINTER(C.c_double)), grid=(C.c_int * 3)(*sys.grid),
            theta_r=_ptr(self.theta_r), v_r=_ptr(self.v_r), n_atoms=sys.n_atoms, n_mt=ip(self._n_mt),
            n_lo=ip(self._n_lo), amat=_ptr(self.amat), h=_ptr(self.h), o=_ptr(self.o), pz=_ptr(self.pz),
            omega=sys.omega, c_light=sys.c_light, occ=sys.occ,
            k_weight=self._kw.ctypes.data_as(C.POINTER(C.c_double)), n_aux=sys.n_aux,
            n_states=sys.n_states, max_cols=self.max_cols, interstitial_route=route)
        wsb = C.c_size_t(0)
        handle = C.c_void_p(0)
        check(self.lib.ltd_create(C.byref(self._desc), precision, C.byref(wsb), C.byref(handle)), "ltd_create")
        self.handle = handle
        self.ws_bytes = wsb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        check(self.lib.ltd_bind_workspace(self.handle, _ptr(self.ws), self.ws_bytes, self.stream()),
              "ltd_bind_workspace")
        self._phis = {}

    # ------------------------------------------------------------------
    def stream(self) -> int:
        return int(_torch().cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.ltd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_status(self) -> int:
        return int(self.lib.ltd_sync_status(self.handle, self.stream()))

    # ------------------------------------------------------------------
    def apply_hs(self, k: int, c, a_z: float = 0.0):
        """H(A) C and S C; c: tensor (n, N_basis) (column-major N_basis x n)."""
        torch = _torch()
        n, nb = c.shape
        hc = torch.empty_like(c)
        sc = torch.empty_like(c)
        a = (C.c_double * 3)(0.0, 0.0, float(a_z))
        check(self.lib.ltd_apply_HS(self.handle, k, a, _ptr(c), nb, n, _ptr(hc), nb, _ptr(sc), nb, self.stream()),
              "ltd_apply_HS")
        return hc, sc

    def project_subspace(self, k: int, phi, c=None):
        """Binds phi (tensor (n_aux, N_basis)); returns H0_sub, S_sub (tensors (n, n),
        column-major) and, if c is given, theta (tensor (n_states, n_aux))."""
        torch = _torch()
        n = self.n_aux
        h0 = torch.empty((n, n), dtype=torch.complex128, device=self.device)
        s = torch.empty_like(h0)
        th = None
        if c is not None:
            th = torch.empty((c.shape[0], n), dtype=torch.complex128, device=self.device)
        self._phis[k] = phi
        check(self.lib.ltd_project_subspace(self.handle, k, _ptr(phi), phi.shape[1], n, _ptr(h0), _ptr(s),
                                            _ptr(c), c.shape[1] if c is not None else 0,
                                            c.shape[0] if c is not None else 0, _ptr(th), self.stream()),
              "ltd_project_subspace")
        return h0, s, th

    def ritz_basis(self, k: int, x):
        """Rotates x (tensor (n_aux, N_basis)) in place into Ritz vectors; returns eps."""
        torch = _torch()
        eps = torch.empty(self.n_aux, dtype=torch.float64, device=self.device)
        check(self.lib.ltd_ritz_basis(self.handle, k, _ptr(x), x.shape[1], _ptr(eps), self.stream()),
              "ltd_ritz_basis")
        return eps

    def propagate_full(self, k: int, c, dt: float, order: int, c0: float, a_mid, cg_max_iter: int = 500,
                       cg_tol: float = 1e-13):
        """Advances c (tensor (n, N_basis), in place) len(a_mid) explicit steps in the
        full basis; returns (largest CG residual, most CG iterations)."""
        a = np.ascontiguousarray(np.asarray(a_mid, dtype=np.float64))
        res, its = C.c_double(), C.c_int()
        fa = _lib.FullArgs(dt=dt, order=order, c0=c0, a_mid=a.ctypes.data_as(C.POINTER(C.c_double)),
                           cg_max_iter=cg_max_iter, cg_tol=cg_tol, cg_resid=C.pointer(res), cg_iters=C.pointer(its))
        n, nb = c.shape
        check(self.lib.ltd_propagate_full(self.handle, k, _ptr(c), nb, n, C.byref(fa), len(a), self.stream()),
              "ltd_propagate_full")
        return res.value, its.value

    def full_spectrum(self, k: int, x0, iters: int = 60, cg_max_iter: int = 500, cg_tol: float = 1e-12):
        """Largest eigenvalue of the full (H0, S) by power iteration from x0 (tensor (N_basis,))."""
        e = C.c_double()
        check(self.lib.ltd_full_spectrum(self.handle, k, _ptr(x0), iters, cg_max_iter, cg_tol, C.byref(e),
                                         self.stream()), "ltd_full_spectrum")
        return e.value

    def subspace_info(self, k: int):
        a, b, d = C.c_double(), C.c_double(), C.c_double()
        check(self.lib.ltd_subspace_info(self.handle, k, C.byref(a), C.byref(b), C.byref(d)), "ltd_subspace_info")
        return a.value, b.value, d.value

    # ------------------------------------------------------------------
    def autotune(self):
        """Times the rebuild's launch shapes and projection split targets on the
        bound subspaces and keeps the fastest; returns the choice and the timings."""
        choice = (C.c_int * 3)()
        times = (C.c_double * 16)()
        check(self.lib.ltd_autotune(self.handle, choice, times, self.stream()), "ltd_autotune")
        return dict(xz_shape=choice[0], projection_blocks=choice[1], n_shapes=choice[2],
                    times_us=list(times[:choice[2] + 4]))

    def state_drift(self, theta, reorthonormalize=False):
        """max |theta^H S_sub theta - I| over the k-points; with reorthonormalize the
        states are replaced (in place) by their Loewdin orthonormalisation."""
        d = C.c_double()
        check(self.lib.ltd_state_drift(self.handle, _ptr(theta), 1 if reorthonormalize else 0, C.byref(d),
                                       self.stream()), "ltd_state_drift")
        return d.value

    def set_tuning(self, xz_shape, projection_blocks):
        """Sets the rebuild's launch shape and the projection split target."""
        choice = (C.c_int * 2)(xz_shape, projection_blocks)
        check(self.lib.ltd_set_tuning(self.handle, choice), "ltd_set_tuning")

    def rebuild_grid(self):
        """FFT lengths (N1, N2, N3) of the per-step rebuild."""
        out = (C.c_int * 3)()
        check(self.lib.ltd_rebuild_grid(self.handle, out), "ltd_rebuild_grid")
        return tuple(out)

    def make_step_args(self, mode, dt, a_t, a_mid, theta, n_steps, c_out=None, v_r_t=None, h_t=None,
                       v_stride=0, h_stride=0, taylor_order=0, nexc=False, theta_hist=None):
        """Device buffers and the StepArgs for a run of n_steps; theta (n_k, n_states, n_aux).
        v_stride / h_stride: elements between the potentials / blocks of consecutive
        steps when v_r_t / h_t hold one per step (0: one for every step).
        taylor_order > 0: the explicit truncated-Taylor step; nexc: also the
        excited-electron series st["nexc"]; theta_hist (hist_len, n_k, n_states,
        n_aux): the states before each step are recorded in slot step mod hist_len."""
        torch = _torch()
        dev = self.device
        st = dict(
            step=torch.zeros(1, dtype=torch.int32, device=dev),
            j=torch.zeros(n_steps + 1, dtype=torch.float64, device=dev),
            e=torch.zeros(n_steps + 1, dtype=torch.float64, device=dev),
            dmu=torch.zeros(n_steps + 1, dtype=torch.float64, device=dev),
            nexc=torch.zeros(n_steps + 1, dtype=torch.float64, device=dev) if nexc else None,
            a_t=a_t, a_mid=a_mid, theta=theta, c_out=c_out, v_r_t=v_r_t, h_t=h_t,
        )
        st["args"] = StepArgs(mode=mode, dt=dt, a_t=_ptr(a_t), a_mid=_ptr(a_mid), step=_ptr(st["step"]),
                              v_r_t=_ptr(v_r_t), h_t=_ptr(h_t), theta=_ptr(theta), c_out=_ptr(c_out),
                              j_out=_ptr(st["j"]), e_out=_ptr(st["e"]), dmu_out=_ptr(st["dmu"]),
                              v_stride=v_stride, h_stride=h_stride, taylor_order=taylor_order,
                              nexc_out=_ptr(st["nexc"]), theta_hist=_ptr(theta_hist),
                              hist_len=0 if theta_hist is None else theta_hist.shape[0])
        st["theta_hist"] = theta_hist
        return st

    def step(self, st):
        check(self.lib.ltd_propagate_step(self.handle, C.byref(st["args"]), self.stream()), "ltd_propagate_step")

    def run(self, st, n_steps: int):
        check(self.lib.ltd_propagate(self.handle, C.byref(st["args"]), n_steps, self.stream()), "ltd_propagate")

    def prepare(self, st, n_steps: int):
        """Captures the graphs a ``run(st, n_steps)`` replays, without running a step."""
        check(self.lib.ltd_propagate_prepare(self.handle, C.byref(st["args"]), n_steps, self.stream()),
              "ltd_propagate_prepare")

    def propagate(self, mode, dt, a_t, a_mid, theta, n_steps, graph=True, c_out=None, v_r_t=None, h_t=None,
                  v_stride=0, h_stride=0, reorth_every=None, taylor_order=0, nexc=False):
        """n_steps steps; reorth_every = K: after every K steps the states are
        reorthonormalised (Loewdin) and the drift before it is kept in st["drift"]."""
        st = self.make_step_args(mode, dt, a_t, a_mid, theta, n_steps, c_out, v_r_t, h_t, v_stride, h_stride,
                                 taylor_order, nexc)
        if reorth_every:
            st["drift"] = []
            done = 0
            while done < n_steps:
                k = min(int(reorth_every), n_steps - done)
                if graph:
                    self.run(st, k)
                else:
                    for _ in range(k):
                        self.step(st)
                done += k
                st["drift"].append(self.state_drift(theta, reorthonormalize=done < n_steps))
            return st
        if graph:
            self.run(st, n_steps)
        else:
            for _ in range(n_steps):
                self.step(st)
        return st

    def profile_steps(self, st, n_steps: int):
        """Mean per-step duration (ms) of each stage over n_steps eager steps (the
        x/z stage: the mean of four back-to-back launches of its kernel)."""
        buf = (C.c_double * _lib.LTD_PROFILE_STAGES)()
        check(self.lib.ltd_profile_steps(self.handle, C.byref(st["args"]), n_steps, buf, self.stream()),
              "ltd_profile_steps")
        return list(buf)

    def profile_apply(self, k: int, c):
        """Stage durations (ms) of one H/S apply of the block c at A = 0."""
        torch = _torch()
        n, nb = c.shape
        hc = torch.empty_like(c)
        sc = torch.empty_like(c)
        buf = (C.c_double * _lib.LTD_PROFILE_STAGES)()
        check(self.lib.ltd_profile_apply(self.handle, k, _ptr(c), nb, n, _ptr(hc), _ptr(sc), nb, buf,
                                         self.stream()), "ltd_profile_apply")
        return list(buf), hc, sc

    def pulse_loss(self, st, n_steps: int):
        """L = delta mu(T) / Omega of a run of n_steps (a device scalar)."""
        torch = _torch()
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        check(self.lib.ltd_pulse_loss(self.handle, _ptr(st["dmu"]), n_steps, _ptr(loss), self.stream()),
              "ltd_pulse_loss")
        return loss

    def adjoint_step(self, st, n, n_steps, mu_next, mu_out, dl_da_mid, dl_da_t, terminal=False):
        a = AdjointArgs(fwd=C.pointer(st["args"]), n=n, terminal=1 if terminal else 0, n_steps=n_steps,
                        mu_next=_ptr(mu_next), mu_out=_ptr(mu_out), dl_da_mid=_ptr(dl_da_mid),
                        dl_da_t=_ptr(dl_da_t))
        check(self.lib.ltd_propagate_step_adjoint(self.handle, C.byref(a), self.stream()),
              "ltd_propagate_step_adjoint")

    def knot_samples(self, q, t_end, dt, n_steps):
        torch = _torch()
        a_t = torch.empty(n_steps + 1, dtype=torch.float64, device=self.device)
        a_mid = torch.empty(n_steps, dtype=torch.float64, device=self.device)
        check(self.lib.ltd_knot_samples(_ptr(q), q.numel(), t_end, dt, n_steps, _ptr(a_t), _ptr(a_mid),
                                        self.stream()), "ltd_knot_samples")
        return a_t, a_mid

    def knot_gradient(self, g_t, g_mid, dt, n_knots, t_end):
        torch = _torch()
        g = torch.empty(n_knots, dtype=torch.float64, device=self.device)
        check(self.lib.ltd_knot_gradient(_ptr(g_t), _ptr(g_mid), g_mid.numel(), dt, n_knots, t_end, _ptr(g),
                                         self.stream()), "ltd_knot_gradient")
        return g


def pulse_samples(kind: int, params, dt: float, n_steps: int, device="cuda"):
    """A(t_n) (n = 0..n_steps) and A(t_n + dt/2) of a pulse kind (LTD_PULSE_*)
    with its four parameters, on the device."""
    torch = _torch()
    lib = _lib.load()
    a_t = torch.empty(n_steps + 1, dtype=torch.float64, device=device)
    a_mid = torch.empty(n_steps, dtype=torch.float64, device=device)
    p = (C.c_double * 4)(*[float(x) for x in params])
    stream = int(torch.cuda.current_stream(a_t.device).cuda_stream)
    check(lib.ltd_pulse_samples(kind, p, dt, n_steps, _ptr(a_t), _ptr(a_mid), stream), "ltd_pulse_samples")
    return a_t, a_mid


def polarizability(j, a_t, dt: float, omega_cell: float, c_light: float, w, gamma: float):
    """alpha_zz(w) (complex tensor, one per frequency of w) from the current series j
    and the potential samples a_t of a run (Eq. (5))."""
    torch = _torch()
    lib = _lib.load()
    out = torch.empty(w.numel(), dtype=torch.complex128, device=j.device)
    stream = int(torch.cuda.current_stream(j.device).cuda_stream)
    check(lib.ltd_polarizability(_ptr(j), _ptr(a_t), j.numel() - 1, dt, omega_cell, c_light, _ptr(w), w.numel(),
                                 gamma, _ptr(out), stream), "ltd_polarizability")
    return out


def chebyshev_coefficients(tau: float, kmax: int):
    lib = _lib.load()
    buf = (C.c_double * (2 * (kmax + 1)))()
    deg = C.c_int(0)
    check(lib.ltd_chebyshev_coefficients(tau, kmax, buf, C.byref(deg)), "ltd_chebyshev_coefficients")
    a = np.frombuffer(buf, dtype=np.float64).copy()
    return a[0::2] + 1j * a[1::2], deg.value


# ----------------------------------------------------------------------
# Pulse gradients: forward propagation with theta checkpoints, backward by
# recomputing each segment and running the adjoint steps in reverse.
# ----------------------------------------------------------------------
def pulse_forward(lt: Ltd, mode, dt, q, t_end, n_steps, theta0, checkpoint=50, potential=None):
    """Propagates theta0 (n_k, n_states, n_aux) under the piecewise-linear pulse
    with knots q; returns (loss, state) with loss = dt sum_n w_n (J_n - J_0).
    potential: optional dict of make_step_args keywords (v_r_t, h_t, v_stride,
    h_stride) for REBUILD with a potential handed in per step."""
    torch = _torch()
    pot = dict(potential or {})
    a_t, a_mid = lt.knot_samples(q, t_end, dt, n_steps)
    theta = theta0.clone()
    st = lt.make_step_args(mode, dt, a_t, a_mid, theta, n_steps, **pot)
    ckpt = {0: theta.clone()}
    done = 0
    while done < n_steps:
        m = min(checkpoint, n_steps - done)
        lt.run(st, m) if m > 1 else lt.step(st)
        done += m
        ckpt[done] = theta.clone()
    loss = lt.pulse_loss(st, n_steps)
    return loss, dict(st=st, ckpt=ckpt, a_t=a_t, a_mid=a_mid, checkpoint=checkpoint, pot=pot)


def pulse_backward(lt: Ltd, mode, dt, q, t_end, n_steps, fw):
    """dL/dq for the forward run ``fw`` (checkpointed adjoint)."""
    torch = _torch()
    dev = lt.device
    shape = (lt.n_k, lt.n_states, lt.n_aux)
    mu = torch.zeros(shape, dtype=torch.complex128, device=dev)
    g_mid = torch.zeros(n_steps, dtype=torch.float64, device=dev)
    g_t = torch.zeros(n_steps + 1, dtype=torch.float64, device=dev)
    ck = fw["checkpoint"]
    pot = fw["pot"]
    # terminal point
    th_n = fw["ckpt"][n_steps]
    sa = lt.make_step_args(mode, dt, fw["a_t"], fw["a_mid"], th_n, n_steps, **pot)
    lt.adjoint_step(sa, n_steps, n_steps, None, mu, None, g_t, terminal=True)
    seg_starts = sorted(s for s in fw["ckpt"] if s < n_steps)
    # each segment is recomputed from its checkpoint by one replayed call that
    # records the states before every step (slot n mod ck)
    theta = torch.empty_like(fw["ckpt"][0])
    hist = torch.empty((ck,) + tuple(theta.shape), dtype=theta.dtype, device=dev)
    rec = lt.make_step_args(mode, dt, fw["a_t"], fw["a_mid"], theta, n_steps, theta_hist=hist, **pot)
    slots = [lt.make_step_args(mode, dt, fw["a_t"], fw["a_mid"], hist[i], n_steps, **pot) for i in range(ck)]
    for s0 in reversed(seg_starts):
        s1 = min(s0 + ck, n_steps)
        theta.copy_(fw["ckpt"][s0])
        rec["step"].fill_(s0)
        lt.run(rec, s1 - s0) if s1 - s0 > 1 else lt.step(rec)
        for n in range(s1 - 1, s0 - 1, -1):
            lt.adjoint_step(slots[n % ck], n, n_steps, mu, mu, g_mid, g_t)
    return lt.knot_gradient(g_t, g_mid, dt, q.numel(), t_end), g_t, g_mid


class PulseLoss:
    """torch.autograd.Function: L(q) = delta mu_z(T)/Omega for knot amplitudes q."""

    @staticmethod
    def apply(lt, q, mode, dt, t_end, n_steps, theta0, checkpoint=50, potential=None):
        torch = _torch()

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, qq):
                loss, fw = pulse_forward(lt, mode, dt, qq.detach(), t_end, n_steps, theta0, checkpoint, potential)
                ctx.fw = fw
                ctx.save_for_backward(qq.detach())
                return loss

            @staticmethod
            def backward(ctx, g):
                (qq,) = ctx.saved_tensors
                grad, _, _ = pulse_backward(lt, mode, dt, qq, t_end, n_steps, ctx.fw)
                return g * grad

        return _F.apply(q)
