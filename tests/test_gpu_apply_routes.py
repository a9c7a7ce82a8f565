"""The two FFT forms of the apply on the GPU against the oracle and each other.

The default FFT route takes box arrays through the rebuild's x/z and y kernels
where the apply grid has them (the molecule's 64^3 rebuild grid, the 72^3 grid
of N_G = 18000); LTD_ROUTE_FFT_PLANES keeps the whole-plane x-y passes and the z
lines on every grid.  Both are the convolution of Sec. 2.3 (second route) and
must agree with the oracle's matrix-free apply and with each other to rounding:
H(t) C and S C at ragged column counts and a nonzero A_z, the four blocks of the
projection mode (through the subspace matrices), and S alone (through one
conventional full-basis step, whose defining identity is checked).

Bar: 1e-10 relative (element maxima against the largest reference element).
"""

import numpy as np
import pytest

from oracle import operators as op
from oracle import subspace as ss
from synth import make_system

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_max(x, ref):
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())


@pytest.fixture(scope="module", params=[dict(), dict(n_g=18000, n_aux=24, n_states=4)], ids=["molecule", "72cubed"])
def routes(request):
    from paper_2403_04351_amd import _lib, ltd

    sys = make_system(1, **request.param)
    box = ltd.Ltd(sys, max_cols=64)
    planes = ltd.Ltd(sys, max_cols=64, route=_lib.LTD_ROUTE_FFT_PLANES)
    yield dict(sys=sys, box=box, planes=planes, ltd=ltd)
    box.close()
    planes.close()


@pytest.mark.parametrize("n", [1, 7, 40])
def test_apply_routes_match_oracle_and_each_other(routes, n):
    import torch

    sys, ltd = routes["sys"], routes["ltd"]
    rng = np.random.default_rng(90 + n)
    c = rng.standard_normal((sys.n_basis(0), n)) + 1j * rng.standard_normal((sys.n_basis(0), n))
    a_z = 0.0043
    out = {}
    for name in ("box", "planes"):
        lt = routes[name]
        hc, sc = lt.apply_hs(0, ltd.colmajor(c, lt.device), a_z)
        torch.cuda.synchronize()
        out[name] = (ltd.to_numpy(hc), ltd.to_numpy(sc))
    hr, sr = op.apply_hs(sys, 0, c, a_z)
    e = [rel_max(out["box"][0], hr), rel_max(out["box"][1], sr), rel_max(out["planes"][0], hr),
         rel_max(out["planes"][1], sr), rel_max(out["box"][0], out["planes"][0])]
    print(f"apply n={n}: box H {e[0]:.2e} S {e[1]:.2e}; planes H {e[2]:.2e} S {e[3]:.2e}; box-planes H {e[4]:.2e}",
          flush=True)
    assert max(e) < TOL


def test_projection_routes_agree(routes):
    import torch

    sys, ltd = routes["sys"], routes["ltd"]
    phi, _ = ss.ground_state(sys, 0)
    ref = ss.project(sys, 0, phi)
    for name in ("box", "planes"):
        lt = routes[name]
        h0, s, _ = lt.project_subspace(0, ltd.colmajor(phi, lt.device))
        torch.cuda.synchronize()
        eh, es = rel_max(ltd.to_numpy(h0), ref["H0"]), rel_max(ltd.to_numpy(s), ref["S"])
        print(f"projection ({name}): H0 {eh:.2e} S {es:.2e}", flush=True)
        assert eh < TOL and es < TOL


def test_s_apply_routes_full_step_identity(routes):
    import torch

    sys, ltd = routes["sys"], routes["ltd"]
    rng = np.random.default_rng(93)
    nb = sys.n_basis(0)
    c = rng.standard_normal((nb, 2)) + 1j * rng.standard_normal((nb, 2))
    dt, c0, a = 0.01, 1.5, 0.21
    hc, sc = op.apply_hs(sys, 0, c, a)
    rhs = -1j * dt * (hc - c0 * sc)
    for name in ("box", "planes"):
        lt = routes[name]
        cd = ltd.colmajor(c, lt.device)
        res, its = lt.propagate_full(0, cd, dt, 1, c0, [a], cg_max_iter=2000, cg_tol=1e-13)
        torch.cuda.synchronize()
        x = ltd.to_numpy(cd)
        _, sd = op.apply_hs(sys, 0, np.exp(1j * dt * c0) * x - c, 0.0)
        err = rel_max(sd, rhs)
        print(f"{name}: order-1 full step identity {err:.2e} (CG residual {res:.1e}, {its} iterations)", flush=True)
        assert res <= 1e-13 and err < TOL
