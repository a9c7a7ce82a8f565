"""Pins for the oracle's LAPW+LO operators (CPU only).

The oracle's three apply routes (dense assembly, FFT, MM) are checked against a
brute-force construction written here from first principles:

* the step-function and potential transforms by direct summation of
  exponentials over every grid point (no FFT library);
* the interstitial velocity-gauge Hamiltonian from the completed square
  1/2 (G+k+A/c z).(G'+k+A/c z) Theta~(g-g') + (Theta V)~(g-g') (Eq. (2) in the
  plane-wave basis), a different formula from the oracle's T + (A/c)P +
  (A^2/2c^2)S split, so a sign or factor slip in either shows up;
* the muffin-tin part by explicit index loops over channels and basis
  functions (Eq. (19); App. A, Eqs. (A.4)-(A.6)).
"""

import numpy as np
import pytest
from hypothesis import HealthCheck, given, reject, settings
from hypothesis import strategies as st

from oracle import operators as op
from synth import make_system


def brute_transform(field, q, grid):
    """(1/N) sum_j f_j exp(-2 pi i q.j/N), one q at a time, direct summation."""
    n1, n2, n3 = grid
    j3, j2, j1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    ph = np.exp(-2j * np.pi * (q[0] * j1 / n1 + q[1] * j2 / n2 + q[2] * j3 / n3))
    return np.sum(field * ph) / (n1 * n2 * n3)


def brute_operators(sys, ik, a_z):
    """Dense H(A) and S from first principles (see module docstring)."""
    kp = sys.kpts[ik]
    ng = kp.n_g
    nb = sys.n_basis(ik)
    g = kp.g_int
    gk = kp.gk
    a = np.array([0.0, 0.0, a_z / sys.c_light])
    h = np.zeros((nb, nb), dtype=complex)
    s = np.zeros((nb, nb), dtype=complex)
    cache = {}
    for i in range(ng):
        for j in range(ng):
            q = tuple(int(x) for x in (g[i] - g[j]))
            if q not in cache:
                cache[q] = (brute_transform(sys.theta, q, sys.grid),
                            brute_transform(sys.theta * sys.vr, q, sys.grid))
            th, thv = cache[q]
            s[i, j] = th
            h[i, j] = 0.5 * np.dot(gk[i] + a, gk[j] + a) * th + thv
    # muffin-tin: explicit loops over (channel r, channel s) of each atom
    a_off, l_off = sys.mt_offsets()
    cl = sys.c_light
    for alpha, at in enumerate(sys.atoms):
        m = at.n_mt
        blk_h = sys.h[alpha] + (a_z / cl) * sys.pz[alpha] + (a_z ** 2 / (2 * cl * cl)) * sys.o[alpha]
        blk_s = sys.o[alpha]

        def coeff(r, nu):
            # value of local channel r of atom alpha in basis function nu
            if r < m:
                return kp.A[a_off[alpha] + r, nu] if nu < ng else 0.0
            return 1.0 if nu == ng + l_off[alpha] + (r - m) else 0.0

        emb = np.array([[coeff(r, nu) for nu in range(nb)] for r in range(at.size)], dtype=complex)
        for nu in range(nb):
            for nu2 in range(nb):
                acc_h = 0.0
                acc_s = 0.0
                for r in range(at.size):
                    cr = np.conj(emb[r, nu])
                    if cr == 0:
                        continue
                    for t in range(at.size):
                        acc_h += cr * blk_h[r, t] * emb[t, nu2]
                        acc_s += cr * blk_s[r, t] * emb[t, nu2]
                h[nu, nu2] += acc_h
                s[nu, nu2] += acc_s
    return h, s


def tiny_system(seed=3, grid=(9, 10, 12), n_g=15, kgrid=(2, 1, 1)):
    atoms = [dict(pos=(1.2, 2.0, 3.1), rmt=0.8, lmax=1, n_rad=1, n_lo=2),
             dict(pos=(3.3, 4.1, 4.6), rmt=0.7, lmax=0, n_rad=2, n_lo=1)]
    return make_system(0, seed=seed, cell=(5.0, 6.0, 7.0), grid=grid, n_g=n_g,
                       atoms=("explicit", atoms), kgrid=kgrid, n_aux=4, n_states=2)


@pytest.fixture(scope="module")
def tiny():
    return tiny_system()


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("a_z", [0.0, 0.37, -1.3])
def test_dense_assembly_matches_brute_force(tiny, a_z):
    ik = 1  # k != 0
    h_ref, s_ref = brute_operators(tiny, ik, a_z)
    d = op.dense_operators(tiny, ik)
    assert rel(op.hamiltonian(d, a_z, tiny.c_light), h_ref) < 1e-13
    assert rel(d["S"], s_ref) < 1e-13


@pytest.mark.parametrize("route", ["fft", "mm"])
def test_matrix_free_routes_match_brute_force(tiny, route):
    ik = 1
    a_z = 0.81
    h_ref, s_ref = brute_operators(tiny, ik, a_z)
    rng = np.random.default_rng(0)
    c = rng.standard_normal((tiny.n_basis(ik), 3)) + 1j * rng.standard_normal((tiny.n_basis(ik), 3))
    hc, sc = op.apply_hs(tiny, ik, c, a_z, route=route)
    assert rel(hc, h_ref @ c) < 1e-13
    assert rel(sc, s_ref @ c) < 1e-13


def test_operators_hermitian_and_overlap_positive(tiny):
    for ik in range(len(tiny.kpts)):
        d = op.dense_operators(tiny, ik)
        for k in ("T", "V", "P", "S", "H0"):
            assert np.abs(d[k] - d[k].conj().T).max() < 1e-14
        # x^H S x > 0 for random x
        rng = np.random.default_rng(ik)
        for _ in range(20):
            x = rng.standard_normal(d["S"].shape[0]) + 1j * rng.standard_normal(d["S"].shape[0])
            assert np.real(x.conj() @ d["S"] @ x) > 0


def test_fft_route_equals_mm_route_on_tiny_config():
    sys = make_system(0)
    rng = np.random.default_rng(5)
    nb = sys.n_basis(0)
    c = rng.standard_normal((nb, 6)) + 1j * rng.standard_normal((nb, 6))
    d = op.dense_operators(sys, 0)
    f = op.apply_ops(sys, 0, c, "fft")
    m = op.apply_ops(sys, 0, c, "mm")
    for k in ("T", "V", "P", "S"):
        assert rel(f[k], d[k] @ c) < 1e-13
        assert rel(m[k], d[k] @ c) < 1e-13


def test_affine_identity():
    """H(A) C = H0 C + (A/c) P C + (A^2/2c^2) S C for several A (Eq. (15))."""
    sys = make_system(0)
    rng = np.random.default_rng(6)
    nb = sys.n_basis(0)
    c = rng.standard_normal((nb, 2)) + 1j * rng.standard_normal((nb, 2))
    h0, _ = op.apply_hs(sys, 0, c, 0.0)
    h1, s1 = op.apply_hs(sys, 0, c, 1.0)
    hm, _ = op.apply_hs(sys, 0, c, -1.0)
    cl = sys.c_light
    # even part gives the overlap term, odd part the momentum term
    assert rel((h1 + hm) / 2 - h0, s1 / (2 * cl * cl)) < 1e-9
    o = op.apply_ops(sys, 0, c)
    assert rel((h1 - hm) / 2, o["P"] / cl) < 1e-12


def test_step_function_and_grid_transform_conventions():
    """Theta~(0) is the interstitial volume fraction; the inverse transform has
    no 1/N so that dft(idft(c)) = c."""
    sys = make_system(0)
    th = op.dft(sys.theta)
    assert abs(th[0, 0, 0].real - sys.theta.mean()) < 1e-15
    rng = np.random.default_rng(0)
    c = rng.standard_normal(sys.theta.shape) + 1j * rng.standard_normal(sys.theta.shape)
    assert rel(op.dft(op.idft(c)), c) < 1e-14
    # a single plane wave of unit coefficient is exp(i q.r) with modulus 1
    e = np.zeros(sys.theta.shape, dtype=complex)
    e[1, 2, 3] = 1.0
    assert np.allclose(np.abs(op.idft(e)), 1.0)


@settings(max_examples=12, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 10_000),
       grid=st.tuples(st.sampled_from([6, 8, 9, 10, 12, 15]), st.sampled_from([5, 8, 9, 10]),
                      st.sampled_from([6, 8, 12, 15])),
       n_g=st.integers(3, 14),
       kgrid=st.sampled_from([None, (2, 2, 1), (3, 1, 2)]),
       lmax=st.integers(0, 2), n_rad=st.integers(1, 2), n_lo=st.integers(0, 3),
       a_z=st.floats(-2.0, 2.0))
def test_random_tiny_systems_fft_route(seed, grid, n_g, kgrid, lmax, n_rad, n_lo, a_z):
    atoms = [dict(pos=(1.0, 1.5, 2.0), rmt=0.6, lmax=lmax, n_rad=n_rad, n_lo=n_lo)]
    try:
        sys = make_system(0, seed=seed, cell=(4.5, 5.5, 6.5), grid=grid, n_g=n_g,
                          atoms=("explicit", atoms), kgrid=kgrid, n_aux=2, n_states=1)
    except ValueError:
        reject()
    ik = len(sys.kpts) - 1
    h_ref, s_ref = brute_operators(sys, ik, a_z)
    rng = np.random.default_rng(seed)
    nb = sys.n_basis(ik)
    c = rng.standard_normal((nb, 2)) + 1j * rng.standard_normal((nb, 2))
    hc, sc = op.apply_hs(sys, ik, c, a_z, "fft")
    assert rel(hc, h_ref @ c) < 1e-12
    assert rel(sc, s_ref @ c) < 1e-12
