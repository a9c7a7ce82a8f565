"""Seeded synthetic inputs with the shapes of the LAPW+LO workloads.

What is drawn, and in which order (one ``numpy.random.default_rng`` stream per
system, seed ``240304351 + cfg`` unless overridden):

1. geometry: atom positions (random only for the heterostructure and the
   batched-k systems; fixed diatomic otherwise);
2. well depths v_alpha ~ U[1, 2] Ha, one per atom;
3. the plane-wave count N_G(k) per k-point (uniform integers for the batched
   system, fixed otherwise);
4. per atom: the random Hermitian blocks h, o, p_z (in that order);
5. per k-point: the matching coefficients A_k ~ CN(0,1)/sqrt(N_G);
6. per k-point: the start block X_k used to build the auxiliary basis;
7. (only if asked for) the time-dependent potential perturbation.

Conventions that both the oracle and the GPU path rely on:

* Real-space grids are numpy arrays of shape (N3, N2, N1): x is the fastest
  index, linear index j = j1 + N1*(j2 + N2*j3), position r_j = (j_i/N_i) L_i.
* A G-vector is an integer triple g = (g1, g2, g3) with G = (2*pi/L_i) g_i; its
  grid index is g mod (N1, N2, N3).
* A basis vector is ordered [plane-wave block (N_G rows); local orbitals of
  atom 0; local orbitals of atom 1; ...].
* The matching coefficients of one k-point form an N_A x N_G matrix whose rows
  are the muffin-tin channels of atom 0, then atom 1, ... (m_alpha rows each,
  m_alpha = n_rad*(lmax+1)^2, channel index (l^2+l+m)*n_rad + rho).
* Muffin-tin blocks are (m_alpha + l_alpha) square Hermitian matrices over
  [muffin-tin channels; local orbitals] of one atom.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# Speed of light in atomic units (CODATA 2018).
C_LIGHT = 137.035999084

_SEED_BASE = 240304351


@dataclasses.dataclass
class Atom:
    pos: np.ndarray      # Cartesian position (bohr), shape (3,)
    rmt: float           # muffin-tin radius (bohr)
    lmax: int
    n_rad: int
    n_lo: int
    v_depth: float       # depth of the Gaussian well (Ha)

    @property
    def n_mt(self) -> int:
        return self.n_rad * (self.lmax + 1) ** 2

    @property
    def size(self) -> int:
        return self.n_mt + self.n_lo


@dataclasses.dataclass
class KPoint:
    k_cart: np.ndarray     # (3,) Cartesian k (bohr^-1)
    weight: float
    g_int: np.ndarray      # (N_G, 3) int32
    gk: np.ndarray         # (N_G, 3) float64, Cartesian G+k
    A: np.ndarray          # (N_A, N_G) complex128 matching coefficients
    start: np.ndarray      # (N_basis, n_aux) complex128 start block

    @property
    def n_g(self) -> int:
        return self.g_int.shape[0]


@dataclasses.dataclass
class System:
    cfg: int
    cell: np.ndarray       # (3,) orthorhombic cell lengths (bohr)
    grid: tuple            # (N1, N2, N3)
    atoms: List[Atom]
    kpts: List[KPoint]
    theta: np.ndarray      # (N3, N2, N1) step function, 1 interstitial / 0 in spheres
    vr: np.ndarray         # (N3, N2, N1) potential on the grid (Ha)
    h: List[np.ndarray]    # per atom, (size, size) complex128
    o: List[np.ndarray]
    pz: List[np.ndarray]
    n_aux: int
    n_states: int
    dt: float
    n_steps: int
    pulse: dict
    occ: float = 2.0
    c_light: float = C_LIGHT

    @property
    def omega(self) -> float:
        return float(np.prod(self.cell))

    @property
    def n_atoms(self) -> int:
        return len(self.atoms)

    @property
    def n_a(self) -> int:
        return sum(a.n_mt for a in self.atoms)

    @property
    def n_lo(self) -> int:
        return sum(a.n_lo for a in self.atoms)

    def n_basis(self, ik: int = 0) -> int:
        return self.kpts[ik].n_g + self.n_lo

    @property
    def n_grid(self) -> int:
        return int(np.prod(self.grid))

    def mt_offsets(self):
        """Row offset of each atom's channels in A, and of its LOs in the LO block."""
        a_off, l_off = [], []
        a = l = 0
        for at in self.atoms:
            a_off.append(a)
            l_off.append(l)
            a += at.n_mt
            l += at.n_lo
        return a_off, l_off


# ---------------------------------------------------------------------------
# Configuration table: the five workloads (sizes as stated for each).
# ---------------------------------------------------------------------------

def _diatomic(cell, lmax, n_lo, rmt=1.0, bond=2.13):
    c = np.asarray(cell, float) / 2.0
    d = np.array([bond / 2.0, 0.0, 0.0])
    return [dict(pos=c - d, rmt=rmt, lmax=lmax, n_lo=n_lo),
            dict(pos=c + d, rmt=rmt, lmax=lmax, n_lo=n_lo)]


WORKLOADS = {
    # Tiny plain FP64 reference.
    0: dict(cell=(10.0, 10.0, 10.0), grid=(16, 16, 16), n_g=200,
            atoms=("diatomic", 3, 4), kgrid=None, n_aux=16, n_states=4,
            dt=0.1, n_steps=100,
            pulse=dict(kind="gauss_sin", amp=0.01, omega=0.3, t0=5.0, width=2.0)),
    # Molecule in a large cell.
    1: dict(cell=(20.0, 20.0, 20.0), grid=(72, 72, 72), n_g=12000,
            atoms=("diatomic", 8, 10), kgrid=None, n_aux=64, n_states=5,
            dt=0.2, n_steps=1000,
            pulse=dict(kind="gauss_sin", amp=0.005, omega=0.2, t0=5.0, width=2.0)),
    # Heterostructure-scale cell: 6 heavy (lmax 8) + 20 light (lmax 6) atoms.
    2: dict(cell=(17.92, 17.92, 27.80), grid=(96, 96, 160), n_g=30000,
            atoms=("random", [(6, 8, 1.1), (20, 6, 0.9)], 8, 2.4), kgrid=None,
            n_aux=300, n_states=60, dt=0.2, n_steps=500,
            pulse=dict(kind="gauss_sin", amp=0.005, omega=0.2, t0=5.0, width=2.0)),
    # Batched k-points: 4x4x1 Monkhorst-Pack set, ragged N_G per k.
    3: dict(cell=(15.0, 15.0, 15.0), grid=(64, 64, 64), n_g=(8000, 9500),
            atoms=("random", [(3, 7, 1.0)], 6, 2.4), kgrid=(4, 4, 1),
            n_aux=80, n_states=20, dt=0.2, n_steps=500,
            pulse=dict(kind="gauss_sin", amp=0.005, omega=0.2, t0=5.0, width=2.0)),
    # Pulse-gradient workload: the molecule system, 64 piecewise-linear knots.
    4: dict(cell=(20.0, 20.0, 20.0), grid=(72, 72, 72), n_g=12000,
            atoms=("diatomic", 8, 10), kgrid=None, n_aux=64, n_states=5,
            dt=0.1, n_steps=2000,
            pulse=dict(kind="knots", n_knots=64, base=dict(
                kind="gauss_sin", amp=0.005, omega=0.2, t0=5.0, width=2.0))),
}


def _cn(rng, shape):
    """Circular complex normal CN(0,1): (x + i y)/sqrt(2), x, y ~ N(0,1)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def _random_hermitian(rng, s):
    """W = (X + X^H) / (2 sqrt(2 s)), X_ij ~ CN(0,1): spectral radius close to 1."""
    x = _cn(rng, (s, s))
    return (x + x.conj().T) / (2.0 * np.sqrt(2.0 * s))


def _min_image_dist(p, q, cell):
    d = p - q
    d -= cell * np.round(d / cell)
    return float(np.sqrt(np.dot(d, d)))


def _random_atoms(rng, cell, groups, n_lo, dmin):
    specs = []
    for count, lmax, rmt in groups:
        specs += [(lmax, rmt)] * count
    out = []
    tries = 0
    while len(out) < len(specs):
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms")
        p = rng.random(3) * cell
        if all(_min_image_dist(p, a["pos"], cell) >= dmin for a in out):
            lmax, rmt = specs[len(out)]
            out.append(dict(pos=p, rmt=rmt, lmax=lmax, n_lo=n_lo))
    return out


def _gk_set(cell, k_cart, n_g, grid):
    """The n_g smallest |G+k|^2, ties broken lexicographically by (g1, g2, g3).

    |G+k|^2 is rounded to 1e-9 bohr^-2 before sorting so that shells that are
    degenerate by symmetry tie exactly whatever the summation order.
    """
    b = 2.0 * np.pi / np.asarray(cell, float)
    gmax = np.sqrt(n_g * 6.0 * np.pi ** 2 / np.prod(cell)) * 1.3 + np.abs(k_cart).max() + 2 * b.max()
    r = np.ceil(gmax / b).astype(int)
    axes = [np.arange(-r[i], r[i] + 1) for i in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    gk = g * b + k_cart
    key = np.round((gk * gk).sum(1) * 1e9).astype(np.int64)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], key))
    sel = order[:n_g]
    if len(order) > n_g and key[order[n_g - 1]] == key[order[n_g]]:
        pass  # a shell is split; the lexicographic tie-break decides
    g = g[sel].astype(np.int32)
    gk = g * b + k_cart
    n = np.asarray(grid)
    if np.any(2 * np.abs(g).max(0) >= n):
        raise ValueError("G set does not map injectively into the FFT grid")
    return g, gk


def _grid_points(cell, grid):
    n1, n2, n3 = grid
    x = np.arange(n1) / n1 * cell[0]
    y = np.arange(n2) / n2 * cell[1]
    z = np.arange(n3) / n3 * cell[2]
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return xx, yy, zz


def _theta_and_v(cell, grid, atoms, sigma=1.5):
    """Step function (0 strictly inside a sphere image) and the Gaussian-well potential."""
    xx, yy, zz = _grid_points(cell, grid)
    theta = np.ones(xx.shape)
    v = np.zeros(xx.shape)
    cell = np.asarray(cell, float)
    for at in atoms:
        for tx in (-1, 0, 1):
            for ty in (-1, 0, 1):
                for tz in (-1, 0, 1):
                    c = at.pos + cell * np.array([tx, ty, tz])
                    d2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
                    theta[d2 < at.rmt ** 2] = 0.0
                    v -= at.v_depth * np.exp(-d2 / (2.0 * sigma ** 2))
    return theta, v


def _mp_kpoints(cell, kgrid):
    b = 2.0 * np.pi / np.asarray(cell, float)
    pts = []
    q1, q2, q3 = kgrid
    for r1 in range(1, q1 + 1):
        for r2 in range(1, q2 + 1):
            for r3 in range(1, q3 + 1):
                u = np.array([(2 * r1 - q1 - 1) / (2 * q1), (2 * r2 - q2 - 1) / (2 * q2),
                              (2 * r3 - q3 - 1) / (2 * q3)])
                pts.append(u * b)
    return pts


def make_system(cfg: int, seed: Optional[int] = None, with_start: bool = True, **over) -> System:
    """Build the synthetic system of workload ``cfg`` (0..4).

    Keyword overrides (``cell``, ``grid``, ``n_g``, ``atoms``, ``kgrid``,
    ``n_aux``, ``n_states``, ``dt``, ``n_steps``, ``pulse``, ``n_k``) give
    scaled variants with the same recipe; ``n_k`` keeps only the first n_k
    k-points.
    """
    p = dict(WORKLOADS[cfg])
    n_k_keep = over.pop("n_k", None)
    p.update(over)
    rng = np.random.default_rng(_SEED_BASE + cfg if seed is None else seed)
    cell = np.asarray(p["cell"], float)
    grid = tuple(int(x) for x in p["grid"])

    # 1. geometry
    spec = p["atoms"]
    if spec[0] == "diatomic":
        raw = _diatomic(cell, spec[1], spec[2])
    elif spec[0] == "random":
        raw = _random_atoms(rng, cell, spec[1], spec[2], spec[3])
    elif spec[0] == "explicit":
        raw = [dict(a) for a in spec[1]]
    else:
        raise ValueError(spec[0])
    # 2. well depths
    atoms = []
    for a in raw:
        atoms.append(Atom(pos=np.asarray(a["pos"], float), rmt=float(a["rmt"]),
                          lmax=int(a["lmax"]), n_rad=int(a.get("n_rad", 2)),
                          n_lo=int(a["n_lo"]), v_depth=float(rng.uniform(1.0, 2.0))))
    # 3. k-points and N_G(k)
    if p["kgrid"] is None:
        kcart = [np.zeros(3)]
    else:
        kcart = _mp_kpoints(cell, p["kgrid"])
    if n_k_keep is not None:
        kcart = kcart[:n_k_keep]
    if isinstance(p["n_g"], tuple):
        lo, hi = p["n_g"]
        ngs = [int(x) for x in rng.integers(lo, hi + 1, size=len(kcart))]
    else:
        ngs = [int(p["n_g"])] * len(kcart)
    # 4. muffin-tin blocks
    h, o, pz = [], [], []
    for at in atoms:
        s = at.size
        h.append(_random_hermitian(rng, s))
        o.append(_random_hermitian(rng, s) + 2.0 * np.eye(s))
        pz.append(0.5 * _random_hermitian(rng, s))
    n_a = sum(a.n_mt for a in atoms)
    n_lo = sum(a.n_lo for a in atoms)
    # 5./6. per-k matching coefficients, then start blocks
    gsets = [_gk_set(cell, kc, ng, grid) for kc, ng in zip(kcart, ngs)]
    amats = [_cn(rng, (n_a, g.shape[0])) / np.sqrt(g.shape[0]) for g, _ in gsets]
    n_aux = int(p["n_aux"])
    starts = []
    for (g, gk) in gsets:
        if with_start:
            damp = 1.0 / (1.0 + 0.5 * (gk * gk).sum(1)) ** 2
            xg = _cn(rng, (g.shape[0], n_aux)) * damp[:, None]
            xl = 0.1 * _cn(rng, (n_lo, n_aux))
            starts.append(np.vstack([xg, xl]))
        else:
            starts.append(None)
    kpts = [KPoint(k_cart=np.asarray(kc), weight=1.0 / len(kcart), g_int=g, gk=gk, A=A, start=st)
            for kc, (g, gk), A, st in zip(kcart, gsets, amats, starts)]
    theta, vr = _theta_and_v(cell, grid, atoms)
    return System(cfg=cfg, cell=cell, grid=grid, atoms=atoms, kpts=kpts, theta=theta, vr=vr,
                  h=h, o=o, pz=pz, n_aux=n_aux, n_states=int(p["n_states"]), dt=float(p["dt"]),
                  n_steps=int(p["n_steps"]), pulse=dict(p["pulse"]))


# ---------------------------------------------------------------------------
# Pulses: the sampled vector potential is an input of the propagation.
# ---------------------------------------------------------------------------

def _gauss_sin(t, amp, omega, t0, width):
    t = np.asarray(t, float)
    return amp * np.sin(omega * t) * np.exp(-((t - t0) / width) ** 2)


def knot_times(n_knots, t_end):
    """Knots placed uniformly on [0, t_end], both ends included."""
    return np.linspace(0.0, t_end, n_knots)


def knot_values(pulse: dict, t_end: float) -> np.ndarray:
    base = pulse["base"]
    tau = knot_times(pulse["n_knots"], t_end)
    return _gauss_sin(tau, base["amp"], base["omega"], base["t0"], base["width"])


def pulse_samples(sys: System, n_steps: Optional[int] = None, knots: Optional[np.ndarray] = None):
    """A_z at t_n = n dt (n = 0..N) and at the midpoints t_n + dt/2 (n = 0..N-1).

    For a knot pulse the samples are the piecewise-linear interpolant of the
    knot values ``knots`` (default: the base pulse at the knots).
    """
    n = sys.n_steps if n_steps is None else n_steps
    t = np.arange(n + 1) * sys.dt
    tm = (np.arange(n) + 0.5) * sys.dt
    pl = sys.pulse
    if pl["kind"] == "gauss_sin":
        f = lambda x: _gauss_sin(x, pl["amp"], pl["omega"], pl["t0"], pl["width"])
        return f(t), f(tm)
    if pl["kind"] == "knots":
        t_end = sys.n_steps * sys.dt
        tau = knot_times(pl["n_knots"], t_end)
        q = knot_values(pl, t_end) if knots is None else np.asarray(knots, float)
        return np.interp(t, tau, q), np.interp(tm, tau, q)
    if pl["kind"] == "zero":
        return np.zeros(n + 1), np.zeros(n)
    raise ValueError(pl["kind"])


def hat_weights(times: np.ndarray, n_knots: int, t_end: float):
    """Piecewise-linear (hat) basis on uniform knots: for each time, the two
    knots it lies between and their weights (phi_k(t) for those two k)."""
    tau = knot_times(n_knots, t_end)
    h = tau[1] - tau[0]
    idx = np.clip(np.floor(times / h).astype(np.int64), 0, n_knots - 2)
    w1 = (times - tau[idx]) / h
    return idx.astype(np.int32), (1.0 - w1), (idx + 1).astype(np.int32), w1


def td_potential(sys: System, eps_v: float = 1e-2, seed: int = 7):
    """Perturbation fields for the time-dependent-potential study: a smooth
    real field W(r) on the grid (unit maximum) and one random Hermitian block
    per atom.  The potential at time t is V + eps_v*s(t)*W and h_alpha +
    eps_v*s(t)*w_alpha, with s(t) = A_z(t)/max|A_z| supplied by the caller."""
    rng = np.random.default_rng(seed)
    xx, yy, zz = _grid_points(sys.cell, sys.grid)
    w = np.zeros(xx.shape)
    for _ in range(4):
        c = rng.random(3) * sys.cell
        s = 1.0 + 2.0 * rng.random()
        d2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
        w += rng.uniform(-1.0, 1.0) * np.exp(-d2 / (2 * s * s))
    w /= np.abs(w).max()
    blocks = [_random_hermitian(rng, at.size) for at in sys.atoms]
    return eps_v, w, blocks


def potential_scale(n_total: int) -> np.ndarray:
    """s_n = sin(0.05 n), n = 0..n_total-1: the scale of the perturbation in the
    potential handed in for step n, V_n = V + eps_v s_n W and h_n = h + eps_v s_n w
    (the per-step potential series of the benchmark and its parity tests)."""
    return np.sin(0.05 * np.arange(n_total))
