"""Seeded generators for the synthetic workloads of the short-range tree force.

The paper's own initial conditions (galaxy collision, LCDM with gas,
collapsing gas sphere; Croker, ngravs, Appendix A) are not available, so the
workloads below stand in for them: uniform boxes, and clustered boxes made of
Plummer spheres plus a uniform background. Species are assigned independently
of position, as the paper does when it redistributes collisionless particles
evenly over the extra types (Appendix A).

Force-factor tables are inputs of the method (the paper lets the user supply
real-space tables for every species pair, section 2): they are built here
from the Newtonian TreePM short-range factor (section 2.4.1) and, for the
modified laws, from that factor times a Yukawa modulation of the form of
Eq. (2).

Everything is deterministic given the seed (numpy PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.special import erfc

__all__ = [
    "Problem", "GRID_R", "GRID_R2", "largest_remainder", "exact_species",
    "uniform_positions", "uniform_lattice", "clustered_positions",
    "newtonian_treepm_factor", "yukawa_product_factor", "table_abscissae",
    "sample_table", "scaled_params", "random_laws", "uniform_4096", "clustered_yukawa_d3", "clustered_d6",
    "clustered_d6_scaled",
    "clustered_problem", "uniform_problem", "batch_box", "serve_request", "poisson_arrivals",
    "accumulator_problem", "yukawa_law", "exact_split_laws", "isolated_problem",
    "newtonian_lattice_correction", "periodic_tree_problem", "transition_problem",
]

GRID_R = "r"     # table samples uniform in r on [0, r_cut]
GRID_R2 = "r2"   # table samples uniform in r^2 on [0, r_cut^2]


@dataclasses.dataclass
class Problem:
    """One force evaluation: particles, laws and walk parameters.

    Positions are given either as float64 ``pos`` (shape (3, n), 0 <= x < box)
    or as 64-bit lattice coordinates ``lattice`` (shape (3, n), uint64, the
    point X * 2**-64 * box). Exactly one of the two is set.
    ``G[a, b]`` and ``tables[a, b]`` act on a sink of species a from a source
    of species b.
    """
    name: str
    n: int
    D: int
    box: float
    species: np.ndarray            # (n,) uint8
    mass: np.ndarray               # (n,) float64
    G: np.ndarray                  # (D, D) float64
    tables: np.ndarray             # (D, D, ntab) float64
    grid: str
    r_s: float
    r_cut: float
    eps: float
    theta: float
    leaf_size: int = 16
    group_size: int = 64
    pos: Optional[np.ndarray] = None       # (3, n) float64
    lattice: Optional[np.ndarray] = None   # (3, n) uint64
    seed: int = 0
    # accumulator laws (section 3.3): {"cored": species indices, "beta": beta}, or None
    accumulator: Optional[dict] = None
    # per-pair Plummer softening (D, D), row = sink species, or None for eps everywhere
    eps_ab: Optional[np.ndarray] = None
    # False: a non-periodic box (pairs interact by their plain separation, no images)
    periodic: bool = True
    # relative opening test: {"alpha": tolerance, "old_acc": (n,) previous |a|}, or None (geometric)
    relative: Optional[dict] = None
    # pure-tree periodic mode: (D, D, n+1, n+1, n+1, 3) lattice correction tables, or None
    lattice_corr: Optional[np.ndarray] = None
    # space-filling curve of the sort (section 2.4): "morton" or "hilbert" (Peano-Hilbert)
    key_order: str = "morton"

    @property
    def ntab(self) -> int:
        return int(self.tables.shape[-1])


# ----------------------------------------------------------------- species --
def largest_remainder(total: int, fractions) -> np.ndarray:
    """Integer counts summing to ``total`` in the given proportions."""
    f = np.asarray(fractions, dtype=np.float64)
    f = f / f.sum()
    raw = f * total
    base = np.floor(raw).astype(np.int64)
    rest = total - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rest]] += 1
    return base


def exact_species(n: int, fractions, rng: np.random.Generator) -> np.ndarray:
    """Species ids with exact counts, placed by a seeded random permutation."""
    counts = largest_remainder(n, fractions)
    s = np.repeat(np.arange(len(counts), dtype=np.uint8), counts)
    return s[rng.permutation(n)]


# --------------------------------------------------------------- positions --
def uniform_positions(n: int, box: float, rng: np.random.Generator) -> np.ndarray:
    x = rng.random((3, n)) * box
    x[x >= box] = 0.0
    return x


def uniform_lattice(n: int, rng: np.random.Generator) -> np.ndarray:
    """Raw uniform 64-bit lattice coordinates, shape (3, n)."""
    return rng.integers(0, np.iinfo(np.uint64).max, size=(3, n),
                        dtype=np.uint64, endpoint=True)


def _plummer_radii(m: int, a: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Plummer-sphere radii for scale radii ``a`` (length m), truncated at 10a."""
    r = np.empty(m)
    todo = np.arange(m)
    while todo.size:
        u = rng.random(todo.size)
        u = np.maximum(u, 1e-300)
        rr = a[todo] / np.sqrt(u ** (-2.0 / 3.0) - 1.0 + 1e-300)
        ok = rr <= 10.0 * a[todo]
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    return r


def clustered_positions(n: int, box: float, rng: np.random.Generator, *,
                        f_cl: float = 0.7, halos: int = 2000,
                        a_min: float = 0.002, a_max: float = 0.02,
                        slope: float = -1.9, w_max: float = 1e3) -> np.ndarray:
    """A fraction ``f_cl`` of the particles in Plummer spheres, the rest uniform.

    Halo centres are uniform; scale radii are log-uniform in [a_min, a_max]
    (units of the box); occupancy weights follow p(w) ~ w**slope on [1, w_max].
    """
    halos = max(1, int(halos))
    n_cl = int(round(f_cl * n))
    centres = rng.random((halos, 3)) * box
    a = np.exp(rng.uniform(math.log(a_min), math.log(a_max), halos)) * box
    u = rng.random(halos)
    e = 1.0 + slope
    w = (1.0 + u * (w_max ** e - 1.0)) ** (1.0 / e)
    occ = largest_remainder(n_cl, w) if n_cl > 0 else np.zeros(halos, np.int64)
    hid = np.repeat(np.arange(halos), occ)
    r = _plummer_radii(hid.size, a[hid], rng)
    d = rng.normal(size=(hid.size, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p_cl = centres[hid] + r[:, None] * d
    p_un = rng.random((n - n_cl, 3)) * box
    p = np.concatenate([p_cl, p_un], axis=0)
    p = np.mod(p, box)
    p[p >= box] = 0.0
    p = p[rng.permutation(n)]
    return np.ascontiguousarray(p.T)


# ------------------------------------------------------------------ tables --
def newtonian_treepm_factor(r, r_s: float):
    """Short-range modulation of the Newtonian force for a Gaussian split of
    scale r_s (section 2.4.1): erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2)."""
    r = np.asarray(r, dtype=np.float64)
    return erfc(r / (2.0 * r_s)) + r / (r_s * math.sqrt(math.pi)) * np.exp(-r * r / (4.0 * r_s * r_s))


def yukawa_product_factor(r, r_s: float, alpha: float, lam: float):
    """Newtonian short-range factor times the force modulation of a Yukawa
    correction of strength alpha and range lam (the Eq. (2) law with C = 1)."""
    r = np.asarray(r, dtype=np.float64)
    return newtonian_treepm_factor(r, r_s) * (1.0 + alpha * (1.0 + r / lam) * np.exp(-r / lam))


def table_abscissae(ntab: int, r_cut: float, grid: str) -> np.ndarray:
    """Radii of the table samples: uniform in r, or uniform in r^2."""
    k = np.arange(ntab, dtype=np.float64)
    if grid == GRID_R:
        return k * (r_cut / (ntab - 1))
    if grid == GRID_R2:
        return np.sqrt(k * (r_cut * r_cut / (ntab - 1)))
    raise ValueError(grid)


def sample_table(fn, ntab: int, r_cut: float, grid: str) -> np.ndarray:
    return np.asarray(fn(table_abscissae(ntab, r_cut, grid)), dtype=np.float64)


def scaled_params(n: int, box: float = 1.0):
    """r_s, r_cut, eps scaled from the 4096-particle setting by mean spacing."""
    s = (4096.0 / n) ** (1.0 / 3.0) * box
    r_s = 1.25 / 64.0 * s
    return r_s, 4.5 * r_s, s / 640.0


def random_laws(D: int, ntab: int, r_s: float, r_cut: float, grid: str,
                rng: np.random.Generator, lam_range=(0.003, 0.03), box: float = 1.0):
    """Random symmetric G in [-1, 2] and a random mix of Newtonian and
    Yukawa-product tables (one law per unordered species pair)."""
    G = np.zeros((D, D))
    tables = np.zeros((D, D, ntab))
    for a in range(D):
        for b in range(a, D):
            g = rng.uniform(-1.0, 2.0)
            if rng.random() < 0.5:
                t = sample_table(lambda r: newtonian_treepm_factor(r, r_s), ntab, r_cut, grid)
            else:
                lam = math.exp(rng.uniform(math.log(lam_range[0]), math.log(lam_range[1]))) * box
                alpha = rng.uniform(-0.5, 1.0)
                t = sample_table(lambda r: yukawa_product_factor(r, r_s, alpha, lam), ntab, r_cut, grid)
            G[a, b] = G[b, a] = g
            tables[a, b] = tables[b, a] = t
    return G, tables


# ----------------------------------------------------------------- configs --
def uniform_4096(seed: int = 1) -> Problem:
    """4096 uniform particles, two equal species, Newtonian short-range laws."""
    n, D, box = 4096, 2, 1.0
    rng = np.random.default_rng(seed)
    lat = uniform_lattice(n, rng)
    species = exact_species(n, [1, 1], rng)
    r_s = 1.25 / 64.0
    r_cut = 4.5 * r_s
    ntab = 1024
    t = sample_table(lambda r: newtonian_treepm_factor(r, r_s), ntab, r_cut, GRID_R)
    return Problem(name=f"uniform-4096-D2-seed{seed}", n=n, D=D, box=box,
                   species=species, mass=np.full(n, 1.0 / n), G=np.ones((D, D)),
                   tables=np.broadcast_to(t, (D, D, ntab)).copy(), grid=GRID_R,
                   r_s=r_s, r_cut=r_cut, eps=1.0 / (40.0 * 16.0), theta=0.5,
                   lattice=lat, seed=seed)


def clustered_yukawa_d3(seed: int = 2, n: int = 2 ** 21) -> Problem:
    """Clustered box, three species (50/30/20), Yukawa-modified laws and a
    repulsive self-interaction of the third species."""
    D, box = 3, 1.0
    rng = np.random.default_rng(seed)
    halos = max(1, int(round(2000 * n / 2 ** 21)))
    pos = clustered_positions(n, box, rng, f_cl=0.7, halos=halos)
    species = exact_species(n, [0.5, 0.3, 0.2], rng)
    r_s, r_cut, eps = scaled_params(n, box)
    ntab = 2048
    lam = 0.01
    alpha = np.array([[0, 0.5, 0], [0.5, 1, -0.3], [0, -0.3, 0]], dtype=np.float64)
    tables = np.zeros((D, D, ntab))
    for a in range(D):
        for b in range(D):
            tables[a, b] = sample_table(lambda r: yukawa_product_factor(r, r_s, alpha[a, b], lam),
                                        ntab, r_cut, GRID_R)
    G = np.ones((D, D))
    G[2, 2] = -1.0
    return Problem(name=f"clustered-{n}-D3-yukawa-seed{seed}", n=n, D=D, box=box,
                   species=species, mass=np.full(n, 1.0 / n), G=G, tables=tables,
                   grid=GRID_R, r_s=r_s, r_cut=r_cut, eps=eps, theta=0.5, pos=pos, seed=seed)


def clustered_problem(n: int, D: int, seed: int, *, f_cl: float = 0.7,
                      grid: str = GRID_R2, ntab: int = 2048, theta: float = 0.5,
                      halos: Optional[int] = None, leaf_size: int = 16,
                      group_size: int = 64, box: float = 1.0) -> Problem:
    """Clustered box with D equal species and random laws."""
    rng = np.random.default_rng(seed)
    if halos is None:
        halos = max(1, int(round(2000 * n / 2 ** 21)))
    pos = clustered_positions(n, box, rng, f_cl=f_cl, halos=halos)
    species = exact_species(n, np.ones(D), rng)
    r_s, r_cut, eps = scaled_params(n, box)
    G, tables = random_laws(D, ntab, r_s, r_cut, grid, rng, box=box)
    return Problem(name=f"clustered-{n}-D{D}-seed{seed}", n=n, D=D, box=box,
                   species=species, mass=np.full(n, 1.0 / n), G=G, tables=tables,
                   grid=grid, r_s=r_s, r_cut=r_cut, eps=eps, theta=theta,
                   leaf_size=leaf_size, group_size=group_size, pos=pos, seed=seed)


def clustered_d6(seed: int = 3, n: int = 2 ** 24, halos: Optional[int] = 2000) -> Problem:
    """Clustered box at scale: six species, random G and random mixed laws.
    By default the same generator as the 2^21 box, 2000 halos whatever n
    (at 2^24 each halo then holds eight times the particles); halos=None
    scales the halo count with n (2000 n / 2^21), keeping the halos' mean
    occupancy of the 2^21 box."""
    p = clustered_problem(n, 6, seed, grid=GRID_R2, ntab=2048, halos=halos)
    h = halos if halos is not None else max(1, int(round(2000 * n / 2 ** 21)))
    p.name = f"clustered-{n}-D6-H{h}-seed{seed}"
    return p


def clustered_d6_scaled(seed: int = 3, n: int = 2 ** 24) -> Problem:
    """The six-species box with the halo count scaled with n (16000 halos at
    2^24)."""
    return clustered_d6(seed, n, halos=None)


def uniform_problem(n: int, D: int, seed: int, *, grid: str = GRID_R,
                    ntab: int = 1024, theta: float = 0.5, leaf_size: int = 16,
                    group_size: int = 64, box: float = 1.0) -> Problem:
    rng = np.random.default_rng(seed)
    pos = uniform_positions(n, box, rng)
    species = exact_species(n, np.ones(D), rng)
    r_s, r_cut, eps = scaled_params(n, box)
    G, tables = random_laws(D, ntab, r_s, r_cut, grid, rng, box=box)
    return Problem(name=f"uniform-{n}-D{D}-seed{seed}", n=n, D=D, box=box,
                   species=species, mass=np.full(n, 1.0 / n), G=G, tables=tables,
                   grid=grid, r_s=r_s, r_cut=r_cut, eps=eps, theta=theta,
                   leaf_size=leaf_size, group_size=group_size, pos=pos, seed=seed)


def batch_box(k: int) -> Problem:
    """Box k of the many-box workload: N log-uniform in [2^12, 2^18], D in
    {1..4}, clustered fraction in [0, 0.8], its own laws."""
    rng = np.random.default_rng(4000 + k)
    n = int(round(2.0 ** rng.uniform(12, 18)))
    D = int(rng.integers(1, 5))
    f_cl = float(rng.uniform(0.0, 0.8))
    return clustered_problem(n, D, 4000 + k, f_cl=f_cl, grid=GRID_R2, ntab=2048)


def serve_request(r: int) -> Problem:
    """Request r of the served workload: a new box with N log-uniform in
    [2^14, 2^20], D in {1..6}, clustered fraction in [0, 0.8] and laws of its
    own (the many-box recipe at larger N)."""
    rng = np.random.default_rng(5000 + r)
    n = int(round(2.0 ** rng.uniform(14, 20)))
    D = int(rng.integers(1, 7))
    f_cl = float(rng.uniform(0.0, 0.8))
    return clustered_problem(n, D, 5000 + r, f_cl=f_cl, grid=GRID_R2, ntab=2048)


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def accumulator_problem(n: int, seed: int, *, D: int = 2, cored=(1,), core_frac: float = 0.25,
                        f_cl: float = 0.7, grid: str = GRID_R2, ntab: int = 2048, theta: float = 0.5,
                        leaf_size: int = 16, group_size: int = 64, box: float = 1.0) -> Problem:
    """The two-species setting of the accumulator test (section 3.3, Fig. 6)
    on the short-range path: clustered box, equal species fractions, unit
    masses 1/n, G = 1 and the Newtonian short-range factor for every pair,
    the species in `cored` cored. beta makes the core radius of one body,
    m / (4 pi beta), core_frac of the mean spacing (the paper's beta is in
    the units of its own runs)."""
    rng = np.random.default_rng(seed)
    halos = max(1, int(round(2000 * n / 2 ** 21)))
    pos = clustered_positions(n, box, rng, f_cl=f_cl, halos=halos)
    species = exact_species(n, np.ones(D), rng)
    r_s, r_cut, eps = scaled_params(n, box)
    t = sample_table(lambda r: newtonian_treepm_factor(r, r_s), ntab, r_cut, grid)
    tables = np.broadcast_to(t, (D, D, ntab)).copy()
    m = 1.0 / n
    beta = m / (4.0 * math.pi * core_frac * box / n ** (1.0 / 3.0))
    return Problem(name=f"accumulator-{n}-D{D}-seed{seed}", n=n, D=D, box=box, species=species,
                   mass=np.full(n, m), G=np.ones((D, D)), tables=tables, grid=grid, r_s=r_s, r_cut=r_cut,
                   eps=eps, theta=theta, leaf_size=leaf_size, group_size=group_size, pos=pos, seed=seed,
                   accumulator={"cored": [int(b) for b in cored], "beta": float(beta)})


def yukawa_law(alpha: float, lam: float):
    """The pair law -(1 + alpha exp(-r/lam)) / r per unit masses (alpha = 0:
    Newton) as the inputs of the exact short-range tables: (phibar(k) =
    k^2 phi(k), f_full(r) = r^2 dphi/dr, decay length). Vectorised."""
    if alpha == 0.0:
        return (lambda k: np.full(np.shape(k), -4.0 * math.pi) if np.ndim(k) else -4.0 * math.pi,
                lambda r: np.ones(np.shape(r)) if np.ndim(r) else 1.0, 0.0)
    mu2 = 1.0 / (lam * lam)
    return (lambda k: -4.0 * math.pi * (1.0 + alpha * k * k / (k * k + mu2)),
            lambda r: 1.0 + alpha * (1.0 + r / lam) * np.exp(-r / lam), lam)


def exact_split_laws(D: int, seed: int, lam_range=(0.003, 0.03), box: float = 1.0):
    """D x D laws (symmetric): Newton with probability 1/2, else Yukawa with
    lam log-uniform in lam_range and alpha uniform in [-0.5, 1]."""
    rng = np.random.default_rng(seed)
    laws = [[None] * D for _ in range(D)]
    for a in range(D):
        for b in range(a, D):
            if rng.random() < 0.5:
                law = yukawa_law(0.0, 1.0)
            else:
                lam = math.exp(rng.uniform(math.log(lam_range[0]), math.log(lam_range[1]))) * box
                law = yukawa_law(float(rng.uniform(-0.5, 1.0)), lam)
            laws[a][b] = laws[b][a] = law
    return laws


def isolated_problem(n: int, D: int, seed: int, *, grid: str = GRID_R2, ntab: int = 2048, theta: float = 0.5,
                     leaf_size: int = 16, group_size: int = 64, box: float = 1.0) -> Problem:
    """A non-periodic box standing in for the paper's isolated runs (the
    galaxy collision of Appendix A): two Plummer spheres of scale 0.05 box,
    centred a third of the box apart, 90% of the particles, the rest uniform;
    D equal species; full laws (no short-range split): Newton with
    probability 1/2, else the Yukawa modulation 1 + alpha (1 + r/lam)
    exp(-r/lam), random G in [0.5, 2]; r_cut = 1.75 box keeps every pair
    (sqrt(3) box is the largest separation)."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(0.9 * n))
    half = n_cl // 2
    centres = np.array([[0.35, 0.4, 0.45], [0.68, 0.6, 0.52]]) * box
    hid = np.concatenate([np.zeros(half, np.int64), np.ones(n_cl - half, np.int64)])
    r = _plummer_radii(hid.size, np.full(hid.size, 0.05 * box), rng)
    d = rng.normal(size=(hid.size, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = np.concatenate([centres[hid] + r[:, None] * d, rng.random((n - n_cl, 3)) * box], axis=0)
    p = np.clip(p, 0.0, np.nextafter(box, 0.0))         # an isolated box has no wrap: keep the few far ones inside
    p = p[rng.permutation(n)]
    species = exact_species(n, np.ones(D), rng)
    r_cut = 1.75 * box
    eps = box / n ** (1.0 / 3.0) / 40.0
    G = np.zeros((D, D))
    tables = np.zeros((D, D, ntab))
    for a in range(D):
        for b in range(a, D):
            G[a, b] = G[b, a] = rng.uniform(0.5, 2.0)
            if rng.random() < 0.5:
                t = np.ones(ntab)
            else:
                lam = math.exp(rng.uniform(math.log(0.01), math.log(0.3))) * box
                alpha = rng.uniform(-0.5, 1.0)
                t = sample_table(lambda x: 1.0 + alpha * (1.0 + x / lam) * np.exp(-x / lam), ntab, r_cut, grid)
            tables[a, b] = tables[b, a] = t
    return Problem(name=f"isolated-{n}-D{D}-seed{seed}", n=n, D=D, box=box, species=species,
                   mass=np.full(n, 1.0 / n), G=G, tables=tables, grid=grid, r_s=0.0, r_cut=r_cut, eps=eps,
                   theta=theta, leaf_size=leaf_size, group_size=group_size, pos=np.ascontiguousarray(p.T), seed=seed,
                   periodic=False)


def newtonian_lattice_correction(EN: int, box: float = 1.0, alpha: float = 2.0, nreal: int = 4,
                                 kmax: int = 6) -> np.ndarray:
    """The lattice correction of Newton's law in a periodic box (section 2.3:
    the tables that correct the nearest-image force for every other image),
    on (EN + 1)^3 points d in [0, box/2]^3, shape (EN + 1, EN + 1, EN + 1, 3):
    the acceleration of a sink whose unit-mass source sits at offset d from
    it (source - sink), summed over all periodic images with a neutralising
    background by Ewald summation (splitting parameter alpha / box, real-space
    images |n_i| <= nreal, wave vectors |m_i| <= kmax), minus the nearest
    image's d / |d|^3. Zero at d = 0."""
    L = float(box)
    a = alpha / L
    g = np.linspace(0.0, L / 2, EN + 1)
    D = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1)       # (EN+1)^3 x 3
    x = -D                                                             # sink - source
    F = np.zeros_like(D)
    rng_ = range(-nreal, nreal + 1)
    for i in rng_:
        for j in rng_:
            for k in rng_:
                r = x - L * np.array([i, j, k])
                rr = np.linalg.norm(r, axis=-1)
                with np.errstate(divide="ignore", invalid="ignore"):
                    fac = (erfc(a * rr) + 2 * a * rr / math.sqrt(math.pi) * np.exp(-a * a * rr * rr)) / rr ** 3
                fac = np.where(rr > 0, fac, 0.0)
                F -= fac[..., None] * r
    mr = range(-kmax, kmax + 1)
    for i in mr:
        for j in mr:
            for k in mr:
                if i == 0 and j == 0 and k == 0:
                    continue
                kv = 2 * math.pi / L * np.array([i, j, k], dtype=np.float64)
                k2 = float(kv @ kv)
                amp = 4 * math.pi / L ** 3 * math.exp(-k2 / (4 * a * a)) / k2
                F -= amp * np.sin(x @ kv)[..., None] * kv
    rr = np.linalg.norm(D, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        near = np.where(rr[..., None] > 0, D / rr[..., None] ** 3, 0.0)
    out = F - near
    out[0, 0, 0] = 0.0
    return out


def periodic_tree_problem(n: int, D: int, seed: int, *, EN: int = 32, ntab: int = 2048, theta: float = 0.5,
                          leaf_size: int = 16, group_size: int = 64, box: float = 1.0) -> Problem:
    """Pure-tree periodic mode with lattice corrections (section 2.3): a
    clustered box, D species in equal shares, Newton for every pair with
    random G in [0.5, 2] (the same correction table for every pair), tables
    of ones on the r^2 grid out to r_cut = 0.9 box (past the farthest
    nearest image, sqrt(3)/2 box), eps of 1/40 the mean spacing."""
    rng = np.random.default_rng(seed)
    pos = clustered_positions(n, box, rng, f_cl=0.6, halos=max(1, n // 400))
    species = exact_species(n, np.ones(D), rng)
    G = rng.uniform(0.5, 2.0, (D, D))
    G = 0.5 * (G + G.T)
    T = newtonian_lattice_correction(EN, box)
    corr = np.broadcast_to(T, (D, D) + T.shape).copy()
    return Problem(name=f"periodic-tree-{n}-D{D}-seed{seed}", n=n, D=D, box=box, species=species,
                   mass=np.full(n, 1.0 / n), G=G, tables=np.ones((D, D, ntab)), grid=GRID_R2, r_s=0.0,
                   r_cut=0.9 * box, eps=box / n ** (1.0 / 3.0) / 40.0, theta=theta, leaf_size=leaf_size,
                   group_size=group_size, pos=pos, seed=seed, lattice_corr=corr)


def transition_problem(seed: int, *, shells: int = 20, per_shell: int = 5000, r_min: float = 1e-3,
                       r_max: float = 0.5, mesh: int = 64, ntab: int = 2048, box: float = 1.0) -> Problem:
    """The transition test of section 3.1: one massive source at a random
    place (species 0, mass 1) and `shells` spherical shells of `per_shell`
    massless test particles (species 1) around it, the shells equal in log r
    between r_min and r_max (so the density falls as 1 / r^3 and every shell
    holds the same number), random directions. Only the test particles feel
    the source (G_10 = 1, every other G_ab = 0: intra-type interactions off);
    Newtonian short-range tables for a mesh of `mesh` points (r_s = 1.25
    cells, r_cut = 4.5 r_s), no softening."""
    rng = np.random.default_rng(seed)
    src = rng.random(3) * box
    edges = np.exp(np.linspace(math.log(r_min), math.log(r_max), shells + 1)) * box
    r = np.concatenate([np.exp(rng.uniform(math.log(edges[k]), math.log(edges[k + 1]), per_shell))
                        for k in range(shells)])
    u = rng.normal(size=(r.size, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    pos = np.mod(np.vstack([src[None, :], src[None, :] + r[:, None] * u]), box)
    pos[pos >= box] = 0.0
    n = pos.shape[0]
    species = np.ones(n, np.uint8)
    species[0] = 0
    mass = np.zeros(n)
    mass[0] = 1.0
    G = np.zeros((2, 2))
    G[1, 0] = 1.0
    r_s = 1.25 * box / mesh
    r_cut = 4.5 * r_s
    t = sample_table(lambda x: newtonian_treepm_factor(x, r_s), ntab, r_cut, GRID_R2)
    return Problem(name=f"transition-seed{seed}", n=n, D=2, box=box, species=species, mass=mass, G=G,
                   tables=np.broadcast_to(t, (2, 2, ntab)).copy(), grid=GRID_R2, r_s=r_s, r_cut=r_cut, eps=0.0,
                   theta=0.5, pos=np.ascontiguousarray(pos.T), seed=seed)
