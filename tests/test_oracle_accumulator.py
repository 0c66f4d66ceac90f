"""Pins of the oracle's accumulator laws (section 3.3, Eqs. (13)-(17)): the
read density against its integral and Fourier transform, the force against
the derivative of the potential, the Newtonian limit, and the exactness of
the N_perp correction for monopoles of coincident bodies."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth


def density(r, M, beta, core):
    """Eq. (15) with core radius `core` (the paper prints M / (2 beta pi))."""
    return M ** 2 / (4 * beta * math.pi ** 3) / (core ** 2 + r ** 2) ** 2


@pytest.mark.parametrize("M,beta", [(1.0, 1.31e-6), (2.5e-4, 2e-3), (3.0, 0.7)])
def test_density_reading_integrates_to_M(M, beta):
    read = M / (4 * beta * math.pi)
    printed = M / (2 * beta * math.pi)
    # integrated in u = r / a so that quad sees a unit scale whatever the core
    total = lambda a: a * integrate.quad(lambda u: 4 * math.pi * (a * u) ** 2 * density(a * u, M, beta, a),
                                         0, np.inf, limit=500)[0]
    assert total(read) == pytest.approx(M, rel=1e-9)
    assert total(printed) == pytest.approx(M / 2, rel=1e-9)     # why the printed radius is not taken


@pytest.mark.parametrize("k", [0.1, 1.0, 3.0])
def test_density_transform_is_exponential(k):
    """The read density's Fourier transform is M exp(-a k): the mutual
    potential of two cores (Eq. (14)) then has the sum of their radii as
    scale, (M + m) / (4 pi beta)."""
    M, beta = 1.7, 0.05
    a = M / (4 * beta * math.pi)
    # Fourier-weighted quadrature (QAWF) for the oscillating tail
    ft = integrate.quad(lambda r: 4 * math.pi * r * density(r, M, beta, a) / k, 0, np.inf,
                        weight="sin", wvar=k)[0]
    assert ft == pytest.approx(M * math.exp(-a * k), rel=1e-7)
    # and exp(-c k) / k^2 transforms back to (2 / pi) atan(r / c) / r
    c, r = 0.3, 0.8
    back = (2 / math.pi) * integrate.quad(lambda q: math.exp(-c * q) / (q * r), 0, np.inf,
                                          weight="sin", wvar=r)[0]
    assert back == pytest.approx((2 / math.pi) * math.atan(r / c) / r, rel=1e-9)


@pytest.mark.parametrize("x", [1e-4, 3e-3, 9.9e-3, 1.01e-2, 0.3, 1.0, 7.0, 300.0])
def test_force_is_derivative_of_potential(x):
    """orc_cored_radial(r, s) * r = -(1/M m) dPhi/dr of Eq. (14), by a
    50-digit derivative of the potential, on both sides of the series
    switch at r / s = 1e-2."""
    s = 0.37
    r = x * s
    with mpmath.workdps(50):
        sm = mpmath.mpf(s)
        dphi = float(mpmath.diff(lambda q: -(2 / (mpmath.pi * q)) * mpmath.atan(q / sm), mpmath.mpf(x) * sm))
    # fp64 loses ~1e-12 next to the switch (series truncation on one side,
    # cancellation in atan x - x / (1 + x^2) on the other)
    assert oracle.cored_radial(r, s) * r == pytest.approx(dphi, rel=5e-12)


def test_limits():
    # s = 0: Newton; r << s: the finite core value (4 / 3 pi) / s^3
    assert oracle.cored_radial(0.25, 0.0) == pytest.approx(64.0, rel=1e-15)
    assert oracle.cored_radial(1e-9, 2.0) == pytest.approx(4.0 / (3.0 * math.pi) / 8.0, rel=1e-12)
    # r >> s: approaches Newton
    assert oracle.cored_radial(1.0, 1e-6) == pytest.approx(1.0, rel=1e-5)


def coincident_clump(nclump, seed):
    """Massless sinks of the point-like species 0 spread in the box, and a
    clump of nclump coincident bodies of the cored species 1 (unit mass)."""
    rng = np.random.default_rng(seed)
    n_spread = 3000
    X = np.empty((3, n_spread + nclump), np.uint64)
    X[:, :n_spread] = rng.integers(0, 2 ** 63, size=(3, n_spread), dtype=np.uint64) << np.uint64(1)
    X[:, n_spread:] = np.uint64(3 << 61)    # 0.375 of the box on every axis
    species = np.concatenate([np.zeros(n_spread, np.uint8), np.ones(nclump, np.uint8)])
    mass = np.concatenate([np.zeros(n_spread), np.ones(nclump)])
    return X, species, mass, slice(0, n_spread)


@pytest.mark.parametrize("track", [True, False])
def test_tracking_makes_coincident_monopoles_exact(track):
    """The only mass sits in N_perp coincident cored bodies, so every
    monopole the walk takes is theirs. With tracking each stands for bodies
    of mass M / N_perp and the tree force equals the direct sum up to
    rounding; without it the core is that of one body of mass M."""
    X, species, mass, spread = coincident_clump(32, 5)
    ntab = 64
    law = oracle.make_law(np.ones((2, 2)), np.ones((2, 2, ntab)), "r", 0.45, 1e-4, 0.9,
                          kind=oracle.LAW_ACCUMULATOR, cored=(1,), beta=1.0 / (4 * math.pi * 0.005),
                          track_counts=track)
    T = oracle.Tree(X, species, mass, 2, 1.0, leaf_size=4)
    T.monopoles()
    T.groups(8)
    acc, _, counts, _ = T.force(law)
    assert counts["pn"] > 200
    direct, _ = oracle.direct(X, species, mass, 2, 1.0, law)
    a, d = acc[:, spread], direct[:, spread]
    live = np.linalg.norm(d, axis=0) > 0
    assert live.sum() > 50
    err = np.linalg.norm(a - d, axis=0)[live] / np.linalg.norm(d, axis=0)[live]
    if track:
        assert np.max(err) < 1e-12
    else:
        assert np.max(err) > 1e-2


def test_tracking_reduces_tree_errors():
    """The claim of section 3.3 (Fig. 6): with N_perp tracked the tree force
    of a Newtonian and a cored species stays close to the direct sum; without
    it the errors grow by about an order of magnitude."""
    p = synth.clustered_problem(3000, 2, 41, f_cl=0.6, ntab=64, grid="r")
    tables = np.ones((2, 2, 64))
    G = np.ones((2, 2))
    beta = 0.5 / (4 * math.pi * 0.01 * 3000)      # core radius of one body ~ 0.005 of the box
    errs = {}
    for track in (True, False):
        law = oracle.make_law(G, tables, "r", 0.45, p.eps, 0.7, kind=oracle.LAW_ACCUMULATOR, cored=(1,),
                              beta=beta, track_counts=track)
        X = oracle.lattice_of(p)
        T = oracle.Tree(X, p.species, p.mass, p.D, p.box, leaf_size=8)
        T.monopoles()
        T.groups(64)
        acc, _, _, _ = T.force(law)
        direct, _ = oracle.direct(X, p.species, p.mass, p.D, p.box, law)
        rel = np.linalg.norm(acc - direct, axis=0) / np.linalg.norm(direct, axis=0)
        errs[track] = float(np.percentile(rel, 90))
    assert errs[True] * 5 < errs[False], errs


def test_direct_sum_brute_force():
    """The direct sum with an accumulator law against a 50-digit brute force
    written from Eqs. (16) and (14): the core scale of a pair adds the cores
    of whichever of the two species carry one, point-like pairs keep the
    softened Newtonian law, and G is taken as G[sink species, source species]."""
    rng = np.random.default_rng(17)
    n, D = 12, 3
    X = rng.integers(0, 2 ** 64, size=(3, n), dtype=np.uint64)
    species = np.array([0, 1, 2] * 4, np.uint8)
    mass = rng.uniform(0.5, 2.0, n)
    G = rng.uniform(0.5, 2.0, (D, D))
    beta, eps, r_cut = 2.0, 0.01, 0.45
    law = oracle.make_law(G, np.ones((D, D, 16)), "r", r_cut, eps, 0.5, kind=oracle.LAW_ACCUMULATOR,
                          cored=(1, 2), beta=beta)
    got, _ = oracle.direct(X, species, mass, D, 1.0, law)
    cored = {1, 2}
    with mpmath.workdps(50):
        for i in range(n):
            a = int(species[i])
            want = [mpmath.mpf(0)] * 3
            for j in range(n):
                if j == i:
                    continue
                b = int(species[j])
                d = []
                for x in range(3):
                    u = (int(X[x, j]) - int(X[x, i])) % 2 ** 64
                    d.append(mpmath.mpf(u - 2 ** 64 if u >= 2 ** 63 else u) / 2 ** 64)
                r = mpmath.sqrt(sum(c * c for c in d))
                if r >= r_cut:
                    continue
                s = ((mass[j] if b in cored else 0) + (mass[i] if a in cored else 0)) / (4 * mpmath.pi * beta)
                if s > 0:
                    g = mpmath.diff(lambda q: -(2 / (mpmath.pi * q)) * mpmath.atan(q / s), r) / r
                else:
                    g = 1 / (r * r + eps * eps) ** mpmath.mpf(1.5)
                for x in range(3):
                    want[x] += G[a, b] * mass[j] * g * d[x]
            assert np.allclose(got[:, i], [float(w) for w in want], rtol=1e-11, atol=0), i
