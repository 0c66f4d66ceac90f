"""Pins of the oracle's particle-mesh step (the PM half of TreePM, sections
2 and 2.4.1): assignment and interpolation by hand values and exactness on
linear fields, the difference stencil's closed-form response, and the whole
chain against the physics it approximates: the Newtonian long-range force
(1 - f_short) m / r^2 of a point mass (with the uniform-background term of
a periodic box), and the Yukawa long-range force from its closed form;
momentum conservation and translation invariance."""
import math

import numpy as np
import pytest
from scipy.special import erfc

from oracle import pm

L = 1.0


def lattice_at(u, N):
    """Lattice coordinates of grid-unit positions u (exact for dyadic u)."""
    return np.array([int(round(x * 2 ** 64 / N)) % 2 ** 64 for x in u], dtype=np.uint64)


def test_cic_weights_exact():
    N = 16
    X = np.stack([lattice_at([3.0, 5.25, 15.5], N)] * 3)
    i, f = pm.cic_weights(X, N)
    assert list(i[0]) == [3, 5, 15]
    assert list(f[0]) == [0.0, 0.25, 0.5]


def test_deposit_by_hand_and_mass():
    N = 8
    h3 = (L / N) ** 3
    X = np.stack([lattice_at([2.0, 4.5], N), lattice_at([1.0, 1.0], N), lattice_at([7.0, 7.5], N)])
    rho = pm.deposit(X, np.array([0, 1]), np.array([2.0, 4.0]), 2, N, L)
    assert rho[0, 2, 1, 7] == pytest.approx(2.0 / h3)
    assert np.count_nonzero(rho[0]) == 1
    # species 1 at (4.5, 1, 7.5): half to x = 4, 5 and half to z = 7, 0 (periodic)
    for x in (4, 5):
        for z in (7, 0):
            assert rho[1, x, 1, z] == pytest.approx(1.0 / h3)
    rng = np.random.default_rng(1)
    Xr = rng.integers(0, 2 ** 64, size=(3, 500), dtype=np.uint64)
    m = rng.uniform(0.1, 1.0, 500)
    s = rng.integers(0, 3, 500)
    rho = pm.deposit(Xr, s, m, 3, N, L)
    for b in range(3):
        assert rho[b].sum() * h3 == pytest.approx(m[s == b].sum(), rel=1e-13)


def test_interpolation_exact_on_linear_fields():
    N = 16
    rng = np.random.default_rng(2)
    # positions away from the periodic seam so the linear field is continuous there
    u = rng.uniform(1.0, 13.0, size=(3, 200))
    X = np.stack([lattice_at(row, N) for row in u])
    g = np.arange(N, dtype=np.float64)
    field = np.stack([np.broadcast_to(c, (N, N, N)) for c in (2 * g[:, None, None] + 1,
                                                              -g[None, :, None] + 0 * g[:, None, None],
                                                              0.5 * g[None, None, :] + 0 * g[:, None, None])])
    out = pm.interpolate(field, X, N)
    uu = X.astype(np.float64) * N * 2.0 ** -64
    assert np.allclose(out[0], 2 * uu[0] + 1, atol=1e-12)
    assert np.allclose(out[1], -uu[1], atol=1e-12)
    assert np.allclose(out[2], 0.5 * uu[2], atol=1e-12)


@pytest.mark.parametrize("m", [1, 3, 7])
def test_stencil_response(m):
    """-d/dx of sin(2 pi m x / L) by the 4-point stencil is
    -cos(2 pi m x / L) [4/3 sin t - 1/6 sin 2t] / h, t = 2 pi m h / L."""
    N = 32
    h = L / N
    x = np.arange(N) * h
    phi = np.broadcast_to(np.sin(2 * math.pi * m * x / L)[:, None, None], (N, N, N)).copy()
    g = pm.gradient(phi, L)
    t = 2 * math.pi * m * h / L
    want = -np.cos(2 * math.pi * m * x / L) * (4.0 / 3.0 * math.sin(t) - math.sin(2 * t) / 6.0) / h
    assert np.allclose(g[0][:, 0, 0], want, atol=1e-12)
    assert np.max(np.abs(g[1])) < 1e-12 and np.max(np.abs(g[2])) < 1e-12


def newton_q(N):
    return np.full((1, 1, pm.max_q(N) + 1), -4 * math.pi)


def f_short_newton(r, r_s):
    return erfc(r / (2 * r_s)) + r / (r_s * math.sqrt(math.pi)) * np.exp(-r * r / (4 * r_s * r_s))


def test_point_mass_long_range_newton():
    """A unit mass and massless test particles at 3..10 mesh cells: the PM
    force is (1 - f_short(r)) / r^2 - (4 pi / 3) r / L^3 (the uniform
    background a periodic box subtracts) to the mesh's accuracy."""
    N = 64
    h = L / N
    r_s = 1.25 * h
    rng = np.random.default_rng(3)
    src = rng.integers(0, 2 ** 64, size=3, dtype=np.uint64)
    n_t = 400
    dirs = rng.normal(size=(3, n_t))
    dirs /= np.linalg.norm(dirs, axis=0)
    r = rng.uniform(3 * h, 10 * h, n_t)
    off = (dirs * r / L * 2.0 ** 64).astype(np.int64).view(np.uint64)
    X = np.concatenate([src[:, None], src[:, None] + off], axis=1)
    mass = np.concatenate([[1.0], np.zeros(n_t)])
    acc = pm.pm_accel(X, np.zeros(n_t + 1, np.int64), mass, 1, L, np.ones((1, 1)), newton_q(N), N, r_s)
    a = acc[:, 1:]
    radial = -np.sum(a * dirs, axis=0)           # toward the source
    want = (1 - f_short_newton(r, r_s)) / r ** 2 - 4 * math.pi / 3 * r / L ** 3
    err = (radial - want) / want
    tang = np.linalg.norm(a + radial * dirs, axis=0) / want
    assert np.sqrt(np.mean(err ** 2)) < 1e-2 and np.max(np.abs(err)) < 4e-2
    assert np.max(tang) < 3e-2


def test_point_mass_long_range_yukawa():
    """The same for -(alpha exp(-r/lam))/r alone: phibar = -4 pi alpha
    k^2/(k^2 + lam^-2); its long-range force is minus the derivative of the
    Gaussian-filtered screened potential (closed form), and a periodic box
    of this short-ranged law needs no background term."""
    N = 64
    h = L / N
    r_s = 1.25 * h
    alpha, lam = 0.8, 6 * h
    mu2 = 1 / lam ** 2
    q = np.arange(pm.max_q(N) + 1) * (2 * math.pi / L) ** 2
    phib = (-4 * math.pi * alpha * q / (q + mu2))[None, None, :]
    rng = np.random.default_rng(4)
    src = rng.integers(0, 2 ** 64, size=3, dtype=np.uint64)
    n_t = 300
    dirs = rng.normal(size=(3, n_t))
    dirs /= np.linalg.norm(dirs, axis=0)
    r = rng.uniform(3 * h, 8 * h, n_t)
    off = (dirs * r / L * 2.0 ** 64).astype(np.int64).view(np.uint64)
    X = np.concatenate([src[:, None], src[:, None] + off], axis=1)
    mass = np.concatenate([[1.0], np.zeros(n_t)])
    acc = pm.pm_accel(X, np.zeros(n_t + 1, np.int64), mass, 1, L, np.ones((1, 1)), phib, N, r_s)
    radial = -np.sum(acc[:, 1:] * dirs, axis=0)

    def long_pot(x):        # Gaussian-filtered -alpha exp(-mu x)/x, mu = 1/lam
        mu = 1 / lam
        c = math.exp(mu * mu * r_s * r_s) / (2 * x)
        y = x / (2 * r_s)
        return -alpha * c * (math.exp(-mu * x) * erfc(mu * r_s - y) - math.exp(mu * x) * erfc(mu * r_s + y))
    dx = 1e-6
    want = np.array([(long_pot(x + dx) - long_pot(x - dx)) / (2 * dx) for x in r])
    err = (radial - want) / np.abs(want)
    assert np.sqrt(np.mean(err ** 2)) < 2e-2


def test_momentum_and_translation():
    N = 32
    rng = np.random.default_rng(5)
    n = 300
    X = rng.integers(0, 2 ** 64, size=(3, n), dtype=np.uint64)
    s = rng.integers(0, 2, n)
    m = rng.uniform(0.5, 1.5, n)
    G = np.array([[1.0, 0.4], [0.4, 2.0]])
    q = np.arange(pm.max_q(N) + 1) * (2 * math.pi / L) ** 2
    phib = np.stack([np.stack([np.full_like(q, -4 * math.pi), -4 * math.pi * (1 + 0.5 * q / (q + 400.0))]),
                     np.stack([-4 * math.pi * (1 + 0.5 * q / (q + 400.0)), np.full_like(q, -4 * math.pi)])])
    r_s = 1.25 / N
    acc = pm.pm_accel(X, s, m, 2, L, G, phib, N, r_s)
    rms = np.sqrt(np.mean(np.sum(acc ** 2, axis=0)))
    assert np.linalg.norm((m * acc).sum(axis=1)) < 1e-12 * rms * m.sum()
    shift = np.uint64(2 ** 64 // N * 3)
    acc2 = pm.pm_accel(X + shift, s, m, 2, L, G, phib, N, r_s)
    assert np.max(np.abs(acc2 - acc)) < 1e-11 * rms
