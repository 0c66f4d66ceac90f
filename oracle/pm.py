"""Particle-mesh long-range accelerations of D species (section 2, the PM
part of TreePM; section 2.4: every species is both a passive and an active
mass for the mesh). TEST INFRASTRUCTURE ONLY, like the rest of this package.

The steps, in the order the paper lists them:
  1. assign each species' particles to a density on a regular periodic grid
     of N^3 points (cloud in cell: a particle at u = x N / L in grid units
     gives weight (1 - f) to point floor(u) and f to the next, per axis,
     f = u - floor(u); density = mass x weight / h^3, h = L / N);
  2. Fourier transform each species' density (numpy.fft.fftn, forward
     exp(-i k.x), unnormalised);
  3. multiply by the k-space Green's function of each species pair and sum
     over source species b for every sink species a:
       Phi_a(k) = sum_b G_ab phi_ab(k) exp(-k^2 r_s^2) / W(k)^2 rho_b(k),
     phi_ab(k) = phibar_ab(k) / k^2 (the law's transform, phibar = k^2 phi(k)
     as in the short-range tables), the Gaussian filter of TreePM mode
     (section 2.4.1), W the cloud-in-cell window prod_axes sinc^2(k_x h / 2)
     divided out once for the assignment and once for the interpolation,
     and k = 0 left out (the periodic mean);
  4. invert the transform (numpy.fft.ifftn): the potential of each sink
     species on the grid;
  5. differentiate with the 4-point centred difference
       dPhi/dx = [2/3 (Phi(i+1) - Phi(i-1)) - 1/12 (Phi(i+2) - Phi(i-2))] / h
     and interpolate -grad Phi_a back to each particle of species a with
     the same cloud-in-cell weights.
This is the scheme of the code the paper extends (GADGET-2): its details
(assignment, window, stencil) are not printed in the paper and are taken as
that code's published scheme.

The law enters through phibar_ab at the mesh's own |k| values: the squared
integer frequency q = i^2 + j^2 + l^2 (signed frequencies, |i| <= N/2) fixes
|k| = 2 pi sqrt(q) / L, so the table phibar_q has entries q = 0 .. 3 (N/2)^2.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["cic_weights", "deposit", "green", "potential", "gradient", "interpolate", "pm_accel", "max_q"]


def max_q(N: int) -> int:
    return 3 * (N // 2) ** 2


def cic_weights(X: np.ndarray, N: int):
    """Lower grid index (3, n) and fraction (3, n) of lattice positions X
    (uint64, the point X 2^-64 L): u = X N 2^-64 exactly, N a power of two."""
    p = int(N).bit_length() - 1
    assert 1 << p == N
    shift = np.uint64(64 - p)
    i = (X >> shift).astype(np.int64)
    f = (X & np.uint64((1 << (64 - p)) - 1)).astype(np.float64) * 2.0 ** -(64 - p)
    return i, f


def deposit(X, species, mass, D: int, N: int, box: float) -> np.ndarray:
    """Step 1: (D, N, N, N) densities."""
    i, f = cic_weights(X, N)
    rho = np.zeros((D, N, N, N))
    h3 = (box / N) ** 3
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                w = mass * wx * wy * wz / h3
                np.add.at(rho, (species.astype(np.int64), (i[0] + cx) % N, (i[1] + cy) % N, (i[2] + cz) % N), w)
    return rho


def _freqs(N: int):
    return np.fft.fftfreq(N, 1.0 / N).astype(np.int64)     # signed integer frequencies


def green(G, phibar_q, N: int, box: float, r_s: float) -> np.ndarray:
    """Step 3's multiplier (D, D, N, N, N): G_ab phibar_ab(q)/k^2 exp(-k^2 r_s^2)/W^2."""
    D = G.shape[0]
    n = _freqs(N)
    q = (n[:, None, None] ** 2 + n[None, :, None] ** 2 + n[None, None, :] ** 2)
    k2 = q * (2.0 * math.pi / box) ** 2
    s = np.sinc(n / N)                                      # sin(pi n/N)/(pi n/N) = sinc(k h / 2)
    W = (s[:, None, None] * s[None, :, None] * s[None, None, :]) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        base = np.where(q > 0, np.exp(-k2 * r_s * r_s) / (k2 * W * W), 0.0)
    out = np.empty((D, D, N, N, N))
    for a in range(D):
        for b in range(D):
            out[a, b] = G[a, b] * phibar_q[a, b][q] * base
    return out


def potential(rho, Gk) -> np.ndarray:
    """Steps 2-4: (D, N, N, N) real potentials of the sink species."""
    D = rho.shape[0]
    rk = np.fft.fftn(rho, axes=(1, 2, 3))
    phi = np.empty_like(rho)
    for a in range(D):
        pk = np.zeros(rho.shape[1:], dtype=np.complex128)
        for b in range(D):
            pk += Gk[a, b] * rk[b]
        phi[a] = np.fft.ifftn(pk).real
    return phi


def gradient(phi_a, box: float) -> np.ndarray:
    """Step 5's difference: (3, N, N, N) = -grad Phi on the grid."""
    N = phi_a.shape[0]
    h = box / N
    out = np.empty((3,) + phi_a.shape)
    for ax in range(3):
        d1 = np.roll(phi_a, -1, axis=ax) - np.roll(phi_a, 1, axis=ax)
        d2 = np.roll(phi_a, -2, axis=ax) - np.roll(phi_a, 2, axis=ax)
        out[ax] = -(2.0 / 3.0 * d1 - 1.0 / 12.0 * d2) / h
    return out


def interpolate(field, X, N: int) -> np.ndarray:
    """Step 5's interpolation of a (3, N, N, N) field to (3, n)."""
    i, f = cic_weights(X, N)
    out = np.zeros((3, X.shape[1]))
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                w = wx * wy * wz
                out += w * field[:, (i[0] + cx) % N, (i[1] + cy) % N, (i[2] + cz) % N]
    return out


def pm_accel(X, species, mass, D: int, box: float, G, phibar_q, N: int, r_s: float) -> np.ndarray:
    """Long-range accelerations (3, n) of every particle."""
    X = np.ascontiguousarray(X, dtype=np.uint64)
    species = np.asarray(species)
    rho = deposit(X, species, np.asarray(mass, dtype=np.float64), D, N, box)
    phi = potential(rho, green(np.asarray(G, dtype=np.float64), np.asarray(phibar_q), N, box, r_s))
    acc = np.zeros((3, X.shape[1]))
    for a in range(D):
        sel = np.nonzero(species == a)[0]
        if sel.size:
            acc[:, sel] = interpolate(gradient(phi[a], box), X[:, sel], N)
    return acc
