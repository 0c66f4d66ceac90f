"""Exact short-range force factors of a general pair law (section 2.4.1,
Eqs. (8)-(11)). TEST INFRASTRUCTURE ONLY, like the rest of this package.

Conventions (the paper leaves them implicit): per unit active and passive
mass a pair potential phi(r) has the 3-D transform
    phi(k) = integral phi(x) exp(-i k.x) d^3x,
so that Newton's phi = -1/r has phi(k) = -4 pi / k^2, and
    phibar(k) = k^2 phi(k)
is the law normalised by the Newtonian Green's function (Newton: -4 pi;
Yukawa -(1 + alpha exp(-r/lam)) / r: -4 pi (1 + alpha k^2 / (k^2 + lam^-2))).
The long-range part is the inverse transform of phi(k) exp(-k^2 r_s^2), the
short-range part phi - phi_long (Eq. (8)). Written radially,
    phi_long(r) = 1 / (2 pi^2 r) * int_0^inf phibar(k) exp(-k^2 r_s^2) sin(k r) / k dk,
the r'-integral of Eq. (10) done in closed form (int_0^r cos(k r') dr' =
sin(k r) / k). Force factors are relative to Newton's 1/r^2: a law's full
factor is f_full(r) = r^2 dphi/dr (Newton: 1), and differentiating under the
integral (Eq. (11)) gives the short-range factor
    f_short(r) = f_full(r) + 1 / (2 pi^2) * int_0^inf phibar(k) exp(-k^2 r_s^2)
                                          [sin(k r) / k - r cos(k r)] dk.
The integral is taken by adaptive Gauss-Kronrod quadrature in float64 up to
the k where the Gaussian has fallen below 1e-17 of its peak. For Newton it
reduces to erfc(r / 2 r_s) + r / (r_s sqrt(pi)) exp(-r^2 / 4 r_s^2), the
paper's own statement for that case.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np
from scipy import integrate

__all__ = ["short_factor", "short_tables"]


def short_factor(phibar: Callable[[float], float], f_full: Callable[[float], float], r_s: float,
                 r: float) -> float:
    """f_short(r) of the law (phibar, f_full) for a Gaussian split of scale r_s."""
    if r == 0.0:
        return float(f_full(0.0))        # the bracket vanishes at r = 0
    kmax = math.sqrt(17.0 * math.log(10.0)) / r_s

    def integrand(k):
        if k == 0.0:
            return 0.0
        kr = k * r
        if kr < 1e-3:                    # sin(kr)/k - r cos(kr) = r (kr)^2 / 3 - r (kr)^4 / 30 + ...
            bracket = r * kr * kr * (1.0 / 3.0 - kr * kr / 30.0)
        else:
            bracket = math.sin(kr) / k - r * math.cos(kr)
        return phibar(k) * math.exp(-(k * r_s) ** 2) * bracket

    val, err = integrate.quad(integrand, 0.0, kmax, limit=2000, epsabs=1e-15, epsrel=1e-13)
    return float(f_full(r)) + val / (2.0 * math.pi ** 2)


def short_tables(phibar_ab, f_full_ab, r_s: float, radii: np.ndarray) -> np.ndarray:
    """Tables D x D x len(radii) of f_short for per-pair callables
    phibar_ab[a][b] and f_full_ab[a][b] at the given radii."""
    D = len(phibar_ab)
    out = np.empty((D, D, len(radii)))
    for a in range(D):
        for b in range(D):
            for i, r in enumerate(radii):
                out[a, b, i] = short_factor(phibar_ab[a][b], f_full_ab[a][b], r_s, float(r))
    return out
