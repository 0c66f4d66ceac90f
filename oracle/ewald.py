"""The exact periodic Newtonian force of one point mass, by Ewald summation:
the reference of the transition test (section 3.1), where the TreePM force
(tree short range plus mesh long range) of a massive source on test
particles is compared with the force of the source and all its periodic
images. TEST INFRASTRUCTURE ONLY, like the rest of this package.

For a sink at offset d = x_source - x_sink in a cube of side L (taken to its
minimum image first, so the result is periodic in d), the acceleration per
unit G M is

    a(d) = sum_n  g(|d + n L|) (d + n L) / |d + n L|^3
           + (4 pi / L^3) sum_{k != 0} exp(-k^2 / (4 a^2)) / k^2  k sin(k . d),
    g(s) = erfc(a s) + (2 a s / sqrt(pi)) exp(-a^2 s^2),

the real-space images n in Z^3 and the wave vectors k = 2 pi m / L, m in Z^3;
the split scale a drops out of the sum (the splitting identity of Ewald), and
the k = 0 term is left out, i.e. the periodic mean density is removed (a
neutralising background, as in every periodic PM). Near the source
a(d) -> d / |d|^3 - (4 pi / 3) d / L^3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

__all__ = ["point_source_accel"]


def point_source_accel(d: np.ndarray, box: float = 1.0, alpha: float = 2.0, nreal: int = 3,
                       kmax: int = 7, chunk: int = 65536) -> np.ndarray:
    """a(d) for offsets d of shape (3, n), per unit G M. alpha is the split
    in units of 1 / box; nreal and kmax the image and wave-vector ranges
    (|n_i| <= nreal, |m_i| <= kmax): with alpha = 2 both sums are converged
    to well below 1e-12 of Newton's force at the box scale."""
    L = float(box)
    d = np.asarray(d, dtype=np.float64)
    d = d - L * np.rint(d / L)                    # the minimum image: the truncated sums are centred on it
    a = alpha / L
    out = np.zeros_like(d)
    ns = np.arange(-nreal, nreal + 1)
    images = np.array(np.meshgrid(ns, ns, ns, indexing="ij")).reshape(3, -1).T * L      # (M, 3)
    ms = np.arange(-kmax, kmax + 1)
    mv = np.array(np.meshgrid(ms, ms, ms, indexing="ij")).reshape(3, -1).T
    mv = mv[np.any(mv != 0, axis=1)]
    kv = 2.0 * math.pi / L * mv                                                          # (K, 3)
    k2 = np.sum(kv * kv, axis=1)
    kamp = (4.0 * math.pi / L ** 3) * np.exp(-k2 / (4.0 * a * a)) / k2                  # (K,)
    for s in range(0, d.shape[1], chunk):
        dd = d[:, s:s + chunk].T                                                         # (c, 3)
        acc = np.zeros_like(dd)
        for img in images:
            r = dd + img
            rr = np.sqrt(np.sum(r * r, axis=1))
            with np.errstate(divide="ignore", invalid="ignore"):
                g = (erfc(a * rr) + 2.0 * a * rr / math.sqrt(math.pi) * np.exp(-a * a * rr * rr)) / rr ** 3
            g = np.where(rr > 0, g, 0.0)
            acc += g[:, None] * r
        acc += np.sin(dd @ kv.T) @ (kamp[:, None] * kv)
        out[:, s:s + chunk] = acc.T
    return out
