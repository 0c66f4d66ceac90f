"""Pins of the oracle's exact short-range factors (section 2.4.1, Eqs.
(8)-(11)) against closed forms: the Newtonian split the paper states, the
screened (Yukawa) split written from the Ewald-type transform of a
Gaussian-filtered exp(-mu r) / r, superposition, and the limits."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import erfc

from oracle.short_range import short_factor

HERE = os.path.dirname(os.path.abspath(__file__))


def newton_closed(r, r_s):
    return erfc(r / (2 * r_s)) + r / (r_s * math.sqrt(math.pi)) * math.exp(-r * r / (4 * r_s * r_s))


def yukawa_long_potential(r, r_s, mu):
    """Inverse transform of 4 pi exp(-k^2 r_s^2) / (k^2 + mu^2): the long-range
    part of exp(-mu r) / r, by completing the square in the Gaussian
    convolution of the screened kernel."""
    c = math.exp(mu * mu * r_s * r_s) / (2 * r)
    x = r / (2 * r_s)
    return c * (math.exp(-mu * r) * erfc(mu * r_s - x) - math.exp(mu * r) * erfc(mu * r_s + x))


def yukawa_short_closed(r, r_s, alpha, lam):
    """Short-range factor of -(1 + alpha exp(-r/lam)) / r: Newton's plus
    alpha times that of the screened part, r^2 d/dr of -(e^{-mu r}/r - long)."""
    mu = 1.0 / lam
    h = r * 1e-5
    full = lambda q: -math.exp(-mu * q) / q
    long_ = lambda q: -yukawa_long_potential(q, r_s, mu)
    d = lambda fn: (fn(r + h) - fn(r - h)) / (2 * h)    # smooth closed forms: centred difference
    return newton_closed(r, r_s) + alpha * r * r * (d(full) - d(long_))


NEWTON = (lambda k: -4 * math.pi, lambda r: 1.0)


def test_paper_newtonian_statement():
    """The golden constant from section 2.4.1 (the Newtonian short-range
    potential is phi erfc(r/2r_s); its derivative is this factor)."""
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as fh:
        c = json.load(fh)["newtonian_short_range_factor"]["value"]
    assert c.startswith("erfc(r/(2 r_s))")
    r_s = 0.0195
    for r in np.linspace(0.0, 5 * r_s, 41):
        assert short_factor(*NEWTON, r_s, float(r)) == pytest.approx(newton_closed(float(r), r_s), abs=2e-13)


@pytest.mark.parametrize("alpha,lam", [(1.0, 0.01), (-0.5, 0.003), (0.7, 0.03)])
def test_yukawa_closed_form(alpha, lam):
    r_s = 0.0025
    mu2 = 1.0 / lam ** 2
    phibar = lambda k: -4 * math.pi * (1 + alpha * k * k / (k * k + mu2))
    f_full = lambda r: 1 + alpha * (1 + r / lam) * math.exp(-r / lam)
    for r in np.linspace(0.1 * r_s, 4.5 * r_s, 23):
        got = short_factor(phibar, f_full, r_s, float(r))
        # the closed form's centred difference limits the agreement to ~1e-9
        assert got == pytest.approx(yukawa_short_closed(float(r), r_s, alpha, lam), abs=2e-8)


def test_superposition_and_scaling():
    """Linear in the law; f_short(r; r_s) depends on r / r_s only for Newton."""
    r_s = 0.01
    lam = 0.02
    yk = (lambda k: -4 * math.pi * k * k / (k * k + lam ** -2), lambda r: (1 + r / lam) * math.exp(-r / lam))
    both = (lambda k: NEWTON[0](k) + 0.3 * yk[0](k), lambda r: 1.0 + 0.3 * yk[1](r))
    for r in (0.003, 0.02, 0.04):
        s = short_factor(*NEWTON, r_s, r) + 0.3 * (short_factor(*yk, r_s, r) - 0.0)
        # yk alone carries no Newtonian part; its own short factor is f_full + integral term
        assert short_factor(*both, r_s, r) == pytest.approx(s, abs=1e-13)
        assert short_factor(*NEWTON, 2 * r_s, 2 * r) == pytest.approx(short_factor(*NEWTON, r_s, r), abs=1e-13)


def test_limits():
    r_s = 0.01
    assert short_factor(*NEWTON, r_s, 0.0) == 1.0
    assert short_factor(*NEWTON, r_s, 1e-6) == pytest.approx(1.0, abs=1e-12)
    assert abs(short_factor(*NEWTON, r_s, 14 * r_s)) < 1e-17 * 1e6
