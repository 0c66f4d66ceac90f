"""Pins of pure-tree periodic mode with lattice corrections (section 2.3):
the Newtonian correction tables against a second, independently
parameterised Ewald sum and against the uniform-background limit; the
oracle's interpolated periodic force of two bodies against the Ewald force
directly; momentum conservation; the tree against the direct sum."""
import math

import numpy as np
import pytest
from scipy.special import erfc

import oracle
import synth


def ewald_force(x, alpha=2.7, nreal=5, kmax=7):
    """Force on a test particle at x (box 1) from unit masses at every lattice
    point with a neutralising background, by Ewald summation with its own
    splitting parameter and cut-offs."""
    F = np.zeros(3)
    for i in range(-nreal, nreal + 1):
        for j in range(-nreal, nreal + 1):
            for k in range(-nreal, nreal + 1):
                r = x - np.array([i, j, k], dtype=np.float64)
                rr = np.linalg.norm(r)
                if rr == 0:
                    continue
                F -= (erfc(alpha * rr) + 2 * alpha * rr / math.sqrt(math.pi) * math.exp(-alpha ** 2 * rr ** 2)) / rr ** 3 * r
    for i in range(-kmax, kmax + 1):
        for j in range(-kmax, kmax + 1):
            for k in range(-kmax, kmax + 1):
                if i == j == k == 0:
                    continue
                kv = 2 * math.pi * np.array([i, j, k], dtype=np.float64)
                k2 = kv @ kv
                F -= 4 * math.pi * math.exp(-k2 / (4 * alpha ** 2)) / k2 * math.sin(kv @ x) * kv
    return F


def test_tables_against_independent_ewald():
    T = synth.newtonian_lattice_correction(8)
    rng = np.random.default_rng(1)
    for _ in range(6):
        idx = rng.integers(0, 9, 3)
        d = idx / 16.0
        if not d.any():
            continue
        want = ewald_force(-d) - d / np.linalg.norm(d) ** 3      # the sink sits at -d from the source
        assert np.allclose(T[tuple(idx)], want, atol=1e-10)


def test_small_offset_is_the_background_term():
    """Near the source the images' pull cancels and the neutralising
    background leaves -(4 pi / 3) d."""
    T = synth.newtonian_lattice_correction(32)
    d = np.array([1, 0, 0]) / 64.0
    assert np.allclose(T[1, 0, 0], -4 * math.pi / 3 * d, rtol=2e-3, atol=1e-12)


def two_body(corr, x0, x1, G=np.ones((1, 1))):
    pos = np.array([x0, x1], dtype=np.float64).T.copy()
    X = oracle.lattice(pos, 1.0)
    law = oracle.make_law(G, np.ones((1, 1, 16)), "r2", 0.9, 0.0, 0.5, corr=corr[None, None])
    acc, _ = oracle.direct(X, np.zeros(2, np.uint8), np.array([1.0, 1.0]), 1, 1.0, law)
    return acc, X


def test_two_body_periodic_force():
    """The interpolated correction plus the nearest image gives the Ewald
    force within the table's trilinear interpolation error."""
    T = synth.newtonian_lattice_correction(32)
    rng = np.random.default_rng(2)
    worst = 0.0
    for _ in range(8):
        x0 = rng.random(3)
        x1 = rng.random(3)
        acc, X = two_body(T, x0, x1)
        d = ((X[:, 1].astype(np.int64) - X[:, 0].astype(np.int64)) * 2.0 ** -64)   # source - sink, nearest image
        want = ewald_force(-d)
        worst = max(worst, np.linalg.norm(acc[:, 0] - want) / np.linalg.norm(want))
        assert np.allclose(acc[:, 1], -acc[:, 0], rtol=1e-12, atol=1e-12)
    assert worst < 2e-3


def test_momentum_and_tree():
    p = synth.periodic_tree_problem(2000, 2, 3, EN=16, ntab=256)
    law = oracle.law_of(p)
    X = oracle.lattice_of(p)
    ref, _ = oracle.direct(X, p.species, p.mass, p.D, p.box, law)
    rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    assert np.linalg.norm((p.mass * ref).sum(axis=1)) < 1e-12 * rms * p.mass.sum()
    T = oracle.Tree.of(p)
    acc, _, cnt, _ = T.force(law)
    assert cnt["pn"] > 0
    rel = np.linalg.norm(acc - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.percentile(rel, 99) < 0.01
