"""The transition test of section 3.1 on the oracle (tree short range plus
the numpy PM long range) against the exact periodic force of the source
(Ewald summation, oracle/ewald.py), and the pins of that reference.

The report: Delta f / f = |a_TreePM - a_exact| / |a_exact| of massless test
particles around one massive source, binned in log r and stacked over seeds.
Where the tree dominates (r well below r_s) the error is that of the tables
(about 1e-5); it peaks in the transition region (a few mesh cells, the mesh's
discreteness) and falls again at large r."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import pm as opm
from oracle.ewald import point_source_accel

EDGES = np.exp(np.linspace(math.log(1e-3), math.log(0.5), 21))


def test_ewald_split_independent_and_symmetric():
    rng = np.random.default_rng(1)
    d = rng.uniform(-0.5, 0.5, (3, 300))
    a1 = point_source_accel(d, alpha=2.0)
    a2 = point_source_accel(d, alpha=2.7, kmax=9)
    assert np.max(np.abs(a1 - a2)) <= 1e-12 * np.max(np.abs(a1))
    assert np.max(np.abs(point_source_accel(-d) + a1)) <= 1e-12 * np.max(np.abs(a1))          # odd
    assert np.max(np.abs(point_source_accel(d[[1, 2, 0]]) - a1[[1, 2, 0]])) <= 1e-12 * np.max(np.abs(a1))
    assert np.max(np.abs(point_source_accel(d + np.array([[1.0], [-2.0], [3.0]])) - a1)) <= 1e-11 * np.max(np.abs(a1))


def test_ewald_near_the_source():
    """Newton plus the neutralising background's (4 pi / 3) d / L^3 pull."""
    rng = np.random.default_rng(2)
    d = rng.normal(size=(3, 100))
    d *= 0.01 / np.linalg.norm(d, axis=0)
    lim = d / np.linalg.norm(d, axis=0) ** 3 - 4.0 * math.pi / 3.0 * d
    assert np.max(np.abs(point_source_accel(d) - lim)) <= 1e-8 * np.max(np.abs(lim))


def treepm_errors(p, mesh):
    T = oracle.Tree.of(p)
    at, _, _, _ = T.force(oracle.law_of(p))
    phib = np.full((2, 2, opm.max_q(mesh) + 1), -4.0 * math.pi)
    al = opm.pm_accel(oracle.lattice_of(p), p.species, p.mass, p.D, p.box, p.G, phib, mesh, p.r_s)
    d = p.pos[:, :1] - p.pos[:, 1:]
    ref = point_source_accel(d, p.box)
    r = np.linalg.norm(d - np.rint(d / p.box) * p.box, axis=0)
    return r, np.linalg.norm((at + al)[:, 1:] - ref, axis=0) / np.linalg.norm(ref, axis=0)


def binned_rms(r, e):
    return np.array([math.sqrt(np.mean(e[(r >= EDGES[k]) & (r < EDGES[k + 1])] ** 2)) for k in range(20)])


def check_profile(rms, r_s):
    mid = np.sqrt(EDGES[:-1] * EDGES[1:])
    assert np.all(rms[mid < 0.25 * r_s] <= 1e-4)          # tree-dominated: the tables' precision
    assert np.all(rms <= 2.5e-2)
    peak = mid[np.argmax(rms)]
    assert r_s <= peak <= 8.0 * r_s                       # the transition region


def test_transition_profile_of_the_oracle():
    mesh = 64
    parts = [treepm_errors(synth.transition_problem(s, per_shell=1000, mesh=mesh), mesh) for s in (1, 2)]
    r = np.concatenate([x[0] for x in parts])
    e = np.concatenate([x[1] for x in parts])
    rms = binned_rms(r, e)
    print("binned rms of Delta f/f:", " ".join(f"{v:.2e}" for v in rms))
    check_profile(rms, 1.25 / mesh)
