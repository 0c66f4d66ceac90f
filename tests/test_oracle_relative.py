"""Pins of the oracle's relative opening test (section 2.2: the walk keeps
the stock code's criterion, the previous acceleration against a Newtonian
estimate of the node's contribution): decisions against exact rational
arithmetic on image-enumerated geometry, the exactness limit alpha -> 0,
and the force accuracy the criterion delivers against the direct sum."""
from fractions import Fraction

import numpy as np

import oracle
import synth
from test_oracle_pins import corner_of, periodic_box_distances


def test_decisions_match_exact_arithmetic(oracle_lib):
    """prune iff gap >= r_cut; open when the group's box reaches into the
    node's cube grown to 1.2 sides; else accept iff M l^2 <= alpha a_min d^4
    (l, d in the box's length units, M the node's mass over all species)
    and the whole cell lies within r_cut. Decisions whose two sides agree to
    1e-12 are skipped (float64 may round either way there)."""
    p = synth.clustered_problem(6000, 3, 8, ntab=16)
    T = oracle_lib.Tree.of(p, group_size=32)
    nd = T.nodes()
    M, _ = T.monopole_arrays()
    rng = np.random.default_rng(4)
    P = 1 << 20
    u = Fraction(p.box) / (1 << 21)
    deep = np.nonzero(nd["level"] >= 2)[0]
    seen = set()
    skipped = 0
    for it in range(1500):
        i = int(rng.choice(deep))
        lvl = int(nd["level"][i])
        c = corner_of(lvl, nd["prefix"][i])
        S = 1 << (20 - lvl)
        lo = rng.integers(0, P - 1, 3)
        hi = np.minimum(lo + rng.integers(1, P // (8 if it % 2 else 512), 3), P)
        gap2 = far2 = 0
        inside = True
        for a in range(3):
            g, f = periodic_box_distances(c[a], c[a] + S, int(lo[a]), int(hi[a]), P)
            gap2 += (2 * g) ** 2
            far2 += (2 * f) ** 2
            # centre distance (half key units) against the grown half-widths
            w = int(hi[a]) - int(lo[a])
            dc = abs(((2 * c[a] + S) - (int(lo[a]) + int(hi[a])) + P) % (2 * P) - P)
            inside &= 5 * dc < 6 * S + 5 * w
        alpha = float(10 ** rng.uniform(-4, -1))
        a_min = float(10 ** rng.uniform(-1, 3))
        mass = sum(Fraction(float(x)) for x in M[:, i])
        for rcut_keys in (3000.0, 30000.0, 200000.0, 400000.0):
            R2 = (2 * rcut_keys) ** 2
            rel_k = alpha * float(u * u)
            d = T.mac_relative(i, lo.astype(np.uint32), hi.astype(np.uint32), R2, rel_k, a_min)
            lhs = mass * 4 * S * S
            rhs = Fraction(rel_k) * Fraction(a_min) * gap2 * gap2
            if gap2 >= R2:
                want = oracle.PRUNE
            elif inside:
                want = oracle.OPEN
            else:
                if rhs > 0 and abs(lhs - rhs) <= Fraction(1, 10 ** 12) * rhs:
                    skipped += 1
                    continue
                want = oracle.ACCEPT if (lhs <= rhs and far2 < R2) else oracle.OPEN
            assert d == want, (it, rcut_keys)
            seen.add(want)
    assert seen == {oracle.PRUNE, oracle.ACCEPT, oracle.OPEN}
    assert skipped < 5


def relative(p, alpha):
    ref, _ = oracle.direct_of(p)
    import dataclasses
    return dataclasses.replace(p, relative={"alpha": alpha, "old_acc": np.linalg.norm(ref, axis=0)}), ref


def test_alpha_to_zero_is_the_direct_sum(oracle_lib):
    p = synth.clustered_problem(3000, 2, 9, ntab=256)
    q, ref = relative(p, 1e-30)
    acc, _, cnt, _ = oracle.Tree.of(q).force(oracle.law_of(q))
    rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    assert cnt["pn"] == 0
    assert np.max(np.abs(acc - ref)) < 1e-12 * rms


def test_accuracy_follows_alpha(oracle_lib):
    """Errors fall with alpha, and at alpha = 0.0025 stay within the paper's
    tree tolerance (0.005) at the 99th percentile."""
    p = synth.clustered_problem(6000, 3, 10, ntab=512)
    errs = []
    for alpha in (0.02, 0.0025):
        q, ref = relative(p, alpha)
        acc, _, cnt, _ = oracle.Tree.of(q).force(oracle.law_of(q))
        live = np.linalg.norm(ref, axis=0) > 0          # some particles have no neighbour within r_cut
        rel = np.linalg.norm(acc - ref, axis=0)[live] / np.linalg.norm(ref, axis=0)[live]
        errs.append(float(np.percentile(rel, 99)))
        assert cnt["pn"] > 0
    assert errs[1] < errs[0]
    assert errs[1] < 0.005, errs
