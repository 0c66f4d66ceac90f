"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one step of the oracle against a worked example, a library
routine, a brute-force construction on a tiny input, a closed form or an
invariant, so that a dropped term, a wrong sign or index, a transposed
operand or a wrong wrap in the oracle fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import erfc

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def paper_constant(name):
    with open(os.path.join(GOLD, "paper_constants.json")) as f:
        return json.load(f)[name]["value"]


# --------------------------------------------------------------- keys -----
def morton_by_string(kx, ky, kz):
    """Independent key: write the 20 digits (x y z bits) from the top down as
    a binary string and parse it."""
    s = "".join(f"{(kx >> b) & 1}{(ky >> b) & 1}{(kz >> b) & 1}" for b in range(19, -1, -1))
    return int(s, 2)


def test_morton_worked_examples(oracle_lib):
    rows = [l.split() for l in open(os.path.join(GOLD, "morton_examples.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 8
    for kx, ky, kz, key in rows:
        assert oracle_lib.morton(int(kx), int(ky), int(kz)) == int(key)


def test_keys_match_bit_string_construction(oracle_lib):
    rng = np.random.default_rng(11)
    n = 2000
    X = synth.uniform_lattice(n, rng)
    s = rng.integers(0, 6, n).astype(np.uint8)
    K = oracle_lib.keys(X, s)
    for i in range(n):
        kx, ky, kz = (int(X[a, i]) >> 44 for a in range(3))
        assert int(K[i]) == (int(s[i]) << 60) | morton_by_string(kx, ky, kz)


def test_keys_decode_roundtrip(oracle_lib):
    rng = np.random.default_rng(12)
    for _ in range(500):
        k = [int(v) for v in rng.integers(0, 1 << 20, 3)]
        m = oracle_lib.morton(*k)
        dec = [0, 0, 0]
        for b in range(20):
            for a in range(3):
                dec[a] |= ((m >> (3 * b + 2 - a)) & 1) << b
        assert dec == k


def test_lattice_conversion(oracle_lib):
    x = np.array([[0.0, 0.5, 0.25, 1.0 - 2.0 ** -53, -0.25, 1.25],
                  [0.0] * 6, [0.75] * 6])
    X = oracle_lib.lattice(x, 1.0)
    assert int(X[0, 0]) == 0
    assert int(X[0, 1]) == 1 << 63
    assert int(X[0, 2]) == 1 << 62
    assert int(X[0, 3]) == (1 << 64) - (1 << 11)
    assert int(X[0, 4]) == 3 << 62          # periodic: -0.25 == 0.75
    assert int(X[0, 5]) == 1 << 62          # periodic: 1.25 == 0.25
    assert all(int(v) == 3 << 62 for v in X[2])
    # box scaling
    X2 = oracle_lib.lattice(x * 7.5, 7.5)
    assert np.array_equal(X, X2)


# --------------------------------------------------------------- sort -----
def test_sort_is_stable_library_sort(oracle_lib):
    rng = np.random.default_rng(13)
    n = 5000
    K = rng.integers(0, 64, n).astype(np.uint64) << np.uint64(58)  # many ties
    perm = oracle_lib.sort(K)
    assert np.array_equal(perm, np.argsort(K, kind="stable").astype(np.uint32))


# --------------------------------------------------------------- tree -----
def brute_tree(kappa, species, D, B):
    """Recursive halving of the 2^20 key cube by explicit cell membership
    (no keys): returns {(level, corner tuple): per-species counts}."""
    out = {}

    def rec(level, corner, idx):
        counts = tuple(int(np.sum(species[idx] == b)) for b in range(D))
        out[(level, corner)] = counts
        if len(idx) <= B or level == 20:
            return
        half = 1 << (20 - level - 1)
        for o in range(8):
            c = (corner[0] + half * ((o >> 2) & 1), corner[1] + half * ((o >> 1) & 1), corner[2] + half * (o & 1))
            inside = np.all((kappa[:, idx] >= np.array(c)[:, None]) & (kappa[:, idx] < np.array(c)[:, None] + half), axis=0)
            sub = idx[inside]
            if len(sub):
                rec(level + 1, c, sub)

    rec(0, (0, 0, 0), np.arange(kappa.shape[1]))
    return out


def corner_of(level, prefix):
    c = [0, 0, 0]
    for d in range(level):
        for a in range(3):
            c[a] |= ((int(prefix) >> (3 * d + 2 - a)) & 1) << d
    return tuple(v << (20 - level) for v in c)


@pytest.mark.parametrize("B", [1, 4])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tree_matches_brute_force_subdivision(oracle_lib, B, seed):
    rng = np.random.default_rng(seed)
    n, D = 48, 3
    # cluster half the points so that the tree goes deep
    X = synth.uniform_lattice(n, rng)
    X[:, : n // 2] = X[:, :1] + (rng.integers(0, 1 << 50, (3, n // 2)).astype(np.uint64))
    s = rng.integers(0, D, n).astype(np.uint8)
    m = rng.random(n)
    T = oracle_lib.Tree(X, s, m, D, 1.0, B)
    nd = T.nodes()
    kappa = (X >> np.uint64(44)).astype(np.int64)
    ref = brute_tree(kappa, s, D, B)
    got = {}
    for i in range(T.n_nodes):
        key = (int(nd["level"][i]), corner_of(int(nd["level"][i]), nd["prefix"][i]))
        got[key] = tuple(int(nd["count"][b, i]) for b in range(D))
    assert got == ref
    # breadth-first order: sorted by (level, prefix)
    order = list(zip(nd["level"].tolist(), nd["prefix"].tolist()))
    assert order == sorted(order)
    # children: contiguous, one level down, counts add up, parent pointers
    for i in range(T.n_nodes):
        nc, fc = int(nd["n_child"][i]), int(nd["first_child"][i])
        total = int(nd["count"][:, i].sum())
        if nc == 0:
            assert total <= B or nd["level"][i] == 20
            continue
        assert total > B
        ch = range(fc, fc + nc)
        assert all(nd["parent"][c] == i and nd["level"][c] == nd["level"][i] + 1 for c in ch)
        assert np.array_equal(nd["count"][:, list(ch)].sum(axis=1), nd["count"][:, i])
    # per-species ranges: inside the species segment, holding that species
    perm, keys = nd["perm"], nd["keys"]
    ss = s[perm]
    for i in range(T.n_nodes):
        for b in range(D):
            st, c = int(nd["start"][b, i]), int(nd["count"][b, i])
            assert np.all(ss[st:st + c] == b)


def test_monopoles_match_exact_rational_sums(oracle_lib):
    rng = np.random.default_rng(21)
    n, D, box = 200, 2, 3.0
    X = synth.uniform_lattice(n, rng)
    X[:, :100] = (X[:, :1] + rng.integers(0, 1 << 56, (3, 100)).astype(np.uint64))
    s = rng.integers(0, D, n).astype(np.uint8)
    m = rng.random(n) + 0.1
    T = oracle_lib.Tree(X, s, m, D, box, 4)
    T.monopoles()
    nd = T.nodes()
    M, com = T.monopole_arrays()
    perm = nd["perm"]
    for i in range(0, T.n_nodes, 3):
        for b in range(D):
            st, c = int(nd["start"][b, i]), int(nd["count"][b, i])
            idx = perm[st:st + c]
            if c == 0:
                assert M[b, i] == 0.0
                continue
            Mq = sum(Fraction(float(v)) for v in m[idx])
            assert abs(M[b, i] - float(Mq)) <= 1e-15 * float(Mq)
            for a in range(3):
                cq = sum(Fraction(float(m[j])) * Fraction(int(X[a, j])) for j in idx) / Mq
                ref = float(cq * Fraction(box) / Fraction(2 ** 64))
                assert abs(com[b, a, i] - ref) <= 1e-14 * box


# --------------------------------------------------------------- groups ---
@pytest.mark.parametrize("Ng", [16, 64])
def test_groups_partition_species_runs(oracle_lib, Ng):
    p = synth.clustered_problem(6000, 3, 5, ntab=64)
    T = oracle_lib.Tree.of(p, group_size=Ng)
    g = T.group_arrays()
    nd = T.nodes()
    perm = nd["perm"]
    X = oracle_lib.lattice_of(p)
    ss = p.species[perm]
    covered = np.zeros(p.n, dtype=np.int64)
    prev_end = {}
    for k in range(T.n_groups):
        a, st, c = int(g["species"][k]), int(g["start"][k]), int(g["count"][k])
        assert 1 <= c <= Ng
        assert np.all(ss[st:st + c] == a)
        covered[st:st + c] += 1
        if a in prev_end:
            assert st == prev_end[a]          # groups of a species are consecutive
        prev_end[a] = st + c
        kap = (X[:, perm[st:st + c]] >> np.uint64(44)).astype(np.int64)
        assert np.array_equal(g["lo"][:, k], kap.min(axis=1))
        assert np.array_equal(g["hi"][:, k], kap.max(axis=1) + 1)
    assert np.all(covered == 1)
    assert np.mean(g["count"]) > 0.35 * Ng   # runs of siblings are merged


# --------------------------------------------------------------- MAC ------
def periodic_box_distances(c0, c1, b0, b1, P):
    """Smallest gap and largest distance between points of [c0,c1) and
    [b0,b1) on a circle of period P, for the image of the box whose centre is
    nearest to the cell's centre, found by trying the images k = -1, 0, 1."""
    best = None
    for k in (-1, 0, 1):
        lo, hi = b0 + k * P, b1 + k * P
        dc = abs((c0 + c1) - (lo + hi))
        if best is None or dc < best[0]:
            gap = max(0, lo - c1, c0 - hi)
            far = max(hi - c0, c1 - lo)
            best = (dc, gap, far)
    return best[1], best[2]


def test_mac_matches_image_enumeration(oracle_lib):
    """The opening test prunes exactly when the periodic cell-box gap is at
    least r_cut, and accepts exactly when S < theta * gap and the whole cell
    lies within r_cut of the whole box; distances from image enumeration."""
    p = synth.clustered_problem(6000, 1, 7, ntab=16)
    T = oracle_lib.Tree.of(p, group_size=32)
    nd = T.nodes()
    rng = np.random.default_rng(3)
    P = 1 << 20
    deep = np.nonzero(nd["level"] >= 3)[0]
    seen = set()
    for _ in range(600):
        i = int(rng.choice(deep))
        lvl = int(nd["level"][i])
        c = corner_of(lvl, nd["prefix"][i])
        S = 1 << (20 - lvl)
        lo = rng.integers(0, P - 1, 3)
        hi = np.minimum(lo + rng.integers(1, P // (8 if _ % 2 else 512), 3), P)
        gap2 = far2 = 0
        for a in range(3):
            g, f = periodic_box_distances(c[a], c[a] + S, int(lo[a]), int(hi[a]), P)
            gap2 += (2 * g) ** 2          # half key units
            far2 += (2 * f) ** 2
        for theta in (0.3, 0.5, 0.9):
            for rcut_keys in (3000.0, 30000.0, 200000.0, 400000.0):
                R2 = (2 * rcut_keys) ** 2
                d = T.mac(i, lo.astype(np.uint32), hi.astype(np.uint32), R2, theta * theta)
                if gap2 >= R2:
                    want = oracle_lib.PRUNE
                elif 4 * S * S < theta * theta * gap2 and far2 < R2:
                    want = oracle_lib.ACCEPT
                else:
                    want = oracle_lib.OPEN
                assert d == want
                seen.add(want)
    assert seen == {oracle_lib.PRUNE, oracle_lib.ACCEPT, oracle_lib.OPEN}


# --------------------------------------------------------------- forces ---
def two_body(oracle_lib, x0, x1, s0, s1, m0, m1, G, tables, grid, r_cut, eps, box=1.0, eps_ab=None):
    pos = np.array([x0, x1], dtype=np.float64).T.copy()
    X = oracle_lib.lattice(pos, box)
    s = np.array([s0, s1], np.uint8)
    m = np.array([m0, m1])
    D = G.shape[0]
    law = oracle_lib.make_law(G, tables, grid, r_cut, eps, 0.5, eps_ab=eps_ab)
    T = oracle_lib.Tree(X, s, m, D, box, 1)
    T.monopoles()
    T.groups(64)
    acc, slack, cnt, _ = T.force(law)
    accd, _ = oracle_lib.direct(X, s, m, D, box, law)
    return acc, accd, X


def wrap_diff(a, b):
    """Signed minimum-image difference of two 64-bit lattice coordinates."""
    d = (int(a) - int(b)) % (1 << 64)
    return d - (1 << 64) if d >= (1 << 63) else d


def lerp_bound(fn, ntab, r_cut, grid):
    """h^2/8 * max|f''| of the sampled variable (r or r^2), from a fine grid."""
    if grid == "r":
        u = np.linspace(0, r_cut, 200001)
        f = fn(u)
        h = r_cut / (ntab - 1)
    else:
        u = np.linspace(0, r_cut * r_cut, 200001)
        f = fn(np.sqrt(u))
        h = r_cut * r_cut / (ntab - 1)
    du = u[1] - u[0]
    f2 = np.abs(np.diff(f, 2)) / du ** 2
    return h * h / 8 * f2.max() * 1.05 + 1e-15


@pytest.mark.parametrize("grid", ["r", "r2"])
def test_two_body_closed_form(oracle_lib, grid):
    """Eq. (1) for two bodies: a_0 = G_ab m_1 f_ab(r) d / (r^2+eps^2)^(3/2),
    with the exact erfc short-range factor, a Yukawa-modified cross law and an
    asymmetric G; within the interpolation error bound of the table."""
    r_s, r_cut, eps = 0.02, 0.09, 0.003
    ntab = 1024
    laws = {
        (0, 0): lambda r: synth.newtonian_treepm_factor(r, r_s),
        (0, 1): lambda r: synth.yukawa_product_factor(r, r_s, 0.7, 0.01),
        (1, 0): lambda r: synth.yukawa_product_factor(r, r_s, -0.4, 0.02),
        (1, 1): lambda r: synth.newtonian_treepm_factor(r, r_s),
    }
    tables = np.zeros((2, 2, ntab))
    for (a, b), fn in laws.items():
        tables[a, b] = synth.sample_table(fn, ntab, r_cut, grid)
    G = np.array([[1.0, 0.6], [-1.7, 2.0]])
    m0, m1 = 0.3, 0.9
    rng = np.random.default_rng(5)
    for r in [0.1 * eps, eps, 0.011, 0.05, 0.99 * r_cut]:
        d = rng.normal(size=3)
        d *= r / np.linalg.norm(d)
        for x0 in [np.array([0.5, 0.5, 0.5]), np.array([0.999, 0.002, 0.5])]:
            x1 = np.mod(x0 + d, 1.0)
            acc, accd, X = two_body(oracle_lib, x0, x1, 0, 1, m0, m1, G, tables, grid, r_cut, eps)
            dl = np.array([wrap_diff(X[a, 1], X[a, 0]) for a in range(3)]) * 2.0 ** -64
            rl = np.linalg.norm(dl)
            k0 = G[0, 1] * m1 * laws[(0, 1)](rl) / (rl * rl + eps * eps) ** 1.5
            k1 = G[1, 0] * m0 * laws[(1, 0)](rl) / (rl * rl + eps * eps) ** 1.5
            tol0 = abs(G[0, 1]) * m1 * lerp_bound(laws[(0, 1)], ntab, r_cut, grid) * rl / (rl * rl + eps * eps) ** 1.5
            tol1 = abs(G[1, 0]) * m0 * lerp_bound(laws[(1, 0)], ntab, r_cut, grid) * rl / (rl * rl + eps * eps) ** 1.5
            assert np.allclose(acc[:, 0], k0 * dl, atol=tol0 + 1e-14 * abs(k0) * rl, rtol=0)
            assert np.allclose(acc[:, 1], -k1 * dl, atol=tol1 + 1e-14 * abs(k1) * rl, rtol=0)
            assert np.allclose(accd, acc, rtol=1e-15, atol=0)
            # direction: attraction pulls sink 0 towards source 1 when G f > 0
            assert np.dot(acc[:, 0], dl) > 0
            assert np.dot(acc[:, 1], -dl) < 0   # G_10 < 0 repels


def test_plummer_kernel_with_flat_factor(oracle_lib):
    """A table of ones leaves the bare softened kernel m d/(r^2+eps^2)^(3/2)."""
    ntab = 8
    tables = np.ones((1, 1, ntab))
    G = np.ones((1, 1))
    eps = 0.01
    for r in [0.001, 0.01, 0.03]:
        x0 = np.array([0.25, 0.25, 0.25])
        x1 = x0 + np.array([r, 0, 0])
        acc, _, X = two_body(oracle_lib, x0, x1, 0, 0, 1.0, 2.0, G, tables, "r", 0.1, eps)
        dl = wrap_diff(X[0, 1], X[0, 0]) * 2.0 ** -64
        assert math.isclose(acc[0, 0], 2.0 * dl / (dl * dl + eps * eps) ** 1.5, rel_tol=1e-14)
        assert math.isclose(acc[0, 1], -1.0 * dl / (dl * dl + eps * eps) ** 1.5, rel_tol=1e-14)
        assert acc[1, 0] == 0 and acc[2, 0] == 0


def test_per_pair_softening(oracle_lib):
    """Section 2's D^2 softenings, each a Plummer length: the sink of species
    a feels m d/(r^2 + eps_ab^2)^(3/2) from a source of species b, with an
    asymmetric eps matrix (row = sink species); a matrix of equal entries
    gives exactly the single-eps result."""
    tables = np.ones((2, 2, 8))
    G = np.ones((2, 2))
    eps_ab = np.array([[0.004, 0.011], [0.02, 0.007]])
    x0 = np.array([0.25, 0.25, 0.25])
    for r in [0.002, 0.012, 0.04]:
        x1 = x0 + np.array([r, 0, 0])
        acc, accd, X = two_body(oracle_lib, x0, x1, 0, 1, 1.0, 2.0, G, tables, "r", 0.1, 0.5, eps_ab=eps_ab)
        dl = wrap_diff(X[0, 1], X[0, 0]) * 2.0 ** -64
        assert math.isclose(acc[0, 0], 2.0 * dl / (dl * dl + eps_ab[0, 1] ** 2) ** 1.5, rel_tol=1e-14)
        assert math.isclose(acc[0, 1], -1.0 * dl / (dl * dl + eps_ab[1, 0] ** 2) ** 1.5, rel_tol=1e-14)
        assert np.allclose(accd, acc, rtol=1e-15, atol=0)
    p = synth.clustered_problem(3000, 3, 6, grid="r2", ntab=256)
    X = oracle_lib.lattice_of(p)
    T = oracle_lib.Tree(X, p.species, p.mass, p.D, p.box, p.leaf_size)
    T.monopoles()
    T.groups(64)
    one = oracle_lib.make_law(p.G, p.tables, p.grid, p.r_cut, p.eps, p.theta)
    mat = oracle_lib.make_law(p.G, p.tables, p.grid, p.r_cut, 7.0, p.theta, eps_ab=np.full((3, 3), p.eps))
    assert np.array_equal(T.force(one)[0], T.force(mat)[0])


def test_cutoff_and_tie_slack(oracle_lib):
    ntab = 16
    tables = np.ones((1, 1, ntab))
    G = np.ones((1, 1))
    r_cut = 0.1
    for r, inside in [(0.0999, True), (0.1001, False)]:
        x0 = np.array([0.25, 0.25, 0.25])
        acc, _, _ = two_body(oracle_lib, x0, x0 + [r, 0, 0], 0, 0, 1.0, 1.0, G, tables, "r", r_cut, 0.0)
        assert (acc[0, 0] != 0) == inside
    # a pair within the tie band reports its magnitude as slack
    pos = np.array([[0.25, 0.25 + r_cut * (1 - 1e-8)], [0.25, 0.25], [0.25, 0.25]])
    X = oracle_lib.lattice(pos, 1.0)
    law = oracle_lib.make_law(G, tables, "r", r_cut, 0.0, 0.5)
    T = oracle_lib.Tree(X, np.zeros(2, np.uint8), np.ones(2), 1, 1.0, 1)
    T.monopoles()
    T.groups(64)
    acc, slack, _, _ = T.force(law)
    assert math.isclose(slack[0], 1.0 / r_cut ** 2, rel_tol=1e-6)


def test_theta_to_zero_reproduces_direct_sum(oracle_lib):
    """With every node opened the walk visits each particle as its own
    monopole and regenerates the direct sum (section 2.2)."""
    p = synth.clustered_problem(5000, 3, 9, ntab=256, grid="r")
    p.theta = 1e-12
    T = oracle_lib.Tree.of(p)
    acc, slack, cnt, _ = T.force(oracle_lib.law_of(p))
    assert cnt["pn"] == 0
    accd, _ = oracle_lib.direct_of(p)
    rms = np.sqrt(np.mean(np.sum(accd ** 2, axis=0)))
    assert np.max(np.abs(acc - accd)) <= 1e-13 * rms


def test_single_species_reduction(oracle_lib):
    """D = 2 with identical laws and G is the D = 1 problem with the species
    merged (direct sum exactly; the tree is at least as accurate)."""
    p2 = synth.clustered_problem(8000, 2, 4, ntab=512, grid="r")
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, p2.r_s), 512, p2.r_cut, "r")
    p2.G = np.ones((2, 2))
    p2.tables = np.broadcast_to(t, (2, 2, 512)).copy()
    p1 = synth.Problem(**{**p2.__dict__, "D": 1, "species": np.zeros(p2.n, np.uint8),
                          "G": np.ones((1, 1)), "tables": t[None, None].copy()})
    a2, _ = oracle_lib.direct_of(p2)
    a1, _ = oracle_lib.direct_of(p1)
    rms = np.sqrt(np.mean(np.sum(a1 ** 2, axis=0)))
    assert np.max(np.abs(a1 - a2)) <= 1e-13 * rms
    errs = []
    for p, ad in ((p1, a1), (p2, a2)):
        acc, _, _, _ = oracle_lib.Tree.of(p).force(oracle_lib.law_of(p))
        nrm = np.linalg.norm(ad, axis=0)
        e = np.linalg.norm(acc - ad, axis=0)[nrm > 0] / nrm[nrm > 0]
        errs.append(np.percentile(e, 99))
    assert errs[1] <= errs[0] * 1.25 + 1e-12


def test_species_relabel_symmetry(oracle_lib):
    """Renaming species (permuting G's rows and columns and the tables with
    the ids) leaves every acceleration unchanged, tree and direct."""
    p = synth.clustered_problem(6000, 3, 8, ntab=256, grid="r2")
    sigma = np.array([2, 0, 1])
    q = synth.Problem(**{**p.__dict__})
    q.species = sigma[p.species].astype(np.uint8)
    inv = np.argsort(sigma)
    q.G = p.G[np.ix_(inv, inv)]
    q.tables = p.tables[np.ix_(inv, inv)]
    ap, _, _, _ = oracle_lib.Tree.of(p).force(oracle_lib.law_of(p))
    aq, _, _, _ = oracle_lib.Tree.of(q).force(oracle_lib.law_of(q))
    rms = np.sqrt(np.mean(np.sum(ap ** 2, axis=0)))
    assert np.max(np.abs(ap - aq)) <= 1e-12 * rms
    dp, _ = oracle_lib.direct_of(p, np.arange(0, p.n, 7, dtype=np.uint32))
    dq, _ = oracle_lib.direct_of(q, np.arange(0, p.n, 7, dtype=np.uint32))
    assert np.max(np.abs(dp - dq)) <= 1e-13 * rms


def test_pair_reciprocity_and_momentum(oracle_lib):
    """For symmetric G f the pair forces are equal and opposite (third law),
    so the direct sum conserves momentum: sum_i m_i a_i = 0."""
    p = synth.clustered_problem(6000, 3, 10, ntab=256, grid="r")
    rng = np.random.default_rng(0)
    p.mass = rng.random(p.n) + 0.5
    ad, _ = oracle_lib.direct_of(p)
    mom = (ad * p.mass).sum(axis=1)
    scale = np.abs(ad * p.mass).sum()
    assert np.all(np.abs(mom) <= 1e-13 * scale)
    # asymmetric G breaks it (so the test can fail)
    p.G = p.G.copy()
    p.G[0, 1] += 0.5
    ad2, _ = oracle_lib.direct_of(p)
    assert np.max(np.abs((ad2 * p.mass).sum(axis=1))) > 1e-6 * scale


def test_cubic_lattice_has_no_net_force(oracle_lib):
    n1 = 16
    g = (np.arange(n1) + 0.5) / n1
    pos = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).copy()
    n = pos.shape[1]
    r_s, r_cut = 0.04, 0.18
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, r_s), 512, r_cut, "r")
    law = oracle_lib.make_law(np.ones((1, 1)), t[None, None], "r", r_cut, 0.002, 0.5)
    X = oracle_lib.lattice(pos, 1.0)
    ad, _ = oracle_lib.direct(X, np.zeros(n, np.uint8), np.full(n, 1.0 / n), 1, 1.0, law)
    s = 1.0 / n1
    assert np.max(np.abs(ad)) <= 1e-12 * (1.0 / n) / s ** 2


@pytest.mark.parametrize("maker", ["yukawa_d3", "mixed_d6", "uniform"])
def test_tree_accuracy_within_paper_tolerance(oracle_lib, maker):
    """Tree versus direct sum at theta = 0.5: the 99th percentile of
    |a_tree - a_dir| / |a_dir| stays within the paper's tree tolerance."""
    alpha = paper_constant("tree_error_tolerance_alpha")
    p = {"yukawa_d3": lambda: synth.clustered_yukawa_d3(2, n=2 ** 15),
         "mixed_d6": lambda: synth.clustered_problem(2 ** 15, 6, 3),
         "uniform": lambda: synth.uniform_problem(2 ** 14, 2, 4)}[maker]()
    T = oracle_lib.Tree.of(p)
    acc, _, cnt, _ = T.force(oracle_lib.law_of(p))
    sinks = np.arange(0, p.n, 3, dtype=np.uint32)
    ad, _ = oracle_lib.direct_of(p, sinks)
    nrm = np.linalg.norm(ad, axis=0)
    keep = nrm > 0
    e = np.linalg.norm(acc[:, sinks] - ad, axis=0)[keep] / nrm[keep]
    assert np.percentile(e, 99) <= alpha


def test_counts_and_self_exclusion(oracle_lib):
    """Interaction counts: every sink meets every particle of its opened
    leaves except itself, plus one monopole per non-empty species of each
    accepted node; summed per group they give the totals."""
    p = synth.clustered_problem(4000, 2, 6, ntab=64)
    T = oracle_lib.Tree.of(p)
    law = oracle_lib.law_of(p)
    acc, _, cnt, gc = T.force(law, group_counts=True)
    assert int(gc[:, 2].sum()) == cnt["pn"] and int(gc[:, 3].sum()) == cnt["pp"]
    nd = T.nodes()
    M, _ = T.monopole_arrays()
    g = T.group_arrays()
    for k in range(0, T.n_groups, 17):
        L = T.group_list(law, k)
        kind = L >> np.uint64(32)
        node = (L & np.uint64(0xffffffff)).astype(np.int64)
        ns = int(g["count"][k])
        pp = int(nd["count"][:, node[kind == 2]].sum()) * ns - ns
        pn = int((M[:, node[kind == 1]] > 0).sum()) * ns
        assert (int(gc[k, 2]), int(gc[k, 3])) == (pn, pp)
        assert len(set(node.tolist())) == len(node)  # each node at most once


def test_counts_per_source_species(oracle_lib):
    """Particle-node interactions split by source species: one per accepted
    node whose species-b monopole is non-empty, times the group's sinks, and
    the split adds up to the total."""
    p = synth.clustered_problem(6000, 3, 8, ntab=64)
    T = oracle_lib.Tree.of(p)
    law = oracle_lib.law_of(p)
    _, _, cnt, gc = T.force(law, group_counts=True)
    assert sum(cnt["pn_species"]) == cnt["pn"]
    M, _ = T.monopole_arrays()
    g = T.group_arrays()
    want = np.zeros(p.D, np.int64)
    for k in range(T.n_groups):
        L = T.group_list(law, k)
        node = (L & np.uint64(0xffffffff)).astype(np.int64)[(L >> np.uint64(32)) == 1]
        want += (M[:, node] > 0).sum(axis=1) * int(g["count"][k])
    assert want.tolist() == cnt["pn_species"]


@pytest.mark.parametrize("rel,ties", [(2.5e-7, 2), (-2.5e-7, 2), (1.5e-6, 0), (-1.5e-6, 0)])
def test_near_tie_count(oracle_lib, rel, ties):
    """Two bodies at r = r_cut (1 + rel) along x: both see the other within
    1e-6 r_cut^2 of the cut-off (|r^2 - r_cut^2| = 2 |rel| r_cut^2 to first
    order) exactly when |rel| < 5e-7, one near tie per sink."""
    r_cut, box = 0.1, 1.0
    d = r_cut * (1.0 + rel)
    X = np.zeros((3, 2), np.uint64)
    X[0, 0] = np.uint64(1) << np.uint64(60)
    X[0, 1] = X[0, 0] + np.uint64(round(d / box * 2.0 ** 64))
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, 0.02), 256, r_cut, "r")
    law = oracle_lib.make_law(np.ones((1, 1)), t[None, None], "r", r_cut, 1e-3, 0.5)
    T = oracle_lib.Tree(X, np.zeros(2, np.uint8), np.full(2, 0.5), 1, box, 16)
    T.monopoles()
    T.groups(64)
    _, slack, cnt, _ = T.force(law)
    assert cnt["pp"] == 2 and cnt["near_ties"] == ties
    assert np.all((slack > 0) == (ties > 0))


@pytest.mark.parametrize("L", [1e-9, 1e12])
def test_length_unit_scaling(oracle_lib, L):
    """The same lattice in a box of side L, with r_s, r_cut and eps scaled
    by L and the same masses and tables (f depends on r / r_s): the tree and
    its lists are unchanged and every acceleration scales as 1 / L^2."""
    p = synth.clustered_problem(4000, 2, 11, ntab=256)
    p.lattice, p.pos = oracle_lib.lattice_of(p), None
    T1 = oracle_lib.Tree.of(p)
    a1, _, c1, _ = T1.force(oracle_lib.law_of(p))
    q = synth.clustered_problem(4000, 2, 11, ntab=256)
    q.lattice, q.pos = p.lattice, None
    q.box, q.r_s, q.r_cut, q.eps = L, p.r_s * L, p.r_cut * L, p.eps * L
    TL = oracle_lib.Tree.of(q)
    aL, _, cL, _ = TL.force(oracle_lib.law_of(q))
    assert (c1["pp"], c1["pn"]) == (cL["pp"], cL["pn"])
    rms = np.sqrt(np.mean(np.sum(a1 ** 2, axis=0)))
    assert np.max(np.abs(aL * L * L - a1)) <= 1e-12 * rms
