"""Pins of the oracle's Peano-Hilbert order (section 2.4: the particles are
sorted along a Peano-Hilbert curve after the type sort), against the
properties that make a curve a Hilbert curve, checked by brute force:

  - a bijection between the 8^k first indices and the cube [0, 2^k)^3;
  - continuity: consecutive points are face neighbours (one coordinate
    changes by one) at every level, including across the boundaries of the
    nested sub-cubes;
  - nesting: the points of an aligned cube of side 2^(20-l) share the top 3l
    index bits, so each tree node is one contiguous key range;
  - encode and decode are inverse on the whole 20-bit lattice.

A Morton order passes the bijection and nesting checks but fails continuity,
and so would a Hilbert transcription with a wrong sign, axis or Gray step.
Then the tree built on Hilbert keys: the same cells as the Morton tree."""
import numpy as np
import pytest

import synth


def decode_all(oracle_lib, hs):
    return np.array([oracle_lib.hilbert_decode(int(h)) for h in hs], dtype=np.int64)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_first_cube_is_a_continuous_bijection(oracle_lib, k):
    pts = decode_all(oracle_lib, range(8 ** k))
    assert pts.min() >= 0 and pts.max() < 2 ** k                      # inside the cube
    assert len({tuple(p) for p in pts}) == 8 ** k                     # every cell once
    step = np.abs(np.diff(pts, axis=0))
    assert np.all(step.sum(axis=1) == 1)                              # unit face steps


@pytest.mark.parametrize("k", [1, 2, 3])
def test_coarse_levels_are_continuous(oracle_lib, k):
    """The cells of level k visited in index order (index q << 3(20-k)) form
    a Hamiltonian path of face neighbours on the 2^k grid."""
    sh = 3 * (20 - k)
    cells = decode_all(oracle_lib, [q << sh for q in range(8 ** k)]) >> (20 - k)
    assert len({tuple(c) for c in cells}) == 8 ** k
    assert np.all(np.abs(np.diff(cells, axis=0)).sum(axis=1) == 1)


def test_continuity_at_random_places(oracle_lib):
    rng = np.random.default_rng(5)
    hs = rng.integers(0, 2 ** 60 - 1, size=3000, dtype=np.uint64)
    a = decode_all(oracle_lib, hs)
    b = decode_all(oracle_lib, hs + np.uint64(1))
    assert np.all(np.abs(a - b).sum(axis=1) == 1)


def test_aligned_cubes_share_a_prefix(oracle_lib):
    rng = np.random.default_rng(6)
    for _ in range(300):
        l = int(rng.integers(1, 20))
        side = 1 << (20 - l)
        corner = (rng.integers(0, 1 << l, size=3) << (20 - l))
        pts = corner + rng.integers(0, side, size=(8, 3))
        pre = {oracle_lib.hilbert(*map(int, p)) >> (3 * (20 - l)) for p in pts}
        assert len(pre) == 1


def test_round_trip(oracle_lib):
    rng = np.random.default_rng(7)
    for h in rng.integers(0, 2 ** 60, size=2000, dtype=np.uint64):
        assert oracle_lib.hilbert(*oracle_lib.hilbert_decode(int(h))) == int(h)
    for p in rng.integers(0, 2 ** 20, size=(2000, 3)):
        assert oracle_lib.hilbert_decode(oracle_lib.hilbert(*map(int, p))) == tuple(map(int, p))


def test_morton_fails_continuity(oracle_lib):
    """The continuity check separates the curves (guards the test itself)."""
    m = [oracle_lib.morton(*oracle_lib.hilbert_decode(h)) for h in range(64)]
    inv = {v: i for i, v in enumerate(m)}
    pts = np.array([oracle_lib.hilbert_decode(h) for h in sorted(range(64), key=lambda h: m[h])])
    assert len(inv) == 64 and not np.all(np.abs(np.diff(pts, axis=0)).sum(axis=1) == 1)


@pytest.mark.parametrize("B", [1, 4, 16])
def test_hilbert_tree_has_the_morton_cells(oracle_lib, B):
    """The curve orders children and particles only: the node set (level and
    cell), per-species counts and leaf rule are those of the Morton tree; each
    node's particles are one key range of its prefix; groups partition the
    sinks as before."""
    p = synth.clustered_problem(3000, 3, 9, ntab=64, leaf_size=B)
    X = oracle_lib.lattice_of(p)
    cells = {}
    for order in ("morton", "hilbert"):
        T = oracle_lib.Tree(X, p.species, p.mass, p.D, p.box, B, order)
        nd = T.nodes()
        K = oracle_lib.keys(X, p.species, order)
        assert np.array_equal(nd["keys"], K[nd["perm"]])
        assert np.all(np.diff(nd["keys"].astype(object)) >= 0)
        lvl = nd["level"].astype(np.int64)
        # each node's particles of every species lie inside its key range
        for i in range(T.n_nodes):
            sh = 3 * (20 - int(lvl[i]))
            for b in range(p.D):
                s0, c = int(nd["start"][b, i]), int(nd["count"][b, i])
                if c:
                    kk = nd["keys"][s0:s0 + c] & np.uint64(2 ** 60 - 1)
                    assert np.all((kk >> np.uint64(sh)) == np.uint64(int(nd["prefix"][i])))
        # the node's cell from its particles' lattice coordinates
        pos = X[:, nd["perm"]] >> np.uint64(44)
        key = set()
        for i in range(T.n_nodes):
            sh = 20 - int(lvl[i])
            j = next(int(nd["start"][b, i]) for b in range(p.D) if nd["count"][b, i])
            corner = tuple(int(v) >> sh for v in pos[:, j])
            counts = tuple(int(nd["count"][b, i]) for b in range(p.D))
            key.add((int(lvl[i]), corner, counts, int(nd["n_child"][i])))
        cells[order] = key
        T.monopoles()
        ng = T.groups(64)
        g = T.group_arrays()
        assert int(g["count"].sum()) == p.n and np.all(g["count"] <= 64)
    assert cells["morton"] == cells["hilbert"]


def test_hilbert_tree_force_limits(oracle_lib):
    """With every node opened (theta -> 0) the Hilbert tree's force is the
    direct sum, so the decoded cells the opening test uses are right; at
    theta = 0.5 its error stays within the tree tolerance."""
    p = synth.clustered_problem(5000, 3, 10, ntab=256)
    p.key_order = "hilbert"
    ad, _ = oracle_lib.direct_of(p)
    rms = np.sqrt(np.mean(np.sum(ad ** 2, axis=0)))
    p.theta = 1e-12
    T = oracle_lib.Tree.of(p)
    at, _, _, _ = T.force(oracle_lib.law_of(p))
    assert np.max(np.linalg.norm(at - ad, axis=0)) <= 1e-13 * rms
    p.theta = 0.5
    T = oracle_lib.Tree.of(p)
    at, _, _, _ = T.force(oracle_lib.law_of(p))
    nrm = np.linalg.norm(ad, axis=0)
    keep = nrm > 0
    assert np.percentile(np.linalg.norm(at - ad, axis=0)[keep] / nrm[keep], 99) <= 0.005
