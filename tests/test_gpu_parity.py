"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Exact for everything integer: lattice coordinates, keys, the sort
permutation, the tree (levels, prefixes, links, per-species ranges), the
groups and every per-group interaction count. Forces per particle within
|a_gpu - a_orc| <= 1e-5 rms|a| + slack, where slack is the oracle's sum of
|term| over pairs within 1e-6 r_cut^2 of the cut-off (a pair there may fall
either side in finite precision). Masses and centres of mass within the
float64 bound of sums taken in different orders.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs, force_gate, gpu_solve

pytestmark = pytest.mark.gpu


def torch_acc(n):
    import torch
    return torch.empty((3, n), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


def full_parity(ctx, p, group_size=None, check_tree=True):
    """Run p on the GPU and compare every stage with the oracle."""
    print(f"case {p.name} n={p.n} D={p.D} grid={p.grid} B={p.leaf_size} Ng={group_size or p.group_size}",
          flush=True)
    gs = group_size or p.group_size
    acc, st, gc, tree = gpu_solve(ctx, p, group_counts=True, keep_tree=True, group_size=gs)
    try:
        T = oracle.Tree.of(p, group_size=gs)
        if check_tree:
            ex = ngr.tree_export(ctx, tree)
            nd = T.nodes()
            assert np.array_equal(ex["perm"], nd["perm"])
            assert np.array_equal(ex["keys"], nd["keys"])
            assert np.array_equal(ex["lattice"], oracle.lattice_of(p)[:, nd["perm"]])
            assert tree.n_nodes == T.n_nodes
            for k in ("level", "prefix", "parent", "first_child", "n_child", "start", "count"):
                assert np.array_equal(ex[k], nd[k]), k
            assert (st["n_nodes"], st["n_leaves"]) == (T.n_nodes, int(np.count_nonzero(nd["n_child"] == 0)))
            M, com = ngr.monopoles_export(ctx, tree)
            Mo, como = T.monopole_arrays()
            # float64 sums of N terms in different orders (bottom-up on the GPU,
            # particle by particle in the oracle) differ by at most ~N 2^-52
            cnt = nd["count"].astype(np.float64)
            assert np.all(np.abs(M - Mo) <= (cnt + 1.0) * 2.0 ** -52 * Mo)
            tol = ((cnt + 1.0) * 2.0 ** -52 + 1e-15)[:, None, :] * p.box
            has = np.broadcast_to((Mo > 0)[:, None, :], com.shape)
            assert np.all(np.abs(com - como)[has] <= np.broadcast_to(tol, com.shape)[has])
            g = ngr.groups_export(ctx, tree, gs)
            go = T.group_arrays()
            for k in go:
                assert np.array_equal(g[k], go[k]), k
        ao, so, co, gco = T.force(oracle.law_of(p), group_counts=True)
        assert (st["interactions_pp"], st["interactions_pn"]) == (co["pp"], co["pn"])
        assert st["interactions_pn_species"][:p.D] == co["pn_species"]
        assert st["near_ties"] == co["near_ties"]
        assert np.array_equal(gc, gco)
        ok, worst, rms, mx = force_gate(acc, ao, so)
        print(f"  interactions={co['pp'] + co['pn']} worst/allowed={worst:.3g} max|da|/rms={mx:.3g}", flush=True)
        assert ok, f"force gate: worst ratio {worst}"
        return acc, st
    finally:
        ngr.tree_free(ctx, tree)


@pytest.mark.parametrize("seed", range(1, 11))
def test_uniform_4096_two_species(ctx, seed):
    full_parity(ctx, synth.uniform_4096(seed))


def test_clustered_three_species_yukawa(ctx):
    full_parity(ctx, synth.clustered_yukawa_d3(2, n=2 ** 15))


def test_clustered_six_species_r2_grid(ctx):
    # D * ntab = 12288: the tables take the value-only LDS layout
    full_parity(ctx, synth.clustered_problem(2 ** 15, 6, 3))


def test_clustered_six_species_pair_tables(ctx):
    full_parity(ctx, synth.clustered_problem(2 ** 15, 6, 4, ntab=512, grid="r"))


def test_single_species(ctx):
    full_parity(ctx, synth.clustered_problem(20000, 1, 5, ntab=2048))


@pytest.mark.parametrize("B", [1, 3, 64])
def test_leaf_sizes(ctx, B):
    p = synth.clustered_problem(6000, 2, 6, ntab=256, grid="r")
    p.leaf_size = B
    full_parity(ctx, p)


@pytest.mark.parametrize("Ng", [16, 32])
def test_group_sizes(ctx, Ng):
    full_parity(ctx, synth.clustered_problem(9000, 3, 7, ntab=512), group_size=Ng)


def test_every_lane_mapping(ctx):
    """Groups of 64 sinks run with one sink per lane (49 to 64 sinks), as
    three blocks of 16 sinks over a quarter of the records each (33 to 48),
    and as two or four copies (17 to 32, at most 16). A clustered box holds
    all four kinds; every stage equals the oracle, near ties included."""
    p = synth.clustered_problem(30000, 3, 12, ntab=512)
    T = oracle.Tree.of(p)
    ns = T.group_arrays()["count"]
    kinds = [int(np.count_nonzero((ns > lo) & (ns <= hi))) for lo, hi in ((0, 16), (16, 32), (32, 48), (48, 64))]
    print(f"groups by lane mapping (<=16, 17-32, 33-48, 49-64): {kinds}")
    assert min(kinds) > 0
    full_parity(ctx, p)


def test_zero_softening(ctx):
    p = synth.uniform_problem(3001, 2, 8, ntab=512)
    p.eps = 0.0
    full_parity(ctx, p)


@pytest.mark.parametrize("n", [1, 2, 7, 65, 129])
def test_tiny_and_ragged(ctx, n):
    # few particles: groups span most of the box and need the per-pair wrap
    p = synth.uniform_problem(n, 2 if n > 1 else 1, 9 + n, ntab=64)
    p.r_s, p.r_cut, p.eps = 0.06, 0.3, 0.01
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, p.r_s), 64, p.r_cut, "r")
    p.tables = np.broadcast_to(t, (p.D, p.D, 64)).copy()
    full_parity(ctx, p)


def test_wide_groups_large_cutoff(ctx):
    p = synth.uniform_problem(300, 1, 21, ntab=128)
    p.r_cut = 0.45
    p.tables = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, 0.1), 128, p.r_cut, "r")[None, None].copy()
    full_parity(ctx, p)


def test_edges_and_coincident_particles(ctx):
    rng = np.random.default_rng(31)
    n = 2000
    pos = synth.uniform_positions(n, 1.0, rng)
    pos[:, :50] = np.nextafter(1.0, 0.0)          # just below the upper face
    pos[:, 50:100] = 0.0                           # on the lower face
    pos[:, 100:140] = pos[:, 140:180]              # coincident pairs
    p = synth.uniform_problem(n, 2, 31, ntab=256)
    p.pos = pos
    full_parity(ctx, p)


def test_masses_unequal_and_zero(ctx):
    p = synth.clustered_problem(8000, 3, 12, ntab=256)
    rng = np.random.default_rng(12)
    p.mass = rng.random(p.n) * 2.0 / p.n
    p.mass[::17] = 0.0
    full_parity(ctx, p)


def test_asymmetric_G_and_laws(ctx):
    p = synth.clustered_problem(8000, 3, 13, ntab=512)
    rng = np.random.default_rng(13)
    p.G = rng.uniform(-1, 2, (3, 3))
    p.tables = p.tables * rng.uniform(0.5, 1.5, (3, 3, 1))
    full_parity(ctx, p)


def test_box_not_unit(ctx):
    p = synth.clustered_problem(8000, 2, 14, ntab=512, box=37.5)
    full_parity(ctx, p)


def test_default_tables_from_split_scale(ctx):
    """tables == NULL: the library tabulates the Newtonian short-range factor
    from r_s; compared with the oracle using the same law tabulated here."""
    import torch
    p = synth.clustered_problem(6000, 2, 15, ntab=1024, grid="r")
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, p.r_s), 1024, p.r_cut, "r")
    p.tables = np.broadcast_to(t, (2, 2, 1024)).copy()
    p.G = np.ones((2, 2))
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **device_inputs(p))
    ngr.compute_monopoles(ctx, tree)
    acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
    ngr.tree_force(ctx, tree, G=p.G, tables=None, ntab=1024, grid="r", r_s=p.r_s, r_cut=p.r_cut, eps=p.eps,
                   theta=p.theta, acc=acc)
    ngr.tree_free(ctx, tree)
    ao, so, _, _ = oracle.Tree.of(p).force(oracle.law_of(p))
    ok, worst, _, _ = force_gate(acc.cpu().numpy(), ao, so)
    assert ok, worst


def test_repeat_is_bitwise_identical(ctx):
    p = synth.clustered_problem(20000, 3, 16, ntab=512)
    a1, _, _, _ = gpu_solve(ctx, p)
    a2, _, _, _ = gpu_solve(ctx, p)
    assert np.array_equal(a1, a2)


def test_empty_input(ctx):
    import torch
    z = torch.zeros(0, dtype=torch.uint8, device="cuda")
    tree = ngr.tree_build(ctx, D=2, box=1.0, species=z, mass=torch.zeros(0, dtype=torch.float64, device="cuda"),
                          pos=torch.zeros((3, 0), dtype=torch.float64, device="cuda"))
    ngr.compute_monopoles(ctx, tree)
    acc = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    st = ngr.tree_force(ctx, tree, G=np.ones((2, 2)), tables=np.ones((2, 2, 8)), grid="r", r_cut=0.1, eps=0.01,
                        theta=0.5, acc=acc)
    assert st["interactions_pp"] == 0 and st["interactions_pn"] == 0 and st["n_groups"] == 0
    ngr.tree_free(ctx, tree)


def _status(fn):
    try:
        fn()
    except ngr.NgravsError as e:
        return e.status
    return ngr.OK


def test_errors_are_reported(ctx):
    import torch
    p = synth.uniform_problem(500, 2, 17, ntab=64)
    t = device_inputs(p)
    bad_species = t["species"].clone()
    bad_species[3] = 2
    assert _status(lambda: ngr.tree_build(ctx, D=2, box=1.0, species=bad_species, mass=t["mass"], pos=t["pos"])) == ngr.EINVAL
    bad_mass = t["mass"].clone()
    bad_mass[7] = -1.0
    assert _status(lambda: ngr.tree_build(ctx, D=2, box=1.0, species=t["species"], mass=bad_mass, pos=t["pos"])) == ngr.EINVAL
    bad_pos = t["pos"].clone()
    bad_pos[1, 9] = float("nan")
    assert _status(lambda: ngr.tree_build(ctx, D=2, box=1.0, species=t["species"], mass=t["mass"], pos=bad_pos)) == ngr.EINVAL
    assert _status(lambda: ngr.tree_build(ctx, D=7, box=1.0, species=t["species"], mass=t["mass"], pos=t["pos"])) == ngr.EINVAL
    assert _status(lambda: ngr.tree_build(ctx, D=2, box=0.0, species=t["species"], mass=t["mass"], pos=t["pos"])) == ngr.EINVAL
    assert _status(lambda: ngr.tree_build(ctx, D=2, box=1.0, species=t["species"], mass=t["mass"], pos=t["pos"],
                                          leaf_size=65)) == ngr.EINVAL
    tree = ngr.tree_build(ctx, D=2, box=1.0, species=t["species"], mass=t["mass"], pos=t["pos"])
    acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
    kw = dict(G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta, acc=acc)
    assert _status(lambda: ngr.tree_force(ctx, tree, **kw)) == ngr.ESTATE
    ngr.compute_monopoles(ctx, tree)
    for change in (dict(r_cut=0.5), dict(r_cut=-1.0), dict(eps=-0.1), dict(theta=0.0), dict(group_size=48),
                   dict(grid=7), dict(G=np.full((2, 2), np.nan)), dict(tables=np.full((2, 2, 64), np.inf)),
                   dict(tables=np.ones((2, 2, 1))), dict(tables=np.ones((2, 2, 7000)))):
        assert _status(lambda: ngr.tree_force(ctx, tree, **{**kw, **change})) == ngr.EINVAL, change
    assert _status(lambda: ngr.tree_force(ctx, tree, **kw)) == ngr.OK
    ngr.tree_free(ctx, tree)


def test_full_parity_at_2_21(ctx, capsys):
    """The three-species clustered box at full size, against the oracle over
    every group: exact counts and the force gate with the oracle's rms."""
    full_box_parity(ctx, capsys, synth.clustered_yukawa_d3(2), chunks=2)


@pytest.mark.slow
@pytest.mark.parametrize("halos", [2000, None], ids=["H2000", "H16000"])
def test_full_parity_at_2_24_six_species(ctx, capsys, halos):
    """The 2^24, six-species workload in the benchmark's launch
    configuration, against the oracle over every group: exact tree, groups,
    per-group and total counts (so the benchmark's interaction count is the
    oracle's), and the per-particle force gate with the oracle's own rms.
    2000 halos is the benchmark box (the generator of the 2^21 box at 2^24);
    halos=None scales the halo count with n (16000)."""
    p = synth.clustered_d6(3, halos=halos)
    full_box_parity(ctx, capsys, p, chunks=8)


def full_box_parity(ctx, capsys, p, chunks):
    def say(msg):
        with capsys.disabled():
            print(msg, flush=True)
    say(f"case {p.name} n={p.n} D={p.D} (full oracle)")
    acc, st, gc, tree = gpu_solve(ctx, p, group_counts=True, keep_tree=True)
    try:
        # the benchmark's instantiation (no counts) gives the same accelerations bit for bit
        plain = torch_acc(p.n)
        ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta,
                       group_size=p.group_size, acc=plain)
        assert np.array_equal(plain.cpu().numpy(), acc)
        del plain
        ex = ngr.tree_export(ctx, tree)
        say("  gpu done")
        T = oracle.Tree.of(p)
        say(f"  oracle tree done: {T.n_nodes} nodes, {T.n_groups} groups")
        nd = T.nodes()
        assert np.array_equal(ex["perm"], nd["perm"]) and np.array_equal(ex["keys"], nd["keys"])
        assert tree.n_nodes == T.n_nodes
        for k in ("level", "prefix", "first_child", "n_child", "start", "count"):
            assert np.array_equal(ex[k], nd[k]), k
        go = T.group_arrays()
        g = ngr.groups_export(ctx, tree, p.group_size)
        for k in go:
            assert np.array_equal(g[k], go[k]), k
    finally:
        ngr.tree_free(ctx, tree)
    law = oracle.law_of(p)
    ao = np.full((3, p.n), np.nan)
    so = np.full(p.n, np.nan)
    pp = pn = ties = 0
    pnb = np.zeros(p.D, np.int64)
    parts = np.array_split(np.arange(T.n_groups, dtype=np.uint32), chunks)
    for c, sel in enumerate(parts):
        a, s, co, gco = T.force(law, groups=sel, group_counts=True)
        assert np.array_equal(gc[sel], gco)
        sinks = np.concatenate([np.arange(go["start"][k], go["start"][k] + go["count"][k]) for k in sel])
        idx = nd["perm"][sinks]
        ao[:, idx] = a[:, idx]
        so[idx] = s[idx]
        pp += co["pp"]
        pn += co["pn"]
        ties += co["near_ties"]
        pnb += np.array(co["pn_species"], np.int64)
        say(f"  oracle chunk {c + 1}/{chunks}: {co['pp'] + co['pn']} interactions")
    assert not np.isnan(ao).any()
    assert (st["interactions_pp"], st["interactions_pn"]) == (pp, pn)
    assert st["interactions_pn_species"][:p.D] == pnb.tolist()
    assert st["near_ties"] == ties
    ok, worst, rms, mx = force_gate(acc, ao, so)
    say(f"  interactions={pp + pn} worst/allowed={worst:.3g} max|da|/rms={mx:.3g}")
    assert ok, f"force gate: worst ratio {worst}"


@pytest.mark.parametrize("L", [1e-9, 1e12])
def test_length_units(ctx, L):
    """Boxes far from unit size: the walk works in units of the box, so the
    float32 kernel factor has the same range (exact counts, force gate)."""
    p = synth.clustered_problem(20000, 3, 41, ntab=512)
    p.lattice, p.pos = oracle.lattice_of(p), None
    p.box, p.r_s, p.r_cut, p.eps = L, p.r_s * L, p.r_cut * L, p.eps * L
    p.name += f"-box{L:g}"
    full_parity(ctx, p)


def test_softening_below_range_is_refused(ctx):
    import torch
    p = synth.uniform_4096(1)
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **t)
    ngr.compute_monopoles(ctx, tree)
    acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
    kw = dict(G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, theta=p.theta, acc=acc)
    assert _status(lambda: ngr.tree_force(ctx, tree, eps=1e-14, **kw)) == ngr.EINVAL
    assert _status(lambda: ngr.tree_force(ctx, tree, eps=0.0, eps_ab=np.full((2, 2), 1e-14), **kw)) == ngr.EINVAL
    assert _status(lambda: ngr.tree_force(ctx, tree, eps=1e-12, **kw)) == ngr.OK
    ngr.tree_free(ctx, tree)
