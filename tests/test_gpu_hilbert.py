"""The Peano-Hilbert key order (section 2.4) on the GPU against the oracle:
keys, sort permutation and every node record bit-exact, the same node cells
as the Morton tree, groups and per-group counts exact, forces within the
gate; a Hilbert box batched beside a Morton box equals its single call."""
import numpy as np
import pytest

import oracle
import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs, gpu_solve
from test_gpu_parity import full_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


def hilbert(p):
    p.key_order = "hilbert"
    p.name += "-hilbert"
    return p


@pytest.mark.parametrize("maker", [
    lambda: synth.uniform_4096(3),
    lambda: synth.clustered_yukawa_d3(2, n=2 ** 15),
    lambda: synth.clustered_problem(2 ** 15, 6, 3),
    lambda: synth.clustered_problem(9000, 1, 5, ntab=512, grid="r"),
], ids=["uniform4096", "yukawa-d3", "mixed-d6", "d1-r"])
def test_parity(ctx, maker):
    full_parity(ctx, hilbert(maker()))


@pytest.mark.parametrize("B,Ng", [(1, 64), (4, 16), (16, 32)])
def test_leaf_and_group_sizes(ctx, B, Ng):
    full_parity(ctx, hilbert(synth.clustered_problem(6000, 3, 7, ntab=512, leaf_size=B)), group_size=Ng)


def test_cells_match_the_morton_tree(ctx):
    """Same (level, cell corner, per-species counts, child count) set under
    both curves; prefixes differ."""
    p = synth.clustered_problem(20000, 3, 8, ntab=256)
    sets = {}
    for order in ("morton", "hilbert"):
        p.key_order = order
        t = device_inputs(p)
        tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, key_order=order, **t)
        ex = ngr.tree_export(ctx, tree)
        ngr.tree_free(ctx, tree)
        lat = oracle.lattice_of(p)[:, ex["perm"]] >> np.uint64(44)
        rows = set()
        for i in range(len(ex["level"])):
            l = int(ex["level"][i])
            j = next(int(ex["start"][b, i]) for b in range(p.D) if ex["count"][b, i])
            rows.add((l, tuple(int(v) >> (20 - l) for v in lat[:, j]),
                      tuple(int(ex["count"][b, i]) for b in range(p.D)), int(ex["n_child"][i])))
        sets[order] = rows
    assert sets["morton"] == sets["hilbert"]


def test_non_periodic_box(ctx):
    full_parity(ctx, hilbert(synth.isolated_problem(6000, 2, 4)))


def test_batch_mixes_curves(ctx):
    import torch
    probs = [synth.clustered_problem(7000, 2, 31, ntab=256), hilbert(synth.clustered_problem(9000, 3, 32, ntab=256))]
    singles = [gpu_solve(ctx, q, group_counts=False)[0] for q in probs]
    boxes, accs = [], []
    for q in probs:
        t = device_inputs(q)
        a = torch.empty((3, q.n), dtype=torch.float64, device="cuda")
        accs.append(a)
        boxes.append(ngr.BatchBox(D=q.D, box=q.box, acc=a, G=q.G, tables=q.tables, grid=q.grid, r_cut=q.r_cut,
                                  eps=q.eps, theta=q.theta, leaf_size=q.leaf_size, group_size=q.group_size,
                                  key_order=q.key_order, **t))
    ngr.batch_build_force(ctx, boxes)
    for a, s in zip(accs, singles):
        assert np.array_equal(a.cpu().numpy(), s)


def test_bad_key_order(ctx):
    p = synth.clustered_problem(500, 1, 33, ntab=64)
    t = device_inputs(p)
    part = ngr.Particles(p.n, p.D, p.box, None, None, ngr._dev(t["species"]), ngr._dev(t["mass"]))
    part.pos = ngr._dev(t["pos"])
    import ctypes as C
    tp = ngr.TreeParams(16, 0, 2)
    h = C.c_void_p()
    assert ngr.lib().ngr_tree_build(ctx.handle, C.byref(part), C.byref(tp), C.byref(h)) == ngr.EINVAL
