"""Non-periodic boxes (section 2: isolated runs use the tree alone) on the
HIP path against the oracle on the same padded lattice: bit-exact lattice and
tree, exact counts, the force gate, full-range laws; two bodies with no
softening, far apart and 1e-14 apart; a non-periodic box in a batch with a
periodic one; positions outside the box, lattice input and a PM force on such
a tree are refused."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs, force_gate, gpu_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,D,grid,gs", [(20000, 3, synth.GRID_R2, 64), (12000, 2, synth.GRID_R, 32),
                                         (3000, 6, synth.GRID_R2, 16)])
def test_parity(ctx, n, D, grid, gs):
    p = synth.isolated_problem(n, D, 10 + D, grid=grid, ntab=1024)
    print(f"case {p.name} grid={grid} Ng={gs}", flush=True)
    acc, st, gc, tree = gpu_solve(ctx, p, group_counts=True, keep_tree=True, group_size=gs)
    try:
        T = oracle.Tree.of(p, group_size=gs)
        ex = ngr.tree_export(ctx, tree)
        nd = T.nodes()
        assert np.array_equal(ex["lattice"], oracle.lattice_of(p)[:, nd["perm"]])
        for k in ("perm", "level", "prefix", "first_child", "start", "count"):
            assert np.array_equal(ex[k], nd[k]), k
    finally:
        ngr.tree_free(ctx, tree)
    ao, so, co, gco = T.force(oracle.law_of(p), group_counts=True)
    assert (st["interactions_pp"], st["interactions_pn"]) == (co["pp"], co["pn"])
    assert np.array_equal(gc, gco)
    ok, worst, _, mx = force_gate(acc, ao, so)
    print(f"  worst/allowed={worst:.3g} max|da|/rms={mx:.3g}", flush=True)
    assert ok


def test_no_images(ctx):
    """Two bodies near opposite faces attract across the box, not through
    the face (a periodic box would pull them the other way)."""
    import torch
    pos = np.array([[0.02, 0.5, 0.5], [0.97, 0.5, 0.5]]).T.copy()
    p = synth.Problem(name="two", n=2, D=1, box=1.0, species=np.zeros(2, np.uint8), mass=np.ones(2),
                      G=np.ones((1, 1)), tables=np.ones((1, 1, 16)), grid=synth.GRID_R, r_s=0.0, r_cut=1.75,
                      eps=0.0, theta=0.5, pos=pos, periodic=False)
    acc = gpu_solve(ctx, p)[0]
    d = 0.95
    # eps = 0: the pair's kernel factor is the float64-refined one (~1e-13);
    # the image through the face would give -1 / 0.05^2
    assert acc[0, 0] == pytest.approx(1 / d ** 2, rel=1e-12) and acc[0, 1] == pytest.approx(-1 / d ** 2, rel=1e-12)


def test_unsoftened_close_pair(ctx):
    """Without softening two bodies 1e-14 apart attract with 1/d^2 ~ 1e28:
    their (r^2)^(-3/2) ~ 1e42 is beyond float32, and the unsoftened kernel
    takes it in float64 (d from the lattice the tree quantises to)."""
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + 1e-14, 0.5, 0.5]]).T.copy()
    p = synth.Problem(name="close-two", n=2, D=1, box=1.0, species=np.zeros(2, np.uint8), mass=np.ones(2),
                      G=np.ones((1, 1)), tables=np.ones((1, 1, 16)), grid=synth.GRID_R, r_s=0.0, r_cut=1.75,
                      eps=0.0, theta=0.5, pos=pos, periodic=False)
    X = oracle.lattice_of(p).astype(np.float64)
    d = (X[0, 1] - X[0, 0]) * oracle.box_of(p) * 2.0 ** -64
    assert 5e-15 < d < 2e-14
    acc = gpu_solve(ctx, p)[0]
    assert np.all(np.isfinite(acc))
    assert acc[0, 0] == pytest.approx(1 / d ** 2, rel=1e-12) and acc[0, 1] == pytest.approx(-1 / d ** 2, rel=1e-12)


def test_batch_with_periodic_box(ctx):
    import torch
    probs = [synth.isolated_problem(6000, 2, 20, ntab=256), synth.clustered_problem(5000, 2, 21, ntab=256)]
    boxes, accs = [], []
    for p in probs:
        acc = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
        b = ngr.BatchBox(D=p.D, box=p.box, acc=acc, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                         theta=p.theta, leaf_size=p.leaf_size, group_size=32, **device_inputs(p))
        b.tree.non_periodic = 0 if p.periodic else 1
        boxes.append(b)
        accs.append(acc)
    ngr.batch_build_force(ctx, boxes)
    for p, acc in zip(probs, accs):
        assert np.array_equal(acc.cpu().numpy(), gpu_solve(ctx, p, group_size=32)[0]), p.name


def test_refusals(ctx):
    import torch
    p = synth.isolated_problem(2000, 2, 22, ntab=64)
    bad = p.pos.copy()
    bad[1, 7] = 1.0                                     # = box: outside [0, box)
    with pytest.raises(ngr.NgravsError, match="outside"):
        gpu_solve(ctx, dataclasses.replace(p, pos=bad))
    bad[1, 7] = -1e-9
    with pytest.raises(ngr.NgravsError, match="outside"):
        gpu_solve(ctx, dataclasses.replace(p, pos=bad))
    with pytest.raises(ngr.NgravsError, match="lattice"):
        gpu_solve(ctx, dataclasses.replace(p, pos=None, lattice=oracle.lattice(p.pos, p.box)))
    tree = ngr.tree_build(ctx, D=2, box=p.box, leaf_size=16, periodic=False, **device_inputs(p))
    try:
        q = 3 * 8 * 8 + 1
        plan = ngr.PM(ctx, N=16, D=2, box=p.box, r_s=0.1, G=np.ones((2, 2)), phibar=np.full((2, 2, q), -4 * math.pi))
        acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        with pytest.raises(ngr.NgravsError, match="non-periodic"):
            plan.force(tree, acc)
        plan.close()
    finally:
        ngr.tree_free(ctx, tree)
