"""Pure-tree periodic mode with lattice corrections (section 2.3) on the HIP
path against the oracle with the same tables: exact interaction counts and
per-group counts, forces within the gate; both table grids, eps = 0, the
relative opening test and per-pair softening under it; boxes with and
without corrections in one batch (each against the oracle, since the batch
then runs every box's groups with the per-pair wrap); refused combinations."""
import dataclasses

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


def check(acc, st, p, gs, gc=None):
    ao, so, co, gco = oracle.Tree.of(p, group_size=gs).force(oracle.law_of(p), group_counts=True)
    assert (st["interactions_pp"], st["interactions_pn"]) == (co["pp"], co["pn"]), p.name
    if gc is not None:
        assert np.array_equal(gc, gco)
    ok, worst, _, mx = force_gate(acc, ao, so)
    print(f"  {p.name}: worst/allowed={worst:.3g} max|da|/rms={mx:.3g} pp={co['pp']} pn={co['pn']}", flush=True)
    assert ok
    return co


@pytest.mark.parametrize("n,D,EN,gs", [(20000, 2, 32, 64), (8000, 3, 16, 32), (4000, 1, 64, 16)])
def test_parity(ctx, n, D, EN, gs):
    p = synth.periodic_tree_problem(n, D, 60 + D, EN=EN, ntab=1024)
    print(f"case {p.name} EN={EN} Ng={gs}", flush=True)
    acc, st, gc, _ = gpu_solve(ctx, p, group_counts=True, group_size=gs)
    co = check(acc, st, p, gs, gc)
    assert co["pn"] > 0


def test_r_grid_eps0_relative_softening(ctx):
    p = synth.periodic_tree_problem(6000, 2, 64, EN=16, ntab=512)
    r = dataclasses.replace(p, grid=synth.GRID_R, eps=0.0)
    check(*gpu_solve(ctx, r)[:2], r, r.group_size)
    a0 = gpu_solve(ctx, p)[0]
    q = dataclasses.replace(p, relative={"alpha": 0.01, "old_acc": np.linalg.norm(a0, axis=0)},
                            eps_ab=p.eps * np.array([[1.0, 2.0], [0.5, 1.0]]))
    check(*gpu_solve(ctx, q, group_size=32)[:2], q, 32)


def test_batch_mixed(ctx):
    import torch
    probs = [synth.periodic_tree_problem(5000, 2, 65, EN=16, ntab=256),
             synth.clustered_problem(6000, 2, 66, ntab=256)]
    boxes, accs = [], []
    for p in probs:
        acc = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
        boxes.append(ngr.BatchBox(D=p.D, box=p.box, acc=acc, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut,
                                  eps=p.eps, theta=p.theta, leaf_size=p.leaf_size, group_size=32,
                                  lattice_corr=p.lattice_corr, **device_inputs(p)))
        accs.append(acc)
    _, pb = ngr.batch_build_force(ctx, boxes, per_box=True)
    for p, acc, st in zip(probs, accs, pb):
        check(acc.cpu().numpy(), st, p, 32)


def test_refusals(ctx):
    p = synth.periodic_tree_problem(1000, 2, 67, EN=8, ntab=64)
    with pytest.raises(ngr.NgravsError, match="sqrt"):
        gpu_solve(ctx, dataclasses.replace(p, r_cut=0.45))
    acc = synth.accumulator_problem(1000, 68, ntab=64)
    with pytest.raises(ngr.NgravsError, match="table laws"):
        gpu_solve(ctx, dataclasses.replace(acc, lattice_corr=p.lattice_corr, r_cut=0.9))
    iso = synth.isolated_problem(1000, 2, 69, ntab=64)
    with pytest.raises(ngr.NgravsError, match="periodic"):
        gpu_solve(ctx, dataclasses.replace(iso, lattice_corr=p.lattice_corr, r_cut=1.9))
    bad = p.lattice_corr.copy()
    bad[0, 1, 2, 3, 4, 1] = float("nan")
    with pytest.raises(ngr.NgravsError, match="not finite"):
        gpu_solve(ctx, dataclasses.replace(p, lattice_corr=bad))
