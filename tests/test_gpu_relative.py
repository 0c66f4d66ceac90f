"""The relative opening test (section 2.2) on the HIP path against the
oracle: exact interaction counts and per-group counts, forces within the
gate, previous accelerations from a first geometric force as a simulation
would have them; tolerances from loose to tight, every group-size path,
the accumulator laws and per-pair softening under it, a non-periodic box,
a batched box, and the error paths."""
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


def with_old_acc(ctx, p, alpha):
    """p with the relative test and |a| of a first (geometric) GPU force."""
    a0 = gpu_solve(ctx, p)[0]
    return dataclasses.replace(p, relative={"alpha": alpha, "old_acc": np.linalg.norm(a0, axis=0)})


def parity(ctx, p, gs):
    print(f"case {p.name} Ng={gs} alpha={p.relative['alpha']}", flush=True)
    acc, st, gc, _ = gpu_solve(ctx, p, group_counts=True, group_size=gs)
    ao, so, co, gco = oracle.Tree.of(p, group_size=gs).force(oracle.law_of(p), group_counts=True)
    print(f"  pp={co['pp']} pn={co['pn']}", flush=True)
    assert (st["interactions_pp"], st["interactions_pn"]) == (co["pp"], co["pn"])
    assert np.array_equal(gc, gco)
    ok, worst, _, _ = force_gate(acc, ao, so)
    assert ok, worst
    return co


@pytest.mark.parametrize("alpha", [0.5, 0.02, 0.0025])
@pytest.mark.parametrize("gs", [64, 32, 16])
def test_clustered(ctx, alpha, gs):
    p = synth.clustered_problem(15000, 3, 50, ntab=512)
    co = parity(ctx, with_old_acc(ctx, p, alpha), gs)
    if alpha == 0.5:
        assert co["pn"] > 0


def test_isolated_box(ctx):
    """A non-periodic box with full-range laws, where the relative test
    accepts many distant nodes."""
    p = synth.isolated_problem(12000, 2, 51, ntab=1024)
    co = parity(ctx, with_old_acc(ctx, p, 0.005), 32)
    assert co["pn"] > 0


def test_with_accumulator_and_softening(ctx):
    p = synth.accumulator_problem(10000, 52, D=3, cored=(1,), ntab=512)
    p = dataclasses.replace(p, eps_ab=p.eps * np.array([[1, 2, 0.5], [3, 1, 1], [1, 0.2, 1.0]]))
    parity(ctx, with_old_acc(ctx, p, 0.05), 32)


def test_zero_old_acc_opens_everything_within_r_cut(ctx):
    p = synth.clustered_problem(6000, 2, 53, ntab=256)
    q = dataclasses.replace(p, relative={"alpha": 0.01, "old_acc": np.zeros(p.n)})
    co = parity(ctx, q, 64)
    assert co["pn"] == 0


def test_batched_box(ctx):
    import torch
    p = with_old_acc(ctx, synth.clustered_problem(7000, 2, 54, ntab=256), 0.05)
    acc = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
    old = torch.from_numpy(p.relative["old_acc"]).cuda()
    box = ngr.BatchBox(D=p.D, box=p.box, acc=acc, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                       theta=p.theta, leaf_size=p.leaf_size, group_size=32,
                       relative={"alpha": 0.05, "old_acc": old}, **device_inputs(p))
    q = synth.clustered_problem(5000, 3, 55, ntab=256)
    acc2 = torch.full((3, q.n), float("nan"), dtype=torch.float64, device="cuda")
    box2 = ngr.BatchBox(D=q.D, box=q.box, acc=acc2, G=q.G, tables=q.tables, grid=q.grid, r_cut=q.r_cut, eps=q.eps,
                        theta=q.theta, leaf_size=q.leaf_size, group_size=32, **device_inputs(q))
    ngr.batch_build_force(ctx, [box2, box])
    assert np.array_equal(acc.cpu().numpy(), gpu_solve(ctx, p, group_size=32)[0])
    assert np.array_equal(acc2.cpu().numpy(), gpu_solve(ctx, q, group_size=32)[0])


def test_errors(ctx):
    p = synth.clustered_problem(1000, 2, 56, ntab=64)
    for rel in ({"alpha": 0.0, "old_acc": np.ones(p.n)}, {"alpha": float("nan"), "old_acc": np.ones(p.n)}):
        with pytest.raises(ngr.NgravsError):
            gpu_solve(ctx, dataclasses.replace(p, relative=rel))
