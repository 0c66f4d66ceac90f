"""Per-pair Plummer softening (section 2's D^2 softening lengths) on the HIP
path against the oracle: exact counts, the force gate, an asymmetric matrix
on both table grids and every group-size path, zero entries (the coincident
guard), the accumulator laws' uncored pairs, a batched box, bad input."""
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


def eps_matrix(p, seed, zero=False):
    rng = np.random.default_rng(seed)
    e = p.eps * rng.uniform(0.2, 5.0, (p.D, p.D))
    if zero:
        e[0, p.D - 1] = 0.0
    return e


def parity(ctx, p, gs):
    print(f"case {p.name} n={p.n} D={p.D} grid={p.grid} Ng={gs} eps_ab={np.round(p.eps_ab / p.eps, 2).tolist()}",
          flush=True)
    acc, st, gc, _ = gpu_solve(ctx, p, group_counts=True, group_size=gs)
    ao, so, co, gco = oracle.Tree.of(p, group_size=gs).force(oracle.law_of(p), group_counts=True)
    assert (st["interactions_pp"], st["interactions_pn"]) == (co["pp"], co["pn"])
    assert np.array_equal(gc, gco)
    ok, worst, _, mx = force_gate(acc, ao, so)
    print(f"  worst/allowed={worst:.3g} max|da|/rms={mx:.3g}", flush=True)
    assert ok
    return acc


@pytest.mark.parametrize("grid", [synth.GRID_R, synth.GRID_R2])
@pytest.mark.parametrize("gs", [64, 32, 16])
def test_asymmetric_matrix(ctx, grid, gs):
    p = synth.clustered_problem(15000, 3, 40, grid=grid, ntab=512)
    parity(ctx, dataclasses.replace(p, eps_ab=eps_matrix(p, 1)), gs)


def test_zero_entries_and_wrap(ctx):
    p = synth.uniform_problem(400, 2, 41, grid=synth.GRID_R2)
    parity(ctx, dataclasses.replace(p, eps_ab=eps_matrix(p, 2, zero=True)), 64)
    p = synth.clustered_problem(8000, 4, 42, grid=synth.GRID_R2, ntab=256)
    parity(ctx, dataclasses.replace(p, eps_ab=eps_matrix(p, 3, zero=True)), 32)


def test_matrix_changes_the_force(ctx):
    p = synth.clustered_problem(8000, 2, 43, grid=synth.GRID_R2, ntab=256)
    a1 = gpu_solve(ctx, p)[0]
    a2 = gpu_solve(ctx, dataclasses.replace(p, eps_ab=np.full((2, 2), p.eps)))[0]
    a3 = gpu_solve(ctx, dataclasses.replace(p, eps_ab=eps_matrix(p, 4)))[0]
    assert np.array_equal(a1, a2)
    rms = np.sqrt(np.mean(np.sum(a1 ** 2, axis=0)))
    assert np.max(np.linalg.norm(a3 - a1, axis=0)) > 1e-3 * rms


def test_with_accumulator_laws(ctx):
    p = synth.accumulator_problem(10000, 44, D=3, cored=(1,), ntab=512)
    parity(ctx, dataclasses.replace(p, eps_ab=eps_matrix(p, 5)), 32)


def test_batched_box(ctx):
    import torch
    probs = [synth.clustered_problem(5000, 2, 45, grid=synth.GRID_R2, ntab=256),
             synth.clustered_problem(7000, 3, 46, grid=synth.GRID_R2, ntab=256)]
    probs = [dataclasses.replace(probs[0], eps_ab=eps_matrix(probs[0], 6)), probs[1]]
    boxes, accs = [], []
    for p in probs:
        acc = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
        boxes.append(ngr.BatchBox(D=p.D, box=p.box, acc=acc, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut,
                                  eps=p.eps, theta=p.theta, leaf_size=p.leaf_size, group_size=32,
                                  eps_ab=p.eps_ab, **device_inputs(p)))
        accs.append(acc)
    ngr.batch_build_force(ctx, boxes)
    for p, acc in zip(probs, accs):
        assert np.array_equal(acc.cpu().numpy(), gpu_solve(ctx, p, group_size=32)[0])


@pytest.mark.parametrize("bad", [-1e-3, float("nan"), float("inf")])
def test_invalid(ctx, bad):
    p = synth.clustered_problem(1000, 2, 47, grid=synth.GRID_R2, ntab=64)
    e = np.full((2, 2), p.eps)
    e[1, 0] = bad
    with pytest.raises(ngr.NgravsError):
        gpu_solve(ctx, dataclasses.replace(p, eps_ab=e))
