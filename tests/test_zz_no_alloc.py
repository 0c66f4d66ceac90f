"""The no-allocation entry point (ngr_tree_force_noalloc) through the C-ABI
against ngr_tree_force on the same tree: bitwise equal accelerations and
equal counts, on two calls in a row (the second on a smaller tree, so the
shared static scratch holds the first call's leftovers), plus its limits."""
import numpy as np
import pytest

import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


def both(ctx, p, device_tables=False):
    """ngr_tree_force with host tables, and ngr_tree_force_noalloc with the
    same tables as host arrays or (device_tables) as a device tensor."""
    import torch
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **t)
    try:
        ngr.compute_monopoles(ctx, tree)
        kw = dict(G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta,
                  group_size=p.group_size, r_s=p.r_s)
        a_ref = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        st_ref = ngr.tree_force(ctx, tree, acc=a_ref, **kw)
        if device_tables:
            kw["tables"] = torch.from_numpy(np.ascontiguousarray(p.tables, dtype=np.float64)).cuda()
        a_na = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
        st_na = ngr.tree_force_noalloc(ctx, tree, acc=a_na, **kw)
        return a_ref.cpu().numpy(), st_ref, a_na.cpu().numpy(), st_na
    finally:
        ngr.tree_free(ctx, tree)


def check(ctx, p, device_tables=False):
    print(f"case {p.name} n={p.n} D={p.D} device tables {device_tables}", flush=True)
    a_ref, st_ref, a_na, st_na = both(ctx, p, device_tables)
    assert np.array_equal(a_ref, a_na)
    for k in ("interactions_pp", "interactions_pn", "n_groups", "group_size", "interactions_pn_species"):
        assert st_ref[k] == st_na[k], k
    assert st_na["near_ties"] == ngr.NOT_COUNTED


def test_two_calls_second_smaller(ctx):
    check(ctx, synth.clustered_problem(2 ** 17, 6, 21))
    check(ctx, synth.clustered_problem(3000, 2, 22, ntab=512, grid="r"))


def test_device_tables(ctx):
    """Tables handed over as a device tensor: the static scratch stages none
    of them, and the result is the host-table call's, bit for bit."""
    check(ctx, synth.clustered_problem(20000, 4, 26, ntab=1024), device_tables=True)
    check(ctx, synth.clustered_problem(3000, 2, 27, ntab=512, grid="r"), device_tables=True)


def test_accumulator_laws_and_softening_zero(ctx):
    p = synth.accumulator_problem(20000, 23)
    import torch
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **t)
    try:
        ngr.compute_monopoles(ctx, tree)
        kw = dict(G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=0.0, theta=p.theta,
                  group_size=32, accumulator=p.accumulator)
        a_ref = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        a_na = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        ngr.tree_force(ctx, tree, acc=a_ref, **kw)
        ngr.tree_force_noalloc(ctx, tree, acc=a_na, **kw)
        assert np.array_equal(a_ref.cpu().numpy(), a_na.cpu().numpy())
    finally:
        ngr.tree_free(ctx, tree)


def test_limits(ctx):
    import torch
    p = synth.clustered_problem(ngr.NOALLOC_MAX_N + 1, 1, 24, ntab=64)
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **t)
    try:
        ngr.compute_monopoles(ctx, tree)
        a = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        with pytest.raises(ngr.NgravsError) as e:
            ngr.tree_force_noalloc(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                                   theta=p.theta, group_size=64, acc=a)
        assert e.value.status == ngr.EINVAL and "NGR_NOALLOC_MAX_N" in str(e.value)
    finally:
        ngr.tree_free(ctx, tree)
    # the context still works afterwards
    check(ctx, synth.clustered_problem(5000, 3, 25, ntab=256))
