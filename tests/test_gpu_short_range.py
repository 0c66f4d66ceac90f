"""Exact short-range tables (section 2.4.1, Eqs. (8)-(11)) from the HIP
path against the oracle's adaptive quadrature: Newton, Yukawa of both signs
and ranges, mixed per species pair, both table grids, to 1e-12 absolute
(the factors are of order one)."""
import math

import numpy as np
import pytest

import paper_1502_07442_amd as ngr
import synth
from oracle.short_range import short_factor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


def newton():
    return (lambda k: -4 * math.pi, lambda r: 1.0, 0.0)


def yukawa(alpha, lam):
    mu2 = lam ** -2
    return (lambda k: -4 * math.pi * (1 + alpha * k * k / (k * k + mu2)),
            lambda r: 1 + alpha * (1 + r / lam) * math.exp(-r / lam), lam)


def build(ctx, laws, r_s, r_cut, ntab, grid):
    D = len(laws)
    rng = max(l[2] for row in laws for l in row)
    nk, dk = ngr.short_range_grid(r_s, r_cut, rng)
    ks = np.arange(nk) * dk
    radii = synth.table_abscissae(ntab, r_cut, grid)
    phib = np.array([[[laws[a][b][0](k) for k in ks] for b in range(D)] for a in range(D)])
    full = np.array([[[laws[a][b][1](r) for r in radii] for b in range(D)] for a in range(D)])
    print(f"case D={D} ntab={ntab} grid={grid} nk={nk}", flush=True)
    return ngr.short_range_tables(ctx, phibar=phib, f_full=full, r_s=r_s, r_cut=r_cut, grid=grid, dk=dk), radii


@pytest.mark.parametrize("grid", [synth.GRID_R, synth.GRID_R2])
def test_newton_matches_closed_form(ctx, grid):
    r_s = 1.25 / 64 / 16
    r_cut = 4.5 * r_s
    t, radii = build(ctx, [[newton()]], r_s, r_cut, 2048, grid)
    ref = synth.newtonian_treepm_factor(radii, r_s)
    assert np.max(np.abs(t[0, 0] - ref)) < 1e-12


@pytest.mark.parametrize("grid", [synth.GRID_R, synth.GRID_R2])
def test_mixed_laws_match_oracle(ctx, grid):
    r_s = 0.0025
    r_cut = 4.5 * r_s
    laws = [[newton(), yukawa(1.0, 0.01), yukawa(-0.5, 0.003)],
            [yukawa(1.0, 0.01), yukawa(0.7, 0.03), newton()],
            [yukawa(-0.5, 0.003), newton(), yukawa(0.2, 0.001)]]
    t, radii = build(ctx, laws, r_s, r_cut, 1024, grid)
    sample = np.unique(np.concatenate([np.arange(0, 1024, 37), [1, 2, 1022, 1023]]))
    for a in range(3):
        for b in range(3):
            ref = np.array([short_factor(laws[a][b][0], laws[a][b][1], r_s, float(radii[i])) for i in sample])
            assert np.max(np.abs(t[a, b, sample] - ref)) < 1e-12, (a, b)


def test_tables_drive_the_walk(ctx):
    """Generated Newtonian tables and the library's default tables give the
    same forces to the tables' own agreement."""
    import torch
    from gpu_util import device_inputs
    p = synth.clustered_problem(20000, 2, 9, grid=synth.GRID_R2, ntab=2048)
    t, _ = build(ctx, [[newton(), newton()], [newton(), newton()]], p.r_s, p.r_cut, 2048, p.grid)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **device_inputs(p))
    try:
        ngr.compute_monopoles(ctx, tree)
        a1 = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        a2 = torch.empty_like(a1)
        ngr.tree_force(ctx, tree, G=p.G, tables=t, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta, acc=a1)
        ngr.tree_force(ctx, tree, G=p.G, tables=None, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta,
                       r_s=p.r_s, ntab=2048, acc=a2)
        a1, a2 = a1.cpu().numpy(), a2.cpu().numpy()
        rms = np.sqrt(np.mean(np.sum(a2 ** 2, axis=0)))
        assert np.max(np.linalg.norm(a1 - a2, axis=0)) < 1e-9 * rms
    finally:
        ngr.tree_free(ctx, tree)


def test_invalid(ctx):
    nk, dk = ngr.short_range_grid(0.01, 0.045, 0.0)
    phib = np.full((1, 1, nk), -4 * math.pi)
    full = np.ones((1, 1, 16))
    for kw in (dict(r_s=0.0), dict(dk=-1.0), dict(r_cut=float("inf"))):
        args = dict(phibar=phib, f_full=full, r_s=0.01, r_cut=0.045, grid="r", dk=dk)
        args.update(kw)
        with pytest.raises(ngr.NgravsError):
            ngr.short_range_tables(ctx, **args)
    bad = phib.copy()
    bad[0, 0, 3] = float("nan")
    with pytest.raises(ngr.NgravsError):
        ngr.short_range_tables(ctx, phibar=bad, f_full=full, r_s=0.01, r_cut=0.045, grid="r", dk=dk)
