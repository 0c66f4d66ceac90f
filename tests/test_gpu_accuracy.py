"""Accuracy of the GPU tree force against the minimum-image direct sum, as
the paper measures force errors (section 3, Eq. (12)):
Delta f / f = |a_tree - a_direct| / |a_direct| per sink, with alpha = 0.005
the tree tolerance of the transition tests (sections 3.1 and 3.2).

alpha is the tolerance of the relative opening criterion that the paper's
tree keeps (section 2.2): a node is used when its Newtonian error estimate is
below alpha times the sink's previous |a|. Its 99th percentile error must
stay within alpha, checked here with the previous accelerations taken from
a first force at theta = 0.5 (the geometric criterion, which needs none).
The geometric criterion at theta = 0.5 meets alpha on the uniform
4096-particle box; on clustered boxes its 99th percentile lies between alpha
and 2 alpha (the densest halos: monopoles accepted at side / distance near
0.5), which is gated at 2 alpha and reported.

The tree force comes from the HIP library through the C-ABI; the direct sum
from the oracle. Sinks with |a_direct| = 0 (no source within r_cut) have no
relative error: they are left out and counted.
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs

pytestmark = pytest.mark.gpu

ALPHA = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))[
    "tree_error_tolerance_alpha"]["value"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ngr.Context(0)
    yield c
    c.close()


def gpu_forces(ctx, p, relative_alpha=None):
    """Geometric force at p.theta, and with relative_alpha the relative
    criterion's force with the previous |a| from the geometric one."""
    import torch
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **t)
    try:
        ngr.compute_monopoles(ctx, tree)
        kw = dict(G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta,
                  group_size=p.group_size, r_s=p.r_s)
        a0 = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        ngr.tree_force(ctx, tree, acc=a0, **kw)
        out = [a0.cpu().numpy()]
        if relative_alpha is not None:
            a1 = torch.empty_like(a0)
            old = torch.linalg.vector_norm(a0, dim=0).contiguous()
            ngr.tree_force(ctx, tree, acc=a1, relative={"alpha": relative_alpha, "old_acc": old}, **kw)
            out.append(a1.cpu().numpy())
        return out
    finally:
        ngr.tree_free(ctx, tree)


def p99_errors(p, forces, sinks=None):
    """p99 of Delta f / f of each force against the oracle's direct sum on
    the sinks (input indices, all when None); and the zero-force count."""
    idx = np.arange(p.n, dtype=np.uint32) if sinks is None else np.sort(sinks).astype(np.uint32)
    ad, _ = oracle.direct_of(p, idx)
    nrm = np.linalg.norm(ad, axis=0)
    keep = nrm > 0
    q = [float(np.percentile(np.linalg.norm(a[:, idx] - ad, axis=0)[keep] / nrm[keep], 99)) for a in forces]
    return q, int((~keep).sum())


@pytest.mark.parametrize("seed", range(1, 11))
def test_p99_uniform_4096_all_sinks(ctx, seed):
    """The 4096-particle, two-species box, every sink of each of ten seeds:
    theta = 0.5 within alpha."""
    p = synth.uniform_4096(seed)
    (q,), zero = p99_errors(p, gpu_forces(ctx, p))
    print(f"case {p.name}: p99 Delta f/f = {q:.3e} ({zero} sinks with zero direct force)")
    assert q <= ALPHA


def clustered_case(ctx, p, nsinks):
    sinks = np.random.default_rng(11).choice(p.n, nsinks, replace=False)
    (qg, qr), zero = p99_errors(p, gpu_forces(ctx, p, relative_alpha=ALPHA), sinks)
    print(f"case {p.name}: p99 Delta f/f theta 0.5 {qg:.3e}, relative alpha {ALPHA}: {qr:.3e} "
          f"over {nsinks - zero} sinks ({zero} with zero direct force)")
    assert qr <= ALPHA
    assert qg <= 2 * ALPHA


def test_p99_clustered_yukawa_2_21(ctx):
    """The 2^21, three-species Yukawa box: 2^16 seeded sinks."""
    clustered_case(ctx, synth.clustered_yukawa_d3(2), 2 ** 16)


@pytest.mark.slow
def test_p99_clustered_d6_2_24(ctx):
    """The benchmark box (2^24, six species, 2000 halos): 2^16 seeded sinks."""
    clustered_case(ctx, synth.clustered_d6(3), 2 ** 16)
