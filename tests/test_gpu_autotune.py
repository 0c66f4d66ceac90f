"""The group-size autotuner: it tunes every class present, later calls with
group_size = 0 resolve to its choices (batched and single-box), each box of
a tuned batch is bitwise its single-box call at the resolved size and its
counts are the oracle's, and a fresh context keeps the default."""
import numpy as np
import pytest

import oracle
import paper_1502_07442_amd as ngr
import synth
from gpu_util import device_inputs, gpu_solve

pytestmark = pytest.mark.gpu


def boxes_of(probs):
    import torch
    boxes, accs = [], []
    for p in probs:
        acc = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
        boxes.append(ngr.BatchBox(D=p.D, box=p.box, acc=acc, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut,
                                  eps=p.eps, theta=p.theta, r_s=p.r_s, leaf_size=p.leaf_size, group_size=0,
                                  **device_inputs(p)))
        accs.append(acc)
    return boxes, accs


def test_tune_then_batch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ngr.Context(0)
    try:
        probs = [synth.batch_box(k) for k in range(12)]
        classes = {(p.D, int(np.floor(np.log2(p.n)))) for p in probs}
        boxes, accs = boxes_of(probs)
        st = ngr.autotune(ctx, boxes)
        print(f"tuned {st}", flush=True)
        assert st["classes"] == len(classes) and st["launches"] == 6 * len(classes)
        chosen = {c: ngr.tuned_group_size(ctx, 2 ** c[1], c[0]) for c in classes}
        assert set(chosen.values()) <= {16, 32, 64}
        _, pb = ngr.batch_build_force(ctx, boxes, per_box=True)
        for p, acc, s in zip(probs, accs, pb):
            assert s["group_size"] == chosen[(p.D, int(np.floor(np.log2(p.n))))]
            a1, s1, _, _ = gpu_solve(ctx, p, group_size=s["group_size"])
            assert np.array_equal(a1, acc.cpu().numpy()), p.name
        for p, s in list(zip(probs, pb))[:3]:
            co = oracle.Tree.of(p, group_size=s["group_size"]).force(oracle.law_of(p))[2]
            assert (s["interactions_pp"], s["interactions_pn"]) == (co["pp"], co["pn"])
        # single-box calls with group_size = 0 resolve the same way
        p = probs[0]
        tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **device_inputs(p))
        ngr.compute_monopoles(ctx, tree)
        a = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
        s = ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps, theta=p.theta,
                           r_s=p.r_s, group_size=0, acc=a)
        ngr.tree_free(ctx, tree)
        assert s["group_size"] == chosen[(p.D, int(np.floor(np.log2(p.n))))]
    finally:
        ctx.close()
    fresh = ngr.Context(0)
    try:
        assert ngr.tuned_group_size(fresh, 5000, 3) == 32
    finally:
        fresh.close()
