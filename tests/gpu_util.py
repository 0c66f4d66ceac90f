"""Helpers shared by the GPU tests: move a synthetic problem to the device,
run the C-ABI pipeline, and compare with the oracle."""
import numpy as np

import oracle
import paper_1502_07442_amd as ngr


def device_inputs(p):
    import torch
    dev = torch.device("cuda", 0)
    species = torch.from_numpy(np.ascontiguousarray(p.species, np.uint8)).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(p.mass, np.float64)).to(dev)
    pos = lat = None
    if p.lattice is not None:
        lat = torch.from_numpy(np.ascontiguousarray(p.lattice).view(np.int64)).to(dev)
    else:
        pos = torch.from_numpy(np.ascontiguousarray(p.pos, np.float64)).to(dev)
    return dict(species=species, mass=mass, pos=pos, lattice=lat)


def gpu_solve(ctx, p, group_counts=False, keep_tree=False, group_size=None, track_counts=True):
    """Build, monopoles and force on the GPU (the accumulator laws when p
    has them). Returns (acc (3, n) numpy, stats, per-group counts or None,
    tree or None)."""
    import torch
    t = device_inputs(p)
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, periodic=getattr(p, "periodic", True),
                          key_order=getattr(p, "key_order", "morton"), **t)
    ngr.compute_monopoles(ctx, tree, track_counts=track_counts)
    acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
    gs = p.group_size if group_size is None else group_size
    rel = getattr(p, "relative", None)
    if rel is not None:
        rel = {"alpha": rel["alpha"], "old_acc": torch.from_numpy(np.ascontiguousarray(rel["old_acc"])).cuda()}
    res = ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                         theta=p.theta, r_s=p.r_s, group_size=gs, acc=acc, group_counts=group_counts,
                         accumulator=getattr(p, "accumulator", None), eps_ab=getattr(p, "eps_ab", None),
                         relative=rel, lattice_corr=getattr(p, "lattice_corr", None))
    st, gc = (res if group_counts else (res, None))
    out = acc.cpu().numpy()
    if not keep_tree:
        ngr.tree_free(ctx, tree)
        tree = None
    return out, st, gc, tree


def force_gate(acc_gpu, acc_orc, slack, rel=1e-5):
    """Per-particle gate |a_gpu - a_orc| <= rel * rms|a_orc| + slack. Returns
    (ok, worst ratio of error to allowance, rms|a|, max |da| / rms)."""
    rms = float(np.sqrt(np.mean(np.sum(acc_orc ** 2, axis=0)))) if acc_orc.size else 0.0
    da = np.linalg.norm(acc_gpu - acc_orc, axis=0)
    allowed = rel * rms + slack
    ok = bool(np.all(da <= allowed))
    ratio = np.divide(da, allowed, out=np.where(da > 0, np.inf, 0.0), where=allowed > 0)
    worst = float(np.max(ratio)) if da.size else 0.0
    return ok, worst, rms, (float(np.max(da)) / rms if rms > 0 and da.size else 0.0)
