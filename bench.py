#!/usr/bin/env python3
"""Benchmark of the short-range multi-species tree force on one MI355X.

One step is the whole hot path on one batch of particles already resident in
HBM: lattice and keys, sort, octree, per-species monopoles, groups and the
tree walk (ngr_tree_build + ngr_compute_monopoles + ngr_tree_force), for the
clustered 2^24-particle, six-species box. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops of one pair term (FMA = 2, transcendental = 1): offsets 3, r^2 5, +eps^2 1,
# rsqrt 1, cube 2, table index 1, floor/fraction 2, lerp 2, mu*f*rho^3 2, three accumulations 6.
FLOPS_PER_INTERACTION = 26
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_traffic():
    """HBM bytes of one walk launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or
    None when the walk sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "walk_clustered_2p24_D6_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("walk_traffic_bytes", "source_sha256"):
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in ("walk.hip", "ngr_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1502_07442_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest() or "walk_traffic_bytes" not in fields:
        return None
    return float(fields["walk_traffic_bytes"])


def cpu_baseline(p, gpu_counts, seconds):
    """The FP64 oracle on a bounded, seeded sample of groups of the same
    workload: interactions per second of its walk on the host cores."""
    import numpy as np

    import oracle
    t0 = time.time()
    T = oracle.Tree.of(p)
    build_s = time.time() - t0
    law = oracle.law_of(p)
    rng = np.random.default_rng(7)
    order = rng.permutation(T.n_groups).astype(np.uint32)
    # grow a seeded random sample of groups until it takes about `seconds`
    take, dt, c1 = 64, 0.0, None
    while True:
        sample = np.sort(order[:take])
        t0 = time.time()
        _, _, c1, _ = T.force(law, groups=sample)
        dt = time.time() - t0
        if dt >= 0.5 * seconds or take >= T.n_groups:
            break
        take = int(min(T.n_groups, take * max(2.0, min(16.0, seconds / max(dt, 1e-3)))))
    inter = c1["pp"] + c1["pn"]
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{take} of {T.n_groups} groups (seeded random), {inter} interactions in {dt:.1f} s; "
                      f"oracle tree build {build_s:.1f} s not included"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2 ** 24, help="particles (the benchmark workload is 2^24)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: the path is built and "
              f"measured for one MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1502_07442_amd as ngr
    import synth

    log(f"generating the clustered workload n={args.n}")
    p = synth.clustered_d6(3, n=args.n)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(p.pos).to(dev)
    species = torch.from_numpy(p.species).to(dev)
    mass = torch.from_numpy(p.mass).to(dev)
    acc = torch.empty((3, p.n), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ctx = ngr.Context(0)

    def step():
        tree = ngr.tree_build(ctx, D=p.D, box=p.box, pos=pos, species=species, mass=mass, leaf_size=p.leaf_size)
        ngr.compute_monopoles(ctx, tree)
        st = ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                            theta=p.theta, group_size=p.group_size, acc=acc)
        ngr.tree_free(ctx, tree)
        return st

    for i in range(args.warmup):
        st = step()
        log(f"warmup {i}: walk {st['ms_walk']:.2f} ms, interactions {st['interactions_pp'] + st['interactions_pn']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(step())
        log(f"step {i}: walk {stats[-1]['ms_walk']:.2f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    inter = stats[-1]["interactions_pp"] + stats[-1]["interactions_pn"]
    assert all(s["interactions_pp"] + s["interactions_pn"] == inter for s in stats)
    ms_walk = float(np.mean([s["ms_walk"] for s in stats]))
    # the walk is one launch per step (every sink species), timed with HIP events on its stream
    achieved = FLOPS_PER_INTERACTION * inter / (ms_walk * 1e-3) / 1e12
    out = {
        "metric": "tree-force interactions/s at 2^24,D=6; batched boxes/s + p50/p99 latency",
        "value": inter / (ms_per_step * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"clustered box, {p.n} particles, {p.D} species (Plummer halos + uniform)",
                   "n": p.n, "D": p.D, "theta": p.theta, "ntab": p.ntab, "grid": p.grid, "leaf_size": p.leaf_size,
                   "group_size": p.group_size, "r_cut": p.r_cut, "eps": p.eps, "seed": p.seed},
        "interactions_per_step": inter,
        "walk_ms": ms_walk,
        "walk_interactions_per_s": inter / (ms_walk * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": walk_traffic()},
    }
    if not args.no_cpu_baseline:
        log("oracle baseline on the host cores")
        out["cpu_baseline"] = cpu_baseline(p, inter, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
