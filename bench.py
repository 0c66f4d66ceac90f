#!/usr/bin/env python3
"""Benchmark of the short-range multi-species tree force on one MI355X.

One step is the whole hot path on one batch of particles already resident in
HBM: lattice and keys, sort, octree, per-species monopoles, groups and the
tree walk (ngr_tree_build + ngr_compute_monopoles + ngr_tree_force), for the
clustered 2^24-particle, six-species box (2000 Plummer halos, as at 2^21).
Prints one JSON line.

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
    None when the walk kernel's source has changed since the counters were
    taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "walk_clustered_2p24_D6_H2000_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("walk_traffic_bytes", "source_sha256"):
            fields[k] = v.strip()
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1502_07442_amd", "csrc", "walk.hip"), "rb") as fh:
        h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest() or "walk_traffic_bytes" not in fields:
        return None
    return float(fields["walk_traffic_bytes"])


def pm_traffic():
    """HBM bytes per launch of the PM's forward x and y passes (together) and
    of the fused z pass, from the committed rocprofv3 counter summary, or None
    when the PM source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pm_mesh1024_2p24_D6_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("fft_xy_traffic_bytes", "green_z_traffic_bytes", "source_sha256"):
            fields[k] = v.strip()
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1502_07442_amd", "csrc", "pm.hip"), "rb") as fh:
        h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest() or len(fields) != 3:
        return None
    return float(fields["fft_xy_traffic_bytes"]), float(fields["green_z_traffic_bytes"])


def batched(ngr, synth, nbox=256, reps=3):
    """The many-box workload: nbox independent boxes in one
    ngr_batch_build_force call (group size chosen by the library), against
    the same boxes looped box by box through the single-box calls on the same
    stream; then the autotuner on the same boxes and the batch at the sizes
    it chose. Inputs, the law tables included, are resident on the device
    before timing; each call includes the build. The batch with the tables
    handed over from host memory (copied inside the call) is timed beside it
    as context."""
    import numpy as np
    import torch
    probs = [synth.batch_box(k) for k in range(nbox)]
    dev = torch.device("cuda", 0)
    inputs = []
    for q in probs:
        inputs.append(dict(species=torch.from_numpy(np.ascontiguousarray(q.species, np.uint8)).to(dev),
                           mass=torch.from_numpy(q.mass).to(dev), pos=torch.from_numpy(q.pos).to(dev)))
    tabs = [None if q.tables is None else torch.from_numpy(np.ascontiguousarray(q.tables, np.float64)).to(dev)
            for q in probs]
    accs = [torch.empty((3, q.n), dtype=torch.float64, device=dev) for q in probs]

    def make_boxes(tables):
        return [ngr.BatchBox(D=q.D, box=q.box, acc=a, G=q.G, tables=tb, grid=q.grid, r_cut=q.r_cut, eps=q.eps,
                             theta=q.theta, r_s=q.r_s, leaf_size=q.leaf_size, group_size=0, **t)
                for q, t, a, tb in zip(probs, inputs, accs, tables)]
    boxes = make_boxes(tabs)
    ctx = ngr.Context(0)

    def timed_batches(bx):
        ngr.batch_build_force(ctx, bx)              # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = ngr.batch_build_force(ctx, bx)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), s
    t_batch, st = timed_batches(boxes)
    t_host_tables, _ = timed_batches(make_boxes([q.tables for q in probs]))
    inter = st["interactions_pp"] + st["interactions_pn"]

    def loop():
        for q, t, a, tb in zip(probs, inputs, accs, tabs):
            tree = ngr.tree_build(ctx, D=q.D, box=q.box, leaf_size=q.leaf_size, **t)
            ngr.compute_monopoles(ctx, tree)
            ngr.tree_force(ctx, tree, G=q.G, tables=tb, grid=q.grid, r_cut=q.r_cut, eps=q.eps, theta=q.theta,
                           r_s=q.r_s, group_size=0, acc=a)
            ngr.tree_free(ctx, tree)
    loop()                                          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    # the autotuner on the same boxes, then the batch at its sizes
    tune = ngr.autotune(ctx, boxes)
    ngr.batch_build_force(ctx, boxes)               # warm-up
    ttimes = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stt = ngr.batch_build_force(ctx, boxes)
        torch.cuda.synchronize()
        ttimes.append(time.perf_counter() - t0)
    t_tuned = float(np.median(ttimes))
    _, pbt = ngr.batch_build_force(ctx, boxes, per_box=True)     # the sizes used (untimed)
    sizes = {g: sum(1 for b in pbt if b["group_size"] == g) for g in (16, 32, 64)}
    # the default size again, after the tuned runs (same context)
    for b in boxes:
        b.force.group_size = 32
    dtimes = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        std = ngr.batch_build_force(ctx, boxes)
        torch.cuda.synchronize()
        dtimes.append(time.perf_counter() - t0)
    for b in boxes:
        b.force.group_size = 0
    t_default_after = float(np.median(dtimes))
    ctx.close()
    return {"workload": f"{nbox} clustered boxes: n log-uniform in [2^12, 2^18], D in 1..4, clustered fraction "
                        f"in [0, 0.8], laws of their own", "n_boxes": nbox, "n_particles": st["n_particles"],
            "interactions": inter, "ms_per_batch": t_batch * 1e3, "boxes_per_s": nbox / t_batch,
            "interactions_per_s": inter / t_batch, "walk_ms": st["ms_walk"], "build_ms": st["ms_build"],
            "ms_per_batch_host_tables": t_host_tables * 1e3,
            "loop_ms": t_loop * 1e3, "loop_boxes_per_s": nbox / t_loop, "speedup_vs_loop": t_loop / t_batch,
            "group_size": "library default (32)",
            "tuned": {"tune_ms": tune["ms"], "classes": tune["classes"], "ms_per_batch": t_tuned * 1e3,
                      "boxes_per_s": nbox / t_tuned, "walk_ms": stt["ms_walk"],
                      "interactions": stt["interactions_pp"] + stt["interactions_pn"],
                      "boxes_by_group_size": sizes, "speedup_vs_loop": t_loop / t_tuned,
                      "build_ms": stt["ms_build"], "groups_ms": stt["ms_groups"],
                      "default_again_ms_per_batch": t_default_after * 1e3, "default_again_groups_ms": std["ms_groups"],
                      "default_again_walk_ms": std["ms_walk"]},
            "groups_ms": st["ms_groups"]}


def served(ngr, synth, nreq=200, warm=25, steps=8, dt=1e-3, loads=(0.5, 0.9)):
    """The served workload: requests of `steps` kick-drift-kick steps on new
    boxes (N log-uniform in [2^14, 2^20], D in 1..6), advanced by one request
    server, one force evaluation of every admitted request per tick. The
    saturated rate comes from submitting every request at once; Poisson
    streams at fractions of it give latencies (arrival to completion; the
    first `warm` requests are not counted). Baseline: the same requests one
    at a time (FIFO) through the single-box calls, each one's service time
    measured alone and queued on the same arrival times."""
    import numpy as np
    import torch
    probs = [synth.serve_request(r) for r in range(nreq)]
    dev = torch.device("cuda", 0)
    inputs = [dict(species=torch.from_numpy(np.ascontiguousarray(q.species, np.uint8)).to(dev),
                   mass=torch.from_numpy(q.mass).to(dev), pos=torch.from_numpy(q.pos).to(dev)) for q in probs]
    torch.cuda.synchronize()
    ctx = ngr.Context(0)

    def submit(srv, j):
        q = probs[j]
        return srv.submit(D=q.D, box=q.box, G=q.G, tables=q.tables, grid=q.grid, r_cut=q.r_cut, eps=q.eps,
                          theta=q.theta, r_s=q.r_s, dt=dt, steps=steps, leaf_size=q.leaf_size, group_size=0,
                          **inputs[j])

    def drive(arrivals):
        """Submit at the arrival times (None: all at once), tick while there is
        work; returns completion times (s from the start) and tick count."""
        srv = ngr.Server(ctx)
        done, ids, k, ticks = {}, {}, 0, 0
        t0 = time.perf_counter()
        while len(done) < nreq:
            now = time.perf_counter() - t0
            while k < nreq and (arrivals is None or arrivals[k] <= now):
                ids[k] = submit(srv, k)
                k += 1
            if not ids:
                time.sleep(max(0.0, min(arrivals[k] - now, 0.01)))
                continue
            srv.tick()
            ticks += 1
            t = time.perf_counter() - t0
            for j, rid in list(ids.items()):
                if srv.status(rid)[0] == ngr.FINISHED:
                    srv.take(rid)
                    done[j] = t
                    del ids[j]
        srv.close()
        return np.array([done[j] for j in range(nreq)]), ticks

    comp, ticks = drive(None)
    sat_s = float(comp.max())
    sat_rate = nreq / sat_s

    # baseline service times: each request alone through the single-box calls,
    # from its lattice (the library's conversion of its positions, taken
    # before timing)
    def lattice0(j):
        q = probs[j]
        tree = ngr.tree_build(ctx, D=q.D, box=q.box, leaf_size=q.leaf_size, **inputs[j])
        ex = ngr.tree_export(ctx, tree)
        ngr.tree_free(ctx, tree)
        X = np.empty((3, q.n), np.uint64)
        X[:, ex["perm"]] = ex["lattice"]
        return torch.from_numpy(X.view(np.int64)).to(dev)

    def alone(j):
        q = probs[j]
        h = 0.5 * dt
        X = lattice0(j)

        def force(lat):
            tree = ngr.tree_build(ctx, D=q.D, box=q.box, leaf_size=q.leaf_size, species=inputs[j]["species"],
                                  mass=inputs[j]["mass"], lattice=lat)
            ngr.compute_monopoles(ctx, tree)
            a = torch.empty((3, q.n), dtype=torch.float64, device=dev)
            ngr.tree_force(ctx, tree, G=q.G, tables=q.tables, grid=q.grid, r_cut=q.r_cut, eps=q.eps, theta=q.theta,
                           r_s=q.r_s, group_size=0, acc=a)
            ngr.tree_free(ctx, tree)
            return a

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = force(X)
        v = torch.zeros_like(a)
        for _ in range(steps):
            v.add_(a, alpha=h)
            d = v * (dt / q.box)
            d -= torch.round(d)
            d.clamp_(-0.5, 0.5 - 2.0 ** -53)
            X += (d * 2.0 ** 64).to(torch.int64)
            a = force(X)
            v.add_(a, alpha=h)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    service = np.array([alone(j) for j in range(nreq)])
    out = {"workload": f"requests of {steps} kick-drift-kick steps (dt {dt}) on new clustered boxes: N log-uniform "
                       f"in [2^14, 2^20], D in 1..6, laws of their own; Poisson arrivals",
           "requests": nreq, "warmup_requests": warm, "steps_per_request": steps,
           "particles_mean": float(np.mean([q.n for q in probs])),
           "saturated": {"requests_per_s": sat_rate, "steps_per_s": steps * nreq / sat_s, "ticks": ticks},
           "fifo_service_ms_mean": float(service.mean() * 1e3)}
    for f in loads:
        rate = f * sat_rate
        arr = synth.poisson_arrivals(nreq, rate, seed=5)
        comp, ticks = drive(arr)
        lat = (comp - arr)[warm:] * 1e3
        fin = np.empty(nreq)
        t = 0.0
        for j in range(nreq):                       # FIFO queue on the same arrivals
            t = max(t, arr[j]) + service[j]
            fin[j] = t
        flat = (fin - arr)[warm:] * 1e3
        out[f"load_{f}"] = {"rate_per_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                            "p99_ms": float(np.percentile(lat, 99)),
                            "steps_per_s": steps * (nreq - warm) / float(comp[warm:].max() - arr[warm]),
                            "fifo_p50_ms": float(np.percentile(flat, 50)), "fifo_p99_ms": float(np.percentile(flat, 99))}
    ctx.close()
    return out


def accumulator(ngr, synth, n=2 ** 22, steps=3):
    """The accumulator laws (section 3.3) on the two-species workload: one
    Newtonian and one cored species, N_perp tracked; a step is the build,
    the monopoles and the force, timed like the main workload. The same
    particles under the table law (no cores) give the overhead of the cored
    pair term."""
    import numpy as np
    import torch
    p = synth.accumulator_problem(n, 3)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(p.pos).to(dev)
    species = torch.from_numpy(np.ascontiguousarray(p.species, np.uint8)).to(dev)
    mass = torch.from_numpy(p.mass).to(dev)
    acc = torch.empty((3, p.n), dtype=torch.float64, device=dev)
    ctx = ngr.Context(0)

    def step(law):
        tree = ngr.tree_build(ctx, D=p.D, box=p.box, pos=pos, species=species, mass=mass, leaf_size=p.leaf_size)
        ngr.compute_monopoles(ctx, tree, track_counts=True)
        st = ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                            theta=p.theta, group_size=p.group_size, acc=acc, accumulator=law)
        ngr.tree_free(ctx, tree)
        return st

    res = {}
    for name, law in (("accumulator", p.accumulator), ("table", None)):
        step(law)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [step(law) for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        inter = sts[-1]["interactions_pp"] + sts[-1]["interactions_pn"]
        res[name] = (ms, float(np.mean([s["ms_walk"] for s in sts])), inter)
    ctx.close()
    ms, walk, inter = res["accumulator"]
    return {"workload": f"clustered box, {p.n} particles, 2 species (one cored, beta {p.accumulator['beta']:.4g}: "
                        f"one body's core 0.25 of the mean spacing), N_perp tracked",
            "n": p.n, "ms_per_step": ms, "interactions": inter, "interactions_per_s": inter / (ms * 1e-3),
            "walk_ms": walk, "walk_interactions_per_s": inter / (walk * 1e-3),
            "table_law_walk_ms": res["table"][1], "cored_walk_over_table_walk": walk / res["table"][1]}


def short_tables(ngr, synth, D=6, ntab=2048, reps=5):
    """Exact short-range tables (section 2.4.1) for D x D random Newton and
    Yukawa laws at the benchmark box's r_s and r_cut: the time of one
    ngr_short_range_tables call (host samples in, host tables out), and the
    Newtonian pairs' largest deviation from the closed-form factor."""
    import numpy as np
    r_s, r_cut, _ = synth.scaled_params(2 ** 24)
    laws = synth.exact_split_laws(D, 7)
    rng = max(l[2] for row in laws for l in row)
    nk, dk = ngr.short_range_grid(r_s, r_cut, rng)
    ks = np.arange(nk) * dk
    radii = synth.table_abscissae(ntab, r_cut, synth.GRID_R2)
    phib = np.array([[laws[a][b][0](ks) for b in range(D)] for a in range(D)])
    full = np.array([[laws[a][b][1](radii) for b in range(D)] for a in range(D)])
    ctx = ngr.Context(0)
    t = ngr.short_range_tables(ctx, phibar=phib, f_full=full, r_s=r_s, r_cut=r_cut, grid=synth.GRID_R2, dk=dk)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        t = ngr.short_range_tables(ctx, phibar=phib, f_full=full, r_s=r_s, r_cut=r_cut, grid=synth.GRID_R2, dk=dk)
        times.append(time.perf_counter() - t0)
    ctx.close()
    newton = [(a, b) for a in range(D) for b in range(D) if laws[a][b][2] == 0.0]
    ref = synth.newtonian_treepm_factor(radii, r_s)
    err = max((float(np.max(np.abs(t[a, b] - ref))) for a, b in newton), default=None)
    return {"workload": f"{D}x{D} random Newton/Yukawa laws, {ntab} samples on the r^2 grid, r_s and r_cut of "
                        f"the 2^24 box", "nk": nk, "ms": float(np.median(times)) * 1e3,
            "newton_max_abs_err_vs_closed_form": err}


def pm_leg(ngr, synth, p, tensors, reps=3):
    """The PM long-range force of the benchmark box (sections 2, 2.4.1): a
    mesh of N = 1.25 box / r_s points per side (the workload's r_s is 1.25
    mesh cells, the usual TreePM choice), D = 6 species, the benchmark's G
    and Newtonian laws. A plan is made once; each force call runs the
    deposit, the forward FFTs, the k-space step, the inverse FFTs and the
    interpolation. The FFT roofline counts one read and one write of every
    mesh per 1-D pass (three passes per 3-D transform)."""
    import math
    import numpy as np
    import torch
    N = int(round(1.25 * p.box / p.r_s))
    q = np.arange(3 * (N // 2) ** 2 + 1)
    phib = np.broadcast_to(np.full(len(q), -4.0 * math.pi), (p.D, p.D, len(q))).copy()
    ctx = ngr.Context(0)
    t0 = time.perf_counter()
    plan = ngr.PM(ctx, N=N, D=p.D, box=p.box, r_s=p.r_s, G=p.G, phibar=phib)
    t_plan = time.perf_counter() - t0
    tree = ngr.tree_build(ctx, D=p.D, box=p.box, leaf_size=p.leaf_size, **tensors)
    acc = torch.empty((3, p.n), dtype=torch.float64, device="cuda")
    plan.force(tree, acc)
    walls, stats = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(plan.force(tree, acc))
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    ngr.tree_free(ctx, tree)
    plan.close()
    ctx.close()
    st = {k: float(np.median([s[k] for s in stats])) for k in stats[0]}
    ngrid = (p.D + 1) // 2
    sweep = 2 * 16.0 * N ** 3 * ngrid                   # read and write every mesh once
    fft_bytes = 2 * sweep                               # the forward x and y passes
    fft_ms = st["ms_fft_forward"]
    achieved = fft_bytes / (fft_ms * 1e-3) / 1e9
    fused = sweep / (st["ms_green"] * 1e-3) / 1e9       # z transforms and the k-space step, one sweep
    traffic = pm_traffic() if N == 1024 and p.D == 6 else None
    return {"workload": f"PM of the benchmark box: {p.n} particles, {p.D} species, mesh {N}^3, "
                        f"{ngrid} complex float64 meshes", "N": N, "ms_per_force": float(np.median(walls)) * 1e3,
            "plan_ms": t_plan * 1e3, **st,
            "fft_roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                             "frac": achieved / 8000.0, "traffic": traffic[0] if traffic else None},
            "green_z_roofline": {"bound": "hbm", "achieved": fused, "peak": 8000.0, "unit": "GB/s",
                                 "frac": fused / 8000.0, "traffic": traffic[1] if traffic else None}}


def cpu_baseline(p, gpu_group_counts, gpu_acc, seconds, gpu_acc_relative=None):
    """The CPU-baseline leg, the one place the benchmark runs the oracle.
    (1) The FP64 oracle on a bounded, seeded sample of groups of the same
    workload: interactions per second of its walk on the host cores; the
    oracle's per-group counts of the sample must equal the GPU's. (2) With
    the GPU's accelerations, the accuracy measure below. Returns (baseline,
    accuracy or None)."""
    import numpy as np

    import oracle
    t0 = time.time()
    T = oracle.Tree.of(p)
    build_s = time.time() - t0
    law = oracle.law_of(p)
    rng = np.random.default_rng(7)
    order = rng.permutation(T.n_groups).astype(np.uint32)
    # grow a seeded random sample of groups until it takes about `seconds`
    take, dt, c1, gc = 64, 0.0, None, None
    while True:
        sample = np.sort(order[:take])
        t0 = time.time()
        _, _, c1, gc = T.force(law, groups=sample, group_counts=True)
        dt = time.time() - t0
        if dt >= 0.5 * seconds or take >= T.n_groups:
            break
        take = int(min(T.n_groups, take * max(2.0, min(16.0, seconds / max(dt, 1e-3)))))
    if gpu_group_counts is not None and not np.array_equal(gpu_group_counts[sample], gc):
        raise SystemExit("the oracle's per-group interaction counts differ from the GPU's on the sample")
    inter = c1["pp"] + c1["pn"]
    base = {"value": inter / dt, "unit": "interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{take} of {T.n_groups} groups (seeded random), {inter} interactions in {dt:.1f} s, "
                      f"per-group counts equal to the GPU's; oracle tree build {build_s:.1f} s not included"}
    del T
    return base, (accuracy(p, gpu_acc, gpu_acc_relative) if gpu_acc is not None else None)


def accuracy(p, acc_gpu, acc_gpu_relative=None, nsinks=2 ** 16, alpha=0.005):
    """The paper's force-error measure (Eq. (12)): Delta f / f =
    |a_tree - a_direct| / |a_direct| of the GPU tree force against the
    oracle's minimum-image direct sum on a seeded sample of sinks; its 99th
    percentile against the tree tolerance alpha of the transition tests, for
    the theta = 0.5 force and the relative criterion's force."""
    import numpy as np

    import oracle
    sinks = np.sort(np.random.default_rng(11).choice(p.n, min(nsinks, p.n), replace=False)).astype(np.uint32)
    t0 = time.time()
    ad, _ = oracle.direct_of(p, sinks)
    dt = time.time() - t0
    nrm = np.linalg.norm(ad, axis=0)
    keep = nrm > 0
    e = np.linalg.norm(acc_gpu[:, sinks] - ad, axis=0)[keep] / nrm[keep]
    q = float(np.percentile(e, 99))
    out = {"p99_rel_err_tree_vs_direct": q, "median_rel_err": float(np.median(e)), "alpha": alpha,
           "within_alpha": q <= alpha, "sinks": int(keep.sum()), "sinks_zero_direct_force": int((~keep).sum()),
           "direct_sum_s": dt}
    if acc_gpu_relative is not None:
        er = np.linalg.norm(acc_gpu_relative[:, sinks] - ad, axis=0)[keep] / nrm[keep]
        qr = float(np.percentile(er, 99))
        out["relative_criterion"] = {"p99_rel_err_tree_vs_direct": qr, "median_rel_err": float(np.median(er)),
                                     "within_alpha": qr <= alpha}
    return out


def copy_calibration(gib=1, reps=3):
    """Device copies of a known size, for scaling rocprofv3's FETCH_SIZE and
    WRITE_SIZE counters to bytes (profile this run with --pmc)."""
    import torch
    n = gib * (1 << 30)
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_per_copy": n, "copies": reps}}), flush=True)


def run_box(ngr, p, steps, warmup, tag, relative=None):
    """Steps (build + monopoles + force) of one box with inputs resident:
    (ms per step, interactions per step, mean walk ms, mean build ms, mean
    monopoles ms, last stats)."""
    import numpy as np
    import torch
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(p.pos).to(dev)
    species = torch.from_numpy(p.species).to(dev)
    mass = torch.from_numpy(p.mass).to(dev)
    acc = torch.empty((3, p.n), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ctx = ngr.Context(0)

    def step(counts=False):
        tree = ngr.tree_build(ctx, D=p.D, box=p.box, pos=pos, species=species, mass=mass, leaf_size=p.leaf_size)
        ngr.compute_monopoles(ctx, tree)
        st = ngr.tree_force(ctx, tree, G=p.G, tables=p.tables, grid=p.grid, r_cut=p.r_cut, eps=p.eps,
                            theta=p.theta, group_size=p.group_size, acc=acc, group_counts=counts,
                            relative=relative)
        ngr.tree_free(ctx, tree)
        return st

    for i in range(warmup):
        st = step()
        log(f"{tag} warmup {i}: walk {st['ms_walk']:.2f} ms, interactions {st['interactions_pp'] + st['interactions_pn']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        stats.append(step())
        log(f"{tag} step {i}: walk {stats[-1]['ms_walk']:.2f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / steps
    inter = stats[-1]["interactions_pp"] + stats[-1]["interactions_pn"]
    assert all(s["interactions_pp"] + s["interactions_pn"] == inter for s in stats)
    mean = lambda k: float(np.mean([s[k] for s in stats]))
    return dict(ctx=ctx, acc=acc, step=step, tensors=dict(pos=pos, species=species, mass=mass), stats=stats,
                ms_per_step=ms_per_step, inter=inter, ms_walk=mean("ms_walk"), ms_build=mean("ms_build"),
                ms_monopoles=mean("ms_monopoles"), ms_groups=mean("ms_groups"), last=stats[-1])


def build_roofline(st, n):
    """Achieved HBM bandwidth of the build phases on their algorithmic bytes
    (device time of each phase from the library's events, host read-backs
    between levels included): ingest (read position 24 B, species 1 B, mass
    8 B; write the lattice-and-mass record 32 B, key 8 B, index 4 B), the
    sort (eight 8-bit passes, each reading and writing key and index, 24 B,
    and reading the key again for the histogram, 8 B) with the one
    reordering (read the index 4 B and one 32-B record; write lattice and
    mass 32 B and the walk's split record 48 B), and the monopoles (read
    every particle's split record once, 48 B, plus 32 B per node and
    species read and written)."""
    ingest = 77.0 * n
    sort = (8 * 32.0 + 116.0) * n
    mono = 48.0 * n + 2 * 32.0 * st["n_nodes"] * 6
    gbps = lambda b, ms: b / (ms * 1e-3) / 1e9 if ms > 0 else None
    return {"ingest_gbps": gbps(ingest, st["ms_build_ingest"]), "sort_and_gather_gbps": gbps(sort, st["ms_build_sort"]),
            "monopoles_gbps": gbps(mono, st["ms_monopoles"]), "peak_gbps": 8000.0,
            "ms_ingest": st["ms_build_ingest"], "ms_sort_and_gather": st["ms_build_sort"],
            "ms_octree": st["ms_build_octree"], "ms_monopoles": st["ms_monopoles"], "ms_groups": st["ms_groups"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2 ** 24, help="particles (the benchmark workload is 2^24)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-accumulator", action="store_true")
    ap.add_argument("--no-pm", action="store_true")
    ap.add_argument("--no-scaled", action="store_true", help="skip the box with the halo count scaled with n")
    ap.add_argument("--no-relative", action="store_true", help="skip the relative-criterion leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device copies of 1 GiB (to scale rocprofv3 byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: the path is built and "
              f"measured for one MI355X", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np

    import paper_1502_07442_amd as ngr
    import synth

    log(f"generating the clustered workload n={args.n} (2000 halos)")
    p = synth.clustered_d6(3, n=args.n)
    r = run_box(ngr, p, args.steps, args.warmup, "H2000")
    ctx, acc, inter = r["ctx"], r["acc"], r["inter"]
    ms_per_step, ms_walk = r["ms_per_step"], r["ms_walk"]
    # the walk is one launch per step (every sink species), timed with HIP events on its stream
    achieved = FLOPS_PER_INTERACTION * inter / (ms_walk * 1e-3) / 1e12
    last = r["last"]
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
        "dtype": "mixed: f64 positions, offsets, r^2 and sums; f32 kernel factor and table lerp",
        "data": "synthetic",
        "config": {"workload": f"clustered box, {p.n} particles, {p.D} species, 2000 Plummer halos (70%) + uniform",
                   "n": p.n, "D": p.D, "halos": 2000, "theta": p.theta, "ntab": p.ntab, "grid": p.grid,
                   "leaf_size": p.leaf_size, "group_size": p.group_size, "r_cut": p.r_cut, "eps": p.eps,
                   "seed": p.seed},
        "interactions_per_step": inter,
        "interactions_pp": last["interactions_pp"],
        "interactions_pn_by_source_species": last["interactions_pn_species"][:p.D],
        "walk_ms": ms_walk,
        "walk_interactions_per_s": inter / (ms_walk * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": walk_traffic()},
        "build": build_roofline(last, p.n),
    }
    # the paper's relative criterion (section 2.2) at its tolerance alpha = 0.005, with the previous
    # accelerations from the theta = 0.5 step (as the stock code does after its first force)
    import torch
    acc_rel = None
    if not args.no_relative:
        old = torch.linalg.vector_norm(acc, dim=0).contiguous()
        rr = run_box(ngr, p, max(2, args.steps // 2), 1, "relative", relative={"alpha": 0.005, "old_acc": old})
        out["relative_criterion"] = {"workload": "the same box, relative opening criterion alpha 0.005 with the "
                                                 "previous |a| from the theta 0.5 force",
                                     "ms_per_step": rr["ms_per_step"], "interactions_per_step": rr["inter"],
                                     "interactions_per_s": rr["inter"] / (rr["ms_per_step"] * 1e-3),
                                     "walk_ms": rr["ms_walk"],
                                     "walk_interactions_per_s": rr["inter"] / (rr["ms_walk"] * 1e-3)}
        acc_rel = rr["acc"].cpu().numpy() if not (args.no_accuracy or args.no_cpu_baseline) else None
        rr["ctx"].close()
        del rr, old
    gpu_gc = None
    if not args.no_cpu_baseline:
        # one more step with per-group counts (untimed), for the baseline's count check
        _, gpu_gc = r["step"](counts=True)
    gpu_acc = acc.cpu().numpy() if not (args.no_accuracy or args.no_cpu_baseline) else None
    tensors = r["tensors"]
    if not args.no_scaled:
        log("the 2^24 box with 16000 halos (halo count scaled with n)")
        q = synth.clustered_d6_scaled(3, n=args.n)
        rs = run_box(ngr, q, max(2, args.steps // 4), 1, "H16000")
        out["scaled_halos"] = {"workload": f"clustered box, {q.n} particles, {q.D} species, 16000 Plummer halos "
                                           f"(70%) + uniform", "ms_per_step": rs["ms_per_step"],
                               "interactions_per_step": rs["inter"],
                               "interactions_per_s": rs["inter"] / (rs["ms_per_step"] * 1e-3), "walk_ms": rs["ms_walk"],
                               "walk_interactions_per_s": rs["inter"] / (rs["ms_walk"] * 1e-3),
                               "roofline_frac": FLOPS_PER_INTERACTION * rs["inter"] / (rs["ms_walk"] * 1e-3) / 1e12
                               / PEAK_FP32_VECTOR_TFLOPS}
        rs["ctx"].close()
        del rs
    if not args.no_batched:
        log("many-box workload: one batched call against the single-box loop")
        out["batched"] = batched(ngr, synth)
        log(f"batched: {out['batched']['ms_per_batch']:.1f} ms per batch, loop {out['batched']['loop_ms']:.1f} ms")
    if not args.no_served:
        log(f"served workload: {args.serve_requests} requests")
        out["served"] = served(ngr, synth, nreq=args.serve_requests)
        log("served: " + json.dumps({k: v for k, v in out["served"].items() if k.startswith(("load", "satur"))}))
    if not args.no_pm:
        log("PM long-range force of the benchmark box")
        out["pm"] = pm_leg(ngr, synth, p, tensors)
        log(f"pm: {out['pm']['ms_per_force']:.1f} ms per force, mesh {out['pm']['N']}^3")
    log("exact short-range tables")
    out["short_tables"] = short_tables(ngr, synth)
    log(f"short-range tables: {out['short_tables']['ms']:.2f} ms")
    if not args.no_accumulator:
        log("accumulator laws: two-species workload")
        out["accumulator"] = accumulator(ngr, synth)
        log(f"accumulator: walk {out['accumulator']['walk_ms']:.2f} ms, "
            f"{out['accumulator']['cored_walk_over_table_walk']:.2f}x the table-law walk")
    ctx.close()
    if not args.no_cpu_baseline:
        log("oracle baseline on the host cores (and the tree-vs-direct accuracy on 2^16 sinks)")
        out["cpu_baseline"], accu = cpu_baseline(p, gpu_gc, gpu_acc, args.cpu_seconds, acc_rel)
        if accu is not None:
            out["accuracy"] = accu
            log(f"accuracy: p99 {accu['p99_rel_err_tree_vs_direct']:.3e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
