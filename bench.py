#!/usr/bin/env python3
"""Throughput of the exact #DNN-Verification count (Alg. 1 with SLR) on one MI355X.

One step = one complete ``count_exact`` on the 5-input, 6x50 ReLU network (He-normal, seed 0)
over [0,1]^5 with the unsafe property y0 - y1 > 0, max depth 40, a 2^20-leaf budget and
65536-box bound launches: every level of the branch-and-bound tree is bounded, classified,
compacted and bisected on the GPU, and the exact leaf volumes are summed.  The network, the
property and the workspace are resident in HBM before the timed region starts.

Prints one JSON line: ``value`` is boxes bounded per second (whole job), ``ms_per_step`` the
time to the final bracket; ``roofline`` rates the bound kernel (the dominant kernel) against
the FP32 MFMA peak from its HIP-event-timed launches; ``cpu_baseline`` times the FP64 oracle
on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "boxes bounded/s + time-to-exact unsafe volume, plain vs batched+α on 1 GPU"
PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0           # GB/s
ALPHA_SELECT = 0.2          # alpha only on boxes within 20% of their bound width from a decision
ALPHA_MIN_DEPTH_BATCH = 8   # first alpha level of the batched-plus-alpha count


def flops_per_box(sizes, rows):
    """Algorithmic flops of the bound kernel per box (contractions only).

    First layer: d multiply-adds for the center and d multiplies for the slopes per neuron
    (3 d flops); each hidden-to-hidden layer: the center equation (d + 1 columns) times W and
    the radius (1 column) times |W|, 2 n_in n_out (d + 2) flops; the folded output rows the same
    with n_out = rows.
    """
    d = sizes[0]
    f = 3 * d * sizes[1]
    hidden = sizes[1:-1]
    for a, b in zip(hidden[:-1], hidden[1:]):
        f += 2 * a * b * (d + 2)
    f += 2 * hidden[-1] * rows * (d + 2)
    return f


def alpha_flops_per_box_step(sizes, rows):
    """Algorithmic flops of one projected-Adam step of one box in alpha mode (contractions only).

    With its own lower slopes a neuron carries two full equations (center and radius, d + 1
    coefficients each), so every hidden-to-hidden layer costs 4 n_in n_out (d + 1) flops forward
    (W times the centers, |W| times the radii) and the same again in the adjoint (W^T, |W|^T);
    the folded output rows likewise with n_out = rows; the first layer 2 d n_1 (centers only).
    """
    d = sizes[0]
    hidden = sizes[1:-1]
    f = 0
    for a, b in zip(hidden[:-1], hidden[1:]):
        f += 4 * a * b * (d + 1)
    f += 4 * hidden[-1] * rows * (d + 1)
    return 2 * f + 2 * d * sizes[1]


def bytes_per_box(d):
    """Algorithmic HBM bytes of the bound kernel per box: corners in, class out."""
    return 2 * d * 4 + 1


KERNEL_SOURCES = ("paper_2312_05890_amd/csrc/slr_device.h", "paper_2312_05890_amd/csrc/slr_kernels.hip")


def kernel_source_hash():
    """Hash of the bound kernel's sources: counter readings taken on other code are stale."""
    m = hashlib.sha256()
    for f in KERNEL_SOURCES:
        m.update(open(os.path.join(ROOT, f), "rb").read())
    return m.hexdigest()[:16]


def measured_traffic(shape):
    """HBM bytes per bound launch from the committed rocprofv3 counter summary, if it was taken
    on the same kernel sources and tile shape."""
    path = os.path.join(ROOT, "profiles", "bound_f32_acas_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if list(rec.get("tile_shape", [])) != list(shape):
        return None
    return rec.get("bytes_per_launch")


def split_report(res):
    """The HBM-bound split kernel of the levels the search continued from: algorithmic bytes
    (every class byte, the undecided parents' corners and paths, two children each, per-tile
    counts) over its HIP-event time, against the 8 TB/s HBM peak.  Taken on a count after the
    timed steps: its events would add to the timed region."""
    ms = sum(r["split_ms"] for r in res)
    nbytes = sum(r["split_bytes"] for r in res)
    if ms <= 0:
        return None
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM, "unit": "GB/s",
            "frac": gbps / PEAK_HBM, "ms_per_step": ms / len(res),
            "bytes_per_step": nbytes // len(res)}


def cpu_baseline(seed, leaves):
    """The FP64 oracle, untuned, on the same network with a smaller leaf budget: once with the
    BLAS thread pool at its default (all the threads it takes on this host; os.cpu_count() is
    recorded beside it) and once on one thread."""
    from oracle import count
    import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    inst = synth.acas(seed)

    def run():
        t0 = time.perf_counter()
        r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, inst.max_depth,
                              leaves)
        return r, time.perf_counter() - t0

    r, dt = run()
    with threadpool_limits(limits=1):
        r1, dt1 = run()
    return {"value": r["n_boxes_bounded"] / dt, "unit": "boxes/s", "cores": cores,
            "kind": "oracle",
            "sample": f"FP64 NumPy oracle count_exact on the same network and property with a "
                      f"{leaves}-leaf budget ({r['n_boxes_bounded']} boxes, levels 0-"
                      f"{r['depth_reached']}), {dt:.1f} s",
            "host_cpu_count": os.cpu_count(),
            "one_core": {"value": r1["n_boxes_bounded"] / dt1, "unit": "boxes/s", "cores": 1,
                         "seconds": dt1}}


def bench_alpha_optimize(E, torch, inst, n, steps, seed, reps=3):
    """alpha_optimize on n boxes of the workload's domain (widths up to 1/16 of the domain):
    one init pass, then steps x (adjoint with fused Adam, forward)."""
    import synth
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    lo, hi = synth.uniform_boxes(inst.lo, inst.hi, n, seed + 101, 1.0 / 16)
    lo = torch.from_numpy(lo).cuda()
    hi = torch.from_numpy(hi).cuda()
    ws = torch.empty(E.alpha_workspace_size(net, prop, n), dtype=torch.uint8, device="cuda")
    E.alpha_optimize(net, prop, lo, hi, steps=steps, workspace=ws)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        r = E.alpha_optimize(net, prop, lo, hi, steps=steps, workspace=ws)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    fps = alpha_flops_per_box_step(inst.sizes, inst.C.shape[0])
    achieved = n * steps * fps / (ms * 1e-3) / 1e12
    cls = r["cls"].cpu().numpy()
    return {"boxes": n, "steps": steps, "ms": ms, "alpha_boxes_per_s": n / (ms * 1e-3),
            "flops_per_box_step": fps, "achieved_tflops": achieved,
            "frac_fp32_mfma": achieved / PEAK_FP32_MFMA,
            "decided": int((cls != 0).sum())}


def bench_count(E, torch, inst, D, M, alpha_steps=0, min_depth=0, reps=1, select=0.0):
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    achunk = 16384 if alpha_steps else 0
    ws = torch.empty(E.workspace_size(net, prop, M, 0, achunk), dtype=torch.uint8, device="cuda")
    kw = dict(workspace=ws, alpha_steps=alpha_steps, alpha_min_depth=min_depth,
              alpha_chunk=achunk, alpha_select=select)
    E.count_exact(net, prop, inst.lo, inst.hi, D, M, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = E.count_exact(net, prop, inst.lo, inst.hi, D, M, **kw)
    dt = (time.perf_counter() - t0) / reps
    return {"time_to_bracket_ms": dt * 1e3, "bracket": [r["unsafe"], r["unsafe"] + r["undecided"]],
            "boxes_bounded": r["n_boxes_bounded"], "depth_reached": r["depth_reached"],
            "alpha_boxes": r["n_alpha_boxes"], "alpha_decided": r["n_alpha_decided"],
            "boxes_per_s": r["n_boxes_bounded"] / dt}


def cpu_alpha_baseline(inst, n, steps, seed):
    """The FP64 torch oracle of the alpha mode (forward + autograd + Adam), untuned."""
    import synth
    from oracle import alpha as oalpha
    import torch
    lo, hi = synth.uniform_boxes(inst.lo, inst.hi, n, seed + 101, 1.0 / 16)
    t0 = time.perf_counter()
    oalpha.optimize(inst.net, inst.C, inst.dvec, lo, hi, steps=steps)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "alpha-optimized boxes/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"FP64 torch oracle, {n} boxes x {steps} Adam steps, {dt:.1f} s"}


def batch_section(E, torch, seed, reps=3):
    """256 uneven instances (d 5..10, 3..6 hidden layers of 32..128, 2..5 outputs, random
    linear property, depth 4 d, 2^16 leaves each) counted as one batch (captured graph, and the
    same launches issued directly) and one instance at a time with count_exact."""
    import synth
    insts = synth.batch(seed)
    items = []
    for inst in insts:
        net = E.Net(inst.net)
        items.append((net, E.Property(net, inst.C, inst.dvec), inst.lo, inst.hi,
                      inst.max_depth, inst.max_leaves))
    t0 = time.perf_counter()
    b = E.Batch(items, use_graph=True)
    t_create = time.perf_counter() - t0
    res = b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = b.run()
    t_graph = (time.perf_counter() - t0) / reps
    d = E.Batch(items, use_graph=False)
    d.run()
    t0 = time.perf_counter()
    d.run()
    t_direct = time.perf_counter() - t0
    ws_bytes = max(E.workspace_size(it[0], it[1], it[5]) for it in items)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    E.count_exact(*items[0][:4], items[0][4], items[0][5], workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [E.count_exact(*it[:4], it[4], it[5], workspace=ws) for it in items]
    t_seq = time.perf_counter() - t0
    boxes = sum(r["n_boxes_bounded"] for r in res)
    flops = sum(r["n_boxes_bounded"] * flops_per_box(inst.sizes, inst.C.shape[0])
                for r, inst in zip(res, insts))
    agree = all(r[k] == q[k] for r, q in zip(res, seq)
                for k in ("unsafe", "safe", "undecided", "n_boxes_bounded"))
    # batched plus alpha (near-decision selection, 20 Adam steps) in the same graph
    ba = E.Batch(items, use_graph=True, alpha_steps=20, alpha_min_depth=ALPHA_MIN_DEPTH_BATCH,
                 alpha_select=ALPHA_SELECT, alpha_chunk=8192)
    ra = ba.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ra = ba.run()
    t_alpha = (time.perf_counter() - t0) / reps
    inside = all(a["unsafe"] >= q["unsafe"] and a["safe"] >= q["safe"] for a, q in zip(ra, seq))
    # time to a bracket inside the plain one: the same batch plus alpha with smaller leaf
    # budgets, counting the instances whose bracket lies inside their plain 2^16-leaf bracket
    smaller = []
    for shift in (1, 2, 3):
        its = [it[:5] + (it[5] >> shift,) for it in items]
        bs = E.Batch(its, use_graph=True, alpha_steps=20, alpha_min_depth=ALPHA_MIN_DEPTH_BATCH,
                     alpha_select=ALPHA_SELECT, alpha_chunk=8192)
        rs = bs.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = bs.run()
        ts = time.perf_counter() - t0
        smaller.append({"leaves": items[0][5] >> shift, "graph_ms": ts * 1e3,
                        "instances_inside_plain": sum(1 for a, q in zip(rs, seq)
                                                      if a["unsafe"] >= q["unsafe"]
                                                      and a["safe"] >= q["safe"]),
                        "speedup_vs_sequential_plain": t_seq / ts})
        del bs
    return {"workload": "256 instances: d 5..10, 3..6 hidden layers of 32/64/96/128, 2..5 "
                        "outputs, c ~ N(0,1), [0,1]^d, depth 4d, 2^16 leaves each (seed %d)" % seed,
            "boxes_per_batch": boxes, "graph_ms": t_graph * 1e3, "direct_ms": t_direct * 1e3,
            "sequential_ms": t_seq * 1e3, "create_ms": t_create * 1e3,
            "boxes_per_s_graph": boxes / t_graph, "boxes_per_s_sequential": boxes / t_seq,
            "speedup_vs_sequential": t_seq / t_graph,
            "achieved_tflops_graph": flops / t_graph / 1e12,
            "results_equal_sequential": agree,
            "instances_resolved": sum(1 for r in res if r["undecided"] == 0.0),
            "batched_alpha": {
                "options": "20 Adam steps from depth %d on boxes within %.1f of a decision, "
                           "8192 boxes per alpha class and level" % (ALPHA_MIN_DEPTH_BATCH,
                                                                      ALPHA_SELECT),
                "graph_ms": t_alpha * 1e3,
                "speedup_vs_sequential_plain": t_seq / t_alpha,
                "brackets_inside_plain": inside,
                "alpha_boxes": sum(r["n_alpha_boxes"] for r in ra),
                "alpha_decided": sum(r["n_alpha_decided"] for r in ra),
                "unsafe_volume_sum": sum(r["unsafe"] for r in ra),
                "unsafe_volume_sum_plain": sum(r["unsafe"] for r in seq),
                "safe_volume_sum": sum(r["safe"] for r in ra),
                "safe_volume_sum_plain": sum(r["safe"] for r in seq),
                "smaller_budgets": smaller}}


def split_section(E, torch, inst, reps=3):
    """The headline count with the crossing-score split rule (first one and two hidden layers)
    beside the widest-side rule: same leaf budget, brackets and time."""
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    ws = torch.empty(E.workspace_size(net, prop, inst.max_leaves), dtype=torch.uint8, device="cuda")
    out = {}
    for k in (0, 1, 2):
        E.count_exact(net, prop, inst.lo, inst.hi, inst.max_depth, inst.max_leaves, chunk=65536,
                      workspace=ws, split_layers=k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = E.count_exact(net, prop, inst.lo, inst.hi, inst.max_depth, inst.max_leaves,
                              chunk=65536, workspace=ws, split_layers=k)
        dt = (time.perf_counter() - t0) / reps
        out["split_layers_%d" % k] = {"time_to_bracket_ms": dt * 1e3,
                                      "bracket": [r["unsafe"], r["unsafe"] + r["undecided"]],
                                      "boxes_bounded": r["n_boxes_bounded"],
                                      "depth_reached": r["depth_reached"]}
    return out


def resolve_section(E, torch, count=256, depth=16, leaves=1 << 16, reps=3):
    """Time to the exact count where the search resolves: ``count`` instances of the 2-16-16-1
    network (seeds 0..count-1, [-1,1]^2, y > 0, depth 16) counted one at a time with
    count_exact, as one batch, and as one batch with the near-decision alpha pass; total time,
    boxes bounded and the summed undecided volume (what is left between the bracket's ends)."""
    import synth
    items = []
    for seed in range(count):
        inst = synth.tiny2d(seed)
        net = E.Net(inst.net)
        items.append((net, E.Property(net, inst.C, inst.dvec), inst.lo, inst.hi, depth, leaves))
    ws = torch.empty(max(E.workspace_size(it[0], it[1], it[5]) for it in items), dtype=torch.uint8,
                     device="cuda")

    def summary(res, dt):
        return {"ms": dt * 1e3, "boxes_bounded": sum(r["n_boxes_bounded"] for r in res),
                "undecided_volume_sum": sum(r["undecided"] for r in res),
                "unsafe_volume_sum": sum(r["unsafe"] for r in res)}

    E.count_exact(*items[0][:4], depth, leaves, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [E.count_exact(*it[:4], depth, leaves, workspace=ws) for it in items]
    out = {"workload": "%d x 2-16-16-1 ReLU (seeds 0..%d), [-1,1]^2, y > 0, depth %d, 2^%d leaves"
                       % (count, count - 1, depth, leaves.bit_length() - 1),
           "sequential_count_exact": summary(seq, time.perf_counter() - t0)}
    for name, kw in (("batch", {}),
                     ("batch_alpha", dict(alpha_steps=5, alpha_min_depth=6, alpha_select=ALPHA_SELECT,
                                          alpha_chunk=1 << 16)),
                     ("batch_alpha_late", dict(alpha_steps=2, alpha_min_depth=12,
                                               alpha_select=ALPHA_SELECT, alpha_chunk=1 << 16))):
        b = E.Batch(items, use_graph=True, **kw)
        res = b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = b.run()
        out[name] = summary(res, (time.perf_counter() - t0) / reps)
        out[name]["brackets_inside_plain"] = all(
            r["unsafe"] >= q["unsafe"] and r["unsafe"] + r["undecided"] <= q["unsafe"] + q["undecided"]
            for r, q in zip(res, seq))
    return out


def relax_section(E, torch, inst, reps=3):
    """The headline count with the two-ratio relaxation (tape-state kernel, widened float32
    classes) beside Eq. 1: same leaf budget, brackets and time."""
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    out = {}
    for relax in ("one", "two"):
        kw = dict(chunk=65536, relax=relax)
        E.count_exact(net, prop, inst.lo, inst.hi, inst.max_depth, inst.max_leaves, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = E.count_exact(net, prop, inst.lo, inst.hi, inst.max_depth, inst.max_leaves, **kw)
        dt = (time.perf_counter() - t0) / reps
        out["relax_" + relax] = {"time_to_bracket_ms": dt * 1e3,
                                 "bracket": [r["unsafe"], r["unsafe"] + r["undecided"]],
                                 "boxes_bounded": r["n_boxes_bounded"],
                                 "depth_reached": r["depth_reached"]}
    return out


def stack_section(E, torch, seed, depth=24, reps=2):
    """count_exact_stack (depth-first chunks, no leaf budget) on the same network past the
    2^20-leaf budget of the headline count."""
    import synth
    inst = synth.acas(seed)
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    ws = torch.empty(E.stack_workspace_size(net, prop, depth), dtype=torch.uint8, device="cuda")
    E.count_exact_stack(net, prop, inst.lo, inst.hi, depth, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = E.count_exact_stack(net, prop, inst.lo, inst.hi, depth, workspace=ws)
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "count_exact_stack, 5-50x6-5 network (seed %d), [0,1]^5, depth %d, "
                        "no leaf budget, 65536-box chunks" % (seed, depth),
            "time_to_bracket_ms": dt * 1e3, "boxes_bounded": r["n_boxes_bounded"],
            "boxes_per_s": r["n_boxes_bounded"] / dt,
            "bracket": [r["unsafe"], r["unsafe"] + r["undecided"]],
            "workspace_mb": ws.numel() / 1e6}


def approx_section(E, torch, seed, cpu):
    """CountingProVe with SLR leaves on the 22-input network (22-64x3-3, y2 strict argmax,
    [0,1]^22): 20 trials, 1000 samples per split, 99% confidence, leaf counts of depth 48 and
    2^16 leaves; the FP64 oracle on a bounded sample of the same procedure beside it."""
    import synth
    inst = synth.nav22(seed)
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    kw = dict(trials=20, samples=1000, confidence=0.99, seed=seed, max_splits=300, grid_bits=16,
              resolve_tol=0.01, leaf_depth=48, leaf_leaves=1 << 16)
    E.count_approx(net, prop, inst.lo, inst.hi, **dict(kw, trials=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = E.count_approx(net, prop, inst.lo, inst.hi, **kw)
    dt = time.perf_counter() - t0
    small = dict(kw, trials=1, leaf_leaves=1 << 10, max_splits=12)
    t0 = time.perf_counter()
    rs = E.count_approx(net, prop, inst.lo, inst.hi, **small)
    dts = time.perf_counter() - t0
    out = {"workload": "count_approx, 22-64x3-3 network (seed %d), [0,1]^22, unsafe iff y2 is the "
                       "strict argmax, 20 trials x 1000 samples, 99%% confidence, <= 300 splits, "
                       "leaves: depth 48, 2^16 leaves, resolved at <= 1%% undecided" % seed,
           "seconds": dt,
           "lower_bound": r["lower_bound"],
           "mean_estimate": sum(r["estimates"]) / len(r["estimates"]),
           "splits": r["splits"],
           "small_sample": {"params": "1 trial, 2^10-leaf leaf counts, <= 12 splits",
                            "seconds": dts, "estimate": rs["estimates"][0],
                            "splits": rs["splits"][0]}}
    if cpu:
        from oracle import count
        t0 = time.perf_counter()
        o = count.count_approx(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, trials=1,
                               samples=1000, confidence=0.99, seed=seed, leaf_depth=48,
                               leaf_leaves=1 << 10, resolve_tol=0.01, max_splits=12,
                               grid_bits=16)
        dto = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / dto, "unit": "trials/s (small sample)",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": "FP64 oracle count_approx, the small-sample parameters, "
                                         "%.1f s, estimate %.6g" % (dto, o["estimates"][0])}
        out["small_sample"]["gpu_trials_per_s"] = 1.0 / dts
    return out


def alpha_section(E, torch, seed, cpu):
    import synth
    a5 = synth.acas(seed)
    b5 = synth.wide20(seed)
    out = {
        "acas_optimize": bench_alpha_optimize(E, torch, a5, 65536, 20, seed),
        "wide20_optimize": bench_alpha_optimize(E, torch, b5, 4096, 20, seed),
        "acas_count_plain": bench_count(E, torch, a5, a5.max_depth, a5.max_leaves),
        "acas_count_alpha": bench_count(E, torch, a5, a5.max_depth, a5.max_leaves, 20, 16),
        "acas_count_alpha_near": bench_count(E, torch, a5, a5.max_depth, a5.max_leaves, 20, 16,
                                             select=ALPHA_SELECT),
        "wide20_count_plain": bench_count(E, torch, b5, b5.max_depth, 1 << 14),
        "wide20_count_alpha": bench_count(E, torch, b5, b5.max_depth, 1 << 14, 20, 8),
        "wide20_count_alpha_near": bench_count(E, torch, b5, b5.max_depth, 1 << 14, 20, 8,
                                               select=ALPHA_SELECT),
    }
    if cpu:
        out["cpu_baseline"] = cpu_alpha_baseline(a5, 32, 20, seed)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-leaves", type=int, default=1 << 15)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-alpha", action="store_true",
                    help="skip the alpha-mode measurements (optimizer throughput, counts with alpha)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-instances measurement")
    ap.add_argument("--no-approx", action="store_true",
                    help="skip the approximate-count measurement")
    ap.add_argument("--no-stack", action="store_true",
                    help="skip the depth-first stack count past the leaf budget")
    ap.add_argument("--no-tile-cache", action="store_true",
                    help="ignore the autotuner's tile-shape cache (default shapes)")
    ap.add_argument("--variant", type=int, default=0,
                    help="bound kernel: 0 automatic, 1 LDS-staged, 2 register-resident")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy a tensor of this many MiB once (a plain copy kernel of "
                         "known size, for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {args.gpus}); the "
              "multi-GPU split of the frontier is described but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    import synth
    import paper_2312_05890_amd as E

    from paper_2312_05890_amd import autotune
    tuned = 0 if args.no_tile_cache else autotune.load()
    E.bound_kernel_variant(args.variant)
    inst = synth.acas(args.seed)
    shape = E.slrcount.current_tile_shape(inst.sizes)
    net = E.Net(inst.net)
    prop = E.Property(net, inst.C, inst.dvec)
    chunk = 65536
    ws = torch.empty(E.workspace_size(net, prop, inst.max_leaves), dtype=torch.uint8,
                     device="cuda")

    def step(timing):
        return E.count_exact(net, prop, inst.lo, inst.hi, inst.max_depth, inst.max_leaves,
                             chunk=chunk, workspace=ws, timing=timing)

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    boxes = sum(r["n_boxes_bounded"] for r in res)
    fpb = flops_per_box(inst.sizes, inst.C.shape[0])
    bound_s = sum(r["bound_ms"] for r in res) / 1e3
    launches = sum(r["bound_launches"] for r in res)
    achieved = boxes * fpb / bound_s / 1e12
    traffic = measured_traffic(shape)
    r0 = res[-1]
    line = {
        "metric": METRIC,
        "value": boxes / dt,
        "unit": "boxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "exact count, 5-50x6-5 ReLU MLP (He-normal seed %d), [0,1]^5, "
                               "unsafe iff y0-y1>0, max depth 40, 2^20-leaf budget, 65536-box "
                               "launches" % args.seed,
                   "mode": "plain", "kernel_variant": args.variant,
                   "tile_shape": list(shape), "tile_cache_entries": tuned},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": traffic},
        "bound_kernel": {"flops_per_box": fpb, "bytes_per_box": bytes_per_box(inst.sizes[0]),
                         "avg_launch_us": bound_s / launches * 1e6,
                         "launches_per_step": launches // args.steps,
                         "boxes_per_s": boxes / bound_s},
        "split_kernel": split_report([step(2)]),
        "time_to_bracket_ms": r0["seconds"] * 1e3,
        "bracket": [r0["unsafe"], r0["unsafe"] + r0["undecided"]],
        "boxes_per_step": r0["n_boxes_bounded"],
        "depth_reached": r0["depth_reached"],
        "recheck64_per_step": r0["n_recheck64"],
    }
    if not args.no_batch:
        line["batch"] = batch_section(E, torch, args.seed)
        line["resolving"] = resolve_section(E, torch)
    if not args.no_stack:
        line["stack"] = stack_section(E, torch, args.seed)
        line["split_rule"] = split_section(E, torch, inst)
        line["relaxation"] = relax_section(E, torch, inst)
    if not args.no_approx:
        line["approx"] = approx_section(E, torch, args.seed, not args.no_cpu_baseline)
    if not args.no_alpha:
        line["alpha"] = alpha_section(E, torch, args.seed, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.seed, args.cpu_leaves)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
