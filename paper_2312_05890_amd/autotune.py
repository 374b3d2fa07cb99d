"""Tile-shape autotuner of the LDS-staged bound kernel, with a JSON cache.

The bound kernel's tile shape (nt 16-box N tiles per workgroup, uw output tiles per wavefront per
layer, nw wavefronts per workgroup) trades LDS footprint, registers and latency hiding; which
shape is fastest depends on the input dimension (state columns) and on the hidden tiles
(mt_max = ceil(max hidden width / 16)).  ``tune`` times every instantiated shape that covers the
network's tiles on a launch of random boxes and keeps the fastest; ``save``/``load`` keep the
choices in a JSON file keyed by (d, mt_max) and install them with ``bound_tile_shape`` (the
library maps d to its column class).  Results never depend on the shape, only speed does.

Usage:  python -m paper_2312_05890_amd.autotune [--out FILE] [--boxes N]
tunes the shapes of the benchmark networks and writes the cache (default: tile_cache.json next
to this file), which ``load()`` installs.
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import slrcount as S

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")
SHAPES: Tuple[Tuple[int, int, int], ...] = ((4, 1, 4), (2, 1, 4), (1, 1, 4), (1, 2, 4),
                                            (1, 1, 8), (1, 4, 4), (1, 2, 8))


def mt_of(sizes: Sequence[int]) -> int:
    return max((w + 15) // 16 for w in sizes[1:-1])


def key(d: int, mt: int) -> str:
    return f"d{d}_mt{mt}"


def candidates(d: int, mt: int) -> List[Tuple[int, int, int]]:
    """Shapes the library accepts for this class (it validates; rejected ones are skipped)."""
    out = []
    for nt, uw, nw in SHAPES:
        if mt * nt > uw * nw:
            continue
        try:
            S.bound_tile_shape(d, mt, nt, uw, nw)
        except S.SlrError:
            continue
        out.append((nt, uw, nw))
    S.bound_tile_shape(d, mt, 0, 0, 0)
    return out


def _time_launches(net, prop, lo, hi, reps: int) -> float:
    import torch
    # bounds only (no classes, hence no FP64 re-decision): the bound kernel alone
    S.bound_boxes(net, prop, lo, hi, want_cls=False)   # warm-up (and LDS attribute)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        S.bound_boxes(net, prop, lo, hi, want_cls=False)
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) * 1e3 / reps   # microseconds per launch


def tune(layers, C, dvec, lo, hi, boxes: int = 65536, reps: int = 5, seed: int = 0) -> Dict:
    """Time every candidate shape for one network on ``boxes`` random boxes inside [lo, hi]
    (widths up to 1/16 of the domain); returns the cache entry and installs the winner."""
    import torch
    net = S.Net(layers)
    prop = S.Property(net, C, dvec)
    d = net.d
    mt = mt_of(net.sizes)
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    w = (hi - lo) / 16 * rng.uniform(0, 1, size=(boxes, d))
    a = lo + (hi - lo - w) * rng.uniform(0, 1, size=(boxes, d))
    blo = torch.from_numpy(a.astype(np.float32)).cuda()
    bhi = torch.from_numpy(np.maximum((a + w).astype(np.float32), a.astype(np.float32))).cuda()
    timings = {}
    for shape in candidates(d, mt):
        S.bound_tile_shape(d, mt, *shape)
        try:
            timings[shape] = _time_launches(net, prop, blo, bhi, reps)
        except S.SlrError:
            continue
    S.bound_tile_shape(d, mt, 0, 0, 0)
    if not timings:
        raise RuntimeError(f"no tile shape runs for d={d}, mt_max={mt}")
    best = min(timings, key=timings.get)
    S.bound_tile_shape(d, mt, *best)
    return {"key": key(d, mt), "d": d, "mt_max": mt, "best": list(best),
            "us_per_launch": {"%d,%d,%d" % s: round(t, 2) for s, t in timings.items()},
            "boxes_per_launch": boxes}


def save(entries: Sequence[Dict], path: str = CACHE) -> None:
    data = {"device": "gfx950", "entries": {e["key"]: e for e in entries}}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(path: str = CACHE) -> int:
    """Install the cached shapes; returns how many were installed (0 without a cache)."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for e in data.get("entries", {}).values():
        try:
            S.bound_tile_shape(int(e["d"]), int(e["mt_max"]), *[int(x) for x in e["best"]])
            n += 1
        except (S.SlrError, KeyError, ValueError):
            continue
    return n


def _bench_networks(seed: int = 0):
    """The benchmark networks: the 5-50x6-5 exact count and one network per (d, width) of the
    256-instance batch (each class tuned once)."""
    import synth
    nets = [synth.acas(seed)]
    seen = set()
    for inst in synth.batch(seed):
        k = (inst.sizes[0], mt_of(inst.sizes))
        if k not in seen:
            seen.add(k)
            nets.append(inst)
    return nets


def main():
    ap = argparse.ArgumentParser(description="tune the bound kernel's tile shapes")
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--boxes", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    entries = []
    for inst in _bench_networks():
        e = tune(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, args.boxes, args.reps)
        entries.append(e)
        print(json.dumps(e), flush=True)
    save(entries, args.out)
    print(f"wrote {len(entries)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
