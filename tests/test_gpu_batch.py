"""Batched exact counts on the GPU, through the C ABI.

The batch runs the same bound tile, FP64 re-decision and bookkeeping code as the single-instance
count, so every instance's result must equal its own ``count_exact`` bit for bit; the single
instance path is pinned to the oracle elsewhere, and a few small instances are compared with the
oracle here as well.  Graph replays are compared with each other and with direct launches, with
unrelated device work and synchronizations between the replays.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import synth
from oracle import count

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("unsafe", "safe", "undecided", "n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded",
        "n_recheck64", "depth_reached", "status")


def E():
    import paper_2312_05890_amd as eng
    return eng


def items_of(insts, depth=None, leaves=None):
    eng = E()
    out = []
    for inst in insts:
        net = eng.Net(inst.net)
        prop = eng.Property(net, inst.C, inst.dvec)
        out.append((net, prop, inst.lo, inst.hi,
                    inst.max_depth if depth is None else depth,
                    inst.max_leaves if leaves is None else leaves))
    return out


def single(it):
    net, prop, lo, hi, D, M = it
    return E().count_exact(net, prop, lo, hi, D, M)


def same(a, b):
    return all(a[k] == b[k] for k in KEYS)


def test_batch_equals_single_instance_counts():
    insts = synth.batch(0, count=24)
    items = items_of(insts, leaves=1 << 12)
    res = E().count_exact_batch(items)
    for it, r in zip(items, res):
        s = single(it)
        assert same(r, s), (r, s)
        assert r["unsafe"] + r["safe"] + r["undecided"] == 1.0


def test_batch_graph_replays_agree():
    insts = synth.batch(1, count=16)
    items = items_of(insts, leaves=1 << 11)
    b = E().Batch(items, use_graph=True)
    ref = E().count_exact_batch(items)
    x = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        res = b.run()
        for r, q in zip(res, ref):
            assert same(r, q), (rep, r, q)
        # unrelated eager work between replays
        x = (x * 1.0001).sin()
        torch.cuda.synchronize()
    d = E().Batch(items, use_graph=False)
    for r, q in zip(d.run(), ref):
        assert same(r, q)


def _one_per_shape(side_log2):
    """The first instance of the 256-instance generator (seed 0) for every pair (inputs d,
    hidden width), 6 x 4 = 24 instances covering every column class and width of the batch.
    Each is restricted to a dyadic sub-box of side 2^-side_log2 at a corner drawn from
    default_rng(instance index): on the whole unit cube these deep random networks decide no
    box within a small leaf budget, on such sub-boxes they decide unsafe and safe boxes."""
    seen = {}
    for i, inst in enumerate(synth.batch(0)):
        seen.setdefault((inst.sizes[0], inst.sizes[1]), (i, inst))
    out = []
    for k in sorted(seen):
        i, inst = seen[k]
        d = inst.sizes[0]
        c = np.floor(np.random.default_rng(i).uniform(0, 1, size=d) * 2 ** side_log2)
        c = c / 2 ** side_log2
        out.append(dataclasses.replace(inst, name=f"batch{i}-d{d}w{inst.sizes[1]}",
                                       lo=c, hi=c + 2.0 ** -side_log2))
    return out


@pytest.mark.parametrize("side_log2", [4, 5])
def test_batch_of_all_shapes_equals_oracle(side_log2):
    """Every (inputs, width) shape of the batch workload, on a 2^-4 and a 2^-5 sub-box, at depth
    4 d with a 2^11-leaf budget: ``count_exact`` is compared box by box with the oracle
    (matched on depth and path id, classes equal wherever the oracle's margin exceeds 1e-5,
    identical leaf counts and volumes unless such a box explains the difference), and the same
    instances run as one batch give the oracle's counts and volumes exactly (or differ in unsafe
    volume by at most the volume of the boxes that explain a difference)."""
    from tests.test_gpu_parity import compare_counts
    insts = _one_per_shape(side_log2)
    items = items_of(insts, leaves=1 << 11)
    res = E().Batch(items).run()
    decided = 0
    for inst, it, r in zip(insts, items, res):
        _, o, diverge = compare_counts(inst, it[4], it[5])
        decided += o["n_unsafe"] + o["n_safe"]
        if not diverge:
            for k in ("n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded", "depth_reached",
                      "status", "unsafe", "safe", "undecided"):
                assert r[k] == o[k], (inst.name, k, r[k], o[k])
        else:
            assert abs(r["unsafe"] - o["unsafe"]) <= sum(2.0 ** -k[0] for k in diverge)
    assert decided > 1000


def test_batch_mixed_shapes_and_budgets_against_oracle():
    insts = [synth.tiny2d(0), synth.tiny2d(3), synth.acas(1)] + synth.batch(2, count=3)
    depth = [12, 10, 30, 12, 14, 16]
    leaves = [1 << 12, 1 << 10, 1 << 10, 1 << 10, 1 << 9, 1 << 10]
    items = []
    eng = E()
    for inst, D, M in zip(insts, depth, leaves):
        net = eng.Net(inst.net)
        items.append((net, eng.Property(net, inst.C, inst.dvec), inst.lo, inst.hi, D, M))
    res = eng.Batch(items).run()
    from tests.test_gpu_parity import compare_counts
    for inst, it, r in zip(insts, items, res):
        assert same(r, single(it))
        _, o, diverge = compare_counts(inst, it[4], it[5])
        if not diverge:
            for k in ("n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded", "unsafe",
                      "safe", "undecided", "depth_reached", "status"):
                assert r[k] == o[k], (inst.name, k, r[k], o[k])
        else:
            assert abs(r["unsafe"] - o["unsafe"]) <= sum(2.0 ** -k[0] for k in diverge)


def _level_loop(it):
    """``count_exact`` with the level-by-level driver for every depth (timing bit 2: no one-pass
    top of the tree)."""
    net, prop, lo, hi, D, M = it
    return E().count_exact(net, prop, lo, hi, D, M, timing=4)


def test_batch_top_of_tree_equals_level_loop():
    """Instances whose counts end inside the batch's first level (the complete subtree of depth
    pk, replayed depth by depth) or right after it, and instances without one: nothing left
    undecided (2-input sub-boxes), the depth limit at pk (depth 5, 4), the leaf budget at pk
    (63 = 2^6 - 1 leaves), no top at all (depth 3, 30 leaves), and ordinary counts past it;
    every result, including the number of FP64 re-decisions, equals the level-by-level
    driver's, and the resolved sub-boxes' volumes are the oracle's."""
    eng = E()
    sub = _one_per_shape(4)[:4]
    def quarter(seed, cx, cy):   # a quarter-side sub-box of a 2-input net's domain
        inst = synth.tiny2d(seed)
        lo = inst.lo + (inst.hi - inst.lo) * np.array([cx, cy]) / 4.0
        return dataclasses.replace(inst, name=f"tiny2d{seed}q{cx}{cy}", lo=lo,
                                   hi=lo + (inst.hi - inst.lo) / 4.0)
    # sub-boxes that the oracle resolves completely at depths 9, 9 and 8
    cases = [(quarter(1, 2, 1), 16, 1 << 16), (quarter(1, 3, 0), 16, 1 << 16),
             (quarter(0, 0, 1), 16, 1 << 16)]
    cases += [(synth.tiny2d(s), 16, 1 << 16) for s in (0, 3)]
    cases += [(synth.acas(0), 5, 1 << 12), (synth.acas(1), 4, 1 << 12), (synth.acas(2), 20, 63),
              (synth.acas(0), 3, 1 << 12), (synth.acas(1), 12, 30), (synth.acas(2), 10, 1 << 10)]
    cases += [(inst, 4 * inst.sizes[0], 1 << 11) for inst in sub]
    items = []
    for inst, D, M in cases:
        net = eng.Net(inst.net)
        items.append((net, eng.Property(net, inst.C, inst.dvec), inst.lo, inst.hi, D, M))
    for use_graph in (True, False):
        res = eng.Batch(items, use_graph=use_graph).run()
        for (inst, D, M), it, r in zip(cases, items, res):
            ref = _level_loop(it)
            assert same(r, ref), (inst.name, D, M, r, ref)
            assert same(single(it), ref), (inst.name, D, M)
    for (inst, D, M), r in list(zip(cases, res))[:3]:
        o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, D, M)
        assert o["status"] == 0 and o["undecided"] == 0.0
        for k in ("unsafe", "safe", "undecided", "n_boxes_bounded", "depth_reached", "status"):
            assert r[k] == o[k], (inst.name, k, r[k], o[k])
    statuses = {r["status"] for r in res}
    assert len(statuses) == 2   # finished and stopped counts both occur
    assert any(r["n_recheck64"] > 0 for r in res)


def test_batch_full_config_counts():
    """256 instances: d 5..10, 3..6 hidden layers of 32..128, 2..5 outputs, depth 4 d, 2^16
    leaves each; spot-check 8 instances against single-instance counts."""
    insts = synth.batch(0)
    items = items_of(insts)
    b = E().Batch(items)
    res = b.run()
    assert len(res) == 256
    for r in res:
        assert r["unsafe"] + r["safe"] + r["undecided"] == 1.0
    for k in range(0, 256, 37):
        assert same(res[k], single(items[k]))


def test_batch_rejects_bad_input():
    eng = E()
    with pytest.raises(eng.SlrError):
        eng.count_exact_batch([])
    inst = synth.nav22(0)                     # d = 22: outside the batch kernels
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact_batch(items_of([inst]))
    assert e.value.code == -5
    inst = synth.tiny2d(0)
    with pytest.raises(eng.SlrError):
        eng.count_exact_batch(items_of([inst], leaves=(1 << 22) + 1))


ALPHA_KEYS = KEYS + ("n_alpha_boxes", "n_alpha_decided")


def _alpha_items():
    """Mixed shapes with decisions: tiny2d seeds 0-3 (depth 12), the 5-input 6x50 network
    (seed 1, depth 30, 2^12 leaves) and every (inputs, width) shape of the batch workload on
    its 2^-4 sub-box (depth 4 d, 2^11 leaves)."""
    insts = [synth.tiny2d(s) for s in range(4)] + [synth.acas(1)] + _one_per_shape(4)
    depth = [12] * 4 + [30] + [i.max_depth for i in insts[5:]]
    leaves = [1 << 12] * 5 + [1 << 11] * (len(insts) - 5)
    eng = E()
    items = []
    for inst, D, M in zip(insts, depth, leaves):
        net = eng.Net(inst.net)
        items.append((net, eng.Property(net, inst.C, inst.dvec), inst.lo, inst.hi, D, M))
    return insts, items


@pytest.mark.parametrize("select", [0.0, 0.2])
def test_batch_alpha_equals_count_exact_alpha(select):
    """The batched alpha pass (fused optimizer per tile, segments per alpha class) gives every
    instance exactly the counts, volumes, alpha boxes and alpha decisions of count_exact with the
    same alpha options, and a bracket inside the plain count's."""
    insts, items = _alpha_items()
    kw = dict(alpha_steps=5, alpha_min_depth=3, alpha_select=select)
    res = E().Batch(items, alpha_chunk=1 << 16, **kw).run()
    decided = 0
    for it, r in zip(items, res):
        net, prop, lo, hi, D, M = it
        s = E().count_exact(net, prop, lo, hi, D, M, alpha_chunk=1 << 16, **kw)
        for k in ALPHA_KEYS:
            assert r[k] == s[k], (k, r[k], s[k])
        p = single(it)
        assert r["unsafe"] >= p["unsafe"] and r["safe"] >= p["safe"]
        decided += r["n_alpha_decided"]
    assert decided > 0


def test_batch_alpha_graph_replays_and_small_chunk():
    """Graph replays equal direct launches; with room for only 16 boxes per class and level the
    counts stay sound: brackets inside the plain ones, containing the full-room alpha ones."""
    insts, items = _alpha_items()
    kw = dict(alpha_steps=4, alpha_min_depth=2, alpha_select=0.2)
    g = E().Batch(items, use_graph=True, alpha_chunk=1 << 16, **kw)
    ref = E().Batch(items, use_graph=False, alpha_chunk=1 << 16, **kw).run()
    x = torch.randn(1 << 18, device="cuda")
    for rep in range(3):
        for r, q in zip(g.run(), ref):
            assert all(r[k] == q[k] for k in ALPHA_KEYS), rep
        x = x.cos()
        torch.cuda.synchronize()
    small = E().Batch(items, alpha_chunk=16, **kw).run()
    for it, r, q in zip(items, small, ref):
        p = single(it)
        assert r["unsafe"] + r["safe"] + r["undecided"] == 1.0
        assert r["unsafe"] >= p["unsafe"] and r["safe"] >= p["safe"]
        assert r["n_alpha_boxes"] <= q["n_alpha_boxes"]


def test_batch_alpha_brackets_inside_oracle_plain():
    """Alpha brackets lie inside the FP64 oracle's plain bracket (up to boxes within 1e-5 of a
    decision, which the parity tests enumerate)."""
    insts, items = _alpha_items()
    res = E().Batch(items, alpha_steps=5, alpha_min_depth=3, alpha_select=0.2,
                    alpha_chunk=1 << 16).run()
    for inst, it, r in zip(insts[:5], items[:5], res[:5]):
        o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, it[4], it[5])
        assert r["unsafe"] >= o["unsafe"] - 2.0 ** -it[4]
        assert r["unsafe"] + r["undecided"] <= o["unsafe"] + o["undecided"] + 2.0 ** -it[4]


def test_batch_rejects_bad_alpha_options():
    insts, items = _alpha_items()
    eng = E()
    for bad in (dict(alpha_steps=-1), dict(alpha_steps=2, alpha_select=float("nan")),
                dict(alpha_steps=2, alpha_min_depth=-1), dict(alpha_steps=2, alpha_chunk=-5)):
        with pytest.raises(eng.SlrError) as e:
            eng.Batch(items[:2], **bad)
        assert e.value.code == -1
