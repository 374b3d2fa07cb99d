"""Depth-first stack count (``count_exact_stack``) on the GPU, through the C ABI.

It bounds exactly the boxes of Alg. 1 with the same depth and no leaf budget, in another order,
so it is compared with the FP64 oracle box by box (matched on depth and path id), with the
oracle's full-size fixture level by level, with ``count_exact`` at a depth beyond the 2^20-leaf
budget, and with itself when the stack spills to host memory or stops on a box budget.
"""
from __future__ import annotations

import hashlib
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import count

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("unsafe", "safe", "undecided", "n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded",
        "depth_reached", "status")


def E():
    import paper_2312_05890_amd as eng
    return eng


def load(inst):
    eng = E()
    net = eng.Net(inst.net)
    return net, eng.Property(net, inst.C, inst.dvec)


@pytest.mark.parametrize("seed", range(10))
def test_stack_matches_oracle_box_by_box(seed):
    """tiny2d, depth 16, no leaf budget: every box of the oracle's tree is bounded once, with the
    oracle's class (margin rule), in chunks of 64 boxes (many launches, mixed depths)."""
    from tests.test_gpu_parity import compare_results
    inst = synth.tiny2d(seed)
    net, prop = load(inst)
    g = E().count_exact_stack(net, prop, inst.lo, inst.hi, 16, chunk=64, trace=True,
                              trace_capacity=1 << 20)
    o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 16, 1 << 40, trace=True)
    assert g["trace_count"] == g["n_boxes_bounded"]
    compare_results(g, o)


def test_stack_matches_full_size_oracle_fixture():
    """The 5-input 6x50 network (seed 0) to depth 20: the boxes of the oracle's 2^20-leaf run
    (its budget stopped it after depth 20, so depth 20 without a budget bounds the same boxes),
    per depth the same path ids and classes (SHA-256 in canonical order) and exact volumes."""
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "acas0_d40_leaves2p20.json")))
    inst = synth.acas(0)
    net, prop = load(inst)
    g = E().count_exact_stack(net, prop, inst.lo, inst.hi, 20, trace=True,
                              trace_capacity=fx["n_boxes_bounded"] + 16)
    assert g["trace_count"] == g["n_boxes_bounded"] == fx["n_boxes_bounded"]
    td, tp, tc = g["trace_depth"], g["trace_path"], g["trace_cls"]
    for lev in fx["levels"]:
        sel = td == lev["depth"]
        order = np.argsort(tp[sel], kind="stable")
        assert hashlib.sha256(tp[sel][order].astype("<u8").tobytes()).hexdigest() == lev["path_sha256"]
        assert hashlib.sha256(tc[sel][order].astype(np.int8).tobytes()).hexdigest() == lev["cls_sha256"]
    for k in ("n_unsafe", "n_safe", "n_undecided", "depth_reached", "status"):
        assert g[k] == fx[k], k
    assert Fraction(g["unsafe"]) == Fraction(fx["unsafe_exact"])
    assert Fraction(g["undecided"]) == Fraction(fx["undecided_exact"])


def test_stack_equals_count_exact_beyond_the_leaf_budget():
    """Depth 25 on the 5-input 6x50 network (seed 0): about 3.3e7 boxes, 32x the 2^20-leaf
    budget; count_exact with a 2^26-leaf budget (a 6.8 GB frontier) visits the same tree."""
    inst = synth.acas(0)
    net, prop = load(inst)
    a = E().count_exact_stack(net, prop, inst.lo, inst.hi, 25)
    b = E().count_exact(net, prop, inst.lo, inst.hi, 25, 1 << 26)
    for k in KEYS + ("n_recheck64",):
        assert a[k] == b[k], (k, a[k], b[k])
    assert a["n_boxes_bounded"] > 30_000_000


def test_stack_spill_to_host_equals_device_only():
    """A device stack of 4 chunks of 1024 boxes spills its bottom to pinned host memory many
    times; results equal the device-only stack and count_exact without a leaf budget."""
    inst = synth.acas(1)
    net, prop = load(inst)
    D = 17
    a = E().count_exact_stack(net, prop, inst.lo, inst.hi, D, chunk=1024)
    host = torch.empty(64 << 20, dtype=torch.uint8, pin_memory=True)
    b = E().count_exact_stack(net, prop, inst.lo, inst.hi, D, chunk=1024, device_boxes=4096,
                              host_spill=host)
    c = E().count_exact(net, prop, inst.lo, inst.hi, D, 1 << 22)
    for k in KEYS + ("n_recheck64",):
        assert a[k] == b[k] == c[k], (k, a[k], b[k], c[k])
    assert a["n_boxes_bounded"] > 100_000


def test_stack_box_budget_gives_an_enclosing_bracket():
    """With a box budget the boxes left on the stack (device and host) count as undecided at
    their depths: volumes still sum to 1 exactly and the bracket encloses the full one."""
    inst = synth.tiny2d(1)
    net, prop = load(inst)
    full = E().count_exact_stack(net, prop, inst.lo, inst.hi, 16, chunk=32)
    host = torch.empty(1 << 20, dtype=torch.uint8, pin_memory=True)
    for budget in (1, 100, full["n_boxes_bounded"] // 3):
        r = E().count_exact_stack(net, prop, inst.lo, inst.hi, 16, chunk=32, max_boxes=budget,
                                  device_boxes=128, host_spill=host)
        assert r["status"] == 1 and r["n_boxes_bounded"] <= budget
        assert r["unsafe"] + r["safe"] + r["undecided"] == 1.0
        assert r["unsafe"] <= full["unsafe"] and r["safe"] <= full["safe"]
        assert r["unsafe"] + r["undecided"] >= full["unsafe"] + full["undecided"]


def test_stack_rejects_bad_options_and_overflow():
    eng = E()
    inst = synth.acas(2)
    net, prop = load(inst)
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact_stack(net, prop, inst.lo, inst.hi, 20, chunk=1024, device_boxes=1000)
    assert e.value.code == -1                                   # device_boxes < 4 chunk
    with pytest.raises(eng.SlrError, match="more than") as e:   # no host spill: stack overflows
        eng.count_exact_stack(net, prop, inst.lo, inst.hi, 20, chunk=1024, device_boxes=4096)
    assert e.value.code == -2
    with pytest.raises(eng.SlrError):
        eng.count_exact_stack(net, prop, inst.lo, inst.hi, 63)
