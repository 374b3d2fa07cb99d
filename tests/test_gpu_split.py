"""Crossing-score split rule (count_exact split_layers) on the GPU against the FP64 oracle.

Boxes are matched on (depth, path id).  Where both sides bound a box: classes agree unless the
oracle's margin is at most 1e-5 (the margin rule of the parity tests), and the side bisected
agrees unless the oracle flagged that choice non-robust (a neuron within 1e-4 of a phase change
could move another side within 1e-5 of the chosen one).  Boxes below a difference of either
kind are excused; with no difference the counts and volumes are identical.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import count, slr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def E():
    import paper_2312_05890_amd as eng
    return eng


def load(inst):
    eng = E()
    net = eng.Net(inst.net)
    return net, eng.Property(net, inst.C, inst.dvec)


def compare_split(inst, D, M, k, chunk=0):
    from tests.test_gpu_parity import _ancestor_in
    net, prop = load(inst)
    g = E().count_exact(net, prop, inst.lo, inst.hi, D, M, chunk=chunk, trace=True, split_layers=k)
    o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, D, M, trace=True,
                          split_layers=k)
    oi = {}
    for lev in o["levels"]:
        mg = slr.decision_margin(lev["g_lo"], lev["g_hi"])
        side = lev.get("side", np.full(lev["cls"].shape[0], -1))
        robust = lev.get("robust", np.ones(lev["cls"].shape[0], bool))
        for p, c, m, sd, rb in zip(lev["path"], lev["cls"], mg, side, robust):
            oi[(lev["depth"], int(p))] = (int(c), float(m), int(sd), bool(rb))
    gi = {(int(a), int(b)): (int(c), int(sd)) for a, b, c, sd in
          zip(g["trace_depth"], g["trace_path"], g["trace_cls"], g["trace_dim"])}
    last = o["depth_reached"]
    diverge = set()
    n_nonrobust = 0
    for key in sorted(oi.keys() & gi.keys()):
        if _ancestor_in(key, diverge):
            continue
        oc, m, osd, rb = oi[key]
        gc, gsd = gi[key]
        if oc != gc:
            assert m <= TOL, f"class mismatch at {key} with margin {m}"
            diverge.add(key)
        elif oc == 0 and key[0] < last and osd >= 0 and gsd != osd:
            assert not rb, f"robust split side differs at {key}: oracle {osd}, GPU {gsd}"
            n_nonrobust += 1
            diverge.add(key)
    for key in oi.keys() ^ gi.keys():
        assert _ancestor_in(key, diverge), f"box {key} visited by one side only"
    compared = sum(1 for key in oi.keys() & gi.keys() if not _ancestor_in(key, diverge))
    print(f"split_layers {k}: {compared} of {len(oi)} oracle boxes compared, "
          f"{len(diverge)} differences, {n_nonrobust} at non-robust splits")
    assert compared >= 0.5 * len(oi)
    if not diverge:
        for f in ("n_unsafe", "n_safe", "n_undecided", "unsafe", "safe", "undecided",
                  "n_boxes_bounded", "depth_reached", "status"):
            assert g[f] == o[f], (f, g[f], o[f])
    assert g["unsafe"] + g["safe"] + g["undecided"] == 1.0
    return g, o, diverge


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("seed", range(8))
def test_split_rule_tiny2d(seed, k):
    compare_split(synth.tiny2d(seed), 14, 1 << 16, k)


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("seed", range(3))
def test_split_rule_five_inputs(seed, k):
    g, o, diverge = compare_split(synth.acas(seed), 40, 1 << 13, k, chunk=1000)
    assert g["n_boxes_bounded"] > 4000


@pytest.mark.parametrize("idx", [1, 2, 7, 11, 14, 19])
def test_split_rule_batch_shapes(idx):
    from tests.test_gpu_batch import _one_per_shape
    inst = _one_per_shape(4)[idx]
    compare_split(inst, inst.max_depth, 1 << 11, 2)


def test_split_rule_rejected_where_unsupported():
    eng = E()
    for inst in (synth.nav22(0), synth.smooth5(0, "tanh")):
        net, prop = load(inst)
        with pytest.raises(eng.SlrError) as e:
            eng.count_exact(net, prop, inst.lo, inst.hi, 10, 1 << 8, split_layers=1)
        assert e.value.code == -5
    inst = synth.acas(0)
    net, prop = load(inst)
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact(net, prop, inst.lo, inst.hi, 10, 1 << 8, split_layers=9)
    assert e.value.code == -1


def test_split_rule_full_size_brackets():
    """The headline workload (depth 40, 2^20 leaves): both rules bound the same number of boxes
    per level budget; the crossing-score rule finds more unsafe volume (printed)."""
    inst = synth.acas(0)
    net, prop = load(inst)
    out = {}
    for k in (0, 1, 2):
        r = E().count_exact(net, prop, inst.lo, inst.hi, 40, 1 << 20, chunk=65536, split_layers=k)
        out[k] = r
        print(k, r["unsafe"], r["undecided"], r["n_boxes_bounded"], r["depth_reached"])
    assert out[1]["unsafe"] > out[0]["unsafe"] and out[2]["unsafe"] > out[0]["unsafe"]
