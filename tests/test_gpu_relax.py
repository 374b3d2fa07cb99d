"""The ReLU relaxation with one ratio per equation on the GPU, through the C ABI.

The tape-state kernel's float32 bounds are compared with the FP64 oracle's (``slr.propagate``
with ``relax="two"``) box by box; ``count_exact`` with ``relax="two"`` (widened float32
bounds) is compared with the oracle's ``count_exact`` box by box (matched on depth and path id, classes equal wherever the oracle's
decision margin exceeds 1e-5; boxes the oracle decides may stay undecided on the GPU, which has
no FP64 re-decision for this relaxation) and, at the full size of the 5-input 6x50 workload,
with the oracle's stored run in tests/golden/.
"""
from __future__ import annotations

import hashlib
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import count, slr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))


def E():
    import paper_2312_05890_amd as eng
    return eng


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def load(inst):
    net = E().Net(inst.net)
    return net, E().Property(net, inst.C, inst.dvec)


def make(name, seed):
    if name == "batch":
        return synth.batch(0, count=seed + 1)[seed]
    return getattr(synth, name)(seed)


# (generator, seed, max bisections of the random boxes)
CASES = [("tiny2d", 0, 10), ("tiny2d", 3, 16), ("acas", 0, 12), ("acas", 1, 33),
         ("acas", 2, 38), ("nav22", 0, 30), ("batch", 0, 20), ("batch", 13, 24),
         ("batch", 14, 12), ("batch", 4, 16)]


def relax_bounds(inst, blo, bhi, relax, raw, want_cls=False):
    net, prop = load(inst)
    g_lo, g_hi, cls = E().bound_boxes_relax(net, prop, dev(blo), dev(bhi), relax=relax, raw=raw,
                                            want_cls=want_cls)
    torch.cuda.synchronize()
    out = g_lo.cpu().numpy().astype(np.float64), g_hi.cpu().numpy().astype(np.float64)
    return out + ((cls.cpu().numpy(),) if want_cls else ())


@pytest.mark.parametrize("relax", ["one", "two"])
@pytest.mark.parametrize("name,seed,depth", CASES)
def test_raw_bounds_match_oracle(name, seed, depth, relax):
    """Unwidened float32 bounds equal the FP64 oracle's to 1e-5 of max(1, |bound|)."""
    inst = make(name, seed)
    blo, bhi = synth.random_boxes(inst.lo, inst.hi, 800, seed + 29, depth)
    o_lo, o_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi, relax=relax)
    g_lo, g_hi = relax_bounds(inst, blo, bhi, relax, raw=True)
    scale = TOL * np.maximum(1.0, np.maximum(np.abs(o_lo), np.abs(o_hi)))
    assert np.max(np.abs(g_lo - o_lo) / scale) <= 1.0
    assert np.max(np.abs(g_hi - o_hi) / scale) <= 1.0


@pytest.mark.parametrize("name,seed,depth", CASES)
def test_widened_bounds_sound_and_around_oracle(name, seed, depth):
    """Widened bounds hold every sampled output and contain the oracle's up to 1e-5; a box they
    decide has the oracle's class wherever its margin exceeds 1e-5, and they decide most boxes
    the oracle decides (this call has no FP64 re-decision: near a threshold the float32
    rounding margin may leave a box undecided)."""
    inst = make(name, seed)
    blo, bhi = synth.random_boxes(inst.lo, inst.hi, 500, seed + 7, depth)
    g_lo, g_hi, cls = relax_bounds(inst, blo, bhi, "two", raw=False, want_cls=True)
    rng = np.random.default_rng(seed)
    for i in range(0, blo.shape[0], 31):
        x = slr.sample_points(blo[i].astype(np.float64), bhi[i].astype(np.float64), 300, rng)
        gv = slr.property_values(inst.net, inst.C, inst.dvec, x)
        assert np.all(g_lo[i] <= gv.min(axis=0)) and np.all(gv.max(axis=0) <= g_hi[i])
    o_lo, o_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi, relax="two")
    scale = TOL * np.maximum(1.0, np.maximum(np.abs(o_lo), np.abs(o_hi)))
    assert np.all(g_lo <= o_lo + scale) and np.all(o_hi - scale <= g_hi)
    big = slr.decision_margin(o_lo, o_hi) > TOL
    o_cls = slr.classify(o_lo, o_hi)
    dec = cls != 0
    assert np.array_equal(cls[dec & big], o_cls[dec & big])
    assert np.sum(dec) >= 0.9 * np.sum(o_cls != 0)


def test_ragged_and_empty_batches():
    inst = synth.acas(4)
    net, prop = load(inst)
    for n in (0, 1, 15, 16, 17, 63, 65, 257):
        blo, bhi = synth.random_boxes(inst.lo, inst.hi, n, n, 25)
        if n == 0:
            blo = np.zeros((0, 5), np.float32)
            bhi = np.zeros((0, 5), np.float32)
        g_lo, g_hi, _ = E().bound_boxes_relax(net, prop, dev(blo), dev(bhi), relax="two", raw=True)
        torch.cuda.synchronize()
        if n == 0:
            assert g_lo.shape == (0, prop.rows)
            continue
        o_lo, o_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi, relax="two")
        assert np.allclose(g_lo.cpu().numpy(), o_lo, rtol=TOL, atol=TOL)
        assert np.allclose(g_hi.cpu().numpy(), o_hi, rtol=TOL, atol=TOL)


def compare_two(g, o):
    """GPU count ``g`` (with a trace) against the oracle's ``o`` (with levels), both with two
    ratios.  The GPU keeps its widened float32 classes (no FP64 re-decision), which contain the
    exact relaxation's bounds: a box it decides has the oracle's class wherever the oracle's
    margin exceeds 1e-5, and a box the oracle decides may stay undecided on the GPU (within the
    float32 rounding margin of a decision).  Boxes visited by one side only descend from such a
    box, on the levels both searches reached.  Returns (boxes the GPU left undecided where the
    oracle decided, boxes whose classes differ within 1e-5 of a decision)."""
    from tests.test_gpu_parity import _ancestor_in, _index
    oi = _index(o["levels"], True)
    gi = _index((g["trace_depth"], g["trace_path"], g["trace_cls"]), False)
    open_gpu, small = set(), set()
    for k in oi.keys() & gi.keys():
        (oc, m), (gc, _) = oi[k], gi[k]
        if oc == gc:
            continue
        if m <= TOL:
            small.add(k)
        else:
            assert gc == 0, f"GPU class {gc} where the oracle decides {oc} with margin {m} at {k}"
            open_gpu.add(k)
    diverge = open_gpu | small
    last = min(g["depth_reached"], o["depth_reached"])
    for k in oi.keys() ^ gi.keys():
        if k[0] <= last:
            assert _ancestor_in(k, diverge), f"box {k} visited by one side only"
    assert g["unsafe"] + g["safe"] + g["undecided"] == 1.0
    if not diverge:
        for k in ("n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded", "depth_reached",
                  "status", "unsafe", "safe", "undecided"):
            assert g[k] == o[k], (k, g[k], o[k])
    else:
        # the GPU's decided volume lies inside the oracle's (up to near-threshold boxes): it
        # decides no box the oracle leaves open, and with more boxes open it meets the leaf
        # budget no later than the oracle
        slack = sum(2.0 ** -k[0] for k in small)
        assert g["unsafe"] <= o["unsafe"] + slack and g["safe"] <= o["safe"] + slack
    return open_gpu, small


def count_pair(inst, D, M, chunk=0):
    net, prop = load(inst)
    g = E().count_exact(net, prop, inst.lo, inst.hi, D, M, chunk=chunk, trace=True, relax="two")
    o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, D, M, trace=True,
                          relax="two")
    open_gpu, small = compare_two(g, o)
    decided = o["n_unsafe"] + o["n_safe"]
    print(f"{inst.name}: oracle decided {decided} leaves, GPU left {len(open_gpu)} of the "
          f"oracle's decided boxes undecided, {len(small)} within 1e-5")
    return g, o, open_gpu


@pytest.mark.parametrize("seed", range(24))
def test_count_exact_tiny2d(seed):
    inst = synth.tiny2d(seed)
    count_pair(inst, 12, 1 << 12)


@pytest.mark.parametrize("seed,D,M", [(0, 40, 1 << 14), (1, 30, 1 << 12), (3, 40, 1 << 13)])
def test_count_exact_acas(seed, D, M):
    count_pair(synth.acas(seed), D, M)


def test_count_exact_nav22_and_chunking():
    inst = synth.nav22(0)
    g, o, diverge = count_pair(inst, 30, 1 << 10)
    g2 = E().count_exact(*load(inst), inst.lo, inst.hi, 30, 1 << 10, chunk=100, relax="two")
    for k in ("unsafe", "safe", "undecided", "n_boxes_bounded", "status", "n_recheck64"):
        assert g2[k] == g[k], k


def test_count_exact_every_batch_shape():
    """Every (inputs, width) shape of the 256-instance batch workload on a 2^-4 sub-box, depth
    4 d, 2^11 leaves."""
    from tests.test_gpu_batch import _one_per_shape
    decided = 0
    for inst in _one_per_shape(4):
        g, o, _ = count_pair(inst, inst.max_depth, 1 << 11)
        decided += o["n_unsafe"] + o["n_safe"]
    assert decided > 1000


def test_count_exact_acas_full_size_against_oracle_fixture():
    """The 5-input 6x50 network (seed 0), depth 40, 2^20 leaves, 65536-box launches, with two
    ratios, against the oracle's full runs (make_acas_full.py, with two ratios and with one):
    up to the first level where the GPU leaves open a box the oracle decided, the same boxes
    with the same classes; the GPU's decided volumes lie inside the oracle's two-ratio ones and
    its unsafe volume exceeds the oracle's one-ratio volume.  (Without an FP64 re-decision the
    GPU keeps open the boxes within its float32 margin of a decision: here it proves about 0.0064
    of the box unsafe against the oracle's 0.0083 with two ratios and 0.0059 with one.)"""
    fx = json.load(open(os.path.join(HERE, "golden", "acas0_d40_leaves2p20_two.json")))
    fx1 = json.load(open(os.path.join(HERE, "golden", "acas0_d40_leaves2p20.json")))
    assert fx["relax"] == "two"
    inst = synth.acas(0)
    net, prop = load(inst)
    g = E().count_exact(net, prop, inst.lo, inst.hi, 40, 1 << 20, chunk=65536, trace=True,
                        trace_capacity=fx["n_boxes_bounded"] + (1 << 20), relax="two")
    td, tp, tc = g["trace_depth"], g["trace_path"], g["trace_cls"]
    same_levels = 0
    for lev in fx["levels"]:
        sel = td == lev["depth"]
        order = np.argsort(tp[sel], kind="stable")
        path = tp[sel][order].astype("<u8")
        cls = tc[sel][order].astype(np.int8)
        if (hashlib.sha256(path.tobytes()).hexdigest() != lev["path_sha256"]
                or hashlib.sha256(cls.tobytes()).hexdigest() != lev["cls_sha256"]):
            break
        same_levels += 1
    print(f"levels identical to the oracle's: {same_levels} of {len(fx['levels'])}; unsafe "
          f"{g['unsafe']:.6g} (oracle two ratios {fx['unsafe']:.6g}, one ratio {fx1['unsafe']:.6g})")
    assert same_levels >= 12
    assert g["unsafe"] <= fx["unsafe"] and g["safe"] <= fx["safe"]
    assert g["unsafe"] > fx1["unsafe"]


def test_noalloc_equals_count_exact():
    inst = synth.acas(1)
    net, prop = load(inst)
    a = E().count_exact(net, prop, inst.lo, inst.hi, 30, 1 << 13, relax="two")
    b = E().count_exact_noalloc(net, prop, inst.lo, inst.hi, 30, 1 << 13, relax="two")
    for k in ("unsafe", "safe", "undecided", "n_unsafe", "n_safe", "n_undecided",
              "n_boxes_bounded", "n_recheck64", "depth_reached", "status"):
        assert a[k] == b[k], k


KEYS = ("unsafe", "safe", "undecided", "n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded",
        "n_recheck64", "depth_reached", "status")


@pytest.mark.parametrize("relax,variant,name,seed,D,M", [
    ("two", 0, "acas", 0, 30, 1 << 14),     # top of depth 12, then levels
    ("two", 0, "tiny2d", 3, 16, 1 << 16),   # top of depth 15, then the last level
    ("two", 0, "acas", 2, 9, 1 << 12),      # the depth limit inside the top
    ("one", 3, "acas", 1, 20, 1 << 13),     # tape-state kernel with one ratio (FP64 re-decision)
    ("one", 3, "nav22", 0, 24, 1 << 12),
])
def test_one_pass_top_on_the_tape_state_kernel(relax, variant, name, seed, D, M):
    """The one-pass top of the tree with the tape-state kernel (two ratios, or the plain slopes
    under bound_kernel_variant 3) gives the level-by-level driver's exact result (timing bit 2
    keeps the level loop), traces included."""
    inst = make(name, seed)
    net, prop = load(inst)
    E().bound_kernel_variant(variant)
    try:
        a = E().count_exact(net, prop, inst.lo, inst.hi, D, M, relax=relax, trace=True)
        b = E().count_exact(net, prop, inst.lo, inst.hi, D, M, relax=relax, trace=True, timing=4)
    finally:
        E().bound_kernel_variant(0)
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])
    for k in ("trace_depth", "trace_path", "trace_cls"):
        assert np.array_equal(a[k], b[k]), k
    assert b["bound_launches"] >= a["bound_launches"]


def test_relax_rejects_bad_options():
    eng = E()
    inst = synth.acas(1)
    net, prop = load(inst)
    with pytest.raises(ValueError):
        eng.count_exact(net, prop, inst.lo, inst.hi, 10, 64, relax="three")
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact(net, prop, inst.lo, inst.hi, 10, 64, relax="two", alpha_steps=2)
    assert e.value.code == -5
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact(net, prop, inst.lo, inst.hi, 10, 64, relax="two", split_layers=1)
    assert e.value.code == -5
    sm = synth.with_activation(inst.net, "tanh")
    snet = eng.Net(sm)
    sprop = eng.Property(snet, inst.C, inst.dvec)
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact(snet, sprop, inst.lo, inst.hi, 10, 64, relax="two")
    assert e.value.code == -5
    # an out-of-range value through the C ABI
    import ctypes as C
    from paper_2312_05890_amd import slrcount
    o, ws = slrcount._exact_opts(net, prop, 10, 64, 0, None, None, 0)
    o.relax = 2
    r = slrcount.CountResult()
    lo = np.ascontiguousarray(inst.lo, np.float64)
    hi = np.ascontiguousarray(inst.hi, np.float64)
    rc = eng.lib().count_exact(net.handle, prop.handle, lo.ctypes.data_as(C.POINTER(C.c_double)),
                               hi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o), C.byref(r))
    assert rc == -1 and "relax" in eng.last_error()
