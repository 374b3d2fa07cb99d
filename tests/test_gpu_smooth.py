"""Tanh and sigmoid networks on the GPU against the FP64 oracle, through the C ABI.

The relaxation is two parallel lines per neuron (chord slope over the pre-activation interval,
offsets bounding s(z) - lam z); the kernels bound the offsets by tangents at the points where
s' = lam, the oracle takes the exact extrema, so raw bounds agree to float32 rounding.  Counts
are compared box by box like the ReLU ones.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import count, slr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
ACTS = ["tanh", "sigmoid"]


def E():
    import paper_2312_05890_amd as eng
    return eng


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def load(inst):
    eng = E()
    net = eng.Net(inst.net)
    return net, eng.Property(net, inst.C, inst.dvec)


def cases(act):
    return [(synth.tanh2d(0, act), 12), (synth.tanh2d(3, act), 16), (synth.smooth5(0, act), 10),
            (synth.smooth5(1, act), 20)]


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("k", range(4))
def test_raw_bounds_match_oracle(act, k):
    inst, depth = cases(act)[k]
    blo, bhi = synth.random_boxes(inst.lo, inst.hi, 800, 31 + k, depth)
    net, prop = load(inst)
    g_lo, g_hi, _ = E().bound_boxes(net, prop, dev(blo), dev(bhi), raw=True)
    o_lo, o_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi)
    scale = TOL * np.maximum(1.0, np.maximum(np.abs(o_lo), np.abs(o_hi)))
    assert np.all(np.abs(g_lo.cpu().numpy() - o_lo) <= scale)
    assert np.all(np.abs(g_hi.cpu().numpy() - o_hi) <= scale)


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("k", range(4))
def test_widened_bounds_sound_and_classes(act, k):
    from tests.test_gpu_parity import margin
    inst, depth = cases(act)[k]
    blo, bhi = synth.random_boxes(inst.lo, inst.hi, 600, 41 + k, depth)
    net, prop = load(inst)
    g_lo, g_hi, cls = E().bound_boxes(net, prop, dev(blo), dev(bhi))
    g_lo, g_hi, cls = g_lo.cpu().numpy(), g_hi.cpu().numpy(), cls.cpu().numpy()
    rng = np.random.default_rng(k)
    for i in range(0, 600, 29):
        x = slr.sample_points(blo[i].astype(np.float64), bhi[i].astype(np.float64), 400, rng)
        gv = slr.property_values(inst.net, inst.C, inst.dvec, x)
        assert np.all(g_lo[i] <= gv.min(axis=0)) and np.all(gv.max(axis=0) <= g_hi[i])
    o_lo, o_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi)
    big = margin(o_lo, o_hi) > TOL
    assert np.array_equal(cls[big], slr.classify(o_lo, o_hi)[big])


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("seed", range(6))
def test_count_exact_box_by_box(act, seed):
    from tests.test_gpu_parity import compare_counts
    inst = synth.tanh2d(seed, act)
    g, o, _ = compare_counts(inst, 14, 1 << 16)
    assert o["n_unsafe"] + o["n_safe"] > 0


@pytest.mark.parametrize("act", ACTS)
def test_count_exact_five_inputs_and_stack(act):
    """5-input 3x32 network, depth 30, 2^13 leaves through count_exact; depth 14 without a leaf
    budget through count_exact_stack; both box by box against the oracle."""
    from tests.test_gpu_parity import compare_counts, compare_results
    inst = synth.smooth5(2, act)
    compare_counts(inst, 30, 1 << 13, chunk=1000)
    net, prop = load(inst)
    g = E().count_exact_stack(net, prop, inst.lo, inst.hi, 14, chunk=512, trace=True,
                              trace_capacity=1 << 16)
    o = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 14, 1 << 40, trace=True)
    compare_results(g, o)


@pytest.mark.parametrize("act", ACTS)
def test_batch_equals_count_exact(act):
    insts = [synth.tanh2d(s, act) for s in range(3)] + [synth.smooth5(s, act) for s in range(3)]
    eng = E()
    items = []
    for inst in insts:
        net, prop = load(inst)
        items.append((net, prop, inst.lo, inst.hi, 12, 1 << 12))
    res = eng.Batch(items).run()
    for it, r in zip(items, res):
        s = eng.count_exact(*it)
        for k in ("unsafe", "safe", "undecided", "n_boxes_bounded", "n_recheck64", "status"):
            assert r[k] == s[k], k


@pytest.mark.parametrize("act", ACTS)
def test_count_approx_matches_oracle_draws(act):
    inst = synth.smooth5(3, act)
    net, prop = load(inst)
    kw = dict(trials=3, samples=300, seed=5, max_splits=6, grid_bits=12, resolve_tol=0.05)
    g = E().count_approx(net, prop, inst.lo, inst.hi, leaf_depth=16, leaf_leaves=1 << 9, **kw)
    o = count.count_approx(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, leaf_depth=16,
                           leaf_leaves=1 << 9, **kw)
    assert g["splits"] == o["splits"]
    assert np.allclose(g["estimates"], o["estimates"], rtol=1e-12, atol=0)


def test_alpha_and_bad_activation_rejected():
    eng = E()
    inst = synth.smooth5(0, "tanh")
    net, prop = load(inst)
    lo, hi = synth.uniform_boxes(inst.lo, inst.hi, 16, 1, 0.2)
    with pytest.raises(eng.SlrError) as e:
        eng.alpha_optimize(net, prop, dev(lo), dev(hi), steps=2)
    assert e.value.code == -5
    with pytest.raises(eng.SlrError) as e:
        eng.count_exact(net, prop, inst.lo, inst.hi, 10, 1 << 10, alpha_steps=2)
    assert e.value.code == -5
    with pytest.raises(ValueError):
        eng.Net(inst.net, act="gelu")
