"""The allocation-free exact count (static device workspace) against count_exact, through the
C ABI: identical results on two calls in a row, the second on a smaller input, and a clear
error for counts that do not fit the static workspace."""
from __future__ import annotations

import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("unsafe", "safe", "undecided", "n_unsafe", "n_safe", "n_undecided", "n_boxes_bounded",
        "n_recheck64", "depth_reached", "status", "bound_launches")


def E():
    import paper_2312_05890_amd as eng
    return eng


def _pair(inst, D, M, **kw):
    eng = E()
    net = eng.Net(inst.net)
    prop = eng.Property(net, inst.C, inst.dvec)
    a = eng.count_exact_noalloc(net, prop, inst.lo, inst.hi, D, M, **kw)
    b = eng.count_exact(net, prop, inst.lo, inst.hi, D, M, **kw)
    return a, b


def test_noalloc_equals_count_exact_two_calls():
    """A large count (5-input 6x50 network, depth 40, 2^19 leaves: 53 MB of the 64 MiB scratch)
    and then a smaller one (2-input network, depth 12) on the same static workspace."""
    a, b = _pair(synth.acas(0), 40, 1 << 19)
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])
    assert a["n_boxes_bounded"] > 500000
    a, b = _pair(synth.tiny2d(0), 12, 1 << 12)
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])
    assert a["n_unsafe"] + a["n_safe"] > 0


def test_noalloc_alpha_and_chunks_equal_count_exact():
    a, b = _pair(synth.acas(1), 40, 1 << 14, chunk=1000, alpha_steps=5, alpha_min_depth=8,
                 alpha_chunk=2048, alpha_select=0.2)
    for k in KEYS + ("n_alpha_boxes", "n_alpha_decided"):
        assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_rejects_oversize_and_bad_options():
    eng = E()
    inst = synth.acas(0)
    net = eng.Net(inst.net)
    prop = eng.Property(net, inst.C, inst.dvec)
    assert eng.count_exact_noalloc_max_bytes() == 64 << 20
    assert eng.workspace_size(net, prop, 1 << 20) > eng.count_exact_noalloc_max_bytes()
    with pytest.raises(eng.SlrError, match="static scratch") as e:
        eng.count_exact_noalloc(net, prop, inst.lo, inst.hi, 40, 1 << 20)
    assert e.value.code == -2                               # SLR_ENOMEM
    # the failed call left the scratch usable
    a = eng.count_exact_noalloc(net, prop, inst.lo, inst.hi, 12, 1 << 10)
    b = eng.count_exact(net, prop, inst.lo, inst.hi, 12, 1 << 10)
    assert all(a[k] == b[k] for k in KEYS)
