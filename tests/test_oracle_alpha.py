"""Pins of the alpha (optimized lower slope) oracle: the float64 torch propagation equals the
NumPy oracle, autograd equals central finite differences away from phase switches, the
optimizer never ends worse than the plain relaxation, and alpha bounds stay sound."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import alpha as A
from oracle import slr

torch = pytest.importorskip("torch")


def _case(seed=0, sizes=(3, 10, 10, 2), n=6):
    net = synth.make_net(list(sizes), seed)
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(2, sizes[-1])).astype(np.float32)
    dv = rng.normal(scale=0.1, size=2).astype(np.float32)
    d = sizes[0]
    lo, hi = synth.uniform_boxes(-np.ones(d), np.ones(d), n, seed + 1, 0.5)
    return net, C, dv, lo.astype(np.float64), hi.astype(np.float64)


def test_torch_forward_matches_numpy_oracle():
    net, C, dv, lo, hi = _case(1)
    rng = np.random.default_rng(2)
    al = rng.uniform(0, 1, size=(lo.shape[0], 20))
    t_lo, t_hi = A.forward_torch(net, C, dv, lo, hi, torch.tensor(al))
    o_lo, o_hi = slr.propagate(net, C, dv, lo, hi, alpha=al)
    assert np.allclose(t_lo.numpy(), o_lo, rtol=1e-10, atol=1e-10)
    assert np.allclose(t_hi.numpy(), o_hi, rtol=1e-10, atol=1e-10)


def _phases(net, C, dv, lo, hi, al):
    _, _, tr = slr.propagate(net, C, dv, lo, hi, alpha=al, keep=True)
    return [((t["hi"] <= 0), (t["lo"] < 0) & (t["hi"] > 0)) for t in tr]


def test_autograd_matches_central_differences():
    net, C, dv, lo, hi = _case(3, n=4)
    rng = np.random.default_rng(4)
    al = rng.uniform(0.1, 0.9, size=(lo.shape[0], 20))
    g = A.gradient(net, C, dv, lo, hi, al)
    h = 1e-6
    base = _phases(net, C, dv, lo, hi, al)
    checked = 0
    for k in range(20):
        e = np.zeros_like(al)
        e[:, k] = h
        p = _phases(net, C, dv, lo, hi, al + e)
        m = _phases(net, C, dv, lo, hi, al - e)
        same = np.ones(lo.shape[0], bool)
        for (d0, c0), (d1, c1), (d2, c2) in zip(base, p, m):
            same &= np.all(d0 == d1, 1) & np.all(c0 == c1, 1) & np.all(d0 == d2, 1) & np.all(c0 == c2, 1)
        fd = (A.objective(net, C, dv, lo, hi, al + e) - A.objective(net, C, dv, lo, hi, al - e)) / (2 * h)
        ok = same & (np.abs(fd) > 1e-7)
        assert np.allclose(g[ok, k], fd[ok], rtol=1e-4, atol=1e-7)
        checked += ok.sum()
    assert checked > 10


def test_alpha_lambda_is_plain_and_optimizer_never_worse():
    net, C, dv, lo, hi = _case(5, n=5)
    lam = A.plain_lambda(net, C, dv, lo, hi)
    j0 = A.objective(net, C, dv, lo, hi, lam)
    best, jb = A.optimize(net, C, dv, lo, hi, steps=20)
    assert np.all(jb <= j0 + 1e-9)
    assert np.all((best >= 0) & (best <= 1))
    g_lo, g_hi = slr.propagate(net, C, dv, lo, hi, alpha=best)
    rng = np.random.default_rng(0)
    for b in range(lo.shape[0]):
        x = slr.sample_points(lo[b], hi[b], 2000, rng)
        gv = slr.property_values(net, C, dv, x)
        assert np.all(g_lo[b] <= gv.min(0)) and np.all(gv.max(0) <= g_hi[b])
