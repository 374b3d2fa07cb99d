"""Exact and approximate counting of unsafe input volume (paper §2.3, §3 Alg. 1, §4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Exact count (Alg. 1, with every box of one branch-and-bound level processed together as in
§3): start from the property's input box; bound every box of the level with ``slr``; a box
whose reachable set lies inside the unsafe set adds its volume to the unsafe total, a box that
cannot reach it adds to the safe total, any other box is bisected.  Volumes are fractions of
the input box: a box at depth t has volume 2^-t, so totals are exact dyadic sums.

Stopping (the paper's loop runs until nothing is undecided, which never happens when the
unsafe boundary crosses the domain): boxes still undecided at ``max_depth`` are not split;
before building level t+1 the search also stops when the leaves so far plus two per
undecided box would exceed ``max_leaves``.  The result is the bracket
[unsafe, unsafe + undecided] on the violation rate.

Approximate count (CountingProVe with the exact count as its leaf backend): per trial,
repeatedly try the exact count on the current subdomain; if more than ``resolve_tol`` of it
stays undecided, draw uniform samples, split one random dimension at the lower median of the
violating samples' coordinates (all samples if none violates), snapped to a fixed dyadic
grid of the domain, and keep a random half; a trial also stops when the drawn dimension of the
subdomain is already narrower than two grid steps, or after ``max_splits``.  A trial that ends
after s splits on a
subdomain holding the fraction v of the domain, with unsafe fraction f (lower end of the
bracket) inside it, estimates E = 2^s v f.  The returned bound is 2^-beta min_i E_i with
beta = log2(1/(1-confidence)) / trials; since E[2^s v f] <= VR for any split points, Markov's
inequality gives P(bound > VR) <= 2^(-beta * trials) = 1 - confidence.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import philox, slr

OK = 0
BUDGET = 1


def _exact_sum(hist):
    """sum_t hist[t] * 2^-t as an exact Fraction."""
    return sum((Fraction(int(n), 1 << t) for t, n in enumerate(hist)), Fraction(0))


def bound_chunked(net, C, dvec, lo, hi, chunk=8192, relax="one"):
    g_lo = []
    g_hi = []
    for s in range(0, lo.shape[0], chunk):
        a, b = slr.propagate(net, C, dvec, lo[s:s + chunk], hi[s:s + chunk], relax=relax)
        g_lo.append(a)
        g_hi.append(b)
    return np.concatenate(g_lo), np.concatenate(g_hi)


def bisect(lo: np.ndarray, hi: np.ndarray, paths: np.ndarray, sides=None):
    """Split every box at the midpoint of its widest side (lowest index on ties), or of the
    given ``sides``.

    Children are emitted in parent order as [lower half, upper half]; the path id of a child
    is 2 * parent + side (the root is 1).
    """
    n, d = lo.shape
    j = np.argmax(hi - lo, axis=1) if sides is None else np.asarray(sides)
    rows = np.arange(n)
    mid = 0.5 * (lo[rows, j] + hi[rows, j])
    lo2 = np.repeat(lo, 2, axis=0)
    hi2 = np.repeat(hi, 2, axis=0)
    hi2[2 * rows, j] = mid
    lo2[2 * rows + 1, j] = mid
    p2 = np.empty(2 * n, np.uint64)
    p2[0::2] = paths * np.uint64(2)
    p2[1::2] = paths * np.uint64(2) + np.uint64(1)
    return lo2, hi2, p2


ASPECT_LOG2 = 6      # split candidates: sides at least 2^-6 of the box's widest side
# crossing tests within BAND[layer] * (|c0| + S) of zero are uncertain: the first layer's
# bounds are exact affine images (a float32 pass is off by ~1e-6 relative); deeper layers
# inherit a float32 pass's worst-case rounding margins, up to ~1e-3 relative
BAND = (1e-4, 1e-2)
TIE = 1e-5           # relative score gap below which a split choice is not robust


def crossing_scores(lo, hi, tr, layers, band=0.0):
    """Per box and input side j: the sum over the crossing neurons of the first ``layers``
    hidden layers of |coefficient of x_j| x (hi_j - lo_j) in the neuron's pre-activation
    equation (the part of the neuron's interval that side j contributes).  A neuron counts as
    crossing when l < -b m and u > b m, m = |centre| + sum of the side terms and
    b = band * BAND[layer]: band = 1 leaves the uncertain ones out, band = -1 counts them in,
    band = 0 is the plain test."""
    w = hi - lo
    s = np.zeros_like(w)
    for li, t in enumerate(tr[:layers]):
        C = 0.5 * (t["L"] + t["U"])
        terms = np.abs(C[..., 1:]) * w[:, None, :]
        centre = C[..., 0] + np.einsum("bkj,bj->bk", C[..., 1:], 0.5 * (lo + hi))
        m = np.abs(centre) + 0.5 * terms.sum(-1)
        bl = band * BAND[min(li, len(BAND) - 1)]
        cross = (t["lo"] < -bl * m) & (t["hi"] > bl * m)
        s += np.einsum("bk,bkj->bj", cross.astype(np.float64), terms)
    return s


def split_sides(lo, hi, tr, layers):
    """The side to bisect and whether that choice is robust.

    layers = 0: the widest side, lowest index on ties (the reading of §2.2's refinement).
    layers > 0: among the sides at least 2^-6 of the widest, the one with the largest
    ``crossing_scores`` (lowest index on ties); the widest if no neuron crosses.  The choice is
    robust unless another candidate's score could reach the chosen one's within TIE when
    neurons within the BAND of a phase change flip (a float32 evaluation may see them either
    way).
    """
    w = hi - lo
    widest = np.argmax(w, axis=1)
    if layers <= 0:
        return widest, np.ones(w.shape[0], bool)
    ok = w >= w.max(axis=1, keepdims=True) * 2.0 ** -ASPECT_LOG2
    s = np.where(ok, crossing_scores(lo, hi, tr, layers), -1.0)
    j = np.argmax(s, axis=1)
    none = s.max(axis=1) <= 0.0
    j = np.where(none, widest, j)
    sure = np.where(ok, crossing_scores(lo, hi, tr, layers, 1.0), -1.0)      # certain crossings
    maybe = np.where(ok, crossing_scores(lo, hi, tr, layers, -1.0), -1.0)    # and uncertain
    rows = np.arange(w.shape[0])
    others = maybe.copy()
    others[rows, j] = -np.inf
    robust = sure[rows, j] * (1.0 - TIE) > others.max(axis=1)
    robust = np.where(none, maybe.max(axis=1) <= 0.0, robust)
    return j, robust


def count_exact(net, C, dvec, lo, hi, max_depth: int, max_leaves: int, trace: bool = False,
                chunk: int = 8192, split_layers: int = 0, relax: str = "one"):
    """Alg. 1, level by level.  Returns a dict with the bracket, counts and histograms.

    With ``trace`` the dict also holds, per level, the boxes' path ids, classes and bounds,
    and for the boxes that were split the side and whether that choice was robust.
    ``split_layers``: the split rule of ``split_sides``.  ``relax``: the ReLU relaxation of
    ``slr.propagate`` ("one": Eq. 1; "two": one ratio per equation).
    """
    lo = np.asarray(lo, np.float64).reshape(1, -1)
    hi = np.asarray(hi, np.float64).reshape(1, -1)
    for v in np.concatenate([lo.ravel(), hi.ravel()]):
        assert slr.dyadic_exact(float(v)), "domain corners must be exact in float32"
    assert np.all(lo <= hi)
    paths = np.ones(1, np.uint64)
    D = int(max_depth)
    h_unsafe = [0] * (D + 1)
    h_safe = [0] * (D + 1)
    h_undec = [0] * (D + 1)
    resolved = 0
    bounded = 0
    status = OK
    levels = []
    depth = 0
    for t in range(D + 1):
        if lo.shape[0] == 0:
            break
        depth = t
        if split_layers > 0:
            g_lo, g_hi, tr = slr.propagate(net, C, dvec, lo, hi, keep=True, relax=relax)
        else:
            g_lo, g_hi = bound_chunked(net, C, dvec, lo, hi, chunk, relax)
        cls = slr.classify(g_lo, g_hi)
        bounded += lo.shape[0]
        if trace:
            levels.append(dict(depth=t, path=paths.copy(), cls=cls.copy(), g_lo=g_lo, g_hi=g_hi,
                               lo=lo.copy(), hi=hi.copy()))
        h_unsafe[t] = int(np.sum(cls == 1))
        h_safe[t] = int(np.sum(cls == 2))
        resolved += h_unsafe[t] + h_safe[t]
        und = cls == 0
        n_und = int(und.sum())
        if n_und == 0:
            lo = lo[:0]
            break
        if t == D or resolved + 2 * n_und > max_leaves:
            h_undec[t] = n_und
            status = BUDGET
            break
        if split_layers > 0:
            tru = [{k: v[und] for k, v in x.items()} for x in tr]
            sides, robust = split_sides(lo[und], hi[und], tru, split_layers)
        else:
            sides, robust = None, None
        if trace:
            levels[-1]["side"] = np.full(cls.shape[0], -1, np.int64)
            levels[-1]["robust"] = np.ones(cls.shape[0], bool)
            if sides is not None:
                levels[-1]["side"][und] = sides
                levels[-1]["robust"][und] = robust
            else:
                levels[-1]["side"][und] = np.argmax(hi[und] - lo[und], axis=1)
        lo, hi, paths = bisect(lo[und], hi[und], paths[und], sides)

    unsafe = _exact_sum(h_unsafe)
    safe = _exact_sum(h_safe)
    undec = _exact_sum(h_undec)
    assert unsafe + safe + undec == 1
    out = dict(status=status, unsafe=float(unsafe), safe=float(safe), undecided=float(undec),
               unsafe_exact=unsafe, safe_exact=safe, undecided_exact=undec,
               n_unsafe=sum(h_unsafe), n_safe=sum(h_safe), n_undecided=sum(h_undec),
               n_boxes_bounded=bounded, depth_reached=depth,
               hist_unsafe=h_unsafe, hist_safe=h_safe, hist_undecided=h_undec)
    if trace:
        out["levels"] = levels
    return out


def snap_split(med: float, a: float, b: float, A: float, B: float, grid_bits: int) -> float:
    """Split point for [a, b] near ``med`` on the grid A + k (B - A) 2^-grid_bits.

    The point is kept at least one grid step inside (a, b); an interval narrower than two
    steps is bisected at its midpoint instead.
    """
    h = (B - A) * 2.0 ** -grid_bits
    if b - a < 2.0 * h or h <= 0.0:
        return 0.5 * (a + b)
    k = math.floor((med - A) / h + 0.5)
    k_lo = math.floor((a - A) / h + 0.5) + 1
    k_hi = math.floor((b - A) / h + 0.5) - 1
    k = min(max(k, k_lo), k_hi)
    return A + k * h


def count_approx(net, C, dvec, lo, hi, trials: int = 20, samples: int = 1000,
                 confidence: float = 0.99, seed: int = 0, leaf_depth: int = 48,
                 leaf_leaves: int = 1 << 16, resolve_tol: float = 0.01, max_splits: int = 60,
                 grid_bits: int = 16):
    """Probabilistic lower bound on the violation rate (see the module docstring)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = lo.shape[0]
    beta = math.log2(1.0 / (1.0 - confidence)) / trials
    estimates, split_counts, details = [], [], []
    for t in range(trials):
        slo, shi = lo.copy(), hi.copy()
        v = Fraction(1)
        s = 0
        while True:
            r = count_exact(net, C, dvec, slo, shi, leaf_depth, leaf_leaves)
            if r["undecided"] <= resolve_tol or s >= max_splits:
                break
            u = np.array(philox.sample_uniforms(seed, t, s, samples, d), np.float64)
            pts = (slo + u * (shi - slo)).astype(np.float32).astype(np.float64)
            viol = np.all(slr.property_values(net, C, dvec, pts) > 0.0, axis=1)
            dim, side = philox.split_choice(seed, t, s, d)
            # the drawn side is already as narrow as two grid steps (or has no width at all,
            # a degenerate side of the domain): the trial stops here
            side_w = float(shi[dim]) - float(slo[dim])
            if side_w < 2.0 * (float(hi[dim]) - float(lo[dim])) * 2.0 ** -grid_bits or side_w <= 0.0:
                break
            vals = pts[viol, dim] if viol.any() else pts[:, dim]
            med = float(np.sort(vals)[(vals.shape[0] - 1) // 2])
            m = snap_split(med, float(slo[dim]), float(shi[dim]), float(lo[dim]),
                           float(hi[dim]), grid_bits)
            assert slr.dyadic_exact(m)
            low = Fraction(m) - Fraction(float(slo[dim]))
            width = Fraction(float(shi[dim])) - Fraction(float(slo[dim]))
            if side == 0:
                shi[dim] = m
                v *= low / width
            else:
                slo[dim] = m
                v *= (width - low) / width
            s += 1
        E = float(Fraction(2) ** s * v * r["unsafe_exact"])
        estimates.append(E)
        split_counts.append(s)
        details.append(dict(splits=s, volume=float(v), leaf=r, lo=slo, hi=shi))
    return dict(lower_bound=2.0 ** (-beta) * min(estimates), estimates=estimates,
                splits=split_counts, beta=beta, trials=details)
