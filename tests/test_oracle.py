"""The FP64 oracle against its pins (CPU only), and mutation tests proving the pins bite."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import alpha as alpha_oracle
from oracle import count, philox, slr
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_soundness_alpha_mode():
    P.pin_soundness(seed=3, n_boxes=4, n_points=2000, alpha=True)


@pytest.mark.parametrize("seed", [1, 2])
def test_dense_grid_more_seeds(seed):
    P.pin_dense_grid(seed, cells=512)


def test_alpha_equal_lambda_is_plain():
    """alpha = lam everywhere reproduces the plain bounds exactly (pins the alpha plumbing)."""
    inst = synth.tiny2d(4)
    blo, bhi = synth.random_boxes(inst.lo, inst.hi, 16, 9, 6)
    g_lo, g_hi, tr = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi, keep=True)
    lam = []
    for t in tr:
        lo_b, hi_b = t["lo"], t["hi"]
        cross = (lo_b < 0) & (hi_b > 0)
        lm = np.where(cross, hi_b / np.where(cross, hi_b - lo_b, 1.0), 1.0)
        lam.append(np.minimum(1.0, lm * (1.0 + 4.0 * slr.UNIT)))
    a_lo, a_hi = slr.propagate(inst.net, inst.C, inst.dvec, blo, bhi, alpha=np.hstack(lam))
    assert np.array_equal(a_lo, g_lo) and np.array_equal(a_hi, g_hi)


def test_scalar_twin_matches_vectorized():
    rng = np.random.default_rng(5)
    for sizes in ([2, 6, 5, 1], [3, 4, 4, 4, 2]):
        net = synth.make_net(sizes, 11)
        C = rng.normal(size=(2, sizes[-1])).astype(np.float32)
        dv = rng.normal(size=2).astype(np.float32)
        blo, bhi = synth.uniform_boxes(-np.ones(sizes[0]), np.ones(sizes[0]), 8, 3, 0.8)
        g_lo, g_hi = slr.propagate(net, C, dv, blo, bhi)
        for i in range(blo.shape[0]):
            s_lo, s_hi = slr.scalar_bounds(net, C, dv, blo[i], bhi[i])
            assert np.allclose(s_lo, g_lo[i], rtol=1e-12, atol=1e-12)
            assert np.allclose(s_hi, g_hi[i], rtol=1e-12, atol=1e-12)


def test_budget_rule_and_status():
    inst = synth.tiny2d(0)
    r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 30, 200)
    assert r["status"] == count.BUDGET
    assert r["n_unsafe"] + r["n_safe"] + r["n_undecided"] <= 200
    assert r["unsafe_exact"] + r["safe_exact"] + r["undecided_exact"] == 1
    # a fully resolved count reports OK
    r = count.count_exact(P.abs_net(), [[1.0]], [0.0], np.zeros(2), np.ones(2), 3, 1 << 20)
    assert r["status"] in (count.OK, count.BUDGET)
    r = count.count_exact(P.relu_identity_net(), [[1.0]], [5.0], [-1.0], [1.0], 4, 16)
    assert r["status"] == count.OK and r["unsafe"] == 1.0 and r["n_boxes_bounded"] == 1


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (tests/golden/philox4x32_10.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10.txt")
    n = 0
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        w = [int(x, 16) for x in line.split()]
        assert philox.philox4x32_10(w[0:4], w[4:6]) == tuple(w[6:10])
        n += 1
    assert n == 3


def test_philox_uniforms_in_range():
    u = np.array(philox.sample_uniforms(7, 0, 0, 500, 3))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.03
    dims = [philox.split_choice(7, 0, s, 5)[0] for s in range(2000)]
    assert set(dims) == set(range(5))


def test_count_approx_lower_bound_closed_form():
    """Irwin-Hall-like net with a large unsafe volume: the 99% bound stays below the truth."""
    net = [(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
           (np.array([[1, 1, 1]], np.float32), np.array([-1.5], np.float32))]
    r = count.count_approx(net, [[1.0]], [0.0], np.zeros(3), np.ones(3), trials=5, samples=200,
                           seed=3, leaf_depth=12, leaf_leaves=1 << 12, resolve_tol=0.05)
    assert 0.0 < r["lower_bound"] <= 0.5
    assert all(e >= 0 for e in r["estimates"])


def test_count_approx_zero_width_side():
    """A domain with one side of zero width (x2 = 1/2 fixed): the rate is that of the 2-d
    slice, x0 + x1 > 3/2, i.e. 1/8.  A trial that draws the fixed side cannot split it and
    stops there (a grid step of zero would divide by zero); the others split as usual."""
    net = [(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
           (np.array([[1, 1, 1]], np.float32), np.array([-2.0], np.float32))]
    lo, hi = np.array([0.0, 0.0, 0.5]), np.array([1.0, 1.0, 0.5])
    r = count.count_approx(net, [[1.0]], [0.0], lo, hi, trials=8, samples=200, seed=11,
                           leaf_depth=12, leaf_leaves=1 << 10, resolve_tol=0.0, max_splits=20,
                           grid_bits=10)
    assert 0.0 <= r["lower_bound"] <= 0.125
    assert all(np.isfinite(r["estimates"]))
    # every trial ends before its split cap: on the first draw of the fixed side
    assert max(r["splits"]) < 20 and len(set(r["splits"])) > 1
    for t in r["trials"]:
        assert t["lo"][2] == 0.5 and t["hi"][2] == 0.5


@pytest.mark.parametrize("weights,bias,d,vr", [
    ([1, 1], -1.0, 2, Fraction(1, 2)),          # x0 + x1 > 1 on the unit square
    ([1, 1, 1], -2.0, 3, Fraction(1, 6)),       # the corner simplex x0 + x1 + x2 > 2
])
def test_count_approx_estimates_are_unbiased(weights, bias, d, vr):
    """Each trial's estimate 2^s v f is, in expectation over the random halves kept, the
    violation rate (per split: a f_low + (1 - a) f_high = f_parent, whatever the split point a);
    with the leaf's unsafe and unsafe+undecided fractions it brackets the exact rate trial by
    trial.  Over 256 seeded trials the rate must lie within 4 standard errors of the two means;
    the same trials evaluated with a volume factor of 1/2 per split, or without the 2^s, miss
    it on both nets."""
    net = [(np.array([weights], np.float32), np.array([bias], np.float32))]
    r = count.count_approx(net, [[1.0]], [0.0], np.zeros(d), np.ones(d), trials=256,
                           samples=200, seed=5, leaf_depth=8, leaf_leaves=1 << 6,
                           resolve_tol=0.02)
    lo = np.array([2.0 ** t["splits"] * t["volume"] * float(t["leaf"]["unsafe_exact"])
                   for t in r["trials"]])
    hi = np.array([2.0 ** t["splits"] * t["volume"] *
                   float(t["leaf"]["unsafe_exact"] + t["leaf"]["undecided_exact"])
                   for t in r["trials"]])
    assert np.allclose(lo, r["estimates"])
    assert max(t["splits"] for t in r["trials"]) >= 2
    se_lo = lo.std() / np.sqrt(lo.size)
    se_hi = hi.std() / np.sqrt(hi.size)
    assert lo.mean() - 4 * se_lo <= float(vr) <= hi.mean() + 4 * se_hi


# ---------------------------------------------------------------------------------------
# Mutation tests: plant a plausible mistake in the oracle and require that a pin fails.
# ---------------------------------------------------------------------------------------

def _swap_wpm_affine(L, U, W, b, xmag, W_err=None, b_err=None):
    return ORIG_AFFINE(L, U, -W, b, xmag, W_err, b_err)


def _relu_no_minus_l(L, U, lo_b, hi_b, xmag, alpha=None):
    """U <- lam U instead of lam (U - l)."""
    dead = hi_b <= 0.0
    cross = (lo_b < 0.0) & (hi_b > 0.0)
    lam = np.where(cross, hi_b / np.where(cross, hi_b - lo_b, 1.0), 1.0)
    Ln = np.where(cross[..., None], lam[..., None] * L, L)
    Un = np.where(cross[..., None], lam[..., None] * U, U)
    Ln[dead] = 0.0
    Un[dead] = 0.0
    return Ln, Un


def _relu_wrong_ratio(L, U, lo_b, hi_b, xmag, alpha=None):
    """lam = -l / (u - l) (the complementary ratio)."""
    dead = hi_b <= 0.0
    cross = (lo_b < 0.0) & (hi_b > 0.0)
    lam = np.where(cross, -lo_b / np.where(cross, hi_b - lo_b, 1.0), 1.0)
    Ln = np.where(cross[..., None], lam[..., None] * L, L)
    S = U.copy()
    S[..., 0] -= np.where(cross, lo_b, 0.0)
    Un = np.where(cross[..., None], lam[..., None] * S, U)
    Ln[dead] = 0.0
    Un[dead] = 0.0
    return Ln, Un


def _concretize_lower_uses_max(L, lo, hi, xmag):
    coef = L[..., 1:]
    return L[..., 0] + np.maximum(coef * lo[:, None, :], coef * hi[:, None, :]).sum(axis=-1)


def _classify_safe_on_lower(g_lo, g_hi):
    return ORIG_CLASSIFY(g_lo, g_lo)


def _bisect_narrowest(lo, hi, paths):
    n, d = lo.shape
    j = np.argmin(hi - lo, axis=1)
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


def _exact_sum_off_by_one(hist):
    from fractions import Fraction
    return sum((Fraction(int(n), 1 << (t + 1)) for t, n in enumerate(hist)), Fraction(0))


def _adam_step_ascends(a, g, m, v, t, lr, betas, eps):
    """Adam step taken along the gradient instead of against it."""
    m = betas[0] * m + (1 - betas[0]) * g
    v = betas[1] * v + (1 - betas[1]) * g * g
    a += lr * (m / (1 - betas[0] ** t)) / ((v / (1 - betas[1] ** t)).sqrt() + eps)
    a.clamp_(0.0, 1.0)
    return m, v


def _adam_step_no_bias_correction(a, g, m, v, t, lr, betas, eps):
    m = betas[0] * m + (1 - betas[0]) * g
    v = betas[1] * v + (1 - betas[1]) * g * g
    a -= lr * m / (v.sqrt() + eps)
    a.clamp_(0.0, 1.0)
    return m, v


def _objective_row_argmax(net, C, dvec, lo, hi):
    center = 0.5 * (np.asarray(lo, np.float64) + np.asarray(hi, np.float64))
    gc = slr.property_values(net, C, dvec, center)
    return np.all(gc > 0, axis=1).astype(np.int64), np.argmax(gc, axis=1)


def _objective_mode_any(net, C, dvec, lo, hi):
    center = 0.5 * (np.asarray(lo, np.float64) + np.asarray(hi, np.float64))
    gc = slr.property_values(net, C, dvec, center)
    return np.any(gc > 0, axis=1).astype(np.int64), np.argmin(gc, axis=1)


def _act_critical_no_sqrt(act, lam):
    """Critical point from 1 - lam instead of its square root (tanh) / 1 - 4 lam (sigmoid)."""
    lam = np.asarray(lam, np.float64)
    if act == "tanh":
        return np.arctanh(np.clip(1.0 - lam, 0.0, 1.0 - 1e-16))
    p = np.minimum(0.5 * (1.0 + np.clip(1.0 - 4.0 * lam, 0.0, 1.0)), 1.0 - 1e-16)
    return np.log(p / (1.0 - p))


def _act_critical_halved(act, lam):
    return 0.5 * ORIG_ACT_CRITICAL(act, lam)


def _act_relax_endpoints_only(L, U, lo_b, hi_b, xmag, act):
    """Parallel lines whose offsets look only at the interval's ends (no critical points)."""
    l = np.asarray(lo_b, np.float64)
    u = np.asarray(hi_b, np.float64)
    w = u - l
    fl, fu = slr.act_fn(act, l), slr.act_fn(act, u)
    lam = np.where(w > 0.0, (fu - fl) / np.where(w > 0.0, w, 1.0), 0.0)
    hl, hu = fl - lam * l, fu - lam * u
    Ln = lam[..., None] * L
    Un = lam[..., None] * U
    Ln[..., 0] += np.minimum(hl, hu)
    Un[..., 0] += np.maximum(hl, hu)
    return Ln, Un


def _split_sides_argmin(lo, hi, tr, layers):
    j, robust = ORIG_SPLIT_SIDES(lo, hi, tr, layers)
    if layers <= 0:
        return j, robust
    w = hi - lo
    s = np.where(w >= w.max(axis=1, keepdims=True) / 64, count.crossing_scores(lo, hi, tr, layers), np.inf)
    return np.argmin(s, axis=1), robust


def _split_sides_no_aspect_guard(lo, hi, tr, layers):
    j, robust = ORIG_SPLIT_SIDES(lo, hi, tr, layers)
    if layers <= 0:
        return j, robust
    s = count.crossing_scores(lo, hi, tr, layers)
    return np.where(s.max(axis=1) > 0, np.argmax(s, axis=1), j), robust


def _two_ratio_shares_the_range(L, U, lo_b, hi_b, lU, uL, xmag):
    """Both equations take the neuron's range [l, u] (the one-ratio form)."""
    return ORIG_RELU_TWO(L, U, lo_b, hi_b, lo_b, hi_b, xmag)


def _two_ratio_upper_shift_by_l(L, U, lo_b, hi_b, lU, uL, xmag):
    """Upper chord through (l, 0) while its slope is taken from [lU, u]."""
    Ln, Un = ORIG_RELU_TWO(L, U, lo_b, hi_b, lU, uL, xmag)
    up = (lo_b < 0.0) & (hi_b > 0.0) & (lU < 0.0)
    lam = np.where(up, hi_b / np.where(up, hi_b - lU, 1.0), 0.0)
    Un[..., 0] += np.where(up, lam * (lU - lo_b), 0.0)
    return Ln, Un


def _two_ratio_lower_keeps_negative(L, U, lo_b, hi_b, lU, uL, xmag):
    """Lower line keeps L when uL <= 0 instead of dropping to 0."""
    Ln, Un = ORIG_RELU_TWO(L, U, lo_b, hi_b, lU, uL, xmag)
    keep = (lo_b < 0.0) & (hi_b > 0.0) & (uL <= 0.0)
    return np.where(keep[..., None], L, Ln), Un


ORIG_AFFINE = slr.affine
ORIG_RELU = slr.relu_relax
ORIG_RELU_TWO = slr.relu_relax_two
ORIG_CLASSIFY = slr.classify
ORIG_BISECT = count.bisect
ORIG_ACT_CRITICAL = slr.act_critical
ORIG_SPLIT_SIDES = count.split_sides

MUTANTS = [
    ("affine swaps W+ and W-", slr, "affine", _swap_wpm_affine),
    ("Eq.1 drops the -l shift", slr, "relu_relax", _relu_no_minus_l),
    ("Eq.1 uses -l/(u-l)", slr, "relu_relax", _relu_wrong_ratio),
    ("lower concretization takes the max", slr, "concretize_lower", _concretize_lower_uses_max),
    ("safe test on the lower bound", slr, "classify", _classify_safe_on_lower),
    ("bisects the narrowest side", count, "bisect", _bisect_narrowest),
    ("volume of depth t taken as 2^-(t+1)", count, "_exact_sum", _exact_sum_off_by_one),
    ("alpha Adam steps along the gradient", alpha_oracle, "adam_step", _adam_step_ascends),
    ("alpha Adam without bias correction", alpha_oracle, "adam_step", _adam_step_no_bias_correction),
    ("alpha objective row is the argmax", alpha_oracle, "objective_weights", _objective_row_argmax),
    ("alpha unsafe mode when any row is positive", alpha_oracle, "objective_weights", _objective_mode_any),
    ("smooth activation: critical point without the square root", slr, "act_critical", _act_critical_no_sqrt),
    ("smooth activation: critical point halved", slr, "act_critical", _act_critical_halved),
    ("smooth activation: offsets from the interval ends only", slr, "act_relax", _act_relax_endpoints_only),
    ("crossing-score split takes the smallest score", count, "split_sides", _split_sides_argmin),
    ("crossing-score split without the aspect guard", count, "split_sides", _split_sides_no_aspect_guard),
    ("two ratios: both from the neuron's range", slr, "relu_relax_two", _two_ratio_shares_the_range),
    ("two ratios: upper chord shifted by l", slr, "relu_relax_two", _two_ratio_upper_shift_by_l),
    ("two ratios: lower keeps L below zero", slr, "relu_relax_two", _two_ratio_lower_keeps_negative),
]


@pytest.mark.parametrize("name,mod,attr,fn", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(monkeypatch, name, mod, attr, fn):
    monkeypatch.setattr(mod, attr, fn)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
        except Exception:                              # a crash also counts as caught
            caught.append(pin.__name__ + "!")
    assert caught, f"no pin caught the planted mistake: {name}"
