"""Checks that pin the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with:
  * hand derivations of Eq. 1 on one- and two-neuron networks,
  * the exact linear program over a box when every ReLU is active (SLR is then exact),
  * brute-force sampling (every sampled point lies inside every propagated bound),
  * closed-form unsafe volumes (Irwin-Hall simplex, |x0 - 1/2| > 1/4),
  * a dense grid of points on tiny random networks (every point in an unsafe leaf is unsafe),
  * exact accounting invariants.
They are plain functions so that the mutation tests can re-run them against an oracle with a
planted mistake and require that at least one of them fails.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import synth
from oracle import count, slr


def _f32(a):
    return np.asarray(a, np.float32)


def relu_identity_net():
    """x in [-1, 1] -> z = x -> y = ReLU(z)."""
    return [(_f32([[1.0]]), _f32([0.0])), (_f32([[1.0]]), _f32([0.0]))]


def two_neuron_net(w_out):
    """z1 = x1 + x2, z2 = x1 - x2 on [-1, 1]^2; y = w_out . ReLU(z)."""
    return [(_f32([[1, 1], [1, -1]]), _f32([0, 0])), (_f32([w_out]), _f32([0.0]))]


def pin_eq1_single_relu():
    """Eq. 1 by hand: z = x on [-1,1] gives l=-1, u=1, lam=1/2, L = x/2, U = (x+1)/2."""
    net = relu_identity_net()
    g_lo, g_hi, tr = slr.propagate(net, [[1.0]], [0.0], [[-1.0]], [[1.0]], keep=True)
    t = tr[0]
    assert abs(t["lo"][0, 0] + 1.0) < 1e-12 and abs(t["hi"][0, 0] - 1.0) < 1e-12
    assert np.allclose(t["Lr"][0, 0], [0.0, 0.5], atol=1e-12)
    assert np.allclose(t["Ur"][0, 0], [0.5, 0.5], atol=1e-12)
    assert abs(g_lo[0, 0] + 0.5) < 1e-12 and abs(g_hi[0, 0] - 1.0) < 1e-12
    assert g_lo[0, 0] <= -0.5 and g_hi[0, 0] >= 1.0           # outward rounding only
    # the same box with d = -1.5 is provably safe, with d = +0.6 provably unsafe
    g_lo, g_hi = slr.propagate(net, [[1.0]], [-1.5], [[-1.0]], [[1.0]])
    assert slr.classify(g_lo, g_hi)[0] == 2
    g_lo, g_hi = slr.propagate(net, [[1.0]], [0.6], [[-1.0]], [[1.0]])
    assert slr.classify(g_lo, g_hi)[0] == 1


def pin_two_neurons():
    """Hand derivation with both signs of output weight (exercises W+ and W-).

    Each hidden neuron has l=-2, u=2, lam=1/2: L1=(x1+x2)/2, U1=(x1+x2+2)/2,
    L2=(x1-x2)/2, U2=(x1-x2+2)/2.  For y = a1 + a2: [L1+L2, U1+U2] = [x1, x1+2] -> [-1, 3].
    For y = a1 - a2: [L1-U2, U1-L2] = [x2-1, x2+1] -> [-2, 2].
    """
    box = ([[-1.0, -1.0]], [[1.0, 1.0]])
    g_lo, g_hi = slr.propagate(two_neuron_net([1, 1]), [[1.0]], [0.0], *box)
    assert abs(g_lo[0, 0] + 1.0) < 1e-12 and abs(g_hi[0, 0] - 3.0) < 1e-12
    g_lo, g_hi = slr.propagate(two_neuron_net([1, -1]), [[1.0]], [0.0], *box)
    assert abs(g_lo[0, 0] + 2.0) < 1e-12 and abs(g_hi[0, 0] - 2.0) < 1e-12
    # on [0,1] x [-1,1] neuron 1 still crosses (l=-1, u=2, lam=2/3) while neuron 2 has
    # l=-1, u=2 as well; y = a1 + a2 gives [L1+L2, U1+U2] = 2/3 [2 x1, 2 x1 + 2] -> [0, 8/3]
    g_lo, g_hi = slr.propagate(two_neuron_net([1, 1]), [[1.0]], [0.0], [[0.0, -1.0]], [[1.0, 1.0]])
    assert abs(g_lo[0, 0] - 0.0) < 1e-12 and abs(g_hi[0, 0] - 8.0 / 3.0) < 1e-12


def pin_linear_regime(seed=0):
    """All ReLUs active (identity first layer on a positive box): bounds equal the exact LP."""
    rng = np.random.default_rng(seed)
    for d in (2, 3, 4):
        W2 = rng.normal(size=(2, d)).astype(np.float32)
        b2 = rng.normal(size=2).astype(np.float32)
        net = [(np.eye(d, dtype=np.float32), np.zeros(d, np.float32)), (W2, b2)]
        C = np.array([[1.0, 0.0], [0.0, -1.0]], np.float32)
        dv = np.zeros(2, np.float32)
        blo, bhi = synth.random_boxes(np.zeros(d), np.ones(d), 20, seed + d, 8)
        g_lo, g_hi = slr.propagate(net, C, dv, blo, bhi)
        corners = np.array(np.meshgrid(*[[0, 1]] * d, indexing="ij")).reshape(d, -1).T
        for i in range(blo.shape[0]):
            v = blo[i].astype(np.float64) + (bhi[i] - blo[i]).astype(np.float64) * corners
            gv = slr.property_values(net, C, dv, v)
            assert np.allclose(g_lo[i], gv.min(axis=0), atol=1e-12, rtol=1e-12)
            assert np.allclose(g_hi[i], gv.max(axis=0), atol=1e-12, rtol=1e-12)


def _eval_eq(E, x):
    return E[..., 0] + np.einsum("ni,pi->pn", E[..., 1:], x) if E.ndim == 2 else None


def pin_soundness(seed=0, n_boxes=6, n_points=4000, alpha=False, act="relu"):
    """Brute force: every sampled point (and every vertex) lies inside every bound."""
    rng = np.random.default_rng(seed)
    shapes = ([2, 16, 16, 1], [3, 8, 8, 2], [4, 10, 10, 10, 3])
    for si, sizes in enumerate(shapes):
        net = synth.make_net(sizes, seed * 10 + si)
        if act != "relu":
            net = synth.with_activation(net, act)
        n_out = sizes[-1]
        C = rng.normal(size=(min(2, n_out), n_out)).astype(np.float32)
        dv = rng.normal(scale=0.1, size=C.shape[0]).astype(np.float32)
        d = sizes[0]
        blo, bhi = synth.uniform_boxes(-np.ones(d), np.ones(d), n_boxes, seed * 7 + si, 0.6)
        al = None
        if alpha:
            al = rng.uniform(0, 1, size=(n_boxes, sum(sizes[1:-1])))
        g_lo, g_hi, tr = slr.propagate(net, C, dv, blo, bhi, alpha=al, keep=True)
        for b in range(n_boxes):
            x = slr.sample_points(blo[b], bhi[b], n_points, rng)
            zs = slr.preactivations(net, x)
            for li, z in enumerate(zs):
                t = tr[li]
                Lx = t["L"][b, :, 0] + x @ t["L"][b, :, 1:].T
                Ux = t["U"][b, :, 0] + x @ t["U"][b, :, 1:].T
                assert np.all(Lx <= z + 1e-12 * (1 + np.abs(z)))
                assert np.all(z <= Ux + 1e-12 * (1 + np.abs(z)))
                assert np.all(t["lo"][b] <= z.min(axis=0))
                assert np.all(z.max(axis=0) <= t["hi"][b])
                a = slr.act_fn(act, z)
                Lr = t["Lr"][b, :, 0] + x @ t["Lr"][b, :, 1:].T
                Ur = t["Ur"][b, :, 0] + x @ t["Ur"][b, :, 1:].T
                assert np.all(Lr <= a + 1e-12 * (1 + a))
                assert np.all(a <= Ur + 1e-12 * (1 + a))
            gv = slr.property_values(net, C, dv, x)
            assert np.all(g_lo[b] <= gv.min(axis=0))
            assert np.all(gv.max(axis=0) <= g_hi[b])


def irwin_hall_net():
    """y = x0 + x1 + x2 + b on [0,1]^3 through an identity hidden layer, b = float32(-2.98)."""
    return [(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
            (_f32([[1, 1, 1]]), _f32([-2.98]))]


def irwin_hall_volume():
    """Exact volume of {x in [0,1]^3 : sum x > -b} = (3 + b)^3 / 6 for the float32 b."""
    t = Fraction(3) + Fraction(float(np.float32(-2.98)))
    return t ** 3 / 6


def pin_irwin_hall():
    net = irwin_hall_net()
    V = irwin_hall_volume()
    lo, hi = np.zeros(3), np.ones(3)
    prev = None
    for D in (18, 24, 30):
        r = count.count_exact(net, [[1.0]], [0.0], lo, hi, D, 1 << 22)
        assert r["unsafe_exact"] <= V <= r["unsafe_exact"] + r["undecided_exact"]
        if prev is not None:
            # six more levels halve every side twice: the undecided shell shrinks ~4x
            assert r["undecided_exact"] <= prev / 2
        prev = r["undecided_exact"]
    # at depth 30 (sides 2^-10) most of the simplex (edge 0.02) is resolved unsafe
    assert r["unsafe_exact"] > V / 2


def abs_net():
    """y = ReLU(x0 - 1/2) + ReLU(1/2 - x0) - 1/4 on [0,1]^2; unsafe (y > 0) volume = 1/2."""
    return [(_f32([[1, 0], [-1, 0]]), _f32([-0.5, 0.5])), (_f32([[1, 1]]), _f32([-0.25]))]


def pin_abs_closed_form():
    net = abs_net()
    r = count.count_exact(net, [[1.0]], [0.0], np.zeros(2), np.ones(2), 14, 1 << 22, trace=True)
    assert r["unsafe_exact"] <= Fraction(1, 2) <= r["unsafe_exact"] + r["undecided_exact"]
    # only the 4 columns of width 2^-7 touching x0 = 1/4 or 3/4 can stay undecided
    assert r["undecided_exact"] <= Fraction(4, 2 ** 7)
    for lev in r["levels"]:
        for i, c in enumerate(lev["cls"]):
            a, b = lev["lo"][i, 0], lev["hi"][i, 0]
            if c == 1:
                assert b <= 0.25 or a >= 0.75
            elif c == 2:
                assert a >= 0.25 and b <= 0.75


def pin_dense_grid(seed=0, cells=1024, act="relu"):
    """tiny2d: leaves classify every point of an aligned grid correctly (no tolerance)."""
    inst = synth.tiny2d(seed) if act == "relu" else synth.tanh2d(seed, act)
    r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, inst.max_depth,
                          inst.max_leaves, trace=True)
    h = 2.0 / cells
    centers = -1.0 + h * (np.arange(cells) + 0.5)
    X, Y = np.meshgrid(centers, centers, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    g = slr.property_values(inst.net, inst.C, inst.dvec, pts)[:, 0]
    unsafe_pt = g > 0.0
    grid_frac = Fraction(int(unsafe_pt.sum()), cells * cells)
    assert r["unsafe_exact"] <= grid_frac <= r["unsafe_exact"] + r["undecided_exact"]
    G = unsafe_pt.reshape(cells, cells)
    for lev in r["levels"]:
        for i, c in enumerate(lev["cls"]):
            if c == 0:
                continue
            i0 = int(round((lev["lo"][i, 0] + 1.0) / h))
            i1 = int(round((lev["hi"][i, 0] + 1.0) / h))
            j0 = int(round((lev["lo"][i, 1] + 1.0) / h))
            j1 = int(round((lev["hi"][i, 1] + 1.0) / h))
            blockv = G[i0:i1, j0:j1]
            assert blockv.size > 0
            if c == 1:
                assert blockv.all()
            else:
                assert not blockv.any()


def pin_accounting(seed=1):
    inst = synth.tiny2d(seed)
    prev = None
    for D in (6, 10, 14):
        r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, D, 1 << 22,
                              trace=True)
        assert r["unsafe_exact"] + r["safe_exact"] + r["undecided_exact"] == 1
        if prev is not None:
            assert prev["unsafe_exact"] <= r["unsafe_exact"]
            assert prev["safe_exact"] <= r["safe_exact"]
        prev = r
        for lev in r["levels"]:
            t = lev["depth"]
            w = lev["hi"] - lev["lo"]
            # on a cube every box of depth t is the cube halved t times, widest side first
            assert np.all(w[:, t % 2] == 2.0 * 2.0 ** -(t // 2))
            assert np.all(lev["path"] >> np.uint64(t) == 1)


def scaled_relu_net(w_out):
    """x in [-1, 1] -> z = x -> y = w_out * ReLU(z) (one crossing neuron, lam = 1/2)."""
    return [(_f32([[1.0]]), _f32([0.0])), (_f32([[w_out]]), _f32([0.0]))]


def pin_alpha_adam_closed_form():
    """Alpha optimizer on one crossing neuron, derived by hand.

    With y = -2 ReLU(x) on [-1, 1] and the row g = y - 0.1, the centre value is -0.1 (not
    unsafe), so the objective is g_hi.  The lower line alpha*x of the ReLU meets the negative
    output weight, so g_hi = max_x(-2 alpha x) - 0.1 = 2 alpha - 0.1: dJ/dalpha = 2 for every
    alpha > 0.  With a constant gradient Adam's bias-corrected moments are m_hat = 2 and
    v_hat = 4 at every step, so each step moves alpha by lr * 2 / (2 + eps) against the
    gradient: from lam = 1/2, three steps of lr = 0.1 end at alpha = 0.2, J = 0.3.
    The mirrored case y = +2 ReLU(x), g = y + 0.1 has an unsafe centre (0.1 > 0), objective
    -g_lo = -(min_x 2 alpha x + 0.1) = 2 alpha - 0.1, and the same trajectory.
    """
    from oracle import alpha as A
    step = 0.1 * 2.0 / (2.0 + 1e-8)
    for w_out, dv, mode in ((-2.0, -0.1, 0), (2.0, 0.1, 1)):
        net = scaled_relu_net(w_out)
        lo, hi = np.array([[-1.0]]), np.array([[1.0]])
        m, r = A.objective_weights(net, [[1.0]], [dv], lo, hi)
        assert m[0] == mode and r[0] == 0
        assert abs(A.plain_lambda(net, [[1.0]], [dv], lo, hi)[0, 0] - 0.5) < 1e-15
        g = A.gradient(net, [[1.0]], [dv], lo, hi, np.array([[0.5]]))
        assert abs(g[0, 0] - 2.0) < 1e-12
        for steps in (1, 3):
            best, jb = A.optimize(net, [[1.0]], [dv], lo, hi, steps=steps, lr=0.1)
            assert abs(best[0, 0] - (0.5 - steps * step)) < 1e-12, (steps, best)
            assert abs(jb[0] - (2.0 * (0.5 - steps * step) - 0.1)) < 1e-12, (steps, jb)
        # past alpha = 0 the projection holds it there: J = -0.1 is the least objective
        best, jb = A.optimize(net, [[1.0]], [dv], lo, hi, steps=8, lr=0.1)
        assert best[0, 0] == 0.0 and abs(jb[0] + 0.1) < 1e-12


def pin_alpha_objective_row():
    """The objective row is the property row with the smallest centre value.

    y = ReLU(x) on [-1, 1] with rows g0 = y + 0.5 and g1 = -y - 0.5: at the centre g0 = 0.5
    and g1 = -0.5, so the box is not unsafe there and the objective is g1_hi.  g1's upper
    bound uses the ReLU's lower line: g1_hi = max_x(-alpha x) - 0.5 = alpha - 0.5, gradient 1,
    while g0_hi = 1.5 does not depend on alpha.  Three Adam steps of lr = 0.1 from lam = 1/2
    give alpha = 0.2; optimizing row 0 (or the unsafe-mode objective, whose min over rows is
    g1_lo = -1.5 for every alpha) would leave alpha at 1/2.
    """
    from oracle import alpha as A
    net = scaled_relu_net(1.0)
    C = [[1.0], [-1.0]]
    dv = [0.5, -0.5]
    lo, hi = np.array([[-1.0]]), np.array([[1.0]])
    m, r = A.objective_weights(net, C, dv, lo, hi)
    assert m[0] == 0 and r[0] == 1
    best, jb = A.optimize(net, C, dv, lo, hi, steps=3, lr=0.1)
    step = 0.1 / (1.0 + 1e-8)
    assert abs(best[0, 0] - (0.5 - 3 * step)) < 1e-12, best
    assert abs(jb[0] - (0.5 - 3 * step - 0.5)) < 1e-12, jb
    # both rows positive at the centre: unsafe mode, J = -min_r g_lo_r
    m, r = A.objective_weights(net, C, [0.5, 0.5], lo, hi)
    assert m[0] == 1


def act_neuron_net(act):
    """x -> z = x -> y = s(z) for s = tanh or the sigmoid."""
    return synth.with_activation([(_f32([[1.0]]), _f32([0.0])), (_f32([[1.0]]), _f32([0.0]))], act)


def pin_act_single_neuron_bruteforce():
    """One tanh / sigmoid neuron on intervals left of, right of, around and far around 0: the
    output bounds equal lam a + min h and lam b + max h, with lam the chord slope over [a, b]
    and min / max of h(z) = s(z) - lam z found by brute force on 2e6 grid points (the exact
    extrema lie within (step)^2 of the grid's), so a wrong critical point or a missing
    candidate shows.  Left of 0 both functions are convex, so the chord is the upper line and
    the upper bound at b is s(b) itself; right of 0 they are concave and the lower bound at a
    is s(a)."""
    for act in ("tanh", "sigmoid"):
        f = (lambda z: np.tanh(z)) if act == "tanh" else (lambda z: 1.0 / (1.0 + np.exp(-z)))
        net = act_neuron_net(act)
        for a, b in ((-3.0, -1.0), (0.5, 2.5), (-1.0, 1.0), (-0.25, 4.0), (-20.0, 20.0),
                     (-6.0, 0.125)):
            g_lo, g_hi = slr.propagate(net, [[1.0]], [0.0], [[a]], [[b]])
            lam = (f(b) - f(a)) / (b - a)
            z = np.linspace(a, b, 2_000_001)
            h = f(z) - lam * z
            step = (b - a) / 2e6
            assert g_lo[0, 0] <= lam * a + h.min() + 1e-12
            assert g_lo[0, 0] >= lam * a + h.min() - step ** 2 - 1e-12, (act, a, b)
            assert g_hi[0, 0] >= lam * b + h.max() - 1e-12
            assert g_hi[0, 0] <= lam * b + h.max() + step ** 2 + 1e-12, (act, a, b)
            if b <= 0.0:                       # convex piece: the chord lies above s
                assert abs(g_hi[0, 0] - f(b)) < 1e-12
            if a >= 0.0:                       # concave piece: the chord lies below s
                assert abs(g_lo[0, 0] - f(a)) < 1e-12


def pin_act_soundness():
    """Random tanh and sigmoid networks: every sampled point lies inside every bound."""
    for act in ("tanh", "sigmoid"):
        pin_soundness(seed=3, n_boxes=4, n_points=2000, act=act)


def pin_act_dense_grid():
    """tanh and sigmoid versions of tiny2d: leaves classify an aligned grid correctly."""
    for act in ("tanh", "sigmoid"):
        pin_dense_grid(seed=1, cells=512, act=act)


def pin_split_rule_hand():
    """Crossing-score split (split_layers = 1), derived by hand.  On [0, 1]^2 with hidden
    neurons z0 = x1 - 0.4 (crossing: l = -0.4, u = 0.6; it depends on x1 only) and
    z1 = x0 + 5 (active), y = ReLU(z0) + ReLU(z1) - 5.2: the only crossing neuron scores side 1
    with |1| * 1 and side 0 with 0, so the root is cut at x1 = 1/2, where widest-first (a tie of
    two unit sides, lowest index) cuts x0.  Below: on x1 in [0, 1/2] z0 still crosses
    (l = -0.4, u = 0.1) and side 1 (score 1/2) is cut again; on x1 in [1/2, 1] z0 is active,
    no neuron crosses and the widest side, x0, is cut.  With x1 confined to [0, 2^-7] and
    z0 = x1 - 2^-8 (crossing, so only side 1 scores) side 1 is narrower than 2^-6 of the
    widest side, no candidate, and side 0 is cut."""
    net = [(_f32([[0.0, 1.0], [1.0, 0.0]]), _f32([-0.4, 5.0])), (_f32([[1.0, 1.0]]), _f32([-5.2]))]
    r = count.count_exact(net, [[1.0]], [0.0], [0.0, 0.0], [1.0, 1.0], 2, 1 << 10, trace=True,
                          split_layers=1)
    assert r["levels"][0]["side"][0] == 1 and r["levels"][0]["robust"][0]
    lev1 = r["levels"][1]
    assert lev1["cls"].tolist() == [0, 0]
    assert lev1["hi"][0, 1] == 0.5 and lev1["lo"][1, 1] == 0.5
    assert lev1["side"].tolist() == [1, 0] and lev1["robust"].all()
    r = count.count_exact(net, [[1.0]], [0.0], [0.0, 0.0], [1.0, 1.0], 1, 1 << 10, trace=True)
    assert r["levels"][0]["side"][0] == 0
    net2 = [(_f32([[0.0, 1.0], [1.0, 0.0]]), _f32([-2.0 ** -8, 5.0])), net[1]]
    r = count.count_exact(net2, [[1.0]], [0.0], [0.0, 0.0], [1.0, 2.0 ** -7], 1, 1 << 10,
                          trace=True, split_layers=1)
    assert r["levels"][0]["cls"][0] == 0 and r["levels"][0]["side"][0] == 0


def pin_split_rule_grid():
    """Dense-grid check and exact accounting with the crossing-score split on tiny2d."""
    inst = synth.tiny2d(2)
    r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 14, 1 << 20,
                          trace=True, split_layers=2)
    assert r["unsafe_exact"] + r["safe_exact"] + r["undecided_exact"] == 1
    cells = 512
    h = 2.0 / cells
    centers = -1.0 + h * (np.arange(cells) + 0.5)
    X, Y = np.meshgrid(centers, centers, indexing="ij")
    G = (slr.property_values(inst.net, inst.C, inst.dvec,
                             np.stack([X.ravel(), Y.ravel()], axis=1))[:, 0] > 0).reshape(cells, cells)
    for lev in r["levels"]:
        for i, c in enumerate(lev["cls"]):
            if c == 0:
                continue
            i0, i1 = (int(round((lev["lo"][i, 0] + 1) / h)), int(round((lev["hi"][i, 0] + 1) / h)))
            j0, j1 = (int(round((lev["lo"][i, 1] + 1) / h)), int(round((lev["hi"][i, 1] + 1) / h)))
            block = G[i0:i1, j0:j1]
            assert block.size > 0 and (block.all() if c == 1 else not block.any())


def pin_two_ratio_hand():
    """Two ratios, derived by hand.  x in [-1, 1], h = ReLU(x), z = h - 1/4, y = ReLU(z).
    The first neuron has L = U = x, so both forms give L = x/2, U = (x + 1)/2.  For z:
    L = x/2 - 1/4 (range [-3/4, 1/4]) and U = x/2 + 1/4 (range [-1/4, 3/4]), so l = -3/4,
    u = 3/4.  Eq. 1 (one ratio 1/2): L' = x/4 - 1/8, U' = (U + 3/4)/2 = x/4 + 1/2, bounds
    [-3/8, 3/4].  Two ratios: lamU = (3/4)/(3/4 + 1/4) = 3/4, U' = 3/4 (U + 1/4) = 3x/8 + 3/8;
    lamL = (1/4)/(1/4 + 3/4) = 1/4, L' = x/8 - 1/16; bounds [-3/16, 3/4]."""
    net = [(_f32([[1.0]]), _f32([0.0])), (_f32([[1.0]]), _f32([-0.25])), (_f32([[1.0]]), _f32([0.0]))]
    for relax, lo_exp, L2, U2 in (("one", -0.375, [-0.125, 0.25], [0.5, 0.25]),
                                  ("two", -0.1875, [-0.0625, 0.125], [0.375, 0.375])):
        g_lo, g_hi, tr = slr.propagate(net, [[1.0]], [0.0], [[-1.0]], [[1.0]], keep=True,
                                       relax=relax)
        assert np.allclose(tr[0]["Lr"][0, 0], [0.0, 0.5], atol=1e-12)
        assert np.allclose(tr[0]["Ur"][0, 0], [0.5, 0.5], atol=1e-12)
        assert np.allclose(tr[1]["Lr"][0, 0], L2, atol=1e-12), (relax, tr[1]["Lr"][0, 0])
        assert np.allclose(tr[1]["Ur"][0, 0], U2, atol=1e-12), (relax, tr[1]["Ur"][0, 0])
        assert abs(g_lo[0, 0] - lo_exp) < 1e-12 and abs(g_hi[0, 0] - 0.75) < 1e-12
    # With z = h + b, b = fl32(-0.6), the lower equation x/2 + b of z stays below zero (its
    # max is 0.5 + b) while the neuron crosses (l = b - 0.5, u = 1 + b).  Two ratios give
    # L' = 0 and, from U = x/2 + 1/2 + b with range [b, 1 + b], U' = (1 + b)(U - b);
    # one ratio lam = u / (u - l) gives L' = lam (x/2 + b) and U' = lam (U - l) = lam (x/2 + 1).
    net[1] = (_f32([[1.0]]), _f32([-0.6]))
    b6 = float(np.float32(-0.6))
    l, u, lU, uL = b6 - 0.5, 1.0 + b6, b6, 0.5 + b6
    assert uL < 0.0 < u and l < lU < 0.0
    for relax in ("one", "two"):
        g_lo, g_hi, tr = slr.propagate(net, [[1.0]], [0.0], [[-1.0]], [[1.0]], keep=True,
                                       relax=relax)
        if relax == "one":
            lam = u / (u - l)
            L2, U2 = [lam * b6, lam * 0.5], [lam, lam * 0.5]
        else:
            lam = u / (u - lU)
            L2, U2 = [0.0, 0.0], [lam * 0.5, lam * 0.5]
        assert np.allclose(tr[1]["Lr"][0, 0], L2, atol=1e-12), (relax, tr[1]["Lr"][0, 0])
        assert np.allclose(tr[1]["Ur"][0, 0], U2, atol=1e-12), (relax, tr[1]["Ur"][0, 0])
        assert abs(g_lo[0, 0] - (L2[0] - L2[1])) < 1e-12
        assert abs(g_hi[0, 0] - (U2[0] + U2[1])) < 1e-12


def pin_two_ratio_soundness_and_grid():
    """Two ratios: sampled soundness of every bound on random networks (as pin_soundness), and
    the dense-grid check of the exact count on tiny2d."""
    rng = np.random.default_rng(5)
    for si, sizes in enumerate(([2, 16, 16, 1], [3, 8, 8, 8, 2], [4, 10, 10, 10, 3])):
        net = synth.make_net(sizes, 70 + si)
        n_out = sizes[-1]
        C = rng.normal(size=(min(2, n_out), n_out)).astype(np.float32)
        dv = rng.normal(scale=0.1, size=C.shape[0]).astype(np.float32)
        blo, bhi = synth.uniform_boxes(-np.ones(sizes[0]), np.ones(sizes[0]), 5, 80 + si, 0.6)
        g_lo, g_hi, tr = slr.propagate(net, C, dv, blo, bhi, keep=True, relax="two")
        for b in range(5):
            x = slr.sample_points(blo[b], bhi[b], 2000, rng)
            for li, z in enumerate(slr.preactivations(net, x)):
                t = tr[li]
                a = np.maximum(z, 0.0)
                Lr = t["Lr"][b, :, 0] + x @ t["Lr"][b, :, 1:].T
                Ur = t["Ur"][b, :, 0] + x @ t["Ur"][b, :, 1:].T
                assert np.all(Lr <= a + 1e-12 * (1 + a)) and np.all(a <= Ur + 1e-12 * (1 + a))
            gv = slr.property_values(net, C, dv, x)
            assert np.all(g_lo[b] <= gv.min(axis=0)) and np.all(gv.max(axis=0) <= g_hi[b])
    inst = synth.tiny2d(4)
    r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 14, 1 << 20,
                          trace=True, relax="two")
    assert r["unsafe_exact"] + r["safe_exact"] + r["undecided_exact"] == 1
    cells = 512
    h = 2.0 / cells
    centers = -1.0 + h * (np.arange(cells) + 0.5)
    X, Y = np.meshgrid(centers, centers, indexing="ij")
    G = (slr.property_values(inst.net, inst.C, inst.dvec,
                             np.stack([X.ravel(), Y.ravel()], axis=1))[:, 0] > 0).reshape(cells, cells)
    for lev in r["levels"]:
        for i, c in enumerate(lev["cls"]):
            if c == 0:
                continue
            i0, i1 = (int(round((lev["lo"][i, 0] + 1) / h)), int(round((lev["hi"][i, 0] + 1) / h)))
            j0, j1 = (int(round((lev["lo"][i, 1] + 1) / h)), int(round((lev["hi"][i, 1] + 1) / h)))
            block = G[i0:i1, j0:j1]
            assert block.size > 0 and (block.all() if c == 1 else not block.any())


ALL_PINS = [pin_eq1_single_relu, pin_two_neurons, pin_linear_regime, pin_soundness,
            pin_irwin_hall, pin_abs_closed_form, pin_dense_grid, pin_accounting,
            pin_alpha_adam_closed_form, pin_alpha_objective_row,
            pin_act_single_neuron_bruteforce, pin_act_soundness, pin_act_dense_grid,
            pin_split_rule_hand, pin_split_rule_grid, pin_two_ratio_hand,
            pin_two_ratio_soundness_and_grid]
