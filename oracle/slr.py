"""FP64 symbolic linear relaxation of a ReLU network over boxes (paper §2.2 and §3, Eq. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Representation.  For a batch of B boxes, every neuron carries two affine functions of the
input x in R^d, a lower one L and an upper one U, stored as arrays of shape [B, n, d+1]:
column 0 is the constant term and column i (1..d) the coefficient of x_i, in the network's
own input coordinates.  For every x in the box the neuron's value lies in [L(x), U(x)].

Steps, in the order of §3:
  * first affine layer: L = U = W1 x + b1, exactly;
  * concretization (§2.2): l = min over the box of L, u = max over the box of U, taking
    min(a*lo, a*hi) per coordinate;
  * ReLU with Eq. 1: dead (u <= 0) -> 0; active (l >= 0) -> unchanged; crossing ->
    L <- lam * L, U <- lam * (U - l) with lam = u / (u - l);
  * next affine layer with weights split into W+ = max(W, 0) and W- = min(W, 0):
    L' = W+ L + W- U + b, U' = W+ U + W- L + b;
  * the property rows C y + d are folded into the last affine layer, and each row's
    concrete lower/upper bound is returned.

Rounding: each step subtracts from L's constant (adds to U's) a bound on the rounding error
of that step over the box, gamma_n * (sum of the magnitudes of the terms), so the output
bounds hold for the exact network whose weights are the float32 values.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

UNIT = 2.0 ** -53          # unit roundoff of binary64, round to nearest


def gamma(n: int) -> float:
    """Higham's gamma_n = n u / (1 - n u): bound on the relative error of n roundings."""
    return n * UNIT / (1.0 - n * UNIT)


def _as64(net):
    return [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in net]


def fold_property(net, C, dvec):
    """Fold the property rows into the last affine layer: g = (C W_L) h + (C b_L + d).

    Returns the folded (W_g, b_g) in FP64 and elementwise bounds on their rounding error.
    """
    W_L, b_L = _as64(net)[-1]
    C = np.asarray(C, np.float64)
    dvec = np.asarray(dvec, np.float64)
    Wg = C @ W_L
    bg = C @ b_L + dvec
    n_out = W_L.shape[0]
    Wg_err = gamma(n_out) * (np.abs(C) @ np.abs(W_L))
    bg_err = gamma(n_out + 1) * (np.abs(C) @ np.abs(b_L) + np.abs(dvec))
    return Wg, bg, Wg_err, bg_err


def magnitude(E: np.ndarray, xmag: np.ndarray) -> np.ndarray:
    """Upper bound on |E(x)| over the box: |e0| + sum_i |e_i| * max(|lo_i|, |hi_i|)."""
    return np.abs(E[..., 0]) + np.einsum("bnd,bd->bn", np.abs(E[..., 1:]), xmag)


def concretize_lower(L: np.ndarray, lo: np.ndarray, hi: np.ndarray, xmag: np.ndarray):
    """min over the box of L(x) = l0 + sum_i min(l_i lo_i, l_i hi_i), minus its rounding bound."""
    coef = L[..., 1:]
    a = coef * lo[:, None, :]
    b = coef * hi[:, None, :]
    val = L[..., 0] + np.minimum(a, b).sum(axis=-1)
    d = lo.shape[1]
    return val - gamma(d + 2) * magnitude(L, xmag)


def concretize_upper(U: np.ndarray, lo: np.ndarray, hi: np.ndarray, xmag: np.ndarray):
    """max over the box of U(x) = u0 + sum_i max(u_i lo_i, u_i hi_i), plus its rounding bound."""
    coef = U[..., 1:]
    a = coef * lo[:, None, :]
    b = coef * hi[:, None, :]
    val = U[..., 0] + np.maximum(a, b).sum(axis=-1)
    d = lo.shape[1]
    return val + gamma(d + 2) * magnitude(U, xmag)


def _matmul(W: np.ndarray, X: np.ndarray) -> np.ndarray:
    """[J, K] times the neuron axis of X [B, K, c] -> [B, J, c] (one library GEMM)."""
    return np.tensordot(X, W, axes=([1], [1])).transpose(0, 2, 1)


def affine(L, U, W, b, xmag, W_err=None, b_err=None):
    """Affine layer on the equations with the W+/W- rule of symbolic propagation.

    L' = W+ L + W- U + b and U' = W+ U + W- L + b; the constant terms are then moved outward
    by the rounding bound gamma_{2K+3} * (sum_k |W_jk| (|L_k| + |U_k|) + |b_j|), plus the
    effect of the error bounds ``W_err``/``b_err`` of the weights themselves if given.
    """
    Wp = np.maximum(W, 0.0)
    Wm = np.minimum(W, 0.0)
    Ln = _matmul(Wp, L) + _matmul(Wm, U)
    Un = _matmul(Wp, U) + _matmul(Wm, L)
    Ln[..., 0] += b
    Un[..., 0] += b
    K = W.shape[1]
    mag = magnitude(L, xmag) + magnitude(U, xmag)          # [B, K]
    err = gamma(2 * K + 3) * (mag @ np.abs(W).T + np.abs(b))
    if W_err is not None:
        err = err + mag @ W_err.T + b_err
    Ln[..., 0] -= err
    Un[..., 0] += err
    return Ln, Un


def relu_relax(L, U, lo_b, hi_b, xmag, alpha=None):
    """ReLU on the equations, Eq. 1.

    ``lo_b``/``hi_b`` are the concrete bounds [B, n] of L and U.  Dead neurons (hi <= 0) get
    L = U = 0; active ones (lo >= 0) are unchanged; crossing ones get
    L <- lam L and U <- lam (U - lo) with lam = hi / (hi - lo), rounded up (capped at 1).
    With ``alpha`` [B, n] the lower line uses slope alpha instead of lam.
    """
    dead = hi_b <= 0.0
    cross = (lo_b < 0.0) & (hi_b > 0.0)
    denom = np.where(cross, hi_b - lo_b, 1.0)
    lam = np.where(cross, hi_b / denom, 1.0)
    lam = np.minimum(1.0, lam * (1.0 + 4.0 * UNIT))
    low_slope = lam if alpha is None else np.where(cross, alpha, 1.0)

    magL = magnitude(L, xmag)
    magU = magnitude(U, xmag)
    Ln = L.copy()
    Un = U.copy()
    c = cross[..., None]
    Ln = np.where(c, low_slope[..., None] * L, Ln)
    shifted = U.copy()
    shifted[..., 0] -= lo_b
    Un = np.where(c, lam[..., None] * shifted, Un)
    Ln[..., 0] -= np.where(cross, gamma(3) * low_slope * magL, 0.0)
    Un[..., 0] += np.where(cross, gamma(3) * lam * (magU + np.abs(lo_b)), 0.0)
    Ln[dead] = 0.0
    Un[dead] = 0.0
    return Ln, Un


def relu_relax_two(L, U, lo_b, hi_b, lU, uL, xmag):
    """ReLU with two ratios, one per equation (the separate-ratio form Eq. 1 is derived from).

    A neuron is dead when u = max U <= 0 and active when l = min L >= 0, as in Eq. 1.  When it
    crosses, each equation gets the chord of its own range: the upper one, with range
    [lU, u], becomes lamU (U - lU), lamU = u / (u - lU) rounded up (or stays U when lU >= 0:
    then ReLU(z) <= ReLU(U) = U); the lower one, with range [l, uL], becomes lamL L,
    lamL = uL / (uL - l) (or 0 when uL <= 0): any slope in [0, 1] gives ReLU(z) >= slope z >=
    slope L.
    """
    dead = hi_b <= 0.0
    cross = (lo_b < 0.0) & (hi_b > 0.0)
    up_chord = cross & (lU < 0.0)
    lamU = np.where(up_chord, hi_b / np.where(up_chord, hi_b - lU, 1.0), 1.0)
    lamU = np.minimum(1.0, lamU * (1.0 + 4.0 * UNIT))
    lo_zero = cross & (uL <= 0.0)
    lo_chord = cross & (uL > 0.0)
    lamL = np.where(lo_chord, uL / np.where(lo_chord, uL - lo_b, 1.0), 1.0)
    lamL = np.where(lo_zero, 0.0, lamL)
    magL = magnitude(L, xmag)
    magU = magnitude(U, xmag)
    Ln = np.where(cross[..., None], lamL[..., None] * L, L)
    shifted = U.copy()
    shifted[..., 0] -= np.where(up_chord, lU, 0.0)
    Un = np.where(up_chord[..., None], lamU[..., None] * shifted, U)
    Ln[..., 0] -= np.where(cross, gamma(3) * lamL * magL, 0.0)
    Un[..., 0] += np.where(up_chord, gamma(3) * lamU * (magU + np.abs(lU)), 0.0)
    Ln[dead] = 0.0
    Un[dead] = 0.0
    return Ln, Un


def activation_of(net) -> str:
    """'relu' (the paper's networks), or 'tanh' / 'sigmoid' for a net that carries ``act``."""
    return getattr(net, "act", "relu")


def act_fn(act: str, z):
    """The activation itself, in float64."""
    z = np.asarray(z, np.float64)
    if act == "relu":
        return np.maximum(z, 0.0)
    if act == "tanh":
        return np.tanh(z)
    if act == "sigmoid":
        return 1.0 / (1.0 + np.exp(-z))
    raise ValueError(act)


def act_critical(act: str, lam):
    """The z >= 0 where the derivative of tanh (1 - tanh^2 z) or of the sigmoid (s (1 - s))
    equals lam; the derivative is even and has one maximum at 0, so +-z are the only points
    with that slope (none when lam exceeds the maximum, which a chord slope never does)."""
    lam = np.asarray(lam, np.float64)
    if act == "tanh":
        t = np.sqrt(np.clip(1.0 - lam, 0.0, 1.0))
        return np.arctanh(np.minimum(t, 1.0 - 1e-16))
    s = np.sqrt(np.clip(1.0 - 4.0 * lam, 0.0, 1.0))
    p = np.minimum(0.5 * (1.0 + s), 1.0 - 1e-16)
    return np.log(p / (1.0 - p))


def act_relax(L, U, lo_b, hi_b, xmag, act):
    """Tanh or sigmoid on the equations, by two parallel lines (the extension of Eq. 1 the paper
    leaves to future work, §3).

    On [l, u] take the chord slope lam = (s(u) - s(l)) / (u - l) (the derivative at l for a
    point); h(z) = s(z) - lam z then has its extrema over [l, u] at l, u or at the points +-z*
    where s'(z) = lam, so lam z + min h <= s(z) <= lam z + max h on [l, u].  With lam > 0 and
    L <= z <= U: L' = lam L + min h, U' = lam U + max h, plus rounding margins.
    """
    l = np.asarray(lo_b, np.float64)
    u = np.asarray(hi_b, np.float64)
    w = u - l
    fl, fu = act_fn(act, l), act_fn(act, u)
    if act == "tanh":
        dl = 1.0 - np.tanh(l) ** 2
    else:
        dl = fl * (1.0 - fl)
    lam = np.where(w > 0.0, (fu - fl) / np.where(w > 0.0, w, 1.0), dl)
    zc = act_critical(act, lam)
    hl, hu = fl - lam * l, fu - lam * u
    bl = np.minimum(hl, hu)
    bh = np.maximum(hl, hu)
    for z in (zc, -zc):
        inside = (z > l) & (z < u)
        hz = act_fn(act, z) - lam * z
        bl = np.where(inside, np.minimum(bl, hz), bl)
        bh = np.where(inside, np.maximum(bh, hz), bh)
    # rounding of the few evaluations above (library tanh/exp within a few ulp)
    m = 16.0 * UNIT * (1.0 + np.abs(lam) * (np.abs(l) + np.abs(u)))
    bl = bl - m
    bh = bh + m
    magL = magnitude(L, xmag)
    magU = magnitude(U, xmag)
    Ln = lam[..., None] * L
    Un = lam[..., None] * U
    Ln[..., 0] += bl - gamma(3) * lam * magL
    Un[..., 0] += bh + gamma(3) * lam * magU
    return Ln, Un


def propagate(net, C, dvec, lo, hi, alpha: Optional[np.ndarray] = None, keep: bool = False,
              equations: bool = False, relax: str = "one"):
    """Output-property bounds for a batch of boxes.

    ``lo``/``hi``: [B, d] box corners.  ``alpha``: optional [B, sum of hidden widths] lower
    slopes in [0, 1] (replacing lam for crossing neurons).  Returns ``(g_lo, g_hi)`` of shape
    [B, rows]; with ``keep`` also a list with, per hidden layer, the pre-activation
    equations and bounds and the post-activation equations (for soundness checks); with
    ``equations`` also the property rows' lower and upper equations ``(L, U)`` [B, rows, d+1]
    (last, after the trace if both are asked for).  ``relax``: "one" (Eq. 1, one ratio) or
    "two" (``relu_relax_two``, ReLU networks without alpha).
    """
    layers = _as64(net)
    lo = np.atleast_2d(np.asarray(lo, np.float64))
    hi = np.atleast_2d(np.asarray(hi, np.float64))
    B, d = lo.shape
    xmag = np.maximum(np.abs(lo), np.abs(hi))
    Wg, bg, Wg_err, bg_err = fold_property(net, C, dvec)

    trace = []
    W1, b1 = layers[0]
    if len(layers) == 1:
        W1, b1 = Wg, bg
    eq = np.zeros((B, W1.shape[0], d + 1))
    eq[..., 0] = b1
    eq[..., 1:] = W1
    L = eq
    U = eq.copy()
    if len(layers) == 1:
        # the folded weights' own error still has to be covered
        err = xmag @ Wg_err.T + bg_err
        L[..., 0] -= err
        U[..., 0] += err
        return concretize_lower(L, lo, hi, xmag), concretize_upper(U, lo, hi, xmag)

    a_off = 0
    for li in range(1, len(layers)):
        lo_b = concretize_lower(L, lo, hi, xmag)
        hi_b = concretize_upper(U, lo, hi, xmag)
        a = None
        if alpha is not None:
            n = L.shape[1]
            a = np.asarray(alpha, np.float64)[:, a_off:a_off + n]
            a_off += n
        act = activation_of(net)
        if act == "relu" and relax == "two":
            assert alpha is None
            lU = concretize_lower(U, lo, hi, xmag)
            uL = concretize_upper(L, lo, hi, xmag)
            Lr, Ur = relu_relax_two(L, U, lo_b, hi_b, lU, uL, xmag)
        elif act == "relu":
            Lr, Ur = relu_relax(L, U, lo_b, hi_b, xmag, a)
        else:
            assert alpha is None, "alpha slopes are defined for ReLU networks only"
            Lr, Ur = act_relax(L, U, lo_b, hi_b, xmag, act)
        if keep:
            trace.append(dict(L=L, U=U, lo=lo_b, hi=hi_b, Lr=Lr, Ur=Ur))
        if li == len(layers) - 1:
            L, U = affine(Lr, Ur, Wg, bg, xmag, Wg_err, bg_err)
        else:
            W, b = layers[li]
            L, U = affine(Lr, Ur, W, b, xmag)
    g_lo = concretize_lower(L, lo, hi, xmag)
    g_hi = concretize_upper(U, lo, hi, xmag)
    out = (g_lo, g_hi)
    if keep:
        out = out + (trace,)
    if equations:
        out = out + ((L, U),)
    return out


def classify(g_lo: np.ndarray, g_hi: np.ndarray) -> np.ndarray:
    """Property test of §3 on rows of C y + d > 0.

    1 = unsafe (every row's lower bound > 0: the reachable set lies in the unsafe set),
    2 = safe (some row's upper bound <= 0: no overlap), 0 = undecided (split further).
    """
    unsafe = np.all(g_lo > 0.0, axis=1)
    safe = np.any(g_hi <= 0.0, axis=1)
    cls = np.zeros(g_lo.shape[0], np.int8)
    cls[safe] = 2
    cls[unsafe] = 1
    return cls


def decision_margin(g_lo: np.ndarray, g_hi: np.ndarray) -> np.ndarray:
    """How far each box's bounds are from changing its ``classify`` decision.

    Unsafe: the smallest row lower bound (it must not reach 0).  Safe: the most negative row
    upper bound, negated (the deciding row must stay <= 0).  Undecided: the smaller of the
    largest negated row lower bound (every row's lower bound must pass 0 to become unsafe)
    and the smallest row upper bound (one row's upper bound reaching 0 makes it safe).
    """
    cls = classify(g_lo, g_hi)
    m_unsafe = g_lo.min(axis=1)
    m_safe = (-g_hi).max(axis=1)
    m_und = np.minimum((-g_lo).max(axis=1), g_hi.min(axis=1))
    return np.where(cls == 1, m_unsafe, np.where(cls == 2, m_safe, m_und))


def forward(net, x: np.ndarray) -> np.ndarray:
    """Concrete FP64 forward pass; ``x`` [N, d] -> outputs [N, n_out]."""
    h = np.asarray(x, np.float64)
    layers = _as64(net)
    act = activation_of(net)
    for i, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if i < len(layers) - 1:
            h = act_fn(act, h)
    return h


def preactivations(net, x: np.ndarray) -> List[np.ndarray]:
    """Pre-activation values of every hidden layer at the points ``x`` [N, d]."""
    h = np.asarray(x, np.float64)
    out = []
    layers = _as64(net)
    act = activation_of(net)
    for W, b in layers[:-1]:
        z = h @ W.T + b
        out.append(z)
        h = act_fn(act, z)
    return out


def property_values(net, C, dvec, x: np.ndarray) -> np.ndarray:
    """Rows of C y + d at the points ``x`` [N, d]."""
    y = forward(net, x)
    return y @ np.asarray(C, np.float64).T + np.asarray(dvec, np.float64)


# ---------------------------------------------------------------------------------------
# Pure-Python per-box twin (tiny networks only): the same steps with explicit loops.
# ---------------------------------------------------------------------------------------

def scalar_bounds(net, C, dvec, lo: Sequence[float], hi: Sequence[float]) -> Tuple[list, list]:
    """One box, plain Python floats and loops; mirrors ``propagate`` step by step."""
    lo = [float(v) for v in lo]
    hi = [float(v) for v in hi]
    d = len(lo)
    xm = [max(abs(a), abs(b)) for a, b in zip(lo, hi)]
    layers = [(np.asarray(W, np.float64).tolist(), np.asarray(b, np.float64).tolist())
              for W, b in net]
    Wg, bg, Wg_err, bg_err = fold_property(net, C, dvec)
    Wg, bg, Wg_err, bg_err = Wg.tolist(), bg.tolist(), Wg_err.tolist(), bg_err.tolist()

    def mag(e):
        return abs(e[0]) + sum(abs(e[i + 1]) * xm[i] for i in range(d))

    def cmin(e):
        s = e[0] + sum(min(e[i + 1] * lo[i], e[i + 1] * hi[i]) for i in range(d))
        return s - gamma(d + 2) * mag(e)

    def cmax(e):
        s = e[0] + sum(max(e[i + 1] * lo[i], e[i + 1] * hi[i]) for i in range(d))
        return s + gamma(d + 2) * mag(e)

    W1, b1 = layers[0]
    L = [[b1[j]] + list(W1[j]) for j in range(len(b1))]
    U = [row[:] for row in L]
    assert len(layers) >= 2, "the scalar twin expects at least one hidden layer"
    for li in range(1, len(layers)):
        nL, nU = [], []
        for j in range(len(L)):
            l_ = cmin(L[j])
            u_ = cmax(U[j])
            if u_ <= 0.0:
                nL.append([0.0] * (d + 1))
                nU.append([0.0] * (d + 1))
            elif l_ >= 0.0:
                nL.append(L[j][:])
                nU.append(U[j][:])
            else:
                lam = min(1.0, (u_ / (u_ - l_)) * (1.0 + 4.0 * UNIT))
                ml, mu = mag(L[j]), mag(U[j])
                a = [lam * v for v in L[j]]
                a[0] -= gamma(3) * lam * ml
                s = U[j][:]
                s[0] -= l_
                bb = [lam * v for v in s]
                bb[0] += gamma(3) * lam * (mu + abs(l_))
                nL.append(a)
                nU.append(bb)
        last = li == len(layers) - 1
        if last:
            W, b = Wg, bg
        else:
            W, b = layers[li]
        K = len(nL)
        mags = [mag(nL[k]) + mag(nU[k]) for k in range(K)]
        L, U = [], []
        for j in range(len(b)):
            lrow = [0.0] * (d + 1)
            urow = [0.0] * (d + 1)
            for k in range(K):
                w = W[j][k]
                for c in range(d + 1):
                    if w >= 0.0:
                        lrow[c] += w * nL[k][c]
                        urow[c] += w * nU[k][c]
                    else:
                        lrow[c] += w * nU[k][c]
                        urow[c] += w * nL[k][c]
            lrow[0] += b[j]
            urow[0] += b[j]
            err = gamma(2 * K + 3) * (sum(abs(W[j][k]) * mags[k] for k in range(K)) + abs(b[j]))
            if last:
                err += sum(Wg_err[j][k] * mags[k] for k in range(K)) + bg_err[j]
            lrow[0] -= err
            urow[0] += err
            L.append(lrow)
            U.append(urow)
    return [cmin(e) for e in L], [cmax(e) for e in U]


def sample_points(lo: np.ndarray, hi: np.ndarray, n: int, rng: np.random.Generator,
                  include_vertices: bool = True) -> np.ndarray:
    """Uniform points of one box plus (for d <= 12) all of its vertices."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = lo.shape[0]
    pts = lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(n, d))
    if include_vertices and d <= 12:
        corners = np.array(np.meshgrid(*[[0, 1]] * d, indexing="ij")).reshape(d, -1).T
        pts = np.vstack([pts, lo + (hi - lo) * corners])
    return pts


def dyadic_exact(x: float) -> bool:
    """True when ``x`` is a finite float representable exactly in float32."""
    return math.isfinite(x) and float(np.float32(x)) == x
