"""Optimized lower slopes for the relaxation of Eq. 1 (test infrastructure only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 1 relaxes a crossing ReLU with the lower line lam * z; any slope alpha in [0, 1] gives a
valid lower line (ReLU(z) >= alpha z), so every crossing neuron of every box can use its own
alpha, optimized by gradient to tighten the bound that decides the box.  Reading used here
(the paper has no alpha; this is the build's addition):

* objective of a box: evaluate the network at the box center; if every property row is
  positive there (the box may be unsafe) maximize min_r g_lo_r, i.e. minimize
  J = -min_r g_lo_r; otherwise minimize J = g_hi_{r*} with r* = argmin_r of the center values;
* alpha starts at lam (so step 0 is the plain relaxation) and takes projected Adam steps
  (lr 0.1, betas (0.9, 0.999), eps 1e-8), clipped to [0, 1]; the best objective seen is kept.

This module writes the alpha-relaxed propagation a second time, in PyTorch float64 on the CPU,
in the same literal lower/upper form as ``slr.propagate`` (without the rounding margins, which
do not change derivatives), so that autograd gives reference gradients.  It is pinned to
``slr.propagate`` and to central finite differences by the tests.
"""
from __future__ import annotations

import math

import numpy as np

from . import slr


def _torch():
    import torch
    return torch


def forward_torch(net, C, dvec, lo, hi, alpha):
    """float64 torch version of ``slr.propagate`` with slopes ``alpha`` [B, sum hidden].

    Returns (g_lo, g_hi) [B, rows] as torch tensors (differentiable in ``alpha``).
    """
    torch = _torch()
    lo = torch.as_tensor(np.asarray(lo, np.float64))
    hi = torch.as_tensor(np.asarray(hi, np.float64))
    B, d = lo.shape
    Wg, bg, _, _ = slr.fold_property(net, C, dvec)
    layers = [(torch.as_tensor(np.asarray(W, np.float64)), torch.as_tensor(np.asarray(b, np.float64)))
              for W, b in net]
    layers[-1] = (torch.as_tensor(Wg), torch.as_tensor(bg))

    def conc_lo(L):
        return L[..., 0] + torch.minimum(L[..., 1:] * lo[:, None, :], L[..., 1:] * hi[:, None, :]).sum(-1)

    def conc_hi(U):
        return U[..., 0] + torch.maximum(U[..., 1:] * lo[:, None, :], U[..., 1:] * hi[:, None, :]).sum(-1)

    W1, b1 = layers[0]
    eq = torch.zeros((B, W1.shape[0], d + 1), dtype=torch.float64)
    eq[..., 0] = b1
    eq[..., 1:] = W1
    L, U = eq, eq.clone()
    off = 0
    for li in range(1, len(layers)):
        l_b = conc_lo(L)
        u_b = conc_hi(U)
        n = L.shape[1]
        a = alpha[:, off:off + n]
        off += n
        dead = u_b <= 0
        cross = (l_b < 0) & (u_b > 0)
        den = torch.where(cross, u_b - l_b, torch.ones_like(u_b))
        lam = torch.where(cross, u_b / den, torch.ones_like(u_b))
        Lc = a[..., None] * L
        shiftU = U.clone()
        shiftU[..., 0] = U[..., 0] - l_b
        Uc = lam[..., None] * shiftU
        keep = ~dead & ~cross
        L = torch.where(cross[..., None], Lc, torch.where(keep[..., None], L, torch.zeros_like(L)))
        U = torch.where(cross[..., None], Uc, torch.where(keep[..., None], U, torch.zeros_like(U)))
        W, b = layers[li]
        Wp = torch.clamp(W, min=0.0)
        Wm = torch.clamp(W, max=0.0)
        Ln = torch.einsum("jk,bkc->bjc", Wp, L) + torch.einsum("jk,bkc->bjc", Wm, U)
        Un = torch.einsum("jk,bkc->bjc", Wp, U) + torch.einsum("jk,bkc->bjc", Wm, L)
        Ln = Ln + torch.cat([b[None, :, None].expand(B, -1, 1), torch.zeros((B, b.shape[0], d), dtype=torch.float64)], -1)
        Un = Un + torch.cat([b[None, :, None].expand(B, -1, 1), torch.zeros((B, b.shape[0], d), dtype=torch.float64)], -1)
        L, U = Ln, Un
    return conc_lo(L), conc_hi(U)


def plain_lambda(net, C, dvec, lo, hi):
    """The ratios lam of the plain relaxation for every hidden neuron, [B, sum hidden]."""
    _, _, tr = slr.propagate(net, C, dvec, lo, hi, keep=True)
    out = []
    for t in tr:
        lo_b, hi_b = t["lo"], t["hi"]
        cross = (lo_b < 0) & (hi_b > 0)
        lam = np.where(cross, hi_b / np.where(cross, hi_b - lo_b, 1.0), 1.0)
        out.append(lam)
    return np.hstack(out)


def objective_weights(net, C, dvec, lo, hi):
    """Per box: (mode, row) with mode 1 = maximize min g_lo (center unsafe), 0 = minimize
    g_hi[row] with row = argmin of the center values."""
    center = 0.5 * (np.asarray(lo, np.float64) + np.asarray(hi, np.float64))
    gc = slr.property_values(net, C, dvec, center)
    unsafe = np.all(gc > 0, axis=1)
    row = np.argmin(gc, axis=1)
    return unsafe.astype(np.int64), row


def objective_torch(g_lo, g_hi, mode, row):
    """J per box (to minimize)."""
    torch = _torch()
    mode_t = torch.as_tensor(mode)
    idx = torch.as_tensor(row)
    j_unsafe = -g_lo.min(dim=1).values
    j_safe = g_hi.gather(1, idx[:, None])[:, 0]
    return torch.where(mode_t == 1, j_unsafe, j_safe)


def gradient(net, C, dvec, lo, hi, alpha):
    """dJ/dalpha by autograd (float64), [B, sum hidden]."""
    torch = _torch()
    mode, row = objective_weights(net, C, dvec, lo, hi)
    a = torch.tensor(np.asarray(alpha, np.float64), requires_grad=True)
    g_lo, g_hi = forward_torch(net, C, dvec, lo, hi, a)
    J = objective_torch(g_lo, g_hi, mode, row).sum()
    J.backward()
    return a.grad.numpy()


def objective(net, C, dvec, lo, hi, alpha):
    """J per box from the numpy oracle (with its rounding margins)."""
    mode, row = objective_weights(net, C, dvec, lo, hi)
    g_lo, g_hi = slr.propagate(net, C, dvec, lo, hi, alpha=alpha)
    return np.where(mode == 1, -g_lo.min(axis=1), g_hi[np.arange(g_hi.shape[0]), row])


def adam_step(a, g, m, v, t, lr, betas, eps):
    """One projected Adam step (Kingma and Ba, Algorithm 1) on ``a`` in place.

    First and second moment estimates with bias correction 1 - beta^t (t counts from 1),
    step lr * m_hat / (sqrt(v_hat) + eps) against the gradient, then projection onto [0, 1].
    Returns the new moments.
    """
    m = betas[0] * m + (1 - betas[0]) * g
    v = betas[1] * v + (1 - betas[1]) * g * g
    mh = m / (1 - betas[0] ** t)
    vh = v / (1 - betas[1] ** t)
    a -= lr * mh / (vh.sqrt() + eps)
    a.clamp_(0.0, 1.0)
    return m, v


def optimize(net, C, dvec, lo, hi, steps=20, lr=0.1, betas=(0.9, 0.999), eps=1e-8):
    """Projected Adam from alpha = lam; returns (best alpha, best J) per box."""
    torch = _torch()
    mode, row = objective_weights(net, C, dvec, lo, hi)
    a = torch.tensor(plain_lambda(net, C, dvec, lo, hi), requires_grad=True)
    m = torch.zeros_like(a)
    v = torch.zeros_like(a)
    best_a = a.detach().clone()
    best_j = torch.full((a.shape[0],), math.inf, dtype=torch.float64)
    for t in range(1, steps + 1):
        g_lo, g_hi = forward_torch(net, C, dvec, lo, hi, a)
        J = objective_torch(g_lo, g_hi, mode, row)
        better = J.detach() < best_j
        best_j = torch.where(better, J.detach(), best_j)
        best_a[better] = a.detach()[better]
        a.grad = None
        J.sum().backward()
        with torch.no_grad():
            m, v = adam_step(a, a.grad, m, v, t, lr, betas, eps)
    g_lo, g_hi = forward_torch(net, C, dvec, lo, hi, a)
    J = objective_torch(g_lo, g_hi, mode, row).detach()
    better = J < best_j
    best_j = torch.where(better, J, best_j)
    best_a[better] = a.detach()[better]
    return best_a.numpy(), best_j.numpy()
