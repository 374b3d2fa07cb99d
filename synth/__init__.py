"""Seeded synthetic verification instances: ReLU networks, input boxes, unsafe properties.

This module only draws numbers. It holds none of the counting method's arithmetic, so both
the FP64 oracle and the GPU engine read their inputs from here without sharing any code of
the method itself.

A network is a list of ``(W, b)`` pairs with ``W`` of shape ``[out, in]`` (row-major) and
``b`` of shape ``[out]``, both float32.  The float32 arrays *are* the network: every consumer
promotes them exactly.  Weights are He-normal, ``N(0, 2/fan_in)``, biases ``U(-0.1, 0.1)``,
drawn per affine layer (weights first, then biases) from ``numpy.random.default_rng(seed)``.

A property is ``(C, d)`` with ``C`` of shape ``[rows, n_out]``: the output ``y`` is unsafe
when every row of ``C y + d`` is strictly positive (the negated postcondition of the
verification tuple <N, P, Q>, paper §2.1 and §3).

A domain is a pair of float64 vectors whose values are exactly representable in float32.

Workloads (the input recipe; the paper's own networks are not available, these are stand-ins
of the same shapes):

* ``tiny2d``   2 -> 16 -> 16 -> 1 on [-1,1]^2, unsafe iff y > 0, max depth 16.
* ``acas``     5 -> 50 x6 -> 5 on [0,1]^5, unsafe iff y0 - y1 > 0 (shape of the ACAS Xu
               networks of §4), 65536 boxes per launch, leaf budget 2^20.
* ``nav22``    22 -> 64 x3 -> 3 on [0,1]^22, unsafe iff y2 is the strict argmax (a scaled-up
               stand-in for the 13-input mapless-navigation model of §4).
* ``batch``    256 instances of 5..10 inputs, 3..6 hidden layers of width 32..128,
               2..5 outputs and a random linear property each.
* ``wide20``   20 -> 256 x4 -> 2 on [0,1]^20, unsafe iff y0 - y1 > 0.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

Net = List[Tuple[np.ndarray, np.ndarray]]


class ActNet(list):
    """A network (list of (W, b) layers) whose hidden activation is ``act`` ('tanh' or
    'sigmoid') instead of ReLU."""

    def __init__(self, layers, act: str):
        super().__init__(layers)
        self.act = act


def with_activation(net, act: str):
    """The same layers with another hidden activation."""
    return ActNet(list(net), act)


def tanh2d(seed: int, act: str = "tanh") -> "Instance":
    """tiny2d's shape with a smooth activation: 2-16-16-1, [-1, 1]^2, y > 0, depth 16."""
    base = tiny2d(seed)
    return dataclasses.replace(base, name=f"{act}2d", net=with_activation(base.net, act))


def smooth5(seed: int, act: str = "tanh", max_depth: int = 30,
            max_leaves: int = 1 << 16) -> "Instance":
    """A 5-input 3x32 network with a smooth activation, [0, 1]^5, y0 - y1 > 0."""
    net = with_activation(make_net([5, 32, 32, 32, 5], seed), act)
    lo, hi = _box(0.0, 1.0, 5)
    C = np.array([[1.0, -1.0, 0.0, 0.0, 0.0]], np.float32)
    return Instance(f"{act}5", net, lo, hi, C, np.zeros(1, np.float32), max_depth, max_leaves)


@dataclasses.dataclass
class Instance:
    """One verification instance: network, input box, property and search limits."""

    name: str
    net: Net
    lo: np.ndarray          # float64 [d], exactly representable in float32
    hi: np.ndarray
    C: np.ndarray           # float32 [rows, n_out]
    dvec: np.ndarray        # float32 [rows]
    max_depth: int
    max_leaves: int

    @property
    def sizes(self) -> List[int]:
        return [self.net[0][0].shape[1]] + [W.shape[0] for W, _ in self.net]


def make_net(sizes, seed: int, rng: np.random.Generator | None = None) -> Net:
    """He-normal weights N(0, 2/fan_in) and biases U(-0.1, 0.1), stored as float32."""
    if rng is None:
        rng = np.random.default_rng(seed)
    net = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(fan_out, fan_in)).astype(np.float32)
        b = rng.uniform(-0.1, 0.1, size=fan_out).astype(np.float32)
        net.append((W, b))
    return net


def _box(lo, hi, d):
    return (np.full(d, lo, dtype=np.float64), np.full(d, hi, dtype=np.float64))


def tiny2d(seed: int) -> Instance:
    net = make_net([2, 16, 16, 1], seed)
    lo, hi = _box(-1.0, 1.0, 2)
    return Instance("tiny2d", net, lo, hi, np.array([[1.0]], np.float32),
                    np.zeros(1, np.float32), max_depth=16, max_leaves=1 << 20)


def acas(seed: int, max_depth: int = 40, max_leaves: int = 1 << 20) -> Instance:
    net = make_net([5, 50, 50, 50, 50, 50, 50, 5], seed)
    lo, hi = _box(0.0, 1.0, 5)
    C = np.array([[1.0, -1.0, 0.0, 0.0, 0.0]], np.float32)
    return Instance("acas", net, lo, hi, C, np.zeros(1, np.float32), max_depth, max_leaves)


def nav22(seed: int, max_depth: int = 48, max_leaves: int = 1 << 16) -> Instance:
    net = make_net([22, 64, 64, 64, 3], seed)
    lo, hi = _box(0.0, 1.0, 22)
    C = np.array([[-1.0, 0.0, 1.0], [0.0, -1.0, 1.0]], np.float32)
    return Instance("nav22", net, lo, hi, C, np.zeros(2, np.float32), max_depth, max_leaves)


def wide20(seed: int, max_depth: int = 40, max_leaves: int = 1 << 20) -> Instance:
    net = make_net([20, 256, 256, 256, 256, 2], seed)
    lo, hi = _box(0.0, 1.0, 20)
    C = np.array([[1.0, -1.0]], np.float32)
    return Instance("wide20", net, lo, hi, C, np.zeros(1, np.float32), max_depth, max_leaves)


def batch(seed: int, count: int = 256) -> List[Instance]:
    """Uneven instances; instance i draws everything from default_rng(seed * 1000 + i)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed * 1000 + i)
        d = int(rng.integers(5, 11))
        depth = int(rng.integers(3, 7))
        width = int(rng.choice([32, 64, 96, 128]))
        n_out = int(rng.integers(2, 6))
        sizes = [d] + [width] * depth + [n_out]
        net = make_net(sizes, 0, rng=rng)
        c = rng.normal(0.0, 1.0, size=(1, n_out)).astype(np.float32)
        lo, hi = _box(0.0, 1.0, d)
        out.append(Instance(f"batch{i}", net, lo, hi, c, np.zeros(1, np.float32),
                            max_depth=4 * d, max_leaves=1 << 16))
    return out


def random_boxes(lo, hi, n: int, seed: int, max_depth: int = 12):
    """Dyadic sub-boxes of [lo, hi]: each is reached by a random sequence of bisections.

    Returns float32 arrays ``(blo, bhi)`` of shape [n, d]; every coordinate is exact.
    """
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = lo.shape[0]
    blo = np.tile(lo, (n, 1))
    bhi = np.tile(hi, (n, 1))
    depths = rng.integers(0, max_depth + 1, size=n)
    for i in range(n):
        for _ in range(int(depths[i])):
            j = int(rng.integers(0, d))
            m = 0.5 * (blo[i, j] + bhi[i, j])
            if rng.integers(0, 2):
                blo[i, j] = m
            else:
                bhi[i, j] = m
    return blo.astype(np.float32), bhi.astype(np.float32)


def uniform_boxes(lo, hi, n: int, seed: int, scale: float = 0.25):
    """Arbitrary (non-dyadic) float32 boxes inside [lo, hi] with widths up to scale*(hi-lo)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    w = (hi - lo) * scale * rng.uniform(0.0, 1.0, size=(n, lo.shape[0]))
    a = lo + (hi - lo - w) * rng.uniform(0.0, 1.0, size=(n, lo.shape[0]))
    blo = a.astype(np.float32)
    bhi = np.maximum((a + w).astype(np.float32), blo)
    return blo, bhi


def save_instance(path: str, inst: Instance) -> None:
    """Plain .npz (no pickled objects) with W0.., b0.., lo, hi, C, d, limits."""
    arrays = {"lo": inst.lo, "hi": inst.hi, "C": inst.C, "d": inst.dvec,
              "limits": np.array([inst.max_depth, inst.max_leaves], np.int64)}
    for i, (W, b) in enumerate(inst.net):
        arrays[f"W{i}"] = W
        arrays[f"b{i}"] = b
    np.savez(path, **arrays)


def load_instance(path: str, name: str = "file") -> Instance:
    z = np.load(path, allow_pickle=False)
    net = []
    i = 0
    while f"W{i}" in z:
        net.append((z[f"W{i}"].astype(np.float32), z[f"b{i}"].astype(np.float32)))
        i += 1
    lim = z["limits"]
    return Instance(name, net, z["lo"], z["hi"], z["C"], z["d"], int(lim[0]), int(lim[1]))
