"""The algorithmic work figures the bench line's roofline is computed from, pinned on the CPU.

The bound kernel's flops per box are the contractions of the center/radius propagation (section
2.2, Eq. 1 keeps one radius column): they are counted here by walking a network's layers and
tallying the multiply-adds of the plain matrix products, and compared with the closed form in
bench.py and with the hand count for the 5-50x6-5 network.
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402


def _walked_flops(sizes, rows):
    """2 flops per multiply-add: the first layer's d center multiply-adds and d slope products
    per neuron (3 d flops), then per hidden-to-hidden layer W times the d + 1 center columns and
    |W| times the radius column, then the folded property rows the same way."""
    d = sizes[0]
    macs = 0
    flops = 3 * d * sizes[1]
    hidden = list(sizes[1:-1])
    layers = list(zip(hidden[:-1], hidden[1:])) + [(hidden[-1], rows)]
    for n_in, n_out in layers:
        for _ in range(n_out):
            for _ in range(n_in):
                macs += (d + 1) + 1
    return flops + 2 * macs


def test_bound_flops_per_box():
    acas = (5, 50, 50, 50, 50, 50, 50, 5)
    assert bench.flops_per_box(acas, 1) == 176450
    assert bench.flops_per_box(acas, 1) == _walked_flops(acas, 1)
    for sizes, rows in (((2, 16, 16, 1), 1), ((22, 64, 64, 64, 3), 2), ((10, 128, 96, 4), 3)):
        assert bench.flops_per_box(sizes, rows) == _walked_flops(sizes, rows)


def test_alpha_flops_per_box_step():
    # forward: W C and |W| R, d + 1 columns each, per hidden layer and the folded rows; the
    # adjoint the same again; the first layer's centers 2 d n1
    acas = (5, 50, 50, 50, 50, 50, 50, 5)
    fwd = 5 * (4 * 50 * 50 * 6) + 4 * 50 * 1 * 6
    assert bench.alpha_flops_per_box_step(acas, 1) == 2 * fwd + 2 * 5 * 50 == 602900


def test_bound_bytes_per_box():
    # two float32 corners of d coordinates in, one class byte out
    assert bench.bytes_per_box(5) == 41
    assert bench.bytes_per_box(22) == 177
