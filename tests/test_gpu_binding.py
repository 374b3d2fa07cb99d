"""The binding on the GPU: loading order of the HIP library and torch."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_before_torch_in_a_fresh_process():
    """Loading a network (the library's first HIP call) before any torch use must leave torch
    able to use the GPU: the binding loads torch's HIP runtime first."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import synth, paper_2312_05890_amd as E\n"
            "net = E.Net(synth.tiny2d(0).net)\n"
            "import torch\n"
            "x = torch.ones(4, device='cuda')\n"
            "print(float(x.sum()))\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("4.0")
