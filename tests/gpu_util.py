"""Helpers shared by the GPU tests (run through the C ABI)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

TOL_C128 = 1e-12   # max |delta amplitude| against the complex128 oracle


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    return torch


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def max_abs_diff(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if len(a) else 0.0
