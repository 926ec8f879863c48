"""Shared helpers of the GPU tests (import only from tests marked gpu)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_20441_amd as p
    return p


def matrix_rel(C, Cref):
    return float(np.max(np.abs(C - Cref)) / np.max(np.abs(Cref)))


def announce(*a):
    print("[case]", *a, flush=True)
