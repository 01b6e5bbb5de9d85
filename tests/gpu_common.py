"""Shared helpers of the GPU parity tests."""
import os

import numpy as np
import pytest

from paper_2606_21125_amd.binding import LIB_PATH


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    if not os.path.exists(LIB_PATH):
        pytest.fail("libdcdft.so missing on a GPU host: build it first")


def l1_over_ne(a, b, dv, ne):
    return dv * float(np.abs(np.asarray(a) - np.asarray(b)).sum()) / ne
