"""Helpers for GPU tests: skip cleanly without a device, load the library."""
import os

import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_17711_amd._lib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("GPU present but libtenso.so is not built")
