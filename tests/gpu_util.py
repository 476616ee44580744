"""Shared helpers of the GPU parity tests: device transfer, the FP32 error
reference (the FP64 oracle evaluated on the FP32-rounded inputs), tolerances."""
import sys

import numpy as np
import pytest

TOL = {np.complex128: 1e-12, np.complex64: 2e-6}


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1008_1366_amd as ic
    ic.lib()  # raises if the library is missing: no silent fallback
    return ic


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to("cuda:0")


def rounded(a, dtype):
    """Inputs as the kernel sees them, upcast to FP64 for the oracle."""
    return np.asarray(a.astype(dtype), dtype=np.complex128)


def rel(x, ref):
    x = np.asarray(x, np.complex128).ravel()
    ref = np.asarray(ref, np.complex128).ravel()
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / d) if d > 0 else float(np.linalg.norm(x))
