"""Helpers shared by the GPU tests."""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def csr_op(A):
    return solver.csr(dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val))


def stencil_coefs(A, dim, n):
    """Coefficients of an interior row of a constant-coefficient 5/7-point CSR matrix."""
    if dim == 2:
        row = n * (n // 2) + n // 2
    else:
        row = n * n * (n // 2) + n * (n // 2) + n // 2
    lo, hi = A.row_ptr[row], A.row_ptr[row + 1]
    return list(A.val[lo:hi])


def say(msg):
    print(msg, flush=True)


def same(a, b):
    """Bitwise equality of float64 arrays (NaN-aware, sign of zero included)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))
