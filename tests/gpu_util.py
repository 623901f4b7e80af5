"""Helpers of the GPU tests: torch device buffers in the library's column-major
layout (N x nrhs, leading dimension ld) and calls through the C ABI."""
from __future__ import annotations

import numpy as np
import torch

from paper_2105_02995_amd import fio as F

CT = {F.FIO_C64: torch.complex64, F.FIO_C128: torch.complex128}


def to_dev(a: np.ndarray, dtype=F.FIO_C128, ld: int | None = None) -> torch.Tensor:
    """(N, B) host array -> device tensor of shape (B, ld) (column-major N x B)."""
    a = a.reshape(a.shape[0], -1)
    N, B = a.shape
    ld = ld or N
    t = torch.zeros((B, ld), dtype=CT[dtype])
    t[:, :N] = torch.from_numpy(np.ascontiguousarray(a.T)).to(CT[dtype])
    return t.cuda()


def from_dev(t: torch.Tensor, N: int) -> np.ndarray:
    torch.cuda.synchronize()
    return t[:, :N].cpu().numpy().T.astype(np.complex128)


def empty(N: int, B: int, dtype=F.FIO_C128, ld: int | None = None) -> torch.Tensor:
    return torch.zeros((B, ld or N), dtype=CT[dtype], device="cuda")


def stream():
    return torch.cuda.current_stream().cuda_stream


def apply(plan, op, dtype, x: np.ndarray, ld=None):
    N = x.shape[0]
    X = to_dev(x, dtype, ld)
    Y = empty(N, X.shape[0], dtype, ld)
    F.fio_apply(plan, op, dtype, X, Y, X.shape[0], X.shape[1], stream())
    return from_dev(Y, N)


def inverse(plan, dtype, u: np.ndarray, ld=None):
    N = u.shape[0]
    U = to_dev(u, dtype, ld)
    Y = empty(N, U.shape[0], dtype, ld)
    F.fio_inverse_apply(plan, dtype, U, Y, U.shape[0], U.shape[1], stream())
    return from_dev(Y, N)


def solve(plan, mode, dtype, u: np.ndarray, tol=0.0, maxit=0, precondition=1, ld=None, spatial=0, restart=0):
    N = u.shape[0]
    U = to_dev(u, F.FIO_C128, ld)
    Y = empty(N, U.shape[0], F.FIO_C128, ld)
    info = F.fio_solve(plan, mode, dtype, U, Y, U.shape[0], U.shape[1], tol=tol, maxit=maxit,
                       precondition=precondition, stream=stream(), spatial=spatial, restart=restart)
    return from_dev(Y, N), info
