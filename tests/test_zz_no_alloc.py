"""fio_inverse_apply_noalloc (the entry point for callers that cannot allocate) against
fio_inverse_apply: two calls in a row, the second with fewer right-hand sides, the
same kernels and launches, so the results must agree bit for bit; both against the
oracle's solve; and the scratch limit is refused with FIO_ERR_ARG."""
import sys

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex
from paper_2105_02995_amd import fio as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("d,n,phase,eps,dtype,widths", [
    (1, 4096, "1d_ex1", 1e-6, F.FIO_C64, (64, 5)),
    (1, 4096, "1d_ex1", 1e-6, F.FIO_C128, (24, 1)),
    (2, 64, "2d_radon", 1e-4, F.FIO_C64, (32, 17)),
])
def test_noalloc_matches_inverse_apply(d, n, phase, eps, dtype, widths):
    log("no-alloc: building %s n=%d" % (phase, n))
    plan = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
    op = O.OracleProblem(d, n, phase, 16.0)
    K = O.dense_K(op)
    N = n ** d
    try:
        for call, B in enumerate(widths):
            fh = gaussian_complex((N, B), 1700 + call)
            u = K @ fh
            ref = O.solve_dense(op, u, K)
            U = G.to_dev(u, dtype)
            Y0 = G.empty(N, B, dtype)
            Y1 = G.empty(N, B, dtype)
            Y1.fill_(float("nan"))  # every entry must be written
            F.fio_inverse_apply(plan, dtype, U, Y0, B, N, G.stream())
            F.fio_inverse_apply_noalloc(plan, dtype, U, Y1, B, N, G.stream())
            torch.cuda.synchronize()
            a, b = G.from_dev(Y0, N), G.from_dev(Y1, N)
            log("no-alloc call %d (%d RHS, dtype %d): max |diff| %.3e, error vs oracle %.2e" % (
                call, B, dtype, np.abs(a - b).max(), O.rel_err(b, ref).max()))
            assert np.array_equal(a, b)
            assert O.rel_err(b, ref).max() < 10 * eps
    finally:
        plan.close()


def test_noalloc_refuses_more_than_its_scratch():
    n = 65536
    plan = F.fio_build(F.make_problem(1, n, "1d_ex1", eps=1e-6, device=0))
    try:
        B = 128  # about 5 MB per complex64 column: more than 256 MiB
        U = torch.zeros((B, n), dtype=torch.complex64, device="cuda")
        Y = torch.zeros_like(U)
        with pytest.raises(F.FioError) as e:
            F.fio_inverse_apply_noalloc(plan, F.FIO_C64, U, Y, B, n, G.stream())
        assert e.value.status == 1 and "scratch" in str(e.value)
        # within the limit the same plan works, and writes every entry
        Y.fill_(float("nan"))
        F.fio_inverse_apply_noalloc(plan, F.FIO_C64, U[:8], Y[:8], 8, n, G.stream())
        torch.cuda.synchronize()
        assert torch.count_nonzero(Y[:8]).item() == 0  # Gd Kd^* 0 = 0
    finally:
        plan.close()
