"""fio_plan_trim: a plan that keeps only the images the refined complex64 solve uses
(Kd^* and Gd in complex64, Kd in complex128) gives the same solves bit for bit with
about half the factor memory, and refuses calls that need a released image."""
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


@pytest.mark.parametrize("d,n,phase,eps", [(1, 4096, "1d_ex1", 1e-6), (2, 64, "2d_radon", 1e-4)])
def test_trimmed_plan_solves_the_same_with_half_the_memory(d, n, phase, eps):
    plan = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
    try:
        op = O.OracleProblem(d, n, phase, 16.0)
        K = O.dense_K(op)
        fh = gaussian_complex((n ** d, 24), 1900)
        u = K @ fh
        before, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=1)
        direct, _ = G.solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C64, u)
        b0 = F.fio_plan_stats(plan)["device_bytes"]
        F.fio_plan_trim(plan, F.FIO_KEEP_REFINE_C64)
        b1 = F.fio_plan_stats(plan)["device_bytes"]
        log("trim %s n=%d: device bytes %.3e -> %.3e" % (phase, n, b0, b1))
        assert b1 < 0.6 * b0
        after, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=1)
        assert np.array_equal(after, before)
        assert np.array_equal(G.solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C64, u)[0], direct)
        assert O.rel_err(after, fh).max() < 10 * eps
        # the kept adjoint chain still applies; the released images are refused
        x = gaussian_complex((n ** d, 3), 1901)
        assert O.rel_err(G.apply(plan, F.FIO_OP_KH, F.FIO_C64, x), K.conj().T @ x).max() < 10 * eps
        for call in (lambda: G.apply(plan, F.FIO_OP_K, F.FIO_C64, x),
                     lambda: G.apply(plan, F.FIO_OP_KH, F.FIO_C128, x),
                     lambda: G.solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C128, u),
                     lambda: G.solve(plan, F.FIO_SOLVE_PCG, F.FIO_C64, u, tol=1e-8, maxit=20)):
            with pytest.raises(F.FioError) as e:
                call()
            assert e.value.status == 6
        # tuning skips what is gone; the multi-instance solve uses only kept images
        F.fio_autotune(plan, F.FIO_C64, 24, 2, G.stream())
        again, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=1)
        assert O.rel_err(again, fh).max() < 10 * eps
        U = G.to_dev(u)
        X = G.empty(n ** d, 24)
        F.fio_solve_multi([plan], F.FIO_SOLVE_REFINE, F.FIO_C64, [U], [X], [24], [n ** d], maxit=1,
                          stream=G.stream())
        assert O.rel_err(G.from_dev(X, n ** d), fh).max() < 10 * eps
    finally:
        plan.close()
