"""Edge cases of the GPU path: single right-hand sides with a padded leading
dimension in every solve mode, the smallest grids, batch widths around the
matrix-core thresholds, workspace growth between calls, empty batches and argument
errors, all against the oracle."""
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

_cache = {}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def setup(d, n, eps):
    key = (d, n, eps)
    if key not in _cache:
        phase = "1d_ex1" if d == 1 else "2d_radon"
        log("building plan %s" % (key,))
        plan = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
        op = O.OracleProblem(d, n, phase, 16.0)
        _cache[key] = (plan, op, O.dense_K(op))
    return _cache[key]


@pytest.mark.parametrize("mode,dtype,kw", [
    (F.FIO_SOLVE_DIRECT, F.FIO_C64, {}), (F.FIO_SOLVE_DIRECT, F.FIO_C128, {}),
    (F.FIO_SOLVE_REFINE, F.FIO_C64, {"maxit": 2}),
    (F.FIO_SOLVE_PCG, F.FIO_C128, {"tol": 1e-8, "maxit": 50}),
    (F.FIO_SOLVE_GMRES, F.FIO_C128, {"tol": 1e-10, "maxit": 30})])
def test_single_rhs_padded_ld_every_mode(mode, dtype, kw):
    n, eps = 1024, 1e-6
    plan, op, K = setup(1, n, eps)
    fh = gaussian_complex((n, 1), 800 + mode)
    u = K @ fh
    x, _ = G.solve(plan, mode, dtype, u, ld=n + 7, **kw)
    err = O.rel_err(x, fh).max()
    log("mode %d dtype %d, 1 RHS, ld=N+7: error %.2e" % (mode, dtype, err))
    assert err < 10 * eps


@pytest.mark.parametrize("d,n,eps", [(1, 16, 1e-6), (1, 32, 1e-6), (2, 16, 1e-4)])
def test_smallest_grids(d, n, eps):
    plan, op, K = setup(d, n, eps)
    fh = gaussian_complex((n ** d, 3), 801)
    u = K @ fh
    y = G.apply(plan, F.FIO_OP_K, F.FIO_C128, fh)
    assert O.rel_err(y, u).max() < eps
    x, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C128, u, maxit=1)
    assert O.rel_err(x, fh).max() < 10 * eps


@pytest.mark.parametrize("B", [1, 7, 15, 16, 17, 31, 33, 63, 65, 129])
def test_batch_widths_around_thresholds(B):
    """Widths below 16 take the vector kernels, 16 and above the matrix-core and
    fused kernels with ragged column tiles; both must agree with the oracle."""
    n, eps = 1024, 1e-6
    plan, op, K = setup(1, n, eps)
    x = gaussian_complex((n, B), 900 + B)
    for dtype, tol in ((F.FIO_C64, 2e-6), (F.FIO_C128, 1e-6)):
        y = G.apply(plan, F.FIO_OP_K, dtype, x)
        yh = G.apply(plan, F.FIO_OP_KH, dtype, x)
        assert O.rel_err(y, K @ x).max() < tol, (B, dtype)
        assert O.rel_err(yh, K.conj().T @ x).max() < tol, (B, dtype)


def test_workspace_grows_and_shrinks_between_calls():
    n, eps = 1024, 1e-6
    plan, op, K = setup(1, n, eps)
    for B in (3, 200, 5, 64, 1):
        fh = gaussian_complex((n, B), 1000 + B)
        x, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, K @ fh, maxit=1)
        assert O.rel_err(x, fh).max() < 10 * eps, B


def test_empty_batches_are_noops():
    n = 1024
    plan, op, K = setup(1, n, 1e-6)
    X = torch.zeros((1, n), dtype=torch.complex128, device="cuda")
    F.fio_apply(plan, F.FIO_OP_K, F.FIO_C64, X, X, 0, n, G.stream())
    F.fio_solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C64, X, X, 0, n, maxit=3, stream=G.stream(), want_info=False)
    F.fio_inverse_dft(plan, X, X, 0, n, G.stream())
    F.fio_stage_pair_apply(plan, F.FIO_OP_K, 1, F.FIO_C64, X, X, 0, G.stream())
    torch.cuda.synchronize()
    assert torch.count_nonzero(X).item() == 0


def test_argument_errors():
    n = 1024
    plan, op, K = setup(1, n, 1e-6)
    X = torch.zeros((2, n), dtype=torch.complex128, device="cuda")
    bad = [lambda: F.fio_solve(plan, 7, F.FIO_C64, X, X, 2, n, stream=G.stream()),
           lambda: F.fio_solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C64, X, X, 2, n, maxit=3, restart=-1, stream=G.stream()),
           lambda: F.fio_solve(plan, F.FIO_SOLVE_PCG, F.FIO_C64, X, X, 2, n, maxit=-1, stream=G.stream()),
           lambda: F.fio_apply(plan, F.FIO_OP_K, F.FIO_C64, X, X, 2, n - 1, G.stream()),
           lambda: F.fio_stage_pair_apply(plan, F.FIO_OP_K, 10_000, F.FIO_C64, X, X, 2, G.stream())]
    for call in bad:
        with pytest.raises(F.FioError) as e:
            call()
        assert e.value.status == 1  # FIO_ERR_ARG


@pytest.mark.parametrize("mode,kw", [
    (F.FIO_SOLVE_PCG, {"tol": 1e-8, "maxit": 50}),
    (F.FIO_SOLVE_REFINE, {"maxit": 2}),
    (F.FIO_SOLVE_GMRES, {"tol": 1e-10, "maxit": 30})])
def test_zero_column_among_gaussian_ones(mode, kw):
    """A zero right-hand side has the exact solution 0: every mode must return 0
    for it (no 0/0 in the per-column scalars) and solve the other columns."""
    n, eps = 1024, 1e-6
    plan, op, K = setup(1, n, eps)
    fh = gaussian_complex((n, 5), 806)
    fh[:, 2] = 0
    u = K @ fh
    x, (its, rr) = G.solve(plan, mode, F.FIO_C128, u, **kw)
    log("mode %d with a zero column: its %d, rel resid %.2e" % (mode, its, rr))
    assert np.isfinite(x).all()
    assert np.abs(x[:, 2]).max() == 0.0
    assert np.isfinite(rr)
    keep = [0, 1, 3, 4]
    assert O.rel_err(x[:, keep], O.solve_dense(op, u[:, keep], K)).max() < 10 * eps


def test_captured_plan_refuses_a_wider_call():
    """A graph captured from a solve keeps the plan's workspace addresses: after
    the capture a wider call must fail (FIO_ERR_ARG) instead of moving the
    workspace, and replays keep matching the eager result."""
    n, eps = 256, 1e-6
    plan = F.fio_build(F.make_problem(1, n, "1d_ex1", eps=eps, device=0))
    try:
        s = torch.cuda.Stream()
        U = torch.from_numpy(np.ascontiguousarray(gaussian_complex((n, 16), 807).T)).cuda()
        X = torch.zeros_like(U)
        with torch.cuda.stream(s):
            F.fio_solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, U, X, 16, n, maxit=1, stream=s, want_info=False)
        s.synchronize()
        eager = X.cpu().clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            F.fio_solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, U, X, 16, n, maxit=1, stream=s, want_info=False)
        U2 = torch.zeros((32, n), dtype=torch.complex128, device="cuda")
        X2 = torch.zeros_like(U2)
        with pytest.raises(F.FioError) as e:
            F.fio_solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C64, U2, X2, 32, n, want_info=False)
        assert e.value.status == 1
        for _ in range(3):
            X.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(X.cpu(), eager)
        del g
    finally:
        plan.close()
