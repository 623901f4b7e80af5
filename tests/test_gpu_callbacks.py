"""Caller-defined FIOs on the GPU (FIO_PHASE_CALLBACK, section 1 eqs. eq3/eq6): device
plans built from the C callbacks of the paper's Examples 1, 2 and 3
(tests/native/fio_callbacks.c), solved through the C ABI and compared with the oracle;
and the plan's error estimates (e_a, e_s, cond) and each solve's est_rel_err against
the errors the oracle measures."""
import sys

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex
from paper_2105_02995_amd import fio as F

from . import callbacks as CB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402

MIX = ((0.2, -0.2), (0.5, 0.2), (0.8, 0.0))
_cache = {}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def case(example, d, n, eps, s2=0.1):
    key = (example, d, n, eps, s2)
    if key not in _cache:
        log("building callback plan %s" % (key,))
        plan = F.fio_build(CB.problem(example, d, n, eps, device=0, sigma2=s2, centres=MIX))
        if example == "ex2":
            op = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=MIX, sigma2=s2)
        else:
            op = O.OracleProblem(d, n, "1d_ex1" if example == "ex1" else "2d_radon", 16.0)
        _cache[key] = (plan, op, O.dense_K(op))
    return _cache[key]


@pytest.mark.parametrize("example,d,n,eps,mode,dtype,kw", [
    ("ex1", 1, 4096, 1e-6, F.FIO_SOLVE_REFINE, F.FIO_C64, {"maxit": 1}),
    ("ex1", 1, 4096, 1e-6, F.FIO_SOLVE_DIRECT, F.FIO_C128, {}),
    ("ex2", 1, 1024, 1e-5, F.FIO_SOLVE_PCG, F.FIO_C128, {"tol": 1e-10, "maxit": 60}),
    ("ex2", 1, 1024, 1e-5, F.FIO_SOLVE_GMRES, F.FIO_C128, {"tol": 1e-10, "maxit": 60}),
    ("radon", 2, 64, 1e-4, F.FIO_SOLVE_REFINE, F.FIO_C64, {"maxit": 1}),
    ("radon", 2, 64, 1e-4, F.FIO_SOLVE_PCG, F.FIO_C128, {"tol": 1e-8, "maxit": 60}),
])
def test_callback_fio_solves_against_the_oracle(example, d, n, eps, mode, dtype, kw):
    plan, op, K = case(example, d, n, eps)
    N = n ** d
    fh = gaussian_complex((N, 8), 1500 + mode)
    u = K @ fh
    ref = O.solve_dense(op, u, K)
    x, (its, rr) = G.solve(plan, mode, dtype, u, **kw)
    err = O.rel_err(x, ref).max()
    log("%s n=%d mode %d dtype %d: %d its, error %.2e" % (example, n, mode, dtype, its, err))
    assert err < 10 * eps


def test_callback_plan_equals_builtin_phase_plan():
    """The same FIO built from callbacks and from the built-in phase: applies agree to
    within the butterfly tolerance (both approximate the same K)."""
    n, eps = 4096, 1e-6
    plan, op, K = case("ex1", 1, n, eps)
    ref_plan = F.fio_build(F.make_problem(1, n, "1d_ex1", eps=eps, device=0))
    x = gaussian_complex((n, 4), 31)
    a = G.apply(plan, F.FIO_OP_K, F.FIO_C128, x)
    b = G.apply(ref_plan, F.FIO_OP_K, F.FIO_C128, x)
    assert O.rel_err(a, K @ x).max() < eps
    assert O.rel_err(a, b).max() < eps
    ref_plan.close()


@pytest.mark.parametrize("example,d,n,eps", [("ex1", 1, 1024, 1e-6), ("ex2", 1, 1024, 1e-5),
                                             ("radon", 2, 32, 1e-4)])
def test_plan_error_estimates(example, d, n, eps):
    """e_a, e_s and cond(Kd) of fio_plan_stats against the dense truth: e_a of the
    plan against ||Kd x - K x|| / ||K x|| on Gaussian vectors, cond against
    cond(K), and e_s against the spectral radius of I - Gd Kd^* Kd, formed densely
    from GPU applies to the identity."""
    plan, op, K = case(example, d, n, eps)
    st = F.fio_plan_stats(plan)
    N = n ** d
    x = gaussian_complex((N, 8), 32)
    ea = O.rel_err(G.apply(plan, F.FIO_OP_K, F.FIO_C128, x), K @ x).max()
    cond = np.linalg.cond(K)
    I = np.eye(N, dtype=np.complex128)
    KdI = G.apply(plan, F.FIO_OP_K, F.FIO_C128, I)            # Kd (dense)
    GdS = G.solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C128, KdI)[0]  # Gd Kd^* Kd
    rho = np.abs(np.linalg.eigvals(I - GdS)).max()
    log("%s: e_a est %.2e vs %.2e; e_s est %.2e vs %.2e; cond est %.3f vs %.3f" % (
        example, st["e_a_est"], ea, st["e_s_est"], rho, st["cond_est"], cond))
    assert 0.1 * ea <= st["e_a_est"] <= 10 * ea
    assert 0.3 * rho <= st["e_s_est"] <= 1.5 * rho
    assert 0.8 * cond <= st["cond_est"] <= 1.25 * cond


@pytest.mark.parametrize("mode,dtype,kw", [
    (F.FIO_SOLVE_DIRECT, F.FIO_C64, {}), (F.FIO_SOLVE_DIRECT, F.FIO_C128, {}),
    (F.FIO_SOLVE_REFINE, F.FIO_C64, {"maxit": 1}), (F.FIO_SOLVE_REFINE, F.FIO_C64, {"maxit": 2}),
    (F.FIO_SOLVE_PCG, F.FIO_C128, {"tol": 1e-8, "maxit": 60}),
    (F.FIO_SOLVE_GMRES, F.FIO_C128, {"tol": 1e-9, "maxit": 60})])
@pytest.mark.parametrize("example,d,n,eps", [("ex1", 1, 4096, 1e-6), ("radon", 2, 64, 1e-4)])
def test_est_rel_err_bounds_the_oracle_error(example, d, n, eps, mode, dtype, kw):
    """fio_solve_info.est_rel_err against the error the oracle measures: it must not
    understate it (within a factor 3).  Where the estimate rests on the solve's own
    residual (REFINE, PCG, GMRES) it must stay within 10 eps when the solve does; the
    direct solve's estimate is the plan's worst-direction e_s (section 6), which a
    Gaussian right-hand side does not reach, so there it must be within 30x of the
    error."""
    plan, op, K = case(example, d, n, eps)
    N = n ** d
    fh = gaussian_complex((N, 6), 1600 + mode)
    u = K @ fh
    ref = O.solve_dense(op, u, K)
    U = G.to_dev(u)
    X = G.empty(N, 6)
    its, rr, est = F.fio_solve(plan, mode, dtype, U, X, 6, N, stream=G.stream(), with_estimate=True, **kw)
    err = O.rel_err(G.from_dev(X, N), ref).max()
    log("%s mode %d dtype %d: error %.2e, estimate %.2e" % (example, mode, dtype, err, est))
    assert err <= 3 * est
    if mode == F.FIO_SOLVE_DIRECT:
        assert est <= max(10 * eps, 30 * err)
    else:
        assert est <= 10 * eps
