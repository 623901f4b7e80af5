"""GMRES on Kd fhat = u with the right preconditioner Gd Kd^* (the alternative to CG
on the normal equations; batched, one Krylov space per column), against the
oracle's exact solve."""
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

_cases = {}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def case(d, n, eps, B):
    key = (d, n, eps, B)
    if key not in _cases:
        phase = "1d_ex1" if d == 1 else "2d_radon"
        log("building plan %s" % (key,))
        plan = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
        op = O.OracleProblem(d, n, phase, 16.0)
        K = O.dense_K(op)
        fh = gaussian_complex((n ** d, B), 600 + n + B)
        u = K @ fh
        _cases[key] = (plan, K, fh, u)
    return _cases[key]


@pytest.mark.parametrize("d,n,eps", [(1, 4096, 1e-6), (2, 64, 1e-4)])
def test_gmres_fp64_converges_in_few_iterations(d, n, eps):
    plan, K, fh, u = case(d, n, eps, 8)
    x, (its, rr) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C128, u, tol=1e-10, maxit=30)
    err = O.rel_err(x, fh).max()
    log("GMRES c128 d=%d n=%d: %d iterations, residual %.2e, error %.2e" % (d, n, its, rr, err))
    assert rr <= 1e-10
    assert its <= 8
    assert err < 10 * eps


@pytest.mark.parametrize("d,n,eps", [(1, 4096, 1e-6), (2, 64, 1e-4)])
def test_gmres_complex64_to_eps(d, n, eps):
    plan, K, fh, u = case(d, n, eps, 8)
    x, (its, rr) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C64, u, tol=eps, maxit=30)
    err = O.rel_err(x, fh).max()
    log("GMRES c64 d=%d n=%d: %d iterations, residual %.2e, error %.2e" % (d, n, its, rr, err))
    assert rr <= eps
    assert err < 10 * eps


def test_gmres_restarted_cycles_reach_the_same_solution():
    plan, K, fh, u = case(1, 4096, 1e-6, 8)
    a, (its_a, _) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C128, u, tol=1e-11, maxit=30)
    b, (its_b, rr_b) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C128, u, tol=1e-11, maxit=30, restart=1)
    log("GMRES restart 1: %d iterations (unrestarted %d), residual %.2e" % (its_b, its_a, rr_b))
    assert rr_b <= 1e-11
    assert its_b >= 2  # several one-step cycles, each from the true residual
    assert O.rel_err(b, a).max() < 1e-9


def test_gmres_residual_estimate_matches_true_residual():
    """The least-squares residual GMRES reports equals ||u - Kd x|| / ||u||, which is
    within e_a of the oracle's ||u - K x|| / ||u||."""
    plan, K, fh, u = case(1, 4096, 1e-6, 8)
    for pre, its in ((0, 6), (1, 2)):
        x, (n_it, rr) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C128, u, tol=0.0, maxit=its, precondition=pre)
        true = (np.linalg.norm(u - K @ x, axis=0) / np.linalg.norm(u, axis=0)).max()
        log("GMRES precondition=%d, %d iterations: estimate %.3e, oracle residual %.3e" % (pre, n_it, rr, true))
        assert n_it == its
        assert abs(rr - true) <= 1e-6 + 1e-3 * true


def test_gmres_spatial_output():
    plan, K, fh, u = case(1, 4096, 1e-6, 8)
    f, (its, rr) = G.solve(plan, F.FIO_SOLVE_GMRES, F.FIO_C128, u, tol=1e-10, maxit=30, spatial=1)
    assert O.rel_err(f, O.idft(fh, 1, 4096)).max() < 1e-5
