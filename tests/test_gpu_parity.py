"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (stated per the method's tolerance): relative 2-norm error per column
<= 10 eps for the factored applies and solves; the tight kernel checks compare
the GPU apply with a host product of the very same saved factors.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex, uniform_indices
from paper_2105_02995_amd import fio as F

from . import factor_file as FF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_plans = {}


def plan_for(n, phase="1d_ex1", eps=1e-6, d=1):
    key = (d, n, phase, eps)
    if key not in _plans:
        log("building plan d=%d n=%d phase=%s eps=%g" % (d, n, phase, eps))
        _plans[key] = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
    return _plans[key]


def oracle_case(n, B, seed, phase="1d_ex1"):
    p = O.OracleProblem(1, n, phase, 16.0)
    K = O.dense_K(p)
    f = gaussian_complex((n, B), seed)
    fh = O.dft(f, 1, n)
    u = K @ fh
    return p, K, f, fh, u


# ---------------------------------------------------------------- butterfly applies
@pytest.mark.parametrize("dtype", [F.FIO_C128, F.FIO_C64])
@pytest.mark.parametrize("n,B", [(256, 1), (256, 5), (4096, 3)])
def test_apply_K_and_KH_vs_oracle(n, B, dtype):
    eps = 1e-6
    plan = plan_for(n)
    p = O.OracleProblem(1, n, "1d_ex1", 16.0)
    K = O.dense_K(p)
    x = gaussian_complex((n, B), 100 + B)
    log("apply K n=%d B=%d dtype=%d" % (n, B, dtype))
    y = G.apply(plan, F.FIO_OP_K, dtype, x)
    assert O.rel_err(y, K @ x).max() < 10 * eps
    yh = G.apply(plan, F.FIO_OP_KH, dtype, x)
    assert O.rel_err(yh, K.conj().T @ x).max() < 10 * eps


def test_apply_matches_saved_factors_tightly(tmp_path):
    """Kernel correctness: the GPU c128 apply equals the host product of the same
    factors up to FP64 rounding (summation order only)."""
    plan = plan_for(256)
    path = str(tmp_path / "p.fio")
    F.fio_save(plan, path)
    f = FF.read(path)
    x = gaussian_complex((256, 7), 7)
    y = G.apply(plan, F.FIO_OP_K, F.FIO_C128, x)
    assert O.rel_err(y, FF.apply_K(f, x)).max() < 1e-13
    yh = G.apply(plan, F.FIO_OP_KH, F.FIO_C128, x)
    assert O.rel_err(yh, FF.apply_KH(f, x)).max() < 1e-13
    z = G.inverse(plan, F.FIO_C128, x)
    assert O.rel_err(z, FF.inverse(f, x)).max() < 1e-12


@pytest.mark.parametrize("n,B", [(256, 64), (256, 70), (4096, 17)])
def test_batched_matrix_core_path_tight(tmp_path, n, B):
    """Batches of >= 16 right-hand sides run on matrix cores (complex products as
    four real MFMAs, 64-column tiles with a ragged tail): complex128 must equal the
    host product of the same factors to FP64 rounding, complex64 to FP32 rounding."""
    plan = plan_for(n)
    path = str(tmp_path / "p.fio")
    F.fio_save(plan, path)
    f = FF.read(path)
    x = gaussian_complex((n, B), 8 + B)
    ref = FF.apply_K(f, x)
    refh = FF.apply_KH(f, x)
    log("matrix-core apply n=%d B=%d" % (n, B))
    assert O.rel_err(G.apply(plan, F.FIO_OP_K, F.FIO_C128, x), ref).max() < 1e-13
    assert O.rel_err(G.apply(plan, F.FIO_OP_KH, F.FIO_C128, x), refh).max() < 1e-13
    assert O.rel_err(G.apply(plan, F.FIO_OP_K, F.FIO_C64, x), ref).max() < 2e-6
    assert O.rel_err(G.apply(plan, F.FIO_OP_KH, F.FIO_C64, x), refh).max() < 2e-6


def test_leading_dimension_and_ragged_batch():
    plan = plan_for(256)
    x = gaussian_complex((256, 37), 9)
    a = G.apply(plan, F.FIO_OP_K, F.FIO_C128, x, ld=300)
    b = G.apply(plan, F.FIO_OP_K, F.FIO_C128, x)
    assert np.abs(a - b).max() == 0.0


def test_zero_rhs_is_a_noop():
    plan = plan_for(256)
    F.fio_apply(plan, F.FIO_OP_K, F.FIO_C128, 0, 0, 0, 256, G.stream())


# ---------------------------------------------------------------- direct inverse (config 0)
@pytest.mark.parametrize("dtype", [F.FIO_C128, F.FIO_C64])
def test_direct_inverse_n256_vs_lu(dtype):
    """1D n=256, c/16, eps=1e-6, one Gaussian RHS: fhat = Gd Kd^* u vs dense LU."""
    eps = 1e-6
    plan = plan_for(256, eps=eps)
    p, K, f, fh, u = oracle_case(256, 1, 1000)
    ref = O.solve_dense(p, u, K)
    log("direct inverse n=256 dtype=%d" % dtype)
    x = G.inverse(plan, dtype, u)
    tol = 10 * eps if dtype == F.FIO_C128 else 10 * eps
    assert O.rel_err(x, ref).max() < tol
    # the recovered spatial f (the oracle's inverse DFT of the GPU result)
    assert O.rel_err(O.idft(x, 1, 256), f).max() < tol


def test_identity_phase_inverse_is_dft():
    """Phi = x.xi: Gd Kd^* u = F u = fft((-1)^k u)/N exactly (rank-0 hierarchy)."""
    n = 4096
    plan = plan_for(n, phase="linear")
    u = gaussian_complex((n, 4), 77)
    x = G.inverse(plan, F.FIO_C128, u)
    ref = np.fft.fft(((-1.0) ** np.arange(n))[:, None] * u, axis=0) / n
    assert O.rel_err(x, ref).max() < 1e-6


# ---------------------------------------------------------------- solves (config 1)
def test_refine_c64_n4096_batch64_vs_lu():
    """1D N=4096, 64 RHS: complex64 factor applies + FP64 refinement <= 10 eps."""
    eps = 1e-6
    plan = plan_for(4096, eps=eps)
    p, K, f, fh, u = oracle_case(4096, 64, 1001)
    ref = O.solve_dense(p, u, K)
    log("refine c64 N=4096 B=64")
    x, (its, rr) = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=2)
    err = O.rel_err(x, ref)
    log("  max rel err %.3e, median %.3e, last correction %.3e" % (err.max(), np.median(err), rr))
    assert err.max() < 10 * eps


def test_plain_fp64_single_rhs_n4096():
    eps = 1e-6
    plan = plan_for(4096, eps=eps)
    p, K, f, fh, u = oracle_case(4096, 1, 1001)
    ref = O.solve_dense(p, u, K)
    x, _ = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C128, u, maxit=1)
    assert O.rel_err(x, ref).max() < 10 * eps


@pytest.mark.parametrize("precondition,max_its", [(1, 4), (0, 20)])
def test_pcg_on_normal_equations(precondition, max_its):
    """pcg(Kd^*Kd, Kd^*u, Gd) to 1e-8 (section 5 and 6): few iterations with Gd,
    the unpreconditioned count (12 for c/16) without."""
    plan = plan_for(4096, eps=1e-6)
    p, K, f, fh, u = oracle_case(4096, 4, 1002)
    ref = O.solve_dense(p, u, K)
    x, (its, rr) = G.solve(plan, F.FIO_SOLVE_PCG, F.FIO_C128, u, tol=1e-8, maxit=100,
                           precondition=precondition)
    log("pcg precondition=%d its=%d resid=%.2e" % (precondition, its, rr))
    assert its <= max_its
    assert O.rel_err(x, ref).max() < 1e-5


def test_refine_n65536_batch64_sampled_columns():
    """The measured configuration (1D N=65536, 64 RHS, c64 + FP64 refinement): four
    columns carry u = K fhat from the oracle's direct summation and must recover
    fhat to <= 10 eps; the other columns are random right-hand sides."""
    n, B, eps = 65536, 64, 1e-6
    plan = plan_for(n, eps=eps)
    p = O.OracleProblem(1, n, "1d_ex1", 16.0)
    fh = gaussian_complex((n, 4), 2001)
    log("oracle direct summation N=65536, 4 columns")
    u_known = O.apply_direct(p, fh)
    u = gaussian_complex((n, B), 2002)
    cols = np.array([0, 17, 40, 63])
    u[:, cols] = u_known
    log("refine c64 N=65536 B=64")
    x, (its, rr) = G.solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=2)
    err = O.rel_err(x[:, cols], fh)
    log("  rel err %s" % err)
    assert err.max() < 10 * eps
    # residual on sampled rows for every column (a property at any size)
    rows = uniform_indices(64, n, 5)
    r = O.apply_direct(p, x, out_idx=rows) - u[rows]
    rel = np.linalg.norm(r, axis=0) / np.linalg.norm(u[rows], axis=0)
    assert rel.max() < 10 * eps


def test_identity_phase_n65536_fft_pin():
    n = 65536
    plan = plan_for(n, phase="linear")
    u = gaussian_complex((n, 2), 78)
    x = G.inverse(plan, F.FIO_C64, u)
    ref = np.fft.fft(((-1.0) ** np.arange(n))[:, None] * u, axis=0) / n
    assert O.rel_err(x, ref).max() < 1e-5


def test_autotuned_variants_give_the_same_results():
    """fio_autotune picks a kernel variant per stage; results stay within FP32
    rounding of the built-in choice (complex64) and FP64 rounding (complex128)."""
    plan = plan_for(4096)
    x = gaussian_complex((4096, 64), 31)
    before64 = G.apply(plan, F.FIO_OP_K, F.FIO_C64, x)
    before128 = G.apply(plan, F.FIO_OP_KH, F.FIO_C128, x)
    F.fio_autotune(plan, F.FIO_C64, 64, 2, G.stream())
    F.fio_autotune(plan, F.FIO_C128, 64, 2, G.stream())
    st = F.fio_plan_stats(plan)
    vs = [F.fio_tune_query(plan, F.FIO_OP_K, s, F.FIO_C64, 64) for s in range(st["n_stages"])]
    log("tuned complex64 variants: %s" % vs)
    assert all(0 <= v <= 6 for v in vs)
    assert O.rel_err(G.apply(plan, F.FIO_OP_K, F.FIO_C64, x), before64).max() < 1e-5
    assert O.rel_err(G.apply(plan, F.FIO_OP_KH, F.FIO_C128, x), before128).max() < 1e-12
