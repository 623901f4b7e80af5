"""Layout out with the optional spatial output: f = F^{-1} fhat = n^d F^* fhat
(section 1) on the GPU, against the oracle's inverse DFT (dense, or by rows at
N = 65536), and solves that return f directly."""
import sys

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex, uniform_indices
from paper_2105_02995_amd import fio as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402

_plans = {}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan(d, n, phase, eps):
    key = (d, n, phase, eps)
    if key not in _plans:
        log("building plan %s" % (key,))
        _plans[key] = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
    return _plans[key]


def gpu_idft(p, fh, ld=None):
    N = fh.shape[0]
    X = G.to_dev(fh, F.FIO_C128, ld)
    Y = G.empty(N, X.shape[0], F.FIO_C128, ld)
    F.fio_inverse_dft(p, X, Y, X.shape[0], X.shape[1], G.stream())
    return G.from_dev(Y, N)


@pytest.mark.parametrize("d,n,B,ld", [(1, 256, 1, None), (1, 4096, 5, 4100), (1, 2048, 3, None),
                                      (2, 64, 4, None), (2, 32, 7, 1030)])
def test_inverse_dft_vs_oracle(d, n, B, ld):
    phase = "1d_ex1" if d == 1 else "2d_radon"
    p = plan(d, n, phase, 1e-6 if d == 1 else 1e-4)
    fh = gaussian_complex((n ** d, B), 40 + n + B)
    got = gpu_idft(p, fh, ld)
    ref = O.idft(fh, d, n)
    err = O.rel_err(got, ref).max()
    log("inverse DFT d=%d n=%d B=%d ld=%s: rel err %.2e" % (d, n, B, ld, err))
    assert err < 1e-12


def test_inverse_dft_in_place():
    p = plan(1, 4096, "1d_ex1", 1e-6)
    fh = gaussian_complex((4096, 3), 71)
    X = G.to_dev(fh)
    F.fio_inverse_dft(p, X, X, 3, 4096, G.stream())
    assert O.rel_err(G.from_dev(X, 4096), O.idft(fh, 1, 4096)).max() < 1e-12


def test_inverse_dft_n65536_sampled_rows():
    n, B = 65536, 8
    p = plan(1, n, "1d_ex1", 1e-6)
    fh = gaussian_complex((n, B), 72)
    got = gpu_idft(p, fh)
    rows = uniform_indices(48, n, 73)
    ref = O.idft_rows(fh, 1, n, rows)
    err = O.rel_err(got[rows], ref).max()
    log("inverse DFT N=65536 sampled rows: rel err %.2e" % err)
    assert err < 1e-11


def test_spatial_solve_identity_phase_returns_u():
    """Linear phase: K = n F^* = F^{-1}, so K fhat = u has fhat = F u and the spatial
    output F^{-1} fhat is u itself."""
    n = 4096
    p = plan(1, n, "linear", 1e-6)
    u = gaussian_complex((n, 4), 74)
    f, _ = G.solve(p, F.FIO_SOLVE_DIRECT, F.FIO_C128, u, spatial=1)
    err = O.rel_err(f, u).max()
    log("identity-phase spatial solve: rel err %.2e" % err)
    assert err < 1e-5


@pytest.mark.parametrize("d,n,eps,mode", [(1, 4096, 1e-6, F.FIO_SOLVE_REFINE), (2, 64, 1e-4, F.FIO_SOLVE_REFINE),
                                          (2, 64, 1e-4, F.FIO_SOLVE_PCG)])
def test_spatial_solve_recovers_generator_f(d, n, eps, mode):
    """u = K F f from the oracle; the solve with the spatial output returns f."""
    phase = "1d_ex1" if d == 1 else "2d_radon"
    p = plan(d, n, phase, eps)
    op = O.OracleProblem(d, n, phase, 16.0)
    f = gaussian_complex((n ** d, 6), 75 + d)
    u = O.forward(op, O.dft(f, d, n))
    maxit = 2 if mode == F.FIO_SOLVE_REFINE else 20
    tol = 0.0 if mode == F.FIO_SOLVE_REFINE else 1e-8
    got, _ = G.solve(p, mode, F.FIO_C64, u, tol=tol, maxit=maxit, spatial=1)
    err = O.rel_err(got, f).max()
    log("spatial solve d=%d n=%d mode=%d: rel err %.2e" % (d, n, mode, err))
    assert err < 10 * eps
