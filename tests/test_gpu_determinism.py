"""Run-to-run determinism: every solve mode, repeated on the same plan and input,
returns the same bits (no atomics in any reduction; column norms and dots are
two-pass), and a batch solved in two halves equals the halves of the whole batch
solved at once (columns are independent, tiles only pad).  A race on shared
workspace or an order-dependent reduction would show up here."""
import sys

import numpy as np
import pytest

from fio_synth import gaussian_complex
from paper_2105_02995_amd import fio as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402

_plan = {}


def plan():
    if "p" not in _plan:
        print("building 1D N=4096 plan", flush=True)
        _plan["p"] = F.fio_build(F.make_problem(1, 4096, "1d_ex1", eps=1e-6, device=0))
    return _plan["p"]


MODES = [(F.FIO_SOLVE_DIRECT, 0.0, 0), (F.FIO_SOLVE_REFINE, 0.0, 2), (F.FIO_SOLVE_PCG, 1e-8, 50),
         (F.FIO_SOLVE_GMRES, 1e-8, 50)]


@pytest.mark.parametrize("mode,tol,maxit", MODES)
@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
def test_repeated_solves_are_bitwise_equal(mode, tol, maxit, dtype):
    p = plan()
    u = gaussian_complex((4096, 40), 77)
    print("mode %d dtype %d" % (mode, dtype), flush=True)
    x1, _ = G.solve(p, mode, dtype, u, tol=tol, maxit=maxit)
    x2, _ = G.solve(p, mode, dtype, u, tol=tol, maxit=maxit)
    x3, _ = G.solve(p, mode, dtype, u, tol=tol, maxit=maxit)
    assert np.array_equal(x1, x2) and np.array_equal(x2, x3)


@pytest.mark.parametrize("mode,tol,maxit", MODES[:2])
def test_split_batch_equals_whole_batch(mode, tol, maxit):
    p = plan()
    u = gaussian_complex((4096, 64), 78)
    whole, _ = G.solve(p, mode, F.FIO_C64, u, tol=tol, maxit=maxit)
    lo, _ = G.solve(p, mode, F.FIO_C64, u[:, :32], tol=tol, maxit=maxit)
    hi, _ = G.solve(p, mode, F.FIO_C64, u[:, 32:], tol=tol, maxit=maxit)
    assert np.array_equal(whole, np.concatenate([lo, hi], axis=1))


def test_tracing_does_not_change_results():
    """fio_set_trace only adds named host ranges: solves with it on equal those with
    it off, bit for bit."""
    p = plan()
    u = gaussian_complex((4096, 24), 79)
    x0, _ = G.solve(p, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=1)
    F.fio_set_trace(True)
    try:
        x1, _ = G.solve(p, F.FIO_SOLVE_REFINE, F.FIO_C64, u, maxit=1)
        x2, _ = G.solve(p, F.FIO_SOLVE_PCG, F.FIO_C64, u, tol=1e-8, maxit=50)
    finally:
        F.fio_set_trace(False)
    x3, _ = G.solve(p, F.FIO_SOLVE_PCG, F.FIO_C64, u, tol=1e-8, maxit=50)
    assert np.array_equal(x0, x1) and np.array_equal(x2, x3)


@pytest.mark.parametrize("d,n,phase,eps", [(1, 4096, "1d_ex1", 1e-6), (2, 32, "2d_radon", 1e-4)])
def test_loaded_plan_equals_built_plan(tmp_path, d, n, phase, eps):
    """A plan saved and loaded onto the device forms its complex64 copies and the
    adjoint chain again on the device (from the stored forward chain): applies of
    Kd, Kd^* and solves equal those of the plan that was built, bit for bit."""
    built = plan() if d == 1 else F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
    path = str(tmp_path / "p.fio")
    F.fio_save(built, path)
    loaded = F.fio_load(path, device=0)
    N = n ** d
    x = gaussian_complex((N, 12), 79)
    for op in (F.FIO_OP_K, F.FIO_OP_KH):
        for dt in (F.FIO_C64, F.FIO_C128):
            assert np.array_equal(G.apply(built, op, dt, x), G.apply(loaded, op, dt, x))
    for mode, tol, maxit in MODES[:2]:
        a, _ = G.solve(built, mode, F.FIO_C64, x, tol=tol, maxit=maxit)
        b, _ = G.solve(loaded, mode, F.FIO_C64, x, tol=tol, maxit=maxit)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [128, 256])
def test_builds_give_identical_factors_2d(n):
    """Two builds of the same 2D problem give bit-identical factors: the fingerprints
    of the butterfly, of every skeletonization step and of the top-level inverse
    agree.  The large skeletonization nodes, their IDs and the top-level inverse run
    through the device's dense routines here (n = 256: 664 device IDs, 89 device
    node factorizations), where concurrent streams once made builds differ."""
    fps = []
    for rep in range(2):
        p = F.fio_build(F.make_problem(2, n, "2d_radon", eps=1e-4, device=0))
        fps.append(F.fio_plan_fingerprints(p))
        st = F.fio_plan_stats(p)
        print("2D n=%d build %d: root %d, %d fingerprints, first %016x" % (n, rep, st["root_size"], len(fps[-1]),
                                                                          fps[-1][0]), flush=True)
        p.close()
    assert len(fps[0]) == st["hif_levels"] + 2
    assert fps[0] == fps[1], [i for i, (a, b) in enumerate(zip(*fps)) if a != b]
