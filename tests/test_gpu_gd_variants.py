"""Every kernel of Gd's skeletonization steps (section 4: the upward sweep with
R_l^*, the FP64 top-level block A_0^{-1}, the downward sweep with R_l): the
LDS-staged node kernel, gathered GEMMs in three tile widths and the fused per-node
matrix-core kernel, each run on every step it applies to, against the host
product of the same saved factors: FP64 rounding for complex128, FP32 rounding
for complex64, full and ragged batches."""
import sys

import numpy as np
import pytest

from fio_synth import gaussian_complex
import oracle as O
from paper_2105_02995_amd import fio as F

from . import factor_file as FF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from . import gpu_util as G  # noqa: E402

_plans = {}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plan_and_factors(d, n, phase, eps, tmp_path):
    key = (d, n, phase, eps)
    if key not in _plans:
        log("building d=%d n=%d %s eps=%g" % key)
        plan = F.fio_build(F.make_problem(d, n, phase, eps=eps, device=0))
        path = str(tmp_path / "gd.fio")
        F.fio_save(plan, path)
        _plans[key] = (plan, FF.read(path))
    return _plans[key]


def gd_gpu(plan, dtype, variant, x):
    N = x.shape[0]
    X = G.to_dev(x, dtype)
    Y = G.empty(N, X.shape[0], dtype)
    F.fio_gd_apply_variant(plan, dtype, variant, X, Y, X.shape[0], X.shape[1], G.stream())
    return G.from_dev(Y, N)


@pytest.mark.parametrize("d,n,phase,eps", [(1, 4096, "1d_ex1", 1e-6), (2, 64, "2d_radon", 1e-4)])
@pytest.mark.parametrize("B", [64, 37, 8, 3, 1])
def test_every_skeletonization_kernel_matches_saved_factors(tmp_path, d, n, phase, eps, B):
    plan, f = plan_and_factors(d, n, phase, eps, tmp_path)
    x = gaussian_complex((n ** d, B), 60 + B)
    ref = FF.from_tree(f, FF.gd(f, FF.to_tree(f, x)))
    for variant in range(-1, 13):
        log("Gd d=%d n=%d B=%d variant %d" % (d, n, B, variant))
        e128 = O.rel_err(gd_gpu(plan, F.FIO_C128, variant, x), ref).max()
        e64 = O.rel_err(gd_gpu(plan, F.FIO_C64, variant, x), ref).max()
        log("  c128 %.2e  c64 %.2e" % (e128, e64))
        assert e128 < 1e-12
        assert e64 < 1e-5


def test_variant_out_of_range_is_an_argument_error(tmp_path):
    plan, _ = plan_and_factors(1, 4096, "1d_ex1", 1e-6, tmp_path)
    X = G.empty(4096, 4)
    with pytest.raises(F.FioError) as e:
        F.fio_gd_apply_variant(plan, F.FIO_C128, 13, X, X, 4, 4096, G.stream())
    assert e.value.status == 1


def test_prescaled_factors_on_every_kernel(tmp_path):
    """Cholesky-prescaled skeletonization (1D): its scaling steps (nodes with only
    redundant DOFs) and skeletonization steps run on every kernel, tightly against the
    saved factors, and the direct inverse meets 10 eps against the oracle."""
    eps = 1e-6
    plan = F.fio_build(F.make_problem(1, 4096, "1d_ex1", eps=eps, device=0, prescale_skel=1))
    path = str(tmp_path / "pre.fio")
    F.fio_save(plan, path)
    f = FF.read(path)
    x = gaussian_complex((4096, 48), 91)
    ref = FF.from_tree(f, FF.gd(f, FF.to_tree(f, x)))
    for variant in range(-1, 13):
        log("prescaled Gd variant %d" % variant)
        assert O.rel_err(gd_gpu(plan, F.FIO_C128, variant, x), ref).max() < 1e-12
        assert O.rel_err(gd_gpu(plan, F.FIO_C64, variant, x), ref).max() < 1e-5
    K = O.dense_K(O.OracleProblem(1, 4096, "1d_ex1", 16.0))
    u = K @ x[:, :8]
    assert O.rel_err(G.inverse(plan, F.FIO_C128, u), x[:, :8]).max() < 10 * eps


@pytest.mark.parametrize("B", [1, 2, 5])
def test_small_batch_kernel_2d_n128(tmp_path, B):
    """The small-batch skeletonization kernel on the large nodes of 2D n=128 (phases
    with few tiles and long k ranges run split over workgroups, their partial sums
    added by a second launch; the others on 16-wave or 4-wave workgroups), against
    the host product of the saved factors."""
    plan, f = plan_and_factors(2, 128, "2d_radon", 1e-4, tmp_path)
    x = gaussian_complex((128 * 128, B), 70 + B)
    ref = FF.from_tree(f, FF.gd(f, FF.to_tree(f, x)))
    for variant in (-1, 12):
        e128 = O.rel_err(gd_gpu(plan, F.FIO_C128, variant, x), ref).max()
        e64 = O.rel_err(gd_gpu(plan, F.FIO_C64, variant, x), ref).max()
        log("Gd 2D n=128 B=%d variant %d: c128 %.2e  c64 %.2e" % (B, variant, e128, e64))
        assert e128 < 1e-12
        assert e64 < 1e-5
