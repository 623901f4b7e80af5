"""CPU tests of the C ABI library: symbols, argument checks and the host-side
factor construction (plans built with device = -1 are never applied on the CPU;
their saved factors are multiplied out with NumPy here).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex
from paper_2105_02995_amd import fio as F

from . import factor_file as FF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return F.load_library()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "fio.h")).read()
    declared = set(re.findall(r"\b(fio_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(F.EXPORTS)


@pytest.mark.parametrize("kw,status", [
    (dict(d=3, n=64), 1),
    (dict(d=1, n=100), 1),
    (dict(d=1, n=256, eps=1.5), 1),
    (dict(d=1, n=256, eps=0.0), 1),
    (dict(d=2, n=64, phase="1d_ex1"), 1),
    (dict(d=1, n=256, phase="2d_radon"), 1),
])
def test_build_rejects_bad_arguments(lib, kw, status):
    args = dict(d=1, n=256, phase="1d_ex1", eps=1e-6, device=-1)
    args.update(kw)
    with pytest.raises(F.FioError) as e:
        F.fio_build(F.make_problem(**args))
    assert e.value.status == status


def _host_plan(tmp_path, n=256, phase="1d_ex1", eps=1e-6, **kw):
    plan = F.fio_build(F.make_problem(1, n, phase, eps=eps, device=-1, **kw))
    path = str(tmp_path / "plan.fio")
    F.fio_save(plan, path)
    return plan, FF.read(path), path


def test_host_only_plan_refuses_applies(tmp_path):
    plan, _, _ = _host_plan(tmp_path)
    with pytest.raises(F.FioError) as e:
        F.fio_apply(plan, F.FIO_OP_K, F.FIO_C128, 1, 1, 1, 256)
    assert e.value.status == 6
    with pytest.raises(F.FioError):
        F.fio_solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C64, 1, 1, 1, 256)
    for call in (lambda: F.fio_inverse_dft(plan, 1, 1, 1, 256),
                 lambda: F.fio_stage_pair_apply(plan, F.FIO_OP_K, 0, F.FIO_C64, 1, 1, 16),
                 lambda: F.fio_solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C64, 1, 1, 1, 256, spatial=1)):
        with pytest.raises(F.FioError) as e:
            call()
        assert e.value.status == 6


def test_butterfly_accuracy_against_oracle(tmp_path):
    """e_a = ||K - Kd|| / ||K|| (section 6) on random vectors, eps_bf = eps/10."""
    eps = 1e-6
    plan, f, _ = _host_plan(tmp_path, eps=eps)
    st = F.fio_plan_stats(plan)
    assert st["n_stages"] == st["L"] + 3
    p = O.OracleProblem(1, 256, "1d_ex1", 16.0)
    K = O.dense_K(p)
    x = gaussian_complex((256, 4), 11)
    assert O.rel_err(FF.apply_K(f, x), K @ x).max() < eps
    assert O.rel_err(FF.apply_KH(f, x), K.conj().T @ x).max() < eps


def test_direct_inverse_within_ten_eps(tmp_path):
    """Gd Kd^* u against the oracle's LU solve: <= 10 eps (section 5, eq:pseudoinv)."""
    eps = 1e-6
    _, f, _ = _host_plan(tmp_path, eps=eps)
    p = O.OracleProblem(1, 256, "1d_ex1", 16.0)
    K = O.dense_K(p)
    fs = gaussian_complex((256, 3), 1000)
    u = K @ O.dft(fs, 1, 256)
    ref = O.solve_dense(p, u, K)
    assert O.rel_err(FF.inverse(f, u), ref).max() < 10 * eps


def test_gd_is_hermitian_positive(tmp_path):
    _, f, _ = _host_plan(tmp_path)
    x = gaussian_complex(256, 3)
    y = gaussian_complex(256, 4)
    a = np.vdot(y, FF.gd(f, x))
    b = np.vdot(FF.gd(f, y), x)
    assert abs(a - b) < 1e-10 * abs(a)
    assert np.vdot(x, FF.gd(f, x)).real > 0


def test_identity_phase_gives_rank_zero_hierarchy(tmp_path):
    """Phi = x.xi: S = N I, every off-diagonal block is empty and Gd Kd^* = F."""
    _, f, _ = _host_plan(tmp_path, phase="linear")
    assert f["max_rank_h"] == 0
    assert f["root"].size == 0
    u = gaussian_complex(256, 5)
    ref = O.dft(u, 1, 256)  # K^{-1} = F when K = N F^*
    assert O.rel_err(FF.inverse(f, u), ref).max() < 1e-6


def test_save_load_roundtrip(tmp_path):
    plan, f, path = _host_plan(tmp_path)
    plan2 = F.fio_load(path, device=-1)
    path2 = str(tmp_path / "plan2.fio")
    F.fio_save(plan2, path2)
    assert open(path, "rb").read() == open(path2, "rb").read()


def test_load_rejects_garbage(tmp_path):
    bad = tmp_path / "bad.fio"
    bad.write_bytes(b"not a plan")
    with pytest.raises(F.FioError) as e:
        F.fio_load(str(bad), device=-1)
    assert e.value.status == 7


def test_2d_host_construction_n32(tmp_path):
    """2D generalized Radon example (section 6, Example 3) at n=32, eps=1e-4: the
    H-matrix peeling (strong admissibility, periodic neighbours) and the cell/edge
    skeletonization inverse give a direct solve within 10 eps, and Gd makes CG on
    the normal equations converge in a few iterations (section 5)."""
    eps = 1e-4
    plan = F.fio_build(F.make_problem(2, 32, "2d_radon", eps=eps, device=-1))
    path = str(tmp_path / "p2.fio")
    F.fio_save(plan, path)
    f = FF.read(path)
    p = O.OracleProblem(2, 32, "2d_radon", 16.0)
    K = O.dense_K(p)
    x = gaussian_complex((1024, 2), 3)
    assert O.rel_err(FF.apply_K(f, x), K @ x).max() < eps
    fs = gaussian_complex((1024, 2), 1002)
    u = K @ O.dft(fs, 2, 32)
    ref = O.solve_dense(p, u, K)
    assert O.rel_err(FF.inverse(f, u), ref).max() < 10 * eps
    pre = lambda r: FF.from_tree(f, FF.gd(f, FF.to_tree(f, r)))
    _, its = O.cg_normal(lambda v: FF.apply_K(f, v), lambda v: FF.apply_KH(f, v), u[:, 0],
                         tol=1e-8, precond=pre)
    assert its <= 4
    # every DOF is eliminated exactly once or kept in the root
    seen = np.concatenate([nd["r"] for st in f["steps"] for nd in st] + [f["root"]])
    assert np.array_equal(np.sort(seen), np.arange(1024))


MIX = ((0.2, -0.2), (0.5, 0.2), (0.8, 0.0))


@pytest.mark.parametrize("s2", [0.1, 0.05])
def test_example2_host_factors(tmp_path, s2):
    """Example 2 (variable amplitude): the butterfly reaches e_a <= eps, and Gd Kd^*
    solves within the accuracy the conditioning allows: the peeling and
    skeletonization tolerances are relative to ||S||, S = Kd^* Kd, so the error of
    Gd S is about eps cond(S) = eps cond(K)^2 (against the oracle's LU solve)."""
    n, eps = 512, 1e-6
    plan, f, _ = _host_plan(tmp_path, n=n, phase="1d_ex2", eps=eps, amp=MIX, amp_sigma2=s2)
    p = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=MIX, sigma2=s2)
    K = O.dense_K(p)
    x = gaussian_complex((n, 4), 13)
    ea = O.rel_err(FF.apply_K(f, x), K @ x).max()
    assert ea < eps
    assert O.rel_err(FF.apply_KH(f, x), K.conj().T @ x).max() < eps
    fs = gaussian_complex((n, 3), 1001)
    u = K @ O.dft(fs, 1, n)
    ref = O.solve_dense(p, u, K)
    es = O.rel_err(FF.inverse(f, u), ref).max()
    cond = np.linalg.cond(K)
    print("sigma2 %.2f: e_a %.2e, e_s %.2e, cond(K) %.1f" % (s2, ea, es, cond))
    assert es < 10 * eps * cond ** 2, (es, cond)


def test_example2_rejects_bad_amplitude_arguments():
    with pytest.raises(F.FioError):
        F.fio_build(F.make_problem(1, 256, "1d_ex2", eps=1e-6, device=-1, amp_sigma2=-1.0))
    with pytest.raises(F.FioError):
        F.fio_build(F.make_problem(2, 64, "1d_ex2", eps=1e-4, device=-1))
    p = F.make_problem(1, 256, "1d_ex2", eps=1e-6, device=-1)
    p.amp_terms = 9
    with pytest.raises(F.FioError):
        F.fio_build(p)


def test_example2_ill_conditioned_pivots_are_shifted(tmp_path):
    """sigma2 = 0.05, eps = 1e-4: cond(S) = cond(K)^2 is about 1e5, so pivot blocks of
    the peeled Sd are not positive definite.  With strict_hpd the build stops with
    FIO_ERR_NOT_HPD; by default those blocks get a small diagonal shift and Gd stays
    a preconditioner: CG on K^*K with Gd converges in a few tens of iterations (the
    eps ||S|| truncation bounds its quality at this conditioning), where K^* alone
    needs well over a thousand (oracle, dense K)."""
    n, eps, s2 = 4096, 1e-4, 0.05
    with pytest.raises(F.FioError) as e:
        F.fio_build(F.make_problem(1, n, "1d_ex2", eps=eps, device=-1, amp=MIX, amp_sigma2=s2, strict_hpd=1))
    assert e.value.status == 4
    plan, f, _ = _host_plan(tmp_path, n=n, phase="1d_ex2", eps=eps, amp=MIX, amp_sigma2=s2)
    shifted = F.fio_plan_stats(plan)["hif_shifted"]
    assert shifted > 0
    p = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=MIX, sigma2=s2)
    K = O.dense_K(p)
    b = K @ gaussian_complex(n, 1002)
    gd_nat = lambda r: FF.from_tree(f, FF.gd(f, FF.to_tree(f, r)))  # noqa: E731
    x, its = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, b, tol=1e-8, maxit=500, precond=gd_nat)
    print("shifted %d pivot blocks; PCG with Gd: %d iterations" % (shifted, its))
    assert its <= 40


def test_c_example_is_built_and_checks_its_arguments():
    """build() compiles the plain-C user of the ABI; without arguments it prints its
    usage and exits with status 2 (no GPU call is made)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2105_02995_amd", "fio_solve_file")
    assert os.path.exists(exe)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


def test_prescaled_skeletonization_matches_the_oracle_and_the_standard_inverse(tmp_path):
    """Cholesky-prescaled skeletonization (section 4, the alternative to the
    elimination step): two steps per level, the first a pure scaling (only
    redundant DOFs, lower-triangular L^{-1}); Gd Hermitian positive; Gd Kd^* u within
    10 eps of the oracle's LU solve, and within eps of the standard variant's Gd."""
    eps = 1e-6
    (tmp_path / "s").mkdir()
    _, fs, _ = _host_plan(tmp_path / "s", n=1024, eps=eps)
    _, fp, _ = _host_plan(tmp_path, n=1024, eps=eps, prescale_skel=1)
    assert len(fp["steps"]) == 2 * len(fs["steps"])
    for k, nodes in enumerate(fp["steps"]):
        if k % 2 == 0:  # the scaling step of a level
            for nd in nodes:
                assert nd["s"].size == 0
                assert np.allclose(np.triu(nd["Linv"], 1), 0)
    x, y = gaussian_complex(1024, 3), gaussian_complex(1024, 4)
    a, b = np.vdot(y, FF.gd(fp, x)), np.vdot(FF.gd(fp, y), x)
    assert abs(a - b) < 1e-10 * abs(a) and np.vdot(x, FF.gd(fp, x)).real > 0
    p = O.OracleProblem(1, 1024, "1d_ex1", 16.0)
    K = O.dense_K(p)
    u = K @ gaussian_complex((1024, 3), 1001)
    ref = O.solve_dense(p, u, K)
    assert O.rel_err(FF.inverse(fp, u), ref).max() < 10 * eps
    assert O.rel_err(FF.inverse(fp, u), FF.inverse(fs, u)).max() < eps


def test_prescaled_identity_phase_inverse_is_the_dft(tmp_path):
    """Phi = x.xi: S = N I, so the scaling is N^{-1/2} I and no DOF survives."""
    _, f, _ = _host_plan(tmp_path, phase="linear", prescale_skel=1)
    assert f["root"].size == 0
    u = gaussian_complex(256, 5)
    assert O.rel_err(FF.inverse(f, u), O.dft(u, 1, 256)).max() < 1e-6


def test_prescaled_skeletonization_is_one_dimensional_only():
    with pytest.raises(F.FioError) as e:
        F.fio_build(F.make_problem(2, 16, "2d_radon", eps=1e-4, device=-1, prescale_skel=1))
    assert e.value.status == 1


def test_column_id_checks_its_arguments():
    """fio_column_id refuses bad shapes, tolerances and null pointers with a status,
    and reports a device error (not a crash) where there is no GPU."""
    import ctypes
    import numpy as np
    lib = F.load_library()
    A = np.zeros((8, 4), dtype=np.complex128, order="F")
    rank = ctypes.c_int()
    perm = np.zeros(4, dtype=np.int32)
    T = np.zeros(16, dtype=np.complex128)
    args = lambda m, n, lda, tol, a=A.ctypes.data: (0, m, n, a, lda, tol, ctypes.byref(rank), perm.ctypes.data,
                                                     T.ctypes.data, 16)
    assert lib.fio_column_id(*args(8, 4, 4, 1e-6)) == 1        # lda < m
    assert lib.fio_column_id(*args(0, 4, 8, 1e-6)) == 1        # empty
    assert lib.fio_column_id(*args(8, 4, 8, -1.0)) == 1        # negative tolerance
    assert lib.fio_column_id(*args(8, 4, 8, 1e-6, None)) == 1  # null matrix
    try:  # a zero matrix has rank 0 where there is a GPU; a clean status where there is none
        skel, red, _ = F.fio_column_id(A, 1e-6, device=0)
        assert len(skel) == 0 and len(red) == 4
    except F.FioError as e:
        assert e.status in (1, 3)  # ordinal out of range or HIP error


def test_fingerprints_identify_identical_factors(tmp_path):
    """Host builds of one problem give equal fingerprints (butterfly, every
    skeletonization step, top-level inverse); a saved and reloaded plan keeps them;
    another tolerance changes them."""
    def build(eps):
        return F.fio_build(F.make_problem(1, 1024, "1d_ex1", eps=eps, device=-1))
    a, b = build(1e-6), build(1e-6)
    fa = F.fio_plan_fingerprints(a)
    assert len(fa) == F.fio_plan_stats(a)["hif_levels"] + 2
    assert fa == F.fio_plan_fingerprints(b)
    path = str(tmp_path / "f.fio")
    F.fio_save(a, path)
    assert F.fio_plan_fingerprints(F.fio_load(path, -1)) == fa
    fc = F.fio_plan_fingerprints(build(1e-4))
    assert fc[0] != fa[0] and fc[-1] != fa[-1]
    n = ctypes.c_int()
    assert F.load_library().fio_plan_fingerprints(a.handle, None, 1, n) == 1   # FIO_ERR_ARG: no array
    assert F.load_library().fio_plan_fingerprints(a.handle, None, 0, None) == 1  # nor count


def test_plan_stats_count_the_factor_entries(tmp_path):
    """fio_plan_stats against the saved factors (section 4): hif_nnz counts every
    entry of T, L^-1 and M; hif_sweep_nnz the entries one sweep of Gd reads, T, M
    and the lower triangle of L^-1 (whose upper part is zero); bf_nnz every entry of
    the butterfly stages (section 2); the root block is square."""
    plan, f, _ = _host_plan(tmp_path)
    st = F.fio_plan_stats(plan)
    full = sweep = 0
    for nodes in f["steps"]:
        for nd in nodes:
            r = nd["Linv"].shape[0]
            assert np.allclose(np.triu(nd["Linv"], 1), 0)
            full += nd["T"].size + nd["Linv"].size + nd["M"].size
            sweep += nd["T"].size + nd["M"].size + r * (r + 1) // 2
    assert st["hif_nnz"] == full
    assert st["hif_sweep_nnz"] == sweep
    assert 0 < sweep < full
    assert st["bf_nnz"] == sum(s["A"].size for s in f["stages"])
    assert st["root_size"] ** 2 == f["A0inv"].size
