"""Fused pairs and triples of butterfly stages (two or three consecutive factors of
Kd in one launch, the intermediate coefficients kept in LDS) against the same
factors applied one launch each, and the launch schedules that the applies use."""
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


@pytest.fixture(scope="module")
def plan():
    log("building 1D plan n=4096")
    return F.fio_build(F.make_problem(1, 4096, "1d_ex1", eps=1e-6, device=0))


def _stage_io(plan, op, s):
    """(input entries, output entries) of factor s of the chain of op."""
    st = F.fio_plan_stats(plan)
    S = st["n_stages"]
    fs = s if op == F.FIO_OP_K else S - 1 - s  # the adjoint chain runs the factors backwards
    i = F.fio_stage_info(plan, fs)
    rows_out = i["n_out"] * i["r_out"]
    # input size: output size of the neighbouring factor on the input side
    if op == F.FIO_OP_K:
        rows_in = st["n"] ** st["d"] if s == 0 else F.fio_stage_info(plan, fs - 1)["n_out"] * F.fio_stage_info(plan, fs - 1)["r_out"]
        return rows_in, rows_out
    return rows_out, (st["n"] ** st["d"] if fs == 0 else F.fio_stage_info(plan, fs - 1)["n_out"] * F.fio_stage_info(plan, fs - 1)["r_out"])


@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
@pytest.mark.parametrize("op", [F.FIO_OP_K, F.FIO_OP_KH])
@pytest.mark.parametrize("B", [16, 40, 64, 100])
def test_fused_pair_equals_two_single_launches(plan, dtype, op, B):
    S = F.fio_plan_stats(plan)["n_stages"]
    ct = G.CT[dtype]
    tol = 1e-5 if dtype == F.FIO_C64 else 1e-13
    fused = 0
    for s in range(S - 1):
        n_in, n_mid = _stage_io(plan, op, s)
        _, n_out = _stage_io(plan, op, s + 1)
        x = torch.from_numpy(np.ascontiguousarray(gaussian_complex((n_in, B), 50 + s))).to(ct).cuda()
        mid = torch.zeros((n_mid, B), dtype=ct, device="cuda")
        ref = torch.zeros((n_out, B), dtype=ct, device="cuda")
        out = torch.full((n_out, B), float("nan"), dtype=ct, device="cuda")
        F.fio_stage_apply(plan, op, s, dtype, x, mid, B, G.stream())
        F.fio_stage_apply(plan, op, s + 1, dtype, mid, ref, B, G.stream())
        try:
            F.fio_stage_pair_apply(plan, op, s, dtype, x, out, B, G.stream())
        except F.FioError as e:
            assert e.status == 6, e  # FIO_ERR_UNSUPPORTED: this pair is not fusable
            continue
        torch.cuda.synchronize()
        a, r = out.cpu().numpy(), ref.cpu().numpy()
        err = np.abs(a - r).max() / max(np.abs(r).max(), 1e-300)
        log("op=%d dtype=%d B=%d pair (%d,%d): rel diff %.2e" % (op, dtype, B, s, s + 1, err))
        assert np.isfinite(a).all()
        assert err < tol
        fused += 1
    assert fused >= (S - 1) // 2  # 1D butterflies fuse every pair of consecutive stages


@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
@pytest.mark.parametrize("op", [F.FIO_OP_K, F.FIO_OP_KH])
@pytest.mark.parametrize("B", [16, 40, 64, 100])
def test_fused_triple_equals_three_single_launches(plan, dtype, op, B):
    """Three consecutive factors in one launch (closed groups of four blocks per
    factor, both intermediates in LDS) equal the three factors launched one by one,
    full and ragged batches (the last column half of a workgroup empty at B = 16 and
    B = 40)."""
    S = F.fio_plan_stats(plan)["n_stages"]
    ct = G.CT[dtype]
    tol = 1e-5 if dtype == F.FIO_C64 else 1e-13
    fused = 0
    for s in range(S - 2):
        n_in, n_m1 = _stage_io(plan, op, s)
        _, n_m2 = _stage_io(plan, op, s + 1)
        _, n_out = _stage_io(plan, op, s + 2)
        x = torch.from_numpy(np.ascontiguousarray(gaussian_complex((n_in, B), 90 + s))).to(ct).cuda()
        m1 = torch.zeros((n_m1, B), dtype=ct, device="cuda")
        m2 = torch.zeros((n_m2, B), dtype=ct, device="cuda")
        ref = torch.zeros((n_out, B), dtype=ct, device="cuda")
        out = torch.full((n_out, B), float("nan"), dtype=ct, device="cuda")
        F.fio_stage_apply(plan, op, s, dtype, x, m1, B, G.stream())
        F.fio_stage_apply(plan, op, s + 1, dtype, m1, m2, B, G.stream())
        F.fio_stage_apply(plan, op, s + 2, dtype, m2, ref, B, G.stream())
        try:
            F.fio_stage_triple_apply(plan, op, s, dtype, x, out, B, G.stream())
        except F.FioError as e:
            assert e.status == 6, e  # FIO_ERR_UNSUPPORTED: these three do not fuse
            continue
        torch.cuda.synchronize()
        a, r = out.cpu().numpy(), ref.cpu().numpy()
        err = np.abs(a - r).max() / max(np.abs(r).max(), 1e-300)
        log("op=%d dtype=%d B=%d triple (%d,%d,%d): rel diff %.2e" % (op, dtype, B, s, s + 1, s + 2, err))
        assert np.isfinite(a).all()
        assert err < tol
        fused += 1
    assert fused >= 1  # the 1D butterfly's consecutive factors form such groups away from the middle


def test_fused_triple_argument_errors(plan):
    S = F.fio_plan_stats(plan)["n_stages"]
    X = torch.zeros(64, dtype=torch.complex64, device="cuda")
    for s in (-1, S - 2):
        with pytest.raises(F.FioError) as e:
            F.fio_stage_triple_apply(plan, F.FIO_OP_K, s, F.FIO_C64, X, X, 1, G.stream())
        assert e.value.status == 1


@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
def test_schedules_cover_every_stage_once_in_order(plan, dtype):
    S = F.fio_plan_stats(plan)["n_stages"]
    for nrhs in (1, 8, 16, 64):
        for op in (F.FIO_OP_K, F.FIO_OP_KH):
            sch = F.fio_chain_schedule(plan, op, dtype, nrhs)
            covered = [f + j for f, c, _ in sch for j in range(c)]
            assert covered == list(range(S)), (nrhs, op, sch)
            if nrhs < 16:
                assert all(c == 1 for _, c, _ in sch)
            else:
                assert any(c == 2 for _, c, _ in sch)
    F.fio_autotune(plan, dtype, 48, 2, G.stream())
    for op in (F.FIO_OP_K, F.FIO_OP_KH):
        sch = F.fio_chain_schedule(plan, op, dtype, 48)
        log("tuned schedule dtype=%d op=%d: %s" % (dtype, op, sch))
        assert [f + j for f, c, _ in sch for j in range(c)] == list(range(S))


@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
def test_tuned_schedule_apply_matches_oracle(plan, dtype):
    """After tuning (single factors, pairs or triples per the timings), Kd and Kd^*
    still match the direct sums."""
    p = O.OracleProblem(1, 4096, "1d_ex1", 16.0)
    x = gaussian_complex((4096, 48), 77)
    rows = np.arange(0, 4096, 97)
    F.fio_autotune(plan, dtype, 48, 2, G.stream())
    for op, adj in ((F.FIO_OP_K, False), (F.FIO_OP_KH, True)):
        log("tuned schedule dtype=%d op=%d: %s" % (dtype, op, F.fio_chain_schedule(plan, op, dtype, 48)))
        ref = O.apply_direct(p, x, adjoint=adj, out_idx=rows)
        y = G.apply(plan, op, dtype, x)
        assert O.rel_err(y[rows], ref).max() < 1e-5


@pytest.mark.parametrize("dtype", [F.FIO_C64, F.FIO_C128])
@pytest.mark.parametrize("op", [F.FIO_OP_K, F.FIO_OP_KH])
@pytest.mark.parametrize("B", [16, 40, 64, 100])
def test_every_fused_variant_equals_two_single_launches(plan, dtype, op, B):
    """Each fused-pair kernel variant (16/32/64 columns per wave, and the stacked form
    where two sibling blocks sharing their inputs form one three-tile operand) equals
    the two stages launched one by one, full and ragged batches."""
    S = F.fio_plan_stats(plan)["n_stages"]
    ct = G.CT[dtype]
    tol = 1e-5 if dtype == F.FIO_C64 else 1e-13
    variants = [1, 2, 4] + ([3] if dtype == F.FIO_C64 else [])
    stacked = 0
    for s in range(S - 1):
        n_in, n_mid = _stage_io(plan, op, s)
        _, n_out = _stage_io(plan, op, s + 1)
        x = torch.from_numpy(np.ascontiguousarray(gaussian_complex((n_in, B), 70 + s))).to(ct).cuda()
        mid = torch.zeros((n_mid, B), dtype=ct, device="cuda")
        ref = torch.zeros((n_out, B), dtype=ct, device="cuda")
        F.fio_stage_apply(plan, op, s, dtype, x, mid, B, G.stream())
        F.fio_stage_apply(plan, op, s + 1, dtype, mid, ref, B, G.stream())
        torch.cuda.synchronize()
        r = ref.cpu().numpy()
        for v in variants:
            out = torch.full((n_out, B), float("nan"), dtype=ct, device="cuda")
            try:
                F.fio_stage_pair_apply_variant(plan, op, s, dtype, v, x, out, B, G.stream())
            except F.FioError as e:
                assert e.status == 6, e  # not fusable, or not stackable
                continue
            torch.cuda.synchronize()
            a = out.cpu().numpy()
            err = np.abs(a - r).max() / max(np.abs(r).max(), 1e-300)
            log("op=%d dtype=%d B=%d pair (%d,%d) variant %d: rel diff %.2e" % (op, dtype, B, s, s + 1, v, err))
            assert np.isfinite(a).all()
            assert err < tol
            stacked += v == 4
    assert stacked >= 1  # ranks of this plan allow the stacked form somewhere
