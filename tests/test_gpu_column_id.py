"""Device column interpolative decomposition (the ID of the large stacked bases in
the 2D skeletonization, section 4): ranks against LAPACK's pivoted QR (scipy), pivot
order against a plain pivoted Householder QR written here, reconstruction error,
exactly zero and duplicated columns, wide and empty inputs."""
import sys

import numpy as np
import pytest
import scipy.linalg as sl

from paper_2105_02995_amd import fio as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lowrank(m, n, r, decay, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    V = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    s = decay ** (np.arange(r) / max(r - 1, 1))
    return (U * s) @ V.conj().T


def cpqr_pivots(A, tol_rel):
    """Pivoted Householder QR, largest trailing norm first (first among equals),
    stopping before the first pivot at or below tol_rel * the largest column norm."""
    A = A.copy()
    m, n = A.shape
    nrm = (abs(A) ** 2).sum(0)
    tol = tol_rel * np.sqrt(nrm.max())
    perm = np.arange(n)
    for k in range(min(m, n)):
        p = k + int(np.argmax(nrm[k:]))
        if np.sqrt(nrm[p]) <= tol:
            return perm[:k]
        A[:, [k, p]] = A[:, [p, k]]
        nrm[[k, p]] = nrm[[p, k]]
        perm[[k, p]] = perm[[p, k]]
        x = A[k:, k]
        a0 = abs(x[0])
        alpha = np.linalg.norm(x)
        w = x.copy()
        w[0] += (x[0] / a0 if a0 > 0 else 1.0) * alpha
        wn2 = np.vdot(w, w).real
        if wn2 > 0:
            A[k:, k + 1:] -= np.outer(w, 2 * (w.conj() @ A[k:, k + 1:]) / wn2)
        nrm[k + 1:] = (abs(A[k + 1:, k + 1:]) ** 2).sum(0)
    return perm[:min(m, n)]


def lapack_rank(A, tol_rel):
    R = sl.qr(A, pivoting=True, mode="r")[0]
    d = abs(np.diag(R))
    tol = tol_rel * np.sqrt((abs(A) ** 2).sum(0).max())
    k = 0
    while k < len(d) and d[k] > tol:
        k += 1
    return k


def check(A, tol, exact_pivots=True):
    skel, red, T = F.fio_column_id(A, tol)
    m, n = A.shape
    k = len(skel)
    assert sorted(np.concatenate([skel, red]).tolist()) == list(range(n))
    assert T.shape == (k, n - k)
    assert np.isfinite(T).all()
    res = np.linalg.norm(A[:, red] - A[:, skel] @ T) if n > k else 0.0
    bound = 2 * np.sqrt(max(n - k, 1)) * tol * np.sqrt((abs(A) ** 2).sum(0).max())
    log("m=%d n=%d tol=%g: rank %d (LAPACK %d), residual %.3e (bound %.3e)" % (m, n, tol, k, lapack_rank(A, tol),
                                                                             res, bound))
    assert res <= bound
    assert abs(k - lapack_rank(A, tol)) <= 1
    if exact_pivots:
        assert np.array_equal(skel, cpqr_pivots(A, tol))
    return skel, red, T


@pytest.mark.parametrize("m,n,r", [(1500, 300, 160), (700, 700, 300), (200, 500, 150), (3000, 64, 64)])
def test_ranks_pivots_and_residual(m, n, r):
    check(lowrank(m, n, r, 1e-10, m + n), 1e-6)


def test_zero_columns_are_redundant_with_zero_coefficients():
    A = lowrank(2000, 400, 200, 1e-9, 11)
    zc = np.random.default_rng(3).choice(400, 90, replace=False)
    A[:, zc] = 0
    skel, red, T = check(A, 1e-5)
    assert not set(zc.tolist()) & set(skel.tolist())
    pos = [red.tolist().index(j) for j in zc]
    assert np.all(T[:, pos] == 0)
    # the rank and skeleton are those of the matrix without the zero columns
    keep = np.setdiff1d(np.arange(400), zc)
    skel2, _, _ = F.fio_column_id(A[:, keep], 1e-5)
    assert np.array_equal(keep[skel2], skel)


def test_duplicated_columns_and_exact_rank():
    B = lowrank(1200, 150, 150, 1e-2, 5)
    A = np.concatenate([B, B[:, :60]], axis=1)  # 60 exact copies: rank stays 150
    skel, red, T = check(A, 1e-8, exact_pivots=False)
    assert len(skel) == 150


def test_zero_matrix_and_single_column():
    skel, red, T = F.fio_column_id(np.zeros((900, 40), dtype=complex), 1e-6)
    assert len(skel) == 0 and len(red) == 40 and T.shape == (0, 40)
    a = np.random.default_rng(1).standard_normal((5000, 1)) + 0j
    skel, red, T = F.fio_column_id(a, 1e-6)
    assert skel.tolist() == [0] and len(red) == 0
