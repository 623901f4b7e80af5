"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-runs the oracle's own formula: each compares it with a
closed form computed by a different route (library FFT, identity matrices), an
invariant, or a value printed in the paper (tests/golden/).
"""
import os

import numpy as np
import pytest

import oracle as O
from fio_synth import gaussian_complex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _shift(d, n):
    """(-1)^(k_1 + ... + k_d) over the X grid, lexicographic order."""
    k = np.arange(n)
    s = (-1.0) ** k
    return s if d == 1 else np.outer(s, s).ravel()


@pytest.mark.parametrize("d,n", [(1, 256), (2, 16)])
def test_identity_phase_closed_forms(d, n):
    """Phi = x.xi, a = 1: K = N F^*, so K F = I and K^*K = N I (section 1)."""
    p = O.OracleProblem(d, n, "linear")
    K = O.dense_K(p)
    F = O.dft_matrix(d, n)
    N = p.N
    assert np.abs(K @ F - np.eye(N)).max() < 1e-12
    assert np.abs(K.conj().T @ K - N * np.eye(N)).max() < 1e-10 * N


@pytest.mark.parametrize("d,n", [(1, 64), (2, 8)])
def test_dft_scaled_unitary(d, n):
    """sqrt(N) F is unitary: N F F^* = I (section 1 normalisation 1/n^d)."""
    F = O.dft_matrix(d, n)
    N = n ** d
    assert np.abs(N * F @ F.conj().T - np.eye(N)).max() < 1e-12


def test_dft_matches_library_fft_1d():
    """F f = fft((-1)^k f)/N, since xi_j = j - n/2 (section 1 grids)."""
    n = 128
    f = gaussian_complex(n, 5)
    ref = np.fft.fft(_shift(1, n) * f) / n
    assert np.abs(O.dft(f, 1, n) - ref).max() < 1e-14


def test_dft_matches_library_fft_2d():
    """2D: F f = fft2((-1)^(k1+k2) f)/N with the first coordinate slowest."""
    n = 16
    f = gaussian_complex(n * n, 6)
    ref = np.fft.fft2((_shift(2, n) * f).reshape(n, n)).ravel() / n ** 2
    assert np.abs(O.dft(f, 2, n) - ref).max() < 1e-14
    assert np.abs(O.idft(O.dft(f, 2, n), 2, n) - f).max() < 1e-12


def test_idft_matches_library_ifft():
    """f = n^d F^* fhat = (-1)^(sum k) N ifft(fhat) (section 1 grids), dense and by rows."""
    n = 128
    fh = gaussian_complex(n, 8)
    ref = _shift(1, n) * n * np.fft.ifft(fh)
    assert np.abs(O.idft(fh, 1, n) - ref).max() < 1e-12
    m = 16
    fh2 = gaussian_complex(m * m, 9)
    ref2 = _shift(2, m) * (m * m) * np.fft.ifft2(fh2.reshape(m, m)).ravel()
    assert np.abs(O.idft(fh2, 2, m) - ref2).max() < 1e-12


@pytest.mark.parametrize("d,n", [(1, 65536), (2, 256)])
def test_idft_rows_at_full_size(d, n):
    """The row-by-row inverse DFT at N = 65536 against the library FFT closed form."""
    N = n ** d
    fh = gaussian_complex((N, 2), 10 + d)
    rows = np.array([0, 1, 777, N // 2, N - 1])
    got = O.idft_rows(fh, d, n, rows)
    if d == 1:
        full = _shift(1, n)[:, None] * N * np.fft.ifft(fh, axis=0)
    else:
        full = _shift(2, n)[:, None] * N * np.fft.ifft2(fh.reshape(n, n, 2), axes=(0, 1)).reshape(N, 2)
    assert np.abs(got - full[rows]).max() / np.abs(full[rows]).max() < 1e-11


def _row_closed_form_1d(n, c, fhat, i):
    """(K fhat)_i when row i has constant c: N F^*(e^{2 pi i c|xi|} fhat) via ifft."""
    xi = np.arange(n) - n // 2
    g = np.exp(2j * np.pi * c * np.abs(xi)) * fhat
    return ((-1.0) ** i * n * np.fft.ifft(g))[i]


def test_constant_c_phase_closed_form():
    """Phi = x xi + c|xi|: K = N F^* diag(e^{2 pi i c |xi|}) (pins |xi| and offsets)."""
    n, c = 256, 0.37
    p = O.OracleProblem(1, n, "1d_const", c)
    fh = gaussian_complex(n, 7)
    xi = np.arange(n) - n // 2
    ref = (-1.0) ** np.arange(n) * n * np.fft.ifft(np.exp(2j * np.pi * c * np.abs(xi)) * fh)
    assert np.abs(O.dense_K(p) @ fh - ref).max() < 1e-10
    assert np.abs(O.apply_direct(p, fh) - ref).max() < 1e-10


@pytest.mark.parametrize("c_div", [8.0, 16.0])
def test_example1_rows_reduce_to_fft(c_div):
    """Example 1 (section 6): row i of K is the constant-c operator with
    c = c(x_i) = (2 + sin 2 pi x_i)/c_div, so (K fhat)_i has an FFT closed form."""
    n = 256
    p = O.OracleProblem(1, n, "1d_ex1", c_div)
    fh = gaussian_complex(n, 8)
    rows = np.array([0, 1, 37, 64, 128, 192, 255])
    dense = O.dense_K(p) @ fh
    direct = O.apply_direct(p, fh, out_idx=rows)
    for t, i in enumerate(rows):
        ci = (2.0 + np.sin(2 * np.pi * i / n)) / c_div
        ref = _row_closed_form_1d(n, ci, fh, i)
        assert abs(dense[i] - ref) < 1e-10
        assert abs(direct[t] - ref) < 1e-10


def test_example3_rows_reduce_to_fft2():
    """Example 3 (section 6): for fixed x, phi = sqrt(c1^2 xi1^2 + c2^2 xi2^2) is a
    diagonal multiplier in xi, so (K fhat)_i is a 2D inverse FFT entry."""
    n = 16
    p = O.OracleProblem(2, n, "2d_radon", 16.0)
    fh = gaussian_complex(n * n, 9)
    xi = np.arange(n) - n // 2
    X1, X2 = np.meshgrid(xi, xi, indexing="ij")
    dense = O.dense_K(p) @ fh
    rows = np.array([0, 5, 17, 100, 255])
    direct = O.apply_direct(p, fh, out_idx=rows)
    for t, i in enumerate(rows):
        k1, k2 = divmod(int(i), n)
        x1, x2 = k1 / n, k2 / n
        c1 = (2 + np.sin(2 * np.pi * x1) * np.sin(2 * np.pi * x2)) / 16
        c2 = (2 + np.cos(2 * np.pi * x1) * np.cos(2 * np.pi * x2)) / 16
        w = np.exp(2j * np.pi * np.sqrt(c1 ** 2 * X1 ** 2 + c2 ** 2 * X2 ** 2))
        g = (w.ravel() * fh).reshape(n, n)
        full = n * n * np.fft.ifft2(g).ravel() * _shift(2, n)
        assert abs(dense[i] - full[i]) < 1e-10
        assert abs(direct[t] - full[i]) < 1e-10


@pytest.mark.parametrize("phase,d,n", [("1d_ex1", 1, 128), ("2d_radon", 2, 12)])
def test_normal_matrix_hermitian_positive_definite(phase, d, n):
    """S = K^*K is Hermitian positive definite (section 3, eq_normal_discr)."""
    K = O.dense_K(O.OracleProblem(d, n, phase, 16.0))
    S = K.conj().T @ K
    assert np.abs(S - S.conj().T).max() < 1e-10 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0.1 * K.shape[0]


@pytest.mark.parametrize("phase,d,n", [("1d_ex1", 1, 512), ("1d_ex2", 1, 512), ("2d_radon", 2, 16)])
def test_direct_sum_adjoint_identity(phase, d, n):
    """<K x, y> = <x, K^* y> for the direct-summation forward and adjoint."""
    p = O.OracleProblem(d, n, phase, 16.0)
    x = gaussian_complex(p.N, 10)
    y = gaussian_complex(p.N, 11)
    lhs = np.vdot(y, O.apply_direct(p, x))
    rhs = np.vdot(O.apply_direct(p, y, adjoint=True), x)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_solves_recover_generator_truth():
    """fhat = F f, u = K fhat; LU and Cholesky on K^*K (section 5) recover f."""
    n = 256
    p = O.OracleProblem(1, n, "1d_ex1", 16.0)
    f = gaussian_complex((n, 3), 1000)
    fh = O.dft(f, 1, n)
    K = O.dense_K(p)
    u = K @ fh
    x_lu = O.solve_dense(p, u, K)
    x_ch = O.solve_normal_cholesky(p, u, K)
    assert O.rel_err(x_lu, fh).max() < 1e-13
    assert O.rel_err(x_ch, fh).max() < 1e-12
    assert O.rel_err(O.idft(x_lu, 1, n), f).max() < 1e-13


def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "paper_cg_counts.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            d, n, phase, c_div, count = line.split()[:5]
            rows.append((int(d), int(n), phase, float(c_div), int(count)))
    return rows


@pytest.mark.parametrize("d,n,phase,c_div,count", _golden_counts())
def test_unpreconditioned_cg_counts_match_paper(d, n, phase, c_div, count):
    """The paper's CG counts without the approximate inverse (section 6 tables)
    depend only on K: they pin the discretisation, phase and stopping rule.
    The paper's right-hand side is unstated, so one iteration of slack is allowed."""
    p = O.OracleProblem(d, n, phase, c_div)
    K = O.dense_K(p)
    for seed in (20, 21):
        b = gaussian_complex(p.N, seed)
        _, its = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, b, tol=1e-8)
        assert abs(its - count) <= 1, (its, count)


def test_cg_count_distinguishes_config_phase():
    """The configuration phase (c divided by 16) is better conditioned than the
    paper's Example 1 (c/8): 12 CG iterations instead of 28 at N = 1024."""
    p = O.OracleProblem(1, 1024, "1d_ex1", 16.0)
    K = O.dense_K(p)
    _, its = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v,
                         gaussian_complex(1024, 20), tol=1e-8)
    assert its < 20


def _ex1_c8(n=256):
    p = O.OracleProblem(1, n, "1d_ex1", 8.0)
    return O.dense_K(p)


def test_pcg_with_exact_inverse_stops_after_one_iteration():
    """Preconditioned branch of cg_normal (section 5): with M = (K^*K)^{-1} the
    first search direction is the exact solution, so one iteration solves K^*K x =
    K^*b to rounding and the iteration stops there."""
    K = _ex1_c8()
    S = K.conj().T @ K
    Sinv = np.linalg.inv(S)
    b = gaussian_complex(K.shape[0], 40)
    x, its = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, b, tol=1e-8,
                         precond=lambda r: Sinv @ r)
    assert its == 1
    assert O.rel_err(x, np.linalg.solve(K, b)).max() < 1e-10


def test_pcg_with_scaled_identity_has_the_iterates_of_cg():
    """M = c I changes neither the step lengths nor the directions of CG: the
    preconditioned branch with c = 7.5 returns the iterate of the plain branch
    after the same number of iterations (and for a fixed iteration cap)."""
    K = _ex1_c8()
    b = gaussian_complex(K.shape[0], 41)
    aK, aKH = (lambda v: K @ v), (lambda v: K.conj().T @ v)
    for cap, tol in ((5, 0.0), (1000, 1e-8)):
        x0, i0 = O.cg_normal(aK, aKH, b, tol=tol, maxit=cap)
        x1, i1 = O.cg_normal(aK, aKH, b, tol=tol, maxit=cap, precond=lambda r: 7.5 * r)
        assert i0 == i1
        assert O.rel_err(x1, x0).max() < 1e-10


def test_pcg_equals_cg_on_the_split_preconditioned_system():
    """PCG with M = D^2 (D diagonal, positive) is CG on (K D)^*(K D) y = (K D)^* b
    with x = D y, a textbook identity of split preconditioning: the preconditioned
    branch must reproduce, iterate by iterate, the plain branch (pinned by the
    paper's counts) run on the transformed operator."""
    K = _ex1_c8()
    n = K.shape[0]
    rng = np.random.default_rng(42)
    dg = np.exp(rng.uniform(-1.0, 1.0, n))
    b = gaussian_complex(n, 43)
    for cap in (1, 2, 3, 6):
        x, i = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, b, tol=0.0, maxit=cap,
                           precond=lambda r: dg ** 2 * r)
        y, j = O.cg_normal(lambda v: K @ (dg * v), lambda v: dg * (K.conj().T @ v), b, tol=0.0, maxit=cap)
        assert i == j == cap
        assert O.rel_err(x, dg * y).max() < 1e-9
    x, i = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, b, tol=1e-8,
                       precond=lambda r: dg ** 2 * r)
    assert O.rel_err(x, np.linalg.solve(K, b)).max() < 1e-6


def test_example2_single_term_is_separable():
    """One Gaussian term factors, a(x, xi) = g(x) h(xi), so K = diag(g) K_1 diag(h)
    with K_1 Example 1's operator: rows reduce to the FFT closed form.  Pins the
    periodic distance in x, the xi/n scaling and sigma2."""
    n, x0, e0, s2 = 256, 0.9, 0.15, 0.07
    p = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=((x0, e0),), sigma2=s2)
    fh = gaussian_complex(n, 12)
    nu = (np.arange(n) - n // 2) / n
    h = np.exp(-(nu - e0) ** 2 / s2)
    rows = np.array([0, 3, 100, 128, 230, 255])
    dense = O.dense_K(p) @ fh
    direct = O.apply_direct(p, fh, out_idx=rows)
    for t, i in enumerate(rows):
        x = i / n
        dx = min(abs(x - x0), 1 - abs(x - x0))
        g = np.exp(-dx ** 2 / s2)
        ci = (2.0 + np.sin(2 * np.pi * x)) / 16.0
        ref = g * _row_closed_form_1d(n, ci, h * fh, i)
        assert abs(dense[i] - ref) < 1e-10 * max(1.0, abs(ref))
        assert abs(direct[t] - ref) < 1e-10 * max(1.0, abs(ref))


def test_example2_mixture_is_additive_and_real():
    """The mixture is a sum over its terms, and a is real: K(A u B) = K(A) + K(B)
    and |K_ij| = a(x_i, xi_j)."""
    n = 128
    A, B = ((0.2, -0.2),), ((0.5, 0.2), (0.8, 0.0))
    pa = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=A, sigma2=0.1)
    pb = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=B, sigma2=0.1)
    pab = O.OracleProblem(1, n, "1d_ex2", 16.0, amp=A + B, sigma2=0.1)
    Kab = O.dense_K(pab)
    assert np.abs(Kab - O.dense_K(pa) - O.dense_K(pb)).max() < 1e-12
    idx = np.arange(n)
    assert np.abs(np.abs(Kab) - O.amplitude(pab, idx, idx)).max() < 1e-12


def test_example2_adjoint_is_a_poor_preconditioner():
    """Section 6, Example 2: with a variable amplitude K^* no longer approximates
    K^{-1}; CG on K^*K needs on the order of a hundred iterations (sigma2 = 0.1)
    and more than a thousand (sigma2 = 0.05) at N = 1024, against 12 for a = 1."""
    counts = []
    for s2 in (0.1, 0.05):
        p = O.OracleProblem(1, 1024, "1d_ex2", 16.0, sigma2=s2)
        K = O.dense_K(p)
        _, its = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v,
                             gaussian_complex(1024, 20), tol=1e-8, maxit=5000)
        counts.append(its)
    assert 100 <= counts[0] <= 400, counts
    assert counts[1] > 1000, counts
