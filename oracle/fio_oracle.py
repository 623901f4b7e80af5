"""Oracle implementation (test infrastructure; see the package docstring).

Every function cites the passage of the paper it follows.  Floating point is
FP64 throughout (complex128).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

__all__ = [
    "OracleProblem", "grid", "phase_mod1", "amplitude", "dense_K", "dft_matrix", "dft",
    "idft", "idft_rows", "apply_direct", "forward", "adjoint", "solve_dense",
    "solve_normal_cholesky", "cg_normal", "rel_err", "build_c", "PHASE_IDS",
]

PHASE_IDS = {"linear": 0, "1d_ex1": 1, "2d_radon": 2, "1d_const": 3, "1d_ex2": 4}
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_direct_sum.so")
_lib = None


@dataclasses.dataclass(frozen=True)
class OracleProblem:
    """A discrete FIO of the section 6 examples.

    phase:  "linear"   Phi = x.xi                              (identity checks)
            "1d_ex1"   Phi = x xi + c(x)|xi|, c = (2 + sin 2 pi x)/param  (Example 1)
            "1d_ex2"   Example 1's phase with the amplitude below          (Example 2)
            "2d_radon" Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2)       (Example 3)
            "1d_const" Phi = x xi + param |xi|                  (closed-form pin)
    param:  the divisor of c (Examples 1 and 3) or the constant c of "1d_const".
    amp, sigma2: Example 2's amplitude, a Gaussian mixture periodic in x,
            a(x, xi) = sum_k exp(-(d(x, x_k)^2 + (xi/n - eta_k)^2) / sigma2),
            d the distance on the unit circle, amp = ((x_k, eta_k), ...).  The
            paper gives neither the centres nor their number; these defaults are
            a choice made here.  a = 1 for the other phases.
    """
    d: int
    n: int
    phase: str
    param: float = 16.0
    amp: tuple = ((0.2, -0.2), (0.5, 0.2), (0.8, 0.0))
    sigma2: float = 0.1

    @property
    def N(self) -> int:
        return self.n ** self.d


def grid(d: int, n: int):
    """Integer coordinates of X and Omega (section 1, eq:X_domain, eq:freq_domain).

    Returns (k, xi), each of shape (N, d): x = k/n with 0 <= k < n and
    xi with -n/2 <= xi < n/2.  Points are lexicographic, first coordinate slowest.
    """
    if n % 2:
        raise ValueError("n must be even (section 1)")
    k1 = np.arange(n, dtype=np.int64)
    j1 = np.arange(n, dtype=np.int64) - n // 2
    if d == 1:
        return k1[:, None], j1[:, None]
    a, b = np.meshgrid(k1, k1, indexing="ij")
    c, e = np.meshgrid(j1, j1, indexing="ij")
    k = np.stack([a.ravel(), b.ravel()], axis=1)
    xi = np.stack([c.ravel(), e.ravel()], axis=1)
    return k, xi


def amplitude(prob: OracleProblem, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """a(x_rows, xi_cols) as a (len(rows), len(cols)) array (Example 2; 1 otherwise)."""
    rows, cols = np.asarray(rows), np.asarray(cols)
    if prob.phase != "1d_ex2":
        return np.ones((rows.size, cols.size))
    k, xi = grid(prob.d, prob.n)
    x = k[rows, 0] / prob.n
    nu = xi[cols, 0] / prob.n
    a = np.zeros((rows.size, cols.size))
    for xk, ek in prob.amp:
        dx = np.abs(x - xk) % 1.0
        dx = np.minimum(dx, 1.0 - dx)
        a += np.exp(-(dx[:, None] ** 2 + (nu[None, :] - ek) ** 2) / prob.sigma2)
    return a


def _nonlinear(prob: OracleProblem, x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """phi(x, xi) of the examples in section 6 (x, xi broadcast against each other)."""
    if prob.phase == "linear":
        return np.zeros(np.broadcast_shapes(x.shape[:-1], xi.shape[:-1]))
    if prob.phase in ("1d_ex1", "1d_ex2"):
        c = (2.0 + np.sin(2 * np.pi * x[..., 0])) / prob.param
        return c * np.abs(xi[..., 0])
    if prob.phase == "1d_const":
        return prob.param * np.abs(xi[..., 0]) + 0.0 * x[..., 0]
    if prob.phase == "2d_radon":
        s1, s2 = np.sin(2 * np.pi * x[..., 0]), np.sin(2 * np.pi * x[..., 1])
        o1, o2 = np.cos(2 * np.pi * x[..., 0]), np.cos(2 * np.pi * x[..., 1])
        c1 = (2.0 + s1 * s2) / prob.param
        c2 = (2.0 + o1 * o2) / prob.param
        return np.sqrt(c1 ** 2 * xi[..., 0] ** 2 + c2 ** 2 * xi[..., 1] ** 2)
    raise ValueError(prob.phase)


def phase_mod1(prob: OracleProblem, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Phi(x_rows, xi_cols) mod 1, as a (len(rows), len(cols)) array.

    The linear part x.xi = (sum_d k_d xi_d)/n is reduced exactly in integers;
    the nonlinear part is reduced mod 1 in FP64 (section 6: Phi = x.xi + phi).
    """
    k, xi = grid(prob.d, prob.n)
    kr = k[rows][:, None, :]
    xc = xi[cols][None, :, :]
    lin = np.mod((kr * xc).sum(axis=-1), prob.n) / prob.n
    nl = _nonlinear(prob, kr.astype(np.float64) / prob.n, xc.astype(np.float64))
    t = lin + (nl - np.floor(nl))
    return t - np.floor(t)


def dense_K(prob: OracleProblem) -> np.ndarray:
    """K_ij = a(x_i, xi_j) exp(2 pi i Phi(x_i, xi_j)) (section 1, eq6)."""
    idx = np.arange(prob.N)
    return amplitude(prob, idx, idx) * np.exp(2j * np.pi * phase_mod1(prob, idx, idx))


def dft_matrix(d: int, n: int) -> np.ndarray:
    """F with F_jk = n^{-d} exp(-2 pi i x_k . xi_j) (section 1): fhat = F f."""
    k, xi = grid(d, n)
    t = np.mod((xi[:, None, :] * k[None, :, :]).sum(axis=-1), n) / n
    return np.exp(-2j * np.pi * t) / float(n ** d)


def dft(f: np.ndarray, d: int, n: int) -> np.ndarray:
    """fhat = F f by the dense definition (section 1)."""
    return dft_matrix(d, n) @ f


def idft(fhat: np.ndarray, d: int, n: int) -> np.ndarray:
    """f = F^{-1} fhat = n^d F^* fhat (the normalised DFT has F^{-1} = n^d F^*)."""
    return float(n ** d) * (dft_matrix(d, n).conj().T @ fhat)


def idft_rows(fhat: np.ndarray, d: int, n: int, rows) -> np.ndarray:
    """Selected entries f[rows] of f = n^d F^* fhat, each summed by the definition
    f_k = sum_j exp(2 pi i x_k . xi_j) fhat_j (section 1); for sizes where the dense
    F does not fit.  The exponent is reduced exactly in integers, as in dft_matrix."""
    k, xi = grid(d, n)
    kk = k[np.asarray(rows)]
    t = np.mod((kk[:, None, :] * xi[None, :, :]).sum(axis=-1), n) / n
    return np.exp(2j * np.pi * t) @ fhat


def build_c(force: bool = False) -> str:
    """Compile the direct-summation oracle (plain C, OpenMP)."""
    src = os.path.join(_HERE, "direct_sum.c")
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_c()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_fio_apply.restype = ctypes.c_int
        lib.oracle_fio_apply.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_double]
        _lib = lib
    return _lib


def apply_direct(prob: OracleProblem, v: np.ndarray, adjoint: bool = False,
                 out_idx=None, nthreads: int = 0) -> np.ndarray:
    """K v (or K^* v) by direct summation in C (section 1, eq3), any N.

    v has shape (N,) or (N, B).  If out_idx is given, only those output
    entries are computed (rows of K v, or rows of K^* v).
    """
    lib = _load()
    vec = v.ndim == 1
    V = np.asfortranarray(v.reshape(prob.N, -1).astype(np.complex128))
    B = V.shape[1]
    if out_idx is None:
        n_out, idx_ptr, idx = prob.N, None, None
    else:
        idx = np.ascontiguousarray(np.asarray(out_idx, dtype=np.int64))
        n_out, idx_ptr = idx.size, idx.ctypes.data
    out = np.zeros((n_out, B), dtype=np.complex128, order="F")
    amp = np.ascontiguousarray(np.asarray(prob.amp, dtype=np.float64).reshape(-1, 2))
    rc = lib.oracle_fio_apply(prob.d, prob.n, PHASE_IDS[prob.phase], float(prob.param),
                              1 if adjoint else 0, B, V.ctypes.data, out.ctypes.data,
                              idx_ptr, n_out, int(nthreads), amp.shape[0], amp.ctypes.data,
                              float(prob.sigma2))
    if rc != 0:
        raise ValueError("oracle_fio_apply rejected its arguments")
    return out[:, 0] if vec else out


def forward(prob: OracleProblem, fhat: np.ndarray) -> np.ndarray:
    """u = K fhat (section 1, eq6): dense product for N <= 4096, else direct sum."""
    if prob.N <= 4096:
        return dense_K(prob) @ fhat
    return apply_direct(prob, fhat)


def adjoint(prob: OracleProblem, u: np.ndarray) -> np.ndarray:
    """K^* u (section 3, eq_adj discretised)."""
    if prob.N <= 4096:
        return dense_K(prob).conj().T @ u
    return apply_direct(prob, u, adjoint=True)


def solve_dense(prob: OracleProblem, u: np.ndarray, K: np.ndarray | None = None) -> np.ndarray:
    """fhat = K^{-1} u by LU with partial pivoting (LAPACK through NumPy)."""
    if K is None:
        K = dense_K(prob)
    return np.linalg.solve(K, u)


def solve_normal_cholesky(prob: OracleProblem, u: np.ndarray,
                          K: np.ndarray | None = None) -> np.ndarray:
    """fhat = (K^*K)^{-1} K^* u (section 5, eq:pseudoinv) by Cholesky of K^*K."""
    if K is None:
        K = dense_K(prob)
    S = K.conj().T @ K
    C = np.linalg.cholesky(S)          # S = C C^*
    y = np.linalg.solve(C, K.conj().T @ u)
    return np.linalg.solve(C.conj().T, y)


def cg_normal(apply_K, apply_KH, b: np.ndarray, tol: float = 1e-8, maxit: int = 1000,
              precond=None):
    """Conjugate gradients on K^*K x = K^* b, x0 = 0 (section 6, eq_NR_1).

    Stops when the residual of the normal equations satisfies
    ||K^*b - K^*K x|| <= tol ||K^*b||.  Returns (x, iterations).  With
    ``precond`` (a callable M^{-1} r) this is preconditioned CG (section 5).
    """
    rhs = apply_KH(b)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = precond(r) if precond else r
    p = z.copy()
    rz = np.vdot(r, z)
    nb = np.linalg.norm(rhs)
    for it in range(1, maxit + 1):
        Ap = apply_KH(apply_K(p))
        alpha = rz / np.vdot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = precond(r) if precond else r
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def rel_err(x: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-column relative 2-norm error ||x - ref|| / ||ref||."""
    x = x.reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)
