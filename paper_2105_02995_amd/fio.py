"""ctypes binding of libfio.so: the C ABI of include/fio.h with the same names.

Argument marshalling only.  Vector arguments may be torch tensors (their device
pointer is passed) or raw integer device addresses.  Every computation happens
in the library's HIP kernels; if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfio.so")

FIO_OK = 0
STATUS = {0: "FIO_OK", 1: "FIO_ERR_ARG", 2: "FIO_ERR_NOMEM", 3: "FIO_ERR_DEVICE",
          4: "FIO_ERR_NOT_HPD", 5: "FIO_ERR_NOT_CONVERGED", 6: "FIO_ERR_UNSUPPORTED",
          7: "FIO_ERR_IO"}
FIO_C64, FIO_C128 = 0, 1
FIO_OP_K, FIO_OP_KH = 0, 1
FIO_PHASE_LINEAR, FIO_PHASE_1D_EX1, FIO_PHASE_2D_RADON, FIO_PHASE_1D_EX2 = 0, 1, 2, 3
FIO_PHASE_CALLBACK = 4
FIO_MAX_AMP_TERMS = 8
FIO_SOLVE_DIRECT, FIO_SOLVE_REFINE, FIO_SOLVE_PCG, FIO_SOLVE_GMRES = 0, 1, 2, 3
PHASES = {"linear": FIO_PHASE_LINEAR, "1d_ex1": FIO_PHASE_1D_EX1, "2d_radon": FIO_PHASE_2D_RADON,
          "1d_ex2": FIO_PHASE_1D_EX2, "callback": FIO_PHASE_CALLBACK}

# fio_phase_fn and fio_amp_fn of fio.h
PHASE_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                            ctypes.c_int, ctypes.c_void_p)
AMP_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double))

EXPORTS = ["fio_build", "fio_apply", "fio_inverse_dft", "fio_stage_apply", "fio_stage_pair_apply", "fio_stage_pair_apply_variant", "fio_stage_triple_apply", "fio_stage_apply_variant", "fio_chain_schedule", "fio_inverse_apply", "fio_inverse_apply_noalloc", "fio_solve_multi", "fio_multi_autotune", "fio_gd_apply", "fio_gd_apply_variant", "fio_solve",
           "fio_autotune", "fio_tune_query",
           "fio_plan_stats", "fio_plan_fingerprints", "fio_plan_trim", "fio_stage_info", "fio_save", "fio_load", "fio_destroy",
           "fio_last_error", "fio_set_trace", "fio_column_id"]


class FioError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class fio_problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("phase", ctypes.c_int),
                ("c_div", ctypes.c_double), ("eps", ctypes.c_double),
                ("eps_bf", ctypes.c_double), ("eps_peel", ctypes.c_double),
                ("eps_hif", ctypes.c_double), ("leaf_bf", ctypes.c_int),
                ("leaf_h", ctypes.c_int), ("oversample", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("device", ctypes.c_int), ("nthreads", ctypes.c_int),
                ("verbose", ctypes.c_int), ("amp_sigma2", ctypes.c_double), ("amp_terms", ctypes.c_int),
                ("amp_x", ctypes.c_double * FIO_MAX_AMP_TERMS), ("amp_eta", ctypes.c_double * FIO_MAX_AMP_TERMS),
                ("strict_hpd", ctypes.c_int), ("host_construction", ctypes.c_int),
                ("prescale_skel", ctypes.c_int), ("phi", PHASE_FN), ("amp_fn", AMP_FN),
                ("user", ctypes.c_void_p),
                ("bf_rank_align", ctypes.c_int)]


class fio_solve_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("precondition", ctypes.c_int), ("spatial", ctypes.c_int), ("restart", ctypes.c_int)]


class fio_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_resid", ctypes.c_double), ("est_rel_err", ctypes.c_double)]


class fio_plan_stats_t(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("L", ctypes.c_int),
                ("L_mid", ctypes.c_int), ("n_stages", ctypes.c_int),
                ("bf_nnz", ctypes.c_int64), ("max_rank_bf", ctypes.c_int),
                ("hif_levels", ctypes.c_int), ("hif_nnz", ctypes.c_int64),
                ("root_size", ctypes.c_int), ("max_rank_h", ctypes.c_int),
                ("device_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("hif_shifted", ctypes.c_int),
                ("bf_seconds", ctypes.c_double), ("bf_device_levels", ctypes.c_int),
                ("hif_device_ids", ctypes.c_int), ("hif_device_nodes", ctypes.c_int),
                ("e_a_est", ctypes.c_double), ("e_s_est", ctypes.c_double), ("cond_est", ctypes.c_double),
                ("hif_sweep_nnz", ctypes.c_int64)]


_lib = None


def load_library():
    """Load libfio.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfio.so is not built; run paper_2105_02995_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, VP = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    lib.fio_build.argtypes = [ctypes.POINTER(fio_problem), ctypes.POINTER(P)]
    lib.fio_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, VP, VP, I64, I64, VP]
    lib.fio_stage_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, VP, VP, I64, VP]
    lib.fio_stage_apply_variant.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, VP, VP, I64,
                                            VP]
    lib.fio_stage_pair_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, VP, VP, I64, VP]
    lib.fio_column_id.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, VP, ctypes.c_int64, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_int), VP, VP, ctypes.c_int64]
    lib.fio_stage_pair_apply_variant.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, VP, VP,
                                                 I64, VP]
    lib.fio_stage_triple_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, VP, VP, I64, VP]
    IP = ctypes.POINTER(ctypes.c_int)
    lib.fio_chain_schedule.argtypes = [P, ctypes.c_int, ctypes.c_int, I64, ctypes.c_int, IP, IP, IP, IP]
    lib.fio_autotune.argtypes = [P, ctypes.c_int, I64, ctypes.c_int, VP]
    lib.fio_tune_query.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, I64,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.fio_inverse_apply.argtypes = [P, ctypes.c_int, VP, VP, I64, I64, VP]
    lib.fio_inverse_apply_noalloc.argtypes = [P, ctypes.c_int, VP, VP, I64, I64, VP]
    lib.fio_solve_multi.argtypes = [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(fio_solve_opts), ctypes.c_int,
                                    ctypes.POINTER(VP), ctypes.POINTER(VP), ctypes.POINTER(I64),
                                    ctypes.POINTER(I64), VP]
    lib.fio_multi_autotune.argtypes = [ctypes.c_int, ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(I64),
                                       ctypes.c_int, VP]
    lib.fio_gd_apply.argtypes = [P, ctypes.c_int, VP, VP, I64, I64, VP]
    lib.fio_gd_apply_variant.argtypes = [P, ctypes.c_int, ctypes.c_int, VP, VP, I64, I64, VP]
    lib.fio_inverse_dft.argtypes = [P, VP, VP, I64, I64, VP]
    lib.fio_solve.argtypes = [P, ctypes.POINTER(fio_solve_opts), ctypes.c_int, VP, VP, I64, I64,
                              ctypes.POINTER(fio_solve_info), VP]
    lib.fio_plan_stats.argtypes = [P, ctypes.POINTER(fio_plan_stats_t)]
    lib.fio_plan_trim.argtypes = [P, ctypes.c_int]
    lib.fio_plan_fingerprints.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]
    lib.fio_stage_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
    lib.fio_save.argtypes = [P, ctypes.c_char_p]
    lib.fio_load.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(P)]
    lib.fio_destroy.argtypes = [P]
    lib.fio_destroy.restype = None
    lib.fio_set_trace.argtypes = [ctypes.c_int]
    lib.fio_set_trace.restype = None
    lib.fio_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("fio_destroy", "fio_last_error", "fio_set_trace"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != FIO_OK:
        raise FioError(rc, load_library().fio_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Plan:
    """Owner of a fio_plan handle."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            load_library().fio_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_problem(d, n, phase="1d_ex1", eps=1e-6, c_div=16.0, device=0, **kw) -> fio_problem:
    p = fio_problem()
    p.d, p.n = d, n
    p.phase = PHASES[phase] if isinstance(phase, str) else int(phase)
    p.c_div, p.eps, p.device = c_div, eps, device
    amp = kw.pop("amp", None)
    if amp is not None:  # Example 2 centres [(x_k, eta_k), ...]
        if len(amp) > FIO_MAX_AMP_TERMS:
            raise ValueError("at most %d amplitude terms" % FIO_MAX_AMP_TERMS)
        p.amp_terms = len(amp)
        for k, (x, e) in enumerate(amp):
            p.amp_x[k], p.amp_eta[k] = x, e
    # FIO_PHASE_CALLBACK: the caller's phase and amplitude, as C function addresses
    # (ints, e.g. from a compiled library) or Python callables with the signatures of
    # fio_phase_fn / fio_amp_fn (correct but slow: every entry of K the build samples
    # is one Python call).  The wrappers stay alive with the problem.
    phi_fn = kw.pop("phi_fn", None)
    amp_fn = kw.pop("amp_fn", None)
    keep = []
    if phi_fn is not None:
        p.phi = ctypes.cast(phi_fn, PHASE_FN) if isinstance(phi_fn, int) else PHASE_FN(phi_fn)
        keep.append(p.phi)
    if amp_fn is not None:
        p.amp_fn = ctypes.cast(amp_fn, AMP_FN) if isinstance(amp_fn, int) else AMP_FN(amp_fn)
        keep.append(p.amp_fn)
    fields = {f[0] for f in fio_problem._fields_}
    for k, v in kw.items():
        if k not in fields:  # a ctypes structure would take an unknown name silently
            raise TypeError("fio_problem has no field %r" % k)
        setattr(p, k, v)
    p._keep = keep
    return p


def fio_build(problem: fio_problem) -> Plan:
    h = ctypes.c_void_p()
    _check(load_library().fio_build(ctypes.byref(problem), ctypes.byref(h)))
    return Plan(h)


def fio_load(path: str, device: int = 0) -> Plan:
    h = ctypes.c_void_p()
    _check(load_library().fio_load(path.encode(), device, ctypes.byref(h)))
    return Plan(h)


def fio_save(plan: Plan, path: str):
    _check(load_library().fio_save(plan.handle, path.encode()))


def fio_set_trace(on: bool):
    """Named roctx ranges of the library's phases (for a profiler's marker trace)."""
    load_library().fio_set_trace(1 if on else 0)


def fio_destroy(plan: Plan):
    plan.close()


def fio_apply(plan: Plan, op: int, dtype: int, x, y, nrhs: int, ld: int, stream=None):
    _check(load_library().fio_apply(plan.handle, op, dtype, _ptr(x), _ptr(y), nrhs, ld,
                                    _stream(stream)))


def fio_stage_apply(plan: Plan, op: int, stage: int, dtype: int, x, y, nrhs: int, stream=None):
    _check(load_library().fio_stage_apply(plan.handle, op, stage, dtype, _ptr(x), _ptr(y), nrhs,
                                          _stream(stream)))


def fio_stage_apply_variant(plan: Plan, op: int, stage: int, dtype: int, variant: int, x, y, nrhs: int,
                            stream=None):
    _check(load_library().fio_stage_apply_variant(plan.handle, op, stage, dtype, variant, _ptr(x), _ptr(y), nrhs,
                                                  _stream(stream)))


def fio_stage_pair_apply_variant(plan: Plan, op: int, stage: int, dtype: int, variant: int, x, y, nrhs: int,
                                 stream=None):
    _check(load_library().fio_stage_pair_apply_variant(plan.handle, op, stage, dtype, variant, _ptr(x), _ptr(y),
                                                       nrhs, _stream(stream)))


def fio_stage_triple_apply(plan: Plan, op: int, stage: int, dtype: int, x, y, nrhs: int, stream=None):
    _check(load_library().fio_stage_triple_apply(plan.handle, op, stage, dtype, _ptr(x), _ptr(y), nrhs,
                                                 _stream(stream)))


def fio_column_id(A, tol_rel: float, device: int = 0):
    """Device column ID of a host complex128 matrix: (skel, redund, T) with
    A[:, redund] ~= A[:, skel] @ T."""
    import numpy as np
    A = np.asfortranarray(np.asarray(A, dtype=np.complex128))
    m, n = A.shape
    rank = ctypes.c_int()
    perm = np.zeros(n, dtype=np.int32)
    T = np.zeros(max(1, (n * n) // 4 + n), dtype=np.complex128)
    _check(load_library().fio_column_id(device, m, n, A.ctypes.data, m, tol_rel, ctypes.byref(rank),
                                        perm.ctypes.data, T.ctypes.data, T.size))
    k = rank.value
    return perm[:k].copy(), perm[k:].copy(), T[:k * (n - k)].reshape(n - k, k).T.copy() if k * (n - k) else \
        np.zeros((k, n - k), dtype=np.complex128)


def fio_stage_pair_apply(plan: Plan, op: int, stage: int, dtype: int, x, y, nrhs: int, stream=None):
    _check(load_library().fio_stage_pair_apply(plan.handle, op, stage, dtype, _ptr(x), _ptr(y), nrhs,
                                               _stream(stream)))


def fio_chain_schedule(plan: Plan, op: int, dtype: int, nrhs: int) -> list:
    """Launches of a chain apply: list of (first_stage, n_stages, variant)."""
    lib = load_library()
    n = ctypes.c_int()
    _check(lib.fio_chain_schedule(plan.handle, op, dtype, nrhs, 0, ctypes.byref(n), None, None, None))
    a, b, c = (ctypes.c_int * max(1, n.value))(), (ctypes.c_int * max(1, n.value))(), (ctypes.c_int * max(1, n.value))()
    _check(lib.fio_chain_schedule(plan.handle, op, dtype, nrhs, n.value, ctypes.byref(n), a, b, c))
    return [(a[j], b[j], c[j]) for j in range(n.value)]


def fio_autotune(plan: Plan, dtype: int, nrhs: int, reps: int = 3, stream=None):
    _check(load_library().fio_autotune(plan.handle, dtype, nrhs, reps, _stream(stream)))


def fio_tune_query(plan: Plan, op: int, stage: int, dtype: int, nrhs: int) -> int:
    v = ctypes.c_int()
    _check(load_library().fio_tune_query(plan.handle, op, stage, dtype, nrhs, ctypes.byref(v)))
    return v.value


def fio_inverse_apply(plan: Plan, dtype: int, u, fhat, nrhs: int, ld: int, stream=None):
    _check(load_library().fio_inverse_apply(plan.handle, dtype, _ptr(u), _ptr(fhat), nrhs, ld,
                                            _stream(stream)))


def fio_inverse_apply_noalloc(plan: Plan, dtype: int, u, fhat, nrhs: int, ld: int, stream=None):
    """fio_inverse_apply with its temporaries in the library's static scratch array."""
    _check(load_library().fio_inverse_apply_noalloc(plan.handle, dtype, _ptr(u), _ptr(fhat), nrhs, ld,
                                                    _stream(stream)))


def fio_inverse_dft(plan: Plan, fhat, f, nrhs: int, ld: int, stream=None):
    _check(load_library().fio_inverse_dft(plan.handle, _ptr(fhat), _ptr(f), nrhs, ld, _stream(stream)))


def fio_gd_apply(plan: Plan, dtype: int, x, y, nrhs: int, ld: int, stream=None):
    _check(load_library().fio_gd_apply(plan.handle, dtype, _ptr(x), _ptr(y), nrhs, ld,
                                       _stream(stream)))


def fio_gd_apply_variant(plan: Plan, dtype: int, variant: int, x, y, nrhs: int, ld: int, stream=None):
    _check(load_library().fio_gd_apply_variant(plan.handle, dtype, variant, _ptr(x), _ptr(y), nrhs, ld,
                                               _stream(stream)))


def fio_solve(plan: Plan, mode: int, dtype: int, u, out, nrhs: int, ld: int, tol: float = 0.0,
              maxit: int = 0, precondition: int = 1, stream=None, want_info: bool = True,
              spatial: int = 0, restart: int = 0, with_estimate: bool = False):
    """Returns (iters, rel_resid), or (iters, rel_resid, est_rel_err) with
    with_estimate, or None without want_info (no synchronisation)."""
    o = fio_solve_opts(mode, tol, maxit, precondition, spatial, restart)
    info = fio_solve_info()
    _check(load_library().fio_solve(plan.handle, ctypes.byref(o), dtype, _ptr(u), _ptr(out), nrhs,
                                    ld, ctypes.byref(info) if (want_info or with_estimate) else None,
                                    _stream(stream)))
    if with_estimate:
        return info.iters, info.rel_resid, info.est_rel_err
    return (info.iters, info.rel_resid) if want_info else None


def fio_solve_multi(plans, mode: int, dtype: int, us, outs, nrhs, lds, maxit: int = 0, stream=None):
    """One pass over several independent solves (one launch per factor level)."""
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    U = (ctypes.c_void_p * n)(*[_ptr(u) for u in us])
    O = (ctypes.c_void_p * n)(*[_ptr(o) for o in outs])
    B = (ctypes.c_int64 * n)(*nrhs)
    L = (ctypes.c_int64 * n)(*lds)
    o = fio_solve_opts(mode, 0.0, maxit, 1, 0, 0)
    _check(load_library().fio_solve_multi(n, P, ctypes.byref(o), dtype, U, O, B, L, _stream(stream)))


def fio_multi_autotune(plans, dtype: int, nrhs, reps: int = 3, stream=None):
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    B = (ctypes.c_int64 * n)(*nrhs)
    _check(load_library().fio_multi_autotune(n, P, dtype, B, reps, _stream(stream)))


FIO_KEEP_ALL, FIO_KEEP_REFINE_C64 = 0, 1


def fio_plan_fingerprints(plan: Plan) -> list:
    lib = load_library()
    n = ctypes.c_int()
    _check(lib.fio_plan_fingerprints(plan.handle, None, 0, ctypes.byref(n)))
    out = (ctypes.c_uint64 * max(n.value, 1))()
    _check(lib.fio_plan_fingerprints(plan.handle, out, n.value, ctypes.byref(n)))
    return list(out[:n.value])


def fio_plan_trim(plan: Plan, keep: int):
    _check(load_library().fio_plan_trim(plan.handle, keep))


def fio_plan_stats(plan: Plan) -> dict:
    s = fio_plan_stats_t()
    _check(load_library().fio_plan_stats(plan.handle, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in s._fields_}


def fio_stage_info(plan: Plan, stage: int) -> dict:
    nnz, nob = ctypes.c_int64(), ctypes.c_int64()
    ro, ri, fan = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().fio_stage_info(plan.handle, stage, ctypes.byref(nnz), ctypes.byref(nob),
                                         ctypes.byref(ro), ctypes.byref(ri), ctypes.byref(fan)))
    return {"nnz": nnz.value, "n_out": nob.value, "r_out": ro.value, "r_in": ri.value,
            "fan": fan.value}
