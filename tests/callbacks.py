"""The test-side callback library (tests/native/fio_callbacks.c): compiled with gcc
on first use, loaded with ctypes, and turned into fio_problem descriptions of the
paper's examples through FIO_PHASE_CALLBACK."""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

from paper_2105_02995_amd import fio as F

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "fio_callbacks.c")


class CbParams(ctypes.Structure):
    _fields_ = [("c_div", ctypes.c_double), ("n", ctypes.c_int), ("terms", ctypes.c_int),
                ("sigma2", ctypes.c_double), ("cx", ctypes.c_double * 8), ("ce", ctypes.c_double * 8)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        out = os.path.join(tempfile.gettempdir(), "fio_callbacks_%d.so" % os.getpid())
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", SRC, "-o", out, "-lm"])
        _lib = ctypes.CDLL(out)
    return _lib


def addr(name: str) -> int:
    return ctypes.cast(getattr(lib(), name), ctypes.c_void_p).value


def problem(example: str, d: int, n: int, eps: float, device: int = 0, sigma2: float = 0.1,
            centres=((0.2, -0.2), (0.5, 0.2), (0.8, 0.0)), **kw):
    """fio_problem of Example 1 ("ex1"), 2 ("ex2") or 3 ("radon") with the phase (and
    amplitude) given by the callback library, c/16."""
    prm = CbParams()
    prm.c_div, prm.n, prm.terms, prm.sigma2 = 16.0, n, len(centres), sigma2
    for k, (x, e) in enumerate(centres):
        prm.cx[k], prm.ce[k] = x, e
    phi = {"ex1": "cb_phase_ex1", "ex2": "cb_phase_ex1", "radon": "cb_phase_radon",
           "bad": "cb_phase_bad"}[example]
    p = F.make_problem(d, n, "callback", eps=eps, device=device, phi_fn=addr(phi),
                       amp_fn=addr("cb_amp_mixture") if example == "ex2" else None,
                       user=ctypes.cast(ctypes.pointer(prm), ctypes.c_void_p), **kw)
    p._keep.append(prm)
    return p
