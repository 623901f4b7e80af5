"""Reader of the library's saved factor files, and NumPy products with the saved
factors, for CPU tests of the host construction (the GPU never runs here).

This is test tooling: it shares nothing with the oracle, and the library never
uses it.
"""
from __future__ import annotations

import struct

import numpy as np


class _Buf:
    def __init__(self, data: bytes):
        self.d, self.o = data, 0

    def take(self, fmt):
        v = struct.unpack_from("<" + fmt, self.d, self.o)
        self.o += struct.calcsize("<" + fmt)
        return v if len(v) > 1 else v[0]

    def arr(self, dtype):
        n = self.take("q")
        a = np.frombuffer(self.d, dtype=dtype, count=n, offset=self.o).copy()
        self.o += a.nbytes
        return a

    def mat(self):
        m, n = self.take("ii")
        a = np.frombuffer(self.d, dtype=np.complex128, count=m * n, offset=self.o).copy()
        self.o += a.nbytes
        return a.reshape(n, m).T  # column-major


def read(path: str) -> dict:
    b = _Buf(open(path, "rb").read())
    assert b.d[:8] == b"FIOPLAN1"
    b.o = 8
    f = {}
    f["d"], f["n"], f["phase"] = b.take("iii")
    f["c_div"], f["eps"], f["eps_bf"], f["eps_peel"], f["eps_hif"] = b.take("ddddd")
    f["leaf_bf"], f["leaf_h"], f["oversample"] = b.take("iii")
    f["seed"] = b.take("Q")
    f["N"] = b.take("q")
    f["L"], f["Lm"], f["m"] = b.take("iii")
    f["perm"] = b.arr(np.int32)
    stages = []
    for _ in range(b.take("i")):
        n_out, n_in = b.take("qq")
        r_out, r_in, fan = b.take("iii")
        idx = b.arr(np.int32).reshape(n_out, fan)
        A = b.arr(np.complex128).reshape(n_out, fan * r_in, r_out).transpose(0, 2, 1)
        stages.append(dict(n_out=n_out, n_in=n_in, r_out=r_out, r_in=r_in, fan=fan, idx=idx, A=A))
    f["stages"] = stages
    b.take("q")
    steps = []
    for _ in range(b.take("i")):
        nodes = []
        for _ in range(b.take("i")):
            ir, is_ = b.arr(np.int32), b.arr(np.int32)
            T, Li, M = b.mat(), b.mat(), b.mat()
            nodes.append(dict(r=ir, s=is_, T=T, Linv=Li, M=M))
        steps.append(nodes)
    f["steps"] = steps
    f["root"] = b.arr(np.int32)
    f["A0inv"] = b.mat()
    f["max_rank_h"] = b.take("i")
    f["build_seconds"] = b.take("d")
    return f


def chain(stages, x):
    """Product of a stage chain with x (rows: first stage's input entries)."""
    cur = x.reshape(-1, x.shape[-1]) if x.ndim > 1 else x[:, None]
    for s in stages:
        xin = cur.reshape(s["n_in"], s["r_in"], -1)
        g = xin[s["idx"]].reshape(s["n_out"], s["fan"] * s["r_in"], -1)
        cur = np.einsum("oak,okb->oab", s["A"], g).reshape(s["n_out"] * s["r_out"], -1)
    return cur if x.ndim > 1 else cur[:, 0]


def adjoint_chain(stages, y):
    """Product of the adjoint of a stage chain with y."""
    cur = y.reshape(-1, y.shape[-1]) if y.ndim > 1 else y[:, None]
    for s in reversed(stages):
        yo = cur.reshape(s["n_out"], s["r_out"], -1)
        contrib = np.einsum("oak,oab->okb", s["A"].conj(), yo).reshape(s["n_out"], s["fan"], s["r_in"], -1)
        out = np.zeros((s["n_in"], s["r_in"], cur.shape[-1]), dtype=np.complex128)
        for q in range(s["fan"]):
            np.add.at(out, s["idx"][:, q], contrib[:, q])
        cur = out.reshape(s["n_in"] * s["r_in"], -1)
    return cur if y.ndim > 1 else cur[:, 0]


def gd(f, x):
    """Gd x = R_L..R_1 A_0^{-1} R_1^*..R_L^* x (x in tree order, one or more columns)."""
    v = x.copy().reshape(x.shape[0], -1)
    for nodes in f["steps"]:
        for nd in nodes:
            r, s = nd["r"], nd["s"]
            xr = v[r] - nd["T"].conj().T @ v[s]
            y = nd["Linv"] @ xr
            v[s] = v[s] - nd["M"] @ y
            v[r] = y
    if f["root"].size:
        v[f["root"]] = f["A0inv"] @ v[f["root"]]
    for nodes in reversed(f["steps"]):
        for nd in nodes:
            r, s = nd["r"], nd["s"]
            t = v[r] - nd["M"].conj().T @ v[s]
            xr = nd["Linv"].conj().T @ t
            v[s] = v[s] - nd["T"] @ xr
            v[r] = xr
    return v.reshape(x.shape)


def to_tree(f, v):
    return v[f["perm"]]


def from_tree(f, v):
    out = np.empty_like(v)
    out[f["perm"]] = v
    return out


def apply_K(f, fhat):
    """Kd fhat in natural order."""
    return from_tree(f, chain(f["stages"], to_tree(f, fhat)))


def apply_KH(f, u):
    return from_tree(f, adjoint_chain(f["stages"], to_tree(f, u)))


def inverse(f, u):
    """Gd Kd^* u in natural order."""
    return from_tree(f, gd(f, adjoint_chain(f["stages"], to_tree(f, u))))
