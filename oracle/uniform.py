"""Uniform H-matrix and H-matrix products by their definitions.  Test infrastructure.

An operator is read through its host layout: a mapping with the keys in
``OPERATOR_KEYS`` whose values are plain numpy arrays (flat complex128 storage, every
per-cluster or per-block matrix column-major at its element offset; ``perm`` maps
cluster position to user index).  Vectors are in user order.

uh_mvp        y = sum_{b=(tau,sigma) in P+} U_tau S_b V_sigma^* x|_sigma
                + sum_{b in P-} A|_b x|_sigma                       (Definition 2.4)
              block by block, recomputing V_sigma^* x|_sigma for every block: nothing is
              shared between blocks, so the sum is the definition written out.
uh_mvp_rows   the same sum restricted to a set of rows (for operators too large for
              uh_mvp to finish quickly; the rows are computed one block at a time).
h_mvp         y = sum_{b in P+} X_b Y_b^* x|_sigma + sum_{b in P-} A|_b x|_sigma
                                                                    (Definition 2.3)
expand_symmetric
              the general image that a symmetric-storage image stands for (Remark 4.4):
              every stored off-diagonal block also gives its mirror, as a transpose.
assemble_factored
              the general image with every coupling formed from its factors,
              S_b = S_{X,b} S_{Y,b}^* (section 4.2).
alg6, alg5    the C implementations of Algorithms 6 and 5 (section 4.4), through ctypes.
optimal_row_basis
              Algorithm 1: the leading left singular vectors of the explicit
              agglomeration matrix A_tau = A|_{tau x F(tau)} (section 4.1).
"""
from __future__ import annotations

import ctypes
import os
from typing import Mapping

import numpy as np

OPERATOR_KEYS = ("n", "perm", "off", "size", "rank_row", "rank_col", "U_off", "V_off", "U", "V",
                 "adm_row", "adm_col", "S_off", "S", "adm_rank", "X_off", "Y_off", "X", "Y",
                 "den_row", "den_col", "D_off", "D")


def _colmajor(flat: np.ndarray, start: int, rows: int, cols: int) -> np.ndarray:
    return flat[start:start + rows * cols].reshape(cols, rows).T


def _basis(op, which: str, c: int) -> np.ndarray:
    rank = op["rank_row"] if which == "U" else op["rank_col"]
    offs = op["U_off"] if which == "U" else op["V_off"]
    return _colmajor(op[which], int(offs[c]), int(op["size"][c]), int(rank[c]))


def _rows_of(op, c: int) -> np.ndarray:
    o = int(op["off"][c])
    return op["perm"][o:o + int(op["size"][c])]


def uh_mvp(op: Mapping, x: np.ndarray) -> np.ndarray:
    n = int(op["n"])
    x2 = np.asarray(x, dtype=np.complex128).reshape(n, -1)
    y = np.zeros_like(x2)
    for b in range(op["adm_row"].shape[0]):
        t, s = int(op["adm_row"][b]), int(op["adm_col"][b])
        lt, ls = int(op["rank_row"][t]), int(op["rank_col"][s])
        Ut, Vs = _basis(op, "U", t), _basis(op, "V", s)
        Sb = _colmajor(op["S"], int(op["S_off"][b]), lt, ls)
        y[_rows_of(op, t)] += Ut @ (Sb @ (Vs.conj().T @ x2[_rows_of(op, s)]))
    for b in range(op["den_row"].shape[0]):
        t, s = int(op["den_row"][b]), int(op["den_col"][b])
        Db = _colmajor(op["D"], int(op["D_off"][b]), int(op["size"][t]), int(op["size"][s]))
        y[_rows_of(op, t)] += Db @ x2[_rows_of(op, s)]
    return y.reshape(np.shape(x))


def uh_mvp_rows(op: Mapping, x: np.ndarray, positions: np.ndarray) -> np.ndarray:
    """(A^UH x) at the cluster positions ``positions``; returns (len(positions), nrhs) in the
    order given, together with the user indices perm[positions]."""
    n = int(op["n"])
    x2 = np.asarray(x, dtype=np.complex128).reshape(n, -1)
    positions = np.asarray(positions, dtype=np.int64)
    want = np.zeros(n, bool)
    want[positions] = True
    acc = np.zeros((n, x2.shape[1]), np.complex128)   # indexed by cluster position
    off, size = op["off"], op["size"]

    def rows_needed(t):
        o = int(off[t])
        r = np.arange(o, o + int(size[t]))
        return r[want[r]]

    for b in range(op["adm_row"].shape[0]):
        t, s = int(op["adm_row"][b]), int(op["adm_col"][b])
        r = rows_needed(t)
        if r.size == 0:
            continue
        lt, ls = int(op["rank_row"][t]), int(op["rank_col"][s])
        Ut, Vs = _basis(op, "U", t), _basis(op, "V", s)
        Sb = _colmajor(op["S"], int(op["S_off"][b]), lt, ls)
        acc[r] += Ut[r - int(off[t])] @ (Sb @ (Vs.conj().T @ x2[_rows_of(op, s)]))
    for b in range(op["den_row"].shape[0]):
        t, s = int(op["den_row"][b]), int(op["den_col"][b])
        r = rows_needed(t)
        if r.size == 0:
            continue
        Db = _colmajor(op["D"], int(op["D_off"][b]), int(size[t]), int(size[s]))
        acc[r] += Db[r - int(off[t])] @ x2[_rows_of(op, s)]
    return acc[positions], op["perm"][positions]


def h_mvp(op: Mapping, x: np.ndarray) -> np.ndarray:
    n = int(op["n"])
    x2 = np.asarray(x, dtype=np.complex128).reshape(n, -1)
    y = np.zeros_like(x2)
    for b in range(op["adm_row"].shape[0]):
        t, s = int(op["adm_row"][b]), int(op["adm_col"][b])
        k = int(op["adm_rank"][b])
        Xb = _colmajor(op["X"], int(op["X_off"][b]), int(op["size"][t]), k)
        Yb = _colmajor(op["Y"], int(op["Y_off"][b]), int(op["size"][s]), k)
        y[_rows_of(op, t)] += Xb @ (Yb.conj().T @ x2[_rows_of(op, s)])
    for b in range(op["den_row"].shape[0]):
        t, s = int(op["den_row"][b]), int(op["den_col"][b])
        Db = _colmajor(op["D"], int(op["D_off"][b]), int(op["size"][t]), int(op["size"][s]))
        y[_rows_of(op, t)] += Db @ x2[_rows_of(op, s)]
    return y.reshape(np.shape(x))


def expand_symmetric(op: Mapping) -> dict:
    """The general UH image that a symmetric-storage image stands for (Remark 4.4).

    A symmetric-storage image has one cluster set with one basis per cluster and lists one
    block of each mirrored pair tau x sigma / sigma x tau (diagonal dense blocks once).
    With V_sigma = conj(U_sigma) the transpose of a stored admissible block is
    (U_tau S_b V_sigma^*)^T = conj(V_sigma) S_b^T U_tau^T = U_sigma S_b^T V_tau^*, so its mirror
    has coupling S_b^T; the mirror of a stored dense block tau x sigma, tau != sigma, is
    (A|_b)^T.  The V, V_off and rank_col entries of the input are not read.  Returns the
    stored blocks followed by their mirrors, with new flat S and D arrays,
    rank_col = rank_row, V = conj(U) and V_off = U_off (the H-form entries are dropped)."""
    out = {k: v for k, v in op.items() if k not in ("adm_rank", "X_off", "Y_off", "X", "Y")}
    rank, size = np.asarray(op["rank_row"]), np.asarray(op["size"])
    out["rank_col"] = rank.copy()
    out["V"] = np.conj(op["U"])
    out["V_off"] = np.asarray(op["U_off"]).copy()
    ar, ac = np.asarray(op["adm_row"]), np.asarray(op["adm_col"])
    if np.any(ar == ac):
        raise ValueError("a cluster is admissible with itself")
    rows, cols, blocks = [], [], []
    for b in range(ar.size):
        t, s = int(ar[b]), int(ac[b])
        Sb = _colmajor(op["S"], int(op["S_off"][b]), int(rank[t]), int(rank[s]))
        rows.append(t), cols.append(s), blocks.append(Sb)
    for b in range(ar.size):
        rows.append(int(ac[b])), cols.append(int(ar[b])), blocks.append(blocks[b].T)
    out["adm_row"], out["adm_col"] = np.array(rows, np.int32), np.array(cols, np.int32)
    out["S_off"], out["S"] = _pack(blocks)
    dr, dc = np.asarray(op["den_row"]), np.asarray(op["den_col"])
    rows, cols, blocks = [], [], []
    for b in range(dr.size):
        t, s = int(dr[b]), int(dc[b])
        rows.append(t), cols.append(s)
        blocks.append(_colmajor(op["D"], int(op["D_off"][b]), int(size[t]), int(size[s])))
    for b in range(dr.size):
        if dr[b] != dc[b]:
            rows.append(int(dc[b])), cols.append(int(dr[b])), blocks.append(blocks[b].T)
    out["den_row"], out["den_col"] = np.array(rows, np.int32), np.array(cols, np.int32)
    out["D_off"], out["D"] = _pack(blocks)
    return out


def assemble_factored(op: Mapping, which: str = "all") -> dict:
    """The general UH image whose couplings are the products of their stored factors,
    S_b = S_{X,b} S_{Y,b}^* (section 4.2), S_{X,b} (l_tau x k_b) at SX_off[b] and S_{Y,b}
    (l_sigma x k_b) at SY_off[b], k_b = adm_rank[b].  which="all" forms every coupling from
    its factors; which="smaller" only those of the blocks whose factors hold fewer elements,
    k_b (l_tau + l_sigma) < l_tau l_sigma, and keeps the stored S_b of the others (the
    operator a per-block choice of the two forms stands for)."""
    out = dict(op)
    rr, rc, k = np.asarray(op["rank_row"]), np.asarray(op["rank_col"]), np.asarray(op["adm_rank"])
    blocks = []
    for b in range(np.asarray(op["adm_row"]).size):
        lt, ls, kb = int(rr[op["adm_row"][b]]), int(rc[op["adm_col"][b]]), int(k[b])
        if which == "smaller" and not kb * (lt + ls) < lt * ls:
            blocks.append(_colmajor(op["S"], int(op["S_off"][b]), lt, ls))
            continue
        sx = _colmajor(op["SX"], int(op["SX_off"][b]), lt, kb)
        sy = _colmajor(op["SY"], int(op["SY_off"][b]), ls, kb)
        blocks.append(sx @ sy.conj().T)
    out["S_off"], out["S"] = _pack(blocks)
    return out


def _pack(blocks):
    offs = np.zeros(len(blocks), np.int64)
    if blocks:
        offs[1:] = np.cumsum([m.size for m in blocks])[:-1]
    flat = np.concatenate([m.ravel(order="F") for m in blocks]) if blocks else np.zeros(0, np.complex128)
    return offs, flat


def assemble_uh(op: Mapping) -> np.ndarray:
    """The dense matrix A^UH (user order); small N only."""
    n = int(op["n"])
    return uh_mvp(op, np.eye(n, dtype=np.complex128))


def assemble_h(op: Mapping) -> np.ndarray:
    n = int(op["n"])
    return h_mvp(op, np.eye(n, dtype=np.complex128))


def optimal_row_basis(a_user: np.ndarray, op: Mapping, t: int, eps: float):
    """Algorithm 1 for one row cluster t of matrix ``a_user`` (user order): SVD of the
    explicit agglomeration A_t = [A(t, s)]_{s in row(t)}; returns (U_t, singular values)
    with the rank chosen as #{sigma_i > eps * sigma_1}."""
    cols = [int(s) for b, s in enumerate(op["adm_col"]) if int(op["adm_row"][b]) == t]
    rows = _rows_of(op, t)
    at = np.concatenate([a_user[np.ix_(rows, _rows_of(op, s))] for s in cols], axis=1)
    u, sv, _ = np.linalg.svd(at, full_matrices=False)
    ell = max(1, int(np.count_nonzero(sv > eps * sv[0])))
    return u[:, :ell], sv


# ------------------------------------------------------------------------- C bindings
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # UHM_ORACLE_LIB selects another build of the same source (the sanitizer test's)
        path = os.environ.get("UHM_ORACLE_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                                "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_uh_mvp_alg6.argtypes = [I64, P, I32, P, P, P, P, P, P, P, P,
                                           I64, P, P, P, P, I64, P, P, P, P, I32, P, P, I32]
        lib.oracle_uh_mvp_alg6.restype = ctypes.c_int
        lib.oracle_h_mvp_alg5.argtypes = [I64, P, P, P, I64, P, P, P, P, P, P, P,
                                          I64, P, P, P, P, I32, P, P, I32]
        lib.oracle_h_mvp_alg5.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def max_threads() -> int:
    return int(_lib().oracle_max_threads())


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def alg6(op: Mapping, x: np.ndarray, nthreads: int = 0) -> np.ndarray:
    n = int(op["n"])
    x2 = np.asfortranarray(np.asarray(x, dtype=np.complex128).reshape(n, -1))
    y = np.zeros_like(x2, order="F")
    keep = [_c(op["perm"], np.int64), _c(op["off"], np.int64), _c(op["size"], np.int64),
            _c(op["rank_row"], np.int32), _c(op["rank_col"], np.int32), _c(op["U_off"], np.int64),
            _c(op["V_off"], np.int64), _c(op["U"], np.complex128), _c(op["V"], np.complex128),
            _c(op["adm_row"], np.int32), _c(op["adm_col"], np.int32), _c(op["S_off"], np.int64),
            _c(op["S"], np.complex128), _c(op["den_row"], np.int32), _c(op["den_col"], np.int32),
            _c(op["D_off"], np.int64), _c(op["D"], np.complex128)]
    (perm, off, size, rr, rc, uo, vo, U, V, ar, ac, so, S, dr, dc, do, D) = keep
    rc_ = _lib().oracle_uh_mvp_alg6(n, _p(perm), off.size, _p(off), _p(size), _p(rr), _p(rc), _p(uo), _p(vo),
                                    _p(U), _p(V), ar.size, _p(ar), _p(ac), _p(so), _p(S), dr.size, _p(dr),
                                    _p(dc), _p(do), _p(D), x2.shape[1], _p(x2), _p(y), int(nthreads))
    if rc_ != 0:
        raise RuntimeError("oracle_uh_mvp_alg6 failed")
    return y.reshape(np.shape(x))


def alg5(op: Mapping, x: np.ndarray, nthreads: int = 0) -> np.ndarray:
    n = int(op["n"])
    x2 = np.asfortranarray(np.asarray(x, dtype=np.complex128).reshape(n, -1))
    y = np.zeros_like(x2, order="F")
    keep = [_c(op["perm"], np.int64), _c(op["off"], np.int64), _c(op["size"], np.int64),
            _c(op["adm_row"], np.int32), _c(op["adm_col"], np.int32), _c(op["adm_rank"], np.int32),
            _c(op["X_off"], np.int64), _c(op["Y_off"], np.int64), _c(op["X"], np.complex128),
            _c(op["Y"], np.complex128), _c(op["den_row"], np.int32), _c(op["den_col"], np.int32),
            _c(op["D_off"], np.int64), _c(op["D"], np.complex128)]
    (perm, off, size, ar, ac, ak, xo, yo, X, Y, dr, dc, do, D) = keep
    rc_ = _lib().oracle_h_mvp_alg5(n, _p(perm), _p(off), _p(size), ar.size, _p(ar), _p(ac), _p(ak), _p(xo),
                                   _p(yo), _p(X), _p(Y), dr.size, _p(dr), _p(dc), _p(do), _p(D),
                                   x2.shape[1], _p(x2), _p(y), int(nthreads))
    if rc_ != 0:
        raise RuntimeError("oracle_h_mvp_alg5 failed")
    return y.reshape(np.shape(x))
