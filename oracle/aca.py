"""Adaptive cross approximation with partial pivoting, and kernel blocks.  Test infrastructure.

Section 2.3 builds the low-rank factors of the admissible blocks by ACA with partial
pivoting (the variant due to Bebendorf that the paper cites); the paper states its cost,
C k (|tau| + |sigma|) (C_elem + C k), but not its steps.  The steps followed here are the
published ones:

  start from row i_1 = 0 of the block R_0 = A|_b; at step k
    row      r = A[i_k, :] - sum_{l<k} u_l[i_k] v_l            (residual row i_k)
             row i_k is now used; if r vanishes, take the next unused row and repeat
    pivot    j_k = argmax_j |r_j|
    factors  v_k = r / r[j_k],   u_k = A[:, j_k] - sum_{l<k} v_l[j_k] u_l
    stop     when |u_k| |v_k| <= eps |S_k|_F,  S_k = sum_{l<=k} u_l v_l^T
    next     i_{k+1} = argmax over unused rows of |u_k[i]|
  and at most min(m, n, cap) terms.

Readings where the published description leaves a choice (the GPU construction takes the
same ones):
  * "largest modulus" is decided on |z|^2 = re^2 + im^2 in FP64, the first index wins a tie;
  * |S_k|_F is the Frobenius norm of the assembled approximation (computed here from
    the dense sum, which is the definition);
  * when a residual row vanishes, the next row tried is the unused row of smallest index.

The entries of a block are those of the point-kernel matrix of ``oracle.kernel``, addressed
by position in the point array (cluster order).  Nothing here is shared with the product
package.

Pins: tests/test_oracle_aca.py (exact low-rank recovery, the cross interpolation property,
agreement of the cross with the block on its pivot rows and columns, a textbook Gaussian
elimination identity, and the error on separated clusters of the Helmholtz kernel).
"""
from __future__ import annotations

import numpy as np

from . import kernel


def kernel_block(points: np.ndarray, kappa: float, diag: float, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """A[rows, cols] of the point-kernel matrix, rows and columns given as positions in
    ``points``; coincident positions (and coincident points) take the diagonal value."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    d = points[rows][:, None, :] - points[cols][None, :, :]
    r = np.sqrt((d * d).sum(-1))
    hit = (r == 0.0) | (rows[:, None] == cols[None, :])
    r[hit] = 1.0
    a = kernel.g(r, kappa)
    a[hit] = diag
    return a


def _mod2(z: np.ndarray) -> np.ndarray:
    return z.real * z.real + z.imag * z.imag


def aca_partial(entry_row, entry_col, m: int, n: int, eps: float, cap: int):
    """ACA with partial pivoting on an m x n block given by its row and column samplers.

    entry_row(i) -> A[i, :] (n,), entry_col(j) -> A[:, j] (m,).
    Returns (u (m x k), v (n x k), rows (k,), cols (k,), converged) with
    A ~ u @ v.T = sum_l u_l v_l^T, the pivot rows i_l and columns j_l of the terms kept,
    and converged False only when the cap stopped the iteration before the criterion
    (cap < min(m, n)).
    """
    kmax = min(m, n, cap)
    us, vs, prow, pcol = [], [], [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    converged = True
    while len(us) < kmax:
        r = np.asarray(entry_row(i), dtype=np.complex128).copy()
        for l in range(len(us)):
            r -= us[l][i] * vs[l]
        used[i] = True
        j = int(np.argmax(_mod2(r)))
        if not _mod2(r)[j] > 0.0:
            free = np.nonzero(~used)[0]
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = np.asarray(entry_col(j), dtype=np.complex128).copy()
        for l in range(len(us)):
            u -= vs[l][j] * us[l]
        us.append(u)
        vs.append(v)
        prow.append(i)
        pcol.append(j)
        S = np.stack(us, 1) @ np.stack(vs, 1).T
        if np.linalg.norm(u) * np.linalg.norm(v) <= eps * np.linalg.norm(S):
            break
        free = np.nonzero(~used)[0]
        if free.size == 0:
            break
        i = int(free[np.argmax(_mod2(u[free]))])
    else:
        converged = kmax < cap or kmax == min(m, n)
    k = len(us)
    U = np.stack(us, 1) if k else np.zeros((m, 0), np.complex128)
    V = np.stack(vs, 1) if k else np.zeros((n, 0), np.complex128)
    return U, V, np.asarray(prow, np.int64), np.asarray(pcol, np.int64), converged


def aca_kernel_block(points, kappa, diag, row_off, m, col_off, n, eps, cap):
    """ACA of the kernel block of positions [row_off, row_off+m) x [col_off, col_off+n)."""
    rows = np.arange(row_off, row_off + m)
    cols = np.arange(col_off, col_off + n)
    return aca_partial(lambda i: kernel_block(points, kappa, diag, rows[i:i + 1], cols)[0],
                       lambda j: kernel_block(points, kappa, diag, rows, cols[j:j + 1])[:, 0],
                       m, n, eps, cap)
