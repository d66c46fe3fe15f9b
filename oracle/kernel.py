"""Brute-force products with the Helmholtz single-layer point kernel.  Test infrastructure.

g(x, y) = exp(i kappa |x - y|) / (4 pi |x - y|)   (section 6.1, the 3D Helmholtz
single-layer kernel), and A_ij = g(x_i, x_j) for i != j.  The diagonal of the point
(Nystrom-like) discretisation is set to a given real value (1/(2h) in every workload).
Nothing here is stored beyond one chunk of rows, so N of a few hundred thousand is fine
for a handful of rows.
"""
import numpy as np


def g(r: np.ndarray, kappa: float) -> np.ndarray:
    """Kernel value at distance r > 0."""
    return np.exp(1j * kappa * r) / (4.0 * np.pi * r)


def dense_matrix(points: np.ndarray, kappa: float, diag: float) -> np.ndarray:
    """The whole matrix A (user order).  For N up to a few thousand."""
    d = points[:, None, :] - points[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, 1.0)
    a = g(r, kappa)
    np.fill_diagonal(a, diag)
    return a


def dense_rows(points: np.ndarray, kappa: float, diag: float, rows: np.ndarray) -> np.ndarray:
    """Rows A[rows, :] of the matrix (user order)."""
    rows = np.asarray(rows, dtype=np.int64)
    d = points[rows][:, None, :] - points[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    hit = r == 0.0
    r[hit] = 1.0
    a = g(r, kappa)
    a[hit] = diag
    a[np.arange(rows.size), rows] = diag
    return a


def dense_matvec(points, kappa, diag, x, rows=None, chunk=512):
    """(A x)[rows] (all rows if rows is None) for x of shape (N,) or (N, r)."""
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    x2 = x.reshape(n, -1)
    out = np.empty((rows.size, x2.shape[1]), dtype=np.complex128)
    for a in range(0, rows.size, chunk):
        out[a:a + chunk] = dense_rows(points, kappa, diag, rows[a:a + chunk]) @ x2
    return out.reshape((rows.size,) + x.shape[1:])

