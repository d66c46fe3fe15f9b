"""GMRES iterates by their definition.  Test infrastructure.

The k-th GMRES iterate from x0 is the vector of the affine Krylov space
x0 + span{r0, A r0, ..., A^{k-1} r0} (r0 = b - A x0) with the smallest residual 2-norm
(Saad and Schultz, 1986).  Here that minimisation is done literally: an orthonormal basis
Q of the Krylov space (the Krylov vectors themselves, orthonormalised by a QR
factorisation with a second Gram-Schmidt sweep against the earlier columns), then the
least-squares problem min_y ||r0 - A Q y|| by numpy's lstsq.  Nothing here uses Hessenberg
matrices or Givens rotations, so it checks the GPU solver's least-squares machinery
against the plain definition.

Restarted GMRES(m) is the same minimisation repeated, each cycle from the previous
iterate.  Iterative refinement with an inner operator (GMRES-IR, one inner cycle per
refinement) takes each cycle's correction from the inner operator's Krylov space and
minimisation, and the next residual from the exact operator.
"""
import numpy as np


def krylov_basis(apply_a, r0: np.ndarray, k: int) -> np.ndarray:
    """Orthonormal basis (n x k) of span{r0, A r0, ..., A^{k-1} r0}."""
    n = r0.shape[0]
    q = np.zeros((n, k), dtype=np.complex128)
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        for _ in range(2):   # classical Gram-Schmidt, twice
            v = v - q[:, :j] @ (q[:, :j].conj().T @ v)
        q[:, j] = v / np.linalg.norm(v)
        v = apply_a(q[:, j])
    return q


def gmres_cycle(apply_a, b: np.ndarray, x0: np.ndarray, k: int) -> np.ndarray:
    """x0 + argmin over the k-dimensional Krylov space of r0 = b - A x0 of ||b - A x||."""
    r0 = b - apply_a(x0)
    if np.linalg.norm(r0) == 0.0:
        return x0.copy()
    q = krylov_basis(apply_a, r0, k)
    aq = np.stack([apply_a(q[:, j]) for j in range(k)], axis=1)
    y = np.linalg.lstsq(aq, r0, rcond=None)[0]
    return x0 + q @ y


def gmres_restarted(apply_a, b: np.ndarray, m: int, iterations: int) -> np.ndarray:
    """GMRES(m) from x0 = 0 after `iterations` Krylov steps (cycles of m, the last one
    shorter if `iterations` is not a multiple of m)."""
    x = np.zeros_like(b, dtype=np.complex128)
    done = 0
    while done < iterations:
        k = min(m, iterations - done)
        x = gmres_cycle(apply_a, b, x, k)
        done += k
    return x


def gmres_ir_cycles(apply_a, apply_inner, b: np.ndarray, m: int, cycles: int) -> np.ndarray:
    """GMRES-IR with one inner GMRES(m) cycle per refinement step, from x0 = 0:
    r = b - A x, d = argmin over K_m(A_inner, r) of ||r - A_inner d||, x += d."""
    x = np.zeros_like(b, dtype=np.complex128)
    for _ in range(cycles):
        r = b - apply_a(x)
        x = x + gmres_cycle(apply_inner, r, np.zeros_like(r), m)
    return x
