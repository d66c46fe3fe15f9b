"""Pins of oracle/krylov.py (GMRES iterates by their definition) to the mathematics.  No GPU.

* With k = n Krylov steps the iterate is the solution A^{-1} b (the Krylov space is the
  whole space for a generic b).
* The residual of the k-th iterate is orthogonal to A K_k (the normal equations of the
  minimisation), and the iterate lies in x0 + K_k.
* The residual norm does not increase with k.
* One step from x0 = 0 has the closed form x1 = alpha b, alpha = (A b)^* b / |A b|^2.
* Restarting with m at least the step count is one cycle; refinement with the exact
  operator as the inner one is restarted GMRES (each cycle minimises over the same space).
* A planted mistake (the Krylov space of b instead of r0 after a restart) is rejected.
"""
import numpy as np

from oracle import krylov


def _system(n=24, seed=0):
    rng = np.random.default_rng(seed)
    a = np.eye(n) * 3.0 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return a, b


def test_full_space_gives_the_solution():
    a, b = _system()
    x = krylov.gmres_cycle(lambda v: a @ v, b, np.zeros_like(b), b.size)
    assert np.linalg.norm(x - np.linalg.solve(a, b)) <= 1e-10 * np.linalg.norm(x)


def test_residual_orthogonal_to_a_krylov_and_iterate_in_space():
    a, b = _system(seed=1)
    x0 = np.full_like(b, 0.3 - 0.1j)
    r0 = b - a @ x0
    for k in (1, 3, 7):
        x = krylov.gmres_cycle(lambda v: a @ v, b, x0, k)
        q = krylov.krylov_basis(lambda v: a @ v, r0, k)
        r = b - a @ x
        aq = a @ q
        # rounding is relative to the size of the data, |r0|, not to the small final residual
        assert np.linalg.norm(aq.conj().T @ r) <= 1e-12 * np.linalg.norm(aq) * np.linalg.norm(r0)
        d = x - x0
        assert np.linalg.norm(d - q @ (q.conj().T @ d)) <= 1e-12 * np.linalg.norm(d)
        # the basis spans the Krylov vectors themselves
        kv = np.stack([np.linalg.matrix_power(a, j) @ r0 for j in range(k)], axis=1)
        assert np.linalg.norm(kv - q @ (q.conj().T @ kv)) <= 1e-10 * np.linalg.norm(kv)


def test_residual_non_increasing():
    a, b = _system(seed=2)
    res = [np.linalg.norm(b - a @ krylov.gmres_cycle(lambda v: a @ v, b, np.zeros_like(b), k)) for k in range(1, 12)]
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))


def test_one_step_closed_form():
    a, b = _system(seed=3)
    ab = a @ b
    alpha = np.vdot(ab, b) / np.vdot(ab, ab)
    x = krylov.gmres_cycle(lambda v: a @ v, b, np.zeros_like(b), 1)
    assert np.linalg.norm(x - alpha * b) <= 1e-13 * np.linalg.norm(x)


def test_restart_and_refinement_consistency():
    a, b = _system(seed=4)
    f = lambda v: a @ v   # noqa: E731
    one = krylov.gmres_cycle(f, b, np.zeros_like(b), 6)
    assert np.linalg.norm(krylov.gmres_restarted(f, b, 10, 6) - one) <= 1e-13 * np.linalg.norm(one)
    rst = krylov.gmres_restarted(f, b, 4, 12)
    ir = krylov.gmres_ir_cycles(f, f, b, 4, 3)
    assert np.linalg.norm(ir - rst) <= 1e-12 * np.linalg.norm(rst)


def test_planted_restart_mistake_rejected():
    """A restart that builds the Krylov space of b instead of the current residual."""
    a, b = _system(seed=5)
    f = lambda v: a @ v   # noqa: E731

    def wrong_cycle(x0, k):
        q = krylov.krylov_basis(f, b, k)
        aq = a @ q
        y = np.linalg.lstsq(aq, b - a @ x0, rcond=None)[0]
        return x0 + q @ y

    x = np.zeros_like(b)
    for _ in range(3):
        x = wrong_cycle(x, 4)
    ref = krylov.gmres_restarted(f, b, 4, 12)
    assert np.linalg.norm(x - ref) > 1e-6 * np.linalg.norm(ref)
