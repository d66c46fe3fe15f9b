"""Pins of the ACA oracle (oracle/aca.py) to what the mathematics fixes (no GPU).

What pins what:
  kernel_block      equals the corresponding block of kernel.dense_matrix (itself pinned
                    by hand-worked values)
  aca_partial       * a matrix of exact rank r is recovered to rounding in r (or r + 1) terms;
                    * the cross interpolation property: the residual A - U V^T vanishes on
                      every pivot row and every pivot column;
                    * the first term is the Gaussian elimination step
                      A[:, j1] A[0, :] / A[0, j1], with j1 = argmax |A[0, :]|, and the second
                      pivot row holds the largest entry of column j1 among the other rows;
                    * with min(m, n) terms and eps = 0 a random matrix is reproduced exactly;
                    * a zero first row is skipped; a rank cap stops the iteration and is
                      reported;
                    * on two separated clusters of the Helmholtz kernel (the stopping rule):
                      the error is at most 3 eps and at least the optimal error of its rank
                      (Eckart-Young, from the block's singular values), and the rank lies
                      between the optimal rank at eps and 3 past the optimal rank at eps/10,
                      so a rule that stops a decade early or late is rejected.
A last test plants plausible mistakes in copies of aca_partial and checks that these pins
reject each one.
"""
import inspect

import numpy as np
import pytest

from oracle import aca, kernel
from paper_2405_15573_amd import inputs


def _rand(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))


def _run(a, eps, cap=None, fn=None):
    fn = fn or aca.aca_partial
    m, n = a.shape
    return fn(lambda i: a[i], lambda j: a[:, j], m, n, eps, cap or min(m, n))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_kernel_block_is_a_block_of_the_dense_matrix():
    cloud = inputs.make_cloud("sphere", 300, seed=2)
    diag = 1.0 / (2.0 * cloud.h)
    a = kernel.dense_matrix(cloud.points, cloud.kappa, diag)
    rows, cols = np.arange(10, 90), np.arange(50, 170)
    blk = aca.kernel_block(cloud.points, cloud.kappa, diag, rows, cols)
    assert np.max(np.abs(blk - a[10:90, 50:170])) <= 1e-15 * np.max(np.abs(a))


def test_exact_low_rank_recovery():
    for seed, (m, n, r) in enumerate([(40, 30, 5), (64, 64, 12), (17, 93, 3)]):
        a = _rand(m, r, seed) @ _rand(r, n, seed + 10)
        u, v, pr, pc, conv = _run(a, 1e-12)
        assert conv and u.shape[1] in (r, r + 1)
        assert _rel(u @ v.T, a) <= 1e-12


def test_cross_interpolation_property():
    """After any number of steps the residual is zero on the pivot rows and columns."""
    cloud = inputs.make_cloud("cube", 400, seed=3)
    diag = 1.0 / (2.0 * cloud.h)
    a = aca.kernel_block(cloud.points, cloud.kappa, diag, np.arange(0, 120), np.arange(200, 380))
    for cap in (1, 4, 9):
        u, v, pr, pc, _ = _run(a, 0.0, cap=cap)
        assert u.shape[1] == cap
        res = a - u @ v.T
        scale = np.max(np.abs(a))
        assert np.max(np.abs(res[pr, :])) <= 1e-13 * scale
        assert np.max(np.abs(res[:, pc])) <= 1e-13 * scale
        assert len(set(pr.tolist())) == cap and len(set(pc.tolist())) == cap


def test_first_step_is_gaussian_elimination():
    a = _rand(25, 31, 7)
    u, v, pr, pc, _ = _run(a, 0.0, cap=2)
    j1 = int(np.argmax(np.abs(a[0])))
    assert pr[0] == 0 and pc[0] == j1
    t1 = np.outer(a[:, j1], a[0]) / a[0, j1]
    assert np.max(np.abs(np.outer(u[:, 0], v[:, 0]) - t1)) <= 1e-14 * np.max(np.abs(t1))
    c = np.abs(a[:, j1])   # u_1 is the residual column j1 before the step: column j1 of A
    c[0] = -1.0
    assert pr[1] == int(np.argmax(c))


def test_full_rank_reproduces_the_matrix():
    a = _rand(8, 6, 11)
    u, v, pr, pc, conv = _run(a, 0.0)
    assert u.shape[1] == 6 and conv
    assert _rel(u @ v.T, a) <= 1e-13


def test_zero_row_skipped_and_cap_reported():
    a = np.outer(_rand(12, 1, 1)[:, 0], _rand(1, 9, 2)[0])
    a[0] = 0.0
    u, v, pr, pc, conv = _run(a, 1e-10)
    assert pr[0] == 1 and conv
    assert _rel(u @ v.T, a) <= 1e-13
    b = _rand(30, 20, 5)
    u, v, pr, pc, conv = _run(b, 1e-10, cap=3)
    assert u.shape[1] == 3 and not conv


def _helmholtz_block():
    rng = np.random.default_rng(9)
    src = rng.uniform(-0.5, 0.5, size=(300, 3))
    dst = rng.uniform(-0.5, 0.5, size=(260, 3)) + np.array([3.0, 0.0, 0.0])
    pts = np.concatenate([src, dst])
    return aca.kernel_block(pts, 4.0, 1.0, np.arange(300), np.arange(300, 560))


def _stopping_rule_failures(fn=None):
    """Checks of the stopping rule on the Helmholtz block; returns the failed ones."""
    a = _helmholtz_block()
    sv = np.linalg.svd(a, compute_uv=False)
    # tail[k]: the smallest relative Frobenius error of any rank-k approximation
    tail = np.append(np.sqrt(np.cumsum((sv ** 2)[::-1])[::-1]) / np.linalg.norm(a), 0.0)
    ropt = lambda e: int(np.argmax(tail <= e))   # noqa: E731
    failed = []
    for eps in (1e-4, 1e-6, 1e-8):
        u, v, pr, pc, conv = _run(a, eps, fn=fn)
        k = u.shape[1]
        err = _rel(u @ v.T, a)
        if not conv:
            failed.append(f"{eps}: not converged")
        if err > 3 * eps:
            failed.append(f"{eps}: error {err:.2e} above 3 eps")
        if err < tail[k] * (1 - 1e-6):
            failed.append(f"{eps}: error below the optimum of rank {k}")
        if not ropt(eps) <= k <= ropt(eps / 10) + 3:
            failed.append(f"{eps}: rank {k} outside [{ropt(eps)}, {ropt(eps / 10) + 3}]")
    return failed


def test_helmholtz_separated_clusters():
    assert _stopping_rule_failures() == []


MISTAKES = {
    "row_update_sign": ("r -= us[l][i] * vs[l]", "r += us[l][i] * vs[l]"),
    "col_update_index": ("u -= vs[l][j] * us[l]", "u -= vs[l][i] * us[l]"),
    "no_pivot_scaling": ("v = r / r[j]", "v = r"),
    "conj_row": ("r = np.asarray(entry_row(i), dtype=np.complex128).copy()",
                 "r = np.conj(np.asarray(entry_row(i), dtype=np.complex128))"),
    "pivot_min": ("j = int(np.argmax(_mod2(r)))", "j = int(np.argmin(_mod2(r)))"),
    "reuse_rows": ("i = int(free[np.argmax(_mod2(u[free]))])", "i = int(np.argmax(_mod2(u)))"),
    "stop_early": ("<= eps * np.linalg.norm(S)", "<= 10 * eps * np.linalg.norm(S)"),
    "stop_late": ("<= eps * np.linalg.norm(S)", "<= 0.1 * eps * np.linalg.norm(S)"),
}


def _planted(name):
    src = inspect.getsource(aca.aca_partial)
    old, new = MISTAKES[name]
    assert old in src
    ns = dict(vars(aca))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    return ns["aca_partial"]


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_pins_reject_planted_mistakes(name):
    fn = _planted(name)
    failed = []
    cloud = inputs.make_cloud("cube", 400, seed=3)
    diag = 1.0 / (2.0 * cloud.h)
    blk = aca.kernel_block(cloud.points, cloud.kappa, diag, np.arange(0, 120), np.arange(200, 380))
    try:
        u, v, pr, pc, _ = _run(blk, 0.0, cap=9, fn=fn)
        res = blk - u @ v.T
        s = np.max(np.abs(blk))
        if np.max(np.abs(res[pr, :])) > 1e-13 * s or np.max(np.abs(res[:, pc])) > 1e-13 * s:
            failed.append("cross")
        if len(set(pr.tolist())) < len(pr):
            failed.append("distinct rows")
    except Exception:
        failed.append("raised")
    a = _rand(25, 31, 7)
    u, v, pr, pc, _ = _run(a, 0.0, cap=2, fn=fn)
    if pc[0] != int(np.argmax(np.abs(a[0]))):
        failed.append("first pivot")
    try:
        failed += _stopping_rule_failures(fn)
    except Exception:
        failed.append("raised")
    assert failed, name
