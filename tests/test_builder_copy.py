"""The builder's native scaled copy (uhmb_scaled_copy), which lays out the agglomerated
block rows X_tau = [U_b Sigma_b ...] and the H-matrix factors, against numpy on strided
views: transposed sources, conjugation, column scaling and zero fill."""
import numpy as np

from paper_2405_15573_amd import builder


def test_scaled_copy_matches_numpy():
    rng = np.random.default_rng(4)
    m, kp = 37, 23
    dst = np.full((m, kp), np.nan + 0j)                      # row-major destination
    dcol = np.full(m * 9, np.nan + 0j)                       # column-major destination
    a = rng.standard_normal((6, m)) + 1j * rng.standard_normal((6, m))   # a.T: m x 6, transposed
    b = rng.standard_normal((m, 9)) + 1j * rng.standard_normal((m, 9))   # C order
    sa, sb = rng.random(6), rng.random(9)
    views = [builder._view(a.T), builder._view(b)]
    base = dst.__array_interface__["data"][0]
    col = dcol.__array_interface__["data"][0]
    recs = [
        (views[0][0], base, sa.__array_interface__["data"][0], views[0][1], views[0][2], kp, 1, m, 6, 0, 0),
        (views[1][0], base + 16 * 6, sb.__array_interface__["data"][0], views[1][1], views[1][2], kp, 1, m, 9,
         1, 0),
        (0, base + 16 * 15, 0, 0, 0, kp, 1, m, kp - 15, 0, 0),
        (views[1][0], col, 0, views[1][1], views[1][2], 1, m, m, 9, 1, 0),
    ]
    builder._scaled_copy(recs)
    ref = np.concatenate([a.T * sa[None, :], np.conj(b) * sb[None, :], np.zeros((m, kp - 15))], axis=1)
    assert np.array_equal(dst, ref)
    assert np.array_equal(dcol.reshape(9, m).T, np.conj(b))


def test_view_copies_what_it_cannot_address():
    x = np.arange(12, dtype=np.float64).reshape(3, 4)
    addr, rs, cs, keep = builder._view(x)          # float64: a complex128 copy is made
    assert keep.dtype == np.complex128 and keep is not x and (rs, cs) == (4, 1)
    y = (np.arange(12) + 0j).reshape(3, 4)[:, ::2]
    addr, rs, cs, keep = builder._view(y)
    assert keep is y and (rs, cs) == (4, 2)
