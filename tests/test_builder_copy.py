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


def _blocks(rng):
    """Stored blocks (t < s) of a few clusters with random factors: U (size t x k), V (size s
    x k) as transposed views, as the recompression leaves them, and Sigma."""
    size = np.array([40, 40, 24, 17, 33])
    keys = [(0, 1), (0, 3), (1, 2), (2, 4), (1, 4), (3, 4)]
    fac_U, fac_V, fac_s = {}, {}, {}
    for t, s in keys:
        k = int(rng.integers(1, 7))
        fac_U[(t, s)] = (rng.standard_normal((k, size[t])) + 1j * rng.standard_normal((k, size[t]))).T
        fac_V[(t, s)] = (rng.standard_normal((k, size[s])) + 1j * rng.standard_normal((k, size[s]))).T
        fac_s[(t, s)] = np.sort(rng.random(k))[::-1].copy()
    adm = np.array(keys + [(s, t) for t, s in keys])
    return size, fac_U, fac_V, fac_s, adm


def test_row_records_lay_out_the_cluster_matrices():
    """X_tau = [U_b Sigma_b ...] over tau's block row (conj(V_b) Sigma_b for a mirrored block),
    row-major and zero-padded: the batch the GPU factorisation of Alg. 2 reads."""
    rng = np.random.default_rng(9)
    size, fac_U, fac_V, fac_s, adm = _blocks(rng)
    row_blocks = {}
    for t, s in adm:
        row_blocks.setdefault(int(t), []).append(int(s))
    fv = builder._factor_views_of(fac_U, fac_V, fac_s)
    part = [(0, 0), (1, 0)]   # a batch holds clusters of one size: 0 and 1 have 40 rows
    nt = 40
    ks = [sum(fac_s[(min(t, s), max(t, s))].size for s in row_blocks[t]) for t, _ in part]
    kp = max(ks) + 3
    buf = np.full((len(part), nt, kp), np.nan + 0j)
    recs, cols = builder._row_records(part, row_blocks, fv, buf.__array_interface__["data"][0], nt, kp)
    builder._scaled_copy(recs)
    for c, (t, _) in enumerate(part):
        ref = []
        for s in row_blocks[t]:
            if t < s:
                ref.append(fac_U[(t, s)] * fac_s[(t, s)][None, :])
            else:
                ref.append(np.conj(fac_V[(s, t)]) * fac_s[(s, t)][None, :])
        ref = np.concatenate(ref + [np.zeros((nt, kp - ks[c]))], axis=1)
        assert np.array_equal(buf[c], ref)
        j = 0
        for (s, j0, kb), s_ref in zip(cols[c], row_blocks[t]):
            assert s == s_ref and j0 == j and kb == fac_s[(min(t, s), max(t, s))].size
            j += kb


def test_hfactor_records_write_both_triangles():
    """X_b = U_b Sigma_b and Y_b = V_b column-major for every admissible block, the mirror of
    a stored block (s, t) taking U_b = conj(V), V_b = conj(U)."""
    rng = np.random.default_rng(10)
    size, fac_U, fac_V, fac_s, adm = _blocks(rng)
    kb = np.array([fac_s[(min(t, s), max(t, s))].size for t, s in adm])
    xs, ys = size[adm[:, 0]] * kb, size[adm[:, 1]] * kb
    X_off = np.concatenate([[0], np.cumsum(xs)[:-1]])
    Y_off = np.concatenate([[0], np.cumsum(ys)[:-1]])
    Xh = np.full(int(xs.sum()), np.nan + 0j)
    Yh = np.full(int(ys.sum()), np.nan + 0j)
    fv = builder._factor_views_of(fac_U, fac_V, fac_s)
    builder._scaled_copy(builder._hfactor_records(adm, kb, size, X_off, Y_off, Xh.__array_interface__["data"][0],
                                                  Yh.__array_interface__["data"][0], fv))
    for b, (t, s) in enumerate(adm):
        X = Xh[X_off[b]:X_off[b] + xs[b]].reshape(kb[b], size[t]).T
        Y = Yh[Y_off[b]:Y_off[b] + ys[b]].reshape(kb[b], size[s]).T
        if t < s:
            Ub, Vb, sb = fac_U[(t, s)], fac_V[(t, s)], fac_s[(t, s)]
        else:
            Ub, Vb, sb = np.conj(fac_V[(s, t)]), np.conj(fac_U[(s, t)]), fac_s[(s, t)]
        assert np.array_equal(X, Ub * sb[None, :]) and np.array_equal(Y, Vb)
