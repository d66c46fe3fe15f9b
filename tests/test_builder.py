"""Host builder invariants and the paper's bounds on the compression (no GPU)."""
import numpy as np
import pytest

from conftest import operator, rel
from oracle import uniform
from paper_2405_15573_amd import builder, inputs


def test_tree_is_a_cluster_tree():
    cloud = inputs.make_cloud("sphere", 3000, seed=1)
    t = builder.build_tree(cloud.points, 64)
    assert sorted(t.perm.tolist()) == list(range(3000))
    leaves = t.leaves()
    assert np.all(t.level[leaves] == t.depth)
    assert np.all(t.size[leaves] <= 64) and np.all(t.size[leaves] >= 1)
    # leaves partition [0, N) in cluster order
    lo = np.sort(t.off[leaves])
    assert lo[0] == 0 and np.all(np.diff(np.append(lo, 3000)) == t.size[leaves][np.argsort(t.off[leaves])])
    for c in range(t.nclusters):
        a, b = t.child[c]
        if a >= 0:
            assert t.off[a] == t.off[c] and t.off[b] == t.off[a] + t.size[a]
            assert t.size[a] + t.size[b] == t.size[c]
            assert t.parent[a] == c and t.parent[b] == c


def test_block_tree_partitions_the_matrix():
    cloud = inputs.make_cloud("sphere", 600, seed=2)
    t = builder.build_tree(cloud.points, 16)
    adm, den = builder.build_block_tree(t, 1.0)
    cover = np.zeros((600, 600), np.int32)
    for (a, b) in np.concatenate([adm, den]):
        cover[t.off[a]:t.off[a] + t.size[a], t.off[b]:t.off[b] + t.size[b]] += 1
    assert np.all(cover == 1)
    diam = t.diam()
    for (a, b) in adm:
        gap = np.maximum(0, np.maximum(t.lo[a] - t.hi[b], t.lo[b] - t.hi[a]))
        assert np.linalg.norm(gap) > min(diam[a], diam[b])
        assert t.level[a] == t.level[b]
    # symmetric block structure
    sa = {(int(a), int(b)) for a, b in adm}
    assert all((b, a) in sa for a, b in sa)


def test_orthogonal_bases_and_conjugate_symmetry(small_op):
    _, op = small_op
    for c in np.nonzero(op.rank_row)[0]:
        n, l = int(op.size[c]), int(op.rank_row[c])
        Uc = op.U[op.U_off[c]:op.U_off[c] + n * l].reshape(l, n).T
        assert np.linalg.norm(Uc.conj().T @ Uc - np.eye(l)) < 1e-13
    assert np.array_equal(op.V, np.conj(op.U))
    assert np.array_equal(op.rank_row, op.rank_col)


def test_couplings_are_optimal(small_op):
    """S_b = U_tau^* (X_b Y_b^*) V_sigma, the optimal coefficient matrix (section 4.1)."""
    _, op = small_op
    for b in range(0, op.nadm, 37):
        t, s = int(op.adm_row[b]), int(op.adm_col[b])
        nt, ns, lt, ls, k = int(op.size[t]), int(op.size[s]), int(op.rank_row[t]), int(op.rank_col[s]), int(op.adm_rank[b])
        Ut = op.U[op.U_off[t]:op.U_off[t] + nt * lt].reshape(lt, nt).T
        Vs = op.V[op.V_off[s]:op.V_off[s] + ns * ls].reshape(ls, ns).T
        Xb = op.X[op.X_off[b]:op.X_off[b] + nt * k].reshape(k, nt).T
        Yb = op.Y[op.Y_off[b]:op.Y_off[b] + ns * k].reshape(k, ns).T
        Sb = op.S[op.S_off[b]:op.S_off[b] + lt * ls].reshape(ls, lt).T
        assert rel(Sb, Ut.conj().T @ (Xb @ Yb.conj().T) @ Vs) < 1e-12


def test_theorem_5_1_and_frobenius_identity(small_op):
    _, op = small_op
    o = vars(op)
    d = uniform.assemble_h(o) - uniform.assemble_uh(o)
    # every cluster is both a row and a column cluster; the column side mirrors the row side
    spec_bound = np.sqrt(2.0) * np.sqrt(2.0 * np.sum(op.sv_dropped ** 2))
    assert np.linalg.norm(d, 2) <= spec_bound
    fro_bound = 2.0 * np.sum(op.sv_tail ** 2)
    assert np.linalg.norm(d) ** 2 <= fro_bound * (1 + 1e-8)


def test_algorithm_1_and_2_give_the_same_basis(small_op):
    """Alg. 2 works on the thin factor X_tau, whose SVD composed with the block-diagonal
    orthogonal Q_tau is the SVD of the agglomeration matrix A_tau (section 4.2).  So Alg. 1
    on the assembled H-matrix finds the same ranks, and the Alg. 2 basis attains Alg. 1's
    optimal projection error sigma_{l+1}(A_tau)."""
    _, op = small_op
    o = vars(op)
    ah = uniform.assemble_h(o)
    checked = 0
    for t in np.nonzero(op.rank_row)[0][::5]:
        t = int(t)
        u1, sv = uniform.optimal_row_basis(ah, o, t, op.eps_comp)
        l = int(op.rank_row[t])
        thr = op.eps_comp * sv[0]
        if np.any(np.abs(sv - thr) < 1e-9 * sv[0]):
            continue  # a singular value sits on the threshold: the rank is rounding-dependent
        assert u1.shape[1] == l
        n = int(op.size[t])
        Ut = op.U[op.U_off[t]:op.U_off[t] + n * l].reshape(l, n).T
        cols = [int(s) for b, s in enumerate(op.adm_col) if int(op.adm_row[b]) == t]
        rows = op.perm[op.off[t]:op.off[t] + n]
        at = np.concatenate([ah[np.ix_(rows, op.perm[op.off[s]:op.off[s] + op.size[s]])] for s in cols], 1)
        err = np.linalg.norm(at - Ut @ (Ut.conj().T @ at), 2)
        best = sv[l] if l < sv.size else 0.0
        assert err <= best * (1 + 1e-6) + 1e-13 * sv[0]
        assert abs(op.sv_dropped[t] - best) <= 1e-6 * best + 1e-13 * sv[0]
        checked += 1
    assert checked > 10


def test_storage_lemma(small_op):
    """Lemma 2.6: N_st^UH <= l_max (L|I| + L|J|) + 2 c_sp l_max^2 min(|I|,|J|)/n_min and
    #P+ <= 2 c_sp min(|I|,|J|)/n_min, with the measured constants."""
    _, op = small_op
    st = op.stats()
    L = op.depth + 1
    n_min = int(op.size.min())
    nst_uh = st["elems_U"] + st["elems_V"] + st["elems_S"]
    assert nst_uh <= st["l_max"] * 2 * L * op.n + 2 * st["c_sp"] * st["l_max"] ** 2 * op.n / n_min
    assert op.nadm <= 2 * st["c_sp"] * op.n / n_min
    nst_h = st["elems_XY"]
    assert nst_h <= st["c_sp"] * st["k_max"] * 2 * L * op.n


def test_save_load_roundtrip(tmp_path, small_op):
    _, op = small_op
    p = str(tmp_path / "op.npz")
    builder.save_operator(op, p)
    op2 = builder.load_operator(p)
    assert op2.n == op.n and op2.kappa == op.kappa
    assert np.array_equal(op2.S, op.S) and np.array_equal(op2.perm, op.perm)


def test_pack_factors_layout():
    """The packing of GPU ACA output for the recompression (builder._pack_factors), on CPU
    tensors: X[c] = u (m x kp), Y[c] = conj(v) (n x kp), zero beyond each block's rank, for
    the selected blocks of a contiguous shape group, whatever the unused columns hold."""
    import torch
    from types import SimpleNamespace
    from paper_2405_15573_amd import builder
    rng = np.random.default_rng(3)
    nb, m, n, c = 5, 7, 4, 3
    ranks = np.array([2, 3, 1, 3, 2])
    U = rng.normal(size=(nb, c, m)) + 1j * rng.normal(size=(nb, c, m))   # column l of block b at [b, l]
    V = rng.normal(size=(nb, c, n)) + 1j * rng.normal(size=(nb, c, n))
    Uf = np.concatenate([np.full(5, 9.0 + 9j), U.ravel()])
    Vf = np.concatenate([np.full(5, 9.0 + 9j), V.ravel()])
    res = SimpleNamespace(U=torch.from_numpy(Uf), V=torch.from_numpy(Vf), rank=np.concatenate([[1], ranks]),
                          cap=np.full(nb + 1, c), u_off=np.concatenate([[0], 5 + np.arange(nb) * c * m]),
                          v_off=np.concatenate([[0], 5 + np.arange(nb) * c * n]))
    pos = np.arange(1, nb + 1)
    rel = np.array([0, 1, 3, 4])
    X, Y = builder._pack_factors(res, pos, rel, m, n)
    kp = 3
    assert X.shape == (4, m, kp) and Y.shape == (4, n, kp)
    for q, r in enumerate(rel):
        k = ranks[r]
        assert np.array_equal(X[q, :, :k], U[r, :k, :].T)
        assert np.array_equal(Y[q, :, :k], np.conj(V[r, :k, :]).T)
        assert np.all(X[q, :, k:] == 0) and np.all(Y[q, :, k:] == 0)


def test_memory_ratio_soft_check():
    """A soft check against the paper's Tables 1-2, not parity: the UH form stores less than
    the H form of the same operator, total memory H/UH within the paper's 1.3-2.7x.  The
    admissible part's ratio (paper: 2.0-3.9x) comes out lower here, 1.6-1.8x, with tolerances
    1e-6 (the paper's experiments use 1e-4) and point clouds."""
    cloud = inputs.make_cloud("sphere", 16384, seed=0)
    op = builder.build_operator(cloud, leaf=64, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
    st = op.stats()
    ratio = st["bytes_h_c128"] / st["bytes_uh_c128"]
    adm = (op.X.size + op.Y.size) / (op.U.size + op.V.size + op.S.size)
    assert 1.3 <= ratio <= 2.7
    assert adm > 1.0


def test_recompression_by_cholesky_qr():
    """builder._recompress_gpu (Cholesky QR of the column-scaled ACA factors, twice, then the
    SVD of the small core), run with CPU tensors, against the Householder-QR recompression of
    the same factors: the same ranks, and U Sigma V^* equal to 1e-12 of |X Y^*|."""
    import torch
    cloud = inputs.make_cloud("cube", 3000, seed=1)
    tree = builder.build_tree(cloud.points, 64)
    pts = np.ascontiguousarray(cloud.points[tree.perm])
    adm, _ = builder.build_block_tree(tree, 1.0)
    low = adm[adm[:, 0] < adm[:, 1]]
    shape = np.stack([tree.size[low[:, 0]], tree.size[low[:, 1]]], 1)
    m, n = (int(v) for v in shape[0])
    sel = low[(shape[:, 0] == m) & (shape[:, 1] == n)][:40]
    lib = builder._native()
    facs = []
    for t, s in sel:
        X = np.empty((m, 64), np.complex128)
        Y = np.empty((n, 64), np.complex128)
        k = lib.uhmb_aca_block(builder._ptr(pts), cloud.kappa, 1.0 / (2 * cloud.h), int(tree.off[t]), m,
                               int(tree.off[s]), n, 1e-6, 64, builder._ptr(X), builder._ptr(Y))
        facs.append((X[:, :k].copy(), Y[:, :k].copy()))
    ranks = np.array([f[0].shape[1] for f in facs])
    kp = int(ranks.max())
    Xb = np.zeros((len(facs), m, kp), np.complex128)
    Yb = np.zeros((len(facs), n, kp), np.complex128)
    for c, (X, Y) in enumerate(facs):
        Xb[c, :, :X.shape[1]] = X
        Yb[c, :, :Y.shape[1]] = Y
    got = builder._recompress_gpu(torch.from_numpy(Xb), torch.from_numpy(Yb), ranks, 1e-7, device="cpu")
    for (X, Y), (Ub, sb, Vb) in zip(facs, got):
        QX, RX = np.linalg.qr(X)
        QY, RY = np.linalg.qr(Y)
        W, sv, Zh = np.linalg.svd(RX @ RY.conj().T)
        r = max(1, int(np.count_nonzero(sv > 1e-7 * sv[0])))
        ref = (QX @ W[:, :r]) * sv[:r] @ (QY @ Zh[:r].conj().T).conj().T
        assert sb.size == r
        assert np.linalg.norm(Ub.conj().T @ Ub - np.eye(r)) < 1e-13
        assert np.linalg.norm((Ub * sb) @ Vb.conj().T - ref) <= 1e-12 * np.linalg.norm(X @ Y.conj().T)


def test_gram_compression_with_cpu_tensors():
    """The Gram-matrix form of Alg. 2's per-cluster step (compress_on="gpu"), run with CPU
    tensors: both of its branches (n_tau <= K and n_tau > K occur on this cloud) give the
    SVD route's ranks, meet the builder's pins, and the same product to 1e-9."""
    cloud = inputs.make_cloud("cube", 3000, seed=0)
    h = builder.build_operator(cloud, leaf=32, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
    g = builder.build_operator(cloud, leaf=32, eta=1.0, eps_aca=1e-6, eps_comp=1e-6, compress_on="gpu",
                               compress_device="cpu")
    has = g.rank_row > 0
    kt = np.bincount(g.adm_row, weights=g.adm_rank, minlength=g.nclusters)
    kmax = {int(sz): int(kt[has & (g.size == sz)].max()) for sz in np.unique(g.size[has])}   # a group's width
    assert any(sz <= k for sz, k in kmax.items()) and any(sz > k for sz, k in kmax.items())
    assert np.array_equal(g.rank_row, h.rank_row)
    for fn in (test_orthogonal_bases_and_conjugate_symmetry, test_couplings_are_optimal,
               test_theorem_5_1_and_frobenius_identity, test_algorithm_1_and_2_give_the_same_basis):
        fn((cloud, g))
    x = inputs.make_rhs(cloud.n, 2, seed=1)
    assert rel(uniform.uh_mvp(vars(g), x), uniform.uh_mvp(vars(h), x)) <= 1e-9
