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
