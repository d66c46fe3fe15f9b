"""Alg. 2's per-cluster factorisation on the GPU (uhm_cluster_basis, section 4.2).

Pins independent of both sides:
* matrices built as Q1 diag(s) Q2^* with orthonormal Q1, Q2 have the singular values s
  (a closed form), so the rank at eps * s_1 is known; the s are spaced so that none lies
  within 1e-6 of the threshold;
* Eckart-Young: the best rank-l projection error is s_{l+1} in the 2-norm and
  sqrt(sum_{i>l} s_i^2) in the Frobenius norm;
* U orthonormal and Sigma V^* = U^* X.
On the builder's own cluster matrices the GPU bases are checked against the oracle's
Alg. 1 (the SVD of the agglomerated block row of the assembled H-matrix): same ranks and
the optimal projection error.

The recompression of ACA factors (uhm_block_recompress, section 2.3) is pinned the same
way: X = Q1 diag(s) G and Y = Q2 G^{-*} with G invertible give X Y^* = Q1 diag(s) Q2^*, whose
truncated SVD is known in closed form.
"""
import numpy as np
import pytest

from conftest import operator
from oracle import uniform

pytestmark = pytest.mark.gpu


def _binding():
    from paper_2405_15573_amd import binding
    return binding


def _prescribed(rng, m, n, s):
    k = s.size
    q1, _ = np.linalg.qr(rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k)))
    q2, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    return (q1 * s) @ q2.conj().T


def _decay(k, ratio, jitter, rng):
    """Geometric singular values with a random jitter, none within 1e-3 (relative) of 1e-6."""
    s = ratio ** np.arange(k) * np.exp(jitter * rng.uniform(-1, 1, k))
    s = np.sort(s)[::-1] / s.max()
    near = np.abs(s / 1e-6 - 1.0) < 1e-3
    s[near] *= 1.01
    return np.sort(s)[::-1]


def _check(X, res, c, eps, s_true=None):
    m, n = X.shape
    U, SV = res.basis(c)
    l = int(res.rank[c])
    assert res.status[c] == 0
    s_ref = np.linalg.svd(X, compute_uv=False) if s_true is None else s_true
    l_ref = max(1, int(np.count_nonzero(s_ref > eps * s_ref[0]))) if s_ref[0] > 0 else 1
    assert l == l_ref
    assert U.shape == (m, l) and SV.shape == (l, n)
    # rounding: Householder QR and Jacobi are backward stable with errors of order
    # eps_mach sqrt(m n) |X| (absolute, in the singular values and the projections), and
    # Gram-Schmidt applied twice leaves about eps_mach per entry of U^* U - I
    emach = np.finfo(float).eps
    ab = max(1e-13, 4 * emach * np.sqrt(m * n)) * s_ref[0]
    assert np.linalg.norm(U.conj().T @ U - np.eye(l)) < max(1e-13, 2 * emach * l)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(SV - U.conj().T @ X) <= 1e-13 * max(nx, 1e-300)
    sv = res.sv.cpu().numpy()[c]
    p = int(res.psteps[c])
    # sigma_i(B)^2 <= sigma_i(X)^2 <= sigma_i(B)^2 + T^2: at and above 1e-9 sigma_1 the two agree
    # to rounding
    kk = int(np.count_nonzero(s_ref[:p] >= 1e-9 * s_ref[0]))
    assert np.all(np.abs(sv[:kk] - s_ref[:kk]) <= ab + 1e-300)
    assert np.all(sv[:p] <= s_ref[:p] * (1 + 1e-13) + ab)
    best2 = s_ref[l] if l < s_ref.size else 0.0
    assert np.linalg.norm(X - U @ SV, 2) <= best2 * (1 + 1e-6) + ab
    bestF = np.sqrt(np.sum(s_ref[l:] ** 2))
    assert abs(res.stats[c, 0] - bestF) <= 1e-6 * bestF + ab
    assert abs(res.stats[c, 1] - best2) <= 1e-6 * best2 + ab
    assert res.stats[c, 2] <= np.sqrt(1e-16 * eps) * nx * (1 + 1e-12)


@pytest.mark.parametrize("m,n,ratio", [(200, 300, 0.9), (300, 120, 0.85), (64, 250, 0.8), (1024, 700, 0.93),
                                       (130, 70, 0.7), (1024, 900, 0.97), (1300, 1300, 0.985)])
def test_prescribed_singular_values(m, n, ratio):
    rng = np.random.default_rng(m * 7 + n)
    batch = 3
    k = min(m, n)
    Xs, ss = [], []
    for c in range(batch):
        s = _decay(k, ratio, 0.2, rng)
        ss.append(s)
        Xs.append(_prescribed(rng, m, n, s))
    res = _binding().cluster_basis(np.stack(Xs), eps=1e-6)
    # the Jacobi orders span both of its forms: all sweeps in LDS (orders up to 64) and one
    # launch per round of the circle schedule (above)
    print(f"  QR steps p = {res.psteps.tolist()}", flush=True)
    for c in range(batch):
        _check(Xs[c], res, c, 1e-6, ss[c])


@pytest.mark.parametrize("m,n,ratio", [(16384, 64, 0.8), (9000, 120, 0.85), (2048, 2048, 0.987)])
def test_maximum_sizes(m, n, ratio):
    """The largest shapes the entry point takes: 16384 rows (the widest QR-step and
    reflector kernels, above 8192 rows), and singular values decaying as 0.987^i, whose QR
    reaches the tolerance 1e-11 only after about 2030 steps: a Jacobi order near pmax's
    limit of 2048."""
    rng = np.random.default_rng(m + 3 * n)
    batch = 2
    k = min(m, n)
    ss = [_decay(k, ratio, 0.2, rng) for _ in range(batch)]
    Xs = [_prescribed(rng, m, n, s) for s in ss]
    res = _binding().cluster_basis(np.stack(Xs), eps=1e-6)
    print(f"  QR steps p = {res.psteps.tolist()}", flush=True)
    for c in range(batch):
        _check(Xs[c], res, c, 1e-6, ss[c])


def test_ragged_batch_with_zero_padding_and_edge_cases():
    """Matrices of one batch with different column counts (zero columns pad them, as the
    builder pads a group of clusters), a zero matrix, and an exact rank-1 matrix."""
    rng = np.random.default_rng(5)
    m, n = 96, 160
    Xs = []
    for kc in (160, 97, 33, 1):
        s = _decay(min(m, kc), 0.85, 0.1, rng)
        X = np.zeros((m, n), complex)
        X[:, :kc] = _prescribed(rng, m, kc, s)
        Xs.append(X)
    Xs.append(np.zeros((m, n), complex))
    u = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Xs.append(np.outer(u, v.conj()))
    res = _binding().cluster_basis(np.stack(Xs), eps=1e-6)
    for c in range(4):
        _check(Xs[c], res, c, 1e-6)
    # the zero matrix: rank 1, a unit vector, zero rows and zero error
    U, SV = res.basis(4)
    assert res.rank[4] == 1 and res.psteps[4] == 0 and res.status[4] == 0
    assert abs(np.linalg.norm(U) - 1.0) < 1e-15 and np.all(SV == 0) and np.all(res.stats[4] == 0)
    # rank 1: one QR step reaches the tolerance
    _check(Xs[5], res, 5, 1e-6)
    assert res.rank[5] == 1 and res.psteps[5] == 1


def test_looser_tolerance_keeps_the_rank_test():
    """The trailing part left by the QR is orthogonal to the kept range, so a singular value
    at the threshold moves by T^2 / (2 eps sigma_1) only: tol = 1e-11 gives the ranks,
    thresholds and projection errors of tol = 1e-14 with fewer QR steps."""
    rng = np.random.default_rng(21)
    X = np.stack([_prescribed(rng, 400, 500, _decay(400, 0.93, 0.2, rng)) for _ in range(3)])
    a = _binding().cluster_basis(X, eps=1e-6, tol=1e-14)
    b = _binding().cluster_basis(X, eps=1e-6, tol=1e-11)
    assert np.array_equal(a.rank, b.rank)
    assert np.all(b.psteps < a.psteps)
    for c in range(3):
        _check(X[c], b, c, 1e-6)
        l = int(a.rank[c])
        assert np.all(np.abs(b.sv.cpu().numpy()[c][:l + 1] - a.sv.cpu().numpy()[c][:l + 1])
                      <= 1e-13 * a.sv.cpu().numpy()[c][0])


def test_capacity_flag():
    """pmax below the QR rank at the tolerance is reported in status bit 0."""
    rng = np.random.default_rng(11)
    X = _prescribed(rng, 120, 150, _decay(120, 0.95, 0.0, rng))
    res = _binding().cluster_basis(X[None], eps=1e-6, pmax=40)
    assert res.status[0] & 1 and res.psteps[0] == 40


def test_rejects_bad_arguments():
    b = _binding()
    with pytest.raises(b.UhmError):
        b.cluster_basis(np.zeros((1, 8, 8), complex), eps=1e-6, pmax=9)
    with pytest.raises(b.UhmError):
        b.cluster_basis(np.zeros((1, 8, 8), complex), eps=-1.0)


def test_builder_clusters_match_algorithm_1():
    """The GPU factorisation of the builder's thin factors X_tau gives Alg. 1's ranks and
    optimal projection error on the assembled H-matrix (the oracle)."""
    _, op = operator("sphere", 3000, leaf=32, seed=3)
    o = vars(op)
    ah = uniform.assemble_h(o)
    b = _binding()
    checked = 0
    for t in np.nonzero(op.rank_row)[0][::7]:
        t = int(t)
        nt = int(op.size[t])
        blocks = [q for q in range(op.nadm) if int(op.adm_row[q]) == t]
        X = np.concatenate([op.X[op.X_off[q]:op.X_off[q] + nt * op.adm_rank[q]].reshape(op.adm_rank[q], nt).T
                            for q in blocks], 1)
        u1, sv = uniform.optimal_row_basis(ah, o, t, op.eps_comp)
        if np.any(np.abs(sv - op.eps_comp * sv[0]) < 1e-9 * sv[0]):
            continue  # a singular value on the threshold: the rank is rounding-dependent
        res = b.cluster_basis(X[None], eps=op.eps_comp)
        assert res.status[0] == 0
        l = int(res.rank[0])
        assert l == u1.shape[1]
        U, _ = res.basis(0)
        assert np.linalg.norm(U.conj().T @ U - np.eye(l)) < 1e-13
        cols = [int(op.adm_col[q]) for q in blocks]
        rows = op.perm[op.off[t]:op.off[t] + nt]
        at = np.concatenate([ah[np.ix_(rows, op.perm[op.off[s]:op.off[s] + op.size[s]])] for s in cols], 1)
        err = np.linalg.norm(at - U @ (U.conj().T @ at), 2)
        best = sv[l] if l < sv.size else 0.0
        assert err <= best * (1 + 1e-6) + 1e-13 * sv[0]
        checked += 1
    assert checked >= 8


def _factor_pair(rng, m, n, s, cond=10.0):
    """X, Y with X Y^* = Q1 diag(s) Q2^* and a mixing G of condition number about cond."""
    k = s.size
    q1, _ = np.linalg.qr(rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k)))
    q2, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    a, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    b, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    g = (a * np.geomspace(1.0, 1.0 / cond, k)) @ b
    return (q1 * s) @ g, q2 @ np.linalg.inv(g).conj().T


def _check_rec(X, Y, U, V, sv, k, eps, s_true):
    A = X @ Y.conj().T
    m, kp = X.shape
    n = Y.shape[0]
    k_ref = max(1, int(np.count_nonzero(s_true > eps * s_true[0]))) if s_true[0] > 0 else 1
    assert k == k_ref
    Uk, Vk = U[:, :k], V[:, :k]
    # rounding, as for the cluster factorisation: eps_mach sqrt(rows kp) |X Y^*| from the
    # QRs of the factors, eps_mach k in the Gram matrices of the twice-orthogonalised sets
    emach = np.finfo(float).eps
    ab = max(1e-12, 4 * emach * np.sqrt(max(m, n) * kp)) * s_true[0]
    orth = max(1e-13, 2 * emach * k)
    assert np.linalg.norm(Uk.conj().T @ Uk - np.eye(k)) < orth
    assert np.linalg.norm(Vk.conj().T @ Vk - np.eye(k)) < orth
    kk = min(s_true.size, sv.size)
    assert np.all(np.abs(sv[:kk] - s_true[:kk]) <= ab)
    best = s_true[k] if k < s_true.size else 0.0
    assert np.linalg.norm(A - (Uk * sv[:k]) @ Vk.conj().T, 2) <= best * (1 + 1e-6) + ab


@pytest.mark.parametrize("m,n,k", [(64, 64, 20), (128, 256, 37), (300, 200, 64), (1024, 512, 90)])
def test_recompression_prescribed(m, n, k):
    rng = np.random.default_rng(m + n + k)
    batch = 4
    eps = 1e-7
    Xs, Ys, ss = [], [], []
    for c in range(batch):
        kc = k - 3 * c   # ragged ranks: zero columns pad the shorter factors
        s = _decay(kc, 0.7, 0.2, rng)
        X, Y = _factor_pair(rng, m, n, s)
        Xp = np.zeros((m, k), complex)
        Yp = np.zeros((n, k), complex)
        Xp[:, :kc], Yp[:, :kc] = X, Y
        Xs.append(Xp)
        Ys.append(Yp)
        ss.append(s)
    U, V, sv, rk, st = _binding().block_recompress(np.stack(Xs), np.stack(Ys), eps)
    assert np.all(st == 0)
    U, V, sv = U.cpu().numpy(), V.cpu().numpy(), sv.cpu().numpy()
    for c in range(batch):
        _check_rec(Xs[c], Ys[c], U[c].T, V[c].T, sv[c], int(rk[c]), eps, ss[c])


@pytest.mark.parametrize("m,n,k,ratio", [(16384, 200, 40, 0.7), (200, 16384, 40, 0.7), (2048, 2048, 2048, 0.99)])
def test_recompression_maximum_sizes(m, n, k, ratio):
    """The largest shapes: 16384 rows on either factor (the widest QR-step and reflector
    kernels), and kp = 2048 (the largest Jacobi order; 0.99^i keeps every singular value
    above the underflow, and about 1600 of them above eps = 1e-7)."""
    rng = np.random.default_rng(m + 2 * n + k)
    batch = 1 if k > 100 else 2
    eps = 1e-7
    ss = [_decay(k, ratio, 0.2, rng) for _ in range(batch)]
    pairs = [_factor_pair(rng, m, n, s) for s in ss]
    X = np.stack([p[0] for p in pairs])
    Y = np.stack([p[1] for p in pairs])
    U, V, sv, rk, st = _binding().block_recompress(X, Y, eps)
    print(f"  ranks {rk.tolist()}", flush=True)
    assert np.all(st == 0)
    U, V, sv = U.cpu().numpy(), V.cpu().numpy(), sv.cpu().numpy()
    for c in range(batch):
        _check_rec(X[c], Y[c], U[c].T, V[c].T, sv[c], int(rk[c]), eps, ss[c])


def test_recompression_degenerate_blocks():
    """A zero block (rank 1, sigma 0) and an exact rank-1 block in one batch."""
    rng = np.random.default_rng(8)
    m, n, k = 80, 50, 6
    X = np.zeros((2, m, k), complex)
    Y = np.zeros((2, n, k), complex)
    X[1, :, 0] = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    Y[1, :, 0] = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    U, V, sv, rk, st = _binding().block_recompress(X, Y, 1e-7)
    sv = sv.cpu().numpy()
    assert np.all(st == 0) and rk[0] == 1 and rk[1] == 1 and np.all(sv[0] == 0)
    assert abs(sv[1, 0] - np.linalg.norm(X[1, :, 0]) * np.linalg.norm(Y[1, :, 0])) <= 1e-13 * sv[1, 0]
    u, v = U.cpu().numpy()[1, 0], V.cpu().numpy()[1, 0]
    assert np.linalg.norm(np.outer(u * sv[1, 0], v.conj()) - X[1] @ Y[1].conj().T) <= 1e-13 * sv[1, 0]



def test_couplings_against_their_formulas():
    """uhm_couplings: S_X = L_t Sigma^{-1}, S_Y = conj(L_s), S = S_X L_s^T for blocks reading
    shared coefficient rows at arbitrary offsets; a descriptor outside the buffers is rejected."""
    import torch
    b = _binding()
    rng = np.random.default_rng(4)
    L = rng.standard_normal(5000) + 1j * rng.standard_normal(5000)
    sig = rng.uniform(0.5, 2.0, 200)
    shapes = [(7, 5, 3), (1, 1, 1), (30, 12, 9), (16, 16, 16)]
    desc = np.zeros(len(shapes), b.COUPLING_DTYPE)
    so = xo = yo = 0
    for q, (lt, ls, kb) in enumerate(shapes):
        desc[q] = (37 * q + 11, 900 + 53 * q, 17 * q, so, xo, yo, lt, ls, kb, 0)
        so, xo, yo = so + lt * ls, xo + lt * kb, yo + ls * kb
    Ld = torch.from_numpy(L).to("cuda")
    S, SX, SY = (t.cpu().numpy() for t in b.couplings(Ld, sig, desc, so, xo, yo))
    for d in desc:
        lt, ls, kb = int(d["lt"]), int(d["ls"]), int(d["kb"])
        A = L[d["a_off"]:d["a_off"] + kb * lt].reshape(kb, lt).T
        B = L[d["b_off"]:d["b_off"] + kb * ls].reshape(kb, ls).T
        sx = A / sig[d["sig_off"]:d["sig_off"] + kb][None, :]
        assert np.allclose(SX[d["x_off"]:d["x_off"] + lt * kb].reshape(kb, lt).T, sx, rtol=1e-15, atol=0)
        assert np.array_equal(SY[d["y_off"]:d["y_off"] + ls * kb].reshape(kb, ls).T, np.conj(B))
        assert np.allclose(S[d["s_off"]:d["s_off"] + lt * ls].reshape(ls, lt).T, sx @ B.T, rtol=1e-13, atol=1e-13)
    bad = desc.copy()
    bad[2]["a_off"] = 5000 - 10   # runs past the end of L
    with pytest.raises(b.UhmError):
        b.couplings(Ld, sig, bad, so, xo, yo)
