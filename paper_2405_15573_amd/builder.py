"""Host-side builder: point cloud -> H-matrix -> uniform H-matrix (UH-matrix).

Steps, in the paper's order:

1. Cluster tree (Definition 2.1): geometric bisection of the longest bounding-box axis at
   the median position, to a fixed depth D = ceil(log2(N/leaf)), so that every leaf sits
   at depth D and holds at most ``leaf`` points.  The children of a cluster partition it
   and are contiguous in cluster order (``perm`` maps cluster order to user order).
2. Block cluster tree (Definition 2.2) with the level-conserving subdivision
   s(tau x sigma) = s(tau) x s(sigma) and the weak admissibility condition
   eta * dist(tau, sigma) > min(diam tau, diam sigma) (section 3.2), with diameters and
   distances measured on axis-aligned bounding boxes (section 6.1).  Inadmissible leaf
   pairs are stored dense.
3. Admissible blocks: ACA with partial pivoting (section 2.3), then algebraic
   recompression A|_b ~ U_b Sigma_b V_b^* from the QRs of both factors and the SVD of the
   small core (section 2.3), truncated relative to the block's largest singular value.
4. Uniform compression (Algorithm 2 with the agglomeration X_{tau|b} = U_b Sigma_b that
   section 4.3 uses): per row cluster, the SVD of X_tau = [U_b Sigma_b]_{sigma in row(tau)}
   gives U_tau (leading left singular vectors above the relative tolerance) and
   U_tau^* U_b Sigma_b = (Sigma V^*)[:l_tau, cols of b].  The coupling matrix is assembled,
   S_b = (U_tau^* U_b Sigma_b) Sigma_b^{-1} (V_sigma^* V_b Sigma_b)^*, and stored whole.
5. Symmetry (Remark 4.4, used in section 6.1): the kernel is symmetric and the rows and
   columns share one tree, so ACA runs on one block of each mirrored pair and the mirrored
   block is its transpose exactly.  Then the column agglomeration of a cluster is the
   complex conjugate of its row agglomeration and V_sigma = conj(U_sigma).  The stored
   operator still carries both triangles and separate U and V, as a general UH-matrix.

The result is a ``HostOperator`` holding both the H form (for the H-MVP comparator) and
the UH form, in the flat, cluster-ordered layout declared in ``include/uhm.h``.

Where the work runs (build_operator's options): the matrix sampling (ACA and the near
field) on the host (OpenMP C++) or on the GPU (uhm_aca, uhm_kernel_blocks); the
recompression on the host (LAPACK QR and SVD) or with its tall products on the GPU
(Cholesky QR); the uniform compression on the host (LAPACK SVD per cluster) or with its
large products on the GPU (the Gram-matrix form of the same subspace).

build_uniform_direct is the direct construction of Algs. 3-4 (section 4.3) with one lock
per block (section 4.4): blocks are approximated on demand and dropped once both of their
clusters have used them, so the H form is never held whole.
"""
from __future__ import annotations

import ctypes
import math
import os
import sys
import time
from dataclasses import dataclass, field

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .inputs import PointCloud

try:  # keep LAPACK single-threaded inside the worker threads
    from threadpoolctl import threadpool_limits
except ImportError:  # pragma: no cover
    threadpool_limits = None

_LIB = None


def _native():
    global _LIB
    if _LIB is None:
        # UHM_BUILDER_LIB selects another build of the same source (a sanitizer build)
        path = os.environ.get("UHM_BUILDER_LIB") or os.path.join(os.path.dirname(__file__), "libuhm_builder.so")
        if not os.path.exists(path):
            raise RuntimeError(
                f"builder library {path} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.uhmb_dense_blocks.argtypes = [P, D, D, I64, P, P, P, P, P, P]
        lib.uhmb_dense_blocks.restype = ctypes.c_int
        lib.uhmb_aca_run.argtypes = [P, D, D, I64, P, P, P, P, D, I32, P]
        lib.uhmb_aca_run.restype = ctypes.c_void_p
        lib.uhmb_aca_copy.argtypes = [P, I64, P, I64, I64, I64, P, P]
        lib.uhmb_aca_copy.restype = ctypes.c_int
        lib.uhmb_aca_free.argtypes = [P]
        lib.uhmb_aca_free.restype = None
        lib.uhmb_aca_block.argtypes = [P, D, D, I64, I64, I64, I64, D, I32, P, P]
        lib.uhmb_aca_block.restype = I32
        lib.uhmb_num_threads.argtypes = []
        lib.uhmb_num_threads.restype = ctypes.c_int
        lib.uhmb_scaled_copy.argtypes = [P, I64]
        lib.uhmb_scaled_copy.restype = ctypes.c_int
        _LIB = lib
    return _LIB


# one record of uhmb_scaled_copy: dst[i drs + q dcs] = f(src[i srs + q scs]) * scale[q]
# (byte addresses, strides in complex elements; f = conj when conj != 0)
COPY_DTYPE = np.dtype([("src", np.uint64), ("dst", np.uint64), ("scale", np.uint64), ("srs", np.int64),
                       ("scs", np.int64), ("drs", np.int64), ("dcs", np.int64), ("rows", np.int32),
                       ("cols", np.int32), ("conj", np.int32), ("pad", np.int32)])


def _scaled_copy(recs):
    """Run uhmb_scaled_copy over a list of COPY_DTYPE tuples (the GIL is released meanwhile)."""
    if not recs:
        return
    arr = np.array(recs, dtype=COPY_DTYPE)
    _native().uhmb_scaled_copy(_ptr(arr), len(arr))


def _view(a: np.ndarray, dtype=np.complex128):
    """(address, row stride, column stride) of a 2-D array, strides in elements; a copy is
    returned beside them when the array is not of that type or its strides are not whole
    elements (the caller keeps it alive)."""
    item = np.dtype(dtype).itemsize
    if a.dtype != dtype or any(st % item for st in a.strides):
        a = np.ascontiguousarray(a, dtype=dtype)
    st = a.strides
    return a.__array_interface__["data"][0], st[0] // item, (st[1] // item if a.ndim > 1 else 0), a


def _row_records(part, row_blocks, factor_views, base: int, nt: int, kp: int):
    """uhmb_scaled_copy records that write the cluster matrices of part (a list of (tau, .))
    as a row-major batch at byte address base, nt x kp each: X_tau = [U_b Sigma_b ...] over
    tau's block row, conj(V_b) Sigma_b for a mirrored block (s, tau), zero columns after.
    factor_views(key) gives a stored block's addresses and strides (as in build_operator).
    Returns the records and, per cluster, its (s, first column, k_b) list."""
    recs, cols = [], []
    for c, (t, _) in enumerate(part):
        j, cl = 0, []
        row0 = base + 16 * c * nt * kp
        for s in row_blocks[t]:
            if t < s:
                ua, urs, ucs, _, _, _, sa, kb, _ = factor_views((t, s))
                recs.append((ua, row0 + 16 * j, sa, urs, ucs, kp, 1, nt, kb, 0, 0))
            else:
                _, _, _, va, vrs, vcs, sa, kb, _ = factor_views((s, t))
                recs.append((va, row0 + 16 * j, sa, vrs, vcs, kp, 1, nt, kb, 1, 0))
            cl.append((s, j, kb))
            j += kb
        if j < kp:
            recs.append((0, row0 + 16 * j, 0, 0, 0, kp, 1, nt, kp - j, 0, 0))
        cols.append(cl)
    return recs, cols


def _hfactor_records(adm, adm_rank, size, X_off, Y_off, xa0: int, ya0: int, factor_views):
    """uhmb_scaled_copy records for the H-matrix factors of every admissible block b = (t, s):
    X_b = U_b Sigma_b and Y_b = V_b, column-major at element offsets X_off[b], Y_off[b] of
    the arrays at byte addresses xa0, ya0; the mirror of a stored block (s, t) has
    U_b = conj(V), V_b = conj(U)."""
    recs = []
    for b in range(adm.shape[0]):
        t, s = int(adm[b, 0]), int(adm[b, 1])
        kb, mt, ms = int(adm_rank[b]), int(size[t]), int(size[s])
        xa, ya = xa0 + 16 * int(X_off[b]), ya0 + 16 * int(Y_off[b])
        if t < s:
            ua, urs, ucs, va, vrs, vcs, sa, _, _ = factor_views((t, s))
            recs.append((ua, xa, sa, urs, ucs, 1, mt, mt, kb, 0, 0))
            recs.append((va, ya, 0, vrs, vcs, 1, ms, ms, kb, 0, 0))
        else:
            ua, urs, ucs, va, vrs, vcs, sa, _, _ = factor_views((s, t))
            recs.append((va, xa, sa, vrs, vcs, 1, mt, mt, kb, 1, 0))
            recs.append((ua, ya, 0, urs, ucs, 1, ms, ms, kb, 1, 0))
    return recs


def _factor_views_of(fac_U, fac_V, fac_s):
    """factor_views(key) over the stored blocks' factors: (U address, row stride, column
    stride, the same for V, Sigma address, k_b, kept arrays), made once per block."""
    views = {}

    def factor_views(key):
        v = views.get(key)
        if v is None:
            ua, urs, ucs, uk = _view(fac_U[key])
            va, vrs, vcs, vk = _view(fac_V[key])
            sv = np.ascontiguousarray(fac_s[key], dtype=np.float64)
            v = (ua, urs, ucs, va, vrs, vcs, sv.__array_interface__["data"][0], int(sv.size), (uk, vk, sv))
            views[key] = v
        return v

    return factor_views


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------- tree
@dataclass
class ClusterTree:
    perm: np.ndarray    # (N,) int64: cluster position -> user index
    off: np.ndarray     # (nc,) int64
    size: np.ndarray    # (nc,) int64
    level: np.ndarray   # (nc,) int32
    parent: np.ndarray  # (nc,) int32, -1 at the root
    child: np.ndarray   # (nc, 2) int32, -1 at leaves
    lo: np.ndarray      # (nc, 3) bounding box
    hi: np.ndarray
    depth: int          # D: leaves are at level D

    @property
    def nclusters(self) -> int:
        return int(self.off.shape[0])

    def diam(self) -> np.ndarray:
        return np.linalg.norm(self.hi - self.lo, axis=1)

    def leaves(self) -> np.ndarray:
        return np.nonzero(self.child[:, 0] < 0)[0]


def build_tree(points: np.ndarray, leaf: int) -> ClusterTree:
    n = points.shape[0]
    if leaf < 2:
        raise ValueError("leaf size must be >= 2")
    depth = max(0, math.ceil(math.log2(n / leaf))) if n > leaf else 0
    perm = np.arange(n, dtype=np.int64)
    off, size, level, parent = [0], [n], [0], [-1]
    child = [[-1, -1]]
    current = [0]
    for lev in range(depth):
        nxt = []
        for c in current:
            o, s = off[c], size[c]
            idx = perm[o:o + s]
            p = points[idx]
            ax = int(np.argmax(p.max(0) - p.min(0)))
            order = np.lexsort((idx, p[:, ax]))
            perm[o:o + s] = idx[order]
            m = s // 2
            kids = []
            for co, cs in ((o, m), (o + m, s - m)):
                kids.append(len(off))
                off.append(co)
                size.append(cs)
                level.append(lev + 1)
                parent.append(c)
                child.append([-1, -1])
            child[c] = kids
            nxt.extend(kids)
        current = nxt
    off_a = np.asarray(off, np.int64)
    size_a = np.asarray(size, np.int64)
    sorted_pts = points[perm]
    # bounding boxes from the cluster-ordered points (reduceat over contiguous segments)
    lo = np.empty((len(off), 3))
    hi = np.empty((len(off), 3))
    for c in range(len(off)):
        seg = sorted_pts[off_a[c]:off_a[c] + size_a[c]]
        lo[c] = seg.min(0)
        hi[c] = seg.max(0)
    return ClusterTree(perm, off_a, size_a, np.asarray(level, np.int32), np.asarray(parent, np.int32),
                       np.asarray(child, np.int32), lo, hi, depth)


def build_block_tree(tree: ClusterTree, eta: float):
    """Return (adm, den): int32 arrays of (row cluster, column cluster) leaf pairs."""
    diam = tree.diam()
    pairs = np.zeros((1, 2), np.int64)
    adm_parts, den_parts = [], []
    while pairs.shape[0]:
        t, s = pairs[:, 0], pairs[:, 1]
        gap = np.maximum(0.0, np.maximum(tree.lo[t] - tree.hi[s], tree.lo[s] - tree.hi[t]))
        dist = np.linalg.norm(gap, axis=1)
        adm = eta * dist > np.minimum(diam[t], diam[s])
        adm_parts.append(pairs[adm])
        rest = pairs[~adm]
        leaf_t = tree.child[rest[:, 0], 0] < 0
        leaf_s = tree.child[rest[:, 1], 0] < 0
        stop = leaf_t | leaf_s
        den_parts.append(rest[stop])
        rest = rest[~stop]
        ct = tree.child[rest[:, 0]]
        cs = tree.child[rest[:, 1]]
        pairs = np.concatenate([np.stack([ct[:, a], cs[:, b]], 1) for a in (0, 1) for b in (0, 1)], 0) \
            if rest.shape[0] else np.zeros((0, 2), np.int64)
    adm = np.concatenate(adm_parts, 0).astype(np.int64)
    den = np.concatenate(den_parts, 0).astype(np.int64)
    adm = adm[np.lexsort((adm[:, 1], adm[:, 0]))]
    den = den[np.lexsort((den[:, 1], den[:, 0]))]
    return adm, den


# --------------------------------------------------------------------------- operator
@dataclass
class HostOperator:
    """Both forms of one operator in the flat, cluster-ordered host layout.

    Complex arrays are complex128 and flat; every per-cluster or per-block matrix is
    column-major at its element offset.
    """
    n: int
    perm: np.ndarray
    off: np.ndarray
    size: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    rank_row: np.ndarray   # int32, l_tau (0 if tau not in L'_I)
    rank_col: np.ndarray   # int32, l_sigma (0 if sigma not in L'_J)
    U_off: np.ndarray      # int64, -1 if no basis
    V_off: np.ndarray
    U: np.ndarray
    V: np.ndarray
    adm_row: np.ndarray    # int32
    adm_col: np.ndarray
    S_off: np.ndarray      # int64
    S: np.ndarray
    adm_rank: np.ndarray   # int32, k_b of the H form
    X_off: np.ndarray      # int64
    Y_off: np.ndarray
    X: np.ndarray          # H form: A|_b ~ X_b Y_b^*, X_b = U_b Sigma_b, Y_b = V_b
    Y: np.ndarray
    den_row: np.ndarray
    den_col: np.ndarray
    D_off: np.ndarray
    D: np.ndarray
    kappa: float
    h: float
    leaf: int
    eta: float
    eps_aca: float
    eps_comp: float
    depth: int
    SX_off: np.ndarray = field(default=None)       # factored couplings S_b = S_{X,b} S_{Y,b}^*:
    SY_off: np.ndarray = field(default=None)       # S_{X,b} l_tau x k_b at SX_off[b],
    SX: np.ndarray = field(default=None)           # S_{Y,b} l_sigma x k_b at SY_off[b]
    SY: np.ndarray = field(default=None)
    sv_dropped: np.ndarray = field(default=None)   # per cluster: sigma_{l+1}(X_tau) (0 if none)
    sv_tail: np.ndarray = field(default=None)      # per cluster: sqrt(sum_{i>l} sigma_i^2)
    timings: dict = field(default_factory=dict)

    @property
    def nclusters(self) -> int:
        return int(self.off.shape[0])

    @property
    def nadm(self) -> int:
        return int(self.adm_row.shape[0])

    @property
    def nden(self) -> int:
        return int(self.den_row.shape[0])

    def stats(self) -> dict:
        r = self.rank_row[self.rank_row > 0]
        rows = np.bincount(self.adm_row, minlength=self.nclusters)
        cols = np.bincount(self.adm_col, minlength=self.nclusters)
        return {
            "n": self.n, "depth": self.depth, "nclusters": self.nclusters,
            "nadm": self.nadm, "nden": self.nden,
            "c_sp": int(max(rows.max(initial=0), cols.max(initial=0))),
            "l_max": int(r.max(initial=0)), "l_mean": float(r.mean()) if r.size else 0.0,
            "k_max": int(self.adm_rank.max(initial=0)),
            "elems_U": int(self.U.size), "elems_V": int(self.V.size), "elems_S": int(self.S.size),
            "elems_D": int(self.D.size), "elems_XY": int(self.X.size + self.Y.size),
            "bytes_uh_c128": 16 * int(self.U.size + self.V.size + self.S.size + self.D.size),
            "bytes_h_c128": 16 * int(self.X.size + self.Y.size + self.D.size),
        }


def _chunks(items, per_item_bytes, budget=1 << 28, parts=1):
    """Split items into pieces of bounded memory, and into at least ``parts`` pieces."""
    step = max(1, int(budget // max(1, per_item_bytes)))
    step = max(1, min(step, -(-len(items) // max(1, parts))))
    for a in range(0, len(items), step):
        yield items[a:a + step]


def _workers() -> int:
    n = os.environ.get("UHM_BUILD_THREADS") or os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1
    return max(1, min(64, int(n)))


def _pmap(fn, items):
    """Map fn over items on a thread pool, with LAPACK/BLAS pinned to one thread each."""
    items = list(items)
    nw = min(_workers(), len(items))
    if nw <= 1:
        return [fn(x) for x in items]
    ctx = threadpool_limits(1) if threadpool_limits is not None else None
    try:
        if ctx is not None:
            ctx.__enter__()
        with ThreadPoolExecutor(nw) as ex:
            return list(ex.map(fn, items))
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)


def _to_host(t):
    """A device tensor copied to the host through page-locked memory (a DMA at the bus rate
    rather than a staged copy through pageable memory); the numpy array views that memory."""
    import torch
    if t.device.type == "cpu":
        return t.numpy()
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t)
    return h.numpy()


# the largest cluster or block side the GPU factorisations take (uhm_cluster_basis,
# uhm_block_recompress); larger ones are factorised on the host
_GPU_MAX_ROWS = 16384


def _copy_into(dst, src, step=1 << 26):
    """The flat device tensor src into the flat host array dst, through one page-locked
    staging buffer of at most `step` elements and torch's threaded host copy."""
    import torch
    n = int(dst.size)
    if n == 0:
        return
    buf = torch.empty(min(n, step), dtype=src.dtype, pin_memory=True)
    d = torch.from_numpy(dst)
    for a in range(0, n, step):
        b = min(n, a + step)
        buf[:b - a].copy_(src[a:b])
        d[a:b].copy_(buf[:b - a])


def _to_host_copy(t):
    """As _to_host, then copied into pageable memory by torch's threaded host copy, so the
    page-locked block goes back to torch's cache for the next transfer (results that the
    builder keeps for the rest of the build would otherwise pin memory for that long)."""
    import torch
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t)
    out = torch.empty(t.shape, dtype=t.dtype)
    out.copy_(h)
    del h
    return out.numpy()


def _pack_factors(res, pos, rel, m, n, device=False):
    """Factors of the blocks pos[rel] of one shape group of an ACA result (blocks pos are
    contiguous, all m x n): X (cnt, m, kp) = u and Y (cnt, n, kp) = conj(v), zero beyond each
    block's rank, kp the group's largest rank.  Packed on the device by uhm_aca_pack and
    copied to the host once, or kept on the device (device=True)."""
    from . import binding
    rank = res.rank[pos[rel]]
    kp = int(rank.max())
    X, Y = binding.aca_pack(res, np.asarray(pos)[rel], int(m), int(n), kp)
    if device:
        return X, Y
    return _to_host(X), _to_host(Y)


def _aca_level_gpu(dev_pts, kappa, diag, roff, rsz, coff, csz, eps, kcap, first_cap=128, device=False):
    """ACA of one level's blocks on the GPU (uhm_aca).  Blocks whose first pass stopped at
    its rank capacity run again with a four times larger one, up to kcap.  Returns the ranks
    and, per (shape, pass) group, (block indices, X (cnt, m, kp), Y (cnt, n, kp)) with
    A|_b ~ X Y^H and zero columns beyond each block's rank (the layout of uhmb_aca_copy);
    host arrays, or device tensors with device=True."""
    from . import binding
    nb = roff.shape[0]
    kout = np.zeros(nb, np.int32)
    groups = []
    todo = np.arange(nb)
    cap_now = first_cap
    kernel_s = 0.0
    while todo.size:
        order = np.lexsort((csz[todo], rsz[todo]))
        idx = todo[order]
        full = np.minimum(np.minimum(rsz[idx], csz[idx]), kcap)
        caps = np.minimum(full, cap_now)
        tk = time.perf_counter()
        res = binding.aca(dev_pts, kappa, diag, roff[idx], rsz[idx], coff[idx], csz[idx], caps, eps)
        kernel_s += time.perf_counter() - tk
        final = (res.status != 0) | (caps >= full)
        kout[idx[final]] = res.rank[final]
        shapes = np.stack([rsz[idx], csz[idx]], 1)
        for (m, n) in np.unique(shapes, axis=0):
            pos = np.nonzero((shapes[:, 0] == m) & (shapes[:, 1] == n))[0]   # contiguous in idx
            keep = pos[final[pos]]
            if keep.size == 0:
                continue
            X, Y = _pack_factors(res, pos, keep - pos[0], int(m), int(n), device=device)
            groups.append((idx[keep], int(m), int(n), X, Y))
        todo = idx[~final]
        cap_now *= 4
        del res
    return kout, groups, kernel_s


def build_operator(cloud: PointCloud, leaf: int = 64, eta: float = 1.0, eps_aca: float = 1e-6,
                   eps_comp: float = 1e-6, eps_rec: float | None = None, kcap: int = 1024,
                   verbose: bool = False, construct: str = "host", factor: str | None = None) -> HostOperator:
    """Build the H form and the UH form of the point-kernel matrix A_ij = g(x_i, x_j),
    A_ii = 1/(2h), for one seeded cloud.

    construct="gpu" samples the matrix on the GPU: ACA of the admissible blocks
    (uhm_aca), whose factors are packed by shape on the device (uhm_aca_pack), and the dense
    near-field blocks (uhm_kernel_blocks); the recompression runs on the host.
    construct="host" does everything on the host (OpenMP C++ and LAPACK).
    factor chooses where Alg. 2's per-cluster SVD runs: "gpu" (uhm_cluster_basis, batched
    over the clusters of one size; the default with construct="gpu") or "host" (LAPACK, the
    default with construct="host")."""
    if construct not in ("host", "gpu"):
        raise ValueError("construct must be 'host' or 'gpu'")
    if factor is None:
        factor = construct
    if factor not in ("host", "gpu"):
        raise ValueError("factor must be 'host' or 'gpu'")
    lib = _native()
    if eps_rec is None:
        eps_rec = eps_aca / 10.0
    t0 = time.perf_counter()
    tim = {}
    tree = build_tree(cloud.points, leaf)
    pts = np.ascontiguousarray(cloud.points[tree.perm])
    diag = 1.0 / (2.0 * cloud.h)
    kappa = cloud.kappa
    adm, den = build_block_tree(tree, eta)
    tim["tree"] = time.perf_counter() - t0
    nc = tree.nclusters
    off, size = tree.off, tree.size

    # ---- admissible blocks: ACA + recompression on one block of each mirrored pair
    dev_pts = None
    if construct == "gpu":
        from . import binding
        binding.load_library()
        dev_pts = binding._points_on_device(pts)
    lower = adm[adm[:, 0] < adm[:, 1]]
    if np.any(adm[:, 0] == adm[:, 1]):
        raise RuntimeError("a cluster is admissible with itself")
    fac_U, fac_V, fac_s = {}, {}, {}   # keyed by (tau, sigma) with tau < sigma
    t1 = time.perf_counter()
    levels = tree.level[lower[:, 0]] if lower.shape[0] else np.zeros(0, np.int32)
    t_aca = t_rec = t_aca_kernel = 0.0
    for lev in np.unique(levels):
        blk = lower[levels == lev]
        nb = blk.shape[0]
        roff = np.ascontiguousarray(off[blk[:, 0]])
        rsz = np.ascontiguousarray(size[blk[:, 0]])
        coff = np.ascontiguousarray(off[blk[:, 1]])
        csz = np.ascontiguousarray(size[blk[:, 1]])
        kout = np.zeros(nb, np.int32)
        ta = time.perf_counter()
        handle = None
        if construct == "gpu":
            kout, gpu_groups, ks = _aca_level_gpu(dev_pts, kappa, diag, roff, rsz, coff, csz, eps_aca, kcap,
                                                  device=factor == "gpu")
            t_aca_kernel += ks
        else:
            handle = lib.uhmb_aca_run(_ptr(pts), kappa, diag, nb, _ptr(roff), _ptr(rsz), _ptr(coff), _ptr(csz),
                                      eps_aca, kcap, _ptr(kout))
            if not handle:
                raise MemoryError("ACA batch allocation failed")
        t_aca += time.perf_counter() - ta
        tr = time.perf_counter()

        def recompress_xy(part, X, Y):
            QX, RX = np.linalg.qr(X)
            QY, RY = np.linalg.qr(Y)
            del X, Y
            W, s, Zh = np.linalg.svd(RX @ np.conj(np.swapaxes(RY, 1, 2)), full_matrices=False)
            out = []
            for c, b in enumerate(part):
                sc = s[c]
                k = max(1, int(np.count_nonzero(sc > eps_rec * sc[0]))) if sc.size and sc[0] > 0.0 else 1
                out.append(((int(blk[b, 0]), int(blk[b, 1])), QX[c] @ W[c][:, :k],
                            QY[c] @ np.conj(Zh[c][:k, :]).T, sc[:k].copy()))
            return out

        def recompress(job):
            if handle is None:
                return recompress_xy(*job)
            part, m, n, kp = job
            cnt = len(part)
            X = np.empty((cnt, m, kp), np.complex128)
            Y = np.empty((cnt, n, kp), np.complex128)
            idx = np.ascontiguousarray(part, dtype=np.int64)
            lib.uhmb_aca_copy(handle, cnt, _ptr(idx), int(m), int(n), kp, _ptr(X), _ptr(Y))
            return recompress_xy(part, X, Y)

        def recompress_dev(sel, X, Y):
            """The recompression of one shape group on the GPU (uhm_block_recompress), in calls of
            at most 65535 blocks and about 4 GiB of factors and workspace."""
            import torch
            from . import binding
            m, kp, n = X.shape[1], X.shape[2], Y.shape[1]
            per = 16 * kp * (6 * (m + n) + 8 * kp)   # factors, their copies, workspace and results
            step = max(1, min(65535, (1 << 32) // per))
            for a in range(0, len(sel), step):
                part = sel[a:a + step]
                tq = time.perf_counter()
                U, V, sv, rk, stt = binding.block_recompress(X[a:a + step], Y[a:a + step], eps_rec)
                torch.cuda.synchronize()
                tq1 = time.perf_counter()
                kmax = int(rk.max())
                Uh = _to_host_copy(U[:, :kmax, :].contiguous())
                Vh = _to_host_copy(V[:, :kmax, :].contiguous())
                svh = sv[:, :kmax].cpu().numpy()
                del U, V, sv
                bad = np.nonzero(stt != 0)[0]
                for c, b in enumerate(part):
                    k = int(rk[c])
                    key = (int(blk[b, 0]), int(blk[b, 1]))
                    fac_U[key] = Uh[c, :k, :].T
                    fac_V[key] = Vh[c, :k, :].T
                    fac_s[key] = svh[c, :k].copy()
                if verbose:
                    print(f"    recompression of {len(part)} blocks {m} x {n}, kp {kp}: GPU {tq1 - tq:.2f} s, "
                          f"host {time.perf_counter() - tq1:.2f} s", file=sys.stderr, flush=True)
                if bad.size:   # Jacobi not converged: the host SVD for those blocks
                    bi = torch.as_tensor(bad, device=X.device)
                    for key, Ub, Vb, sb in recompress_xy([part[c] for c in bad], X[a:a + step][bi].cpu().numpy(),
                                                         Y[a:a + step][bi].cpu().numpy()):
                        fac_U[key], fac_V[key], fac_s[key] = Ub, Vb, sb
                    tim["recompress_host_fallback"] = tim.get("recompress_host_fallback", 0) + int(bad.size)

        try:
            jobs = []
            if handle is None and factor == "gpu":
                for sel, m, n, X, Y in gpu_groups:
                    if max(m, n) > _GPU_MAX_ROWS:   # beyond the GPU kernels' row limit: the host SVD
                        for key, Ub, Vb, sb in recompress_xy(sel, _to_host(X), _to_host(Y)):
                            fac_U[key], fac_V[key], fac_s[key] = Ub, Vb, sb
                    else:
                        recompress_dev(sel, X, Y)
                del gpu_groups
            elif handle is None:
                for sel, m, n, X, Y in gpu_groups:
                    kp = X.shape[2]
                    step = max(1, len(list(_chunks(sel, 16 * (m + n) * kp * 4, parts=4 * _workers()))[0]))
                    for a in range(0, len(sel), step):
                        jobs.append((sel[a:a + step], X[a:a + step], Y[a:a + step]))
                del gpu_groups
            else:
                shapes = np.stack([rsz, csz], 1)
                for (m, n) in np.unique(shapes, axis=0):
                    sel = np.nonzero((rsz == m) & (csz == n))[0]
                    kp = int(kout[sel].max())
                    for part in _chunks(sel, 16 * (m + n) * kp * 4, parts=4 * _workers()):
                        jobs.append((part, int(m), int(n), kp))
            for res in _pmap(recompress, jobs):
                for key, Ub, Vb, sb in res:
                    fac_U[key] = Ub
                    fac_V[key] = Vb
                    fac_s[key] = sb
        finally:
            if handle is not None:
                lib.uhmb_aca_free(handle)
        t_rec += time.perf_counter() - tr
        if verbose:
            print(f"  level {lev}: {nb} ACA blocks, k_max {int(kout.max())}", file=sys.stderr, flush=True)
    tim["aca"] = t_aca
    if construct == "gpu":
        tim["aca_gpu_calls"] = t_aca_kernel
    tim["recompress"] = t_rec
    if verbose:
        print(f"  ACA {t_aca:.1f} s, recompression {t_rec:.1f} s", file=sys.stderr, flush=True)

    def block_factors(t, s):
        """(U_b, Sigma_b, V_b) of block t x s, using the mirror for t > s."""
        if t < s:
            return fac_U[(t, s)], fac_s[(t, s)], fac_V[(t, s)]
        return np.conj(fac_V[(s, t)]), fac_s[(s, t)], np.conj(fac_U[(s, t)])

    # stored block (t < s) -> addresses and strides of U_b, V_b, Sigma_b, for uhmb_scaled_copy
    factor_views = _factor_views_of(fac_U, fac_V, fac_s)

    # ---- uniform compression, one SVD per cluster (row side; column side by symmetry)
    t2 = time.perf_counter()
    row_blocks = {}
    for t, s in adm:
        row_blocks.setdefault(int(t), []).append(int(s))
    rank = np.zeros(nc, np.int32)
    Ubasis = {}
    Lmat = {}  # (t, s) -> U_t^* U_b Sigma_b   (l_t x k_b)
    sv_dropped = np.zeros(nc)
    sv_tail = np.zeros(nc)
    clusters = np.array(sorted(row_blocks), dtype=np.int64)
    groups = {}
    for t in clusters:
        ks = sum(fac_s[(min(t, s), max(t, s))].size for s in row_blocks[t])
        groups.setdefault((int(size[t])), []).append((int(t), ks))
    def agglomerate(part):
        nt = int(size[part[0][0]])
        kp = max(k for _, k in part)
        Xb = np.zeros((len(part), nt, kp), np.complex128)
        cols = []
        for c, (t, _) in enumerate(part):
            j = 0
            cl = []
            for s in row_blocks[t]:
                Ub, sb, _ = block_factors(t, s)
                kb = sb.size
                Xb[c, :, j:j + kb] = Ub * sb[None, :]
                cl.append((s, j, kb))
                j += kb
            cols.append(cl)
        return Xb, cols

    def compress(part):
        Xb, cols = agglomerate(part)
        Uh, sh, Vh = np.linalg.svd(Xb, full_matrices=False)
        del Xb
        out = []
        for c, (t, ks) in enumerate(part):
            sv = sh[c]
            l = max(1, int(np.count_nonzero(sv > eps_comp * sv[0]))) if sv[0] > 0 else 1
            l = min(l, ks)
            SV = sv[:l, None] * Vh[c][:l, :]
            out.append((t, l, np.ascontiguousarray(Uh[c][:, :l]), sv[l] if l < sv.size else 0.0,
                        float(np.sqrt(np.sum(sv[l:] ** 2))),
                        [(s, np.ascontiguousarray(SV[:, j:j + kb])) for s, j, kb in cols[c]]))
        return out

    def compress_gpu_all(jobs):
        """Alg. 2's SVDs on the GPU, one batched call per chunk of same-size clusters.  The next
        chunk's cluster matrices are written into page-locked host memory by the thread pool
        meanwhile (one DMA each way).  A cluster the GPU flags (step cap before the tolerance,
        or Jacobi not converged) is taken by the host SVD instead."""
        import torch
        from . import binding
        out = []
        tw = {"compress_fill_wait": 0.0, "compress_gpu": 0.0, "compress_post": 0.0, "compress_host_fallback_s": 0.0}
        fallback = 0
        per_size = {}

        def fill(part):
            """The batch's matrices X_tau = [U_b Sigma_b ...] (conj(V_b) Sigma_b for a mirrored
            block) written by the native copy into page-locked memory, zero columns after."""
            t0 = time.perf_counter()
            nt = int(size[part[0][0]])
            kp = max(k for _, k in part)
            buf = torch.empty((len(part), nt, kp), dtype=torch.complex128, pin_memory=True)
            recs, cols = _row_records(part, row_blocks, factor_views, buf.data_ptr(), nt, kp)
            _scaled_copy(recs)
            return buf, cols, time.perf_counter() - t0

        # fills run back to back on one thread, up to two batches ahead of the GPU
        depth = 2
        fill_s = 0.0
        with ThreadPoolExecutor(1) as pre:
            ahead = [pre.submit(fill, jobs[i]) for i in range(min(depth, len(jobs)))]
            for q, part in enumerate(jobs):
                ta = time.perf_counter()
                buf, cols, tf = ahead.pop(0).result()
                fill_s += tf
                if q + depth < len(jobs):
                    ahead.append(pre.submit(fill, jobs[q + depth]))
                tb = time.perf_counter()
                nt, kp = buf.shape[1], buf.shape[2]
                res = binding.cluster_basis(buf.to("cuda", non_blocking=True), eps=eps_comp,
                                            pmax=min(nt, kp, 2048))
                tc = time.perf_counter()
                bad = set(np.nonzero(res.status != 0)[0].tolist())
                lmax = int(res.rank.max())
                Uh = _to_host_copy(res.U[:, :lmax, :].contiguous())
                # Sigma V^* stays on the device for the couplings: per cluster (ks x l) at [c, :ks, :l]
                dev_L.append(([t for t, _ in part], [ks for _, ks in part], res.rank.copy(), bad,
                              res.SV[:, :, :lmax].contiguous()))
                del res.U, res.SV, res.sv, buf
                for c, (t, ks) in enumerate(part):
                    if c in bad:
                        continue
                    l = int(res.rank[c])
                    out.append((t, l, Uh[c, :l, :].T, float(res.stats[c, 1]), float(res.stats[c, 0]), []))
                td = time.perf_counter()
                if bad:
                    fallback += len(bad)
                    out.extend(compress([part[c] for c in sorted(bad)]))
                te = time.perf_counter()
                del Uh
                tw["compress_fill_wait"] += tb - ta
                tw["compress_gpu"] += tc - tb
                tw["compress_post"] += td - tc
                tw["compress_host_fallback_s"] += te - td
                e = per_size.setdefault(int(nt), [0, 0, 0, 0.0, 0.0])
                e[0] += len(part)
                e[1] = max(e[1], int(res.psteps.max()))
                e[2] = max(e[2], lmax)
                e[3] += tc - tb
                e[4] += te - tc
        tw["compress_fill"] = fill_s
        tim.update(tw)
        tim["compress_host_fallback"] = fallback
        if verbose:
            for nt in sorted(per_size):
                c, pm, lm, g, hp = per_size[nt]
                print(f"  uniform compression, {c} clusters of {nt}: p <= {pm}, l <= {lm}, GPU {g:.2f} s, "
                      f"host {hp:.2f} s", file=sys.stderr, flush=True)
        return [out]

    dev_L = []   # per GPU chunk: (clusters, their column counts, ranks, flagged, Sigma V^* on the device)
    jobs = []
    if factor == "gpu":
        host_jobs = []
        for nt, members in groups.items():
            kp_all = max(k for _, k in members)
            if nt > _GPU_MAX_ROWS:   # beyond the GPU kernels' row limit: the host SVD
                host_jobs.extend(_chunks(members, 16 * nt * kp_all * 3, parts=2 * _workers()))
                continue
            # about 4 GiB of cluster matrices per call, at most 65535 clusters
            for part in _chunks(members, 16 * nt * kp_all, budget=1 << 32):
                jobs.extend(part[a:a + 65535] for a in range(0, len(part), 65535))
        # the smallest clusters first, their first batch an eighth of the rest: the GPU starts
        # after a short fill, and the later fills run while it works
        jobs.sort(key=lambda part: int(size[part[0][0]]))
        if jobs and len(jobs[0]) >= 16:
            head = len(jobs[0]) // 8
            jobs[:1] = [jobs[0][:head], jobs[0][head:]]
        results = compress_gpu_all(jobs) + _pmap(compress, host_jobs)
    else:
        for nt, members in groups.items():
            kp_all = max(k for _, k in members)
            jobs.extend(_chunks(members, 16 * nt * kp_all * 3, parts=2 * _workers()))
        results = _pmap(compress, jobs)
    host_L = {}   # GPU mode: Sigma V^* (l x ks) of the clusters the host factorised
    for res in results:
        for t, l, Ut, dropped, tail, Ls in res:
            if factor == "gpu" and Ls:
                host_L[t] = np.concatenate([Lb for _, Lb in Ls], axis=1)
            rank[t] = l
            Ubasis[t] = Ut
            sv_dropped[t] = dropped
            sv_tail[t] = tail
            for s, Lb in Ls:
                Lmat[(t, s)] = Lb
    tim["compress"] = time.perf_counter() - t2
    if verbose:
        print(f"  uniform compression {tim['compress']:.1f} s", file=sys.stderr, flush=True)

    # ---- couplings S_b = L_b Sigma_b^{-1} L_{b~}^T, b~ the mirrored block
    t3 = time.perf_counter()
    nadm = adm.shape[0]
    S_off = np.zeros(nadm, np.int64)
    sizes = rank[adm[:, 0]].astype(np.int64) * rank[adm[:, 1]].astype(np.int64)
    S_off[1:] = np.cumsum(sizes)[:-1]
    S = np.empty(int(sizes.sum()), np.complex128)
    adm_rank = np.array([fac_s[(min(int(t), int(s)), max(int(t), int(s)))].size for t, s in adm], np.int32) \
        if nadm else np.zeros(0, np.int32)
    # factored couplings S_b = S_{X,b} S_{Y,b}^* (section 4.2): S_{X,b} = U_tau^* U_b (l_tau x k_b),
    # S_{Y,b} = V_sigma^* V_b (l_sigma x k_b), with V_b's scale folded into S_{X,b}
    xsz = rank[adm[:, 0]].astype(np.int64) * adm_rank
    ysz = rank[adm[:, 1]].astype(np.int64) * adm_rank
    SX_off = np.concatenate([[0], np.cumsum(xsz)[:-1]]).astype(np.int64)[:nadm]
    SY_off = np.concatenate([[0], np.cumsum(ysz)[:-1]]).astype(np.int64)[:nadm]
    SX = np.empty(int(xsz.sum()), np.complex128)
    SY = np.empty(int(ysz.sum()), np.complex128)
    lt_of, ls_of = rank[adm[:, 0]], rank[adm[:, 1]]

    def couplings_gpu():
        """All couplings on the GPU (uhm_couplings) from the clusters' Sigma V^* rows, which the
        GPU factorisation left on the device (the host factorisation's, for flagged clusters,
        are uploaded); S, S_X and S_Y come back through page-locked staging."""
        import torch
        from . import binding
        ks_of = np.zeros(nc, np.int64)
        for members in groups.values():
            for t, ks in members:
                ks_of[t] = ks
        lsz = ks_of * rank.astype(np.int64)
        L_off = np.concatenate([[0], np.cumsum(lsz)[:-1]]).astype(np.int64)
        Lbuf = torch.empty(max(1, int(lsz.sum())), dtype=torch.complex128, device="cuda")
        for clist, kslist, rk, bad, SVd in dev_L:
            for c, t in enumerate(clist):
                if c in bad:
                    continue
                ks, l = int(kslist[c]), int(rank[t])
                Lbuf[L_off[t]:L_off[t] + ks * l].view(ks, l).copy_(SVd[c, :ks, :l])
        dev_L.clear()
        for t, Lh in host_L.items():
            ks, l = int(ks_of[t]), int(rank[t])
            Lbuf[L_off[t]:L_off[t] + ks * l].view(ks, l).copy_(torch.from_numpy(np.ascontiguousarray(Lh.T)))
        # j: the first column of block b in its row cluster's agglomeration (row_blocks order,
        # which is the order of adm); the mirrored block by its key
        order = np.argsort(adm[:, 0], kind="stable")
        rk_s = adm_rank[order].astype(np.int64)
        rows_s = adm[order, 0]
        csum = np.cumsum(rk_s) - rk_s
        first = np.r_[True, rows_s[1:] != rows_s[:-1]] if nadm else np.zeros(0, bool)
        start = np.maximum.accumulate(np.where(first, np.arange(nadm), 0)) if nadm else np.zeros(0, np.int64)
        j_of = np.empty(nadm, np.int64)
        j_of[order] = csum - csum[start]
        key = adm[:, 0].astype(np.int64) * nc + adm[:, 1]
        mkey = adm[:, 1].astype(np.int64) * nc + adm[:, 0]
        ko = np.argsort(key)
        mirror = ko[np.searchsorted(key[ko], mkey)]
        if not np.array_equal(key[mirror], mkey):
            raise RuntimeError("a block without its mirror")
        sig = np.concatenate([fac_s[(min(int(t), int(s)), max(int(t), int(s)))] for t, s in adm]) if nadm \
            else np.zeros(1)
        desc = np.zeros(nadm, binding.COUPLING_DTYPE)
        t_, s_ = adm[:, 0].astype(np.int64), adm[:, 1].astype(np.int64)
        desc["a_off"] = L_off[t_] + j_of * rank[t_]
        desc["b_off"] = L_off[s_] + j_of[mirror] * rank[s_]
        desc["sig_off"] = np.cumsum(adm_rank.astype(np.int64)) - adm_rank
        desc["s_off"], desc["x_off"], desc["y_off"] = S_off, SX_off, SY_off
        desc["lt"], desc["ls"], desc["kb"] = rank[t_], rank[s_], adm_rank
        Sd, SXd, SYd = binding.couplings(Lbuf, sig, desc, S.size, SX.size, SY.size)
        del Lbuf
        for dst, src in ((S, Sd), (SX, SXd), (SY, SYd)):
            _copy_into(dst, src)

    def couple(bs):
        """Blocks bs written straight into their column-major places (disjoint slices; numpy
        drops the GIL in the copies, so the thread pool also spreads the first-touch faults of
        the fresh arrays)."""
        for b in bs:
            t, s = int(adm[b, 0]), int(adm[b, 1])
            sb = fac_s[(min(t, s), max(t, s))]
            lt, ls, kb = int(lt_of[b]), int(ls_of[b]), int(adm_rank[b])
            Xf = SX[SX_off[b]:SX_off[b] + xsz[b]].reshape(kb, lt).T
            np.divide(Lmat[(t, s)], sb[None, :], out=Xf)
            np.conjugate(Lmat[(s, t)], out=SY[SY_off[b]:SY_off[b] + ysz[b]].reshape(kb, ls).T)
            S[S_off[b]:S_off[b] + sizes[b]].reshape(ls, lt).T[...] = Xf @ Lmat[(s, t)].T

    if factor == "gpu":
        couplings_gpu()
    else:
        _pmap(couple, np.array_split(np.arange(nadm), max(1, min(nadm, 8 * _workers()))))
    tim["couplings"] = time.perf_counter() - t3
    if verbose:
        print(f"  couplings {tim['couplings']:.1f} s", file=sys.stderr, flush=True)

    # ---- bases (V = conj(U) by symmetry), H factors
    t5 = time.perf_counter()
    U_off = np.full(nc, -1, np.int64)
    usz = size * rank
    has = rank > 0
    U_off[has] = np.concatenate([[0], np.cumsum(usz[has])[:-1]]) if has.any() else []
    U = np.empty(int(usz.sum()), np.complex128)
    V = np.empty_like(U)

    def bases(ts):
        for t in ts:
            t = int(t)
            u = U[U_off[t]:U_off[t] + usz[t]]
            u.reshape(int(rank[t]), int(size[t])).T[...] = Ubasis[t]
            np.conjugate(u, out=V[U_off[t]:U_off[t] + usz[t]])

    with_basis = np.array(sorted(Ubasis), dtype=np.int64)
    _pmap(bases, np.array_split(with_basis, max(1, min(len(with_basis), 8 * _workers()))))

    xs = size[adm[:, 0]] * adm_rank
    ys = size[adm[:, 1]] * adm_rank
    X_off = np.concatenate([[0], np.cumsum(xs)[:-1]]).astype(np.int64)[:nadm]
    Y_off = np.concatenate([[0], np.cumsum(ys)[:-1]]).astype(np.int64)[:nadm]
    Xh = np.empty(int(xs.sum()), np.complex128)
    Yh = np.empty(int(ys.sum()), np.complex128)

    # X_b = U_b Sigma_b and Y_b = V_b column-major, by the native copy
    _scaled_copy(_hfactor_records(adm, adm_rank, size, X_off, Y_off, Xh.__array_interface__["data"][0],
                                  Yh.__array_interface__["data"][0], factor_views))
    del factor_views, fac_U, fac_V, Lmat
    tim["factors"] = time.perf_counter() - t5

    # ---- dense near field
    t4 = time.perf_counter()
    nden = den.shape[0]
    dsz = size[den[:, 0]] * size[den[:, 1]]
    D_off = np.concatenate([[0], np.cumsum(dsz)[:-1]]).astype(np.int64) if nden else np.zeros(0, np.int64)
    D = np.empty(int(dsz.sum()), np.complex128)
    if nden and construct == "gpu":
        Dd, doff = binding.kernel_blocks(dev_pts, kappa, diag, off[den[:, 0]], size[den[:, 0]], off[den[:, 1]],
                                         size[den[:, 1]])
        assert np.array_equal(doff, D_off)
        D = _to_host(Dd)
        del Dd
    elif nden:
        d_ro = np.ascontiguousarray(off[den[:, 0]])
        d_rs = np.ascontiguousarray(size[den[:, 0]])
        d_co = np.ascontiguousarray(off[den[:, 1]])
        d_cs = np.ascontiguousarray(size[den[:, 1]])
        lib.uhmb_dense_blocks(_ptr(pts), kappa, diag, nden, _ptr(d_ro), _ptr(d_rs), _ptr(d_co), _ptr(d_cs),
                              _ptr(D_off), _ptr(D))
    tim["dense"] = time.perf_counter() - t4
    tim["total"] = time.perf_counter() - t0

    return HostOperator(
        n=cloud.n, perm=tree.perm, off=tree.off, size=tree.size, level=tree.level, parent=tree.parent,
        rank_row=rank.copy(), rank_col=rank.copy(), U_off=U_off, V_off=U_off.copy(), U=U, V=V,
        adm_row=adm[:, 0].astype(np.int32), adm_col=adm[:, 1].astype(np.int32), S_off=S_off, S=S,
        adm_rank=adm_rank, X_off=X_off, Y_off=Y_off, X=Xh, Y=Yh,
        den_row=den[:, 0].astype(np.int32), den_col=den[:, 1].astype(np.int32), D_off=D_off, D=D,
        kappa=kappa, h=cloud.h, leaf=leaf, eta=eta, eps_aca=eps_aca, eps_comp=eps_comp, depth=tree.depth,
        SX_off=SX_off, SY_off=SY_off, SX=SX, SY=SY,
        sv_dropped=sv_dropped, sv_tail=sv_tail, timings=tim)


def build_uniform_direct(cloud: PointCloud, leaf: int = 64, eta: float = 1.0, eps_aca: float = 1e-6,
                         eps_comp: float = 1e-6, eps_rec: float | None = None, kcap: int = 1024,
                         threads: int | None = None) -> HostOperator:
    """Direct construction of the UH form from matrix entries (Algs. 3-4, section 4.3), in
    parallel with one lock per admissible block (section 4.4), in the symmetric form of
    Remark 4.4: one set of clusters, one approximation per mirrored pair of blocks.

    The clusters are processed from large to small.  Building cluster tau takes, for each
    block tau x sigma, the block's recompressed factors U_b Sigma_b V_b^*, approximating the
    block first (ACA + recompression, section 2.3) if no thread has yet; the block's lock
    makes the second thread wait for the first.  Its columns U_b Sigma_b (or conj(V_b)
    Sigma_b for the mirrored orientation) go into X_tau, and once both clusters of a block
    have taken them the factors are dropped; only Sigma_b is kept, for the couplings.  The
    SVD of X_tau gives U_tau and U_tau^* U_b Sigma_b as in build_operator, and the couplings
    S_b = S_{X,b} S_{Y,b}^* are formed the same way.  The H form is never held whole, so the
    returned operator carries no X and Y (adm_rank is set); timings["peak_factor_bytes"] is
    the largest amount of block factors held at once and timings["total_factor_bytes"] what
    the H form would hold."""
    import threading
    lib = _native()
    if eps_rec is None:
        eps_rec = eps_aca / 10.0
    t0 = time.perf_counter()
    tim = {}
    tree = build_tree(cloud.points, leaf)
    pts = np.ascontiguousarray(cloud.points[tree.perm])
    diag = 1.0 / (2.0 * cloud.h)
    kappa = cloud.kappa
    adm, den = build_block_tree(tree, eta)
    nc = tree.nclusters
    off, size = tree.off, tree.size
    if np.any(adm[:, 0] == adm[:, 1]):
        raise RuntimeError("a cluster is admissible with itself")
    lower = adm[adm[:, 0] < adm[:, 1]]
    index = {(int(t), int(s)): b for b, (t, s) in enumerate(lower)}
    row_blocks = {}
    for t, s in adm:
        row_blocks.setdefault(int(t), []).append(int(s))
    order = sorted(row_blocks, key=lambda c: (-int(size[c]), c))
    nlow = lower.shape[0]
    locks = [threading.Lock() for _ in range(nlow)]
    fac = [None] * nlow
    sigma = [None] * nlow
    uses = [2] * nlow
    book = threading.Lock()
    acct = {"live": 0, "peak": 0, "total": 0, "waits": 0}

    def approximate(b):
        t, s = int(lower[b, 0]), int(lower[b, 1])
        m, n = int(size[t]), int(size[s])
        full = min(m, n, kcap)
        cap = min(full, 128)
        while True:
            X = np.empty((m, cap), np.complex128)
            Y = np.empty((n, cap), np.complex128)
            k = lib.uhmb_aca_block(_ptr(pts), kappa, diag, int(off[t]), m, int(off[s]), n, eps_aca, cap, _ptr(X), _ptr(Y))
            if k < cap or cap >= full:
                break
            cap = min(full, 4 * cap)
        QX, RX = np.linalg.qr(X[:, :k])
        QY, RY = np.linalg.qr(Y[:, :k])
        W, sv, Zh = np.linalg.svd(RX @ RY.conj().T)
        r = max(1, int(np.count_nonzero(sv > eps_rec * sv[0]))) if sv.size and sv[0] > 0.0 else 1
        return QX @ W[:, :r], sv[:r].copy(), QY @ Zh[:r, :].conj().T

    def factors(b):
        if not locks[b].acquire(blocking=False):
            with book:
                acct["waits"] += 1
            locks[b].acquire()
        try:
            if fac[b] is None and sigma[b] is None:
                Ub, sb, Vb = approximate(b)
                fac[b], sigma[b] = (Ub, Vb), sb
                nbytes = Ub.nbytes + Vb.nbytes
                with book:
                    acct["live"] += nbytes
                    acct["total"] += nbytes
                    acct["peak"] = max(acct["peak"], acct["live"])
            return fac[b], sigma[b]
        finally:
            locks[b].release()

    def release(b):
        with book:
            uses[b] -= 1
            if uses[b] == 0:
                acct["live"] -= fac[b][0].nbytes + fac[b][1].nbytes
                fac[b] = None

    def build_cluster(t):
        cols, parts = [], []
        for s in row_blocks[t]:
            b = index[(min(t, s), max(t, s))]
            (Ub, Vb), sb = factors(b)
            parts.append(Ub * sb[None, :] if t < s else np.conj(Vb) * sb[None, :])
            cols.append((s, sb.size))
            release(b)
        X = np.concatenate(parts, 1)
        Uh, sv, Vh = np.linalg.svd(X, full_matrices=False)
        l = max(1, int(np.count_nonzero(sv > eps_comp * sv[0]))) if sv[0] > 0 else 1
        l = min(l, X.shape[1])
        SV = sv[:l, None] * Vh[:l, :]
        out, j = [], 0
        for s, kb in cols:
            out.append((s, np.ascontiguousarray(SV[:, j:j + kb])))
            j += kb
        return (t, l, np.ascontiguousarray(Uh[:, :l]), sv[l] if l < sv.size else 0.0,
                float(np.sqrt(np.sum(sv[l:] ** 2))), out)

    t1 = time.perf_counter()
    nw = max(1, int(threads or _workers()))
    ctx = threadpool_limits(1) if threadpool_limits is not None else None
    try:
        if ctx is not None:
            ctx.__enter__()
        if nw == 1:
            results = [build_cluster(t) for t in order]
        else:
            with ThreadPoolExecutor(nw) as ex:
                results = list(ex.map(build_cluster, order))
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    tim["clusters"] = time.perf_counter() - t1
    rank = np.zeros(nc, np.int32)
    Ubasis, Lmat = {}, {}
    sv_dropped = np.zeros(nc)
    sv_tail = np.zeros(nc)
    for t, l, Ut, dropped, tail, Ls in results:
        rank[t] = l
        Ubasis[t] = Ut
        sv_dropped[t] = dropped
        sv_tail[t] = tail
        for s, Lb in Ls:
            Lmat[(t, s)] = Lb
    del results

    # couplings S_b = L_b Sigma_b^{-1} L_{b~}^T and their factors, as in build_operator
    nadm = adm.shape[0]
    kb_all = np.array([sigma[index[(min(int(t), int(s)), max(int(t), int(s)))]].size for t, s in adm], np.int32) \
        if nadm else np.zeros(0, np.int32)
    sizes = rank[adm[:, 0]].astype(np.int64) * rank[adm[:, 1]].astype(np.int64)
    S_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)[:nadm]
    S = np.empty(int(sizes.sum()), np.complex128)
    xsz = rank[adm[:, 0]].astype(np.int64) * kb_all
    ysz = rank[adm[:, 1]].astype(np.int64) * kb_all
    SX_off = np.concatenate([[0], np.cumsum(xsz)[:-1]]).astype(np.int64)[:nadm]
    SY_off = np.concatenate([[0], np.cumsum(ysz)[:-1]]).astype(np.int64)[:nadm]
    SX = np.empty(int(xsz.sum()), np.complex128)
    SY = np.empty(int(ysz.sum()), np.complex128)
    for b in range(nadm):
        t, s = int(adm[b, 0]), int(adm[b, 1])
        sb = sigma[index[(min(t, s), max(t, s))]]
        Xf = Lmat[(t, s)] / sb[None, :]
        S[S_off[b]:S_off[b] + sizes[b]] = (Xf @ Lmat[(s, t)].T).ravel(order="F")
        SX[SX_off[b]:SX_off[b] + xsz[b]] = Xf.ravel(order="F")
        SY[SY_off[b]:SY_off[b] + ysz[b]] = np.conj(Lmat[(s, t)]).ravel(order="F")
    U_off = np.full(nc, -1, np.int64)
    usz = size * rank
    has = rank > 0
    U_off[has] = np.concatenate([[0], np.cumsum(usz[has])[:-1]]) if has.any() else []
    U = np.empty(int(usz.sum()), np.complex128)
    for t, Ut in Ubasis.items():
        U[U_off[t]:U_off[t] + usz[t]] = Ut.ravel(order="F")

    nden = den.shape[0]
    dsz = size[den[:, 0]] * size[den[:, 1]]
    D_off = np.concatenate([[0], np.cumsum(dsz)[:-1]]).astype(np.int64) if nden else np.zeros(0, np.int64)
    D = np.empty(int(dsz.sum()), np.complex128)
    if nden:
        # the index arrays are named so that they outlive the call
        d_ro = np.ascontiguousarray(off[den[:, 0]])
        d_rs = np.ascontiguousarray(size[den[:, 0]])
        d_co = np.ascontiguousarray(off[den[:, 1]])
        d_cs = np.ascontiguousarray(size[den[:, 1]])
        lib.uhmb_dense_blocks(_ptr(pts), kappa, diag, nden, _ptr(d_ro), _ptr(d_rs), _ptr(d_co), _ptr(d_cs),
                              _ptr(D_off), _ptr(D))
    tim["total"] = time.perf_counter() - t0
    tim["peak_factor_bytes"] = acct["peak"]
    tim["total_factor_bytes"] = acct["total"]
    tim["lock_waits"] = acct["waits"]
    tim["threads"] = nw
    zero = np.zeros(nadm, np.int64)
    return HostOperator(
        n=cloud.n, perm=tree.perm, off=tree.off, size=tree.size, level=tree.level, parent=tree.parent,
        rank_row=rank.copy(), rank_col=rank.copy(), U_off=U_off, V_off=U_off.copy(), U=U, V=np.conj(U),
        adm_row=adm[:, 0].astype(np.int32), adm_col=adm[:, 1].astype(np.int32), S_off=S_off, S=S,
        adm_rank=kb_all, X_off=zero, Y_off=zero.copy(), X=np.zeros(0, np.complex128), Y=np.zeros(0, np.complex128),
        den_row=den[:, 0].astype(np.int32), den_col=den[:, 1].astype(np.int32), D_off=D_off, D=D,
        kappa=kappa, h=cloud.h, leaf=leaf, eta=eta, eps_aca=eps_aca, eps_comp=eps_comp, depth=tree.depth,
        SX_off=SX_off, SY_off=SY_off, SX=SX, SY=SY, sv_dropped=sv_dropped, sv_tail=sv_tail, timings=tim)


def symmetric_image(op: HostOperator) -> dict:
    """The symmetric-storage image of an operator (Remark 4.4, as in section 6.1): one block
    of each mirrored pair, the one whose row cluster has the smaller index, and every
    diagonal dense block.  The flat arrays are shared with ``op`` (the blocks left out are
    simply not listed); V_sigma = conj(U_sigma) and the mirrors are implied, so an upload
    with symmetric storage reads only U, the listed couplings and the listed dense blocks."""
    d = {k: getattr(op, k) for k in ("n", "perm", "off", "size", "level", "parent", "rank_row", "rank_col",
                                     "U_off", "V_off", "U", "V", "S", "D", "kappa", "h", "leaf", "eta",
                                     "eps_aca", "eps_comp", "depth")}
    ka = op.adm_row < op.adm_col
    kd = op.den_row <= op.den_col
    d.update(adm_row=op.adm_row[ka], adm_col=op.adm_col[ka], S_off=op.S_off[ka],
             den_row=op.den_row[kd], den_col=op.den_col[kd], D_off=op.D_off[kd])
    rs = op.rank_row.astype(np.int64)
    d["elems_S_stored"] = int(np.sum(rs[d["adm_row"]] * rs[d["adm_col"]]))
    d["elems_D_stored"] = int(np.sum(op.size[d["den_row"]] * op.size[d["den_col"]]))
    return d


def save_operator(op: HostOperator, path: str) -> None:
    arrays = {k: v for k, v in op.__dict__.items() if isinstance(v, np.ndarray)}
    scalars = {k: v for k, v in op.__dict__.items() if isinstance(v, (int, float)) and not isinstance(v, bool)}
    np.savez(path, **arrays, **{"_scalar_" + k: np.asarray(v) for k, v in scalars.items()})


def load_operator(path: str) -> HostOperator:
    z = np.load(path, allow_pickle=False)
    kw = {}
    for k in z.files:
        if k.startswith("_scalar_"):
            v = z[k]
            kw[k[8:]] = v.item()
        else:
            kw[k] = z[k]
    for k in ("n", "leaf", "depth"):
        kw[k] = int(kw[k])
    return HostOperator(**kw)
