"""Python binding of libuhm.so (include/uhm.h): argument marshalling only.

Every step of the product runs in the HIP library.  PyTorch is used for device memory
(the vectors are torch tensors on a HIP device) and for streams.  If libuhm.so is
missing this module raises on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuhm.so")

UHM_OK, UHM_EINVAL, UHM_ENOMEM, UHM_EHIP, UHM_ENOCONV, UHM_ENOTSUP = 0, -1, -2, -3, -4, -5
STORAGE = {"c128": 0, "c64": 1, "bf16pair": 2, "c128multi": 3, "c128sym": 4, "c128fact": 5, "c64fact": 6,
           "bf16pairfact": 7, "c128multifact": 8, "c64stream": 9, "bf16pairstream": 10}
FACTORED_FORMS = ("c128fact", "c64fact", "bf16pairfact", "c128multifact")
C128_FORMS = ("c128", "c128multi", "c128sym", "c128fact", "c128multifact")

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32


class HostOperator(ctypes.Structure):
    _fields_ = [("n", I64), ("perm", P), ("nclusters", I32), ("off", P), ("size", P), ("parent", P),
                ("rank_row", P), ("rank_col", P), ("U_off", P), ("V_off", P),
                ("U", P), ("U_len", I64), ("V", P), ("V_len", I64),
                ("nadm", I64), ("adm_row", P), ("adm_col", P), ("S_off", P), ("S", P), ("S_len", I64),
                ("nden", I64), ("den_row", P), ("den_col", P), ("D_off", P), ("D", P), ("D_len", I64),
                ("adm_rank", P), ("SX_off", P), ("SY_off", P), ("SX", P), ("SX_len", I64), ("SY", P), ("SY_len", I64)]


class HostHMatrix(ctypes.Structure):
    _fields_ = [("n", I64), ("perm", P), ("nclusters", I32), ("off", P), ("size", P), ("parent", P),
                ("nadm", I64), ("adm_row", P), ("adm_col", P), ("adm_rank", P), ("X_off", P), ("Y_off", P),
                ("X", P), ("X_len", I64), ("Y", P), ("Y_len", I64),
                ("nden", I64), ("den_row", P), ("den_col", P), ("D_off", P), ("D", P), ("D_len", I64)]


class OpInfo(ctypes.Structure):
    _fields_ = [("n", I64), ("kind", I32), ("storage", I32), ("nleaves", I32), ("elem_bytes", I32),
                ("nadm", I64), ("nden", I64), ("elems_forward", I64), ("elems_coupling", I64),
                ("elems_backward", I64), ("elems_near", I64), ("rank_space", I64), ("device_bytes", I64),
                ("partial_coupling", I64), ("partial_near", I64), ("elems_coupling_in", I64),
                ("scratch_bytes", I64)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("restart", I32), ("max_iterations", I32), ("max_refinements", I32), ("inner_tol", ctypes.c_double),
                ("inner_cycles", I32)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iterations", I32), ("restarts", I32), ("refinements", I32), ("converged", I32),
                ("rel_residual", ctypes.c_double), ("seconds_total", ctypes.c_double),
                ("seconds_products", ctypes.c_double), ("seconds_arnoldi", ctypes.c_double),
                ("second_passes", I64)]


class BlockDesc(ctypes.Structure):
    _fields_ = [("row_off", I64), ("col_off", I64), ("rows", I32), ("cols", I32), ("cap", I32), ("reserved", I32),
                ("a_off", I64), ("b_off", I64), ("p_off", I64)]


# the same layout as a numpy record, to fill many descriptors at once
BLOCK_DTYPE = np.dtype({"names": [f for f, _ in BlockDesc._fields_],
                        "formats": [np.int64 if t is I64 else np.int32 for _, t in BlockDesc._fields_],
                        "offsets": [getattr(BlockDesc, f).offset for f, _ in BlockDesc._fields_],
                        "itemsize": ctypes.sizeof(BlockDesc)})


class CouplingDesc(ctypes.Structure):
    _fields_ = [("a_off", I64), ("b_off", I64), ("sig_off", I64), ("s_off", I64), ("x_off", I64), ("y_off", I64),
                ("lt", I32), ("ls", I32), ("kb", I32), ("reserved", I32)]


COUPLING_DTYPE = np.dtype({"names": [f for f, _ in CouplingDesc._fields_],
                           "formats": [np.int64 if t is I64 else np.int32 for _, t in CouplingDesc._fields_],
                           "offsets": [getattr(CouplingDesc, f).offset for f, _ in CouplingDesc._fields_],
                           "itemsize": ctypes.sizeof(CouplingDesc)})

KRYLOV_DONE, KRYLOV_PRODUCT_HIGH, KRYLOV_PRODUCT_LOW = 0, 1, 2

EXPORTS = ("uhm_upload", "uhm_upload_h", "uhm_matvec", "uhm_matvec_noalloc", "uhm_solve_gmres", "uhm_krylov_create", "uhm_krylov_next",
           "uhm_krylov_advance", "uhm_krylov_result", "uhm_krylov_free", "uhm_krylov_step",
           "uhm_batch_create", "uhm_batch_run",
           "uhm_batch_tune", "uhm_batch_capture", "uhm_batch_free", "uhm_op_info_get", "uhm_set_timing",
           "uhm_kernel_times", "uhm_free", "uhm_strerror", "uhm_last_error", "uhm_version",
           "uhm_kernel_blocks", "uhm_aca", "uhm_aca_pack", "uhm_cluster_basis", "uhm_cluster_basis_work",
           "uhm_block_recompress", "uhm_block_recompress_work", "uhm_couplings")

_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libuhm.so and declare its signatures.  Raises if the library is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    lib.uhm_upload.argtypes = [ctypes.POINTER(HostOperator), I32, P, ctypes.POINTER(P)]
    lib.uhm_upload.restype = ctypes.c_int
    lib.uhm_upload_h.argtypes = [ctypes.POINTER(HostHMatrix), I32, P, ctypes.POINTER(P)]
    lib.uhm_upload_h.restype = ctypes.c_int
    lib.uhm_matvec.argtypes = [P, P, I64, P, I64, I32, P]
    lib.uhm_matvec.restype = ctypes.c_int
    lib.uhm_matvec_noalloc.argtypes = [P, P, I64, P, I64, I32, P]
    lib.uhm_matvec_noalloc.restype = ctypes.c_int
    lib.uhm_solve_gmres.argtypes = [P, P, P, I64, P, I64, I32, ctypes.c_double, ctypes.POINTER(GmresOpts),
                                    ctypes.POINTER(GmresInfo), P]
    lib.uhm_solve_gmres.restype = ctypes.c_int
    lib.uhm_krylov_create.argtypes = [I64, I32, P, I64, ctypes.c_double, I32, ctypes.POINTER(GmresOpts), P,
                                      ctypes.POINTER(P)]
    lib.uhm_krylov_create.restype = ctypes.c_int
    lib.uhm_krylov_next.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P)]
    lib.uhm_krylov_next.restype = ctypes.c_int
    lib.uhm_krylov_advance.argtypes = [P]
    lib.uhm_krylov_advance.restype = ctypes.c_int
    lib.uhm_krylov_result.argtypes = [P, P, I64, ctypes.POINTER(GmresInfo)]
    lib.uhm_krylov_result.restype = ctypes.c_int
    lib.uhm_krylov_free.argtypes = [P]
    lib.uhm_krylov_free.restype = None
    lib.uhm_krylov_step.argtypes = [ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), I32, P]
    lib.uhm_krylov_step.restype = ctypes.c_int
    lib.uhm_batch_create.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(P),
                                     ctypes.POINTER(I64), ctypes.POINTER(I32), P, ctypes.POINTER(P)]
    lib.uhm_batch_create.restype = ctypes.c_int
    lib.uhm_batch_run.argtypes = [P, P]
    lib.uhm_batch_run.restype = ctypes.c_int
    lib.uhm_batch_tune.argtypes = [P, P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]
    lib.uhm_batch_tune.restype = ctypes.c_int
    lib.uhm_batch_capture.argtypes = [P, P]
    lib.uhm_batch_capture.restype = ctypes.c_int
    lib.uhm_batch_free.argtypes = [P]
    lib.uhm_batch_free.restype = None
    lib.uhm_op_info_get.argtypes = [P, ctypes.POINTER(OpInfo)]
    lib.uhm_op_info_get.restype = ctypes.c_int
    lib.uhm_set_timing.argtypes = [P, ctypes.c_int]
    lib.uhm_set_timing.restype = ctypes.c_int
    lib.uhm_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(I64), I32]
    lib.uhm_kernel_times.restype = ctypes.c_int
    lib.uhm_free.argtypes = [P]
    lib.uhm_free.restype = None
    lib.uhm_strerror.argtypes = [ctypes.c_int]
    lib.uhm_strerror.restype = ctypes.c_char_p
    lib.uhm_last_error.argtypes = []
    lib.uhm_last_error.restype = ctypes.c_char_p
    lib.uhm_version.restype = ctypes.c_int
    D = ctypes.c_double
    lib.uhm_kernel_blocks.argtypes = [P, I64, D, D, P, I64, P, I64, P, P]
    lib.uhm_kernel_blocks.restype = ctypes.c_int
    lib.uhm_aca.argtypes = [P, I64, D, D, P, I64, I32, I32, D, P, I64, P, I64, P, I64, P, P, P]
    lib.uhm_aca_pack.argtypes = [P, I64, P, P, I64, P, I64, P, I32, I32, I32, I32, P, P, P, P]
    lib.uhm_aca_pack.restype = ctypes.c_int
    lib.uhm_aca.restype = ctypes.c_int
    lib.uhm_cluster_basis.argtypes = [P, I32, I32, I32, I32, D, D, P, P, P, P, P, P, P, P, I64, P]
    lib.uhm_cluster_basis.restype = ctypes.c_int
    lib.uhm_cluster_basis_work.argtypes = [I32, I32, I32, I32]
    lib.uhm_cluster_basis_work.restype = I64
    lib.uhm_block_recompress.argtypes = [P, P, I32, I32, I32, I32, D, P, P, P, P, P, P, I64, P]
    lib.uhm_block_recompress.restype = ctypes.c_int
    lib.uhm_block_recompress_work.argtypes = [I32, I32, I32, I32]
    lib.uhm_block_recompress_work.restype = I64
    lib.uhm_couplings.argtypes = [P, I64, P, I64, P, I64, P, I64, P, I64, P, I64, P, P]
    lib.uhm_couplings.restype = ctypes.c_int
    _LIB = lib
    return lib


class UhmError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load_library()
        self.code = code
        super().__init__(f"{where}: {lib.uhm_strerror(code).decode()} ({code}): {lib.uhm_last_error().decode()}")


def _check(rc: int, where: str):
    if rc != UHM_OK:
        raise UhmError(rc, where)


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class DeviceOperator:
    """An operator uploaded to the current HIP device (UH form or H form)."""

    def __init__(self, handle, kind: str, storage: str, n: int):
        self._h = handle
        self.kind = kind
        self.storage = storage
        self.n = n

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = OpInfo()
        _check(load_library().uhm_op_info_get(self._h, ctypes.byref(inf)), "uhm_op_info_get")
        return {name: getattr(inf, name) for name, _ in OpInfo._fields_}

    def matvec(self, x, y=None, stream=None):
        """y = A x for a torch tensor x (n,) or (n, r) on the device; returns y."""
        return self._product("uhm_matvec", x, y, stream)

    def matvec_noalloc(self, x, y=None, stream=None):
        """y = A x through uhm_matvec_noalloc (no device allocation in the library; the
        product scratch is the library's file-scope array).  Pass y to keep the call itself
        free of allocations: without it this wrapper allocates y with torch."""
        return self._product("uhm_matvec_noalloc", x, y, stream)

    def _product(self, entry, x, y, stream):
        import torch
        want = torch.complex128 if self.storage in C128_FORMS else torch.complex64
        if x.dtype != want or not x.is_cuda:
            raise ValueError(f"x must be a {want} device tensor")
        vec = x.dim() == 1
        x2 = x.reshape(self.n, 1) if vec else x
        if x2.shape[0] != self.n:
            raise ValueError("x has the wrong number of rows")
        # column-major view: stride (1, ld)
        if x2.stride(0) != 1:
            x2 = x2.t().contiguous().t()
        nrhs = x2.shape[1]
        if y is None:
            y2 = torch.empty((nrhs, self.n), dtype=want, device=x.device).t()
        else:
            y2 = y.reshape(self.n, 1) if y.dim() == 1 else y
            if y2.stride(0) != 1 or y2.dtype != want or tuple(y2.shape) != (self.n, nrhs):
                raise ValueError("y must be a column-major (n, nrhs) tensor of the operator's dtype")
        ldx = x2.stride(1) if nrhs > 1 else self.n
        ldy = y2.stride(1) if nrhs > 1 else self.n
        sh, _ = _stream_handle(stream)
        rc = getattr(load_library(), entry)(self._h, ctypes.c_void_p(x2.data_ptr()), ldx,
                                            ctypes.c_void_p(y2.data_ptr()), ldy, nrhs, sh)
        _check(rc, entry)
        if y is not None:
            return y
        return y2.reshape(self.n) if vec else y2

    def set_timing(self, enabled: bool):
        _check(load_library().uhm_set_timing(self._h, int(bool(enabled))), "uhm_set_timing")

    def kernel_times(self) -> dict:
        cap = 32
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (I64 * cap)()
        k = load_library().uhm_kernel_times(self._h, names, ms, cnt, cap)
        if k < 0:
            _check(k, "uhm_kernel_times")
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(k, cap))}

    def free(self):
        if self._h:
            load_library().uhm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def upload(op, storage: str = "c128", stream=None) -> DeviceOperator:
    """Upload the UH form of a host operator (builder.HostOperator or a mapping with the
    same keys)."""
    g = (lambda k: op[k]) if isinstance(op, dict) else (lambda k: getattr(op, k))
    keep = {}

    def a(name, dtype):
        arr, p = _arr(g(name), dtype)
        keep[name] = arr
        return p

    h = HostOperator()
    h.n = int(g("n"))
    h.perm = a("perm", np.int64)
    h.nclusters = int(np.asarray(g("off")).size)
    h.off = a("off", np.int64)
    h.size = a("size", np.int64)
    h.parent = a("parent", np.int32)
    h.rank_row = a("rank_row", np.int32)
    h.rank_col = a("rank_col", np.int32)
    h.U_off = a("U_off", np.int64)
    h.V_off = a("V_off", np.int64)
    h.U = a("U", np.complex128)
    h.U_len = keep["U"].size
    h.V = a("V", np.complex128)
    h.V_len = keep["V"].size
    h.nadm = int(np.asarray(g("adm_row")).size)
    h.adm_row = a("adm_row", np.int32)
    h.adm_col = a("adm_col", np.int32)
    h.S_off = a("S_off", np.int64)
    h.S = a("S", np.complex128)
    h.S_len = keep["S"].size
    h.nden = int(np.asarray(g("den_row")).size)
    h.den_row = a("den_row", np.int32)
    h.den_col = a("den_col", np.int32)
    h.D_off = a("D_off", np.int64)
    h.D = a("D", np.complex128)
    h.D_len = keep["D"].size
    if storage in FACTORED_FORMS:
        h.adm_rank = a("adm_rank", np.int32)
        h.SX_off = a("SX_off", np.int64)
        h.SY_off = a("SY_off", np.int64)
        h.SX = a("SX", np.complex128)
        h.SX_len = keep["SX"].size
        h.SY = a("SY", np.complex128)
        h.SY_len = keep["SY"].size
    out = P()
    sh, _ = _stream_handle(stream)
    _check(load_library().uhm_upload(ctypes.byref(h), STORAGE[storage], sh, ctypes.byref(out)), "uhm_upload")
    return DeviceOperator(out, "uh", storage, h.n)


def upload_h(op, storage: str = "c128", stream=None) -> DeviceOperator:
    """Upload the H form (X_b, Y_b and the dense blocks) of a host operator."""
    g = (lambda k: op[k]) if isinstance(op, dict) else (lambda k: getattr(op, k))
    keep = {}

    def a(name, dtype):
        arr, p = _arr(g(name), dtype)
        keep[name] = arr
        return p

    h = HostHMatrix()
    h.n = int(g("n"))
    h.perm = a("perm", np.int64)
    h.nclusters = int(np.asarray(g("off")).size)
    h.off = a("off", np.int64)
    h.size = a("size", np.int64)
    h.parent = a("parent", np.int32)
    h.nadm = int(np.asarray(g("adm_row")).size)
    h.adm_row = a("adm_row", np.int32)
    h.adm_col = a("adm_col", np.int32)
    h.adm_rank = a("adm_rank", np.int32)
    h.X_off = a("X_off", np.int64)
    h.Y_off = a("Y_off", np.int64)
    h.X = a("X", np.complex128)
    h.X_len = keep["X"].size
    h.Y = a("Y", np.complex128)
    h.Y_len = keep["Y"].size
    h.nden = int(np.asarray(g("den_row")).size)
    h.den_row = a("den_row", np.int32)
    h.den_col = a("den_col", np.int32)
    h.D_off = a("D_off", np.int64)
    h.D = a("D", np.complex128)
    h.D_len = keep["D"].size
    out = P()
    sh, _ = _stream_handle(stream)
    _check(load_library().uhm_upload_h(ctypes.byref(h), STORAGE[storage], sh, ctypes.byref(out)), "uhm_upload_h")
    return DeviceOperator(out, "h", storage, h.n)


def solve_gmres(op: DeviceOperator, b, tol: float, inner: DeviceOperator | None = None, restart: int = 50,
                max_iterations: int = 2000, max_refinements: int = 30, inner_tol: float = 1e-4, x=None,
                stream=None, raise_on_noconv: bool = True, inner_cycles: int = 0):
    """Solve A X = B with GMRES(restart) (inner=None) or GMRES-IR with the low-precision
    operator `inner` (inner_cycles > 0: an inner solve also ends after that many cycles).
    b: complex128 device tensor (n,) or (n, r).  Returns (x, info dict, code)."""
    import torch
    if op.storage not in C128_FORMS:
        raise ValueError("the residual operator must be complex128")
    vec = b.dim() == 1
    b2 = b.reshape(op.n, 1) if vec else b
    if b2.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    if b2.stride(0) != 1:
        b2 = b2.t().contiguous().t()
    r = b2.shape[1]
    if x is None:
        x2 = torch.empty((r, op.n), dtype=torch.complex128, device=b.device).t()
    else:
        x2 = x.reshape(op.n, 1) if x.dim() == 1 else x
    ldb = b2.stride(1) if r > 1 else op.n
    ldx = x2.stride(1) if r > 1 else op.n
    o = GmresOpts(restart, max_iterations, max_refinements, inner_tol, inner_cycles)
    inf = GmresInfo()
    sh, _ = _stream_handle(stream)
    rc = load_library().uhm_solve_gmres(op.handle, inner.handle if inner is not None else None,
                                        ctypes.c_void_p(b2.data_ptr()), ldb, ctypes.c_void_p(x2.data_ptr()), ldx, r,
                                        float(tol), ctypes.byref(o), ctypes.byref(inf), sh)
    info = {name: getattr(inf, name) for name, _ in GmresInfo._fields_}
    if rc not in (UHM_OK, UHM_ENOCONV) or (rc == UHM_ENOCONV and raise_on_noconv):
        raise UhmError(rc, "uhm_solve_gmres")
    out = x if x is not None else (x2.reshape(op.n) if vec else x2)
    return out, info, rc


class Batch:
    """A bound set of products Y_k = A_k X_k run stage by stage in shared launches.

    xs, ys: column-major device tensors (n_k, r_k) (or (n_k,)) of the operators' dtype;
    they stay bound to the batch (keep them alive)."""

    def __init__(self, ops, xs, ys, stream=None):
        import torch
        k = len(ops)
        self._keep = (list(ops), list(xs), list(ys))
        oph = (P * k)(*[o.handle for o in ops])
        xp, yp = (P * k)(), (P * k)()
        ldx, ldy, nr = (I64 * k)(), (I64 * k)(), (I32 * k)()
        for i, (o, x, y) in enumerate(zip(ops, xs, ys)):
            want = torch.complex128 if o.storage in C128_FORMS else torch.complex64
            x2 = x.reshape(o.n, 1) if x.dim() == 1 else x
            y2 = y.reshape(o.n, 1) if y.dim() == 1 else y
            if x2.dtype != want or y2.dtype != want or x2.stride(0) != 1 or y2.stride(0) != 1:
                raise ValueError("batch vectors must be column-major tensors of the operator's dtype")
            xp[i] = x2.data_ptr()
            yp[i] = y2.data_ptr()
            ldx[i] = x2.stride(1) if x2.shape[1] > 1 else o.n
            ldy[i] = y2.stride(1) if y2.shape[1] > 1 else o.n
            nr[i] = x2.shape[1]
        out = P()
        sh, _ = _stream_handle(stream)
        _check(load_library().uhm_batch_create(oph, k, xp, ldx, yp, ldy, nr, sh, ctypes.byref(out)), "uhm_batch_create")
        self._h = out

    def run(self, stream=None):
        sh, _ = _stream_handle(stream)
        _check(load_library().uhm_batch_run(self._h, sh), "uhm_batch_run")

    def tune(self, stream=None):
        w, o, ms = I32(), I32(), ctypes.c_double()
        sh, _ = _stream_handle(stream)
        _check(load_library().uhm_batch_tune(self._h, sh, ctypes.byref(w), ctypes.byref(o), ctypes.byref(ms)),
               "uhm_batch_tune")
        return {"tile_width": w.value, "order": o.value, "best_ms": ms.value}

    def capture(self, stream):
        sh, _ = _stream_handle(stream)
        _check(load_library().uhm_batch_capture(self._h, sh), "uhm_batch_capture")

    def free(self):
        if getattr(self, "_h", None):
            load_library().uhm_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Krylov:
    """A resumable GMRES / GMRES-IR solve of A X = B (reverse communication).

    The products are performed by the caller: alone through `product`, or for many solves
    at once through `krylov_step`."""

    def __init__(self, b, tol: float, mixed: bool, restart: int = 50, max_iterations: int = 2000,
                 max_refinements: int = 30, inner_tol: float = 1e-4, stream=None, inner_cycles: int = 0):
        import torch
        b2 = b.reshape(-1, 1) if b.dim() == 1 else b
        if b2.dtype != torch.complex128:
            raise ValueError("b must be complex128")
        if b2.stride(0) != 1:
            b2 = b2.t().contiguous().t()
        self.n, self.r = b2.shape
        ldb = b2.stride(1) if self.r > 1 else self.n
        o = GmresOpts(restart, max_iterations, max_refinements, inner_tol, inner_cycles)
        out = P()
        sh, _ = _stream_handle(stream)
        _check(load_library().uhm_krylov_create(self.n, self.r, ctypes.c_void_p(b2.data_ptr()), ldb, float(tol),
                                                int(bool(mixed)), ctypes.byref(o), sh, ctypes.byref(out)),
               "uhm_krylov_create")
        self._h = out
        self.mixed = bool(mixed)

    @property
    def handle(self):
        return self._h

    def pending(self) -> int:
        return load_library().uhm_krylov_next(self._h, None, None)

    def result(self, x=None):
        """Returns (x, info, code); x: (n, r) complex128 tensor (allocated if None)."""
        import torch
        if x is None:
            x = torch.empty((self.r, self.n), dtype=torch.complex128, device="cuda").t()
        ldx = x.stride(1) if self.r > 1 else self.n
        inf = GmresInfo()
        rc = load_library().uhm_krylov_result(self._h, ctypes.c_void_p(x.data_ptr()), ldx, ctypes.byref(inf))
        if rc not in (UHM_OK, UHM_ENOCONV):
            raise UhmError(rc, "uhm_krylov_result")
        return x, {name: getattr(inf, name) for name, _ in GmresInfo._fields_}, rc

    def free(self):
        if getattr(self, "_h", None):
            load_library().uhm_krylov_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def krylov_step(solves, highs, lows=None, stream=None) -> int:
    """Advance many solves by one product each (grouped per operator).  Returns the number
    still running."""
    k = len(solves)
    hs = (P * k)(*[s.handle for s in solves])
    hi = (P * k)(*[o.handle for o in highs])
    lo = (P * k)(*[(o.handle if o is not None else None) for o in lows]) if lows is not None else None
    sh, _ = _stream_handle(stream)
    rc = load_library().uhm_krylov_step(hs, hi, lo, k, sh)
    if rc < 0:
        raise UhmError(rc, "uhm_krylov_step")
    return rc


# --------------------------------------------------------------------------- construction
def _points_on_device(points):
    import torch
    if isinstance(points, torch.Tensor):
        if points.device.type != "cuda" or points.dtype != torch.float64 or points.dim() != 2 \
                or points.shape[1] != 3 or not points.is_contiguous():
            raise ValueError("points must be a contiguous (n, 3) float64 tensor on the HIP device")
        return points
    a = np.ascontiguousarray(points, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("points must have shape (n, 3)")
    return torch.from_numpy(a).to("cuda")


def _descs(row_off, rows, col_off, cols, cap=None):
    nb = len(rows)
    d = np.zeros(nb, BLOCK_DTYPE)
    d["row_off"], d["rows"], d["col_off"], d["cols"] = row_off, rows, col_off, cols
    if cap is not None:
        d["cap"] = cap
    return d


def _to_device(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8)).to("cuda")


def kernel_blocks(points, kappa: float, diag: float, row_off, rows, col_off, cols, stream=None):
    """Dense blocks A[row_off:row_off+rows, col_off:col_off+cols] of the point-kernel matrix,
    computed on the device (uhm_kernel_blocks).  Returns (D, offsets): D a flat complex128
    device tensor holding block b column-major at offsets[b]."""
    import torch
    lib = load_library()
    pts = _points_on_device(points)
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    d = _descs(row_off, rows, col_off, cols)
    sz = rows * cols
    d["a_off"] = np.concatenate([[0], np.cumsum(sz)[:-1]]) if len(sz) else []
    total = int(sz.sum())
    h, stream = _stream_handle(stream)
    with torch.cuda.stream(stream):   # allocations, copies and the launch in one stream order
        D = torch.empty(total, dtype=torch.complex128, device="cuda")
        status = torch.empty(len(rows), dtype=torch.int32, device="cuda")
        dd = _to_device(d)
        _check(lib.uhm_kernel_blocks(ctypes.c_void_p(pts.data_ptr()), pts.shape[0], float(kappa), float(diag),
                                     ctypes.c_void_p(dd.data_ptr()), len(rows), ctypes.c_void_p(D.data_ptr()), total,
                                     ctypes.c_void_p(status.data_ptr()), h), "uhm_kernel_blocks")
        st = status.cpu().numpy()
    if (st != 1).any():
        raise UhmError(UHM_EINVAL, f"uhm_kernel_blocks: {int((st != 1).sum())} descriptors rejected")
    return D, d["a_off"].copy()


class AcaResult:
    """Device outputs of uhm_aca for a list of blocks: U, V (flat complex128 tensors), piv
    (int32 tensor), the host arrays rank, status, and the per-block offsets u_off, v_off, p_off
    and caps."""

    def __init__(self, U, V, piv, rank, status, desc, desc_dev=None, rank_dev=None):
        self.U, self.V, self.piv = U, V, piv
        self.rank, self.status = rank, status
        self.desc_dev, self.rank_dev = desc_dev, rank_dev   # the call's device descriptors and ranks
        self.u_off, self.v_off, self.p_off = desc["a_off"].copy(), desc["b_off"].copy(), desc["p_off"].copy()
        self.rows, self.cols, self.cap = (desc["rows"].astype(np.int64), desc["cols"].astype(np.int64),
                                          desc["cap"].astype(np.int64))

    def factors(self, b: int):
        """(u (m x k), v (n x k), pivot rows, pivot columns) of block b, on the host."""
        m, n, k, c = int(self.rows[b]), int(self.cols[b]), int(self.rank[b]), int(self.cap[b])
        u = self.U[self.u_off[b]:self.u_off[b] + m * k].cpu().numpy().reshape(k, m).T
        v = self.V[self.v_off[b]:self.v_off[b] + n * k].cpu().numpy().reshape(k, n).T
        p = self.piv[self.p_off[b]:self.p_off[b] + 2 * c].cpu().numpy()
        return u, v, p[:k].astype(np.int64), p[c:c + k].astype(np.int64)


def aca(points, kappa: float, diag: float, row_off, rows, col_off, cols, cap, eps: float, stream=None) -> AcaResult:
    """ACA with partial pivoting of every block on the device (uhm_aca), one workgroup per
    block, in the order given.  cap: most terms per block (scalar or per block)."""
    import torch
    lib = load_library()
    pts = _points_on_device(points)
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    nb = len(rows)
    cap = np.broadcast_to(np.asarray(cap, np.int64), (nb,)).copy()
    d = _descs(row_off, rows, col_off, cols, cap)
    usz, vsz, psz = rows * cap, cols * cap, 2 * cap
    d["a_off"] = np.concatenate([[0], np.cumsum(usz)[:-1]]) if nb else []
    d["b_off"] = np.concatenate([[0], np.cumsum(vsz)[:-1]]) if nb else []
    d["p_off"] = np.concatenate([[0], np.cumsum(psz)[:-1]]) if nb else []
    h, stream = _stream_handle(stream)
    max_rows = int(rows.max()) if nb else 1
    max_cap = int(cap.max()) if nb else 1
    with torch.cuda.stream(stream):   # allocations, copies and the launch in one stream order
        U = torch.zeros(int(usz.sum()), dtype=torch.complex128, device="cuda")
        V = torch.zeros(int(vsz.sum()), dtype=torch.complex128, device="cuda")
        piv = torch.full((int(psz.sum()),), -1, dtype=torch.int32, device="cuda")
        rank = torch.zeros(nb, dtype=torch.int32, device="cuda")
        status = torch.zeros(nb, dtype=torch.int32, device="cuda")
        dd = _to_device(d)
        _check(lib.uhm_aca(ctypes.c_void_p(pts.data_ptr()), pts.shape[0], float(kappa), float(diag),
                           ctypes.c_void_p(dd.data_ptr()), nb, max_rows, max_cap, float(eps),
                           ctypes.c_void_p(U.data_ptr()), U.numel(), ctypes.c_void_p(V.data_ptr()), V.numel(),
                           ctypes.c_void_p(piv.data_ptr()), piv.numel(), ctypes.c_void_p(rank.data_ptr()),
                           ctypes.c_void_p(status.data_ptr()), h), "uhm_aca")
        st = status.cpu().numpy()
        rk = rank.cpu().numpy()
    if (st < 0).any():
        raise UhmError(UHM_EINVAL, f"uhm_aca: {int((st < 0).sum())} descriptors rejected")
    return AcaResult(U, V, piv, rk, st, d, dd, rank)


def aca_pack(res: AcaResult, sel, m: int, n: int, kp: int, stream=None):
    """The factors of blocks `sel` of an ACA result (all m x n) packed by uhm_aca_pack:
    X (cnt, m, kp) and Y (cnt, n, kp) device tensors with A|_b ~ X Y^H, zero columns beyond
    each block's rank."""
    import torch
    lib = load_library()
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    cnt = int(sel.size)
    h, stream = _stream_handle(stream)
    with torch.cuda.stream(stream):
        X = torch.empty((cnt, m, kp), dtype=torch.complex128, device="cuda")
        Y = torch.empty((cnt, n, kp), dtype=torch.complex128, device="cuda")
        status = torch.empty(max(1, cnt), dtype=torch.int32, device="cuda")
        sd = torch.from_numpy(sel).to("cuda")
        _check(lib.uhm_aca_pack(ctypes.c_void_p(res.desc_dev.data_ptr()), len(res.rows),
                                ctypes.c_void_p(res.rank_dev.data_ptr()), ctypes.c_void_p(res.U.data_ptr()),
                                res.U.numel(), ctypes.c_void_p(res.V.data_ptr()), res.V.numel(),
                                ctypes.c_void_p(sd.data_ptr()), cnt, int(m), int(n), int(kp),
                                ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                ctypes.c_void_p(status.data_ptr()), h), "uhm_aca_pack")
        st = status.cpu().numpy()[:cnt]
    if (st != 1).any():
        raise UhmError(UHM_EINVAL, f"uhm_aca_pack: {int((st != 1).sum())} blocks rejected")
    return X, Y


class ClusterBasis:
    """Results of uhm_cluster_basis for a batch: device tensors U (batch, pmax, m) holding
    U_c^T row by row (column i of U_c is U[c, i, :]), SV (batch, n, pmax) holding (Sigma
    V^*)^T, sv (batch, pmax); host arrays rank, psteps, stats (batch, 3) and status."""

    def __init__(self, U, SV, sv, rank, psteps, stats, status):
        self.U, self.SV, self.sv = U, SV, sv
        self.rank, self.psteps, self.stats, self.status = rank, psteps, stats, status

    def basis(self, c: int):
        """U_c (m x l) and Sigma V^* (l x n) of matrix c as host arrays."""
        l = int(self.rank[c])
        return self.U[c, :l, :].cpu().numpy().T, self.SV[c, :, :l].cpu().numpy().T


def cluster_basis(X, eps: float, tol: float | None = None, pmax: int | None = None, stream=None) -> ClusterBasis:
    """Alg. 2's factorisation of a batch of cluster matrices X (batch, m, n), complex128
    (host or device, row-major; the library only reads it), on the device (uhm_cluster_basis).
    tol defaults to sqrt(1e-16 eps), where the rank test is that of a full SVD up to rounding."""
    import torch
    lib = load_library()
    Xt = torch.as_tensor(X)
    batch, m, n = (int(v) for v in Xt.shape)
    pmax = int(min(m, n, 2048) if pmax is None else pmax)
    if tol is None:
        tol = float(np.sqrt(1e-16 * max(eps, 0.0)))
    h, stream = _stream_handle(stream)
    with torch.cuda.stream(stream):
        Xd = Xt.to(device="cuda", dtype=torch.complex128).contiguous()
        need = int(lib.uhm_cluster_basis_work(batch, m, n, pmax))
        if need < 0:
            raise UhmError(UHM_EINVAL, "uhm_cluster_basis_work: sizes rejected")
        work = torch.empty(max(1, need), dtype=torch.float64, device="cuda")
        U = torch.empty((batch, pmax, m), dtype=torch.complex128, device="cuda")
        SV = torch.empty((batch, n, pmax), dtype=torch.complex128, device="cuda")
        sv = torch.empty((batch, pmax), dtype=torch.float64, device="cuda")
        rank = torch.empty(max(1, batch), dtype=torch.int32, device="cuda")
        psteps = torch.empty(max(1, batch), dtype=torch.int32, device="cuda")
        stats = torch.empty((max(1, batch), 3), dtype=torch.float64, device="cuda")
        status = torch.empty(max(1, batch), dtype=torch.int32, device="cuda")
        _check(lib.uhm_cluster_basis(ctypes.c_void_p(Xd.data_ptr()), batch, m, n, pmax, float(tol), float(eps),
                                     ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(SV.data_ptr()),
                                     ctypes.c_void_p(sv.data_ptr()), ctypes.c_void_p(rank.data_ptr()),
                                     ctypes.c_void_p(psteps.data_ptr()), ctypes.c_void_p(stats.data_ptr()),
                                     ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(work.data_ptr()), need, h),
               "uhm_cluster_basis")
        res = ClusterBasis(U, SV, sv, rank.cpu().numpy()[:batch], psteps.cpu().numpy()[:batch],
                           stats.cpu().numpy()[:batch], status.cpu().numpy()[:batch])
        del Xd, work
    return res


def block_recompress(X, Y, eps: float, stream=None):
    """The recompression of a batch of ACA factor pairs (uhm_block_recompress): X (batch, m,
    kp) and Y (batch, n, kp) complex128 with A|_b ~ X[c] Y[c]^H (host or device, row-major;
    only read).
    Returns device tensors U (batch, kp, m) and V (batch, kp, n) holding U_c^T and V_c^T row
    by row, sv (batch, kp), and host arrays rank and status."""
    import torch
    lib = load_library()
    Xt, Yt = torch.as_tensor(X), torch.as_tensor(Y)
    batch, m, kp = (int(v) for v in Xt.shape)
    n = int(Yt.shape[1])
    if tuple(Yt.shape) != (batch, n, kp):
        raise UhmError(UHM_EINVAL, "block_recompress: X and Y disagree in batch or kp")
    h, stream = _stream_handle(stream)
    with torch.cuda.stream(stream):
        Xd = Xt.to(device="cuda", dtype=torch.complex128).contiguous()
        Yd = Yt.to(device="cuda", dtype=torch.complex128).contiguous()
        need = int(lib.uhm_block_recompress_work(batch, m, n, kp))
        if need < 0:
            raise UhmError(UHM_EINVAL, "uhm_block_recompress_work: sizes rejected")
        work = torch.empty(max(1, need), dtype=torch.float64, device="cuda")
        U = torch.empty((batch, kp, m), dtype=torch.complex128, device="cuda")
        V = torch.empty((batch, kp, n), dtype=torch.complex128, device="cuda")
        sv = torch.empty((batch, kp), dtype=torch.float64, device="cuda")
        rank = torch.empty(max(1, batch), dtype=torch.int32, device="cuda")
        status = torch.empty(max(1, batch), dtype=torch.int32, device="cuda")
        _check(lib.uhm_block_recompress(ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Yd.data_ptr()), batch, m, n,
                                        kp, float(eps), ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                        ctypes.c_void_p(sv.data_ptr()), ctypes.c_void_p(rank.data_ptr()),
                                        ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(work.data_ptr()), need, h),
               "uhm_block_recompress")
        rk = rank.cpu().numpy()[:batch]
        stt = status.cpu().numpy()[:batch]
        del Xd, Yd, work
    return U, V, sv, rk, stt


def couplings(L, sigma, desc, S_len: int, SX_len: int, SY_len: int, stream=None):
    """The couplings S_b, S_{X,b}, S_{Y,b} of every block in desc (a COUPLING_DTYPE record array)
    on the device (uhm_couplings).  L: complex128 device tensor of the clusters' coefficient
    rows, sigma: float64 (host or device).  Returns flat complex128 device tensors S, SX, SY."""
    import torch
    lib = load_library()
    desc = np.ascontiguousarray(desc, dtype=COUPLING_DTYPE)
    nb = int(desc.shape[0])
    h, stream = _stream_handle(stream)
    with torch.cuda.stream(stream):
        sig = torch.as_tensor(sigma).to(device="cuda", dtype=torch.float64).contiguous()
        S = torch.empty(max(1, S_len), dtype=torch.complex128, device="cuda")
        SX = torch.empty(max(1, SX_len), dtype=torch.complex128, device="cuda")
        SY = torch.empty(max(1, SY_len), dtype=torch.complex128, device="cuda")
        status = torch.zeros(max(1, nb), dtype=torch.int32, device="cuda")
        dd = torch.from_numpy(desc.view(np.uint8)).to("cuda") if nb else torch.empty(1, dtype=torch.uint8,
                                                                                      device="cuda")
        _check(lib.uhm_couplings(ctypes.c_void_p(L.data_ptr()), int(L.numel()), ctypes.c_void_p(sig.data_ptr()),
                                 int(sig.numel()), ctypes.c_void_p(dd.data_ptr()), nb, ctypes.c_void_p(S.data_ptr()),
                                 int(S_len), ctypes.c_void_p(SX.data_ptr()), int(SX_len),
                                 ctypes.c_void_p(SY.data_ptr()), int(SY_len), ctypes.c_void_p(status.data_ptr()), h),
               "uhm_couplings")
        st = status.cpu().numpy()[:nb]
    if (st != 1).any():
        raise UhmError(UHM_EINVAL, f"uhm_couplings: {int((st != 1).sum())} descriptors rejected")
    return S, SX, SY

