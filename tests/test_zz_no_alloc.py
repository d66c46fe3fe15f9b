"""uhm_matvec_noalloc: the product without any device allocation in the library.

The entry point takes its scratch from a file-scope device array instead of the
operator's workspace.  It is called here through the C-ABI (ctypes, caller-allocated
output) twice in a row, the second time with a smaller operator and fewer right-hand
sides, and each result is compared with uhm_matvec's on the same operator (same kernels in
the same order: bitwise equal) and with the CPU oracle (the FP64 parity bar, 1e-12 per
right-hand side).  Storage forms: general, symmetric (Remark 4.4) and factored
(section 4.2) UH storage, and the H-matrix comparator (Algorithm 5).
"""
import ctypes

import numpy as np
import pytest

from conftest import operator
from oracle import uniform
from paper_2405_15573_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    from paper_2405_15573_amd import binding
    binding.load_library()
    return torch


def _colmajor(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda").t()


def _abi_noalloc(torch, dop, xt):
    """uhm_matvec_noalloc through ctypes, into a column-major output allocated here."""
    from paper_2405_15573_amd import binding
    n, r = xt.shape
    yt = torch.empty((r, n), dtype=xt.dtype, device=xt.device).t()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # a single column's leading dimension is n (torch gives its transposed view stride 1)
    ldx, ldy = (xt.stride(1), yt.stride(1)) if r > 1 else (n, n)
    rc = binding.load_library().uhm_matvec_noalloc(dop._h, ctypes.c_void_p(xt.data_ptr()), ldx,
                                                   ctypes.c_void_p(yt.data_ptr()), ldy, r, stream)
    assert rc == 0, binding.load_library().uhm_last_error()
    return yt


def _images(op, form):
    from paper_2405_15573_amd import builder
    if form == "c128":
        return op, vars(op)
    if form == "c128sym":
        sym = builder.symmetric_image(op)
        return sym, uniform.expand_symmetric(sym)
    if form == "c128fact":
        return op, uniform.assemble_factored(vars(op), "smaller")
    raise ValueError(form)


@pytest.mark.parametrize("form", ["c128", "c128sym", "c128fact", "h"])
def test_noalloc_equals_matvec_twice(torch_dev, form):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    # the second call has the smaller operator and fewer right-hand sides
    for surface, n, seed, leaf, r in (("sphere", 6000, 11, 64, 3), ("cube", 1300, 5, 32, 1)):
        print(f"case noalloc {form} {surface} n={n} seed={seed} nrhs={r}", flush=True)
        cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
        if form == "h":
            dop = binding.upload_h(op)
            ref_img = None
        else:
            img, ref_img = _images(op, form)
            dop = binding.upload(img, form)
        x = inputs.make_rhs(cloud.n, r, seed=seed)
        xt = _colmajor(torch, x)
        y_na = _abi_noalloc(torch, dop, xt)
        y_mv = dop.matvec(xt)
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_mv.cpu().numpy()
        dop.free()
        assert np.array_equal(a, b), "uhm_matvec_noalloc differs from uhm_matvec"
        ref = uniform.h_mvp(vars(op), x) if form == "h" else uniform.uh_mvp(ref_img, x)
        errs = [float(np.linalg.norm(a[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j])) for j in range(r)]
        print(f"  parity vs oracle {max(errs):.2e}", flush=True)
        assert max(errs) <= TOL


def test_noalloc_rejects_many_rhs_storage(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    cloud, op = operator()
    dop = binding.upload(op, "c64")
    xt = _colmajor(torch, inputs.make_rhs(cloud.n, 1, seed=0).astype(np.complex64))
    yt = torch.empty_like(xt)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = binding.load_library().uhm_matvec_noalloc(dop._h, ctypes.c_void_p(xt.data_ptr()), cloud.n,
                                                   ctypes.c_void_p(yt.data_ptr()), cloud.n, 1, stream)
    dop.free()
    assert rc == binding.UHM_ENOTSUP
