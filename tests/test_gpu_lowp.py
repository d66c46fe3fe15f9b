"""GPU parity of the low-precision storage forms (complex64 and bf16 pairs, FP32 accumulation,
MFMA kernels), one to many right-hand sides.

Two comparisons per case:
  * against the FP64 definition applied to the same operator rounded to the storage
    format (isolates the kernels' FP32 arithmetic): <= 2e-5 relative per column;
  * against the FP64 definition on the FP64 operator: complex64 <= 1e-5 (the bar for the
    FP32 form); bf16 pairs: the error is stated (storage rounding 2^-9), <= 2e-2.
"""
import numpy as np
import pytest

from conftest import operator
from oracle import precision, uniform
from paper_2405_15573_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    from paper_2405_15573_amd import binding
    binding.load_library()
    return torch


def _col_rel(y, ref):
    y = y.reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.array([np.linalg.norm(y[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j]) for j in range(ref.shape[1])])


def _run(torch, dop, x, ld_pad=0):
    n, r = x.shape
    ld = n + ld_pad
    buf = torch.zeros((r, ld), dtype=torch.complex64, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(x.T.astype(np.complex64))).to("cuda")
    xv = buf.t()[:n]
    ybuf = torch.zeros((r, ld + 3), dtype=torch.complex64, device="cuda")
    yv = ybuf.t()[:n]
    dop.matvec(xv, yv)
    torch.cuda.synchronize()
    return yv.cpu().numpy().astype(np.complex128)


CASES = [("sphere", 2048, 0, 32), ("sphere", 3000, 3, 64), ("cube", 1300, 5, 32), ("ellipsoid", 1500, 4, 32)]


@pytest.mark.parametrize("storage", ["c64", "bf16pair", "c64stream", "bf16pairstream"])
@pytest.mark.parametrize("surface,n,seed,leaf", CASES)
def test_lowp_single_rhs(torch_dev, storage, surface, n, seed, leaf):
    """The MFMA forms (one column padded to 16) and the streaming forms (one lane per panel
    column or row, the complex128 layout with compact elements)."""
    from paper_2405_15573_amd import binding
    print(f"case {storage} {surface} n={n} seed={seed} leaf={leaf}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    dop = binding.upload(op, storage=storage)
    x = inputs.make_rhs(cloud.n, 1, seed=seed).astype(np.complex64).astype(np.complex128)
    y = _run(torch_dev, dop, x)
    ref_r = uniform.uh_mvp(precision.round_operator(vars(op), storage.replace("stream", "")), x)
    ref = uniform.uh_mvp(vars(op), x)
    e_arith = _col_rel(y, ref_r).max()
    e_full = _col_rel(y, ref).max()
    print(f"  arithmetic err {e_arith:.2e}  vs FP64 operator {e_full:.2e}", flush=True)
    assert e_arith <= 2e-5
    assert e_full <= (1e-5 if storage.startswith("c64") else 2e-2)
    assert dop.info()["storage"] == binding.STORAGE[storage]


@pytest.mark.parametrize("storage", ["c64", "bf16pair"])
@pytest.mark.parametrize("nrhs", [2, 16, 17, 64, 70])
def test_lowp_multi_rhs(torch_dev, storage, nrhs):
    from paper_2405_15573_amd import binding
    print(f"case {storage} nrhs={nrhs}", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    dop = binding.upload(op, storage=storage)
    x = inputs.make_rhs(cloud.n, nrhs, seed=40 + nrhs).astype(np.complex64).astype(np.complex128)
    y = _run(torch_dev, dop, x, ld_pad=5)
    ref_r = uniform.uh_mvp(precision.round_operator(vars(op), storage), x)
    assert _col_rel(y, ref_r).max() <= 2e-5
    # every column equals the single-column product (same reduction order per column)
    y0 = _run(torch_dev, dop, x[:, :1])
    assert np.linalg.norm(y[:, 0] - y0[:, 0]) / np.linalg.norm(y0[:, 0]) <= 1e-6


@pytest.mark.parametrize("storage", ["c64stream", "bf16pairstream"])
def test_stream_forms_several_columns_and_errors(torch_dev, storage):
    """The streaming forms with several right-hand sides and padded leading dimensions (one
    column after another: each equals its single-column product bitwise), and the calls they
    refuse: the solver step and the allocation-free product take other forms."""
    from paper_2405_15573_amd import binding
    torch = torch_dev
    print(f"case {storage} several columns", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    dop = binding.upload(op, storage=storage)
    x = inputs.make_rhs(cloud.n, 5, seed=45).astype(np.complex64).astype(np.complex128)
    y = _run(torch, dop, x, ld_pad=5)
    ref_r = uniform.uh_mvp(precision.round_operator(vars(op), storage.replace("stream", "")), x)
    assert _col_rel(y, ref_r).max() <= 2e-5
    y2 = _run(torch, dop, x[:, 2:3])
    assert np.array_equal(y[:, 2], y2[:, 0])
    info = dop.info()
    assert info["elem_bytes"] == (8 if storage == "c64stream" else 4) and info["scratch_bytes"] == 0
    xt = torch.from_numpy(np.ascontiguousarray(x[:, 0].astype(np.complex64))).to("cuda")
    with pytest.raises(binding.UhmError):
        dop.matvec_noalloc(xt, torch.empty_like(xt))


def test_lowp_dense_only(torch_dev):
    from paper_2405_15573_amd import binding
    for storage in ("c64", "bf16pair", "c64stream", "bf16pairstream"):
        cloud, op = operator(n=60, leaf=32)
        dop = binding.upload(op, storage=storage)
        x = inputs.make_rhs(cloud.n, 3, seed=1).astype(np.complex64).astype(np.complex128)
        y = _run(torch_dev, dop, x)
        ref_r = uniform.uh_mvp(precision.round_operator(vars(op), storage.replace("stream", "")), x)
        assert _col_rel(y, ref_r).max() <= 2e-5


@pytest.mark.parametrize("storage", ["c128multi", "c128multifact"])
@pytest.mark.parametrize("nrhs", [1, 3, 16, 17, 64, 70])
def test_c128multi_parity(torch_dev, nrhs, storage):
    """complex128 storage in the many-RHS layout (FP64 MFMA), also with factored couplings:
    the FP64 bar, 1e-12 per column."""
    from paper_2405_15573_amd import binding
    torch = torch_dev
    print(f"case {storage} nrhs={nrhs}", flush=True)
    for surface, n, seed, leaf in (("sphere", 3000, 3, 64), ("cube", 1300, 5, 32)):
        cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
        dop = binding.upload(op, storage=storage)
        x = inputs.make_rhs(cloud.n, nrhs, seed=50 + nrhs)
        ld = cloud.n + 7
        buf = torch.zeros((nrhs, ld), dtype=torch.complex128, device="cuda")
        buf[:, :cloud.n] = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")
        ybuf = torch.zeros((nrhs, ld), dtype=torch.complex128, device="cuda")
        dop.matvec(buf.t()[:cloud.n], ybuf.t()[:cloud.n])
        torch.cuda.synchronize()
        y = ybuf.t()[:cloud.n].cpu().numpy()
        ref_op = uniform.assemble_factored(vars(op), "smaller") if storage.endswith("fact") else vars(op)
        assert _col_rel(y, uniform.uh_mvp(ref_op, x)).max() <= 1e-12


@pytest.mark.parametrize("storage", ["c64fact", "bf16pairfact"])
@pytest.mark.parametrize("surface,n,seed,leaf,nrhs", [("sphere", 2048, 0, 32, 1), ("sphere", 3000, 3, 64, 17),
                                                      ("cube", 1300, 5, 32, 64), ("ellipsoid", 1500, 4, 32, 3)])
def test_lowp_factored_couplings(torch_dev, storage, surface, n, seed, leaf, nrhs):
    """Factored couplings on the matrix cores: a first coupling pass forms S_{Y,b}^* u_sigma,
    the main pass applies S_{X,b}.  Reference: the FP64 definition with S_b = S_{X,b} S_{Y,b}^*
    formed from the factors rounded to the storage format where the factors are stored, and
    the rounded S_b elsewhere (the two roundings differ by the storage precision)."""
    from paper_2405_15573_amd import binding
    base = storage[:-4]
    print(f"case {storage} {surface} n={n} nrhs={nrhs}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    dop = binding.upload(op, storage=storage)
    x = inputs.make_rhs(cloud.n, nrhs, seed=seed + 60).astype(np.complex64).astype(np.complex128)
    y = _run(torch_dev, dop, x, ld_pad=3)
    ref_r = uniform.uh_mvp(uniform.assemble_factored(precision.round_operator(vars(op), base), "smaller"), x)
    ref = uniform.uh_mvp(vars(op), x)
    e_arith = _col_rel(y, ref_r).max()
    e_full = _col_rel(y, ref).max()
    print(f"  arithmetic err {e_arith:.2e}  vs FP64 operator {e_full:.2e}", flush=True)
    assert e_arith <= 2e-5
    assert e_full <= (1e-5 if base == "c64" else 2e-2)
    info = dop.info()
    assert info["storage"] == binding.STORAGE[storage]
    lt = op.rank_row[op.adm_row].astype(np.int64)
    ls = op.rank_col[op.adm_col].astype(np.int64)
    k = op.adm_rank.astype(np.int64)
    assert info["elems_coupling"] + info["elems_coupling_in"] == int(np.minimum(lt * ls, k * (lt + ls)).sum())
