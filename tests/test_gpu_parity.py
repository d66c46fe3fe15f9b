"""GPU parity: the HIP products through the C-ABI against the CPU oracle, element by element.

Bar (FP64): ||y_gpu - y_oracle||_2 / ||y_oracle||_2 <= 1e-12 per right-hand side.  The
GPU and the oracle read one host operator; the oracle computes the plain block-wise
definition, the GPU the staged product.
"""
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


def _cols_rel(y, ref):
    y = y.reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return [float(np.linalg.norm(y[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j])) for j in range(ref.shape[1])]


def _run(torch, dop, x):
    xt = torch.from_numpy(np.asfortranarray(x)).to("cuda")
    if x.ndim == 2:
        xt = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda").t()
    y = dop.matvec(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


CASES = [
    ("sphere", 2048, 0, 32), ("sphere", 2048, 1, 32), ("sphere", 2048, 2, 32),
    ("sphere", 3000, 3, 64), ("ellipsoid", 1500, 4, 32), ("cube", 1300, 5, 32), ("sphere", 9000, 6, 64),
]


@pytest.mark.parametrize("surface,n,seed,leaf", CASES)
def test_uh_matvec_parity(torch_dev, surface, n, seed, leaf):
    from paper_2405_15573_amd import binding
    print(f"case uh {surface} n={n} seed={seed} leaf={leaf}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    dop = binding.upload(op)
    x = inputs.make_rhs(cloud.n, 1, seed=seed)[:, 0]
    y = _run(torch_dev, dop, x)
    ref = uniform.uh_mvp(vars(op), x)
    assert max(_cols_rel(y, ref)) <= TOL
    info = dop.info()
    assert info["n"] == cloud.n and info["kind"] == 0


@pytest.mark.parametrize("surface,n,seed,leaf", CASES[:1] + CASES[3:6])
def test_h_matvec_parity(torch_dev, surface, n, seed, leaf):
    from paper_2405_15573_amd import binding
    print(f"case h {surface} n={n} seed={seed} leaf={leaf}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    dop = binding.upload_h(op)
    x = inputs.make_rhs(cloud.n, 1, seed=seed + 100)[:, 0]
    y = _run(torch_dev, dop, x)
    assert max(_cols_rel(y, uniform.h_mvp(vars(op), x))) <= TOL


def test_multi_rhs_and_leading_dimension(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    print("case multi-rhs ld", flush=True)
    cloud, op = operator()
    dop = binding.upload(op)
    n, r, ld = cloud.n, 3, cloud.n + 17
    x = inputs.make_rhs(n, r, seed=21)
    xbuf = torch.zeros((r, ld), dtype=torch.complex128, device="cuda")
    xbuf[:, :n] = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")
    ybuf = torch.full((r, ld + 5), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    xv = xbuf.t()[:n]     # (n, r) with leading dimension ld
    yv = ybuf.t()[:n]     # (n, r) with leading dimension ld + 5
    dop.matvec(xv, yv)
    torch.cuda.synchronize()
    y = yv.cpu().numpy()
    assert max(_cols_rel(y, uniform.uh_mvp(vars(op), x))) <= TOL
    # padding rows beyond n are untouched
    assert torch.all(ybuf.t()[n:] == 7.0 + 0j).item()


def test_dense_only_and_tiny(torch_dev):
    from paper_2405_15573_amd import binding
    for n, leaf in ((60, 32), (5, 4), (1, 2)):
        print(f"case tiny n={n} leaf={leaf}", flush=True)
        cloud, op = operator(n=n, leaf=leaf)
        dop = binding.upload(op)
        x = inputs.make_rhs(cloud.n, 1, seed=n)[:, 0]
        y = _run(torch_dev, dop, x)
        assert max(_cols_rel(y, uniform.uh_mvp(vars(op), x))) <= TOL


def test_deterministic(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    cloud, op = operator(n=3000, seed=3, leaf=64)
    dop = binding.upload(op)
    x = torch.from_numpy(inputs.make_rhs(cloud.n, 1, seed=9)[:, 0]).to("cuda")
    y1 = dop.matvec(x).clone()
    y2 = dop.matvec(x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_argument_errors(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    cloud, op = operator()
    dop = binding.upload(op)
    lib = binding.load_library()
    import ctypes
    x = torch.zeros(cloud.n, dtype=torch.complex128, device="cuda")
    y = torch.zeros(cloud.n, dtype=torch.complex128, device="cuda")
    P = ctypes.c_void_p
    h = dop.handle
    assert lib.uhm_matvec(h, P(x.data_ptr()), cloud.n, P(y.data_ptr()), cloud.n, 0, None) == binding.UHM_OK
    assert lib.uhm_matvec(h, P(x.data_ptr()), cloud.n, P(y.data_ptr()), cloud.n, -1, None) == binding.UHM_EINVAL
    assert lib.uhm_matvec(h, P(x.data_ptr()), cloud.n - 1, P(y.data_ptr()), cloud.n, 1, None) == binding.UHM_EINVAL
    assert lib.uhm_matvec(h, P(x.data_ptr()), cloud.n, P(x.data_ptr()), cloud.n, 1, None) == binding.UHM_EINVAL
    assert lib.uhm_matvec(h, None, cloud.n, P(y.data_ptr()), cloud.n, 1, None) == binding.UHM_EINVAL
    assert lib.uhm_matvec(None, P(x.data_ptr()), cloud.n, P(y.data_ptr()), cloud.n, 1, None) == binding.UHM_EINVAL
    # an inconsistent operator is rejected before anything reaches the device
    bad = dict(vars(op))
    bad["S_off"] = op.S_off.copy()
    bad["S_off"][-1] = op.S.size  # block runs past the end of S
    with pytest.raises(binding.UhmError) as e:
        binding.upload(bad)
    assert e.value.code == binding.UHM_EINVAL
    bad = dict(vars(op))
    bad["perm"] = op.perm.copy()
    bad["perm"][0] = bad["perm"][1]
    with pytest.raises(binding.UhmError):
        binding.upload(bad)


SYM_CASES = CASES + [("sphere", 60, 0, 32), ("sphere", 5, 0, 4), ("sphere", 1, 0, 2)]


@pytest.mark.parametrize("surface,n,seed,leaf", SYM_CASES)
def test_symmetric_storage_parity(torch_dev, surface, n, seed, leaf):
    """Symmetric storage (one block per mirrored pair, each applied as itself and as its
    transpose) against the oracle's product of the expanded operator."""
    from paper_2405_15573_amd import binding, builder
    print(f"case sym {surface} n={n} seed={seed} leaf={leaf}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    sym = builder.symmetric_image(op)
    dop = binding.upload(sym, "c128sym")
    x = inputs.make_rhs(cloud.n, 2, seed=seed + 7)
    y = _run(torch_dev, dop, x)
    ref = uniform.uh_mvp(uniform.expand_symmetric(sym), x)
    assert max(_cols_rel(y, ref)) <= TOL
    info = dop.info()
    assert info["storage"] == 4 and info["elems_coupling"] == sym["elems_S_stored"]
    assert info["elems_near"] == sym["elems_D_stored"]
    # the same operator in general storage gives the same product to rounding
    full = _run(torch_dev, binding.upload(op), x)
    assert max(_cols_rel(y, full)) <= TOL


def test_symmetric_storage_deterministic_and_rejects_mirrors(torch_dev):
    from paper_2405_15573_amd import binding, builder
    torch = torch_dev
    print("case sym determinism", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    sym = builder.symmetric_image(op)
    dop = binding.upload(sym, "c128sym")
    x = torch.from_numpy(inputs.make_rhs(cloud.n, 1, seed=9)[:, 0]).to("cuda")
    y1 = dop.matvec(x).clone()
    y2 = dop.matvec(x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    # the general image lists both blocks of every mirrored pair: not a symmetric image
    with pytest.raises(binding.UhmError):
        binding.upload(op, "c128sym")


@pytest.mark.parametrize("surface,n,seed,leaf", CASES + [("sphere", 60, 0, 32), ("sphere", 1, 0, 2)])
def test_factored_couplings_parity(torch_dev, surface, n, seed, leaf):
    """Factored couplings (two-step S_{X,b} (S_{Y,b}^* u_sigma) where that stores fewer
    elements) against the oracle's product with S_b = S_{X,b} S_{Y,b}^* for every block."""
    from paper_2405_15573_amd import binding
    print(f"case factored {surface} n={n} seed={seed} leaf={leaf}", flush=True)
    cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
    dop = binding.upload(op, "c128fact")
    x = inputs.make_rhs(cloud.n, 2, seed=seed + 9)
    y = _run(torch_dev, dop, x)
    ref = uniform.uh_mvp(uniform.assemble_factored(vars(op)), x)
    assert max(_cols_rel(y, ref)) <= TOL
    info = dop.info()
    assert info["storage"] == 5
    if op.nadm:
        lt = op.rank_row[op.adm_row].astype(np.int64)
        ls = op.rank_col[op.adm_col].astype(np.int64)
        k = op.adm_rank.astype(np.int64)
        assert info["elems_coupling"] + info["elems_coupling_in"] == int(np.minimum(lt * ls, k * (lt + ls)).sum())
        assert info["elems_coupling_in"] == int((ls * k)[k * (lt + ls) < lt * ls].sum())


@pytest.mark.parametrize("form", ["c128sym", "c128fact"])
def test_symmetric_and_factored_multi_rhs_and_leading_dimension(torch_dev, form):
    from paper_2405_15573_amd import binding, builder
    torch = torch_dev
    print(f"case {form} multi-rhs ld", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    if form == "c128sym":
        img = builder.symmetric_image(op)
        ref_op = uniform.expand_symmetric(img)
    else:
        img = op
        ref_op = uniform.assemble_factored(vars(op))
    dop = binding.upload(img, form)
    n, r, ld = cloud.n, 3, cloud.n + 5
    x = inputs.make_rhs(n, r, seed=22)
    xbuf = torch.zeros((r, ld), dtype=torch.complex128, device="cuda")
    xbuf[:, :n] = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")
    ybuf = torch.full((r, ld + 3), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    dop.matvec(xbuf.t()[:n], ybuf.t()[:n])
    torch.cuda.synchronize()
    assert max(_cols_rel(ybuf.t()[:n].cpu().numpy(), uniform.uh_mvp(ref_op, x))) <= TOL
    assert torch.all(ybuf.t()[n:] == 7.0 + 0j).item()


def test_factored_upload_needs_the_factors(torch_dev):
    from paper_2405_15573_amd import binding
    cloud, op = operator()
    bad = dict(vars(op))
    bad["SX_off"] = op.SX_off.copy()
    bad["SX_off"][-1] = op.SX.size  # factor runs past the end of SX
    with pytest.raises(binding.UhmError):
        binding.upload(bad, "c128fact")
