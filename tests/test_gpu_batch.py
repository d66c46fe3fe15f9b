"""Batched products of many operators (stage-wise shared launches, hipGraph, tuner).

Each product in a batch must equal the operator's own product: bitwise under the default
schedule (same tiles, same reduction order), to FP32 rounding after the tuner changes the
coupling tiles; graph replays must equal eager runs every time.
"""
import numpy as np
import pytest

from conftest import operator
from oracle import precision, uniform
from paper_2405_15573_amd import inputs

pytestmark = pytest.mark.gpu

MIX = [("sphere", 2048, 0, 32), ("ellipsoid", 1500, 4, 32), ("cube", 1300, 5, 32), ("sphere", 3000, 3, 64),
       ("sphere", 60, 0, 32)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    from paper_2405_15573_amd import binding
    binding.load_library()
    return torch


def _setup(torch, storage, rhs):
    from paper_2405_15573_amd import binding
    dtype = torch.complex128 if storage == "c128multi" else torch.complex64
    ops, dops, xs, ys, xn = [], [], [], [], []
    for k, (surface, n, seed, leaf) in enumerate(MIX):
        cloud, op = operator(surface=surface, n=n, seed=seed, leaf=leaf)
        ops.append(op)
        dops.append(binding.upload(op, storage=storage))
        r = rhs[k % len(rhs)]
        x = inputs.make_rhs(cloud.n, r, seed=60 + k)
        if dtype == torch.complex64:
            x = x.astype(np.complex64).astype(np.complex128)
        xn.append(x)
        xs.append(torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda", dtype).t())
        ys.append(torch.zeros((r, cloud.n), dtype=dtype, device="cuda").t())
    return ops, dops, xs, ys, xn


@pytest.mark.parametrize("storage", ["c64", "bf16pair", "c128multi", "c64fact"])
def test_batch_equals_individual_products(torch_dev, storage):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    print(f"case batch {storage}", flush=True)
    ops, dops, xs, ys, xn = _setup(torch, storage, [1, 5, 16, 3, 9])
    b = binding.Batch(dops, xs, ys)
    b.run()
    torch.cuda.synchronize()
    for k, (op, dop) in enumerate(zip(ops, dops)):
        alone = dop.matvec(xs[k])
        torch.cuda.synchronize()
        assert torch.equal(alone, ys[k]), k
        y = ys[k].cpu().numpy().astype(np.complex128)
        if storage == "c128multi":
            ref = uniform.uh_mvp(vars(op), xn[k])
            tol = 1e-12
        elif storage.endswith("fact"):
            ref = uniform.uh_mvp(uniform.assemble_factored(precision.round_operator(vars(op), storage[:-4]), "smaller"), xn[k])
            tol = 2e-5
        else:
            ref = uniform.uh_mvp(precision.round_operator(vars(op), storage), xn[k])
            tol = 2e-5
        err = np.linalg.norm(y - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= tol, (k, err.max())


def test_batch_tune_and_graph_replays(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    ops, dops, xs, ys, xn = _setup(torch, "c64", [16, 2, 7, 16, 1])
    stream = torch.cuda.Stream()
    b = binding.Batch(dops, xs, ys, stream=stream)
    choice = b.tune(stream=stream)
    print(f"  tuned: {choice}", flush=True)
    assert choice["tile_width"] in (256, 512, 1024, 2048) and choice["order"] in (0, 1, 2)
    b.run(stream=stream)
    torch.cuda.synchronize()
    eager = [y.clone() for y in ys]
    for k, dop in enumerate(dops):
        alone = dop.matvec(xs[k])
        torch.cuda.synchronize()
        diff = (torch.linalg.norm(alone - eager[k]) / torch.linalg.norm(alone)).item()
        assert diff <= 1e-5, (k, diff)
    b.capture(stream)
    for rep in range(4):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        b.run(stream=stream)
        torch.cuda.synchronize()
        for k in range(len(ys)):
            assert torch.equal(ys[k], eager[k]), (rep, k)
        # eager work between replays
        _ = dops[0].matvec(xs[0])
        torch.cuda.synchronize()
    # a second batch with the same signature reuses the tuned schedule without re-timing
    b2 = binding.Batch(dops, xs, ys, stream=stream)
    again = b2.tune(stream=stream)
    assert again["tile_width"] == choice["tile_width"] and again["order"] == choice["order"]
    assert again["best_ms"] < 0  # cache hit: nothing timed


def test_batch_argument_errors(torch_dev):
    from paper_2405_15573_amd import binding
    torch = torch_dev
    cloud, op = operator()
    d128 = binding.upload(op)  # single-RHS layout
    x = torch.zeros(cloud.n, dtype=torch.complex128, device="cuda")
    y = torch.zeros(cloud.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.UhmError):
        binding.Batch([d128], [x], [y])
    d64 = binding.upload(op, storage="c64")
    dbf = binding.upload(op, storage="bf16pair")
    x32 = torch.zeros(cloud.n, dtype=torch.complex64, device="cuda")
    y32 = torch.zeros(cloud.n, dtype=torch.complex64, device="cuda")
    with pytest.raises(binding.UhmError):
        binding.Batch([d64, dbf], [x32, x32], [y32, torch.zeros_like(y32)])
