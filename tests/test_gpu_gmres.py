"""GMRES(m) and GMRES-IR on the GPU through the C-ABI, checked by the CPU oracle.

The oracle's reference solution is the plain definition x* = A^{-1} b, from a dense LU
solve of the assembled FP64 UH-matrix (numpy), and the true residual ||b - A x|| / ||b|| is
recomputed with the oracle's block-wise product.
"""
import numpy as np
import pytest

from conftest import operator, rel
from oracle import krylov, precision, uniform
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


def _solve(torch, op, b, tol, inner_storage=None, **kw):
    from paper_2405_15573_amd import binding
    dop = binding.upload(op)
    inner = binding.upload(op, storage=inner_storage) if inner_storage else None
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda").t()
    x, info, rc = binding.solve_gmres(dop, bt, tol, inner=inner, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info, rc


@pytest.mark.parametrize("inner,cycles", [(None, 0), ("c64", 0), ("bf16pair", 0), ("c64fact", 0),
                                          ("bf16pairfact", 0), ("c64", 1), ("bf16pair", 1), ("bf16pairfact", 1)])
def test_gmres_solves_against_dense_solution(torch_dev, inner, cycles):
    print(f"case gmres inner={inner} inner_cycles={cycles}", flush=True)
    cloud, op = operator()
    o = vars(op)
    b = inputs.make_rhs(cloud.n, 2, seed=31)
    tol = 1e-8
    kw = {"inner_cycles": cycles, "max_refinements": 100} if inner else {}
    x, info, rc = _solve(torch_dev, op, b, tol, inner, restart=50, **kw)
    print(f"  {info}", flush=True)
    assert rc == 0 and info["converged"] == 2
    res = np.linalg.norm(b - uniform.uh_mvp(o, x), axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= tol * 1.01
    assert abs(res.max() - info["rel_residual"]) <= 1e-3 * tol + 1e-14
    a = uniform.assemble_uh(o)
    xs = np.linalg.solve(a, b)
    cond = np.linalg.cond(a)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= max(cond * tol, 1e-12)
    if inner is not None:
        assert info["refinements"] >= 1


def test_gmres_restarts_and_ragged(torch_dev):
    # restart 20 on a ragged cube cloud: several cycles (very short restarts stagnate on this
    # indefinite Helmholtz system, a property of restarted GMRES)
    cloud, op = operator(surface="cube", n=1300, seed=5)
    b = inputs.make_rhs(cloud.n, 1, seed=32)
    x, info, rc = _solve(torch_dev, op, b, 1e-8, None, restart=20)
    assert rc == 0 and info["restarts"] >= 1
    res = np.linalg.norm(b - uniform.uh_mvp(vars(op), x)) / np.linalg.norm(b)
    assert res <= 1e-8 * 1.01


def test_gmres_iteration_cap_reports_noconv(torch_dev):
    from paper_2405_15573_amd import binding
    cloud, op = operator()
    b = inputs.make_rhs(cloud.n, 1, seed=33)
    x, info, rc = _solve(torch_dev, op, b, 1e-12, None, restart=50, max_iterations=1, raise_on_noconv=False)
    # forced from the host: the cap stops the solve, X holds the last iterate
    assert rc == binding.UHM_ENOCONV and info["iterations"] == 1 and info["converged"] == 0
    res = np.linalg.norm(b - uniform.uh_mvp(vars(op), x)) / np.linalg.norm(b)
    assert abs(res - info["rel_residual"]) <= 1e-10 and res < 1.0


def test_gmres_batch_equals_alone(torch_dev):
    """Each right-hand side has its own Krylov space: solving it alone or in a batch gives
    the same iterate (same products, same reductions per column)."""
    cloud, op = operator(n=3000, seed=3, leaf=64)
    b = inputs.make_rhs(cloud.n, 3, seed=34)
    for inner in (None, "c64"):
        xb, _, _ = _solve(torch_dev, op, b, 1e-8, inner)
        for j in range(3):
            xa, _, _ = _solve(torch_dev, op, b[:, j:j + 1], 1e-8, inner)
            assert np.array_equal(xa[:, 0], xb[:, j]), (inner, j)


@pytest.mark.parametrize("storage", ["c128multi", "c128multifact"])
def test_gmres_with_multi_rhs_fp64_operator(torch_dev, storage):
    """The FP64 operator in its many-RHS layout (also with factored couplings) drives both
    plain GMRES and the refinement."""
    from paper_2405_15573_amd import binding
    torch = torch_dev
    print(f"case gmres residual operator {storage}", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    b = inputs.make_rhs(cloud.n, 5, seed=35)
    dop = binding.upload(op, storage=storage)
    inner = binding.upload(op, storage="bf16pair")
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda").t()
    for inn in (None, inner):
        x, info, rc = binding.solve_gmres(dop, bt, 1e-8, inner=inn)
        torch.cuda.synchronize()
        x = x.cpu().numpy()
        res = np.linalg.norm(b - uniform.uh_mvp(vars(op), x), axis=0) / np.linalg.norm(b, axis=0)
        assert rc == 0 and res.max() <= 1e-8 * 1.01


def test_gmres_with_symmetric_storage_operator(torch_dev):
    """The symmetric-storage FP64 operator (Remark 4.4) as the residual operator of plain
    GMRES and of the refinement; residuals checked with the oracle's expanded operator."""
    from paper_2405_15573_amd import binding, builder
    torch = torch_dev
    print("case gmres symmetric storage", flush=True)
    cloud, op = operator(n=3000, seed=3, leaf=64)
    sym = builder.symmetric_image(op)
    ex = uniform.expand_symmetric(sym)
    b = inputs.make_rhs(cloud.n, 3, seed=36)
    dop = binding.upload(sym, storage="c128sym")
    inner = binding.upload(op, storage="c64")
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda").t()
    for inn in (None, inner):
        x, info, rc = binding.solve_gmres(dop, bt, 1e-8, inner=inn)
        torch.cuda.synchronize()
        x = x.cpu().numpy()
        res = np.linalg.norm(b - uniform.uh_mvp(ex, x), axis=0) / np.linalg.norm(b, axis=0)
        assert rc == 0 and info["converged"] == 3 and res.max() <= 1e-8 * 1.01


@pytest.mark.parametrize("iters,restart", [(7, 50), (23, 10)])
def test_gmres_iterate_is_the_minimal_residual_iterate(torch_dev, iters, restart):
    """After a fixed number of Krylov steps (the iteration cap; the tolerance is out of
    reach), each column of the GPU iterate is the minimal-residual iterate over the same
    Krylov spaces, computed by the oracle as a literal least-squares minimisation
    (oracle.krylov): a check of the device-side Hessenberg, Givens and triangular-solve
    steps, cycle by cycle."""
    print(f"case gmres iterate {iters} steps, restart {restart}", flush=True)
    cloud, op = operator()
    o = vars(op)
    b = inputs.make_rhs(cloud.n, 2, seed=40)
    x, info, rc = _solve(torch_dev, op, b, 1e-15, None, restart=restart, max_iterations=iters,
                         raise_on_noconv=False)
    assert info["iterations"] == iters and info["converged"] == 0
    for j in range(2):
        ref = krylov.gmres_restarted(lambda v: uniform.alg6(o, v), b[:, j], restart, iters)
        err = rel(x[:, j], ref)
        print(f"  column {j}: {err:.2e}", flush=True)
        assert err <= 1e-10


def test_ir_one_cycle_per_refinement_is_the_oracle_refinement(torch_dev):
    """GMRES-IR with one inner cycle per refinement (inner_cycles = 1) against the oracle's
    refinement (oracle.krylov.gmres_ir_cycles): residuals with the FP64 operator, each
    correction the minimal-residual iterate of the complex64-rounded operator over its
    Krylov space.  The GPU's inner products accumulate in FP32, hence the 1e-5 bar."""
    print("case gmres-ir per-cycle refinement vs oracle", flush=True)
    cloud, op = operator()
    o = vars(op)
    lo = precision.round_operator(o, "c64")
    b = inputs.make_rhs(cloud.n, 2, seed=41)
    x, info, rc = _solve(torch_dev, op, b, 1e-15, "c64", restart=10, max_iterations=30, inner_cycles=1,
                         inner_tol=1e-12, max_refinements=100, raise_on_noconv=False)
    assert info["iterations"] == 30 and info["refinements"] == 3
    for j in range(2):
        ref = krylov.gmres_ir_cycles(lambda v: uniform.alg6(o, v), lambda v: uniform.alg6(lo, v), b[:, j], 10, 3)
        err = rel(x[:, j], ref)
        print(f"  column {j}: {err:.2e}", flush=True)
        assert err <= 1e-5
