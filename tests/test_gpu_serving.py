"""Serving loop on the GPU: continuous batching of GMRES-IR solves over resident operators.

Checks: every solve reaches its tolerance (true FP64 residual, recomputed by the oracle);
a solve's result is identical alone and in a mix of concurrent solves on several
operators; requests queued behind a small memory budget are admitted as memory frees.
"""
import numpy as np
import pytest

from conftest import operator
from oracle import uniform
from paper_2405_15573_amd import inputs

pytestmark = pytest.mark.gpu

OPS = [("sphere", 2048, 0, 32), ("cube", 1300, 5, 32), ("ellipsoid", 1500, 4, 32)]


@pytest.fixture(scope="module")
def server_env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    from paper_2405_15573_amd import binding
    binding.load_library()
    host = [operator(surface=s, n=n, seed=sd, leaf=lf)[1] for s, n, sd, lf in OPS]
    return torch, host


def _requests(torch, host, spec):
    from paper_2405_15573_amd.serving import Request
    out = []
    for rid, (op, r, tol, t) in enumerate(spec):
        b = inputs.make_rhs(host[op].n, r, seed=100 + rid)
        bt = torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda").t()
        out.append(Request(rid=rid, op=op, b=bt, tol=tol, arrival=t))
    return out


SPEC = [(0, 2, 1e-8, 0.0), (1, 1, 1e-6, 0.0), (2, 3, 1e-8, 0.001), (0, 1, 1e-6, 0.002), (1, 4, 1e-8, 0.003)]


@pytest.mark.parametrize("low", ["c64", "c64fact"])
def test_mix_equals_alone_and_converges(server_env, low):
    torch, host = server_env
    from paper_2405_15573_amd.serving import Server
    print(f"case serving mix, inner {low}", flush=True)
    srv = Server(host, low_storage=low, keep_solutions=True)
    mix = srv.serve(_requests(torch, host, SPEC))
    rep = Server.report(mix)
    print(f"  mix report {rep}", flush=True)
    assert rep["completed"] == len(SPEC) and rep["converged"] == len(SPEC)
    for q in mix:
        b = q.b.cpu().numpy()
        x = q.x.cpu().numpy()
        res = np.linalg.norm(b - uniform.uh_mvp(vars(host[q.op]), x), axis=0) / np.linalg.norm(b, axis=0)
        assert res.max() <= q.tol * 1.01, (q.rid, res.max())
    from paper_2405_15573_amd.serving import Request
    for q in mix:
        alone = srv.serve([Request(rid=q.rid, op=q.op, b=q.b, tol=q.tol, arrival=0.0)])[0]
        assert torch.equal(alone.x, q.x), q.rid
        assert alone.info["iterations"] == q.info["iterations"]
    srv.free()


def test_small_budget_queues_and_admits_on_free(server_env):
    torch, host = server_env
    from paper_2405_15573_amd.serving import Server, solve_footprint
    # room for one 2048-point single-RHS solve at a time
    budget = solve_footprint(2048, 1, 50) + 1
    srv = Server(host, low_storage="bf16pair", hbm_budget=budget)
    reqs = srv.serve(_requests(torch, host, [(0, 1, 1e-6, 0.0), (0, 1, 1e-6, 0.0), (1, 1, 1e-6, 0.0)]))
    assert all(q.code == 0 for q in reqs)
    starts = sorted(q.start for q in reqs)
    fins = sorted(q.finish for q in reqs)
    # at most one at a time: each start follows the previous finish
    assert starts[1] >= fins[0] and starts[2] >= fins[1]
    assert srv.admission.used == 0 and srv.admission.active == 0
    srv.free()


def test_wide_mix_equals_alone(server_env):
    """58 columns on one operator share each product (four column blocks) while the solves
    alone use one or two; a column's arithmetic must not depend on that."""
    torch, host = server_env
    from paper_2405_15573_amd.serving import Request, Server
    spec = [(0, 8, 1e-8, 0.0), (0, 30, 1e-6, 0.0), (0, 20, 1e-6, 0.0), (1, 2, 1e-8, 0.0)]
    srv = Server(host, low_storage="c64", keep_solutions=True)
    mix = srv.serve(_requests(torch, host, spec))
    assert all(q.code == 0 for q in mix)
    for q in (mix[0], mix[3]):
        alone = srv.serve([Request(rid=q.rid, op=q.op, b=q.b, tol=q.tol, arrival=0.0)])[0]
        assert torch.equal(alone.x, q.x), q.rid
        assert alone.info["iterations"] == q.info["iterations"]
    srv.free()
