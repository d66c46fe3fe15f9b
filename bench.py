"""Benchmark: FP64 uniform H-matrix MVP against the plain H-matrix MVP of the same operator.

Default workload: N = 262144 quasi-uniform points on the unit sphere (seeded jittered
Fibonacci lattice), kernel exp(i kappa r)/(4 pi r) with kappa*h = 0.6, diagonal 1/(2h),
geometric bisection tree with leaf 64, weak admissibility eta = 1, ACA and compression
tolerance 1e-6, one complex128 right-hand side x ~ CN(0,1).

One step = one product y = A x through the C-ABI (forward, coupling, backward and near
field kernels), with the operator and x already resident in HBM.  Also reported: the
H-matrix product of the same operator on the same GPU, per-kernel times, a roofline line
for the dominant kernel, sampled parity against the CPU oracle, and the CPU oracle
(Algorithm 6 in C/OpenMP) timed on this host's cores on a bounded sample.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "uniform-H MVP GB/s & MVPs/s vs plain H-MVP at N=256K; p99 GMRES solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SYM_STORAGE = 4  # symmetric storage form (one block per mirrored pair)
C128_STORAGES = (0, 3, 4, 5, 8)  # storage forms with complex128 vectors


def algorithmic_bytes(info: dict, n: int, nrhs: int = 1) -> dict:
    """Bytes each kernel must move per product: stored operator elements once, vectors once."""
    e = info["elem_bytes"]
    f = 16 if info["storage"] in C128_STORAGES else 8  # vector element: complex128 or complex64
    rs = info["rank_space"]
    out = {
        "k_forward_tiles": e * info["elems_forward"] + f * nrhs * (n + rs),
        "k_backward": e * (info["elems_backward"] + info["elems_near"]) + f * nrhs * (2 * n),
    }
    if info["storage"] == SYM_STORAGE:
        # symmetric storage: the transposed products also write (and a second kernel reads) partial sums
        tc, tn = info["partial_coupling"], info["partial_near"]
        out["k_coupling_sym"] = e * info["elems_coupling"] + f * nrhs * (2 * rs + tc)
        out["k_backward_sym"] = out.pop("k_backward") + f * nrhs * (rs + tn)
        out["total"] = (e * (info["elems_forward"] + info["elems_coupling"] + info["elems_backward"]
                             + info["elems_near"]) + f * nrhs * (2 * n + 4 * rs + 2 * tc + 2 * tn))
        return out
    ci = info.get("elems_coupling_in", 0)
    if info["kind"] == 0:
        out["k_coupling"] = e * info["elems_coupling"] + f * nrhs * 2 * rs
        out["k_backward"] += f * nrhs * rs
        if ci:  # factored couplings: first step S_Y^* u, then S_X (and the assembled S_b) in k_coupling
            out["k_factor_in"] = e * ci + f * nrhs * 2 * rs
    else:
        out["k_backward"] += f * nrhs * rs
    out["total"] = (e * (info["elems_forward"] + info["elems_coupling"] + ci + info["elems_backward"]
                         + info["elems_near"])
                    + f * nrhs * (2 * n + 2 * rs + (2 * rs if info["kind"] == 0 else 0) + (2 * rs if ci else 0)))
    return out


def time_products(torch, dop, x, y, steps, warmup, stream, per_product=None):
    """Mean wall time per product over `steps` products (synchronised before and after),
    and per-kernel HIP-event times.  per_product: a dict that receives the HIP-event time
    of every product (events on `stream` around each) as mean / min / p50 in ms."""
    import numpy as np
    for _ in range(warmup):
        dop.matvec(x, y, stream=stream)
    torch.cuda.synchronize()
    dop.set_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)] \
        if per_product is not None else None
    t0 = time.perf_counter()
    for k in range(steps):
        if ev:
            ev[k][0].record(stream)
        dop.matvec(x, y, stream=stream)
        if ev:
            ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = dop.kernel_times()
    dop.set_timing(False)
    if ev:
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        per_product.update(mean_ms=float(ms.mean()), min_ms=float(ms.min()), p50_ms=float(np.median(ms)),
                           max_ms=float(ms.max()), count=int(ms.size))
    return (t1 - t0) / steps, {k: (v[0] / max(1, v[1]), v[1]) for k, v in kt.items() if v[1] > 0}


def stream_context(torch):
    """Rates plain torch kernels reach on this GPU: a 2 GiB device copy (read + write) and a
    2 GiB sum (read).  Context for the roofline fraction, which stays against the 8 TB/s
    peak."""
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * a.numel() * 8),
                             ("sum", lambda: a.sum(), a.numel() * 8)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[f"torch_{name}_gbs"] = nbytes / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


DEFAULT_INNER_TOL = {"c64": 1e-3, "bf16pair": 1e-2, "c64fact": 1e-3, "bf16pairfact": 1e-2}


def run_gmres_cases(torch, binding, op, n, r, tol, maxit, stream, seed, cases=None, inner_tols=None, inner_cycles=1):
    """Plain FP64 GMRES(50) against GMRES-IR with complex64 and bf16-pair inner products
    (cases: names to run, default all; inner_tols: inner tolerance per inner storage;
    inner_cycles: GMRES(50) cycles per inner solve, 1 = every restart is a refinement step
    with the true FP64 residual, 0 = inner solves run to their tolerance)."""
    import numpy as np

    from paper_2405_15573_amd import inputs
    out = {}
    Bn = inputs.make_rhs(n, r, seed=seed + 11)
    Bd = torch.from_numpy(np.ascontiguousarray(Bn.T)).to("cuda").t()
    dmulti = binding.upload(op, storage="c128multi", stream=stream)
    dmulti_f = None
    # inner tolerances: the residual reduction asked of each inner solve (complex64 products
    # are accurate to ~1e-6, bf16 pairs to ~3e-3)
    itol = dict(DEFAULT_INNER_TOL, **(inner_tols or {}))
    for name, inner_st in (("fp64", None), ("fp64fact", None), ("ir_c64", "c64"), ("ir_bf16pair", "bf16pair"),
                           ("ir_c64fact", "c64fact"), ("ir_bf16pairfact", "bf16pairfact")):
        if cases and name not in cases:
            continue
        inner_tol = itol[inner_st] if inner_st else None
        inner = binding.upload(op, storage=inner_st, stream=stream) if inner_st else None
        if name == "fp64fact":  # plain FP64 GMRES on the FP64 operator with factored couplings
            dmulti_f = binding.upload(op, storage="c128multifact", stream=stream)
        torch.cuda.synchronize()
        t0g = time.perf_counter()
        kw = {"inner": inner, "inner_tol": inner_tol, "inner_cycles": inner_cycles,
              "max_refinements": maxit // 50 + 50} if inner_st else {}
        X, ginfo, rc = binding.solve_gmres(dmulti_f if name == "fp64fact" else dmulti, Bd, tol, restart=50,
                                           max_iterations=maxit, stream=stream, raise_on_noconv=False, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0g
        out[name] = dict(ginfo, wall_s=wall, nrhs=r, tol=tol, iteration_cap=maxit, inner_tol=inner_tol,
                         inner_cycles=inner_cycles if inner_st else None,
                         status="converged" if rc == 0 else "iteration cap")
        log(f"GMRES N={n} {name}: {wall:.2f} s, {ginfo['iterations']} it, {ginfo['refinements']} ref, "
            f"res {ginfo['rel_residual']:.2e}, products {ginfo['seconds_products']:.2f} s, "
            f"arnoldi {ginfo['seconds_arnoldi']:.2f} s")
        if inner is not None:
            inner.free()
        del X
    # speed-ups against the faster plain FP64 solve
    fp = [out[k]["wall_s"] for k in ("fp64", "fp64fact") if k in out and out[k]["status"] == "converged"]
    if fp:
        for k in ("ir_c64", "ir_bf16pair", "ir_c64fact", "ir_bf16pairfact"):
            if k in out and out[k]["status"] == "converged":
                out[k]["speedup_vs_fp64"] = min(fp) / out[k]["wall_s"]
    dmulti.free()
    if dmulti_f is not None:
        dmulti_f.free()
    return out


def mixed_population(count, lo, hi, seed, surf=("sphere", "ellipsoid", "cube")):
    """Seeded operator population: N log-uniform in [lo, hi], surfaces in turn."""
    from paper_2405_15573_amd import inputs
    sizes = inputs.log_uniform_sizes(count, lo, hi, seed)
    return [(surf[k % len(surf)], int(sizes[k])) for k in range(count)]


def run_batched(args):
    """Many operators of uneven size (complex64, 1-16 RHS each) in shared stage launches,
    tuned and captured in a hipGraph, against one operator at a time."""
    import numpy as np
    import torch

    from paper_2405_15573_amd import binding, builder, inputs
    pop = mixed_population(args.nops, 4096, args.max_n, args.seed)
    rng = np.random.default_rng([args.seed, 4])
    stream = torch.cuda.Stream()
    ops, hosts, xs, ys, bytes_total, flops_total, rsum = [], [], [], [], 0, 0.0, 0
    t0 = time.perf_counter()
    for k, (surf, n) in enumerate(pop):
        cloud = inputs.make_cloud(surf, n, seed=args.seed + k)
        h = builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                   construct=args.construct)
        d = binding.upload(h, storage=args.batch_storage, stream=stream)
        r = int(rng.integers(1, 17))
        inf = d.info()
        M = (inf["elems_forward"] + inf["elems_coupling"] + inf["elems_coupling_in"] + inf["elems_backward"]
             + inf["elems_near"])
        eb = 4 if args.batch_storage.startswith("bf16") else 8   # stored element bytes
        bytes_total += eb * M + 8 * r * 2 * cloud.n
        flops_total += 8.0 * r * M
        rsum += r
        x = inputs.make_rhs(cloud.n, r, seed=args.seed + 100 + k).astype(np.complex64)
        xs.append(torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda").t())
        ys.append(torch.empty((r, cloud.n), dtype=torch.complex64, device="cuda").t())
        ops.append(d)
        hosts.append((surf, cloud.n, r))
        log(f"  op {k}: {surf} N={cloud.n} r={r} built {h.timings['total']:.1f}s")
        del h
    log(f"population built in {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def one_at_a_time():
        for d, x, y in zip(ops, xs, ys):
            d.matvec(x, y, stream=stream)

    t_seq = timed(one_at_a_time, args.steps)
    ref = [y.clone() for y in ys]
    batch = binding.Batch(ops, xs, ys, stream=stream)
    t_untuned = timed(lambda: batch.run(stream=stream), args.steps)
    choice = batch.tune(stream=stream)
    t_tuned = timed(lambda: batch.run(stream=stream), args.steps)
    batch.capture(stream)
    t_graph = timed(lambda: batch.run(stream=stream), args.steps)
    err = max(float((torch.linalg.norm(y - r_) / torch.linalg.norm(r_)).item()) for y, r_ in zip(ys, ref))
    line = {
        "metric": f"batched uniform-H MVPs: right-hand-side products per second, {args.batch_storage}, shared launches",
        "value": rsum / (t_graph * 1e-3), "unit": "RHS-products/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 3, "ms_per_step": t_graph, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.nops} operators, N log-uniform in [4096, {args.max_n}], sphere/ellipsoid/cube, "
                               f"1-16 RHS each, {args.batch_storage} storage", "operators": hosts},
        "ms_one_operator_at_a_time": t_seq, "ms_batched_untuned": t_untuned, "ms_batched_tuned": t_tuned,
        "ms_batched_graph": t_graph, "speedup_vs_one_at_a_time": t_seq / t_graph, "tuned_schedule": choice,
        "gbs": bytes_total / (t_graph * 1e-3) / 1e9, "tflops": flops_total / (t_graph * 1e-3) / 1e12,
        "hbm_frac": bytes_total / (t_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "mfma_frac": flops_total / (t_graph * 1e-3) / 1e12 / (2500.0 if args.batch_storage.startswith("bf16")
                                                             else 157.3),
        "algorithmic_bytes": bytes_total, "algorithmic_flops": flops_total,
        "max_rel_diff_vs_one_at_a_time": err,
    }
    print(json.dumps(line), flush=True)


def run_gmres_sizes(args):
    """Time to tolerance of FP64 GMRES(50) and GMRES-IR on spheres of several sizes."""
    import torch

    from paper_2405_15573_amd import binding, builder, inputs
    stream = torch.cuda.Stream()
    res = {}
    for n in [int(v) for v in args.gmres_sizes.split(",")]:
        cloud = inputs.make_cloud("sphere", n, seed=args.seed)
        h = builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                   construct=args.construct)
        log(f"N={cloud.n} built in {h.timings['total']:.1f} s")
        cases = args.gmres_cases.split(",") if args.gmres_cases else None
        tols = {k: float(v) for k, v in (kv.split("=") for kv in args.inner_tols.split(","))} if args.inner_tols else None
        res[str(cloud.n)] = run_gmres_cases(torch, binding, h, cloud.n, args.gmres_rhs, args.gmres_tol,
                                             args.gmres_tol_maxit, stream, args.seed, cases, tols,
                                             inner_cycles=args.inner_cycles)
        del h
    line = {
        "metric": "GMRES time to tolerance, FP64 vs mixed-precision GMRES-IR", "value": None, "unit": "s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32/bf16", "data": "synthetic",
        "config": {"workload": f"spheres N={args.gmres_sizes}, kappa*h=0.6, {args.gmres_rhs} RHS, tol "
                               f"{args.gmres_tol}, GMRES(50), iteration cap {args.gmres_tol_maxit}, "
                               f"{args.inner_cycles} inner cycle(s) per refinement"},
        "per_size": res,
    }
    print(json.dumps(line), flush=True)


def run_construct(args):
    """Sampling the matrix on the GPU (ACA of every admissible block, uhm_aca, and the dense
    near-field blocks, uhm_kernel_blocks) against the host builder's OpenMP C++ on the same
    blocks: times, rank agreement, and sampled parity of the GPU factors with the oracle."""
    import numpy as np
    import torch

    from oracle import aca as oaca
    from paper_2405_15573_amd import binding, builder, inputs
    cloud = inputs.make_cloud("sphere", args.n, seed=args.seed)
    tree = builder.build_tree(cloud.points, args.leaf)
    pts = np.ascontiguousarray(cloud.points[tree.perm])
    diag = 1.0 / (2.0 * cloud.h)
    adm, den = builder.build_block_tree(tree, 1.0)
    low = adm[adm[:, 0] < adm[:, 1]]
    levs = tree.level[low[:, 0]]
    dev_pts = binding._points_on_device(pts)
    lib = builder._native()
    P = builder._ptr
    eps, kcap = 1e-6, 1024
    stream = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # warm-up launch (module load)
    binding.aca(dev_pts, cloud.kappa, diag, [0], [8], [64], [8], [4], eps, stream=stream)
    torch.cuda.synchronize()
    per_level, tot = {}, {"gpu_ms": 0.0, "host_s": 0.0, "entries": 0, "update_flops": 0, "blocks": 0,
                          "rank_equal": 0, "reruns": 0}
    sample = []
    for lev in np.unique(levs):
        blk = low[levs == lev]
        ro, rs = tree.off[blk[:, 0]], tree.size[blk[:, 0]]
        co, cs = tree.off[blk[:, 1]], tree.size[blk[:, 1]]
        order = np.argsort(-(rs + cs), kind="stable")
        ro, rs, co, cs = ro[order], rs[order], co[order], cs[order]
        full = np.minimum(np.minimum(rs, cs), kcap)
        rank = np.zeros(len(ro), np.int64)
        todo, cap_now, ms = np.arange(len(ro)), 128, 0.0
        first = None
        while todo.size:
            caps = np.minimum(full[todo], cap_now)
            torch.cuda.synchronize()
            e0.record(stream)
            res = binding.aca(dev_pts, cloud.kappa, diag, ro[todo], rs[todo], co[todo], cs[todo], caps, eps,
                              stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            done = (res.status != 0) | (caps >= full[todo])
            rank[todo[done]] = res.rank[done]
            if first is None:
                first = (res, todo.copy())
            else:
                tot["reruns"] += int(done.sum())
            todo = todo[~done]
            cap_now *= 4
        kout = np.zeros(len(ro), np.int32)
        t = time.perf_counter()
        args_c = [np.ascontiguousarray(a, dtype=np.int64) for a in (ro, rs, co, cs)]   # alive during the call
        h = lib.uhmb_aca_run(P(pts), cloud.kappa, diag, len(ro), *[P(a) for a in args_c], eps, kcap, P(kout))
        host_s = time.perf_counter() - t
        lib.uhmb_aca_free(h)
        entries = int(np.sum(rank * (rs + cs)))
        flops = int(np.sum(8 * rank * (rank - 1) * (rs + cs)))  # residual updates + norm cross terms
        eq = int(np.sum(rank == kout))
        per_level[int(lev)] = {"blocks": len(ro), "rows": int(rs.max()), "k_max": int(rank.max()),
                               "gpu_ms": round(ms, 3), "host_s": round(host_s, 3), "rank_equal_host": eq}
        log(f"level {lev}: {len(ro)} blocks of {int(rs.max())}, k_max {int(rank.max())}: GPU {ms:.2f} ms, "
            f"host {host_s:.2f} s, ranks equal {eq}/{len(ro)}")
        for key, v in (("gpu_ms", ms), ("host_s", host_s), ("entries", entries), ("update_flops", flops),
                       ("blocks", len(ro)), ("rank_equal", eq)):
            tot[key] += v
        # sampled parity with the oracle: two blocks of each level up to 1024 rows (first pass, full rank)
        res, idx = first
        if int(rs.max()) <= 1024:
            for b in (0, len(idx) - 1):
                if res.status[b] == 0:
                    continue
                j = int(idx[b])
                u, v, pr, pc, conv = oaca.aca_kernel_block(pts, cloud.kappa, diag, int(ro[j]), int(rs[j]), int(co[j]),
                                                           int(cs[j]), eps, int(res.cap[b]))
                gu, gv, gpr, gpc = res.factors(b)
                ok = (np.array_equal(gpr, pr) and np.array_equal(gpc, pc) and gu.shape == u.shape)
                blk = oaca.kernel_block(pts, cloud.kappa, diag, np.arange(ro[j], ro[j] + rs[j]),
                                        np.arange(co[j], co[j] + cs[j]))
                err = float(np.linalg.norm(gu @ gv.T - u @ v.T) / np.linalg.norm(blk)) if ok else float("inf")
                sample.append({"level": int(lev), "rows": int(rs[j]), "k": int(u.shape[1]), "pivots_equal": ok,
                               "approx_rel_diff": err, "aca_rel_err": float(np.linalg.norm(gu @ gv.T - blk)
                                                                             / np.linalg.norm(blk))})
        del first, res
    # dense near field
    ro, rs, co, cs = tree.off[den[:, 0]], tree.size[den[:, 0]], tree.off[den[:, 1]], tree.size[den[:, 1]]
    torch.cuda.synchronize()
    e0.record(stream)
    Dd, doff = binding.kernel_blocks(dev_pts, cloud.kappa, diag, ro, rs, co, cs, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dense_ms = e0.elapsed_time(e1)
    Dh = np.empty(int(np.sum(rs * cs)), np.complex128)
    t = time.perf_counter()
    args_c = [np.ascontiguousarray(a, dtype=np.int64) for a in (ro, rs, co, cs, doff)]   # alive during the call
    lib.uhmb_dense_blocks(P(pts), cloud.kappa, diag, len(ro), *[P(a) for a in args_c], P(Dh))
    dense_host_s = time.perf_counter() - t
    dense_err = float(np.max(np.abs(Dd.cpu().numpy() - Dh)) / np.max(np.abs(Dh)))
    del Dd, Dh
    worst = max((sm["approx_rel_diff"] for sm in sample), default=None)
    build = None
    if args.full_build:
        # the whole operator built with the GPU sampling (ACA, packing, near field), checked on
        # sampled rows against the dense matrix (within 10 eps |(A x) on those rows|)
        from oracle import kernel, uniform
        del dev_pts
        torch.cuda.empty_cache()
        t = time.perf_counter()
        op = builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=eps, eps_comp=1e-6, construct="gpu",
                                    verbose=True)
        total = time.perf_counter() - t
        leaves = np.nonzero(np.bincount(op.parent[op.parent >= 0], minlength=op.nclusters) == 0)[0]
        pick = np.random.default_rng(12345).choice(leaves, size=4, replace=False)
        pos = np.concatenate([np.arange(op.off[c], op.off[c] + op.size[c]) for c in pick])
        x = inputs.make_rhs(cloud.n, 1, seed=0)[:, 0]
        ref, users = uniform.uh_mvp_rows(vars(op), x, pos)
        dense = kernel.dense_matvec(cloud.points, cloud.kappa, diag, x, rows=users, chunk=64)
        dop = binding.upload(op, "c128")
        yfull = float(np.linalg.norm(dop.matvec(torch.from_numpy(x).to("cuda")).cpu().numpy()))
        dop.free()
        build = {"construct": "gpu", "seconds": round(total, 2),
                 **{k: round(v, 3) for k, v in op.timings.items()},
                 "sampled_err_vs_dense": float(np.linalg.norm(ref[:, 0] - dense)),
                 "ten_eps_norm_Ax_sampled_rows": 10 * 1e-6 * float(np.linalg.norm(dense)),
                 "ten_eps_norm_Ax": 10 * 1e-6 * yfull,
                 "l_max": int(op.rank_row.max()), "k_max": int(op.adm_rank.max())}
        log(f"full build {total:.1f} s: {json.dumps(build)}")
    gpu_s = (tot["gpu_ms"] + dense_ms) / 1e3
    host_s = tot["host_s"] + dense_host_s
    line = {
        "metric": "matrix sampling for construction: ACA of every admissible block + dense near field",
        "value": round(gpu_s, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(gpu_s * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sphere N={cloud.n}, leaf {args.leaf}, eta 1, ACA eps {eps}, kappa*h=0.6"},
        "aca": {"gpu_ms": round(tot["gpu_ms"], 3), "host_s": round(tot["host_s"], 3),
                "speedup": round(tot["host_s"] * 1e3 / tot["gpu_ms"], 1), "blocks": tot["blocks"],
                "rank_equal_host": tot["rank_equal"], "reruns_at_larger_cap": tot["reruns"],
                "entries_sampled": tot["entries"], "entries_per_s": round(tot["entries"] / (tot["gpu_ms"] / 1e3), 1),
                "update_tflops": round(tot["update_flops"] / (tot["gpu_ms"] / 1e3) / 1e12, 3),
                "per_level": per_level},
        "dense": {"gpu_ms": round(dense_ms, 3), "host_s": round(dense_host_s, 3), "entries": int(np.sum(rs * cs)),
                  "max_rel_diff_host": dense_err},
        "host_threads": int(lib.uhmb_num_threads()),
        "parity_sample": {"blocks": len(sample), "pivots_equal": all(sm["pivots_equal"] for sm in sample),
                          "worst_approx_rel_diff": worst},
        "full_build": build,
    }
    print(json.dumps(line), flush=True)


def run_direct(args):
    """Direct UH construction (Algs. 3-4 with per-block locks) against the two-phase builder
    (H-matrix, then Alg. 2) on one cloud, on the host: times, the block factors held at once,
    and agreement of the two operators on sampled rows (oracle, block by block)."""
    import numpy as np

    from oracle import uniform
    from paper_2405_15573_amd import builder, inputs
    import resource
    cloud = inputs.make_cloud("sphere", args.n, seed=args.seed)
    t = time.perf_counter()
    direct = builder.build_uniform_direct(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
    t_dir = time.perf_counter() - t
    rss_direct = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2**20
    log(f"direct {t_dir:.1f} s, peak resident set {rss_direct:.1f} GB: {json.dumps(direct.timings)}")
    two = None
    if not args.direct_only:
        t = time.perf_counter()
        two = builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6)
        t_two = time.perf_counter() - t
        log(f"two-phase {t_two:.1f} s")
        leaves = np.nonzero(np.bincount(two.parent[two.parent >= 0], minlength=two.nclusters) == 0)[0]
        pick = np.random.default_rng(7).choice(leaves, size=4, replace=False)
        pos = np.concatenate([np.arange(two.off[c], two.off[c] + two.size[c]) for c in pick])
        x = inputs.make_rhs(cloud.n, 1, seed=args.seed)
        a, _ = uniform.uh_mvp_rows(vars(two), x, pos)
        b, _ = uniform.uh_mvp_rows(vars(direct), x, pos)
    st = direct.stats()
    tm = direct.timings
    line = {
        "metric": "direct UH construction (Algs. 3-4, per-block locks) vs H-matrix then Alg. 2",
        "value": round(t_dir, 2), "unit": "s", "n_gpus": 0, "steps": 1, "warmup": 0, "ms_per_step": round(t_dir * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"sphere N={cloud.n}, leaf {args.leaf}, eta 1, tolerances 1e-6, host threads "
                               f"{tm['threads']}"},
        "direct_s": round(t_dir, 2), "direct_peak_rss_gb": round(rss_direct, 2),
        "peak_factor_bytes": tm["peak_factor_bytes"], "total_factor_bytes": tm["total_factor_bytes"],
        "uh_bytes": st["bytes_uh_c128"], "lock_waits": tm["lock_waits"],
        "l_max": st["l_max"], "k_max": st["k_max"],
    }
    if two is not None:
        line.update({
            "two_phase_s": round(t_two, 2), "h_bytes": two.stats()["bytes_h_c128"],
            "ranks_equal": bool(np.array_equal(two.rank_row, direct.rank_row)
                                and np.array_equal(two.adm_rank, direct.adm_rank)),
            "sampled_rel_diff": float(np.linalg.norm(a - b) / np.linalg.norm(a))})
    print(json.dumps(line), flush=True)


def run_serving(args):
    """Poisson arrivals of GMRES-IR solve requests over resident operators."""
    import numpy as np
    import torch

    from paper_2405_15573_amd import builder, inputs
    from paper_2405_15573_amd.serving import Request, Server, solve_footprint
    # no ellipsoids: GMRES(50) stalls near 1e-2 on the ellipsoid operators at kappa*h = 0.6,
    # in FP64 as in mixed precision, so their requests would only measure the iteration cap
    pop = mixed_population(16, 4096, args.serve_max_n, args.seed + 1, surf=("sphere", "cube"))
    hosts = []
    t0 = time.perf_counter()
    for k, (surf, n) in enumerate(pop):
        cloud = inputs.make_cloud(surf, n, seed=args.seed + k)
        hosts.append(builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                            construct=args.construct))
        log(f"  op {k}: {surf} N={cloud.n} built {hosts[-1].timings['total']:.1f}s")
    log(f"population built in {time.perf_counter() - t0:.1f} s")
    srv = Server(hosts, low_storage=args.serve_storage, inner_tol=1e-3, max_iterations=args.serve_maxit,
                 inner_cycles=args.inner_cycles)
    budget = srv.admission.budget
    results = {}
    runs = [(float(v), None) for v in args.rates.split(",")]
    if args.serve_budget_mb > 0:   # the highest rate again, under a small HBM budget
        runs.append((max(r for r, _ in runs), int(args.serve_budget_mb) << 20))
    for rate, cap in runs:
        rng = np.random.default_rng([args.seed, 5, int(rate)])
        t = np.cumsum(rng.exponential(1.0 / rate, size=args.requests))
        reqs = []
        for i in range(args.requests):
            op = int(rng.integers(0, len(hosts)))
            r = int(rng.integers(1, 9))
            tol = 1e-6 if rng.random() < 0.5 else 1e-8
            b = inputs.make_rhs(hosts[op].n, r, seed=int(rate) * 100000 + i)
            reqs.append(Request(rid=i, op=op, b=torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda").t(), tol=tol,
                                arrival=float(t[i])))
        srv.admission.budget = cap if cap is not None else budget
        srv.step_s, srv.steps, srv.step_solves = 0.0, 0, 0
        key = str(int(rate)) + ("" if cap is None else f"_budget{args.serve_budget_mb}MB")
        log(f"rate {rate}/s: {args.requests} requests, HBM budget {srv.admission.budget / 2**20:.0f} MB")
        done = srv.serve(reqs, log=log)
        rep = Server.report(done)
        rep.update(step_ms_mean=1e3 * srv.step_s / max(1, srv.steps), steps=srv.steps,
                   solves_per_step_mean=srv.step_solves / max(1, srv.steps),
                   capped_fraction=1.0 - rep.get("converged", 0) / max(1, rep.get("completed", 1)),
                   hbm_budget_bytes=srv.admission.budget,
                   largest_request_bytes=max(srv.footprint(q) for q in reqs))
        results[key] = rep
        log(f"  {rep}")
        del reqs, done
    srv.admission.budget = budget
    worst = max((v for k, v in results.items() if "budget" not in k), key=lambda v: v.get("p99_converged_s") or 0.0)
    line = {
        "metric": "p99 GMRES solve latency over converged solves (served, continuous batching)",
        "value": worst.get("p99_converged_s"),
        "unit": "s", "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": worst.get("step_ms_mean"),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"16 resident operators (sphere, cube), N log-uniform in [4096, {args.serve_max_n}], "
                               f"GMRES-IR ({args.serve_storage} inner, FP64 residual, {args.inner_cycles} inner "
                               f"cycle(s) per refinement), Poisson arrivals {args.rates}/s, {args.requests} requests "
                               f"per rate, 1-8 RHS, tol 1e-6 or 1e-8, iteration cap {args.serve_maxit}",
                   "operators": [(p[0], int(h.n)) for p, h in zip(pop, hosts)]},
        "capped_fraction_at_worst_rate": worst.get("capped_fraction"),
        "per_rate": results,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", type=str, default="",
                    help="headline: also time the headline product on the operators of these seeds "
                         "(e.g. 0,1,2; each adds one operator build)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-h", action="store_true")
    ap.add_argument("--no-sym", action="store_true", help="skip the symmetric storage form")
    ap.add_argument("--no-factored", action="store_true", help="skip the factored-coupling form")
    ap.add_argument("--no-lowp", action="store_true", help="skip the complex64 / bf16-pair multi-RHS forms")
    ap.add_argument("--lowp-rhs", type=int, default=64)
    ap.add_argument("--lowp-forms", type=str, default="c64,bf16pair,c64fact,bf16pairfact,c128multi,c64stream,bf16pairstream",
                    help="comma list of the precision forms to time")
    ap.add_argument("--no-gmres", action="store_true", help="skip the time-to-solution comparison")
    ap.add_argument("--gmres-rhs", type=int, default=64)
    ap.add_argument("--gmres-tol", type=float, default=1e-8)
    ap.add_argument("--gmres-maxit", type=int, default=200)
    ap.add_argument("--gmres-small-n", type=int, default=65536,
                    help="size of the sphere at which the time-to-tolerance comparison runs to convergence")
    ap.add_argument("--gmres-tol-rhs", type=int, default=16,
                    help="right-hand sides of the time-to-tolerance comparison")
    ap.add_argument("--gmres-tol-maxit", type=int, default=6000,
                    help="iteration cap of the time-to-tolerance comparison")
    ap.add_argument("--inner-cycles", type=int, default=1,
                    help="GMRES-IR: GMRES(50) cycles per inner solve (1: every restart is a refinement step; "
                         "0: inner solves run to their inner tolerance)")
    ap.add_argument("--mode", choices=("headline", "batched", "serving", "gmres", "construct", "direct"),
                    default="headline",
                    help="headline: the FP64 workload and its side measurements; batched: many operators in "
                         "shared launches; serving: Poisson arrivals of GMRES solves; gmres: time to tolerance "
                         "of FP64 GMRES and GMRES-IR over sphere sizes; construct: ACA and near-field "
                         "sampling on the GPU vs the host builder; direct: direct UH construction vs the "
                         "two-phase builder (host only)")
    ap.add_argument("--gmres-sizes", type=str, default="16384,32768,65536",
                    help="sphere sizes of --mode gmres")
    ap.add_argument("--gmres-cases", type=str, default="", help="gmres mode: comma list of cases to run")
    ap.add_argument("--inner-tols", type=str, default="",
                    help="gmres mode: inner tolerances, e.g. c64fact=1e-4,bf16pairfact=1e-3")
    ap.add_argument("--nops", type=int, default=32)
    ap.add_argument("--rates", type=str, default="50,100,200,400")
    ap.add_argument("--requests", type=int, default=200, help="requests per arrival rate (serving)")
    ap.add_argument("--max-n", type=int, default=65536, help="largest operator of the batched mix")
    ap.add_argument("--serve-max-n", type=int, default=65536,
                    help="largest operator of the serving mix (GMRES(50) on larger spheres of this wavenumber "
                         "does not reach 1e-8 in thousands of iterations)")
    ap.add_argument("--serve-maxit", type=int, default=6000, help="iteration cap of a served solve")
    ap.add_argument("--serve-budget-mb", type=int, default=2048,
                    help="serving: run the highest rate once more under this HBM budget (0: skip)")
    ap.add_argument("--batch-storage", choices=("c64", "c64fact", "bf16pair", "bf16pairfact"), default="c64fact",
                    help="storage of the operators of the batched mode")
    ap.add_argument("--serve-storage", choices=("c64", "c64fact", "bf16pair", "bf16pairfact"), default="c64fact",
                    help="storage of the inner (low-precision) operators of the serving loop")
    ap.add_argument("--parity-leaves", type=int, default=6)
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "traffic_sphere262k_c128.json"),
                    help="JSON file with counter-derived HBM bytes per launch (used only if it was taken on the "
                         "current kernel source)")
    ap.add_argument("--construct", choices=("gpu", "host"), default="gpu",
                    help="headline: sample the operator's blocks (ACA, near field) on the GPU or on the host")
    ap.add_argument("--direct-only", action="store_true",
                    help="direct mode: skip the two-phase build (which holds the H and UH forms at once)")
    ap.add_argument("--full-build", action="store_true",
                    help="construct mode: also build the whole operator and check it against the dense matrix")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (the calibration kernel for the byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is a design "
              "described in DESIGN.md and is not built", file=sys.stderr)
        sys.exit(2)

    if args.mode == "direct":
        return run_direct(args)

    import numpy as np
    import torch

    from paper_2405_15573_amd import binding, builder, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    binding.load_library()
    if args.copy_calibration:
        a = torch.empty(1 << 26, dtype=torch.complex128, device="cuda")  # 1 GiB
        a.fill_(1.0)
        b = torch.empty_like(a)
        from paper_2405_15573_amd import traffic as trmod
        for _ in range(trmod.CALIBRATION_COPIES):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"copy calibration: {trmod.CALIBRATION_COPIES} copies of 1 GiB")

    if args.mode == "batched":
        return run_batched(args)
    if args.mode == "serving":
        return run_serving(args)
    if args.mode == "gmres":
        return run_gmres_sizes(args)
    if args.mode == "construct":
        return run_construct(args)

    t0 = time.perf_counter()
    cloud = inputs.make_cloud("sphere", args.n, seed=args.seed)
    log(f"building operator N={cloud.n} kappa={cloud.kappa:.3f} h={cloud.h:.5f}")
    op = builder.build_operator(cloud, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6, verbose=True,
                                construct=args.construct)
    st = op.stats()
    log(f"built in {time.perf_counter() - t0:.1f} s: {json.dumps(op.timings)}")
    log(json.dumps(st))

    stream = torch.cuda.Stream()
    t1 = time.perf_counter()
    duh = binding.upload(op, stream=stream)
    log(f"UH upload {time.perf_counter() - t1:.1f} s")
    info = duh.info()
    x_np = inputs.make_rhs(cloud.n, 1, seed=args.seed)[:, 0]
    x = torch.from_numpy(x_np).to("cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()

    pp_uh = {}
    t_uh, k_uh = time_products(torch, duh, x, y, args.steps, args.warmup, stream, per_product=pp_uh)
    y_uh = y.cpu().numpy()
    ab = algorithmic_bytes(info, cloud.n)
    log(f"UH MVP {t_uh * 1e3:.3f} ms; kernels " + json.dumps({k: round(v[0], 4) for k, v in k_uh.items()}))

    ctx = stream_context(torch)
    log(f"plain torch kernels: {json.dumps(ctx)}")

    # sampled parity at full size against the oracle (block-wise definition, restricted rows)
    from oracle import uniform
    leaves = np.nonzero(np.bincount(op.parent[op.parent >= 0], minlength=op.nclusters) == 0)[0]
    rng = np.random.default_rng(12345)
    pick = rng.choice(leaves, size=min(args.parity_leaves, leaves.size), replace=False)
    pos = np.concatenate([np.arange(op.off[c], op.off[c] + op.size[c]) for c in pick])
    tp = time.perf_counter()
    ref, users = uniform.uh_mvp_rows(vars(op), x_np, pos)
    parity = float(np.linalg.norm(y_uh[users] - ref[:, 0]) / np.linalg.norm(ref[:, 0]))
    log(f"sampled parity ({pos.size} rows) {parity:.3e} in {time.perf_counter() - tp:.1f} s")

    # symmetric storage (Remark 4.4): one block of each mirrored pair, applied both ways
    sym = None
    if not args.no_sym:
        ts = time.perf_counter()
        simg = builder.symmetric_image(op)
        dsym = binding.upload(simg, "c128sym", stream=stream)
        log(f"symmetric upload {time.perf_counter() - ts:.1f} s")
        sinfo = dsym.info()
        ys = torch.empty_like(x)
        pp_sy = {}
        t_sy, k_sy = time_products(torch, dsym, x, ys, args.steps, args.warmup, stream, per_product=pp_sy)
        y_sy = ys.cpu().numpy()
        abs_ = algorithmic_bytes(sinfo, cloud.n)
        tp = time.perf_counter()
        ref_s, users_s = uniform.uh_mvp_rows(uniform.expand_symmetric(simg), x_np, pos)
        par_s = float(np.linalg.norm(y_sy[users_s] - ref_s[:, 0]) / np.linalg.norm(ref_s[:, 0]))
        log(f"symmetric sampled parity {par_s:.3e} in {time.perf_counter() - tp:.1f} s")
        sym = {"ms_per_mvp": t_sy * 1e3, "mvps_per_s": 1.0 / t_sy, "gbs": abs_["total"] / t_sy / 1e9,
               "per_product_ms": pp_sy, "scratch_bytes": sinfo["scratch_bytes"],
               "vs_general_speedup": t_uh / t_sy,
               "bytes": abs_["total"], "bytes_per_kernel": abs_,
               "kernels_ms": {k: v[0] for k, v in k_sy.items()},
               "parity_sampled_rel_err": par_s,
               "rel_diff_vs_general": float(np.linalg.norm(y_sy - y_uh) / np.linalg.norm(y_uh)),
               "elems_coupling": sinfo["elems_coupling"], "elems_near": sinfo["elems_near"],
               "partial_coupling": sinfo["partial_coupling"], "partial_near": sinfo["partial_near"]}
        log(f"symmetric UH MVP {t_sy * 1e3:.3f} ms; kernels " + json.dumps({k: round(v[0], 4) for k, v in k_sy.items()}))
        dsym.free()
        del ys

    # factored couplings (section 4.2) in general storage, where they store fewer elements
    fact = None
    if not args.no_factored:
        tf = time.perf_counter()
        dfa = binding.upload(op, "c128fact", stream=stream)
        log(f"factored upload {time.perf_counter() - tf:.1f} s")
        finfo = dfa.info()
        yf = torch.empty_like(x)
        t_fa, k_fa = time_products(torch, dfa, x, yf, args.steps, args.warmup, stream)
        y_fa = yf.cpu().numpy()
        abf = algorithmic_bytes(finfo, cloud.n)
        tp = time.perf_counter()
        ref_f, users_f = uniform.uh_mvp_rows(uniform.assemble_factored(vars(op)), x_np, pos)
        par_f = float(np.linalg.norm(y_fa[users_f] - ref_f[:, 0]) / np.linalg.norm(ref_f[:, 0]))
        log(f"factored sampled parity {par_f:.3e} in {time.perf_counter() - tp:.1f} s")
        fact = {"ms_per_mvp": t_fa * 1e3, "mvps_per_s": 1.0 / t_fa, "gbs": abf["total"] / t_fa / 1e9,
                "bytes": abf["total"], "bytes_per_kernel": abf, "vs_general_speedup": t_uh / t_fa,
                "kernels_ms": {k: v[0] for k, v in k_fa.items()}, "parity_sampled_rel_err": par_f,
                "elems_coupling": finfo["elems_coupling"], "elems_coupling_in": finfo["elems_coupling_in"]}
        log(f"factored UH MVP {t_fa * 1e3:.3f} ms; kernels " + json.dumps({k: round(v[0], 4) for k, v in k_fa.items()}))
        dfa.free()
        del yf

    res_h = None
    if not args.no_h:
        t2 = time.perf_counter()
        dh = binding.upload_h(op, stream=stream)
        log(f"H upload {time.perf_counter() - t2:.1f} s")
        t_h, k_h = time_products(torch, dh, x, y, args.steps, args.warmup, stream)
        hinfo = dh.info()
        abh = algorithmic_bytes(hinfo, cloud.n)
        res_h = {"ms_per_mvp": t_h * 1e3, "mvps_per_s": 1.0 / t_h, "gbs": abh["total"] / t_h / 1e9,
                 "bytes": abh["total"], "kernels_ms": {k: v[0] for k, v in k_h.items()}}
        log(f"H MVP {t_h * 1e3:.3f} ms")
        dh.free()

    lowp = None
    if not args.no_lowp:
        lowp = {}
        r = args.lowp_rhs
        X64 = inputs.make_rhs(cloud.n, r, seed=args.seed + 7)
        Xd32 = torch.from_numpy(np.ascontiguousarray(X64.T.astype(np.complex64))).to("cuda").t()
        Yd32 = torch.empty((r, cloud.n), dtype=torch.complex64, device="cuda").t()
        Xd128 = torch.from_numpy(np.ascontiguousarray(X64.T)).to("cuda").t()
        Yd128 = torch.empty((r, cloud.n), dtype=torch.complex128, device="cuda").t()
        x1 = x.to(torch.complex64)
        y1 = torch.empty_like(x1)
        # many right-hand sides on the matrix cores (bound by them for complex64 and FP64,
        # by HBM for bf16 pairs: 8 r / e flop per operator byte), and one right-hand side in
        # the streaming forms (HBM-bound)
        wanted = [f for f in args.lowp_forms.split(",") if f]
        forms = (("c64", 157.3, 8), ("bf16pair", 2500.0, 4), ("c64fact", 157.3, 8), ("bf16pairfact", 2500.0, 4),
                 ("c128multi", 78.6, 16), ("c64stream", None, 8), ("bf16pairstream", None, 4))
        unknown = set(wanted) - {f[0] for f in forms}
        if unknown:
            raise SystemExit(f"unknown precision forms: {sorted(unknown)}")
        for st_name, peak_tf, e_bytes in (f for f in forms if f[0] in wanted):
            tl = time.perf_counter()
            dl = binding.upload(op, storage=st_name, stream=stream)
            log(f"{st_name} upload {time.perf_counter() - tl:.1f} s")
            li = dl.info()
            # elements the form multiplies (the factored forms apply fewer coupling elements)
            M_uh = li["elems_forward"] + li["elems_coupling"] + li["elems_coupling_in"] + li["elems_backward"] + \
                li["elems_near"]
            ve = 16 if st_name == "c128multi" else 8   # vector element bytes
            ent = {"nrhs": r}
            if peak_tf is not None:
                Xd, Yd = (Xd128, Yd128) if ve == 16 else (Xd32, Yd32)
                t_r, k_r = time_products(torch, dl, Xd, Yd, max(5, args.steps // 5), 2, stream)
                flops = 8.0 * r * M_uh
                bytes_r = e_bytes * M_uh + ve * r * (2 * cloud.n + 4 * info["rank_space"])
                ent.update({
                    "ms_per_mvp": t_r * 1e3, "rhs_per_s": r / t_r,
                    "tflops": flops / t_r / 1e12, "mfma_peak_tflops": peak_tf,
                    "mfma_frac": flops / t_r / 1e12 / peak_tf,
                    "gbs": bytes_r / t_r / 1e9, "hbm_frac": bytes_r / t_r / 1e9 / HBM_PEAK_GBS,
                    "kernels_ms": {k: v[0] for k, v in k_r.items()}})
                log(f"{st_name}: {r} RHS {t_r * 1e3:.3f} ms ({flops / t_r / 1e12:.1f} TFLOP/s, "
                    f"{bytes_r / t_r / 1e9:.0f} GB/s)")
            if ve == 16:
                xs1, ys1 = x, torch.empty_like(x)
            else:
                xs1, ys1 = x1, y1
            t_1, k_1 = time_products(torch, dl, xs1, ys1, args.steps, args.warmup, stream)
            y1n = ys1.cpu().numpy().astype(np.complex128)
            err_vs_fp64 = float(np.linalg.norm(y1n - y_uh) / np.linalg.norm(y_uh))
            g1 = (e_bytes * M_uh + 2 * ve * cloud.n) / t_1 / 1e9
            ent.update({"single_rhs_ms": t_1 * 1e3, "single_rhs_gbs": g1, "single_rhs_hbm_frac": g1 / HBM_PEAK_GBS,
                        "single_rhs_kernels_ms": {k: v[0] for k, v in k_1.items()},
                        "rel_err_vs_fp64": err_vs_fp64, "elem_bytes": e_bytes})
            lowp[st_name] = ent
            log(f"{st_name}: 1 RHS {t_1 * 1e3:.3f} ms ({g1:.0f} GB/s), err vs FP64 {err_vs_fp64:.2e}")
            dl.free()
        del Xd32, Yd32, Xd128, Yd128

    gm = None
    if not args.no_gmres:
        # the full-size operator at a fixed iteration cap (it does not reach 1e-8 within
        # thousands of iterations: the sphere at this wavenumber is near an interior resonance)
        gm = {"full_size": run_gmres_cases(torch, binding, op, cloud.n, args.gmres_rhs, args.gmres_tol,
                                           args.gmres_maxit, stream, args.seed, inner_cycles=args.inner_cycles)}
        gm["full_size"].update(n=cloud.n, nrhs=args.gmres_rhs, status="iteration cap (1e-8 not reached)")
        cs = inputs.make_cloud("sphere", args.gmres_small_n, seed=args.seed)
        log(f"building the N={cs.n} sphere for the time-to-tolerance comparison")
        ops_small = builder.build_operator(cs, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                           construct=args.construct)
        gm["to_tolerance"] = run_gmres_cases(torch, binding, ops_small, cs.n, args.gmres_tol_rhs, args.gmres_tol,
                                             args.gmres_tol_maxit, stream, args.seed, inner_cycles=args.inner_cycles)
        gm["to_tolerance"].update(n=cs.n, nrhs=args.gmres_tol_rhs)
        del ops_small

    cpu = None
    if not args.no_cpu:
        import numpy as _np
        ncores = uniform.max_threads()

        def cpu_times(fn, budget):
            """Three warm-ups (the first touches the operator pages), then up to 10 timed
            products within the budget; per-product seconds."""
            tw = time.perf_counter()
            fn()
            first = time.perf_counter() - tw
            fn()
            fn()
            reps = max(3, min(10, int(budget / max(first, 1e-3))))
            ts = []
            for _ in range(reps):
                tc = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - tc)
            return _np.array(ts)

        t6 = cpu_times(lambda: uniform.alg6(vars(op), x_np), args.cpu_seconds)
        t5 = cpu_times(lambda: uniform.alg5(vars(op), x_np), args.cpu_seconds / 2)
        tcpu = float(t6.mean())
        cpu = {"value": 1.0 / tcpu, "unit": "MVPs/s", "cores": ncores, "kind": "oracle",
               "sample": f"{t6.size} full products of the same N={cloud.n} operator with the C Algorithm 6 "
                         f"oracle (OpenMP, {ncores} threads) after three warm-ups",
               "gbs": ab["total"] / tcpu / 1e9, "ms_per_mvp": tcpu * 1e3,
               "ms_per_mvp_min": float(t6.min()) * 1e3, "ms_per_mvp_p50": float(_np.median(t6)) * 1e3,
               "h_mvp_alg5": {"ms_per_mvp": float(t5.mean()) * 1e3, "ms_per_mvp_min": float(t5.min()) * 1e3,
                              "ms_per_mvp_p50": float(_np.median(t5)) * 1e3, "products": int(t5.size),
                              "gbs": (abh["total"] / float(t5.mean()) / 1e9) if res_h else None},
               "h_over_uh": float(t5.mean()) / tcpu}
        log(f"CPU oracle {tcpu * 1e3:.1f} ms per MVP (Alg. 6), H-MVP {t5.mean() * 1e3:.1f} ms (Alg. 5) "
            f"on {ncores} threads")

    # further operator instances (the paper's protocol averages three): the headline product
    # on the operators of the other seeds, built and timed the same way
    per_seed = None
    extra = [int(v) for v in args.seeds.split(",") if v.strip() and int(v) != args.seed]
    if extra:
        import numpy as _np
        per_seed = {str(args.seed): pp_sy if sym is not None else pp_uh}
        for sd in extra:
            cl = inputs.make_cloud("sphere", args.n, seed=sd)
            tb = time.perf_counter()
            op_s = builder.build_operator(cl, leaf=args.leaf, eta=1.0, eps_aca=1e-6, eps_comp=1e-6,
                                          construct=args.construct)
            log(f"seed {sd}: built in {time.perf_counter() - tb:.1f} s")
            img = builder.symmetric_image(op_s) if sym is not None else op_s
            d_s = binding.upload(img, "c128sym" if sym is not None else "c128", stream=stream)
            xs = torch.from_numpy(inputs.make_rhs(cl.n, 1, seed=sd)[:, 0]).to("cuda")
            ys_ = torch.empty_like(xs)
            pp = {}
            t_s, _ = time_products(torch, d_s, xs, ys_, args.steps, args.warmup, stream, per_product=pp)
            pp["wall_ms_per_mvp"] = t_s * 1e3
            per_seed[str(sd)] = pp
            log(f"seed {sd}: {t_s * 1e3:.3f} ms per MVP, events {json.dumps(pp)}")
            d_s.free()
            del op_s, img, xs, ys_
        means = _np.array([v["mean_ms"] for v in per_seed.values()])
        per_seed["over_seeds"] = {"mean_ms": float(means.mean()), "min_ms": float(min(v["min_ms"] for v in per_seed.values())),
                                  "p50_of_means_ms": float(_np.median(means)), "seeds": [args.seed] + extra}

    # headline: the symmetric storage the paper's experiments use (Remark 4.4, section 6.1)
    # when it was run, else the general storage; both are reported
    general = {"ms_per_mvp": t_uh * 1e3, "mvps_per_s": 1.0 / t_uh, "gbs": ab["total"] / t_uh / 1e9,
               "per_product_ms": pp_uh, "scratch_bytes": info["scratch_bytes"],
               "bytes": ab["total"], "kernels_ms": {k: v[0] for k, v in k_uh.items()},
               "parity_sampled_rel_err": parity}
    if sym is not None:
        t_hd, k_hd, ab_hd, par_hd, storage = t_sy, k_sy, abs_, par_s, "complex128, symmetric (one block per mirrored pair)"
    else:
        t_hd, k_hd, ab_hd, par_hd, storage = t_uh, k_uh, ab, parity, "complex128, general (both triangles)"
    # dominant kernel and its roofline
    dom = max((k for k in k_hd if k in ab_hd), key=lambda k: k_hd[k][0])
    achieved = ab_hd[dom] / (k_hd[dom][0] * 1e-3) / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        from paper_2405_15573_amd import traffic as trmod
        tr = json.load(open(args.traffic))
        if tr.get("source_sha256") == trmod.kernel_source_sha256() and tr.get("n") == cloud.n:
            traffic = tr.get("bytes_per_launch", {}).get(dom)
    line = {
        "metric": METRIC,
        "value": 1.0 / t_hd,
        "unit": "MVPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_hd * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"uniform-H MVP, sphere N={cloud.n}, kappa*h=0.6, leaf {args.leaf}, eta 1, "
                               f"ACA/compression tol 1e-6, 1 RHS complex128",
                   "n": cloud.n, "nrhs": 1, "storage": storage, "leaf": args.leaf, "eta": 1.0, "eps": 1e-6,
                   "seed": args.seed},
        "gbs": ab_hd["total"] / t_hd / 1e9,
        "bytes_per_mvp": ab_hd["total"],
        "kernels_ms": {k: v[0] for k, v in k_hd.items()},
        "general_storage": general,
        "symmetric": sym,
        "general_factored": fact,
        "h_mvp": res_h,
        "uh_speedup_over_h": (res_h["ms_per_mvp"] / (t_uh * 1e3)) if res_h else None,
        "uh_symmetric_speedup_over_h": (res_h["ms_per_mvp"] / (t_sy * 1e3)) if (res_h and sym) else None,
        "parity_sampled_rel_err": par_hd,
        "per_product_ms": pp_sy if sym is not None else pp_uh,
        "per_seed": per_seed,
        "operator": {k: st[k] for k in ("nadm", "nden", "c_sp", "l_max", "k_max", "bytes_uh_c128", "bytes_h_c128")},
        "build": {"construct": args.construct, **{k: round(v, 3) for k, v in op.timings.items()}},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "hbm_context": ctx,
        "precision_forms": lowp,
        "gmres": gm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
