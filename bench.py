"""Benchmark: preconditioned Schur matvecs per second at N = 5000, p = 16.

Workload (the 5000-particle configuration): 5000 star particles
r(t) = 0.25 + 0.05 cos 5t of wavenumber 15 at uniform random rotations in a
400 x 38 strip of the middle layer (d = 40), layers k = (6, 9, 12), expansion
order p = 16, 1024 Sommerfeld nodes; seeded synthetic layout.  One step is one
matvec y = x - S (T + T_R) x of the GMRES operator (all steps of the hot path:
M2S, reflection, S2L, all-pairs M2L, scattering-matrix apply) in complex64
with FP32 accumulation (the mixed-precision configuration); the FP64 matvec
is timed beside it.  Inputs are resident in device memory before timing.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12   # MI355X FP32, TFLOP/s (vector and dense matrix cores alike)
PEAK_FP64 = 78.6e12    # MI355X FP64, TFLOP/s (vector and dense matrix cores alike)

# M2L launch variants (mpsl_set_tuning): kernel, bound, committed HBM-traffic
# summary and the source region its hash covers
M2L_VARIANTS = {
    0: ("k_m2l<{t},16,-1> (all-pairs M2L, one lane per target)", "alu", "m2l_5000stars_p16_hbm_traffic.md",
        ("// Row a1: all-pairs free-space M2L", "// FMM near field:")),
    1: ("k_m2l<{t},16,0|1> (all-pairs M2L, output halves)", "alu", None, None),
    2: ("k_m2l_mfma<{t},16,1> (all-pairs M2L on the matrix cores)", "mfma",
        "m2l_mfma_5000stars_p16_hbm_traffic.md",
        ("// Row a1 on the matrix cores, one right-hand side.", "// Row a1 for many right-hand sides")),
    3: ("k_m2l_mfma<{t},16,2> (all-pairs M2L on the matrix cores, 32 targets per wave)", "mfma", None, None),
}


def m2l_source_sha256(variant=0):
    """Hash of the source of one M2L kernel variant (its device code)."""
    region = M2L_VARIANTS[variant][3]
    with open(os.path.join(ROOT, "paper_1407_3868_amd", "csrc", "kernels.hip")) as fh:
        src = fh.read()
    a = src.index(region[0])
    b = src.index(region[1], a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def _m2l_traffic(variant, chunks=None):
    """Scaled HBM bytes per launch of the FP32 M2L kernel of this variant at this workload
    from the committed rocprofv3 counter summary; None when there is none, when the kernel
    source has changed since, or when the summary was taken at another number of source
    chunks than this run uses (the partial outputs scale with it)."""
    name = M2L_VARIANTS[variant][2]
    if name is None:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"m2l_traffic_bytes_fp32: (\d+)", text)
    h = re.search(r"m2l_source_sha256: ([0-9a-f]+)", text)
    if not m or not h or h.group(1) != m2l_source_sha256(variant):
        return None
    c = re.search(r"m2l_chunks_fp32: (\d+)", text)
    if chunks is not None and c and int(c.group(1)) != chunks:
        return None
    return int(m.group(1))


def _matvec_rate(ctx, torch, prec, x_np, steps, warmup):
    import numpy as np
    dt = np.complex64 if prec == 1 else np.complex128
    xd = torch.from_numpy(x_np.astype(dt)).cuda()
    yd = torch.zeros_like(xd)
    for _ in range(warmup):
        ctx.apply_dev(prec, xd, yd)
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.apply_dev(prec, xd, yd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m2l_ms, cnt = ctx.profile_read()
    ctx.profile(False)
    finite = bool(torch.isfinite(torch.view_as_real(yd)).all().item())
    return (t1 - t0), m2l_ms, cnt, finite


def _oracle_m2l_part(args):
    """One worker of the all-core oracle timing: the oracle's M2L for some targets."""
    xy, k2, p, x, targets = args
    from threadpoolctl import threadpool_limits

    from oracle import operators as oo
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oo.m2l_apply(xy, k2, p, x, targets=targets)
        return time.perf_counter() - t0


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def _cpu_baseline(wl, S, x, n_targets=24):
    """The FP64 oracle's matvec, timed on a bounded sample of the workload: on
    one host thread, and on every core available to the process (the sampled
    targets' M2L spread over one worker process per core, the BLAS parts
    threaded over all cores)."""
    import concurrent.futures

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import contour as oc
    from oracle import operators as oo
    from oracle import system as osys

    model, cores = _host_cpu()
    lam, w = oc.contour(wl.n_nodes, wl.b, wl.t_max, [wl.k1, wl.k2, wl.k3])
    pr = osys.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, S, wl.xy, wl.rot, lam, w)
    tg = list(np.linspace(0, wl.n - 1, n_targets).astype(int))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oo.m2l_apply(wl.xy, wl.k2, wl.p, x, targets=tg)
        t1 = time.perf_counter()
        sig = pr.sigma(beta=x)
        t2 = time.perf_counter()
        a = oo.s2l(sig[:, 1], sig[:, 2], wl.xy, lam, w, wl.k2, wl.d, wl.p)
        t3 = time.perf_counter()
        pr.apply_S(a[tg], targets=tg)
        t4 = time.perf_counter()
    one = (t1 - t0) * wl.n / n_targets + (t2 - t1) + (t3 - t2) + (t4 - t3) * wl.n / n_targets
    # all cores: n_targets per worker, one worker per core
    tall = list(np.linspace(0, wl.n - 1, n_targets * cores).astype(int))
    parts = [(wl.xy, wl.k2, wl.p, x, tall[i::cores]) for i in range(cores)]
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_m2l_part, parts[:cores]))       # start-up of the workers, untimed
        a0 = time.perf_counter()
        list(ex.map(_oracle_m2l_part, parts))
        a1 = time.perf_counter()
    with threadpool_limits(limits=cores):
        a2 = time.perf_counter()
        sig = pr.sigma(beta=x)
        a = oo.s2l(sig[:, 1], sig[:, 2], wl.xy, lam, w, wl.k2, wl.d, wl.p)
        a3 = time.perf_counter()
    allc = (a1 - a0) * wl.n / len(tall) + (a3 - a2) + (t4 - t3) * wl.n / n_targets / cores
    return {"value": 1.0 / allc, "unit": "matvecs/s", "cores": cores, "kind": "oracle", "cpu_model": model,
            "one_thread": {"value": 1.0 / one, "seconds_per_matvec": one},
            "seconds_per_matvec": allc,
            "sample": (f"FP64 numpy/scipy oracle on {model}: all-pairs M2L for {len(tall)} of {wl.n} targets "
                       f"in {cores} worker processes (one per core, scaled by {wl.n}/{len(tall)}), M2S, 4x4 node "
                       f"solves and S2L in full with {cores} BLAS threads, S-apply scaled from one thread; "
                       f"{allc:.1f} s per full matvec on all cores, {one:.1f} s on one thread "
                       f"({n_targets} targets)")}


def _cpu_baseline_full(args):
    """The rest of the oracle timing plan, on the host alone (no GPU): the
    dense assembly of eq. (49) and its LU solve for the 16-disk (C1) and the
    1000-star (C2) recipes with BLAS threads on every core, and the oracle's
    matrix-free matvec for two right-hand sides and two of the perturbed
    configurations of the 2000-star batching recipe (C4).  The 5000-star
    dense system (436 GB) is out of reach; its matrix-free matvec is the
    default run's cpu_baseline."""
    import concurrent.futures

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import contour as oc
    from oracle import mie as omie
    from oracle import star as ostar
    from oracle import system as osys
    from synth import make_workload, perturbed_layout, rejection_layout

    model, cores = _host_cpu()
    out = {"kind": "oracle", "cpu_model": model, "cores": cores}

    def problem(wl, S, xy=None, rot=None, d=None, b=None):
        lam, w = oc.contour(wl.n_nodes, wl.b if b is None else b, wl.t_max, [wl.k1, wl.k2, wl.k3])
        return osys.Problem(wl.k1, wl.k2, wl.k3, wl.d if d is None else d, wl.p, S,
                            wl.xy if xy is None else xy, wl.rot if rot is None else rot, lam, w)

    def smatrix(wl):
        if wl.shape == "disk":
            return np.diag(omie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
        a1, a2, a3 = wl.shape_params
        return ostar.star_smatrix(a1, a2, a3, wl.k2, wl.kp, wl.p, nb=256)

    for name in ("c1", "c2"):
        wl = make_workload(name)
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            S = smatrix(wl)
            t1 = time.perf_counter()
            pr = problem(wl, S)
            K = pr.dense()
            t2 = time.perf_counter()
            print(f"# cpu {name}: assembled {wl.n * wl.P} unknowns in {t2 - t1:.1f} s", file=sys.stderr, flush=True)
            b = pr.rhs(wl.src[0]).reshape(-1)
            beta = np.linalg.solve(K, b)
            t3 = time.perf_counter()
        res = float(np.linalg.norm(K @ beta - b) / np.linalg.norm(b))
        del K
        out[name] = {"particles": wl.n, "unknowns": wl.n * wl.P, "scattering_matrix_s": t1 - t0,
                     "assembly_s": t2 - t1, "lu_solve_s": t3 - t2, "relative_residual": res}
        print(f"# cpu {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)

    wl = make_workload("c4", n_rhs=2, src_seed=4)
    with threadpool_limits(limits=cores):
        S = smatrix(wl)
    rng = np.random.default_rng(5)
    ns = np.round(np.exp(rng.uniform(np.log(500), np.log(4000), 32))).astype(int)
    cases = [("rhs 0", wl.xy, wl.rot, wl.d, wl.b, wl.src[0]), ("rhs 1", wl.xy, wl.rot, wl.d, wl.b, wl.src[1])]
    for i in range(2):
        width = ns[i] / (0.3 * 18.0)
        xy, rot = rejection_layout(int(ns[i]), (-width / 2, width / 2), (-19.0, -1.0), 0.75, 100 + i)
        xy, rot = perturbed_layout(xy, rot, 0.05, 200 + i, 0.75, y_range=(-19.6, -0.4))
        cases.append((f"config {i} (N = {ns[i]})", xy, rot, 20.0, min(0.2, 2.0 / width), (0.0, 2.0)))
    c4 = []
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores) as ex:
        for label, xy, rot, d, b, src in cases:
            pr = problem(wl, S, xy, rot, d, b)
            x = pr.rhs(src)
            n = xy.shape[0]
            tg = list(range(n))
            parts = [(xy, wl.k2, wl.p, x, tg[i::cores]) for i in range(cores)]
            a0 = time.perf_counter()
            list(ex.map(_oracle_m2l_part, parts))
            a1 = time.perf_counter()
            with threadpool_limits(limits=cores):
                pr.apply_S(pr.layer_local(beta=x))   # M2S, node solves, S2L and the S apply
                a2 = time.perf_counter()
            c4.append({"case": label, "particles": int(n), "m2l_s": a1 - a0, "layered_s": a2 - a1,
                       "matvec_s": a2 - a0})
            print(f"# cpu c4 {label}: {json.dumps(c4[-1])}", file=sys.stderr, flush=True)
    out["c4_matvecs"] = c4
    out["c3_note"] = ("5000 stars: dense LU needs 436 GB; the matrix-free matvec is the default run's "
                      "cpu_baseline, and a 1450-iteration GMRES at that rate is the matvec time times 1450")
    return out


def _batch_workload(args, torch, mp):
    """64 sources over one 2000-star p = 12 geometry, and 32 perturbed configurations."""
    import numpy as np

    from synth import make_workload, perturbed_layout, rejection_layout

    wl = make_workload("c4", n_rhs=64, src_seed=4)
    a1, a2, a3 = wl.shape_params
    S = mp.compute_star_smatrix(a1, a2, a3, wl.k2, wl.kp, wl.p, 256)
    stream = torch.cuda.current_stream().cuda_stream

    def context(xy, rot, d, b):
        c = mp.Context(0)
        c.set_stream(stream)
        c.set_layers(wl.k1, wl.k2, wl.k3, d)
        c.set_scattering_matrix(wl.p, wl.r_enclose, S)
        c.set_geometry(xy, rot)
        c.set_contour(wl.n_nodes, b, wl.t_max)
        return c

    out = {"workload": "64 point sources over 2000 stars (p=12, 512 nodes); 32 perturbed configurations, "
                       "N log-uniform in [500, 4000]"}
    ctx = context(wl.xy, wl.rot, wl.d, wl.b)
    R = wl.src.shape[0]
    X = np.stack([ctx.rhs(s) for s in wl.src])
    res = {}
    for name, prec in (("fp32", 1), ("fp64", 0)):
        ctx.autotune(prec)
        npdt = np.complex64 if prec == 1 else np.complex128
        xd = torch.from_numpy(X.astype(npdt)).cuda()
        yd = torch.zeros_like(xd)
        for _ in range(args.warmup):
            ctx.apply_batch_dev(prec, R, xd, yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.apply_batch_dev(prec, R, xd, yd)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / args.steps
        x1, y1 = xd[0].contiguous(), yd[0].clone()
        for _ in range(args.warmup):
            ctx.apply_dev(prec, x1, y1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for r in range(R):
                ctx.apply_dev(prec, xd[r], yd[r])
        torch.cuda.synchronize()
        t_loop = (time.perf_counter() - t0) / args.steps
        flops = 8.0 * wl.P ** 2 * wl.n * (wl.n - 1) * R
        res[name] = {"rhs_matvecs_per_s": R / t_batch, "ms_per_batch": t_batch * 1e3,
                     "ms_per_64_single_matvecs": t_loop * 1e3, "batched_vs_loop": t_loop / t_batch,
                     "m2l_tflops_equivalent": flops / t_batch / 1e12}
    out["multi_rhs"] = res

    rng = np.random.default_rng(5)
    ns = np.round(np.exp(rng.uniform(np.log(500), np.log(4000), 32))).astype(int)
    ctxs, xs, ys, pairs = [], [], [], 0
    for i, n in enumerate(ns):
        width = n / (0.3 * 18.0)
        xy, rot = rejection_layout(int(n), (-width / 2, width / 2), (-19.0, -1.0), 0.75, 100 + i)
        xy, rot = perturbed_layout(xy, rot, 0.05, 200 + i, 0.75, y_range=(-19.6, -0.4))
        c = context(xy, rot, 20.0, min(0.2, 2.0 / width))
        ctxs.append(c)
        pairs += int(n) * (int(n) - 1)
    cfg = {}
    for name, prec in (("fp32", 1), ("fp64", 0)):
        npdt = np.complex64 if prec == 1 else np.complex128
        xs = [torch.from_numpy(np.stack([c.rhs(np.array([0.0, 2.0]))]).astype(npdt)).cuda() for c in ctxs]
        ys = [torch.zeros_like(x) for x in xs]
        t0 = time.perf_counter()
        batch = mp.Batch([(c, prec, 1, x, y) for c, x, y in zip(ctxs, xs, ys)])
        t_cap = time.perf_counter() - t0
        for _ in range(args.warmup):
            batch.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.launch(stream)
        torch.cuda.synchronize()
        t_graph = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for c, x, y in zip(ctxs, xs, ys):
                c.apply_dev(prec, x, y)
        torch.cuda.synchronize()
        t_eager = (time.perf_counter() - t0) / args.steps
        batch.close()
        cfg[name] = {"config_matvecs_per_s": len(ctxs) / t_graph, "ms_per_graph": t_graph * 1e3,
                     "ms_eager_sequence": t_eager * 1e3, "graph_vs_eager": t_eager / t_graph,
                     "capture_s": t_cap,
                     "m2l_tflops_equivalent": 8.0 * wl.P ** 2 * pairs / t_graph / 1e12}
    out["multi_config"] = cfg
    out["configs_n"] = [int(n) for n in ns]
    return out


def _serve_requests(mp, nreq, prec, n_max=20000):
    """The design-loop request stream: N log-uniform in [200, n_max], p in
    {8, 12, 16}, star or disk, k2 ~ U[6, 12], d ~ U[8, 60], strip of height
    d - 2 and width N / (0.3 (d - 2)), source at (0, 2); span-rule contours
    resolving the strip's width (h = 12 / X for the mixed solves' 1e-6, 6 / X
    for FP64's 1e-10) with the interpolated Sommerfeld transforms, except
    where that rule would pass 2^19 nodes (count rule, 1024 nodes, reported);
    the cluster-block preconditioner; tol 1e-6 (mixed) / 1e-10 (FP64)."""
    import numpy as np

    from synth import rejection_layout

    rng = np.random.default_rng(6)
    tol = 1e-6 if prec == 1 else 1e-10
    reqs = []
    for i in range(nreq):
        n = int(round(np.exp(rng.uniform(np.log(200), np.log(n_max)))))
        p = int(rng.choice([8, 12, 16]))
        star = bool(rng.integers(0, 2))
        k2 = float(rng.uniform(6.0, 12.0))
        d = float(rng.uniform(8.0, 60.0))
        h = d - 2.0
        width = n / (0.3 * h)
        xy, rot = rejection_layout(n, (-width / 2, width / 2), (-d + 1.0, -1.0), 0.75, 1000 + i)
        b, hmax = mp.span_contour_params(width, tol)
        ns = len(mp.compute_contour_span((6.0, k2, 12.0), b, 24.0, hmax)[0]) if width < 40000 else 1 << 30
        r = dict(k=(6.0, k2, 12.0), d=d, particle=1 if star else 0, shape=(0.25, 0.05, 5) if star else (0.25,),
                 kp=15.0, p=p, xy=xy, rot=rot, src=(0.0, 2.0), tol=tol, maxiter=3000, n_bdry=128, precision=prec,
                 precond=mp.PRECOND_CLUSTER, inner_tol=1e-5)
        if ns <= (1 << 19):
            r.update(contour=1, n_nodes=0, b=b, t_max=24.0, h_max=hmax, sommerfeld=mp.SOMM_INTERP)
        else:
            r.update(contour=0, n_nodes=1024, b=min(0.2, 2.0 / width), t_max=32.0)
        reqs.append((r, ns))
    return reqs


def _serve_workload(args, torch, mp, n_max=20000):
    """A Poisson stream of design-loop requests through the continuous-batching server."""
    import numpy as np

    nreq = args.requests
    far = " (FMM far field above 8000)" if n_max > 8000 else ""
    out = {"workload": (f"{nreq} requests: N log-uniform [200, {n_max}]{far}, p in {{8, 12, 16}}, "
                        "star or disk, k2 ~ U[6, 12], d ~ U[8, 60], span-rule contours (interpolated transforms) "
                        "resolving each strip, cluster-block preconditioner, tol 1e-6 mixed / 1e-10 FP64; "
                        "Poisson arrivals at 0.8 / (mean isolated service time)")}
    modes = [(name, prec) for name, prec in (("mixed", 1), ("fp64", 0)) if name in args.serve_modes.split(",")]
    for name, prec in modes:
        reqs = _serve_requests(mp, nreq, prec, n_max)
        # isolated service time on a calibration sample
        srv = mp.Server(0, hbm_budget=200 << 30, max_active=1)
        cal = []
        for i, (r, ns) in enumerate(reqs[:args.serve_calibration]):
            cal.append(srv.wait(srv.submit(**r)))
            print(f"# serve {name} calibration {i}: N {r['xy'].shape[0]}, p {r['p']}, {ns} nodes, "
                  f"{cal[-1]['iterations']} its, {cal[-1]['t_finish'] - cal[-1]['t_submit']:.2f} s, "
                  f"status {cal[-1]['status']}", file=sys.stderr, flush=True)
        srv.close()
        mean_service = float(np.mean([c["t_finish"] - c["t_submit"] for c in cal]))
        qps = 0.8 / mean_service
        gaps = np.random.default_rng(7).exponential(1.0 / qps, nreq)
        srv = mp.Server(0, hbm_budget=200 << 30, max_active=16)
        t0 = time.perf_counter()
        tickets = []
        for i, ((r, ns), g) in enumerate(zip(reqs, gaps)):
            time.sleep(float(g))
            tickets.append(srv.submit(**r))
            print(f"# serve {name} submitted {i} at {time.perf_counter() - t0:.1f} s: N {r['xy'].shape[0]}, "
                  f"p {r['p']}, {ns} nodes", file=sys.stderr, flush=True)
        res = [None] * len(tickets)
        pending = list(range(len(tickets)))
        while pending:  # in order of completion
            left = []
            for i in pending:
                r = srv.wait(tickets[i], timeout=0.0)
                if r is None:
                    left.append(i)
                    continue
                res[i] = r
                print(f"# serve {name} request {i}: {r['iterations']} its, "
                      f"{r['t_finish'] - r['t_submit']:.2f} s, status {r['status']}", file=sys.stderr, flush=True)
            pending = left
            if pending:
                time.sleep(0.05)
        wall = time.perf_counter() - t0
        srv.close()
        lat = np.array([r["t_finish"] - r["t_submit"] for r in res]) * 1e3
        ok = np.array([r["status"] == 0 for r in res])
        resolved = sum(1 for r, _ in reqs if r["contour"] == 1)
        out[name] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                     "mean_ms": float(lat.mean()), "throughput_req_s": nreq / wall, "qps_offered": qps,
                     "mean_isolated_service_ms": mean_service * 1e3, "converged": int(ok.sum()), "requests": nreq,
                     "p50_ms_converged": float(np.percentile(lat[ok], 50)) if ok.any() else None,
                     "p99_ms_converged": float(np.percentile(lat[ok], 99)) if ok.any() else None,
                     "span_rule_requests": resolved, "max_nodes": int(max(ns for _, ns in reqs)),
                     "iterations_mean": float(np.mean([r["iterations"] for r in res])),
                     "statuses": sorted(set(int(r["status"]) for r in res))}
        print(f"# serve {name}: p50 {out[name]['p50_ms']:.1f} ms, p99 {out[name]['p99_ms']:.1f} ms, "
              f"{int(ok.sum())}/{nreq} converged", file=sys.stderr, flush=True)
    return out


def _fmm_workload(args, torch, mp):
    """20000 stars, p = 16: the FMM far field (the default above 8000
    particles) against the direct all-pairs M2L on the same context."""
    import numpy as np

    from synth import make_workload

    wl = make_workload("c5max")
    a1, a2, a3 = wl.shape_params
    stream = torch.cuda.current_stream().cuda_stream
    ctx = mp.Context(0)
    ctx.set_stream(stream)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_particle_star(a1, a2, a3, wl.kp, wl.p, 256)
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    S = ctx.get_scattering_matrix()
    rng = np.random.default_rng(1)
    r = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    n = np.arange(-wl.p, wl.p + 1)
    x = np.stack([np.exp(1j * (n[None, :] - n[:, None]) * wl.rot[l]) * S @ r[l] for l in range(wl.n)])
    out = {"metric": "GMRES matvecs/s", "unit": "matvec/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "config": {"workload": "20000 stars, p=16, 1024 contour nodes, strip 1754 x 38, "
                                                      "FMM far field (MPSL_FAR_AUTO)"}}
    res = {}
    y_ref = {}
    for mode, method in (("fmm", mp.FAR_AUTO), ("direct", mp.FAR_DIRECT)):
        ctx.set_far_field(method)
        t0 = time.perf_counter()
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros_like(xd)
        ctx.apply_dev(0, xd, yd)   # builds the tables of this far-field method
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        y_ref[mode] = yd.cpu().numpy()
        steps = args.steps if mode == "fmm" else max(2, args.steps // 10)
        for name, prec in (("fp32", 1), ("fp64", 0)):
            dt, far_ms, cnt, finite = _matvec_rate(ctx, torch, prec, x, steps, 1)
            res.setdefault(mode, {})[name] = {"matvecs_per_s": steps / dt, "ms_per_matvec": dt / steps * 1e3,
                                              "far_field_ms": far_ms, "finite": finite, "steps": steps}
            if mode == "fmm":
                res[mode][name]["info"] = ctx.fmm_info(prec)
        res[mode]["setup_s"] = setup
    err = float(np.linalg.norm(y_ref["fmm"] - y_ref["direct"]) / np.linalg.norm(y_ref["direct"]))
    out["fmm"] = res["fmm"]
    out["direct"] = res["direct"]
    out["fmm_vs_direct_fp64_matvec_rel_err"] = err
    for name in ("fp32", "fp64"):
        out["fmm"][name]["speedup_vs_direct"] = (res["direct"][name]["ms_per_matvec"] /
                                                 res["fmm"][name]["ms_per_matvec"])
    out["value"] = res["fmm"]["fp32"]["matvecs_per_s"]
    out["dtype"] = "f32 (f64 tables)"
    return out


def _solve_leg(args, mp, ctx, wl, flops):
    """Solves of eq. (49) at the benchmark configuration to tol 1e-6, with the
    cluster-block right preconditioner (built once per geometry, timed as
    setup), for seeded point sources: p50 / p99 per precision, and the field
    of the mixed-precision solution against the FP64 one at 4096 seeded
    receivers in all three layers."""
    import numpy as np

    from synth import receivers

    rng = np.random.default_rng(1003)
    srcs = [np.array([0.0, 2.0])] + [np.array([rng.uniform(-200.0, 200.0), rng.uniform(1.0, 3.0)])
                                     for _ in range(args.solve_sources - 1)]
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, args.cluster)
    res = {"tol": wl.tol, "preconditioner": {"kind": "cluster blocks", "cluster_size": args.cluster}}
    betas = {}
    for name, prec in (("mixed", 1), ("fp64", 0)):
        secs, its, conv, metas = [], [], 0, []
        for i, src in enumerate(srcs):
            beta, meta = ctx.solve(src, precision=prec, tol=wl.tol, maxiter=args.solve_maxiter, inner_tol=1e-5)
            secs.append(meta["seconds"] - meta["precond_seconds"])
            its.append(meta["iterations"])
            conv += meta["status"] == 0
            metas.append(meta)
            if i == 0:
                betas[name] = beta
            print(f"# solve {name} source {i}: {meta['iterations']} its, {secs[-1]:.2f} s, "
                  f"res {meta['rel_residual']:.2e}", file=sys.stderr, flush=True)
        ms = np.array(secs) * 1e3
        ms_it = float(np.sum(ms) / max(1, np.sum(its)))
        peak = PEAK_FP32 if prec == 1 else PEAK_FP64
        res[name] = {"sources": len(srcs), "converged": int(conv), "p50_ms": float(np.percentile(ms, 50)),
                     "p99_ms": float(np.percentile(ms, 99)), "mean_ms": float(ms.mean()),
                     "iterations": its, "refinements": [m["refinements"] for m in metas],
                     "rel_residual_max": float(max(m["rel_residual"] for m in metas)),
                     "ms_per_iteration": ms_it,
                     # ideal time of the iteration's M2L at the peak / measured time per iteration
                     "iteration_roofline_frac": flops / peak * 1e3 / ms_it}
    res["preconditioner"].update(ctx.precond_info())
    xs = wl.xy[:, 0]
    rcv = receivers(4096, (xs.min() - 2.0, xs.max() + 2.0), (-wl.d - 2.0, 3.0), wl.xy, 1002, particle_excl=0.35,
                    source=srcs[0], source_excl=0.05)
    u32 = ctx.eval_field(srcs[0], betas["mixed"], rcv)
    u64 = ctx.eval_field(srcs[0], betas["fp64"], rcv)
    res["field_4096_receivers"] = {
        "mixed_vs_fp64_rel_l2": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64)),
        "mixed_vs_fp64_max_rel": float(np.max(np.abs(u32 - u64)) / np.max(np.abs(u64))),
        "note": "both solves to relative residual 1e-6; the difference is that tolerance amplified by the "
                "conditioning, not the error of the FP32 arithmetic"}
    # the mixed-precision field error itself: mixed to 1e-8 against an FP64 reference to 1e-10
    bt, mt = ctx.solve(srcs[0], precision=1, tol=1e-8, maxiter=args.solve_maxiter, inner_tol=1e-5)
    br, mr = ctx.solve(srcs[0], precision=0, tol=1e-10, maxiter=args.solve_maxiter)
    ut, ur = ctx.eval_field(srcs[0], bt, rcv), ctx.eval_field(srcs[0], br, rcv)
    res["field_4096_receivers"]["tight"] = {
        "mixed_tol": 1e-8, "fp64_tol": 1e-10, "mixed_iterations": mt["iterations"],
        "fp64_iterations": mr["iterations"], "converged": bool(mt["status"] == 0 and mr["status"] == 0),
        "mixed_seconds": mt["seconds"], "fp64_seconds": mr["seconds"],
        "mixed_vs_fp64_rel_l2": float(np.linalg.norm(ut - ur) / np.linalg.norm(ur)),
        "mixed_vs_fp64_max_rel": float(np.max(np.abs(ut - ur)) / np.max(np.abs(ur)))}
    print(f"# tight pair: {json.dumps(res['field_4096_receivers']['tight'])}", file=sys.stderr, flush=True)
    return res


def _span_leg(args, torch, mp, wl, x, y_count):
    """The same 5000-particle matvec on span-rule contours (panels no longer
    than h = 12/X and 6/X for the strip's extent X, b = 2/X, t_max = 24), which
    resolve e^{i lambda x} across the strip; the workload's 1024-node contour
    does not.  Reports rates and how far the 1024-node matvec is from the
    converged one."""
    import numpy as np

    a1, a2, a3 = wl.shape_params
    X = float(wl.xy[:, 0].max() - wl.xy[:, 0].min())
    res = {"extent_x": X, "b": 2.0 / X, "t_max": 24.0}
    y6 = None
    for label, hf, method in (("h12", 12.0, mp.SOMM_DIRECT), ("h6", 6.0, mp.SOMM_DIRECT),
                              ("h12_interp", 12.0, mp.SOMM_INTERP), ("h6_interp", 6.0, mp.SOMM_INTERP)):
        ctx = mp.Context(0)
        ctx.set_sommerfeld_method(method)
        ctx.set_stream(torch.cuda.current_stream().cuda_stream)
        ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
        ctx.set_particle_star(a1, a2, a3, wl.kp, wl.p, 256)
        ctx.set_geometry(wl.xy, wl.rot)
        ns = ctx.set_contour_span(min(0.2, 2.0 / X), 24.0, hf / X)
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros_like(xd)
        ctx.apply_dev(0, xd, yd)
        torch.cuda.synchronize()
        leg = {"h_max": hf / X, "n_nodes": ns, "sommerfeld": "interp" if method == mp.SOMM_INTERP else "direct"}
        if method == mp.SOMM_INTERP:
            leg["somm_plan"] = ctx.somm_info()
        for name, prec in (("fp32", 1), ("fp64", 0)):
            dt, m2l_ms, _, fin = _matvec_rate(ctx, torch, prec, x, args.steps, args.warmup)
            leg[name] = {"matvecs_per_s": args.steps / dt, "ms_per_matvec": dt / args.steps * 1e3,
                         "m2l_ms": m2l_ms, "finite": fin}
        if label == "h6":
            y6 = yd.cpu().numpy()
        elif label == "h12":
            y12 = yd.cpu().numpy()
        else:
            leg["fp64_matvec_rel_diff_vs_direct"] = float(
                np.linalg.norm(yd.cpu().numpy() - (y6 if label == "h6_interp" else y12)) /
                np.linalg.norm(y6 if label == "h6_interp" else y12))
        res[label] = leg
        del ctx
        torch.cuda.empty_cache()
    ref = np.linalg.norm(y6)
    res["fp64_matvec_rel_diff_h12_vs_h6"] = float(np.linalg.norm(y12 - y6) / ref)
    res["fp64_matvec_rel_diff_1024_nodes_vs_h6"] = float(np.linalg.norm(y_count - y6) / ref)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-solve", action="store_true", help="skip the solve timings")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--solve-maxiter", type=int, default=4000)
    ap.add_argument("--solve-sources", type=int, default=10, help="seeded point sources per precision")
    ap.add_argument("--cluster", type=int, default=160, help="largest cluster of the block preconditioner")
    ap.add_argument("--no-batch", action="store_true", help="skip the short many-RHS / many-config leg")
    ap.add_argument("--no-autotune", action="store_true", help="use the default M2L launch shape")
    ap.add_argument("--no-fmm", action="store_true", help="skip the FMM far-field comparison")
    ap.add_argument("--no-span", action="store_true", help="skip the span-rule contour legs")
    ap.add_argument("--workload", choices=["c3", "batch", "serve", "fmm", "cpu"], default="c3",
                    help="c3: the 5000-particle matvec (default); batch: multi-RHS and multi-config batching; "
                         "serve: Poisson request stream through the server; fmm: 20000 particles, FMM vs direct; "
                         "cpu: the oracle's dense assembly and LU (16 disks, 1000 stars) and matvecs of the "
                         "2000-star batching recipe on the host (no GPU)")
    ap.add_argument("--requests", type=int, default=40, help="serve: number of requests")
    ap.add_argument("--serve-calibration", type=int, default=6, help="serve: requests timed alone for the QPS")
    ap.add_argument("--serve-modes", default="mixed,fp64", help="serve: precisions to run (mixed, fp64)")
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving leg")
    ap.add_argument("--no-fmm20k", action="store_true", help="skip the short 20000-particle FMM leg")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "cpu":
        print(json.dumps({"cpu_baseline_full": _cpu_baseline_full(args)}), flush=True)
        return

    import numpy as np
    import torch

    import paper_1407_3868_amd as mp
    from synth import make_workload

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.workload == "batch":
        print(json.dumps(_batch_workload(args, torch, mp)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(_serve_workload(args, torch, mp)), flush=True)
        return
    if args.workload == "fmm":
        print(json.dumps(_fmm_workload(args, torch, mp)), flush=True)
        return
    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = make_workload("c3")
    a1, a2, a3 = wl.shape_params

    t_setup0 = time.perf_counter()
    ctx = mp.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_particle_star(a1, a2, a3, wl.kp, wl.p, 256)
    t_smat = time.perf_counter()
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    S = ctx.get_scattering_matrix()
    rng = np.random.default_rng(1)
    r = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    n = np.arange(-wl.p, wl.p + 1)
    x = np.stack([np.exp(1j * (n[None, :] - n[:, None]) * wl.rot[l]) * S @ r[l] for l in range(wl.n)])
    # first call builds the per-pair and per-node device tables
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros_like(xd)
    ctx.apply_dev(0, xd, yd)
    torch.cuda.synchronize()
    t_setup1 = time.perf_counter()
    # launch-shape autotuning of the M2L kernel, per precision (before timing)
    tuning = {}
    for name, prec in (("fp32", 1), ("fp64", 0)):
        if not args.no_autotune:
            ctx.autotune(prec)
        tuning[name] = ctx.get_tuning(prec)
    t_tune = time.perf_counter()

    el32, m2l32, cnt32, fin32 = _matvec_rate(ctx, torch, 1, x, args.steps, args.warmup)
    el64, m2l64, cnt64, fin64 = _matvec_rate(ctx, torch, 0, x, args.steps, args.warmup)
    flops = 8.0 * wl.P ** 2 * wl.n * (wl.n - 1)
    v32, v64 = tuning["fp32"]["variant"], tuning["fp64"]["variant"]
    ach32 = flops / (m2l32 * 1e-3)
    ach64 = flops / (m2l64 * 1e-3)
    value = args.steps / el32
    value64 = args.steps / el64

    out = {
        "metric": "GMRES matvecs/s at N=5000,p=16",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": ("5000 stars r=0.25+0.05cos5t, kp=15, p=16, k=(6,9,12), d=40, 400x38 strip, "
                         "1024 Sommerfeld nodes; one Schur matvec in complex64 (mixed-precision mode)"),
            "n_particles": wl.n, "p": wl.p, "n_nodes": wl.n_nodes, "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": M2L_VARIANTS[v32][0].format(t="float"),
            "bound": M2L_VARIANTS[v32][1],
            "achieved": ach32 / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": ach32 / PEAK_FP32,
            "traffic": _m2l_traffic(v32, tuning["fp32"]["chunks"]),
            "avg_ms": m2l32,
            "launches": cnt32,
            "algorithmic_flops_per_launch": flops,
        },
        "fp64": {
            "value": value64, "unit": "matvecs/s", "ms_per_step": el64 / args.steps * 1e3,
            "roofline": {"kernel": M2L_VARIANTS[v64][0].format(t="double"), "bound": M2L_VARIANTS[v64][1],
                         "achieved": ach64 / 1e12,
                         "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": ach64 / PEAK_FP64,
                         "avg_ms": m2l64, "launches": cnt64},
        },
        "mixed_vs_fp64_matvec_speedup": value / value64,
        "setup_s": {"scattering_matrix": t_smat - t_setup0, "tables_and_first_matvec": t_setup1 - t_smat,
                    "autotune": t_tune - t_setup1},
        "m2l_tuning": tuning,
        "finite_outputs": fin32 and fin64,
    }

    if not args.no_fmm:
        # the same matvec with the FMM far field (the paper's own route at large M);
        # reported beside the all-pairs headline, which it does not replace
        xd64 = torch.from_numpy(x).cuda()
        y_dir = torch.zeros_like(xd64)
        ctx.apply_dev(0, xd64, y_dir)
        ctx.set_far_field(mp.FAR_FMM)
        fm = {}
        for name, prec in (("fp32", 1), ("fp64", 0)):
            dt, far_ms, _, fin = _matvec_rate(ctx, torch, prec, x, args.steps, args.warmup)
            fm[name] = {"matvecs_per_s": args.steps / dt, "ms_per_matvec": dt / args.steps * 1e3,
                        "far_field_ms": far_ms, "finite": fin}
        y_fmm = torch.zeros_like(xd64)
        ctx.apply_dev(0, xd64, y_fmm)
        torch.cuda.synchronize()
        a, b = y_fmm.cpu().numpy(), y_dir.cpu().numpy()
        fm["fp64_rel_err_vs_all_pairs"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        fm["info"] = ctx.fmm_info(1)
        ctx.set_far_field(mp.FAR_AUTO)
        out["fmm_far_field"] = fm

    if not args.no_solve:
        out["solve"] = _solve_leg(args, mp, ctx, wl, flops)
        sv = out["solve"]
        if sv["mixed"]["converged"] == sv["mixed"]["sources"] and sv["fp64"]["converged"] == sv["fp64"]["sources"]:
            out["mixed_vs_fp64_solve_speedup"] = sv["fp64"]["p50_ms"] / sv["mixed"]["p50_ms"]

    if not args.no_span:
        yc = torch.zeros_like(xd)
        ctx.apply_dev(0, xd, yc)
        torch.cuda.synchronize()
        y_count = yc.cpu().numpy()
        del ctx
        torch.cuda.empty_cache()
        out["span_contour"] = _span_leg(args, torch, mp, wl, x, y_count)
        print(f"# span legs: {json.dumps(out['span_contour'])}", file=sys.stderr, flush=True)

    if not args.no_batch:
        short = argparse.Namespace(**vars(args))
        short.steps, short.warmup = 5, 1
        out["batch"] = _batch_workload(short, torch, mp)
        print(f"# batch: {json.dumps(out['batch'])}", file=sys.stderr, flush=True)
    if not args.no_fmm20k:
        short = argparse.Namespace(**vars(args))
        short.steps = 10
        out["fmm_20000"] = _fmm_workload(short, torch, mp)
        print(f"# fmm 20000: {json.dumps(out['fmm_20000'])}", file=sys.stderr, flush=True)
    if not args.no_serve:
        # a short request stream of the serving mix with N up to 2000 (the
        # full mix: --workload serve)
        short = argparse.Namespace(**vars(args))
        short.requests, short.serve_calibration, short.serve_modes = 8, 4, "mixed,fp64"
        out["serve_short"] = _serve_workload(short, torch, mp, n_max=2000)
        print(f"# serve (short): {json.dumps(out['serve_short'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(wl, S, x)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
