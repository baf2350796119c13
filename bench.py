#!/usr/bin/env python3
"""Benchmark of the MI355X matrix-free IPM solver (one JSON line on stdout).

A step is one complete call of the hot path on inputs that already sit in
device memory: every IPM iteration with its PCG solves, residuals, step
lengths, correctors and the final x = u - v, for every instance of the call.
The default workload is the uneven dense batch: 256 independent instances in
one launch, n_i = 64 U{16..128}, m_i = n_i/4, A_i i.i.d. N(0, 1/m_i),
k_i = floor(n_i/50) N(0,1) spikes, noise sigma = 1e-3,
tau_i = 1e-2 ||A_i^T b_i||_inf; `value` is solves per second of that batch.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workloads: batched_dense (default), pdct_hdr (partial DCT n = 2^20),
grad (32 signals sharing a partial DCT, n = 2^18, forward + adjoint),
shared_dense (256 signals sharing one 2048 x 8192 dense A, FP64 MFMA),
phase (a phase-transition sweep of small partial-DCT instances),
pdct (partial DCT n = 2^16), dense (256 x 1024), wht / wht_hdr (partial
Walsh-Hadamard n = 2^16 / 2^20, with the recipes of pdct / pdct_hdr), dst
(partial DST-II n = 2^16, the pdct recipe),
direct (exact Newton directions by Cholesky, n = 4096, with the n = 2^5 ..
2^12 sweep of both variants).

Roofline: algorithmic bytes (or flops) of the timed launch divided by its
duration measured with HIP events on the library's stream (average over the
timed launches).  Per PCG iteration the method must move the vector state
(read x, r, p, Theta^{-1}; write x, r, p: 7 x 2n doubles = 112 n bytes) and
the operator's compulsory traffic (partial DCT: 16 (n + m) bytes; dense: the
matrix once, 8 m n bytes); per direction computation (IPM iteration or
corrector) and per residual evaluation it moves ten 2n-vector passes
(160 n bytes) plus one operator application.  The shared-dense workload is
bound by FP64 MFMA: 4 m n flops per signal per operator application.

cpu_baseline: the CPU oracle (plain NumPy/SciPy FP64) on a bounded sample of
the same workload, in worker processes (one host core each) forked from a
server started before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
METRIC = "l1-LS solves/sec + PCG matvec HBM GB/s (% peak), batched & grad vs plain"


def alg_bytes(kind: str, n: int, m: int, info: dict, reduced: bool = False) -> float:
    op = 16.0 * (n + m) if kind in ("pdct", "wht", "dst") else 8.0 * m * n
    vec = 56.0 * n if reduced else 112.0 * n  # reduced: x, r, p, Theta_bar^{-1} are n-vectors
    pcg = info["pcg_iters"] * (vec + op)
    ipm = (info["ipm_iters"] + info["correctors"] + 1) * (160.0 * n + op)
    return pcg + ipm


def adjoint_bytes(kind: str, n: int, m: int, info: dict, reduced: bool = False) -> float:
    op = 16.0 * (n + m) if kind in ("pdct", "wht", "dst") else 8.0 * m * n
    vec = 56.0 * n if reduced else 112.0 * n
    return info["pcg_iters"] * (vec + op) + 2 * (160.0 * n + op)


def kernel_src_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1208_5435_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("src_hash") != kernel_src_hash():
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def _counter_rows(path: str):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def write_traffic(workload: str, fetch_csv: str, write_csv: str, calib_mb: int):
    """Turns two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; each with
    --copy-calib-mb) into profiles/traffic.json: per-launch bytes of the
    solve kernel, each counter scaled by what it reads for the device copy of
    calib_mb MiB (calib_mb MiB fetched and written)."""
    rec = {"src_hash": kernel_src_hash()}
    for what, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _counter_rows(path)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        solves = [r for r in rows if "k_mfipm" in r["Kernel_Name"]]
        if not copies or not solves:
            raise SystemExit(f"{path}: no calibration copy or no solve kernel in the counter file")
        scale = (calib_mb << 20) / (max(copies) * 1024.0)
        # one step may launch several solve kernels (forward and adjoint): the
        # per-step figure is the sum over kernels of each one's mean per launch
        by_kernel = {}
        for r in solves:
            by_kernel.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        kib = sum(float(np.mean(v)) for v in by_kernel.values())
        rec[f"{what}_scale"] = scale
        rec[f"{what}_bytes_per_launch"] = kib * 1024.0 * scale
        rec[f"{what}_kib_raw_per_launch"] = kib
        rec["kernel"] = " + ".join(sorted(by_kernel))
        rec["launches"] = {k: len(v) for k, v in sorted(by_kernel.items())}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[workload] = rec
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps({workload: rec}))


def _line(value, unit, args, ms_step, config, roofline, higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": config, "roofline": roofline}


_COPY_GBS = None
_COPY_PROBE = True  # off in counter runs, whose only copy must be the calibration copy


def measured_copy_gbs():
    """Device-to-device copy rate of this GPU (1 GiB read + 1 GiB written per
    copy, best of five after a warm-up, HIP events): the achievable streaming
    bandwidth the algorithmic GB/s is also compared with."""
    global _COPY_GBS
    if not _COPY_PROBE:
        return None
    if _COPY_GBS is None:
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        best = None
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        _COPY_GBS = 2.0 * (1 << 30) / (best * 1e-3) / 1e9
        del src, dst
    return _COPY_GBS


def _hbm_roofline(ab, kernel_ms, kernel, workload):
    achieved = ab / (kernel_ms * 1e-3) / 1e9
    copy = measured_copy_gbs()
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(workload),
            "kernel": kernel, "alg_bytes_per_launch": ab, "copy_gbs": round(copy, 1) if copy else None,
            "frac_of_copy": round(achieved / copy, 4) if copy else None}


def _params(args):
    """Solver parameters of the run: the paper's defaults, or the reduced
    n x n PCG system (--reduced)."""
    return {"reduced": 1} if getattr(args, "reduced", False) else {}


def _timed(run, args, torch):
    """Warmup, then exactly args.steps timed calls between synchronisations.
    Returns (wall seconds, kernel ms per call, last result)."""
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    kms = []
    r = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = run()
        kms.append(r[1] if isinstance(r, tuple) else r.kernel_ms)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kms, r


# ----------------------------------------------------------------- CPU baselines --

def cpu_baseline_single(kind, inst, budget_s):
    """Full oracle solves of the same instance on one host core (BLAS limited
    to one thread; scipy.fft single worker), as many as fit in the budget."""
    from threadpoolctl import threadpool_limits
    from oracle import mfipm_ref as R
    if kind == "dense":
        op = R.DenseOperator(inst.A)
    elif kind == "wht":
        op = R.PartialWHTOperator(inst.n, inst.rows)
    elif kind == "dst":
        op = R.PartialDSTOperator(inst.n, inst.rows)
    else:
        op = R.PartialDCTOperator(inst.n, inst.rows)
    times = []
    with threadpool_limits(1):
        t_end = time.perf_counter() + budget_s
        while True:
            t0 = time.perf_counter()
            R.solve(op, inst.b, inst.tau)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() + times[-1] > t_end or len(times) >= 50:
                break
    from oracle import pool
    return {"value": round(len(times) / sum(times), 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host": pool.host_model(),
            "sample": f"{len(times)} full oracle solves of the same instance ({sum(times):.1f} s on one core)"}


def cpu_baseline_batched_dense(sizes, stride):
    """Every `stride`-th instance of the batch (by size) solved by the oracle
    in parallel worker processes; the rate is scaled to the whole batch by
    the sum of m n (the oracle's cost is its matrix passes)."""
    from oracle import pool
    order = np.argsort(-sizes, kind="stable")
    sample = [int(i) for i in order[::stride]]
    cores = min(pool.host_cores(), len(sample))
    with pool.executor(cores) as ex:
        pool.warm(ex, cores)
        t0 = time.perf_counter()
        res = list(ex.map(pool.time_batched_dense, sample, [int(sizes[i]) for i in sample]))
        wall = time.perf_counter() - t0
    mn = lambda n: (n // 4) * n  # noqa: E731
    full = float(sum(mn(int(n)) for n in sizes))
    part = float(sum(mn(int(sizes[i])) for i in sample))
    est = wall * full / part
    return {"value": round(len(sizes) / est, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "host": pool.host_model(),
            "sample": f"{len(sample)} of {len(sizes)} instances (every {stride}th by size, "
                      f"{part / full:.3f} of the batch's sum m*n) on {cores} worker processes: "
                      f"{wall:.1f} s wall incl. drawing each instance ({sum(r[0] for r in res):.1f} s of it); "
                      f"scaled to the batch by sum m*n",
            "oracle_ipm_iters_sample": [r[2] for r in res]}


def cpu_baseline_grad(n, batch, signals):
    from oracle import pool
    cores = min(pool.host_cores(), signals)
    with pool.executor(cores) as ex:
        pool.warm(ex, cores)
        t0 = time.perf_counter()
        res = list(ex.map(pool.time_grad_signal, range(signals), [n] * signals, [batch] * signals))
        wall = time.perf_counter() - t0
    return {"value": round(signals / wall, 4), "unit": "signals/s (forward+gradient)", "cores": cores,
            "kind": "oracle", "host": pool.host_model(),
            "sample": f"signals 0..{signals - 1} of {batch}: oracle forward solve + oracle adjoint "
                      f"(PCG to 1e-12) each, {cores} worker processes, {wall:.1f} s wall; "
                      f"forward {np.mean([r[0] for r in res]):.1f} s and adjoint "
                      f"{np.mean([r[1] for r in res]):.1f} s per signal"}


def cpu_baseline_phase(grid, stride):
    """Every `stride`-th instance of the sweep through the oracle in worker
    processes; the rate is scaled to the whole sweep by the instance count."""
    from oracle import pool
    sample = [g[3] for g in grid[::stride]]
    cores = min(pool.host_cores(), len(sample))
    with pool.executor(cores) as ex:
        pool.warm(ex, cores)
        t0 = time.perf_counter()
        res = list(ex.map(pool.time_phase_instance, sample))
        wall = time.perf_counter() - t0
    return {"value": round(len(sample) / wall, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "host": pool.host_model(),
            "sample": f"{len(sample)} of {len(grid)} instances (every {stride}th), {cores} worker processes, "
                      f"{wall:.1f} s wall, {np.mean(res):.2f} s per solve"}


def cpu_baseline_direct(n):
    """One oracle direct-variant solve of the same instance (Cholesky of the
    explicit 2n system by LAPACK), BLAS on all usable host cores, in a worker
    process."""
    from oracle import pool
    cores = pool.host_cores()
    with pool.executor(1) as ex:
        pool.warm(ex, 1)
        sec, its, status = ex.submit(pool.time_direct, n, cores).result()
    return {"value": round(1.0 / sec, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "host": pool.host_model(),
            "sample": f"1 full oracle direct solve of the same instance ({its} IPM iterations, {sec:.1f} s, "
                      f"BLAS on {cores} threads)"}


def cpu_baseline_shared_dense(batch, signals):
    from oracle import pool
    cores = min(pool.host_cores(), signals)
    with pool.executor(cores) as ex:
        pool.warm(ex, cores)
        t0 = time.perf_counter()
        res = list(ex.map(pool.time_shared_dense, range(signals), [batch] * signals))
        wall = time.perf_counter() - t0
    return {"value": round(signals / wall, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "host": pool.host_model(),
            "sample": f"signals 0..{signals - 1} of {batch} (each worker draws A and its signal, then "
                      f"solves): {cores} worker processes, {wall:.1f} s wall, "
                      f"{np.mean([r[0] for r in res]):.1f} s per solve"}


# ------------------------------------------------------------------ workloads --

def make_single(name: str):
    import workloads as W
    if name == "pdct":
        inst = W.config_pdct()
        return "pdct", inst, f"pdct_n{inst.n}_m{inst.m}_k{inst.n // 100}"
    if name == "pdct_hdr":
        inst = W.config_pdct_hdr()
        return "pdct", inst, f"pdct_hdr_n{inst.n}_m{inst.m}_k{inst.n // 200}"
    if name == "dst":
        inst = W.config_dst()
        return "dst", inst, f"dst_n{inst.n}_m{inst.m}_k{inst.n // 100}"
    if name == "wht":
        inst = W.config_wht()
        return "wht", inst, f"wht_n{inst.n}_m{inst.m}_k{inst.n // 100}"
    if name == "wht_hdr":
        inst = W.config_wht_hdr()
        return "wht", inst, f"wht_hdr_n{inst.n}_m{inst.m}_k{inst.n // 200}"
    if name == "dense":
        inst = W.config_dense_256x1024()
        return "dense", inst, "dense_256x1024_k20"
    raise SystemExit(f"unknown workload {name}")


def bench_single(args, torch, Solver):
    kind, inst, wl = make_single(args.workload)
    wl += "_reduced" if args.reduced else ""
    dev = torch.device("cuda", 0)
    solver = Solver(device=dev, params=_params(args))
    try:
        solver.set_launch(args.workgroups, 0, args.tile)
        b = torch.from_numpy(inst.b).to(dev)
        if kind == "dense":
            A = torch.from_numpy(inst.A).to(dev)
            call = lambda: solver.solve(b, inst.tau, A=A)  # noqa: E731
        else:
            rows = torch.from_numpy(inst.rows).to(dev)
            call = lambda: solver.solve(b, inst.tau, rows=rows, n=inst.n, transform=inst.transform)  # noqa: E731
        _calibration_copy(args, torch, dev)
        wall, kms, r = _timed(call, args, torch)
    finally:
        solver.close()
    info = r.infos[0]
    if info["status"] != 0:
        print(f"bench.py: solve did not converge: {info}", file=sys.stderr)
    n, m = inst.n, inst.m
    kms_mean = float(np.mean(kms))
    cfg = {"workload": wl, "n": n, "m": m, "tau": inst.tau, "tol": 1e-8, "tolpcg": 1e-2, "reduced": int(args.reduced),
           "ipm_iters": info["ipm_iters"], "pcg_iters": info["pcg_iters"], "correctors": info["correctors"],
           "nmat": info["nmat"], "rel_gap": info["rel_gap"], "kernel_ms_mean": round(kms_mean, 4),
           "kernel_ms_min": round(float(np.min(kms)), 4)}
    kern = {"pdct": "k_mfipm<OpPdct,0>", "dst": "k_mfipm<OpPdct,0>", "wht": "k_mfipm<OpWht,0>",
            "dense": "k_mfipm<OpDense,0>"}[kind]
    out = _line(round(args.steps / wall, 3), "solves/s", args, 1e3 * wall / args.steps, cfg,
                _hbm_roofline(alg_bytes(kind, n, m, info, args.reduced), kms_mean, kern, wl))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_single(kind, inst, args.cpu_seconds)
    return out


def _calibration_copy(args, torch, dev):
    if args.copy_calib_mb > 0:
        src = torch.empty(args.copy_calib_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def batched_dense_inputs(args, torch):
    import workloads as W
    from concurrent.futures import ThreadPoolExecutor
    sizes = W.batched_dense_sizes(batch=args.batch)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:
        insts = list(ex.map(lambda iv: W.batched_dense_instance(iv[0], int(iv[1])), enumerate(sizes)))
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    n_off = np.concatenate([[0], np.cumsum([i.n for i in insts])]).astype(np.int64)
    m_off = np.concatenate([[0], np.cumsum([i.m for i in insts])]).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum([i.m * i.n for i in insts])]).astype(np.int64)
    A = torch.empty(int(a_off[-1]), dtype=torch.float64, device=dev)
    for j, i in enumerate(insts):
        A[a_off[j]:a_off[j + 1]].copy_(torch.from_numpy(i.A.reshape(-1)))
    b = torch.from_numpy(np.concatenate([i.b for i in insts])).to(dev)
    taus = np.array([i.tau for i in insts])
    return sizes, insts, gen_s, dev, n_off, m_off, a_off, A, b, taus


def bench_batched_dense(args, torch, Solver):
    """The uneven dense batch in one launch, against one launch per instance."""
    sizes, insts, gen_s, dev, n_off, m_off, a_off, A, b, taus = batched_dense_inputs(args, torch)
    del insts
    solver = Solver(device=dev, params=_params(args))
    try:
        solver.set_launch(args.workgroups, args.team, args.tile)
        run = lambda: solver.solve_batched(b, taus, n_off, m_off, A_packed=A, a_off=a_off)  # noqa: E731
        _calibration_copy(args, torch, dev)
        wall, kms, r = _timed(run, args, torch)
        infos = r.infos
        plain = None
        if not args.no_plain:
            solver.set_launch(0, 0, args.tile)
            t1 = time.perf_counter()
            plain_iters = 0
            for j in range(len(sizes)):
                nj, mj = int(n_off[j + 1] - n_off[j]), int(m_off[j + 1] - m_off[j])
                rr = solver.solve(b[m_off[j]:m_off[j + 1]], float(taus[j]),
                                  A=A[a_off[j]:a_off[j + 1]].view(mj, nj))
                plain_iters += rr.infos[0]["ipm_iters"]
            torch.cuda.synchronize()
            plain = (time.perf_counter() - t1, plain_iters)
    finally:
        solver.close()
    B = len(sizes)
    bad = [k for k, i in enumerate(infos) if i["status"] != 0]
    ab = sum(alg_bytes("dense", int(n_off[j + 1] - n_off[j]), int(m_off[j + 1] - m_off[j]), infos[j])
             for j in range(B))
    kms_mean = float(np.mean(kms))
    value = B * args.steps / wall
    wl = f"batched_dense_{B}_n64x16-128_m=n/4"
    cfg = {"workload": wl, "batch": B, "sum_mn": int(a_off[-1]), "gen_s": round(gen_s, 1),
           "not_converged": bad, "ipm_iters_sum": sum(i["ipm_iters"] for i in infos),
           "pcg_iters_sum": sum(i["pcg_iters"] for i in infos), "kernel_ms_mean": round(kms_mean, 3)}
    if plain:
        cfg.update({"plain_solves_per_s": round(B / plain[0], 3), "plain_ipm_iters_sum": plain[1],
                    "batched_over_plain": round(value / (B / plain[0]), 3)})
    out = _line(round(value, 3), "solves/s", args, 1e3 * wall / args.steps, cfg,
                _hbm_roofline(ab, kms_mean, "k_mfipm<OpDense,0>", wl))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched_dense(sizes, stride=8)
    return out


def bench_grad(args, torch, Solver):
    """32 signals sharing a partial DCT: batched forward + adjoint, against
    one forward and one adjoint launch per signal."""
    import workloads as W
    B = args.batch if args.batch != 256 else 32
    inst = W.config_dct_batch(n=args.grad_n, batch=B)
    dev = torch.device("cuda", 0)
    m = inst.m
    n = inst.n
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    rows = torch.from_numpy(inst.rows).to(dev)
    b = torch.from_numpy(inst.b.reshape(-1)).to(dev)
    xt = torch.from_numpy(inst.x_true.reshape(-1)).to(dev)
    solver = Solver(device=dev, params=_params(args))
    try:
        solver.set_launch(args.workgroups, args.team, args.tile)

        def fwd_bwd():
            r = solver.solve_batched(b, inst.tau, n_off, m_off, rows=rows, shared_op=True)
            f_ms = r.kernel_ms
            gb, gt, binf = solver.backward(r.state, r.x - xt, n_off, m_off, rows=rows, shared_op=True)
            return (r, f_ms, solver.last_kernel_ms(), binf)
        _calibration_copy(args, torch, dev)
        for _ in range(args.warmup):
            fwd_bwd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fms, bms = [], []
        for _ in range(args.steps):
            r, f_ms, b_ms, binf = fwd_bwd()
            fms.append(f_ms)
            bms.append(b_ms)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        plain_s = None
        if not args.no_plain:
            solver.set_launch(0, 0, args.tile)
            one = np.array([0, n], np.int64)
            onem = np.array([0, m], np.int64)
            t1 = time.perf_counter()
            for j in range(B):
                rj = solver.solve(b[j * m:(j + 1) * m], float(inst.tau[j]), rows=rows, n=n)
                solver.backward(rj.state, rj.x - xt[j * n:(j + 1) * n], one, onem, rows=rows)
            torch.cuda.synchronize()
            plain_s = time.perf_counter() - t1
    finally:
        solver.close()
    infos = r.infos
    ab_f = sum(alg_bytes("pdct", n, m, i, args.reduced) for i in infos)
    ab_b = sum(adjoint_bytes("pdct", n, m, i, args.reduced) for i in binf)
    f_mean, b_mean = float(np.mean(fms)), float(np.mean(bms))
    value = B * args.steps / wall
    wl = f"grad_pdct_batch{B}_n{n}_m{m}" + ("_reduced" if args.reduced else "")
    cfg = {"workload": wl, "forward_kernel_ms": round(f_mean, 3), "backward_kernel_ms": round(b_mean, 3),
           "ipm_iters": [i["ipm_iters"] for i in infos], "adjoint_pcg_iters": [i["pcg_iters"] for i in binf],
           "not_converged": [j for j, i in enumerate(infos) if i["status"] != 0],
           "adjoint_status": sorted({i["status"] for i in binf})}
    if plain_s:
        cfg.update({"plain_signals_per_s": round(B / plain_s, 3),
                    "batched_over_plain": round(value / (B / plain_s), 3)})
    roof = _hbm_roofline(ab_f + ab_b, f_mean + b_mean, "k_mfipm<OpPdct,0> + k_mfipm<OpPdct,1>", wl)
    out = _line(round(value, 3), "signals/s (forward+gradient)", args, 1e3 * wall / args.steps, cfg, roof)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_grad(n, B, min(16, B))
    return out


def bench_shared_dense(args, torch, Solver):
    """256 signals sharing one 2048 x 8192 dense A in one lock-step launch
    (operator = two FP64 MFMA matrix products per round), against one launch
    per signal on the same A."""
    import workloads as W
    B = args.batch
    inst = W.config_shared_dense(batch=B)
    dev = torch.device("cuda", 0)
    m, n = inst.m, inst.n
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    A = torch.from_numpy(inst.A).to(dev)
    b = torch.from_numpy(inst.b.reshape(-1)).to(dev)
    solver = Solver(device=dev, params=_params(args))
    try:
        solver.set_launch(args.workgroups, 0, 0)
        run = lambda: solver.solve_batched(b, inst.tau, n_off, m_off, A_packed=A, shared_op=True)  # noqa: E731
        _calibration_copy(args, torch, dev)
        wall, kms, r = _timed(run, args, torch)
        plain = None
        if not args.no_plain:
            solver.set_launch(0, 0, 0)
            t1 = time.perf_counter()
            for j in range(B):
                solver.solve(b[j * m:(j + 1) * m], float(inst.tau[j]), A=A)
            torch.cuda.synchronize()
            plain = time.perf_counter() - t1
    finally:
        solver.close()
    infos = r.infos
    kms_mean = float(np.mean(kms))
    flops = sum(2.0 * m * n * i["nmat"] for i in infos)  # each product with A or A^T: 2 m n
    achieved = flops / (kms_mean * 1e-3) / 1e12
    value = B * args.steps / wall
    wl = f"shared_dense_{B}_m{m}_n{n}"
    cfg = {"workload": wl, "batch": B, "m": m, "n": n, "kernel_ms_mean": round(kms_mean, 3),
           "not_converged": [j for j, i in enumerate(infos) if i["status"] != 0],
           "ipm_iters": [min(i["ipm_iters"] for i in infos), max(i["ipm_iters"] for i in infos)],
           "nmat_max": max(i["nmat"] for i in infos), "nmat_sum": sum(i["nmat"] for i in infos)}
    if plain:
        cfg.update({"plain_solves_per_s": round(B / plain, 3), "batched_over_plain": round(value / (B / plain), 3)})
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": counter_traffic(wl),
            "kernel": "k_mfipm_lockstep", "alg_flops_per_launch": flops}
    out = _line(round(value, 3), "solves/s", args, 1e3 * wall / args.steps, cfg, roof)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_shared_dense(B, 16)
    return out


def direct_flops(n: int, m: int, info: dict) -> float:
    """Algorithmic flops of one direct-variant solve: K = A^T A once (its
    lower half, m n^2), a Cholesky factorisation per IPM iteration (n^3 / 3),
    two triangular sweeps per Newton direction (2 n^2), and the residuals'
    products with A and A^T (2 m n each)."""
    return (m * n * n + info["ipm_iters"] * n ** 3 / 3.0 + (info["ipm_iters"] + info["correctors"]) * 2.0 * n * n
            + info["nmat"] * 2.0 * m * n)


def bench_direct(args, torch, Solver):
    """The direct-solver variant (Section 5.7): the Gaussian, noiseless,
    tau = 1e-3 problem with n = 4096, m = 1024 solved with exact Newton
    directions (Cholesky of the n x n system on FP64 MFMA), plus the paper's
    size sweep n = 2^5 .. 2^12 with both variants (time and IPM iterations)."""
    import workloads as W
    dev = torch.device("cuda", 0)
    n = args.direct_n
    inst = W.direct_scaling_instance(n)
    m = inst.m
    A = torch.from_numpy(inst.A).to(dev)
    b = torch.from_numpy(inst.b).to(dev)
    sd = Solver(device=dev, params={**_params(args), "direct": 1})
    sp = Solver(device=dev, params=_params(args))
    sweep = []
    try:
        run = lambda: sd.solve(b, inst.tau, A=A)  # noqa: E731
        _calibration_copy(args, torch, dev)
        wall, kms, r = _timed(run, args, torch)
        if not args.no_plain:
            for nn in W.DIRECT_SCALING_NS:
                q = W.direct_scaling_instance(nn)
                Aq = torch.from_numpy(q.A).to(dev)
                bq = torch.from_numpy(q.b).to(dev)
                row = {"n": nn, "m": q.m}
                for name, s in (("direct", sd), ("pcg", sp)):
                    s.solve(bq, q.tau, A=Aq)
                    rr = s.solve(bq, q.tau, A=Aq)
                    i = rr.infos[0]
                    row[name] = {"ms": round(rr.kernel_ms, 3), "ipm_iters": i["ipm_iters"],
                                 "pcg_iters": i["pcg_iters"], "status": i["status_name"]}
                sweep.append(row)
    finally:
        sd.close()
        sp.close()
    info = r.infos[0]
    if info["status"] != 0:
        print(f"bench.py: direct solve did not converge: {info}", file=sys.stderr)
    kms_mean = float(np.mean(kms))
    flops = direct_flops(n, m, info)
    achieved = flops / (kms_mean * 1e-3) / 1e12
    wl = f"direct_n{n}_m{m}"
    cfg = {"workload": wl, "n": n, "m": m, "tau": inst.tau, "tol": 1e-8, "direct": 1,
           "ipm_iters": info["ipm_iters"], "correctors": info["correctors"], "rel_gap": info["rel_gap"],
           "kernel_ms_mean": round(kms_mean, 3), "sweep_n_2e5_to_2e12": sweep}
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": counter_traffic(wl),
            "kernel": "k_mfipm<OpDenseDirect,0>", "alg_flops_per_launch": flops}
    out = _line(round(args.steps / wall, 3), "solves/s", args, 1e3 * wall / args.steps, cfg, roof)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_direct(n)
    return out


def bench_phase(args, torch, Solver):
    """The average phase-transition sweep (noiseless partial DCT, n = 1024,
    delta = m/n in 0.1..0.9, rho = k/m in 0.05..0.95, +-1 spikes) as one
    batched launch of many small instances, each with its own rows."""
    import workloads as W
    grid = W.phase_transition_grid(trials=args.phase_trials)
    insts = [g[3] for g in grid]
    B, n = len(insts), insts[0].n
    dev = torch.device("cuda", 0)
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.concatenate([[0], np.cumsum([i.m for i in insts])]).astype(np.int64)
    rows = torch.from_numpy(np.concatenate([i.rows for i in insts])).to(dev)
    b = torch.from_numpy(np.concatenate([i.b for i in insts])).to(dev)
    taus = np.array([i.tau for i in insts])
    solver = Solver(device=dev, params={**W.PHASE_PARAMS, **_params(args)})
    try:
        solver.set_launch(args.workgroups, args.team, args.tile)
        run = lambda: solver.solve_batched(b, taus, n_off, m_off, rows=rows)  # noqa: E731
        _calibration_copy(args, torch, dev)
        wall, kms, r = _timed(run, args, torch)
    finally:
        solver.close()
    x = r.x.cpu().numpy().reshape(B, n)
    re = [float(np.linalg.norm(x[j] - insts[j].x_true) / np.linalg.norm(insts[j].x_true)) for j in range(B)]
    rate = {}
    for (d, rho, _, _), e in zip(grid, re):
        rate.setdefault(d, {}).setdefault(rho, []).append(e <= 1e-5)
    transition = {str(d): max([rho for rho, v in sorted(rs.items()) if np.mean(v) >= 0.5], default=0.0)
                  for d, rs in rate.items()}
    infos = r.infos
    kms_mean = float(np.mean(kms))
    ab = sum(alg_bytes("pdct", n, insts[j].m, infos[j], args.reduced) for j in range(B))
    value = B * args.steps / wall
    wl = f"phase_transition_pdct_n{n}_{B}"
    statuses = {}
    for i in infos:
        statuses[i["status_name"]] = statuses.get(i["status_name"], 0) + 1
    cfg = {"workload": wl, "batch": B, "n": n, "trials": args.phase_trials, "tol": W.PHASE_PARAMS["tol"],
           "tolpcg": W.PHASE_PARAMS["tolpcg"], "c_tau": W.PHASE_C_TAU, "kernel_ms_mean": round(kms_mean, 3),
           "statuses": statuses, "rho_50pct_by_delta": transition}
    out = _line(round(value, 3), "solves/s", args, 1e3 * wall / args.steps, cfg,
                _hbm_roofline(ab, kms_mean, "k_mfipm<OpPdct,0>", wl))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_phase(grid, stride=20)
    return out


def tune_workload(args, torch, Solver):
    """Autotunes the launch shape of one workload (forward, and backward for
    the gradient batch) and writes it to the package's shipped table."""
    from paper_1208_5435_amd import autotune
    dev = torch.device("cuda", 0)
    solver = Solver(device=dev, params=_params(args))
    out = args.tune_out or autotune.SHIPPED
    jobs = []
    if args.workload in ("pdct", "pdct_hdr", "wht", "wht_hdr", "dst", "dense"):
        kind, inst, _ = make_single(args.workload)
        b = torch.from_numpy(inst.b).to(dev)
        if kind == "dense":
            A = torch.from_numpy(inst.A).to(dev)
            call = lambda: solver.solve(b, inst.tau, A=A)  # noqa: E731
            op = 0
        else:
            rows = torch.from_numpy(inst.rows).to(dev)
            call = lambda: solver.solve(b, inst.tau, rows=rows, n=inst.n, transform=inst.transform)  # noqa: E731
            op = {"wht": 2, "dst": 3}.get(kind, 1)
        jobs.append((solver.tune_key(op, inst.n, inst.m, 1, True), call,
                     autotune.candidates(op, inst.n, inst.m, 1, solver.num_cu)))
    elif args.workload == "grad":
        import workloads as W
        inst = W.config_dct_batch(n=args.grad_n, batch=32)
        B, m = inst.b.shape
        n_off = np.arange(B + 1, dtype=np.int64) * inst.n
        m_off = np.arange(B + 1, dtype=np.int64) * m
        rows = torch.from_numpy(inst.rows).to(dev)
        b = torch.from_numpy(inst.b.reshape(-1)).to(dev)
        xt = torch.from_numpy(inst.x_true.reshape(-1)).to(dev)
        res = solver.solve_batched(b, inst.tau, n_off, m_off, rows=rows, shared_op=True)
        fwd = lambda: solver.solve_batched(b, inst.tau, n_off, m_off, rows=rows, shared_op=True)  # noqa: E731
        bwd = lambda: solver.backward(res.state, res.x - xt, n_off, m_off, rows=rows, shared_op=True)  # noqa
        cands = autotune.candidates(1, inst.n, m, B, solver.num_cu)
        jobs.append((solver.tune_key(1, inst.n, m, B, True), fwd, cands))
        jobs.append((solver.tune_key(1, inst.n, m, B, True, backward=True), bwd, cands))
    elif args.workload == "batched_dense":
        sizes, insts, _, _, n_off, m_off, a_off, A, b, taus = batched_dense_inputs(args, torch)
        call = lambda: solver.solve_batched(b, taus, n_off, m_off, A_packed=A, a_off=a_off)  # noqa: E731
        nmax = int(np.diff(n_off).max())
        mmax = int(np.diff(m_off).max())
        jobs.append((solver.tune_key(0, nmax, mmax, len(insts), False), call,
                     autotune.candidates(0, nmax, mmax, len(insts), solver.num_cu)))
    else:
        raise SystemExit("--tune supports pdct, pdct_hdr, wht, wht_hdr, dense, batched_dense, grad")
    try:
        for key, call, cands in jobs:
            best, ms, table = autotune.tune(solver, call, key, cands, reps=3, path=out, verbose=True)
            print(json.dumps({"key": key, "best": best, "kernel_ms": ms,
                              "table": [[list(s), round(t, 4)] for s, t in table]}), flush=True)
    finally:
        solver.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched_dense",
                    choices=["batched_dense", "pdct_hdr", "grad", "shared_dense", "phase", "pdct", "dense", "wht",
                             "wht_hdr", "dst", "direct"])
    ap.add_argument("--direct-n", type=int, default=4096, help="n of the direct workload (m = n/4)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--grad-n", type=int, default=1 << 18)
    ap.add_argument("--phase-trials", type=int, default=10)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the one-launch-per-instance comparison (profiling runs)")
    ap.add_argument("--reduced", action="store_true",
                    help="PCG on the reduced n x n system (half the vector traffic per PCG iteration)")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch shape of this workload and record it in the shipped table")
    ap.add_argument("--tune-out", default=None, help="tuning table to write (default: the shipped one)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="write profiles/traffic.json for --workload from two rocprofv3 counter files "
                         "(needs --copy-calib-mb as used in those runs); runs nothing on the GPU")
    ap.add_argument("--traffic-key", default=None, help="workload key for --traffic-from")
    args = ap.parse_args()
    global _COPY_PROBE
    _COPY_PROBE = args.copy_calib_mb <= 0
    if args.traffic_from:
        write_traffic(args.traffic_key or args.workload, args.traffic_from[0], args.traffic_from[1],
                      args.copy_calib_mb)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(instances shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        raise SystemExit(2)
    if not args.no_cpu_baseline:
        from oracle import pool
        pool.start()  # worker server forked before any GPU call

    import torch
    from paper_1208_5435_amd import Solver

    torch.cuda.set_device(0)
    if args.tune:
        tune_workload(args, torch, Solver)
        return
    fn = {"batched_dense": bench_batched_dense, "grad": bench_grad, "shared_dense": bench_shared_dense,
          "phase": bench_phase, "direct": bench_direct}.get(args.workload, bench_single)
    out = fn(args, torch, Solver)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
