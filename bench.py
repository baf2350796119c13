#!/usr/bin/env python3
"""Benchmark of the MI355X matrix-free IPM solver (one JSON line on stdout).

A step is one complete solve (every IPM iteration with its PCG solves,
residuals, step lengths, correctors) of one synthetic instance whose inputs
already sit in device memory.  The default workload is the partial DCT with
n = 2^16, m = n/4, k = floor(n/100) N(0,1) spikes, noise sigma = 1e-2,
tau = 1e-2 ||A^T b||_inf.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Roofline: algorithmic bytes of one solve launch divided by the kernel's
duration measured with HIP events on the library's stream (average over
the timed launches).  Per PCG iteration the method must move the vector
state (read x, r, p, Theta^{-1}; write x, r, p: 7 * 2n doubles = 112 n
bytes) and the operator's compulsory traffic (partial DCT: 16 (n + m) bytes;
dense: the matrix once, 8 m n bytes); per direction computation (IPM
iteration or corrector) and per residual evaluation it moves ten 2n-vector
passes (160 n bytes) plus one operator application.

cpu_baseline: the CPU oracle (plain NumPy/SciPy FP64) timed on the host on
a bounded sample of the same workload.
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
METRIC = "l1-LS solves/sec + PCG matvec HBM GB/s (% peak), batched & grad vs plain"


def alg_bytes(kind: str, n: int, m: int, info: dict) -> float:
    op = 16.0 * (n + m) if kind == "pdct" else 8.0 * m * n
    pcg = info["pcg_iters"] * (112.0 * n + op)
    ipm = (info["ipm_iters"] + info["correctors"] + 1) * (160.0 * n + op)
    return pcg + ipm


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
        per_launch = float(np.mean([float(r["Counter_Value"]) for r in solves])) * 1024.0 * scale
        rec[f"{what}_scale"] = scale
        rec[f"{what}_bytes_per_launch"] = per_launch
        rec[f"{what}_kib_raw_per_launch"] = float(np.mean([float(r["Counter_Value"]) for r in solves]))
        rec["kernel"] = solves[0]["Kernel_Name"]
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


def make_workload(name: str):
    import workloads as W
    if name == "pdct":
        inst = W.config_pdct()
        return "pdct", inst, f"pdct_n{inst.n}_m{inst.m}_k{inst.n // 100}"
    if name == "pdct_hdr":
        inst = W.config_pdct_hdr()
        return "pdct", inst, f"pdct_hdr_n{inst.n}_m{inst.m}_k{inst.n // 200}"
    if name == "dense":
        inst = W.config_dense_256x1024()
        return "dense", inst, "dense_256x1024_k20"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(kind, inst, budget_s: float):
    """Times the oracle on the host: as many full solves of the same instance
    as fit in the budget (at least one)."""
    from oracle import mfipm_ref as R
    op = R.DenseOperator(inst.A) if kind == "dense" else R.PartialDCTOperator(inst.n, inst.rows)
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        R.solve(op, inst.b, inst.tau)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() + times[-1] > t_end or len(times) >= 50:
            break
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    cores = 1 if kind == "pdct" else int(blas_threads)
    return {"value": round(len(times) / sum(times), 4), "unit": "solves/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{len(times)} full oracle solves of the same instance "
                      f"({sum(times):.1f} s of host time; scipy.fft single worker, numpy elementwise)"}


def _pool_map(fn, items, workers=16):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def batched_dense_inputs(args, torch):
    import workloads as W
    sizes = W.batched_dense_sizes(batch=args.batch)
    t0 = time.perf_counter()
    insts = _pool_map(lambda iv: W.batched_dense_instance(iv[0], int(iv[1])), list(enumerate(sizes)))
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
    return insts, gen_s, dev, n_off, m_off, a_off, A, b, taus


def bench_batched_dense(args, torch, Solver):
    """256 uneven dense instances in one launch vs one launch per instance."""
    insts, gen_s, dev, n_off, m_off, a_off, A, b, taus = batched_dense_inputs(args, torch)
    solver = Solver(device=dev)
    solver.set_launch(args.workgroups, args.team, args.tile)
    run = lambda: solver.solve_batched(b, taus, n_off, m_off, A_packed=A, a_off=a_off)  # noqa: E731
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    kms, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        r = run()
        kms.append(r.kernel_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = r.infos
    bad = [k for k, i in enumerate(infos) if i["status"] != 0]
    ab = sum(alg_bytes("dense", int(n_off[j + 1] - n_off[j]), int(m_off[j + 1] - m_off[j]), infos[j])
             for j in range(len(insts)))
    # plain: one launch per instance, same parameters
    solver.set_launch(0, 0, args.tile)
    t1 = time.perf_counter()
    plain_iters = 0
    for j, i in enumerate(insts):
        rr = solver.solve(b[m_off[j]:m_off[j + 1]], i.tau,
                          A=A[a_off[j]:a_off[j + 1]].view(i.m, i.n))
        plain_iters += rr.infos[0]["ipm_iters"]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    kms_mean = float(np.mean(kms))
    achieved = ab / (kms_mean * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": round(len(insts) * args.steps / wall, 3), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched_dense_{len(insts)}_n64x16-128_m=n/4",
                   "batch": len(insts), "sum_mn": int(a_off[-1]), "gen_s": round(gen_s, 1),
                   "not_converged": bad, "ipm_iters_sum": sum(i["ipm_iters"] for i in infos),
                   "plain_ipm_iters_sum": plain_iters,
                   "kernel_ms_mean": round(kms_mean, 3),
                   "plain_solves_per_s": round(len(insts) / plain_s, 3),
                   "batched_over_plain": round((len(insts) * args.steps / wall) / (len(insts) / plain_s), 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_mfipm<OpDense,0>", "alg_bytes_per_launch": ab},
    }


def bench_grad(args, torch, Solver):
    """32 signals sharing a partial DCT: batched forward + adjoint vs per-signal calls."""
    import workloads as W
    inst = W.config_dct_batch(n=args.grad_n, batch=args.batch if args.batch != 256 else 32)
    dev = torch.device("cuda", 0)
    B, m = inst.b.shape
    n = inst.n
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    rows = torch.from_numpy(inst.rows).to(dev)
    b = torch.from_numpy(inst.b.reshape(-1)).to(dev)
    xt = torch.from_numpy(inst.x_true.reshape(-1)).to(dev)
    solver = Solver(device=dev)
    solver.set_launch(args.workgroups, args.team, args.tile)

    def fwd_bwd():
        r = solver.solve_batched(b, inst.tau, n_off, m_off, rows=rows, shared_op=True)
        f_ms = r.kernel_ms
        gb, gt, binf = solver.backward(r.state, r.x - xt, n_off, m_off, rows=rows, shared_op=True)
        return r, f_ms, solver.last_kernel_ms(), binf
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
    # plain: one forward + one adjoint launch per signal
    solver.set_launch(0, 0, args.tile)
    one = np.array([0, n], np.int64)
    onem = np.array([0, m], np.int64)
    t1 = time.perf_counter()
    for j in range(B):
        rj = solver.solve(b[j * m:(j + 1) * m], float(inst.tau[j]), rows=rows, n=n)
        solver.backward(rj.state, rj.x - xt[j * n:(j + 1) * n], one, onem, rows=rows)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    infos = r.infos
    ab_f = sum(alg_bytes("pdct", n, m, i) for i in infos)
    ab_b = sum(binf[j]["pcg_iters"] * (112.0 * n + 16.0 * (n + m)) + 2 * (160.0 * n + 16.0 * (n + m))
               for j in range(B))
    f_mean, b_mean = float(np.mean(fms)), float(np.mean(bms))
    achieved = (ab_f + ab_b) / ((f_mean + b_mean) * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": round(B * args.steps / wall, 3), "unit": "signals/s (forward+gradient)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"grad_pdct_batch{B}_n{n}_m{m}", "forward_kernel_ms": round(f_mean, 3),
                   "backward_kernel_ms": round(b_mean, 3),
                   "ipm_iters": [i["ipm_iters"] for i in infos],
                   "adjoint_pcg_iters": [i["pcg_iters"] for i in binf],
                   "plain_signals_per_s": round(B / plain_s, 3),
                   "batched_over_plain": round((B * args.steps / wall) / (B / plain_s), 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_mfipm<OpPdct,0> + k_mfipm<OpPdct,1>",
                     "alg_bytes_per_launch": ab_f + ab_b},
    }


def tune_workload(args, torch, Solver):
    """Autotunes the launch shape of one workload (forward, and backward for
    the gradient batch) and writes it to the package's shipped table."""
    from paper_1208_5435_amd import autotune
    dev = torch.device("cuda", 0)
    solver = Solver(device=dev)
    out = args.tune_out or autotune.SHIPPED
    jobs = []
    if args.workload in ("pdct", "pdct_hdr", "dense"):
        kind, inst, _ = make_workload(args.workload)
        b = torch.from_numpy(inst.b).to(dev)
        if kind == "dense":
            A = torch.from_numpy(inst.A).to(dev)
            call = lambda: solver.solve(b, inst.tau, A=A)  # noqa: E731
            op = 0
        else:
            rows = torch.from_numpy(inst.rows).to(dev)
            call = lambda: solver.solve(b, inst.tau, rows=rows, n=inst.n)  # noqa: E731
            op = 1
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
        insts, _, _, n_off, m_off, a_off, A, b, taus = batched_dense_inputs(args, torch)
        call = lambda: solver.solve_batched(b, taus, n_off, m_off, A_packed=A, a_off=a_off)  # noqa: E731
        nmax = int(np.diff(n_off).max())
        mmax = int(np.diff(m_off).max())
        jobs.append((solver.tune_key(0, nmax, mmax, len(insts), False), call,
                     autotune.candidates(0, nmax, mmax, len(insts), solver.num_cu)))
    else:
        raise SystemExit("--tune supports pdct, pdct_hdr, dense, batched_dense, grad")
    for key, call, cands in jobs:
        best, ms, table = autotune.tune(solver, call, key, cands, reps=3, path=out, verbose=True)
        print(json.dumps({"key": key, "best": best, "kernel_ms": ms,
                          "table": [[list(s), round(t, 4)] for s, t in table]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pdct",
                    choices=["pdct", "pdct_hdr", "dense", "batched_dense", "grad"])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--grad-n", type=int, default=1 << 18)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(make_workload(args.workload)[2], args.traffic_from[0], args.traffic_from[1],
                      args.copy_calib_mb)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(instances shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_1208_5435_amd import Solver

    if args.tune:
        tune_workload(args, torch, Solver)
        return
    if args.workload in ("batched_dense", "grad"):
        fn = bench_batched_dense if args.workload == "batched_dense" else bench_grad
        print(json.dumps(fn(args, torch, Solver)), flush=True)
        return
    kind, inst, wl = make_workload(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    solver = Solver(device=dev)
    solver.set_launch(args.workgroups, 0, args.tile)
    b = torch.from_numpy(inst.b).to(dev)
    if kind == "dense":
        A = torch.from_numpy(inst.A).to(dev)
        call = lambda: solver.solve(b, inst.tau, A=A)  # noqa: E731
        n, m = inst.n, inst.m
    else:
        rows = torch.from_numpy(inst.rows).to(dev)
        call = lambda: solver.solve(b, inst.tau, rows=rows, n=inst.n)  # noqa: E731
        n, m = inst.n, inst.m
    if args.copy_calib_mb > 0:
        src = torch.empty(args.copy_calib_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    kms = []
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = call()
        kms.append(r.kernel_ms)
        infos.append(r.infos[0])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = infos[-1]
    if info["status"] != 0:
        print(f"bench.py: solve did not converge: {info}", file=sys.stderr)
    ms_step = 1e3 * wall / args.steps
    kms_mean = float(np.mean(kms))
    ab = alg_bytes(kind, n, m, info)
    achieved = ab / (kms_mean * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(args.steps / wall, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl, "n": n, "m": m, "tau": inst.tau, "tol": solver.params.tol,
                   "tolpcg": solver.params.tolpcg, "ipm_iters": info["ipm_iters"],
                   "pcg_iters": info["pcg_iters"], "correctors": info["correctors"], "nmat": info["nmat"],
                   "rel_gap": info["rel_gap"], "kernel_ms_mean": round(kms_mean, 4),
                   "kernel_ms_min": round(float(np.min(kms)), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(wl),
                     "kernel": "k_mfipm<OpPdct,0>" if kind == "pdct" else "k_mfipm<OpDense,0>",
                     "alg_bytes_per_launch": ab},
    }
    solver.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(kind, inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
