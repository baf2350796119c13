"""Process pool that runs the CPU oracle on many instances at once.

TEST INFRASTRUCTURE, like the rest of this package: only the test suite and
the CPU-baseline leg of the benchmark use it.  Workers are forked from a
multiprocessing forkserver that the caller starts (`start()`) before it
touches the GPU, so no worker inherits device state and nothing is exec'd
from a process that holds it.  Every worker limits its BLAS to one thread, so
`workers` processes use `workers` host cores.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time
from concurrent.futures import ProcessPoolExecutor

_CTX = None


def start():
    """Starts the forkserver now (call before the first GPU call)."""
    global _CTX
    if _CTX is None:
        _CTX = mp.get_context("forkserver")
        _CTX.set_forkserver_preload(["numpy", "scipy.fft", "oracle.mfipm_ref", "workloads"])
        from multiprocessing import forkserver
        forkserver.ensure_running()
    return _CTX


def host_cores(cap: int = 16) -> int:
    """Usable host cores (affinity), at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def host_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def executor(workers: int | None = None) -> ProcessPoolExecutor:
    ctx = start()
    return ProcessPoolExecutor(max_workers=workers or host_cores(), mp_context=ctx, initializer=_init_worker)


def _ready(_):
    import oracle.mfipm_ref  # noqa: F401
    import workloads  # noqa: F401
    time.sleep(0.2)
    return os.getpid()


def warm(ex: ProcessPoolExecutor, workers: int):
    """Starts every worker of `ex` before a timed map."""
    list(ex.map(_ready, range(workers)))


# --- timing tasks (CPU baseline) ---------------------------------------------------

def time_batched_dense(i: int, n: int):
    """Draws instance i of the uneven dense batch and solves it with the
    oracle.  Returns (generation s, solve s, IPM iterations, status)."""
    import workloads as W
    from oracle import mfipm_ref as R
    t0 = time.perf_counter()
    inst = W.batched_dense_instance(i, n)
    t1 = time.perf_counter()
    r = R.solve(R.DenseOperator(inst.A), inst.b, inst.tau)
    return t1 - t0, time.perf_counter() - t1, r.ipm_iters, r.status


def time_shared_dense(j: int, batch: int):
    """Signal j of the shared-dense batch: oracle solve time."""
    import workloads as W
    from oracle import mfipm_ref as R
    inst = W.config_shared_dense(batch=batch, signals=[j])
    t0 = time.perf_counter()
    r = R.solve(R.DenseOperator(inst.A), inst.b[0], inst.tau[0])
    return time.perf_counter() - t0, r.ipm_iters, r.status


def time_grad_signal(j: int, n: int, batch: int):
    """Signal j of the shared partial-DCT batch: oracle forward solve, then
    the oracle adjoint of L = 1/2 ||x - x_true||^2 at its final point.
    Returns (forward s, adjoint s, IPM iterations, status)."""
    import workloads as W
    from oracle import mfipm_ref as R
    inst = W.config_dct_batch(n=n, batch=batch)
    op = R.PartialDCTOperator(inst.n, inst.rows)
    t0 = time.perf_counter()
    r = R.solve(op, inst.b[j], inst.tau[j])
    t1 = time.perf_counter()
    R.backward(op, r.z, r.s, r.x - inst.x_true[j])
    return t1 - t0, time.perf_counter() - t1, r.ipm_iters, r.status


def time_phase_instance(inst):
    """One instance of the phase-transition sweep: oracle solve time."""
    import workloads as W
    from oracle import mfipm_ref as R
    t0 = time.perf_counter()
    R.solve(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau, R.Params(**W.PHASE_PARAMS))
    return time.perf_counter() - t0


def time_direct(n: int, threads: int):
    """Draws the Section 5.7 problem of length n and solves it with the
    oracle's direct variant (Cholesky of the explicit 2n system), BLAS on
    `threads` threads.  Returns (solve s, IPM iterations, status)."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import mfipm_ref as R
    inst = W.direct_scaling_instance(n)
    with threadpool_limits(threads):
        t0 = time.perf_counter()
        r = R.solve(R.DenseOperator(inst.A), inst.b, inst.tau, R.Params(direct=1))
        return time.perf_counter() - t0, r.ipm_iters, r.status
