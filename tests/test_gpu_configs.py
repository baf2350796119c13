"""Parity at the full sizes of the named workloads, in the launch shapes the
benchmark uses (GPU).  Every instance of the batches is compared with the
oracle at the strict bar (no escalation); the oracle runs in host worker
processes (oracle/pool.py) so that the whole batch fits the test's time."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mfipm_ref as R
from oracle import pool
from tests import gpu_util as U
from tests import parity_tasks as T

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver(gpu_lib):
    from paper_1208_5435_amd import Solver
    s = Solver()
    yield s
    s.close()


def test_pdct_hdr_2p20(solver):
    """Partial DCT n=2^20, m=n/4, high dynamic range: full oracle comparison."""
    inst = W.config_pdct_hdr()
    say("pdct n=2^20 high dynamic range")
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
    ref = U.check_against_oracle(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau,
                                 res.x.cpu().numpy(), res.infos[0], res.state.cpu().numpy(), label="hdr",
                                 strict=True)
    say("  gpu", res.infos[0]["ipm_iters"], res.infos[0]["pcg_iters"], "oracle", ref.ipm_iters, ref.pcg_iters)


def test_batched_dense_256(solver):
    """The 256-instance uneven dense batch in one launch: all 256 instances
    against the oracle at the strict bar."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    sizes = [int(v) for v in W.batched_dense_sizes(batch=256)]
    with ThreadPoolExecutor(16) as ex:
        insts = list(ex.map(lambda iv: W.batched_dense_instance(iv[0], iv[1]), enumerate(sizes)))
    say("batched dense 256, sum m*n =", sum(i.m * i.n for i in insts))
    dev = solver.device
    n_off = np.concatenate([[0], np.cumsum([i.n for i in insts])]).astype(np.int64)
    m_off = np.concatenate([[0], np.cumsum([i.m for i in insts])]).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum([i.m * i.n for i in insts])]).astype(np.int64)
    A = torch.empty(int(a_off[-1]), dtype=torch.float64, device=dev)
    for j, i in enumerate(insts):
        A[a_off[j]:a_off[j + 1]].copy_(torch.from_numpy(i.A.reshape(-1)))
    b = np.concatenate([i.b for i in insts])
    taus = [i.tau for i in insts]
    del insts
    res = solver.solve_batched(b, taus, n_off, m_off, A_packed=A, a_off=a_off)
    del A
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    assert all(i["status"] == 0 for i in res.infos), [j for j, i in enumerate(res.infos) if i["status"]]
    say(f"  kernel {res.kernel_ms:.1f} ms; oracle on {pool.host_cores()} host processes")
    args = [(j, sizes[j], x[n_off[j]:n_off[j + 1]], st[4 * n_off[j]:4 * n_off[j + 1]], res.infos[j])
            for j in range(256)]
    order = sorted(range(256), key=lambda j: -sizes[j])
    worst = 0.0
    with pool.executor() as ex:
        futs = [ex.submit(T.batched_dense_instance, *args[j]) for j in order]
        for k, f in enumerate(futs):
            j, it_ref, it_gpu, r = f.result()
            worst = max(worst, r)
            if k % 32 == 31:
                say(f"  {k + 1}/256 instances checked, worst rel(x) {worst:.2e}")
    say(f"  all 256 instances at the strict bar; worst rel(x) {worst:.2e}")


def test_grad_batch_32_2p18(solver):
    """32 signals sharing a partial DCT, n=2^18: batched forward and adjoint.
    Every signal: x at the strict bar; dL/db, dL/dtau against the oracle's
    adjoint at the GPU's own final point (1e-8) and against the closed form
    on the GPU's support (1e-5)."""
    inst = W.config_dct_batch()
    B, m = inst.b.shape
    n = inst.n
    say("grad batch 32 x 2^18")
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    res = solver.solve_batched(inst.b.reshape(-1), inst.tau, n_off, m_off, rows=inst.rows, shared_op=True)
    x = res.x.cpu().numpy()
    gx = x - inst.x_true.reshape(-1)
    gb, gt, binf = solver.backward(res.state, gx, n_off, m_off, rows=inst.rows, shared_op=True)
    gb = gb.cpu().numpy().reshape(B, m)
    gt = gt.cpu().numpy()
    st = res.state.cpu().numpy()
    assert all(i["status"] == 0 for i in res.infos)
    assert all(i["status"] == 0 for i in binf)
    say(f"  forward {res.kernel_ms:.1f} ms, adjoint {solver.last_kernel_ms():.1f} ms; "
        f"oracle on {pool.host_cores()} host processes")
    worst = [0.0, 0.0]
    with pool.executor() as ex:
        futs = [ex.submit(T.grad_signal, j, n, B, x[j * n:(j + 1) * n], st[4 * n * j:4 * n * (j + 1)],
                          res.infos[j], gb[j], float(gt[j]), binf[j]) for j in range(B)]
        for f in futs:
            j, eb, et, eb_cf, et_cf, ns = f.result()
            worst = [max(worst[0], eb, et), max(worst[1], eb_cf, et_cf)]
            say(f"  signal {j}: |S|={ns} adjoint vs oracle {max(eb, et):.1e}, vs closed form "
                f"{max(eb_cf, et_cf):.1e}")
    say(f"  all 32 signals: worst adjoint-vs-oracle {worst[0]:.2e}, worst closed-form {worst[1]:.2e}")
