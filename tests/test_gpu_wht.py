"""Partial Walsh-Hadamard operator (GPU) against the oracle's
PartialWHTOperator: single solves over the range of lengths (odd and even
log2 n, so both split shapes), the n = 2^16 and n = 2^20 workloads at the
strict bar, forced column lengths, uneven and shared-row batches, the
adjoint, the reduced n x n variant and the no-allocation entry point."""
import sys

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import mfipm_ref as R
from tests import gpu_util as U

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


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def _check(solver, inst, res, label, j=None, params=None, strict=False, **kw):
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    return U.check_against_oracle(R.PartialWHTOperator(inst.n, inst.rows), inst.b, inst.tau, x, res.infos[0], st,
                                  params=params, label=label, strict=strict,
                                  resolve=None if strict else U.resolver(solver, b=inst.b, tau=inst.tau,
                                                                         rows=inst.rows, n=inst.n,
                                                                         transform="wht"), **kw)


@pytest.mark.parametrize("n,m,k,seed", [(64, 16, 2, 1), (128, 40, 3, 2), (1024, 256, 10, 3),
                                        (1024, 1000, 20, 4), (2048, 700, 15, 7), (4096, 1023, 40, 5),
                                        (8192, 2048, 81, 6), (1 << 15, 8191, 300, 8)])
def test_wht_small(solver, n, m, k, seed):
    say(f"wht n={n} m={m} seed={seed}")
    inst = W.dct_instance(n, m, k, seed=seed, amp="normal", sigma=1e-2, c_tau=1e-2, transform="wht")
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n, transform="wht")
    _check(solver, inst, res, f"wht{n}/{m}")


@pytest.mark.parametrize("l1", [2, 5, 9, 13])
def test_wht_column_lengths(solver, l1):
    """Every column length of the two-step split gives the same answer."""
    n = 1 << 14
    say(f"wht n={n} forced l1={l1}")
    inst = W.dct_instance(n, n // 4, 100, seed=21, amp="normal", sigma=1e-2, c_tau=1e-2, transform="wht")
    solver.set_launch(0, 0, l1)
    try:
        res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n, transform="wht")
    finally:
        solver.set_launch(0, 0, 0)
    _check(solver, inst, res, f"wht l1={l1}")


def test_wht_2p16(solver):
    say("wht n=2^16 workload")
    inst = W.config_wht()
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n, transform="wht")
    ref = _check(solver, inst, res, "wht 2^16", strict=True)
    say("  gpu", res.infos[0], "oracle", ref.ipm_iters, ref.pcg_iters, "ms", res.kernel_ms)


def test_wht_2p20_hdr(solver):
    say("wht n=2^20 high-dynamic-range workload")
    inst = W.config_wht_hdr()
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n, transform="wht")
    ref = _check(solver, inst, res, "wht 2^20 hdr", strict=True)
    say("  gpu", res.infos[0], "oracle", ref.ipm_iters, ref.pcg_iters, "ms", res.kernel_ms)


def test_wht_operator_is_the_transform(solver):
    """All rows kept: A is W itself, so the minimiser is the
    soft threshold of W b (the closed form of the separable problem)."""
    n = 1024
    rng = np.random.default_rng(np.random.PCG64(31))
    rows = np.arange(n, dtype=np.int32)
    b = rng.standard_normal(n)
    tau = 0.3
    solver.set_params(tol=1e-12)
    try:
        res = solver.solve(b, tau, rows=rows, n=n, transform="wht")
    finally:
        solver.set_params(tol=1e-8)
    c = scipy.linalg.hadamard(n) @ b / np.sqrt(n)
    x_cf = np.sign(c) * np.maximum(np.abs(c) - tau, 0.0)
    assert res.infos[0]["status"] == 0
    assert U.rel(res.x.cpu().numpy(), x_cf) <= 1e-7


def test_wht_batched_uneven(solver):
    ns = [64, 256, 1024, 4096, 512, 1 << 15, 128]
    insts = [W.dct_instance(n, n // 4, max(1, n // 100), seed=700 + i, transform="wht") for i, n in enumerate(ns)]
    say("batched wht", ns)
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    rows = np.concatenate([i.rows for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, rows=rows, transform="wht")
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    for j, inst in enumerate(insts):
        U.check_against_oracle(R.PartialWHTOperator(inst.n, inst.rows), inst.b, inst.tau,
                               x[n_off[j]:n_off[j + 1]], res.infos[j], st[4 * n_off[j]:4 * n_off[j + 1]],
                               label=f"batch wht {j}",
                               resolve=U.resolver(solver, b=inst.b, tau=inst.tau, rows=inst.rows, n=inst.n,
                                                  transform="wht"))


@pytest.mark.parametrize("reduced", [0, 1])
def test_wht_shared_and_adjoint(solver, reduced):
    """Signals sharing one row set; every signal and its adjoint against the
    oracle (the adjoint at the GPU's final point)."""
    inst = W.config_dct_batch(n=4096, batch=5, transform="wht")
    B, m = inst.b.shape
    n = inst.n
    prm = R.Params(reduced=reduced)
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    old = solver.params.reduced
    solver.set_params(reduced=reduced)
    try:
        res = solver.solve_batched(inst.b.reshape(-1), inst.tau, n_off, m_off, rows=inst.rows, shared_op=True,
                                   transform="wht")
        x = res.x.cpu().numpy()
        st = res.state.cpu().numpy()
        gx = x - inst.x_true.reshape(-1)
        gb, gt, binf = solver.backward(res.state, gx, n_off, m_off, rows=inst.rows, shared_op=True,
                                       transform="wht")
        op = R.PartialWHTOperator(n, inst.rows)
        gb = gb.cpu().numpy().reshape(B, m)
        gt = gt.cpu().numpy()
        for j in range(B):
            sl = slice(j * n, (j + 1) * n)
            U.check_against_oracle(op, inst.b[j], inst.tau[j], x[sl], res.infos[j], st[4 * n * j:4 * n * (j + 1)],
                                   params=prm, label=f"wht shared {j} reduced={reduced}",
                                   resolve=U.resolver(solver, b=inst.b[j], tau=float(inst.tau[j]), rows=inst.rows,
                                                      n=n, transform="wht"))
            assert binf[j]["status"] == 0, binf[j]
            z, s = U.zs_from_state(st[4 * n * j:4 * n * (j + 1)], n)
            ref = R.backward(op, z, s, gx[sl], prm)
            assert U.rel(gb[j], ref.grad_b) <= 1e-8, j
            assert abs(gt[j] - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau), j
    finally:
        solver.set_params(reduced=old)


def test_wht_noalloc_matches_solve(solver):
    """The no-allocation entry point takes the Walsh-Hadamard operator too:
    same status, iterations within the slack and x within the parity bar of
    the workspace entry point."""
    import torch
    inst = W.dct_instance(4096, 1024, 40, seed=41, transform="wht")
    ref = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n, transform="wht")
    dev = solver.device
    b = torch.as_tensor(inst.b, dtype=torch.float64, device=dev)
    rows = torch.as_tensor(inst.rows, dtype=torch.int32, device=dev)
    x = torch.empty(inst.n, dtype=torch.float64, device=dev)
    info = solver.solve_noalloc(b, inst.tau, x, rows=rows, n=inst.n, transform="wht")
    assert info["status"] == ref.infos[0]["status"] == 0
    assert abs(info["ipm_iters"] - ref.infos[0]["ipm_iters"]) <= U.ITER_SLACK
    assert U.rel(x.cpu().numpy(), ref.x.cpu().numpy()) <= U.X_REL
