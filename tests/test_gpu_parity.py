"""HIP solver against the CPU oracle on identical seeded inputs (GPU)."""
import math
import sys

import numpy as np
import pytest

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


def _dense(m, n, k, seed, sigma=1e-3, c_tau=1e-2):
    inst = W.dense_instance(m, n, k, seed=seed, amp="normal", sigma=sigma, c_tau=c_tau)
    return inst


@pytest.mark.parametrize("m,n,k,seed", [(16, 64, 2, 1), (40, 200, 4, 2), (64, 300, 6, 3),
                                        (100, 1000, 10, 4), (128, 129, 3, 5)])
def test_dense_small(solver, m, n, k, seed):
    say(f"dense small m={m} n={n} seed={seed}")
    inst = _dense(m, n, k, seed)
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                           res.state.cpu().numpy(), label=f"dense{m}x{n}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


def test_dense_256x1024(solver):
    say("dense 256x1024 configuration")
    inst = W.config_dense_256x1024()
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    ref = U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(),
                                 res.infos[0], res.state.cpu().numpy(), label="C1", strict=True)
    say("  gpu", res.infos[0], "oracle iters", ref.ipm_iters, ref.pcg_iters)


@pytest.mark.parametrize("n,m,k,seed", [(64, 16, 2, 1), (128, 40, 3, 2), (1024, 256, 10, 3),
                                        (1024, 1000, 20, 4), (4096, 1023, 40, 5), (8192, 2048, 81, 6)])
def test_pdct_small(solver, n, m, k, seed):
    say(f"pdct small n={n} m={m} seed={seed}")
    inst = W.dct_instance(n, m, k, seed=seed, amp="normal", sigma=1e-2, c_tau=1e-2)
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
    U.check_against_oracle(R.PartialDCTOperator(n, inst.rows), inst.b, inst.tau, res.x.cpu().numpy(),
                           res.infos[0], res.state.cpu().numpy(), label=f"pdct{n}/{m}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, rows=inst.rows, n=n))


@pytest.mark.parametrize("l1", [2, 4, 6])
def test_pdct_tile_choices(solver, l1):
    """Every column-FFT length gives the same answer (four-step split)."""
    n = 4096
    say(f"pdct tile l1={l1}")
    inst = W.dct_instance(n, 1024, 30, seed=11, amp="normal", sigma=1e-2, c_tau=1e-2)
    solver.set_launch(0, 0, l1)
    try:
        res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
    finally:
        solver.set_launch(0, 0, 0)
    U.check_against_oracle(R.PartialDCTOperator(n, inst.rows), inst.b, inst.tau, res.x.cpu().numpy(),
                           res.infos[0], res.state.cpu().numpy(), label=f"l1={l1}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, rows=inst.rows, n=n))


def test_pdct_2p16(solver):
    say("pdct n=2^16 configuration")
    inst = W.config_pdct()
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
    ref = U.check_against_oracle(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau,
                                 res.x.cpu().numpy(), res.infos[0], res.state.cpu().numpy(), label="C2",
                                 strict=True)
    say("  gpu", res.infos[0], "oracle", ref.ipm_iters, ref.pcg_iters, "ms", res.kernel_ms)


def test_zero_solution(solver):
    inst = _dense(30, 90, 3, seed=21)
    tau = 1.5 * float(np.max(np.abs(inst.A.T @ inst.b)))
    res = solver.solve(inst.b, tau, A=inst.A)
    assert res.infos[0]["status"] == 0
    assert float(res.x.abs().max()) <= 1e-8 * (1 + np.max(np.abs(inst.b)))


def test_full_dct_soft_threshold(solver):
    n = 256
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n)
    rows = np.arange(n, dtype=np.int32)
    solver.set_params(tol=1e-12)
    try:
        res = solver.solve(b, 0.5, rows=rows, n=n)
    finally:
        solver.set_params(tol=1e-8)
    op = R.PartialDCTOperator(n, rows)
    ref = R.soft_threshold(op.rmatvec(b), 0.5)
    assert U.rel(res.x.cpu().numpy(), ref) <= 1e-7


def test_identity_soft_threshold(solver):
    n = 128
    rng = np.random.default_rng(6)
    b = rng.standard_normal(n)
    solver.set_params(tol=1e-12)
    try:
        res = solver.solve(b, 0.7, A=np.eye(n))
    finally:
        solver.set_params(tol=1e-8)
    assert U.rel(res.x.cpu().numpy(), R.soft_threshold(b, 0.7)) <= 1e-7


def test_status_paths(solver):
    from paper_1208_5435_amd import MfipmError
    inst = _dense(16, 64, 2, seed=8)
    solver.set_params(maxiters=1)
    try:
        res = solver.solve(inst.b, inst.tau, A=inst.A)
    finally:
        solver.set_params(maxiters=100)
    assert res.infos[0]["status"] == 1 and res.infos[0]["ipm_iters"] == 1
    bb = inst.b.copy()
    bb[0] = np.nan
    res = solver.solve(bb, inst.tau, A=inst.A)
    assert res.infos[0]["status"] == 3
    with pytest.raises(MfipmError):
        solver.solve(inst.b, -1.0, A=inst.A)
    with pytest.raises(MfipmError):   # n not a power of two
        solver.solve(np.zeros(10), 1.0, rows=np.arange(10, dtype=np.int32), n=100)
    with pytest.raises(MfipmError):   # unsorted rows: device-side check
        solver.solve(np.ones(4), 1.0, rows=np.array([5, 3, 9, 20], dtype=np.int32), n=64)
    # the handle still works afterwards
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    assert res.infos[0]["status"] == 0


def test_mxiterpcg_one(solver):
    """A PCG cap of one iteration is not an error; the IPM still ends."""
    inst = _dense(32, 128, 3, seed=9)
    solver.set_params(mxiterpcg=1)
    try:
        res = solver.solve(inst.b, inst.tau, A=inst.A)
    finally:
        solver.set_params(mxiterpcg=200)
    p = R.Params(mxiterpcg=1)
    ref = R.solve(R.DenseOperator(inst.A), inst.b, inst.tau, p)
    assert res.infos[0]["status"] == ref.status
    assert abs(res.infos[0]["ipm_iters"] - ref.ipm_iters) <= 1
