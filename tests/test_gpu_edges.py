"""Edge cases (GPU): the dense two-pass operator path (n above the fused
path's 8192, and odd n), with the reduced variant and the adjoint on it;
the smallest instances (one measurement); and argument checks at the size
limits and for empty batches."""
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


@pytest.mark.parametrize("m,n,k,seed", [(500, 10000, 40, 11), (768, 12288, 50, 12), (250, 1001, 10, 13)])
def test_dense_two_pass(solver, m, n, k, seed):
    say(f"dense two-pass m={m} n={n}")
    inst = W.dense_instance(m, n, k, seed=seed, amp="normal", sigma=1e-3, c_tau=1e-2)
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                           res.state.cpu().numpy(), label=f"dense2p {m}x{n}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


def test_dense_two_pass_reduced_and_adjoint(solver):
    inst = W.dense_instance(400, 9000, 30, seed=14, amp="normal", sigma=1e-3, c_tau=2e-2)
    n, m = inst.n, inst.m
    red = R.Params(reduced=1)
    solver.set_params(reduced=1)
    try:
        res = solver.solve(inst.b, inst.tau, A=inst.A)
        U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                               res.state.cpu().numpy(), params=red, label="dense2p reduced",
                               resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))
        gx = res.x.cpu().numpy() - inst.x_true
        n_off = np.array([0, n], np.int64)
        m_off = np.array([0, m], np.int64)
        a_off = np.array([0, m * n], np.int64)
        gb, gt, infos = solver.backward(res.state, gx, n_off, m_off, A_packed=inst.A.reshape(-1), a_off=a_off)
    finally:
        solver.set_params(reduced=0)
    z, s = U.zs_from_state(res.state.cpu().numpy(), n)
    ref = R.backward(R.DenseOperator(inst.A), z, s, gx, red)
    assert infos[0]["status"] == 0
    assert U.rel(gb.cpu().numpy(), ref.grad_b) <= 1e-8
    assert abs(float(gt.cpu()[0]) - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau)


@pytest.mark.parametrize("kind", ["dense", "dct", "wht", "dst"])
def test_one_measurement(solver, kind):
    """m = 1: a single measurement."""
    rng = np.random.default_rng(np.random.PCG64(77))
    n = 64
    if kind == "dense":
        A = rng.standard_normal((1, n))
        b = np.array([1.5])
        tau = 0.1 * float(np.max(np.abs(A.T @ b)))
        op = R.DenseOperator(A)
        res = solver.solve(b, tau, A=A)
        rs = U.resolver(solver, b=b, tau=tau, A=A)
    else:
        rows = np.array([5], dtype=np.int32)
        op = {"dct": R.PartialDCTOperator, "wht": R.PartialWHTOperator, "dst": R.PartialDSTOperator}[kind](n, rows)
        b = np.array([0.7])
        tau = 0.1 * float(np.max(np.abs(op.rmatvec(b))))
        res = solver.solve(b, tau, rows=rows, n=n, transform=kind)
        rs = U.resolver(solver, b=b, tau=tau, rows=rows, n=n, transform=kind)
    U.check_against_oracle(op, b, tau, res.x.cpu().numpy(), res.infos[0], res.state.cpu().numpy(),
                           label=f"m=1 {kind}", resolve=rs)


def test_limits_and_empty_batch(solver):
    from paper_1208_5435_amd import MfipmError
    rng = np.random.default_rng(5)
    # transform longer than 2^20
    n = 1 << 21
    with pytest.raises(MfipmError) as e:
        solver.solve(np.ones(4), 1.0, rows=np.array([1, 2, 3, 4], dtype=np.int32), n=n)
    assert e.value.code == -1
    # more rows than the transform length
    with pytest.raises(MfipmError) as e:
        solver.solve(np.ones(65), 1.0, rows=np.arange(65, dtype=np.int32), n=64)
    assert e.value.code == -1
    # an empty batch
    with pytest.raises(MfipmError) as e:
        solver.solve_batched(np.zeros(0), np.zeros(0), np.zeros(1, np.int64), np.zeros(1, np.int64),
                             rows=np.zeros(0, np.int32))
    assert e.value.code == -1
    # the handle still works
    inst = W.dense_instance(16, 64, 2, seed=3)
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    assert res.infos[0]["status"] == 0
    _ = rng
