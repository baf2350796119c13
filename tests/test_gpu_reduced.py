"""The reduced n x n PCG variant (GPU) against the oracle's reduced variant:
the same IPM with PCG on (Theta_bar^{-1} + A^T A) d = Theta_bar^{-1}
(Theta_u r_u - Theta_v r_v) and the back-substituted 2n direction."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mfipm_ref as R
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

RED = R.Params(reduced=1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver(gpu_lib):
    from paper_1208_5435_amd import Solver
    s = Solver(params=dict(reduced=1))
    yield s
    s.close()


@pytest.mark.parametrize("m,n,k,seed", [(40, 200, 4, 2), (100, 1000, 10, 4), (128, 129, 3, 5)])
def test_reduced_dense(solver, m, n, k, seed):
    inst = W.dense_instance(m, n, k, seed=seed, amp="normal", sigma=1e-3, c_tau=1e-2)
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                           res.state.cpu().numpy(), params=RED, label=f"red dense{m}x{n}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


@pytest.mark.parametrize("n,m,k,seed", [(1024, 256, 10, 3), (4096, 1023, 40, 5), (8192, 2048, 81, 6)])
def test_reduced_pdct(solver, n, m, k, seed):
    inst = W.dct_instance(n, m, k, seed=seed, amp="normal", sigma=1e-2, c_tau=1e-2)
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
    U.check_against_oracle(R.PartialDCTOperator(n, inst.rows), inst.b, inst.tau, res.x.cpu().numpy(),
                           res.infos[0], res.state.cpu().numpy(), params=RED, label=f"red pdct{n}/{m}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, rows=inst.rows, n=n))


def test_reduced_configs(solver):
    """Dense 256 x 1024 and partial DCT n = 2^16 at the strict bar."""
    inst = W.config_dense_256x1024()
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    ref = U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                                 res.state.cpu().numpy(), params=RED, label="red C1", strict=True)
    say(f"reduced dense 256x1024: gpu {res.infos[0]['ipm_iters']} IPM {res.infos[0]['pcg_iters']} PCG, oracle "
        f"{ref.ipm_iters} {ref.pcg_iters}")
    inst = W.config_pdct()
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
    ref = U.check_against_oracle(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau, res.x.cpu().numpy(),
                                 res.infos[0], res.state.cpu().numpy(), params=RED, label="red C2", strict=True)
    say(f"reduced pdct 2^16: gpu {res.infos[0]['ipm_iters']} IPM {res.infos[0]['pcg_iters']} PCG "
        f"{res.kernel_ms:.2f} ms, oracle {ref.ipm_iters} {ref.pcg_iters}")


def test_reduced_batched_and_adjoint(solver):
    """A batch of partial DCT signals sharing rows; every signal against the
    oracle, and the adjoint against the oracle's reduced adjoint at the GPU's
    final point."""
    inst = W.config_dct_batch(n=4096, batch=5)
    B, m = inst.b.shape
    n = inst.n
    n_off = np.arange(B + 1, dtype=np.int64) * n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    res = solver.solve_batched(inst.b.reshape(-1), inst.tau, n_off, m_off, rows=inst.rows, shared_op=True)
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    op = R.PartialDCTOperator(n, inst.rows)
    gx = x - inst.x_true.reshape(-1)
    gb, gt, binf = solver.backward(res.state, gx, n_off, m_off, rows=inst.rows, shared_op=True)
    gb = gb.cpu().numpy().reshape(B, m)
    gt = gt.cpu().numpy()
    for j in range(B):
        sl = slice(j * n, (j + 1) * n)
        U.check_against_oracle(op, inst.b[j], inst.tau[j], x[sl], res.infos[j], st[4 * n * j:4 * n * (j + 1)],
                               params=RED, label=f"red batch {j}",
                               resolve=U.resolver(solver, b=inst.b[j], tau=float(inst.tau[j]), rows=inst.rows, n=n))
        assert binf[j]["status"] == 0, binf[j]
        z, s = U.zs_from_state(st[4 * n * j:4 * n * (j + 1)], n)
        ref = R.backward(op, z, s, gx[sl], RED)
        assert U.rel(gb[j], ref.grad_b) <= 1e-8, j
        assert abs(gt[j] - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau), j
