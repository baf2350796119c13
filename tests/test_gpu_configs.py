"""Parity at the full sizes of the named workloads, in the launch shapes the
benchmark uses (GPU).  Where the oracle cannot run every instance in seconds,
sampled instances are compared one by one and every instance is checked
against properties that hold at any size (status, gap certificate)."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import scipy.sparse.linalg as sla

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


def _state_zs(st, n):
    z = st[:2 * n].reshape(n, 2).T.reshape(-1)
    s = st[2 * n:].reshape(n, 2).T.reshape(-1)
    return z, s


def test_pdct_hdr_2p20(solver):
    """Partial DCT n=2^20, m=n/4, high dynamic range: full oracle comparison."""
    inst = W.config_pdct_hdr()
    say("pdct n=2^20 high dynamic range")
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
    ref = U.check_against_oracle(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau,
                                 res.x.cpu().numpy(), res.infos[0], res.state.cpu().numpy(), label="hdr")
    say("  gpu", res.infos[0]["ipm_iters"], res.infos[0]["pcg_iters"], "oracle", ref.ipm_iters, ref.pcg_iters)


def test_batched_dense_256(solver):
    """The 256-instance uneven dense batch in one launch: every instance
    converged with a gap certificate <= 1e-7 recomputed on the CPU from the
    GPU's x; the smallest, a middle and the largest instance against the
    oracle."""
    sizes = W.batched_dense_sizes(batch=256)
    with ThreadPoolExecutor(16) as ex:
        insts = list(ex.map(lambda iv: W.batched_dense_instance(iv[0], int(iv[1])), enumerate(sizes)))
    say("batched dense 256, sum m*n =", sum(i.m * i.n for i in insts))
    import torch
    dev = solver.device
    n_off = np.concatenate([[0], np.cumsum([i.n for i in insts])]).astype(np.int64)
    m_off = np.concatenate([[0], np.cumsum([i.m for i in insts])]).astype(np.int64)
    a_off = np.concatenate([[0], np.cumsum([i.m * i.n for i in insts])]).astype(np.int64)
    A = torch.empty(int(a_off[-1]), dtype=torch.float64, device=dev)
    for j, i in enumerate(insts):
        A[a_off[j]:a_off[j + 1]].copy_(torch.from_numpy(i.A.reshape(-1)))
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, A_packed=A, a_off=a_off)
    del A
    x = res.x.cpu().numpy()

    def cert(j):
        inst = insts[j]
        xj = x[n_off[j]:n_off[j + 1]]
        z = np.concatenate([np.maximum(xj, 0), np.maximum(-xj, 0)])
        _, r, g, primal = R.objective_terms(R.DenseOperator(inst.A), inst.b, inst.tau, z)
        return R.relative_gap(inst.b, inst.tau, r, g, primal)[0]
    with ThreadPoolExecutor(16) as ex:
        gaps = list(ex.map(cert, range(len(insts))))
    assert all(i["status"] == 0 for i in res.infos), [j for j, i in enumerate(res.infos) if i["status"]]
    assert max(gaps) <= 1e-7, max(gaps)
    order = np.argsort(sizes, kind="stable")
    for j in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        inst = insts[j]
        say("  sampled instance", j, "n =", inst.n)
        U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, x[n_off[j]:n_off[j + 1]],
                               res.infos[j], label=f"batch256 {j}")


def test_grad_batch_32_2p18(solver):
    """32 signals sharing a partial DCT, n=2^18: batched forward and adjoint.
    Sampled signals: x against the oracle; dL/db, dL/dtau against the
    oracle's adjoint at the GPU's own final point and against the closed form
    on the GPU's support (x_S affine in (b, tau) there), to 1e-5.  A
    directional central difference through the GPU solver at tolerance 1e-12
    is reported, not gated (solver noise swamps h = 1e-6 differences)."""
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
    op = R.PartialDCTOperator(n, inst.rows)
    for j in (0, 17):
        say("  signal", j)
        xj = x[j * n:(j + 1) * n]
        U.check_against_oracle(op, inst.b[j], inst.tau[j], xj, res.infos[j], st[4 * n * j:4 * n * (j + 1)],
                               label=f"grad {j}")
        z, s = _state_zs(st[4 * n * j:4 * n * (j + 1)], n)
        ref = R.backward(op, z, s, gx[j * n:(j + 1) * n])
        assert U.rel(gb[j], ref.grad_b) <= 1e-8, j
        assert abs(gt[j] - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau), j
        # closed form on the support, by CG through the DCT on A_S^T A_S
        S, sg = R.support_from_state(z, s, n)

        def AS(v):
            full = np.zeros(n)
            full[S] = v
            return op.matvec(full)
        G = sla.LinearOperator((len(S), len(S)), matvec=lambda v: op.rmatvec(AS(v))[S], dtype=np.float64)
        v, info = sla.cg(G, xj[S] - inst.x_true[j][S], rtol=1e-13, maxiter=5000)
        assert info == 0
        gb_cf = AS(v)
        gt_cf = -float(sg @ v)
        say(f"    |S|={len(S)} rel(grad_b, closed form)={U.rel(gb[j], gb_cf):.2e} "
            f"rel(grad_tau)={abs(gt[j] - gt_cf) / abs(gt_cf):.2e}")
        assert U.rel(gb[j], gb_cf) <= 1e-5, j
        assert abs(gt[j] - gt_cf) <= 1e-5 * abs(gt_cf), j
    # directional central difference through the GPU solver at a tight
    # tolerance (reported, not gated)
    h = 1e-6
    d = inst.extra["fd_direction"][0]
    tight = dict(tol=1e-12, tolpcg=1e-8, mxiterpcg=2000)
    solver.set_params(**tight)
    try:
        one = np.array([0, n], np.int64)
        onem = np.array([0, m], np.int64)
        r0 = solver.solve_batched(inst.b[0], inst.tau[:1], one, onem, rows=inst.rows, shared_op=True)
        g0, _, _ = solver.backward(r0.state, r0.x.cpu().numpy() - inst.x_true[0], one, onem, rows=inst.rows,
                                   shared_op=True)

        def loss(bb):
            rr = solver.solve_batched(bb, inst.tau[:1], one, onem, rows=inst.rows, shared_op=True)
            return 0.5 * float(np.sum((rr.x.cpu().numpy() - inst.x_true[0]) ** 2))
        fd = (loss(inst.b[0] + h * d) - loss(inst.b[0] - h * d)) / (2 * h)
        an = float(g0.cpu().numpy() @ d)
        say(f"  directional FD (tol 1e-12, h=1e-6): fd={fd:.8e} adjoint={an:.8e} "
            f"rel={abs(fd - an) / abs(an):.2e}")
    finally:
        solver.set_params(tol=1e-8, tolpcg=1e-2, mxiterpcg=200)
