"""Batched solves and the adjoint (GPU) against the CPU oracle."""
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


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def test_batched_dense_uneven(solver):
    ns = [64, 128, 200, 256, 320, 512, 1000]
    insts = [W.dense_instance(n // 4, n, max(1, n // 50), seed=300 + i, amp="normal", sigma=1e-3, c_tau=1e-2)
             for i, n in enumerate(ns)]
    say("batched dense", ns)
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    a_off = _offsets([i.m * i.n for i in insts])
    A = np.concatenate([i.A.reshape(-1) for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, A_packed=A, a_off=a_off)
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    for j, inst in enumerate(insts):
        U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, x[n_off[j]:n_off[j + 1]],
                               res.infos[j], st[4 * n_off[j]:4 * n_off[j + 1]], label=f"batch dense {j}",
                               resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


def test_batched_equals_single_bitwise(solver):
    """Reductions are fixed-order over items, so the team size does not change
    a single bit of the result."""
    insts = [W.dct_instance(2048, 512, 20, seed=400 + i) for i in range(3)]
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    rows = np.concatenate([i.rows for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, rows=rows)
    xb = res.x.cpu().numpy()
    for j, inst in enumerate(insts):
        r1 = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
        assert np.array_equal(r1.x.cpu().numpy(), xb[n_off[j]:n_off[j + 1]]), j
        assert r1.infos[0]["ipm_iters"] == res.infos[j]["ipm_iters"]


@pytest.mark.parametrize("logn,team", [(18, 64), (20, 128)])
def test_write_through_team_equals_one_workgroup(solver, logn, team):
    """A team of several workgroups stores the exchange buffers and the PCG
    vectors through the L2 (the write-through path of multi-workgroup teams at
    n >= 2^18) and synchronises over the XCDs; a team of one workgroup does
    neither.  At these team sizes both cut the work into the same items, so
    the fixed-order reductions give bit-identical results."""
    n = 1 << logn
    inst = W.dct_instance(n, n // 4, n // 100, seed=4242 + logn, sigma=1e-2, c_tau=5e-3)
    out = {}
    try:
        for wg in (1, team):
            say(f"write-through check: n=2^{logn}, {wg} workgroup(s)")
            solver.set_launch(wg, 0, 0)
            r = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
            out[wg] = (r.x.cpu().numpy(), r.infos[0])
    finally:
        solver.set_launch(0, 0, 0)
    (x1, i1), (xt, it) = out[1], out[team]
    assert i1["status"] == it["status"] == 0, (i1, it)
    assert (i1["ipm_iters"], i1["pcg_iters"]) == (it["ipm_iters"], it["pcg_iters"])
    assert np.array_equal(x1, xt)


def test_batched_pdct_uneven_lengths(solver):
    """Different n in one launch: per-instance twiddle resolution."""
    ns = [64, 256, 1024, 4096, 512]
    insts = [W.dct_instance(n, n // 4, max(1, n // 100), seed=500 + i) for i, n in enumerate(ns)]
    say("batched pdct", ns)
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    rows = np.concatenate([i.rows for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, rows=rows)
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    for j, inst in enumerate(insts):
        U.check_against_oracle(R.PartialDCTOperator(inst.n, inst.rows), inst.b, inst.tau,
                               x[n_off[j]:n_off[j + 1]], res.infos[j], st[4 * n_off[j]:4 * n_off[j + 1]],
                               label=f"batch pdct {j}",
                               resolve=U.resolver(solver, b=inst.b, tau=inst.tau, rows=inst.rows, n=inst.n))


def test_batched_pdct_shared_rows(solver):
    inst = W.config_dct_batch(n=4096, batch=6)
    say("batched pdct shared rows n=4096 x6")
    B, m = inst.b.shape
    n_off = np.arange(B + 1, dtype=np.int64) * inst.n
    m_off = np.arange(B + 1, dtype=np.int64) * m
    res = solver.solve_batched(inst.b.reshape(-1), inst.tau, n_off, m_off, rows=inst.rows, shared_op=True)
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    op = R.PartialDCTOperator(inst.n, inst.rows)
    for j in range(B):
        U.check_against_oracle(op, inst.b[j], inst.tau[j], x[n_off[j]:n_off[j + 1]], res.infos[j],
                               st[4 * n_off[j]:4 * n_off[j + 1]], label=f"shared {j}",
                               resolve=U.resolver(solver, b=inst.b[j], tau=inst.tau[j], rows=inst.rows,
                                                  n=inst.n))


def test_batched_dense_12_of_workload(solver):
    """The first 12 instances of the uneven dense workload (n multiple of 64
    in [1024, 8192]) in one launch: every instance against its own gap
    certificate and against the oracle at the strict bar."""
    sizes = W.batched_dense_sizes(batch=12)
    insts = [W.batched_dense_instance(i, int(n)) for i, n in enumerate(sizes)]
    say("batched dense sampled", list(sizes))
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    a_off = _offsets([i.m * i.n for i in insts])
    A = np.concatenate([i.A.reshape(-1) for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, A_packed=A, a_off=a_off)
    x = res.x.cpu().numpy()
    for j, inst in enumerate(insts):
        assert res.infos[j]["status"] == 0, (j, res.infos[j])
        xj = x[n_off[j]:n_off[j + 1]]
        op = R.DenseOperator(inst.A)
        z = np.concatenate([np.maximum(xj, 0), np.maximum(-xj, 0)])
        _, r, g, primal = R.objective_terms(op, inst.b, inst.tau, z)
        gap, _ = R.relative_gap(inst.b, inst.tau, r, g, primal)
        assert gap <= 1e-7, (j, gap)
    st = res.state.cpu().numpy()
    for j in range(len(insts)):
        inst = insts[j]
        U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, x[n_off[j]:n_off[j + 1]],
                               res.infos[j], st[4 * n_off[j]:4 * n_off[j + 1]], label=f"batch12 {j}",
                               strict=True)


# ---------------------------------------------------------------- adjoint --------

def _closed_form(op_dense, b, tau, xt, z, s):
    S, sg = R.support_from_state(z, s, op_dense.n)
    x = z[:op_dense.n] - z[op_dense.n:]
    return R.closed_form_gradient(op_dense.dense()[:, S], sg, x[S], xt[S])


def test_backward_dense_vs_oracle_and_closed_form(solver):
    inst = W.dense_instance(40, 120, 4, seed=55, amp="normal", sigma=1e-3, c_tau=5e-2)
    solver.set_params(tol=1e-12, tolpcg=1e-8, mxiterpcg=2000)
    try:
        res = solver.solve(inst.b, inst.tau, A=inst.A)
        n = inst.n
        x = res.x.cpu().numpy()
        gx = x - inst.x_true
        n_off = np.array([0, n], np.int64)
        m_off = np.array([0, inst.m], np.int64)
        gb, gt, infos = solver.backward(res.state, gx, n_off, m_off, A_packed=inst.A,
                                        a_off=np.array([0, inst.m * n], np.int64))
    finally:
        solver.set_params(tol=1e-8, tolpcg=1e-2, mxiterpcg=200)
    st = res.state.cpu().numpy()
    z = st[:2 * n].reshape(n, 2).T.reshape(-1)
    s = st[2 * n:].reshape(n, 2).T.reshape(-1)
    op = R.DenseOperator(inst.A)
    ref = R.backward(op, z, s, gx)
    gbn = gb.cpu().numpy()
    gtn = float(gt.cpu().numpy()[0])
    assert infos[0]["status"] == 0
    assert U.rel(gbn, ref.grad_b) <= 1e-8
    assert abs(gtn - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau)
    gb_cf, gt_cf = _closed_form(op, inst.b, inst.tau, inst.x_true, z, s)
    assert U.rel(gbn, gb_cf) <= 1e-5
    assert abs(gtn - gt_cf) <= 1e-5 * abs(gt_cf)


def test_backward_pdct_vs_oracle(solver):
    inst = W.dct_instance(2048, 512, 10, seed=66, sigma=1e-2, c_tau=2e-2)
    n = inst.n
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
    gx = res.x.cpu().numpy() - inst.x_true
    n_off = np.array([0, n], np.int64)
    m_off = np.array([0, inst.m], np.int64)
    gb, gt, infos = solver.backward(res.state, gx, n_off, m_off, rows=inst.rows)
    st = res.state.cpu().numpy()
    z = st[:2 * n].reshape(n, 2).T.reshape(-1)
    s = st[2 * n:].reshape(n, 2).T.reshape(-1)
    ref = R.backward(R.PartialDCTOperator(n, inst.rows), z, s, gx)
    assert infos[0]["status"] == 0
    assert U.rel(gb.cpu().numpy(), ref.grad_b) <= 1e-8
    assert abs(float(gt.cpu()[0]) - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau)


def test_autograd_batched_shared_dct(solver):
    """torch.autograd through the batched solve.  Every signal: gradients
    against the oracle's adjoint at the GPU's own final point.  Signals where
    the closed form on the support is well posed (the tightly converged
    oracle adjoint agrees with it to 1e-7; it does not when a support entry
    is so small that its Theta stays moderate): also against the closed form
    to 1e-5."""
    import torch
    from paper_1208_5435_amd.autograd import MfipmSolve
    inst = W.config_dct_batch(n=1024, batch=4, c_tau=2e-2)
    dev = solver.device
    b = torch.tensor(inst.b, device=dev, requires_grad=True)
    tau = torch.tensor(inst.tau, device=dev, requires_grad=True)
    xt = torch.tensor(inst.x_true, device=dev)
    tight = dict(tol=1e-12, tolpcg=1e-8, mxiterpcg=2000)
    solver.set_params(**tight)
    try:
        x = MfipmSolve.apply(b, tau, solver, None, torch.tensor(inst.rows, device=dev), inst.n)
        loss = 0.5 * ((x - xt) ** 2).sum()
        gb, gt = torch.autograd.grad(loss, (b, tau))
        # the state the autograd forward kept (same inputs, bitwise-identical run)
        n = inst.n
        B = inst.b.shape[0]
        res = solver.solve_batched(inst.b.reshape(-1), inst.tau, np.arange(B + 1) * n,
                                   np.arange(B + 1) * inst.m, rows=inst.rows, shared_op=True)
    finally:
        solver.set_params(tol=1e-8, tolpcg=1e-2, mxiterpcg=200)
    op = R.PartialDCTOperator(inst.n, inst.rows)
    Ad = op.dense()
    xs = x.detach().cpu().numpy()
    assert np.array_equal(xs.reshape(-1), res.x.cpu().numpy())
    st = res.state.cpu().numpy()
    P = R.Params(**tight)
    well_posed = 0
    for j in range(B):
        sj = st[4 * n * j:4 * n * (j + 1)]
        z = sj[:2 * n].reshape(n, 2).T.reshape(-1)
        s = sj[2 * n:].reshape(n, 2).T.reshape(-1)
        ref = R.backward(op, z, s, xs[j] - inst.x_true[j], P)
        assert U.rel(gb[j].cpu().numpy(), ref.grad_b) <= 1e-8, j
        assert abs(float(gt[j]) - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau), j
        orc = R.solve(op, inst.b[j], inst.tau[j], P)
        S, sg = R.support_from_state(orc.z, orc.s, n)
        gb_cf, gt_cf = R.closed_form_gradient(Ad[:, S], sg, orc.x[S], inst.x_true[j][S])
        go = R.backward(op, orc.z, orc.s, orc.x - inst.x_true[j], P)
        if U.rel(go.grad_b, gb_cf) <= 1e-7:
            well_posed += 1
            gb_cf, gt_cf = R.closed_form_gradient(Ad[:, S], sg, xs[j][S], inst.x_true[j][S])
            assert U.rel(gb[j].cpu().numpy(), gb_cf) <= 1e-5, j
            assert abs(float(gt[j]) - gt_cf) <= 1e-5 * abs(gt_cf), j
    assert well_posed >= 2


@pytest.mark.parametrize("team,total", [(1, 0), (1, 5), (3, 0), (5, 40), (7, 21), (12, 0)])
def test_batched_odd_team_sizes(solver, team, total):
    """Teams whose workgroups spread unevenly over the XCDs (the team barrier
    groups a team's workgroups by the XCD they run on): every instance of an
    uneven batch converges and agrees with its single solve to the parity bar,
    whatever the team size and number of teams (the item shape, and so the
    last bits, may differ from the single solve's)."""
    insts = [W.dct_instance(n, n // 4, max(2, n // 100), seed=900 + i)
             for i, n in enumerate([1024, 4096, 2048, 8192, 512, 4096, 1024, 2048, 16384])]
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    rows = np.concatenate([i.rows for i in insts])
    b = np.concatenate([i.b for i in insts])
    say(f"odd teams: team={team} workgroups={total}")
    solver.set_launch(total, team, 0)
    try:
        res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, rows=rows)
    finally:
        solver.set_launch(0, 0, 0)
    xb = res.x.cpu().numpy()
    for j, inst in enumerate(insts):
        r1 = solver.solve(inst.b, inst.tau, rows=inst.rows, n=inst.n)
        x1 = r1.x.cpu().numpy()
        assert res.infos[j]["status"] == 0, (j, res.infos[j])
        assert np.linalg.norm(x1 - xb[n_off[j]:n_off[j + 1]]) <= 1e-6 * (1.0 + np.linalg.norm(x1)), j
