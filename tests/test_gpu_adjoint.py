"""The adjoint (GPU): central finite differences of the solve map, and the
status paths of the adjoint solve."""
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


TIGHT14 = dict(tol=1e-14, tolpcg=1e-10, mxiterpcg=5000, maxiters=200)
DEFAULTS = dict(tol=1e-8, tolpcg=1e-2, mxiterpcg=200, maxiters=100, tolpcg_adj=1e-12, mxiterpcg_adj=1000)


def test_adjoint_vs_central_fd():
    """Shape of the differentiation workload scaled to n = 2^12 (m = n/4,
    k = n/100, sigma = 1e-2, tau = 5e-3 ||A^T b||_inf), solved to relative
    gap 1e-14 so that solver noise is far below the h = 1e-6 differences.
    x* is affine in (b, tau) on a fixed support, so central differences are
    exact up to that noise: directional dL/db . d and dL/dtau from the GPU
    adjoint against central differences of GPU solves, to 1e-5 (the oracle
    reaches ~1e-8 on this instance)."""
    from paper_1208_5435_amd import Solver
    n = 1 << 12
    inst = W.config_dct_batch(n=n, batch=2)
    m = inst.m
    b0, tau0, xt = inst.b[0], float(inst.tau[0]), inst.x_true[0]
    d = inst.extra["fd_direction"][0]
    s = Solver(params=TIGHT14)
    try:
        r0 = s.solve(b0, tau0, rows=inst.rows, n=n)
        assert r0.infos[0]["status"] == 0, r0.infos[0]
        x0 = r0.x.cpu().numpy()
        gb, gt, binf = s.backward(r0.state, x0 - xt, np.array([0, n], np.int64), np.array([0, m], np.int64),
                                  rows=inst.rows)
        assert binf[0]["status"] == 0, binf[0]
        an_b = float(gb.cpu().numpy() @ d)
        an_t = float(gt.cpu().numpy()[0])

        def loss(bb, tt):
            rr = s.solve(bb, tt, rows=inst.rows, n=n)
            assert rr.infos[0]["status"] == 0, rr.infos[0]
            return 0.5 * float(np.sum((rr.x.cpu().numpy() - xt) ** 2))
        h = 1e-6
        fd_b = (loss(b0 + h * d, tau0) - loss(b0 - h * d, tau0)) / (2 * h)
        ht = h * tau0
        fd_t = (loss(b0, tau0 + ht) - loss(b0, tau0 - ht)) / (2 * ht)
    finally:
        s.close()
    eb = abs(fd_b - an_b) / abs(an_b)
    et = abs(fd_t - an_t) / abs(an_t)
    say(f"FD n={n} tol 1e-14 h=1e-6: dL/db.d adjoint {an_b:.10e} fd {fd_b:.10e} rel {eb:.2e}; "
        f"dL/dtau adjoint {an_t:.10e} fd {fd_t:.10e} rel {et:.2e}")
    assert eb <= 1e-5, eb
    assert et <= 1e-5, et
    # and the GPU adjoint against the oracle's adjoint at the GPU's final point
    op = R.PartialDCTOperator(n, inst.rows)
    z, sv = U.zs_from_state(r0.state.cpu().numpy(), n)
    ref = R.backward(op, z, sv, x0 - xt)
    assert U.rel(gb.cpu().numpy(), ref.grad_b) <= 1e-8
    assert abs(an_t - ref.grad_tau) <= 1e-8 * abs(ref.grad_tau)


def test_adjoint_cap_is_reported(solver):
    """An adjoint PCG stopped by its iteration cap reports PCG_MAXITER, and
    the autograd wrapper refuses to return such a gradient."""
    import torch
    from paper_1208_5435_amd.autograd import MfipmSolve, SolveStatusError
    inst = W.dct_instance(1024, 256, 10, seed=71, sigma=1e-2, c_tau=2e-2)
    n, m = inst.n, inst.m
    res = solver.solve(inst.b, inst.tau, rows=inst.rows, n=n)
    solver.set_params(mxiterpcg_adj=1)
    try:
        gb, gt, binf = solver.backward(res.state, res.x.cpu().numpy() - inst.x_true, np.array([0, n], np.int64),
                                       np.array([0, m], np.int64), rows=inst.rows)
        assert binf[0]["status"] == 7 and binf[0]["status_name"] == "PCG_MAXITER", binf[0]
        assert binf[0]["pcg_iters"] == 1
        assert np.all(np.isfinite(gb.cpu().numpy()))
        dev = solver.device
        b = torch.tensor(inst.b, device=dev, requires_grad=True)
        tau = torch.tensor(inst.tau, device=dev, dtype=torch.float64, requires_grad=True)
        x = MfipmSolve.apply(b, tau, solver, None, torch.tensor(inst.rows, device=dev), n)
        loss = 0.5 * (x ** 2).sum()
        with pytest.raises(SolveStatusError):
            loss.backward()
    finally:
        solver.set_params(**DEFAULTS)


def test_adjoint_breakdown_gives_nan(solver):
    """A state with s = -z makes Theta^{-1} = -1, so p^T H p turns
    non-positive and the adjoint PCG breaks down (the oracle's does too); the
    instance's gradients are then NaN, never stale memory."""
    n, m = 256, 64
    inst = W.dct_instance(n, m, 3, seed=72)
    z = np.ones(2 * n)
    s = -np.ones(2 * n)
    state = np.concatenate([np.stack([z[:n], z[n:]], 1).reshape(-1), np.stack([s[:n], s[n:]], 1).reshape(-1)])
    gx = np.random.default_rng(3).standard_normal(n)
    ref = R.backward(R.PartialDCTOperator(n, inst.rows), z, s, gx)
    assert ref.status == R.PCG_BREAKDOWN
    import torch
    st = torch.tensor(state, device=solver.device)
    gb, gt, binf = solver.backward(st, gx, np.array([0, n], np.int64), np.array([0, m], np.int64), rows=inst.rows)
    assert binf[0]["status"] == 2, binf[0]
    assert np.all(np.isnan(gb.cpu().numpy()))
    assert np.isnan(float(gt.cpu()[0]))
