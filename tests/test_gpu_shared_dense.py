"""Many signals through one dense A (GPU): the lock-step path, whose operator
is two FP64 MFMA matrix products per round, against the oracle signal by
signal, against the per-instance batched path, and at the full size of the
shared-matrix workload (256 signals, A 2048 x 8192)."""
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


def _run(solver, inst, team=0):
    B = inst.b.shape[0]
    n_off = np.arange(B + 1, dtype=np.int64) * inst.n
    m_off = np.arange(B + 1, dtype=np.int64) * inst.m
    solver.set_launch(0, team, 0)
    try:
        return solver.solve_batched(inst.b.reshape(-1), inst.tau, n_off, m_off, A_packed=inst.A, shared_op=True)
    finally:
        solver.set_launch(0, 0, 0)


@pytest.mark.parametrize("m,n,B", [(128, 512, 24), (100, 300, 9), (64, 256, 70), (101, 300, 9)])
def test_lockstep_vs_oracle(solver, m, n, B):
    """Ragged shapes: m, n not multiples of the 64 x 64 tiles or the 32-wide
    K chunks; B not a multiple of the 64-signal column groups."""
    inst = W.config_shared_dense(m=m, n=n, batch=B, seed=7000 + n)
    say(f"lock-step m={m} n={n} B={B}")
    res = _run(solver, inst)
    x = res.x.cpu().numpy().reshape(B, n)
    st = res.state.cpu().numpy().reshape(B, 4 * n)
    op = R.DenseOperator(inst.A)
    for j in range(B):
        U.check_against_oracle(op, inst.b[j], inst.tau[j], x[j], res.infos[j], st[j], label=f"ls {m}x{n} [{j}]",
                               resolve=U.resolver(solver, b=inst.b[j], tau=float(inst.tau[j]), A=inst.A))


def test_lockstep_equals_team_path(solver):
    """The same batch through the lock-step path and the per-instance team
    path (forced by a team size): same statuses and iteration counts, x to
    the parity bar."""
    inst = W.config_shared_dense(m=256, n=1024, batch=16, seed=7101)
    a = _run(solver, inst)
    b = _run(solver, inst, team=4)
    xa = a.x.cpu().numpy().reshape(16, -1)
    xb = b.x.cpu().numpy().reshape(16, -1)
    for j in range(16):
        assert a.infos[j]["status"] == b.infos[j]["status"] == 0, (j, a.infos[j], b.infos[j])
        assert abs(a.infos[j]["ipm_iters"] - b.infos[j]["ipm_iters"]) <= U.ITER_SLACK
        assert U.rel(xa[j], xb[j]) <= U.X_REL, j


def test_shared_dense_256(solver):
    """256 signals sharing one 2048 x 8192 N(0, 1/2048) matrix in one
    lock-step launch: every signal converged with a gap certificate <= 1e-7
    recomputed on the host from the GPU's x; 32 signals (every 8th) against
    the oracle at the strict bar."""
    inst = W.config_shared_dense()
    B, n, m = inst.b.shape[0], inst.n, inst.m
    res = _run(solver, inst)
    say(f"shared dense 256 x (2048 x 8192): kernel {res.kernel_ms:.1f} ms, IPM iterations "
        f"{min(i['ipm_iters'] for i in res.infos)}..{max(i['ipm_iters'] for i in res.infos)}")
    assert all(i["status"] == 0 for i in res.infos), [j for j, i in enumerate(res.infos) if i["status"]]
    x = res.x.cpu().numpy().reshape(B, n)
    st = res.state.cpu().numpy().reshape(B, 4 * n)
    op = R.DenseOperator(inst.A)
    gaps = []
    for j in range(B):
        z = np.concatenate([np.maximum(x[j], 0), np.maximum(-x[j], 0)])
        _, r, g, primal = R.objective_terms(op, inst.b[j], inst.tau[j], z)
        gaps.append(R.relative_gap(inst.b[j], inst.tau[j], r, g, primal)[0])
    say(f"  largest gap certificate {max(gaps):.2e}")
    assert max(gaps) <= 1e-7
    sample = list(range(0, B, 8))
    with pool.executor() as ex:
        futs = [ex.submit(T.shared_dense_signal, j, x[j], st[j], res.infos[j], B) for j in sample]
        worst = 0.0
        for f in futs:
            j, it_ref, it_gpu, r = f.result()
            worst = max(worst, r)
    say(f"  {len(sample)} signals at the strict bar; worst rel(x) {worst:.2e}")
