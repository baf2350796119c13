"""The direct-solver variant (GPU): the IPM with exact Newton directions from
a Cholesky factorisation (params.direct = 1, Section 5.7) against the
oracle's direct variant (Cholesky of the explicit 2n system), on the Section
5.7 comparison problems (n = 2^5 .. 2^11, m = n/4, noiseless, tau = 1e-3),
on lengths that are not multiples of the 64-wide tiles, in a batch of uneven
instances, and its argument checks."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mfipm_ref as R
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

DIRECT = R.Params(direct=1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver(gpu_lib):
    from paper_1208_5435_amd import Solver
    s = Solver(params=dict(direct=1))
    yield s
    s.close()


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


@pytest.mark.parametrize("n", W.DIRECT_SCALING_NS[:7])
def test_direct_section57_problems(solver, n):
    inst = W.direct_scaling_instance(n)
    say(f"direct n={n} m={inst.m}")
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    ref = U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                                 res.state.cpu().numpy(), params=DIRECT, label=f"direct n={n}",
                                 resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))
    assert res.infos[0]["pcg_iters"] == 0
    say(f"  gpu {res.infos[0]['ipm_iters']} IPM ({res.infos[0]['correctors']} corr) {res.kernel_ms:.2f} ms, "
        f"oracle {ref.ipm_iters}")


@pytest.mark.parametrize("m,n,k,seed", [(16, 40, 2, 1), (40, 200, 4, 2), (100, 1000, 10, 4), (128, 129, 3, 5),
                                        (300, 1500, 20, 6)])
def test_direct_ragged_lengths(solver, m, n, k, seed):
    """n not a multiple of 64: the padded tiles carry the identity."""
    inst = W.dense_instance(m, n, k, seed=seed, amp="normal", sigma=1e-3, c_tau=1e-2)
    say(f"direct ragged m={m} n={n}")
    res = solver.solve(inst.b, inst.tau, A=inst.A)
    U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, res.x.cpu().numpy(), res.infos[0],
                           res.state.cpu().numpy(), params=DIRECT, label=f"direct {m}x{n}",
                           resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


def test_direct_batched_uneven(solver):
    """Instances of different sizes in one launch, one team each."""
    ns = [64, 320, 128, 1024, 96, 512]
    insts = [W.dense_instance(n // 4, n, max(1, n // 50), seed=900 + i, amp="normal", sigma=1e-3, c_tau=1e-2)
             for i, n in enumerate(ns)]
    say("direct batch", ns)
    n_off = _offsets([i.n for i in insts])
    m_off = _offsets([i.m for i in insts])
    a_off = _offsets([i.m * i.n for i in insts])
    A = np.concatenate([i.A.reshape(-1) for i in insts])
    b = np.concatenate([i.b for i in insts])
    res = solver.solve_batched(b, [i.tau for i in insts], n_off, m_off, A_packed=A, a_off=a_off)
    x = res.x.cpu().numpy()
    st = res.state.cpu().numpy()
    for j, inst in enumerate(insts):
        U.check_against_oracle(R.DenseOperator(inst.A), inst.b, inst.tau, x[n_off[j]:n_off[j + 1]], res.infos[j],
                               st[4 * n_off[j]:4 * n_off[j + 1]], params=DIRECT, label=f"direct batch {j}",
                               resolve=U.resolver(solver, b=inst.b, tau=inst.tau, A=inst.A))


def test_direct_matches_tight_pcg(gpu_lib):
    """Exact and inexact Newton directions reach the same minimiser: the
    direct variant's x against the PCG variant's at tolerance 1e-12."""
    from paper_1208_5435_amd import Solver
    inst = W.direct_scaling_instance(1024)
    with_d = Solver(params=dict(direct=1, tol=1e-12))
    with_p = Solver(params=dict(tol=1e-12, tolpcg=1e-8, mxiterpcg=2000))
    try:
        rd = with_d.solve(inst.b, inst.tau, A=inst.A)
        rp = with_p.solve(inst.b, inst.tau, A=inst.A)
    finally:
        with_d.close()
        with_p.close()
    assert rd.infos[0]["status"] == rp.infos[0]["status"] == 0
    assert U.rel(rd.x.cpu().numpy(), rp.x.cpu().numpy()) <= 1e-6
    say(f"direct {rd.infos[0]['ipm_iters']} IPM, pcg {rp.infos[0]['ipm_iters']} IPM")


def test_direct_argument_checks(solver):
    from paper_1208_5435_amd import MfipmError
    d = W.dct_instance(1024, 256, 10, seed=8)
    with pytest.raises(MfipmError) as e:
        solver.solve(d.b, d.tau, rows=d.rows, n=d.n)
    assert e.value.code == -1
    rng = np.random.default_rng(3)
    A = rng.standard_normal((8, 8192 + 64))
    with pytest.raises(MfipmError) as e:
        solver.solve(rng.standard_normal(8), 0.1, A=A)
    assert e.value.code == -1


def test_direct_noalloc_matches_solve(solver):
    """The no-allocation entry point with exact Newton directions: the
    factorisation's matrices fit the static scratch at this size."""
    import torch
    inst = W.direct_scaling_instance(512)
    ref = solver.solve(inst.b, inst.tau, A=inst.A)
    dev = solver.device
    A = torch.as_tensor(inst.A, dtype=torch.float64, device=dev)
    b = torch.as_tensor(inst.b, dtype=torch.float64, device=dev)
    x = torch.empty(inst.n, dtype=torch.float64, device=dev)
    info = solver.solve_noalloc(b, inst.tau, x, A=A)
    assert info["status"] == ref.infos[0]["status"] == 0
    assert abs(info["ipm_iters"] - ref.infos[0]["ipm_iters"]) <= U.ITER_SLACK
    assert U.rel(x.cpu().numpy(), ref.x.cpu().numpy()) <= U.X_REL
