"""The noiseless regime (GPU): b = A x_true exactly, tau from the paper's
table of regularisation parameters for noiseless problems (1e-10 to 1e-2,
Section 5.4, Table regparams), tol 1e-14 and tolpcg 1e-6 (the ends of the
noiseless ranges in Section 5.4).  The oracle runs first on the same inputs;
the GPU must reproduce its status (including MAXITER where the gap stalls
above 1e-14), its IPM iteration count within +-1 and its x to 1e-6."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mfipm_ref as R
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

PRM = dict(tol=1e-14, tolpcg=1e-6)
DEFAULTS = dict(tol=1e-8, tolpcg=1e-2)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver(gpu_lib):
    from paper_1208_5435_amd import Solver
    s = Solver()
    yield s
    s.close()


def _case(name):
    if name == "dense256x1024":
        inst = W.dense_instance(256, 1024, 20, seed=120801, amp="pm1", sigma=0.0, c_tau=1e-2)
        return R.DenseOperator(inst.A), inst.b, inst.x_true, dict(A=inst.A)
    n = int(name[4:])
    inst = W.dct_instance(n, n // 4, n // 100, seed=777 + n, amp="normal", sigma=0.0, c_tau=1e-2)
    return R.PartialDCTOperator(n, inst.rows), inst.b, inst.x_true, dict(rows=inst.rows, n=n)


@pytest.mark.parametrize("name", ["dense256x1024", "pdct4096", "pdct65536"])
@pytest.mark.parametrize("tau", [1e-10, 1e-6, 1e-2])
def test_noiseless(solver, name, tau):
    op, b, xt, kw = _case(name)
    ref = R.solve(op, b, tau, R.Params(**PRM))
    say(f"noiseless {name} tau={tau:g}: oracle {R.STATUS_NAMES[ref.status]} {ref.ipm_iters} IPM "
        f"{ref.pcg_iters} PCG, rel gap {ref.rel_gap:.1e}")
    solver.set_params(**PRM)
    try:
        res = solver.solve(b, tau, **kw)
    finally:
        solver.set_params(**DEFAULTS)
    info = res.infos[0]
    x = res.x.cpu().numpy()
    say(f"   gpu {info['status_name']} {info['ipm_iters']} IPM {info['pcg_iters']} PCG, rel gap "
        f"{info['rel_gap']:.1e}; rel(x) {U.rel(x, ref.x):.2e}; recovery error {U.rel(x, xt):.1e}")
    assert info["status"] == ref.status, (info, ref.status)
    assert abs(info["ipm_iters"] - ref.ipm_iters) <= U.ITER_SLACK
    assert U.rel(x, ref.x) <= U.X_REL
    z, s = U.zs_from_state(res.state.cpu().numpy(), op.n)
    kkt_gpu = U.kkt_of(op, b, tau, x, z, s)
    kkt_ref = U.kkt_of(op, b, tau, ref.x, ref.z, ref.s)
    if kkt_ref <= U.KKT_TOL:
        assert kkt_gpu <= U.KKT_TOL, (kkt_gpu, kkt_ref)
    else:
        # with tau ~ 1e-10 a residual relative to tau says little: the
        # gradient itself is ~1e-11
        say(f"   oracle KKT {kkt_ref:.1e} > {U.KKT_TOL}; GPU {kkt_gpu:.1e} gated at twice the oracle's")
        assert kkt_gpu <= 2.0 * kkt_ref
