"""mfipm_solve_noalloc (GPU): the entry point for callers that cannot
allocate, against mfipm_solve on the same inputs, two calls in a row with the
second one smaller, for both operators; and its size limit."""
import sys

import numpy as np
import pytest

import workloads as W
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


def _compare(solver, inst, kind, label):
    import torch
    dev = solver.device
    b = torch.from_numpy(inst.b).to(dev)
    if kind == "dense":
        A = torch.from_numpy(inst.A).to(dev)
        ref = solver.solve(b, inst.tau, A=A)
        kw = dict(A=A)
    else:
        rows = torch.from_numpy(inst.rows).to(dev)
        ref = solver.solve(b, inst.tau, rows=rows, n=inst.n)
        kw = dict(rows=rows, n=inst.n)
    x = torch.full((inst.n,), float("nan"), dtype=torch.float64, device=dev)
    st = torch.full((4 * inst.n,), float("nan"), dtype=torch.float64, device=dev)
    info = solver.solve_noalloc(b, inst.tau, x, st, **kw)
    xr, xn = ref.x.cpu().numpy(), x.cpu().numpy()
    r = U.rel(xn, xr)
    say(f"{label}: solve {ref.infos[0]['status_name']} {ref.infos[0]['ipm_iters']} IPM; noalloc "
        f"{info['status_name']} {info['ipm_iters']} IPM; rel(x) {r:.2e}; bitwise {np.array_equal(xn, xr)}")
    assert info["status"] == ref.infos[0]["status"] == 0
    assert abs(info["ipm_iters"] - ref.infos[0]["ipm_iters"]) <= U.ITER_SLACK
    assert r <= U.X_REL
    assert U.rel(st.cpu().numpy(), ref.state.cpu().numpy()) <= U.X_REL


def test_noalloc_pdct_two_calls(solver):
    _compare(solver, W.config_pdct(), "pdct", "pdct n=2^16")
    _compare(solver, W.dct_instance(4096, 1024, 40, seed=81), "pdct", "pdct n=4096 (second, smaller)")


def test_noalloc_dense_two_calls(solver):
    _compare(solver, W.config_dense_256x1024(), "dense", "dense 256x1024")
    _compare(solver, W.dense_instance(64, 256, 5, seed=82), "dense", "dense 64x256 (second, smaller)")


def test_noalloc_rejects_too_large(solver):
    """Partial DCT n = 2^18 needs more than the 64 MiB scratch: refused on
    the host before any launch."""
    import torch
    from paper_1208_5435_amd import MfipmError
    n = 1 << 18
    dev = solver.device
    rows = torch.arange(0, n, 4, dtype=torch.int32, device=dev)
    b = torch.zeros(n // 4, dtype=torch.float64, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    with pytest.raises(MfipmError) as e:
        solver.solve_noalloc(b, 1.0, x, rows=rows, n=n)
    assert e.value.code == -6
