"""Per-instance oracle comparisons run in host worker processes (see
oracle/pool.py), so that every instance of the full-size batches is checked
against the oracle at the strict bar within the test's time."""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

import workloads as W
from oracle import mfipm_ref as R
from tests import gpu_util as U


def batched_dense_instance(i, n, x, state, info):
    """Instance i of the uneven dense batch: oracle solve and the strict bar.
    Returns (i, oracle IPM iterations, GPU IPM iterations, rel(x))."""
    inst = W.batched_dense_instance(i, n)
    op = R.DenseOperator(inst.A)
    ref = U.check_against_oracle(op, inst.b, inst.tau, x, info, state, label=f"batched_dense[{i}] n={n}",
                                 strict=True)
    return i, ref.ipm_iters, info["ipm_iters"], U.rel(x, ref.x)


_DCT = {}


def _dct_batch(n, batch):
    key = (n, batch)
    if key not in _DCT:
        _DCT[key] = W.config_dct_batch(n=n, batch=batch)
    return _DCT[key]


def grad_signal(j, n, batch, x, state, info, grad_b, grad_tau, binfo):
    """Signal j of the shared partial-DCT batch: forward x at the strict bar;
    the adjoint against the oracle's adjoint at the GPU's own final point
    (1e-8) and against the closed form on the GPU's support (1e-5), where x_S
    is affine in (b, tau): dL/db = A_S (A_S^T A_S)^{-1} (x_S - xt_S),
    dL/dtau = -sign_S^T (A_S^T A_S)^{-1} (x_S - xt_S), solved by CG through
    the DCT.  Returns the measured errors."""
    inst = _dct_batch(n, batch)
    op = R.PartialDCTOperator(inst.n, inst.rows)
    U.check_against_oracle(op, inst.b[j], inst.tau[j], x, info, state, label=f"grad[{j}]", strict=True)
    assert binfo["status"] == 0, (j, binfo)
    z, s = U.zs_from_state(state, n)
    gx = x - inst.x_true[j]
    ref = R.backward(op, z, s, gx)
    eb = U.rel(grad_b, ref.grad_b)
    et = abs(grad_tau - ref.grad_tau) / abs(ref.grad_tau)
    assert eb <= 1e-8 and et <= 1e-8, (j, eb, et)
    S, sg = R.support_from_state(z, s, n)

    def AS(v):
        full = np.zeros(n)
        full[S] = v
        return op.matvec(full)
    G = sla.LinearOperator((len(S), len(S)), matvec=lambda v: op.rmatvec(AS(v))[S], dtype=np.float64)
    v, cg_info = sla.cg(G, gx[S], rtol=1e-13, maxiter=5000)
    assert cg_info == 0, (j, cg_info)
    gb_cf = AS(v)
    gt_cf = -float(sg @ v)
    eb_cf = U.rel(grad_b, gb_cf)
    et_cf = abs(grad_tau - gt_cf) / abs(gt_cf)
    assert eb_cf <= 1e-5 and et_cf <= 1e-5, (j, eb_cf, et_cf)
    return j, eb, et, eb_cf, et_cf, len(S)


def shared_dense_signal(j, x, state, info, batch):
    """Signal j of the shared-dense batch (A drawn again from its seed):
    oracle solve and the strict bar."""
    inst = W.config_shared_dense(batch=batch, signals=[j])
    op = R.DenseOperator(inst.A)
    ref = U.check_against_oracle(op, inst.b[0], inst.tau[0], x, info, state, label=f"shared_dense[{j}]",
                                 strict=True)
    return j, ref.ipm_iters, info["ipm_iters"], U.rel(x, ref.x)


def phase_instance(n, rows, b, tau, x_true, x_gpu, info):
    """One phase-transition instance: the oracle's solve at the sweep's
    parameters.  Returns (oracle status, oracle IPM iterations, oracle r.e.,
    GPU r.e., rel(x_gpu, x_oracle))."""
    op = R.PartialDCTOperator(n, rows)
    ref = R.solve(op, b, tau, R.Params(**W.PHASE_PARAMS))
    re_o = float(np.linalg.norm(ref.x - x_true) / np.linalg.norm(x_true))
    re_g = float(np.linalg.norm(x_gpu - x_true) / np.linalg.norm(x_true))
    return ref.status, ref.ipm_iters, re_o, re_g, U.rel(x_gpu, ref.x)
