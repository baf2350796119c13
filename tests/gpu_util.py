"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
from __future__ import annotations

import numpy as np

from oracle import mfipm_ref as R

# Parity bar: ||x_gpu - x_cpu|| / ||x_cpu|| <= 1e-6 at IPM tol 1e-8, KKT <= 1e-6,
# IPM iteration counts within +-1 of the oracle.
X_REL = 1e-6
KKT_TOL = 1e-6
ITER_SLACK = 1


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


def check_against_oracle(op, b, tau, x_gpu, info, state=None, params=None, label=""):
    """Runs the oracle on the same inputs and applies the parity bar."""
    ref = R.solve(op, b, tau, params)
    assert info["status"] == ref.status, (label, info, R.STATUS_NAMES[ref.status])
    assert abs(info["ipm_iters"] - ref.ipm_iters) <= ITER_SLACK, (label, info["ipm_iters"], ref.ipm_iters)
    xg = np.asarray(x_gpu)
    if np.max(np.abs(ref.x)) <= 1e-8 * (1 + np.max(np.abs(b))):
        # degenerate x* = 0: absolute gate
        assert np.max(np.abs(xg)) <= 1e-8 * (1 + np.max(np.abs(b))), label
    elif rel(xg, ref.x) > X_REL:
        # The gap test only fixes x to O(gap): when the objective is tiny the
        # tolerance leaves x loose.  Then both answers are compared with a
        # tightly converged oracle solution; the GPU's may be no farther from
        # it than twice the oracle's own distance (plus the bar).
        tight = R.solve(op, b, tau, R.Params(tol=1e-12, tolpcg=1e-8, mxiterpcg=2000))
        d_ref = rel(ref.x, tight.x)
        d_gpu = rel(xg, tight.x)
        assert d_ref > X_REL / 10, (label, "tolerance determines x, yet GPU differs", rel(xg, ref.x))
        assert d_gpu <= 2 * d_ref + X_REL, (label, d_gpu, d_ref)
    if ref.status == R.CONVERGED:
        if state is not None:
            n = op.n
            st = np.asarray(state)
            z = st[: 2 * n].reshape(n, 2).T.reshape(-1)   # interleaved (u,v) -> [u; v]
            s = st[2 * n:].reshape(n, 2).T.reshape(-1)
            S, sg = R.support_from_state(z, s, n)
        else:
            S, sg = R.support_from_state(ref.z, ref.s, op.n)
        kkt = R.kkt_residual(op, b, tau, xg, S, sg)
        kkt_ref = R.kkt_residual(op, b, tau, ref.x, *R.support_from_state(ref.z, ref.s, op.n))
        assert kkt <= max(KKT_TOL, 10 * kkt_ref), (label, kkt, kkt_ref)
    return ref
