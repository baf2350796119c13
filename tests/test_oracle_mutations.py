"""Planted mistakes in the CPU oracle must be caught by at least one pin.

Each case monkeypatches one oracle function with a plausible slip (a sign,
a dropped term, a transposed operand) and checks that the pin meant to guard
that function now reports an error far above its pass threshold.
"""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import mfipm_ref as R
from tests import oracle_pins as PIN


def _tiny():
    return PIN.dense_problem(5, 8, 2, seed=101, sigma=0.05, c_tau=0.1)


def _small_ops():
    rng = PIN.rng_for(31)
    n = 32
    return [R.DenseOperator(rng.standard_normal((8, n)) / math.sqrt(8)),
            R.PartialDCTOperator(n, np.sort(rng.choice(n, 8, replace=False)))]


def _newton_sign_flip(op, theta_inv, p):
    n = op.n
    d = p[:n] + p[n:]          # slip: u + v instead of u - v
    t = op.rmatvec(op.matvec(d))
    return theta_inv * p + np.concatenate([t, -t])


def _newton_block_sign(op, theta_inv, p):
    n = op.n
    d = p[:n] - p[n:]
    t = op.rmatvec(op.matvec(d))
    return theta_inv * p + np.concatenate([t, t])   # slip: lost minus sign


def _precond_no_rho_cross(theta_inv, rho, r):
    n = r.shape[0] // 2
    tu, tv = theta_inv[:n], theta_inv[n:]
    ru, rv = r[:n], r[n:]
    det = tu * tv + rho * (tu + tv)
    return np.concatenate([((tv + rho) * ru) / det, ((tu + rho) * rv) / det])  # slip: dropped rho r


def _gap_without_half(b, tau, r, g, primal):
    ginf = float(np.max(np.abs(g)))
    theta = 1.0 if ginf <= tau else tau / ginf
    nu = theta * r
    dual = -float(nu @ nu) - float(b @ nu)   # slip: dropped 1/2
    return (primal - dual) / (1.0 + abs(primal)), dual


def _objective_wrong_split(op, b, tau, z):
    n = op.n
    x = z[:n] + z[n:]                        # slip: x = u + v
    r = op.matvec(x) - b
    g = op.rmatvec(r)
    return x, r, g, tau * float(np.sum(z)) + 0.5 * float(r @ r)


def test_newton_sign_slip_caught(monkeypatch):
    monkeypatch.setattr(R, "newton_apply", _newton_sign_flip)
    assert max(PIN.pin_newton_blocks(op, 4) for op in _small_ops()) > 1e-3


def test_newton_block_sign_caught(monkeypatch):
    monkeypatch.setattr(R, "newton_apply", _newton_block_sign)
    assert max(PIN.pin_newton_blocks(op, 4) for op in _small_ops()) > 1e-3
    A, b, tau, _ = _tiny()
    try:
        err = PIN.pin_brute_force(A, b, tau)
    except AssertionError:
        err = math.inf
    assert err > 1e-3


def test_preconditioner_slip_caught(monkeypatch):
    monkeypatch.setattr(R, "precond_solve", _precond_no_rho_cross)
    assert max(PIN.pin_newton_blocks(op, 4) for op in _small_ops()) > 1e-3


def test_dual_half_slip_caught(monkeypatch):
    monkeypatch.setattr(R, "relative_gap", _gap_without_half)
    A, b, tau, _ = _tiny()
    assert PIN.pin_duality(A, b, tau) > 1e-3


def test_split_slip_caught(monkeypatch):
    monkeypatch.setattr(R, "objective_terms", _objective_wrong_split)
    A, b, tau, _ = _tiny()
    try:
        err = PIN.pin_brute_force(A, b, tau)
    except AssertionError:
        err = math.inf
    assert err > 1e-3


def test_dct_transposed_slip_caught(monkeypatch):
    def bad_matvec(self, x):
        return scipy.fft.dct(x, type=3, norm="ortho")[self.rows]  # slip: DCT-III rows
    monkeypatch.setattr(R.PartialDCTOperator, "matvec", bad_matvec)
    assert PIN.pin_dct_definition(64, 16, seed=64) > 1e-3


def test_dct_unnormalised_slip_caught(monkeypatch):
    def bad_rmatvec(self, y):
        full = np.zeros(self.n)
        full[self.rows] = y
        return scipy.fft.idct(full, type=2)      # slip: not orthonormal
    monkeypatch.setattr(R.PartialDCTOperator, "rmatvec", bad_rmatvec)
    assert PIN.pin_dct_definition(64, 16, seed=64) > 1e-3


def test_gradient_sign_slip_caught(monkeypatch):
    orig = R.backward

    def bad_backward(*a, **k):
        g = orig(*a, **k)
        g.grad_tau = -g.grad_tau                  # slip: dL/dtau = +1^T w
        return g
    monkeypatch.setattr(R, "backward", bad_backward)
    A, b, tau, xt = PIN.dense_problem(40, 120, 4, seed=55, sigma=1e-3, c_tau=5e-2)
    assert PIN.pin_gradient(A, b, tau, xt) > 1e-3


@pytest.mark.parametrize("field,value", [("sigma1", 0.2), ("alpha_tilde", 0.3)])
def test_parameter_slip_caught(field, value):
    """A wrong default is caught by the golden parameter file."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_params.json")) as f:
        gold = json.load(f)["values"]
    assert gold[field]["value"] != value


def test_rho_denominator_slip_caught(monkeypatch):
    """rho = ||A||_F^2 / m instead of / n."""
    def bad_frob2(self):
        return float(np.sum(self.A * self.A)) * self.n / self.m
    monkeypatch.setattr(R.DenseOperator, "frob2", bad_frob2)
    A, b, tau, _ = PIN.dense_problem(12, 48, 2, seed=41)
    assert PIN.pin_rho(R.DenseOperator(A), b, tau) > 1e-3


def test_rho_unsquared_slip_caught(monkeypatch):
    """Frobenius norm instead of its square."""
    def bad_frob2(self):
        return float(np.sqrt(np.sum(self.A * self.A)))
    monkeypatch.setattr(R.DenseOperator, "frob2", bad_frob2)
    A, b, tau, _ = PIN.dense_problem(12, 48, 2, seed=42)
    assert PIN.pin_rho(R.DenseOperator(3.0 * A), b, tau) > 1e-3


def test_rho_dct_slip_caught(monkeypatch):
    """A partial DCT whose rho ignores the sampled rows (rho = 1)."""
    monkeypatch.setattr(R.PartialDCTOperator, "frob2", lambda self: float(self.n))
    rng = PIN.rng_for(41)
    op = R.PartialDCTOperator(48, np.sort(rng.choice(48, 12, replace=False)))
    assert PIN.pin_rho(op, rng.standard_normal(12), 0.1) > 1e-3


def _kkt_no_offsupport(op, b, tau, x, support=None, signs=None):
    g = op.rmatvec(op.matvec(x) - b)
    on = float(np.max(np.abs(g[support] + tau * signs))) if len(support) else 0.0
    return on / tau                     # slip: dropped the |g_i| <= tau term


def _kkt_sign(op, b, tau, x, support=None, signs=None):
    g = op.rmatvec(op.matvec(x) - b)
    viol = float(np.max(np.maximum(np.abs(g) - tau, 0.0)))
    on = float(np.max(np.abs(g[support] - tau * signs))) if len(support) else 0.0   # slip: sign
    return max(viol, on) / tau


def _kkt_unscaled(op, b, tau, x, support=None, signs=None):
    g = op.rmatvec(op.matvec(x) - b)
    viol = float(np.max(np.maximum(np.abs(g) - tau, 0.0)))
    on = float(np.max(np.abs(g[support] + tau * signs))) if len(support) else 0.0
    return max(viol, on)                 # slip: not relative to tau


def _kkt_zero(op, b, tau, x, support=None, signs=None):
    return 0.0                           # slip: a residual that never reports


@pytest.mark.parametrize("bad", [_kkt_no_offsupport, _kkt_sign, _kkt_unscaled, _kkt_zero])
def test_kkt_residual_slip_caught(monkeypatch, bad):
    monkeypatch.setattr(R, "kkt_residual", bad)
    assert PIN.pin_kkt_handbuilt() > 1e-3


def test_back_substitution_slip_caught(monkeypatch):
    """du = (r_u + r_v + tu d) / (tu + tv): the wrong diagonal."""
    def bad(theta_inv, rhs, d):
        n = rhs.shape[0] // 2
        tu, tv = theta_inv[:n], theta_inv[n:]
        du = (rhs[:n] + rhs[n:] + tu * d) / (tu + tv)
        return np.concatenate([du, du - d])
    monkeypatch.setattr(R, "back_substitute", bad)
    assert PIN.pin_reduced_direction(_small_ops()[0], seed=5) > 1e-3


def test_reduced_rhs_slip_caught(monkeypatch):
    """The reduced right-hand side with a sign slip."""
    def bad(theta_inv, rhs):
        n = rhs.shape[0] // 2
        tu, tv = theta_inv[:n], theta_inv[n:]
        return tu * tv / (tu + tv), (tv * rhs[:n] + tu * rhs[n:]) / (tu + tv)
    monkeypatch.setattr(R, "reduced_system", bad)
    assert PIN.pin_reduced_direction(_small_ops()[1], seed=5) > 1e-3


def test_wht_ordering_slip_caught(monkeypatch):
    """A transform in the wrong order (pairs combined as (a - b, a + b))."""
    def bad_fwht(x):
        y = np.array(x, dtype=np.float64, copy=True)
        n = y.shape[0]
        h = 1
        while h < n:
            y = y.reshape(-1, 2, h)
            a = y[:, 0, :].copy()
            b = y[:, 1, :]
            y = np.stack([a - b, a + b], axis=1).reshape(n)
            h *= 2
        return y
    monkeypatch.setattr(R, "fwht", bad_fwht)
    assert PIN.pin_wht_definition(64, 16, seed=67) > 1e-3


def test_dst_type_slip_caught(monkeypatch):
    """A DST-I in place of the DST-II is caught by the sine-sum pin."""
    real_dst = R.scipy.fft.dst

    def bad_dst(x, type=2, norm=None):
        return real_dst(x, type=1, norm=norm)

    monkeypatch.setattr(R.scipy.fft, "dst", bad_dst)
    assert PIN.pin_dst_definition(64, 16, seed=69) > 1e-3
