"""CPU oracle against closed forms, invariants and brute force (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mfipm_ref as R
from tests import oracle_pins as PIN

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_parameters_are_defaults():
    """Defaults equal the values the paper states (golden file cites them)."""
    with open(os.path.join(GOLDEN, "paper_params.json")) as f:
        gold = json.load(f)
    p = R.Params()
    for key, entry in gold["values"].items():
        assert getattr(p, key) == entry["value"], key
    # tol and tolpcg lie in the ranges the paper gives for noisy problems
    lo, hi = gold["ranges"]["tol_noisy"]["value"]
    assert lo <= p.tol <= hi
    lo, hi = gold["ranges"]["tolpcg_noisy"]["value"]
    assert lo <= p.tolpcg <= hi


def test_worked_constant_C():
    """Section 4: for |tau_hat| <= 17/20 with rho = 1/4 the separator constant is
    C = 20 (0.75 + delta + 2 sqrt(1+delta))^2 / 3; the paper prints ~139.74 for
    delta <= 1 and ~50.41 for delta = 0."""
    with open(os.path.join(GOLDEN, "paper_params.json")) as f:
        gold = json.load(f)["worked_constants"]
    for delta, key in ((1.0, "C_delta1"), (0.0, "C_delta0")):
        C = 20.0 * (0.75 + delta + 2.0 * math.sqrt(1.0 + delta)) ** 2 / 3.0
        assert abs(C - gold[key]["value"]) < 0.01
        # the same C makes the Lemma's bound (nearly orthonormal rows,
        # delta_l = 1/4) equal to 17/20
        rho, dl = 0.25, 0.25
        bound = dl + 0.25 * (1 + delta - rho + 2 * math.sqrt(1 + delta)) ** 2 / (rho * dl * C)
        assert abs(bound - 0.85) < 1e-12


@pytest.mark.parametrize("kind", ["dense", "dct"])
def test_zero_solution(kind):
    rng = PIN.rng_for(11)
    if kind == "dense":
        A, b, _, _ = PIN.dense_problem(24, 64, 4, seed=3)
        op = R.DenseOperator(A)
    else:
        n = 128
        rows = np.sort(rng.choice(n, 32, replace=False))
        op = R.PartialDCTOperator(n, rows)
        b = rng.standard_normal(32)
    assert PIN.pin_zero_solution(op, b) <= 1e-8


def test_identity_soft_threshold():
    rng = PIN.rng_for(5)
    n = 64
    b = rng.standard_normal(n)
    tau = 0.7
    assert PIN.pin_orthonormal_soft_threshold(R.DenseOperator(np.eye(n)), b, tau) <= 1e-7


def test_full_dct_soft_threshold():
    """All rows of the orthonormal DCT: A^T A = I, x* = soft(A^T b, tau)."""
    rng = PIN.rng_for(6)
    n = 128
    op = R.PartialDCTOperator(n, np.arange(n))
    b = rng.standard_normal(n)
    assert PIN.pin_orthonormal_soft_threshold(op, b, 0.5) <= 1e-7


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_tiny(seed):
    A, b, tau, _ = PIN.dense_problem(5, 8, 2, seed=100 + seed, sigma=0.05, c_tau=0.1)
    assert PIN.pin_brute_force(A, b, tau) <= 1e-6


@pytest.mark.parametrize("m,n,seed", [(32, 128, 1), (64, 256, 2)])
def test_kkt_dense(m, n, seed):
    A, b, tau, _ = PIN.dense_problem(m, n, max(1, n // 50), seed=seed)
    kkt8, res = PIN.pin_kkt(R.DenseOperator(A), b, tau)
    assert res.status == R.CONVERGED
    kkt, res = PIN.pin_kkt(R.DenseOperator(A), b, tau, R.Params(tol=1e-11))
    assert res.status == R.CONVERGED
    assert kkt <= 1e-7 and kkt <= kkt8


def test_kkt_dct():
    rng = PIN.rng_for(21)
    n, m = 1024, 256
    rows = np.sort(rng.choice(n, m, replace=False))
    op = R.PartialDCTOperator(n, rows)
    x = np.zeros(n)
    x[rng.choice(n, 10, replace=False)] = rng.standard_normal(10)
    b = op.matvec(x) + 1e-2 * rng.standard_normal(m)
    tau = 1e-2 * float(np.max(np.abs(op.rmatvec(b))))
    kkt, res = PIN.pin_kkt(op, b, tau, R.Params(tol=1e-11))
    assert res.status == R.CONVERGED
    assert kkt <= 1e-7


@pytest.mark.parametrize("kind", ["dense", "dct"])
def test_newton_blocks_and_theorem(kind):
    rng = PIN.rng_for(31)
    n = 32
    if kind == "dense":
        op = R.DenseOperator(rng.standard_normal((8, n)) / math.sqrt(8))
    else:
        op = R.PartialDCTOperator(n, np.sort(rng.choice(n, 8, replace=False)))
    assert PIN.pin_newton_blocks(op, seed=4) <= 1e-7


@pytest.mark.parametrize("n,m", [(64, 16), (256, 100), (1024, 256)])
def test_dct_definition(n, m):
    assert PIN.pin_dct_definition(n, m, seed=n) <= 1e-12


@pytest.mark.parametrize("n", [32, 64, 128])
def test_pcg_matches_direct_newton(n):
    """Section 5.7 setup: Gaussian A, m = n/4, k = ceil(m/20), tau = 1e-3,
    noiseless."""
    m = n // 4
    k = math.ceil(m / 20)
    rng = PIN.rng_for(n)
    A = rng.standard_normal((m, n)) / math.sqrt(m)
    x = np.zeros(n)
    x[rng.choice(n, k, replace=False)] = rng.choice([-1.0, 1.0], k)
    b = A @ x
    dit, dx = PIN.pin_pcg_vs_direct(A, b, 1e-3)
    assert dit == 0
    assert dx <= 1e-8


def test_duality_certificate():
    A, b, tau, _ = PIN.dense_problem(5, 8, 2, seed=77, sigma=0.05, c_tau=0.1)
    assert PIN.pin_duality(A, b, tau) <= 1e-10


def test_step_length_brute():
    rng = PIN.rng_for(9)
    v = np.abs(rng.standard_normal(50)) + 0.1
    dv = rng.standard_normal(50)
    a = R.max_step(v, dv)
    assert np.all(v + a * (1 - 1e-12) * dv > 0)
    assert np.min(v + a * (1 + 1e-9) * dv) < 0
    assert R.max_step(v, np.abs(dv)) == math.inf
    assert R.step_length(v, np.abs(dv), 0.995) == 1.0


def test_gradient_closed_form_dense():
    A, b, tau, xt = PIN.dense_problem(40, 120, 4, seed=55, sigma=1e-3, c_tau=5e-2)
    assert PIN.pin_gradient(A, b, tau, xt) <= 1e-5


def test_gradient_central_fd_on_support():
    """On a fixed support with fixed signs x_S is affine in (b, tau) and the
    loss is quadratic, so central differences of the closed form are exact up
    to rounding; they must agree with the closed-form gradient."""
    A, b, tau, xt = PIN.dense_problem(40, 120, 4, seed=55, sigma=1e-3, c_tau=5e-2)
    op = R.DenseOperator(A)
    res = R.solve(op, b, tau, R.Params(tol=1e-13, tolpcg=1e-10, mxiterpcg=2000))
    S, sg = R.support_from_state(res.z, res.s, op.n)
    A_S = A[:, S]

    def loss(bb, tt):
        xs = R.closed_form_on_support(A_S, bb, tt, sg)
        return 0.5 * float(np.sum((xs - xt[S]) ** 2)) + 0.5 * float(np.sum(xt[np.setdiff1d(
            np.arange(op.n), S)] ** 2))

    xs = R.closed_form_on_support(A_S, b, tau, sg)
    gb, gt = R.closed_form_gradient(A_S, sg, xs, xt[S])
    d = PIN.rng_for(56).standard_normal(b.shape[0])
    d /= np.linalg.norm(d)
    h = 1e-6
    fd = (loss(b + h * d, tau) - loss(b - h * d, tau)) / (2 * h)
    assert abs(fd - gb @ d) <= 1e-7 * max(1.0, abs(gb @ d))
    fdt = (loss(b, tau + h) - loss(b, tau - h)) / (2 * h)
    assert abs(fdt - gt) <= 1e-7 * max(1.0, abs(gt))
    # and the solver's x equals the closed form on that support
    assert np.linalg.norm(res.x[S] - xs) <= 1e-6 * np.linalg.norm(xs)


def test_backward_pcg_matches_dense():
    A, b, tau, xt = PIN.dense_problem(40, 120, 4, seed=57)
    op = R.DenseOperator(A)
    res = R.solve(op, b, tau)
    g1 = R.backward(op, res.z, res.s, res.x - xt)
    g2 = R.backward(op, res.z, res.s, res.x - xt, method="dense")
    assert np.linalg.norm(g1.grad_b - g2.grad_b) <= 1e-8 * np.linalg.norm(g2.grad_b)
    assert abs(g1.grad_tau - g2.grad_tau) <= 1e-8 * abs(g2.grad_tau)


def test_status_maxiter_and_nonfinite():
    A, b, tau, _ = PIN.dense_problem(16, 64, 2, seed=8)
    op = R.DenseOperator(A)
    r = R.solve(op, b, tau, R.Params(maxiters=1))
    assert r.status == R.MAXITER and r.ipm_iters == 1
    bb = b.copy()
    bb[0] = np.nan
    r = R.solve(op, bb, tau)
    assert r.status == R.NONFINITE


@pytest.mark.parametrize("kind", ["dense", "dct", "scaled"])
def test_rho_is_frobenius_closest(kind):
    rng = PIN.rng_for(41)
    n = 48
    if kind == "dense":
        A, b, tau, _ = PIN.dense_problem(12, n, 2, seed=41)
        op = R.DenseOperator(A)
    elif kind == "scaled":  # rows far from orthonormal: rho must follow ||A||_F
        A, b, tau, _ = PIN.dense_problem(12, n, 2, seed=42)
        op = R.DenseOperator(3.0 * A)
    else:
        op = R.PartialDCTOperator(n, np.sort(rng.choice(n, 12, replace=False)))
        b = rng.standard_normal(12)
        tau = 0.1
    assert PIN.pin_rho(op, b, tau) <= 1e-9
    if kind == "dct":
        assert R.solve(op, b, tau, R.Params(maxiters=1)).rho == 12 / n


def test_kkt_residual_handbuilt():
    assert PIN.pin_kkt_handbuilt() <= 1e-12


@pytest.mark.parametrize("kind", ["dense", "dct"])
def test_reduced_direction_is_the_newton_direction(kind):
    rng = PIN.rng_for(51)
    n = 40
    if kind == "dense":
        op = R.DenseOperator(rng.standard_normal((12, n)) / math.sqrt(12))
    else:
        op = R.PartialDCTOperator(n, np.sort(rng.choice(n, 12, replace=False)))
    assert PIN.pin_reduced_direction(op, seed=5) <= 1e-9


@pytest.mark.parametrize("n", [32, 64])
def test_reduced_pcg_matches_direct_newton(n):
    m = n // 4
    rng = PIN.rng_for(n + 1)
    A = rng.standard_normal((m, n)) / math.sqrt(m)
    x = np.zeros(n)
    x[rng.choice(n, 2, replace=False)] = rng.choice([-1.0, 1.0], 2)
    dit, dx = PIN.pin_reduced_vs_direct(A, A @ x, 1e-3)
    assert dit == 0
    assert dx <= 1e-8


def test_reduced_adjoint_matches_dense():
    A, b, tau, xt = PIN.dense_problem(40, 120, 4, seed=57)
    op = R.DenseOperator(A)
    res = R.solve(op, b, tau, R.Params(reduced=1))
    g1 = R.backward(op, res.z, res.s, res.x - xt, R.Params(reduced=1))
    g2 = R.backward(op, res.z, res.s, res.x - xt, method="dense")
    assert np.linalg.norm(g1.grad_b - g2.grad_b) <= 1e-8 * np.linalg.norm(g2.grad_b)
    assert abs(g1.grad_tau - g2.grad_tau) <= 1e-8 * abs(g2.grad_tau)


@pytest.mark.parametrize("n,m", [(64, 16), (256, 100)])
def test_wht_definition(n, m):
    assert PIN.pin_wht_definition(n, m, seed=n + 3) <= 1e-12


def test_wht_full_soft_threshold():
    """All rows of the orthonormal Walsh-Hadamard matrix: x* = soft(W b, tau)."""
    rng = PIN.rng_for(61)
    n = 128
    op = R.PartialWHTOperator(n, np.arange(n))
    b = rng.standard_normal(n)
    assert PIN.pin_orthonormal_soft_threshold(op, b, 0.5) <= 1e-7


@pytest.mark.parametrize("kind", ["wht"])
def test_wht_newton_blocks_and_theorem(kind):
    rng = PIN.rng_for(62)
    n = 32
    op = R.PartialWHTOperator(n, np.sort(rng.choice(n, 8, replace=False)))
    assert PIN.pin_newton_blocks(op, seed=4) <= 1e-7


@pytest.mark.parametrize("n,m", [(64, 16), (128, 100)])
def test_dst_definition(n, m):
    assert PIN.pin_dst_definition(n, m, seed=n + 5) <= 1e-12


def test_dst_full_soft_threshold():
    """All rows of the orthonormal DST-II: x* = soft(S^T b, tau)."""
    rng = PIN.rng_for(63)
    n = 128
    op = R.PartialDSTOperator(n, np.arange(n))
    b = rng.standard_normal(n)
    assert PIN.pin_orthonormal_soft_threshold(op, b, 0.5) <= 1e-7


def test_dst_newton_blocks_and_theorem():
    rng = PIN.rng_for(64)
    n = 32
    op = R.PartialDSTOperator(n, np.sort(rng.choice(n, 8, replace=False)))
    assert PIN.pin_newton_blocks(op, seed=6) <= 1e-7
