"""Pins for the CPU oracle: checks against facts that the paper or plain
mathematics fix, written so that a plausible slip anywhere in the oracle
(a dropped term, a wrong sign, a transposed operand) changes at least one of
the returned error measures.  Each function returns an error (0 when exact);
tests compare it against a threshold and the mutation tests check that planted
mistakes push it over.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import mfipm_ref as R


def rng_for(seed):
    return np.random.default_rng(np.random.PCG64(seed))


def dense_problem(m, n, k, seed, sigma=1e-3, c_tau=1e-2):
    rng = rng_for(seed)
    A = rng.standard_normal((m, n)) / math.sqrt(m)
    x = np.zeros(n)
    S = rng.choice(n, k, replace=False)
    x[S] = rng.standard_normal(k)
    b = A @ x + sigma * rng.standard_normal(m)
    tau = c_tau * float(np.max(np.abs(A.T @ b)))
    return A, b, tau, x


def pin_zero_solution(op, b, scale=1.5):
    """tau >= ||A^T b||_inf makes x = 0 optimal (0 is in the subdifferential).
    Returns ||x||_inf / (1 + ||b||_inf)."""
    tau = scale * float(np.max(np.abs(op.rmatvec(b))))
    res = R.solve(op, b, tau)
    assert res.status == R.CONVERGED, res.status
    return float(np.max(np.abs(res.x))) / (1.0 + float(np.max(np.abs(b))))


def pin_orthonormal_soft_threshold(op, b, tau):
    """A^T A = I  =>  x* = soft(A^T b, tau).  Returns the relative error."""
    res = R.solve(op, b, tau, R.Params(tol=1e-12))
    ref = R.soft_threshold(op.rmatvec(b), tau)
    return float(np.linalg.norm(res.x - ref) / max(np.linalg.norm(ref), 1e-300))


def pin_brute_force(A, b, tau):
    """Relative distance of the oracle solution from the enumerated minimiser."""
    xb, _ = R.brute_force_bpdn(A, b, tau)
    res = R.solve(R.DenseOperator(A), b, tau, R.Params(tol=1e-12))
    return float(np.linalg.norm(res.x - xb) / max(np.linalg.norm(xb), 1e-300))


def pin_kkt(op, b, tau, params=None):
    """KKT residual of the oracle solution (|g_i| <= tau, g_S = -tau sign x_S)."""
    res = R.solve(op, b, tau, params)
    S, sg = R.support_from_state(res.z, res.s, op.n)
    return R.kkt_residual(op, b, tau, res.x, S, sg), res


def pin_newton_blocks(op, seed):
    """H-apply and P^{-1} against their dense block definitions, and
    Theorem (thm:ne2_prec): P^{-1} H has eigenvalue 1 with multiplicity n, the
    other n eigenvalues are those of the n x n pair with Theta_u + Theta_v.
    Returns the largest of the discrepancies."""
    n = op.n
    rng = rng_for(seed)
    theta_inv = 10.0 ** rng.uniform(-4, 4, 2 * n)
    rho = op.frob2() / n
    H = R.dense_newton_matrix(op, theta_inv)
    P = R.dense_preconditioner(theta_inv, rho)
    p = rng.standard_normal(2 * n)
    e1 = np.linalg.norm(R.newton_apply(op, theta_inv, p) - H @ p) / np.linalg.norm(H @ p)
    e2 = np.linalg.norm(R.precond_solve(theta_inv, rho, p) - np.linalg.solve(P, p)) / \
        np.linalg.norm(np.linalg.solve(P, p))
    # the explicit H itself against the product definition Theta^{-1} + F F^T
    A = op.dense()
    F = np.vstack([A.T, -A.T])  # F = [A^T; -A^T] so that F^T = [A, -A]
    e0 = np.linalg.norm(H - (np.diag(theta_inv) + F @ F.T)) / np.linalg.norm(H)
    # spectrum: generalized symmetric problem H v = lambda P v
    import scipy.linalg
    lam = np.sort(scipy.linalg.eigh(H, P, eigvals_only=True))
    ones = np.abs(lam - 1.0) < 1e-8 * max(1.0, float(np.max(np.abs(lam))))
    e3 = abs(int(np.sum(ones)) - n)  # exactly n unit eigenvalues
    th = 1.0 / theta_inv
    tbar_inv = 1.0 / (th[:n] + th[n:])
    Hn = A.T @ A + np.diag(tbar_inv)
    Pn = np.diag(tbar_inv + rho)
    lam_n = np.sort(scipy.linalg.eigh(Hn, Pn, eigvals_only=True))
    rest = np.sort(np.concatenate([lam[~ones], np.ones(int(np.sum(ones)) - n)])) \
        if np.sum(ones) >= n else lam
    lam_all = np.sort(np.concatenate([np.ones(n), lam_n]))
    e4 = float(np.max(np.abs(lam_all - lam)) / max(1.0, float(np.max(lam))))
    del rest
    return max(e0, e1, e2, float(e3), e4)


def pin_dct_definition(n, m, seed):
    """Partial DCT against the cosine-sum definition and A A^T = I_m."""
    rng = rng_for(seed)
    rows = np.sort(rng.choice(n, m, replace=False))
    op = R.PartialDCTOperator(n, rows)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    # cosine sum written out directly (independent of op.dense())
    j = np.arange(n)
    ref = np.array([(math.sqrt(1.0 / n) if k == 0 else math.sqrt(2.0 / n)) *
                    np.sum(x * np.cos(math.pi * (2 * j + 1) * k / (2 * n))) for k in rows])
    e1 = np.linalg.norm(op.matvec(x) - ref) / np.linalg.norm(ref)
    # adjoint identity <A x, y> = <x, A^T y>
    e2 = abs(op.matvec(x) @ y - x @ op.rmatvec(y)) / (np.linalg.norm(x) * np.linalg.norm(y))
    # orthonormal rows
    e3 = np.linalg.norm(op.matvec(op.rmatvec(y)) - y) / np.linalg.norm(y)
    return max(e1, e2, e3)


def pin_pcg_vs_direct(A, b, tau):
    """With PCG run to 1e-12 the IPM takes the same iterations and reaches the
    same point as with exact (Cholesky) Newton directions (Section 5.7:
    PCG needs as few IPM iterations as the direct solver).  Returns
    (|iteration difference|, relative x difference)."""
    op = R.DenseOperator(A)
    p_it = R.Params(tolpcg=1e-12, mxiterpcg=10 * A.shape[1])
    r1 = R.solve(op, b, tau, p_it)
    r2 = R.solve(op, b, tau, p_it, linsolve="direct")
    return abs(r1.ipm_iters - r2.ipm_iters), float(np.linalg.norm(r1.x - r2.x) / np.linalg.norm(r2.x))


def pin_duality(A, b, tau):
    """At the exact minimiser the gap certificate is zero (strong duality), and
    it is non-negative at any z (weak duality).  Returns max(|gap at x*|,
    largest negative gap over random z)."""
    op = R.DenseOperator(A)
    xb, _ = R.brute_force_bpdn(A, b, tau)
    z = np.concatenate([np.maximum(xb, 0), np.maximum(-xb, 0)])
    _, r, g, primal = R.objective_terms(op, b, tau, z)
    gap0, _ = R.relative_gap(b, tau, r, g, primal)
    worst = 0.0
    rng = rng_for(7)
    for _ in range(20):
        zz = np.abs(rng.standard_normal(2 * A.shape[1]))
        _, r, g, primal = R.objective_terms(op, b, tau, zz)
        gp, _ = R.relative_gap(b, tau, r, g, primal)
        worst = max(worst, -gp)
    # the primal value equals the BPDN objective of x = u - v when u, v have
    # disjoint supports
    fb = R.bpdn_objective(op, b, tau, xb)
    _, _, _, pz = R.objective_terms(op, b, tau, z)
    return max(abs(gap0), worst, abs(fb - pz) / (1 + abs(fb)))


def pin_gradient(A, b, tau, x_true):
    """Adjoint gradient at a tightly converged solve against the closed form
    on the support.  Returns the largest relative error over dL/db, dL/dtau."""
    op = R.DenseOperator(A)
    prm = R.Params(tol=1e-13, tolpcg=1e-10, mxiterpcg=2000)
    res = R.solve(op, b, tau, prm)
    S, sg = R.support_from_state(res.z, res.s, op.n)
    gx = res.x - x_true
    gb_cf, gt_cf = R.closed_form_gradient(A[:, S], sg, res.x[S], x_true[S])
    gr = R.backward(op, res.z, res.s, gx, prm)
    eb = np.linalg.norm(gr.grad_b - gb_cf) / np.linalg.norm(gb_cf)
    et = abs(gr.grad_tau - gt_cf) / abs(gt_cf)
    return max(eb, et)


def pin_rho(op, b, tau):
    """The preconditioner scalar the solver uses against the paper's
    criterion, found by a one-dimensional search rather than a formula: rho is
    the multiple of the identity closest to A^T A in the Frobenius norm
    (Section 4, before eq. (eq:ne2_P)).  For orthonormal rows (partial DCT)
    this is m/n.  ||A^T A - r I||_F^2 is a parabola in r, so its minimiser is
    the vertex through three evaluations of the distance itself (explicit A).
    Returns the relative distance of the solver's rho from that vertex."""
    res = R.solve(op, b, tau, R.Params(maxiters=1))
    A = op.dense()
    K = A.T @ A
    f = [float(np.linalg.norm(K - r * np.eye(op.n)) ** 2) for r in (0.0, 1.0, 2.0)]
    a2 = (f[2] - 2.0 * f[1] + f[0]) / 2.0
    a1 = f[1] - f[0] - a2
    vertex = -a1 / (2.0 * a2)
    return abs(res.rho - vertex) / vertex


def pin_kkt_handbuilt():
    """kkt_residual on points with a known answer.  With A = I the gradient
    of the least-squares term is g = x - b.  Case 1: x = soft(b, tau) is the
    minimiser, residual 0.  Case 2: entry j off the support with
    |b_j| = tau (1 + eps): residual eps.  Case 3: a support entry moved by
    delta: |g_j + tau sign x_j| = delta, residual delta / tau.  Case 4: a
    support entry with the wrong sign of g: residual 2.  Returns the largest
    deviation from the known values."""
    n, tau = 16, 0.5
    rng = rng_for(13)
    b = rng.standard_normal(n) * 2.0
    b[np.abs(b) < 0.7] += 1.0  # keep entries away from the threshold
    b[0], b[1] = 0.1, -0.2    # two entries off the support
    op = R.DenseOperator(np.eye(n))
    x = R.soft_threshold(b, tau)
    S = np.nonzero(x)[0]
    sg = np.sign(x[S])
    errs = [abs(R.kkt_residual(op, b, tau, x, S, sg) - 0.0)]
    eps = 0.25
    b2 = b.copy()
    b2[0] = tau * (1 + eps)          # x_0 = 0 stays, so |g_0| = tau (1 + eps)
    errs.append(abs(R.kkt_residual(op, b2, tau, x, S, sg) - eps))
    delta = 1e-3
    x3 = x.copy()
    j = S[0]
    x3[j] += delta
    errs.append(abs(R.kkt_residual(op, b, tau, x3, S, sg) - delta / tau))
    sg4 = sg.copy()
    sg4[0] = -sg4[0]
    errs.append(abs(R.kkt_residual(op, b, tau, x, S, sg4) - 2.0))
    return max(errs)


def pin_reduced_direction(op, seed):
    """The reduced system's exact solution, back-substituted, against the
    exact 2n Newton direction (Cholesky of the explicit H): the elimination
    of Section 4's block rows loses nothing.  Also the reduced PCG at a tight
    tolerance against the same direction.  Returns the larger relative error."""
    n = op.n
    rng = rng_for(seed)
    theta_inv = 10.0 ** rng.uniform(-3, 3, 2 * n)
    rhs = rng.standard_normal(2 * n)
    exact = np.linalg.solve(R.dense_newton_matrix(op, theta_inv), rhs)
    tb, rb = R.reduced_system(theta_inv, rhs)
    A = op.dense()
    d = np.linalg.solve(np.diag(tb) + A.T @ A, rb)
    e1 = np.linalg.norm(R.back_substitute(theta_inv, rhs, d) - exact) / np.linalg.norm(exact)
    res = R.pcg_reduced(op, theta_inv, op.frob2() / n, rhs, 1e-13, 50 * n)
    e2 = np.linalg.norm(res.x - exact) / np.linalg.norm(exact)
    return max(e1, e2)


def pin_reduced_vs_direct(A, b, tau):
    """The IPM with reduced-system PCG at tolpcg 1e-12 takes the iterations of
    the exact-Newton IPM and reaches its point (Section 5.7 comparison, with
    the reduced system).  Returns (|iteration difference|, relative x
    difference)."""
    op = R.DenseOperator(A)
    p_it = R.Params(tolpcg=1e-12, mxiterpcg=10 * A.shape[1], reduced=1)
    r1 = R.solve(op, b, tau, p_it)
    r2 = R.solve(op, b, tau, p_it, linsolve="direct")
    return abs(r1.ipm_iters - r2.ipm_iters), float(np.linalg.norm(r1.x - r2.x) / np.linalg.norm(r2.x))


def pin_wht_definition(n, m, seed):
    """Partial Walsh-Hadamard operator against the matrix entries written
    out from their closed form, H[k, j] = (-1)^{popcount(k & j)} (Sylvester
    order), the adjoint identity and A A^T = I.  Returns the largest error."""
    rng = rng_for(seed)
    rows = np.sort(rng.choice(n, m, replace=False))
    op = R.PartialWHTOperator(n, rows)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    j = np.arange(n)
    ref = np.array([np.sum(x * (-1.0) ** np.array([bin(int(k) & int(jj)).count("1") for jj in j]))
                    for k in rows]) / math.sqrt(n)
    e1 = np.linalg.norm(op.matvec(x) - ref) / np.linalg.norm(ref)
    e2 = abs(op.matvec(x) @ y - x @ op.rmatvec(y)) / (np.linalg.norm(x) * np.linalg.norm(y))
    e3 = np.linalg.norm(op.matvec(op.rmatvec(y)) - y) / np.linalg.norm(y)
    e4 = np.linalg.norm(op.dense() @ x - op.matvec(x)) / np.linalg.norm(ref)
    return max(e1, e2, e3, e4)


def pin_dst_definition(n, m, seed):
    """Partial DST operator against its entries written out from the sine sum
    S[k, j] = c_k sin(pi (k + 1)(2 j + 1) / (2 n)), c_k = sqrt(2/n) (sqrt(1/n)
    for k = n - 1), with the sum taken term by term here; plus the adjoint
    identity and A A^T = I.  Returns the largest error."""
    rng = rng_for(seed)
    rows = np.sort(rng.choice(n, m, replace=False))
    op = R.PartialDSTOperator(n, rows)
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    ref = np.zeros(m)
    for a, k in enumerate(rows):
        c = math.sqrt((1.0 if k == n - 1 else 2.0) / n)
        ref[a] = c * sum(x[j] * math.sin(math.pi * (k + 1) * (2 * j + 1) / (2 * n)) for j in range(n))
    e1 = np.linalg.norm(op.matvec(x) - ref) / np.linalg.norm(ref)
    e2 = abs(op.matvec(x) @ y - x @ op.rmatvec(y)) / (np.linalg.norm(x) * np.linalg.norm(y))
    e3 = np.linalg.norm(op.matvec(op.rmatvec(y)) - y) / np.linalg.norm(y)
    return max(e1, e2, e3)
