"""FP64 CPU oracle of the single-corrector primal-dual matrix-free IPM.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU library never calls it,
and it shares no code with the GPU path (only the seeded input generators in
`workloads.py` serve both sides).

What it computes (paper: Fountoulakis, Gondzio, Zhlobich, "Matrix-free
interior point method for compressed sensing problems"):

  BPDN   min_x  tau*||x||_1 + 1/2 ||A x - b||^2               (Section 1, eq.
         (formulationsnoisy1); the 1/2 follows the smooth QP below)
  split  x = u - v, u, v >= 0, z = [u; v]                     (Section 1, eqs.
         (uvDef), (lintechni))
  primal min_z tau 1^T z + 1/2 ||F^T z - b||^2,  z >= 0,      (eq. (wrightBPDN))
         F^T = [A, -A]
  dual   max -1/2 z^T F F^T z  s.t. c + F F^T z - s = 0, z,s >= 0,
         c = [tau - A^T b; tau + A^T b]                       (Section 3, eq.
         (dualquadraticBPDN))
  Newton residuals f_z = s - c - F F^T z, f_s = sigma mu e - Z S e,
         mu = z^T s / (2n)                                    (eq. (fzfs))
  reduced system (Theta^{-1} + F F^T) dz = f_z + Z^{-1} f_s,
         ds = Z^{-1} f_s - Theta^{-1} dz, Theta = S^{-1} Z     (eq. (redNewton))
  PCG preconditioner P = [[Theta_u^{-1} + rho I, -rho I],
                          [-rho I, Theta_v^{-1} + rho I]]     (Section 4, eq.
         (eq:ne2_P)), rho = Frobenius-closest scalar to A^T A
  IPM loop: single-corrector primal-dual method, Section 5.1 algorithm,
         with the parameter values listed after it and in Section 5.4.

Only products with A and A^T are used inside the method (Section 3: only
matrix-vector products with F are allowed).  The function `dense_newton_matrix`
builds H explicitly for the direct-solver variant (Section 5.7) and for tests.

Readings where the paper is silent (each is a parameter or documented rule):
  * 1/2 on the least-squares term (as in (wrightBPDN) and the vector c);
  * rho = ||A||_F^2 / n (equals m/n for orthonormal rows);
  * z0 = s0 = 1;
  * step length = min(1, eta * largest feasible step), eta = 0.995;
  * relative duality gap = (P(z) - D(nu)) / (1 + |P(z)|) with
    nu = min(1, tau/||g||_inf) (A x - b), g = A^T (A x - b),
    D(nu) = -1/2 ||nu||^2 - b^T nu;
  * corrector: only f_z, f_s (and mu) are evaluated at the trial point;
    Theta and the Z^{-1} of the reduced system stay at the current iterate;
  * sigma choice uses the final step sizes of the previous iteration;
  * PCG: x0 = 0, stop when ||r||_2 <= tolpcg ||rhs||_2 (checked before each
    operator apply), breakdown when p^T q is not > 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np
import scipy.fft
import scipy.linalg

# solver outcome codes
CONVERGED, MAXITER, PCG_BREAKDOWN, NONFINITE, STEP_UNDERFLOW = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "CONVERGED", 1: "MAXITER", 2: "PCG_BREAKDOWN", 3: "NONFINITE",
                4: "STEP_UNDERFLOW"}


@dataclass
class Params:
    """Solver parameters.  Paper values: sigma1..3 and the two step thresholds
    (Section 5.1, after the algorithm); maxiters and mxiterpcg (Section 5.4);
    tol and tolpcg inside the ranges Section 5.4 gives for noisy problems."""
    tol: float = 1e-8
    maxiters: int = 100
    tolpcg: float = 1e-2
    mxiterpcg: int = 200
    sigma1: float = 0.1
    sigma2: float = 0.5
    sigma3: float = 0.8
    alpha_bar: float = 0.5
    alpha_tilde: float = 0.1
    eta: float = 0.995
    rho: float = 0.0          # <= 0: ||A||_F^2 / n
    z0: float = 1.0
    s0: float = 1.0
    tolpcg_adj: float = 1e-12
    mxiterpcg_adj: int = 1000
    step_min: float = 1e-14   # both step sizes below this -> STEP_UNDERFLOW
    reduced: int = 0          # 1: PCG on the n x n system of the Theorem (see pcg_reduced)
    direct: int = 0           # 1: exact Newton directions by Cholesky (Section 5.7; see direct_solve)


# --- operators ----------------------------------------------------------------

class DenseOperator:
    """Explicit m x n matrix; A x and A^T y by numpy products."""

    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.m, self.n = self.A.shape

    def matvec(self, x):
        return self.A @ x

    def rmatvec(self, y):
        return self.A.T @ y

    def frob2(self) -> float:
        return float(np.sum(self.A * self.A))

    def dense(self) -> np.ndarray:
        return self.A


class PartialDCTOperator:
    """A = R_m C: rows `rows` of the orthonormal DCT-II of length n.

    A x   = dct(x, type 2, orthonormal)[rows]
    A^T y = orthonormal DCT-III (= inverse DCT-II) of y zero-filled to length n.
    """

    def __init__(self, n: int, rows: np.ndarray):
        self.n = int(n)
        self.rows = np.asarray(rows, dtype=np.int64)
        self.m = int(self.rows.shape[0])

    def matvec(self, x):
        return scipy.fft.dct(x, type=2, norm="ortho")[self.rows]

    def rmatvec(self, y):
        full = np.zeros(self.n)
        full[self.rows] = y
        return scipy.fft.idct(full, type=2, norm="ortho")

    def frob2(self) -> float:
        return float(self.m)  # orthonormal rows: each has unit norm

    def dense(self) -> np.ndarray:
        """Explicit rows from the cosine definition (small n only)."""
        n = self.n
        k = self.rows[:, None].astype(np.float64)
        j = np.arange(n)[None, :].astype(np.float64)
        alpha = np.where(k == 0, math.sqrt(1.0 / n), math.sqrt(2.0 / n))
        return alpha * np.cos(math.pi * (2.0 * j + 1.0) * k / (2.0 * n))


def fwht(x: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform in natural (Sylvester) order:
    H_1 = [1], H_2n = [[H_n, H_n], [H_n, -H_n]], applied by the recursive
    definition (pairs at distance h combined as (a + b, a - b) for
    h = 1, 2, 4, ...)."""
    y = np.array(x, dtype=np.float64, copy=True)
    n = y.shape[0]
    h = 1
    while h < n:
        y = y.reshape(-1, 2, h)
        a = y[:, 0, :].copy()
        b = y[:, 1, :]
        y = np.stack([a + b, a - b], axis=1).reshape(n)
        h *= 2
    return y


class PartialWHTOperator:
    """A = R_m W: rows `rows` of the orthonormal Walsh-Hadamard matrix
    W = H_n / sqrt(n) (natural order; n a power of two), one of the fast
    partial transforms the paper names beside the DCT.  W is symmetric and
    orthogonal, so A^T y = W (zero-fill of y) and A A^T = I."""

    def __init__(self, n: int, rows: np.ndarray):
        self.n = int(n)
        self.rows = np.asarray(rows, dtype=np.int64)
        self.m = int(self.rows.shape[0])

    def matvec(self, x):
        return fwht(x)[self.rows] / math.sqrt(self.n)

    def rmatvec(self, y):
        full = np.zeros(self.n)
        full[self.rows] = y
        return fwht(full) / math.sqrt(self.n)

    def frob2(self) -> float:
        return float(self.m)

    def dense(self) -> np.ndarray:
        """Explicit rows from Sylvester's construction (small n only)."""
        return scipy.linalg.hadamard(self.n)[self.rows] / math.sqrt(self.n)


class PartialDSTOperator:
    """A = R_m S: rows `rows` of the orthonormal DST-II of length n (another
    fast transform with orthonormal rows); A^T y is the orthonormal DST-III
    of the zero-filled y."""

    def __init__(self, n: int, rows: np.ndarray):
        self.n = int(n)
        self.rows = np.asarray(rows, dtype=np.int64)
        self.m = int(self.rows.shape[0])

    def matvec(self, x):
        return scipy.fft.dst(np.asarray(x, dtype=np.float64), type=2, norm="ortho")[self.rows]

    def rmatvec(self, y):
        full = np.zeros(self.n)
        full[self.rows] = y
        return scipy.fft.idst(full, type=2, norm="ortho")

    def frob2(self) -> float:
        return float(self.m)

    def dense(self) -> np.ndarray:
        """Explicit rows from the sine-sum definition (small n only):
        S[k, j] = s_k sqrt(2/n) sin(pi (k + 1)(2 j + 1) / (2 n)), s_{n-1} = 1/sqrt(2)."""
        n = self.n
        k = self.rows[:, None].astype(np.float64)
        j = np.arange(n, dtype=np.float64)[None, :]
        S = math.sqrt(2.0 / n) * np.sin(math.pi * (k + 1.0) * (2.0 * j + 1.0) / (2.0 * n))
        S[self.rows == n - 1, :] *= 1.0 / math.sqrt(2.0)
        return S


def make_operator(A=None, n=None, rows=None):
    if A is not None:
        return DenseOperator(A)
    return PartialDCTOperator(n, rows)


# --- pieces of the Newton step --------------------------------------------------

def newton_apply(op, theta_inv: np.ndarray, p: np.ndarray) -> np.ndarray:
    """H p = Theta^{-1} p + F F^T p with F F^T w = [K d; -K d], d = w_u - w_v,
    K = A^T A (block form eq. (eq:ne2_H)).  Two operator products."""
    n = op.n
    d = p[:n] - p[n:]
    t = op.rmatvec(op.matvec(d))
    return theta_inv * p + np.concatenate([t, -t])


def precond_solve(theta_inv: np.ndarray, rho: float, r: np.ndarray) -> np.ndarray:
    """P^{-1} r for the block preconditioner (eq. (eq:ne2_P)).  P is a 2x2
    matrix [[a, -rho], [-rho, c]] per index i with a = Theta_u^{-1}+rho,
    c = Theta_v^{-1}+rho; its inverse is [[c, rho], [rho, a]] / (a c - rho^2),
    and a c - rho^2 = tu tv + rho (tu + tv)."""
    n = r.shape[0] // 2
    tu, tv = theta_inv[:n], theta_inv[n:]
    ru, rv = r[:n], r[n:]
    det = tu * tv + rho * (tu + tv)
    return np.concatenate([((tv + rho) * ru + rho * rv) / det,
                           (rho * ru + (tu + rho) * rv) / det])


def dense_newton_matrix(op, theta_inv: np.ndarray) -> np.ndarray:
    """H = diag(Theta^{-1}) + [[K, -K], [-K, K]] explicitly (eq. (eq:ne2_H))."""
    A = op.dense()
    K = A.T @ A
    H = np.block([[K, -K], [-K, K]])
    H[np.diag_indices_from(H)] += theta_inv
    return H


def dense_preconditioner(theta_inv: np.ndarray, rho: float) -> np.ndarray:
    n = theta_inv.shape[0] // 2
    I = np.eye(n)
    P = np.block([[rho * I, -rho * I], [-rho * I, rho * I]])
    P[np.diag_indices_from(P)] += theta_inv
    return P


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    status: int          # 0 ok (converged or hit the cap), PCG_BREAKDOWN, NONFINITE
    hit_cap: bool
    rel_res: float


def pcg(op, theta_inv, rho, rhs, tol, maxit) -> PCGResult:
    """Preconditioned conjugate gradients on (eq:ne2_matrix) with P of
    (eq:ne2_P) (Section 4).  x0 = 0; the test ||r|| <= tol ||rhs|| (squared
    form) precedes every operator apply; `iters` counts operator applies."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    rhs2 = float(rhs @ rhs)
    y = precond_solve(theta_inv, rho, r)
    p = y.copy()
    rty = float(r @ y)
    it = 0
    status = 0
    hit_cap = False
    while True:
        rr = float(r @ r)
        if not math.isfinite(rr):
            status = NONFINITE
            break
        if rr <= tol * tol * rhs2:
            break
        if it == maxit:
            hit_cap = True
            break
        q = newton_apply(op, theta_inv, p)
        it += 1
        pq = float(p @ q)
        if not pq > 0.0:
            status = NONFINITE if not math.isfinite(pq) else PCG_BREAKDOWN
            break
        alpha = rty / pq
        x += alpha * p
        r -= alpha * q
        y = precond_solve(theta_inv, rho, r)
        rty_new = float(r @ y)
        beta = rty_new / rty
        rty = rty_new
        p = y + beta * p
    rel = math.sqrt(float(r @ r) / rhs2) if rhs2 > 0 else 0.0
    return PCGResult(x=x, iters=it, status=status, hit_cap=hit_cap, rel_res=rel)


def reduced_system(theta_inv, rhs):
    """The n x n system behind the Theorem (thm:ne2_prec) of Section 4.
    Writing the two block rows of (eq:ne2_H) with d = du - dv,
        Theta_u^{-1} du + A^T A d = r_u,    Theta_v^{-1} dv - A^T A d = r_v,
    and eliminating du = Theta_u (r_u - A^T A d), dv = Theta_v (r_v + A^T A d)
    gives (Theta_bar^{-1} + A^T A) d = Theta_bar^{-1} (Theta_u r_u - Theta_v r_v)
    with Theta_bar = Theta_u + Theta_v.  Returns (Theta_bar^{-1}, right-hand
    side), both written with Theta^{-1} entries only:
    Theta_bar^{-1} = tu tv / (tu + tv), rhs = (tv r_u - tu r_v) / (tu + tv)."""
    n = rhs.shape[0] // 2
    tu, tv = theta_inv[:n], theta_inv[n:]
    ru, rv = rhs[:n], rhs[n:]
    return tu * tv / (tu + tv), (tv * ru - tu * rv) / (tu + tv)


def back_substitute(theta_inv, rhs, d):
    """The 2n direction from d = du - dv: adding the two block rows gives
    Theta_u^{-1} du + Theta_v^{-1} dv = r_u + r_v, so
    du = (r_u + r_v + tv d) / (tu + tv) and dv = du - d (no operator product)."""
    n = rhs.shape[0] // 2
    tu, tv = theta_inv[:n], theta_inv[n:]
    du = (rhs[:n] + rhs[n:] + tv * d) / (tu + tv)
    return np.concatenate([du, du - d])


def pcg_reduced(op, theta_inv, rho, rhs, tol, maxit) -> PCGResult:
    """PCG on the reduced system with the n x n preconditioner
    Theta_bar^{-1} + rho I of the Theorem (the same non-unit spectrum as the
    2n block-preconditioned system), then the back-substitution.  x0 = 0; the
    test ||r|| <= tol ||rhs_bar|| on the reduced residual precedes every
    operator apply; `iters` counts operator applies."""
    tb, rb = reduced_system(theta_inv, rhs)
    x = np.zeros_like(rb)
    r = rb.copy()
    rhs2 = float(rb @ rb)
    y = r / (tb + rho)
    p = y.copy()
    rty = float(r @ y)
    it = 0
    status = 0
    hit_cap = False
    while True:
        rr = float(r @ r)
        if not math.isfinite(rr):
            status = NONFINITE
            break
        if rr <= tol * tol * rhs2:
            break
        if it == maxit:
            hit_cap = True
            break
        q = tb * p + op.rmatvec(op.matvec(p))
        it += 1
        pq = float(p @ q)
        if not pq > 0.0:
            status = NONFINITE if not math.isfinite(pq) else PCG_BREAKDOWN
            break
        alpha = rty / pq
        x += alpha * p
        r -= alpha * q
        y = r / (tb + rho)
        rty_new = float(r @ y)
        beta = rty_new / rty
        rty = rty_new
        p = y + beta * p
    rel = math.sqrt(float(r @ r) / rhs2) if rhs2 > 0 else 0.0
    return PCGResult(x=back_substitute(theta_inv, rhs, x), iters=it, status=status, hit_cap=hit_cap,
                     rel_res=rel)


def direct_solve(op, theta_inv, rhs) -> PCGResult:
    """Exact Newton direction by Cholesky of the explicit H (Section 5.7)."""
    H = dense_newton_matrix(op, theta_inv)
    c = scipy.linalg.cho_factor(H)
    return PCGResult(x=scipy.linalg.cho_solve(c, rhs), iters=0, status=0, hit_cap=False,
                     rel_res=0.0)


def max_step(v: np.ndarray, dv: np.ndarray) -> float:
    """Largest alpha with v + alpha dv > 0 (inf when dv >= 0)."""
    neg = dv < 0
    if not np.any(neg):
        return math.inf
    return float(np.min(-v[neg] / dv[neg]))


def step_length(v, dv, eta) -> float:
    """Step in [0, 1]: min(1, eta * largest feasible step) (Section 5.1)."""
    return min(1.0, eta * max_step(v, dv))


def objective_terms(op, b, tau, z):
    """Residual-side quantities at z: r = A x - b, g = A^T r, primal value."""
    n = op.n
    x = z[:n] - z[n:]
    r = op.matvec(x) - b
    g = op.rmatvec(r)
    primal = tau * float(np.sum(z)) + 0.5 * float(r @ r)
    return x, r, g, primal


def relative_gap(b, tau, r, g, primal):
    """(P - D(nu)) / (1 + |P|) with the dual-feasible scaling
    nu = min(1, tau / ||g||_inf) r and D(nu) = -1/2 ||nu||^2 - b^T nu."""
    ginf = float(np.max(np.abs(g))) if g.size else 0.0
    theta = 1.0 if ginf <= tau else tau / ginf
    nu = theta * r
    dual = -0.5 * float(nu @ nu) - float(b @ nu)
    return (primal - dual) / (1.0 + abs(primal)), dual


@dataclass
class SolveResult:
    x: np.ndarray
    z: np.ndarray
    s: np.ndarray
    status: int
    ipm_iters: int
    pcg_iters: int
    correctors: int
    nmat: int
    rel_gap: float
    mu: float
    primal_obj: float
    dual_obj: float
    rho: float
    history: list = field(default_factory=list)


def solve(op, b, tau, params: Params | None = None, linsolve: str = "pcg",
          record: bool = False) -> SolveResult:
    """Single-corrector primal-dual matrix-free IPM (Section 5.1 algorithm)."""
    p = params or Params()
    n = op.n
    b = np.asarray(b, dtype=np.float64)
    tau = float(tau)
    rho = p.rho if p.rho > 0 else op.frob2() / n
    z = np.full(2 * n, p.z0)
    s = np.full(2 * n, p.s0)
    k = 1
    aP_prev = aD_prev = 1.0
    nmat = pcg_total = ncorr = 0
    status = MAXITER
    hist = []
    mu = float(z @ s) / (2 * n)

    def lin(theta_inv, rhs):
        if linsolve == "direct" or p.direct:
            return direct_solve(op, theta_inv, rhs)
        if p.reduced:
            return pcg_reduced(op, theta_inv, rho, rhs, p.tolpcg, p.mxiterpcg)
        return pcg(op, theta_inv, rho, rhs, p.tolpcg, p.mxiterpcg)

    while True:
        x, r, g, primal = objective_terms(op, b, tau, z)
        nmat += 2
        relgap, dual = relative_gap(b, tau, r, g, primal)
        mu = float(z @ s) / (2 * n)
        if record:
            hist.append(dict(k=k, relgap=relgap, mu=mu, primal=primal))
        if not math.isfinite(relgap):
            status = NONFINITE
            break
        if relgap <= p.tol:
            status = CONVERGED
            break
        if k > p.maxiters:
            status = MAXITER
            break
        # centring parameter from the previous step sizes
        sigma = p.sigma2 if (k != 1 and (aP_prev <= p.alpha_bar or aD_prev <= p.alpha_bar)) \
            else p.sigma1
        # predictor: residuals (fzfs) and reduced Newton system (redNewton)
        fz = s - np.concatenate([tau + g, tau - g])
        fs = sigma * mu - z * s
        theta_inv = s / z
        rhs = fz + fs / z
        res = lin(theta_inv, rhs)
        pcg_total += res.iters
        nmat += 2 * res.iters
        if res.status:
            status = res.status
            break
        dz = res.x
        ds = fs / z - theta_inv * dz
        aP = step_length(z, dz, p.eta)
        aD = step_length(s, ds, p.eta)
        # corrector when a step is short
        if aP <= p.alpha_tilde or aD <= p.alpha_tilde:
            zt = z + aP * dz
            st = s + aD * ds
            xt = zt[:n] - zt[n:]
            gt = op.rmatvec(op.matvec(xt) - b)
            nmat += 2
            mut = float(zt @ st) / (2 * n)
            fzt = st - np.concatenate([tau + gt, tau - gt])
            fst = p.sigma3 * mut - zt * st
            rhst = fzt + fst / z
            res = lin(theta_inv, rhst)
            pcg_total += res.iters
            nmat += 2 * res.iters
            if res.status:
                status = res.status
                break
            dzt = res.x
            dst = fst / z - theta_inv * dzt
            dz = dz + dzt
            ds = ds + dst
            aP = step_length(z, dz, p.eta)
            aD = step_length(s, ds, p.eta)
            ncorr += 1
        if aP < p.step_min and aD < p.step_min:
            status = STEP_UNDERFLOW
            break
        z = z + aP * dz
        s = s + aD * ds
        aP_prev, aD_prev = aP, aD
        k += 1
    x = z[:n] - z[n:]
    return SolveResult(x=x, z=z, s=s, status=status, ipm_iters=k - 1, pcg_iters=pcg_total,
                       correctors=ncorr, nmat=nmat, rel_gap=relgap, mu=mu,
                       primal_obj=primal, dual_obj=dual, rho=rho, history=hist)


# --- adjoint ----------------------------------------------------------------------

@dataclass
class GradResult:
    grad_b: np.ndarray
    grad_tau: float
    w: np.ndarray
    pcg_iters: int
    status: int


def backward(op, z, s, grad_x, params: Params | None = None, rho: float | None = None,
             method: str = "pcg") -> GradResult:
    """Implicit derivative of x* = u - v through the perturbed optimality
    conditions of the primal-dual pair at the final (z, s): differentiating
    c + F F^T z - s = 0 and Z S e = mu e (mu fixed) gives
    (Theta^{-1} + F F^T) dz = F db - 1 dtau.  With H w = [g_x; -g_x]:
    dL/db = A (w_u - w_v),  dL/dtau = -1^T w.
    `method` is "pcg" (the same PCG as the forward solve, 2n or reduced per
    params.reduced, at the adjoint tolerance) or "dense" (Cholesky)."""
    p = params or Params()
    n = op.n
    if rho is None:
        rho = p.rho if p.rho > 0 else op.frob2() / n
    theta_inv = s / z
    rhs = np.concatenate([grad_x, -grad_x])
    if method == "dense":
        res = direct_solve(op, theta_inv, rhs)
    elif p.reduced:
        res = pcg_reduced(op, theta_inv, rho, rhs, p.tolpcg_adj, p.mxiterpcg_adj)
    else:
        res = pcg(op, theta_inv, rho, rhs, p.tolpcg_adj, p.mxiterpcg_adj)
    w = res.x
    return GradResult(grad_b=op.matvec(w[:n] - w[n:]), grad_tau=-float(np.sum(w)), w=w,
                      pcg_iters=res.iters, status=res.status)


# --- certificates and closed forms ------------------------------------------------

def soft_threshold(v, t):
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def support_from_state(z, s, n):
    """Index set B of the paper (Section 4, eq. (eq:thetas_split)):
    Theta_j = z_j / s_j >> 1.  Returns (support indices, signs)."""
    th = z / s
    tu, tv = th[:n], th[n:]
    on = (tu > 1.0) | (tv > 1.0)
    idx = np.nonzero(on)[0]
    sgn = np.where(tu[idx] > tv[idx], 1.0, -1.0)
    return idx, sgn


def kkt_residual(op, b, tau, x, support=None, signs=None):
    """max( max_i (|g_i| - tau)_+, max_{i in S} |g_i + tau sign_i| ) / tau with
    g = A^T (A x - b); optimality of BPDN requires |g_i| <= tau everywhere and
    g_i = -tau sign(x_i) on the support."""
    g = op.rmatvec(op.matvec(x) - b)
    viol = float(np.max(np.maximum(np.abs(g) - tau, 0.0)))
    if support is None:
        support = np.nonzero(x)[0]
        signs = np.sign(x[support])
    on = float(np.max(np.abs(g[support] + tau * signs))) if len(support) else 0.0
    return max(viol, on) / tau


def prox_residual(op, b, tau, x):
    """||x - soft(x - g, tau)||_inf / (1 + ||x||_inf)."""
    g = op.rmatvec(op.matvec(x) - b)
    return float(np.max(np.abs(x - soft_threshold(x - g, tau)))) / (1.0 + float(np.max(np.abs(x))))


def bpdn_objective(A_op, b, tau, x):
    r = A_op.matvec(x) - b
    return tau * float(np.sum(np.abs(x))) + 0.5 * float(r @ r)


def closed_form_on_support(A_S: np.ndarray, b, tau, signs):
    """x_S = (A_S^T A_S)^{-1} (A_S^T b - tau sign_S): stationarity of BPDN
    restricted to a fixed support with fixed signs."""
    G = A_S.T @ A_S
    return np.linalg.solve(G, A_S.T @ b - tau * signs)


def closed_form_gradient(A_S: np.ndarray, signs, x_S, xtrue_S):
    """For L = 1/2 ||x* - x_true||^2 with x*_S affine in (b, tau):
    dL/db = A_S (A_S^T A_S)^{-1} (x_S - xt_S),
    dL/dtau = -sign_S^T (A_S^T A_S)^{-1} (x_S - xt_S)."""
    G = A_S.T @ A_S
    v = np.linalg.solve(G, x_S - xtrue_S)
    return A_S @ v, -float(signs @ v)


def brute_force_bpdn(A: np.ndarray, b, tau):
    """Global minimiser of tau||x||_1 + 1/2||Ax-b||^2 by enumerating the 3^n
    sign patterns (tiny n only): for each pattern solve the restricted
    stationarity equations and keep sign- and KKT-consistent candidates."""
    m, n = A.shape
    best = None
    best_val = math.inf
    for code in range(3 ** n):
        sg = np.zeros(n)
        c = code
        for i in range(n):
            sg[i] = (c % 3) - 1
            c //= 3
        S = np.nonzero(sg)[0]
        x = np.zeros(n)
        if len(S):
            if len(S) > m:
                continue
            A_S = A[:, S]
            G = A_S.T @ A_S
            if np.linalg.cond(G) > 1e12:
                continue
            xs = np.linalg.solve(G, A_S.T @ b - tau * sg[S])
            if np.any(np.sign(xs) != sg[S]):
                continue
            x[S] = xs
        g = A.T @ (A @ x - b)
        if np.max(np.abs(g)) > tau * (1 + 1e-9):
            continue
        val = tau * np.sum(np.abs(x)) + 0.5 * np.sum((A @ x - b) ** 2)
        if val < best_val:
            best_val, best = val, x
    return best, best_val
