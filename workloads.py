"""Seeded synthetic inputs for the l1-regularised least-squares solver.

This module only *draws* problem instances: measurement operators (a dense
Gaussian matrix or a set of sampled DCT rows), sparse signals, noise, the
observations b and the regularisation weight tau.  It contains none of the
solver's arithmetic and is shared, as input, by the CPU oracle tests and by
the GPU harness (tests, bench).

Problem family (paper, Section 1, eqs. (incomplsysnoisy) and
(formulationsnoisy1)): b = A x_true + e with e_i ~ N(0, sigma^2), and
tau = c_tau * ||A^T b||_inf.

Operators:
  * dense: A with i.i.d. N(0, 1/m) entries, row-major (C order), m x n;
  * partial DCT: A = R_m C, where C is the orthonormal DCT-II of length n and
    R_m keeps m distinct rows drawn uniformly without replacement, sorted
    ascending (paper, Section 2 orthonormal rows, eq. (eq:orthonormality), and
    Section 5.8 phase-transition setup "normalized DCT");
  * partial DST: A = R_m S with S the orthonormal DST-II, rows as for the DCT;
  * partial Walsh-Hadamard: A = R_m W, W = H_n / sqrt(n) with H_n the
    Sylvester-ordered Hadamard matrix, rows drawn as for the DCT (another fast
    orthonormal transform, paper Sections 1-2).

Draw order inside one instance is fixed: operator (A or rows) -> support ->
amplitudes / signs -> noise.  Every generator is numpy's PCG64 with the stated
seed.  The observation b is formed on the host in FP64 (matmul or
scipy.fft.dct); tau from A^T b likewise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.fft

__all__ = [
    "DenseInstance", "DCTInstance", "dense_instance", "dct_instance",
    "config_dense_256x1024", "config_pdct", "config_pdct_hdr",
    "batched_dense_sizes", "batched_dense_instance", "config_dct_batch",
    "dct_apply", "dct_apply_t", "SharedDenseInstance", "config_shared_dense",
    "wht_apply", "wht_apply_t", "config_wht", "config_wht_hdr", "direct_scaling_instance",
    "dst_apply", "dst_apply_t", "config_dst",
    "DIRECT_SCALING_NS",
]


def dct_apply(rows: np.ndarray, n: int, x: np.ndarray) -> np.ndarray:
    """Rows `rows` of the orthonormal DCT-II of x (input synthesis only)."""
    return scipy.fft.dct(np.asarray(x, np.float64), type=2, norm="ortho")[rows]


def dct_apply_t(rows: np.ndarray, n: int, y: np.ndarray) -> np.ndarray:
    """Transpose of dct_apply: zero-fill to length n, orthonormal DCT-III."""
    full = np.zeros(n, np.float64)
    full[rows] = y
    return scipy.fft.idct(full, type=2, norm="ortho")


def _hadamard_unnormalised(x: np.ndarray) -> np.ndarray:
    """H_n x for the Sylvester-ordered Hadamard matrix (input synthesis only)."""
    v = np.array(x, np.float64, copy=True)
    n = v.shape[0]
    h = 1
    while h < n:
        v = v.reshape(-1, 2, h)
        v = np.stack([v[:, 0] + v[:, 1], v[:, 0] - v[:, 1]], axis=1).reshape(n)
        h *= 2
    return v


def wht_apply(rows: np.ndarray, n: int, x: np.ndarray) -> np.ndarray:
    """Rows `rows` of H_n x / sqrt(n) (input synthesis only)."""
    return _hadamard_unnormalised(x)[rows] / np.sqrt(n)


def wht_apply_t(rows: np.ndarray, n: int, y: np.ndarray) -> np.ndarray:
    """Transpose of wht_apply: zero-fill to length n, then H_n / sqrt(n)."""
    full = np.zeros(n, np.float64)
    full[rows] = y
    return _hadamard_unnormalised(full) / np.sqrt(n)


def dst_apply(rows: np.ndarray, n: int, x: np.ndarray) -> np.ndarray:
    """Rows `rows` of the orthonormal DST-II of x (input synthesis only)."""
    return scipy.fft.dst(np.asarray(x, np.float64), type=2, norm="ortho")[rows]


def dst_apply_t(rows: np.ndarray, n: int, y: np.ndarray) -> np.ndarray:
    """Transpose of dst_apply: zero-fill to length n, orthonormal DST-III."""
    full = np.zeros(n, np.float64)
    full[rows] = y
    return scipy.fft.idst(full, type=2, norm="ortho")


_APPLY = {"dct": (dct_apply, dct_apply_t), "wht": (wht_apply, wht_apply_t), "dst": (dst_apply, dst_apply_t)}


def _sparse_signal(rng: np.random.Generator, n: int, k: int, amp: str) -> np.ndarray:
    x = np.zeros(n, np.float64)
    supp = rng.choice(n, size=k, replace=False)
    if amp == "pm1":
        x[supp] = rng.choice(np.array([-1.0, 1.0]), size=k)
    elif amp == "normal":
        x[supp] = rng.standard_normal(k)
    elif amp == "hdr":  # +-10^(3U), U ~ U(0,1), random sign
        mag = 10.0 ** (3.0 * rng.random(k))
        sgn = rng.choice(np.array([-1.0, 1.0]), size=k)
        x[supp] = sgn * mag
    else:
        raise ValueError(amp)
    return x


@dataclass
class DenseInstance:
    A: np.ndarray          # (m, n) float64, C order
    b: np.ndarray          # (m,)
    tau: float
    x_true: np.ndarray     # (n,)
    seed: int
    label: str = ""

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


@dataclass
class DCTInstance:
    n: int
    rows: np.ndarray       # (m,) int32, sorted, distinct
    b: np.ndarray          # (m,) or (B, m)
    tau: np.ndarray | float
    x_true: np.ndarray     # (n,) or (B, n)
    seed: int
    label: str = ""
    extra: dict = field(default_factory=dict)
    transform: str = "dct"  # "dct" or "wht": which transform's rows A keeps

    @property
    def m(self) -> int:
        return int(self.rows.shape[0])


def dense_instance(m: int, n: int, k: int, seed: int, amp: str = "normal",
                   sigma: float = 1e-3, c_tau: float = 1e-2, label: str = "") -> DenseInstance:
    rng = np.random.default_rng(np.random.PCG64(seed))
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x = _sparse_signal(rng, n, k, amp)
    e = sigma * rng.standard_normal(m)
    b = A @ x + e
    tau = float(c_tau * np.max(np.abs(A.T @ b)))
    return DenseInstance(A=np.ascontiguousarray(A), b=b, tau=tau, x_true=x, seed=seed, label=label)


def dct_instance(n: int, m: int, k: int, seed: int, amp: str = "normal",
                 sigma: float = 1e-2, c_tau: float = 1e-2, label: str = "",
                 transform: str = "dct") -> DCTInstance:
    """Rows of a fast transform ("dct" or "wht"), a k-sparse signal, noise."""
    fwd, adj = _APPLY[transform]
    rng = np.random.default_rng(np.random.PCG64(seed))
    rows = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    x = _sparse_signal(rng, n, k, amp)
    e = sigma * rng.standard_normal(m)
    b = fwd(rows, n, x) + e
    tau = float(c_tau * np.max(np.abs(adj(rows, n, b))))
    return DCTInstance(n=n, rows=rows, b=b, tau=tau, x_true=x, seed=seed, label=label, transform=transform)


# --- the five named workloads -------------------------------------------------

def config_dense_256x1024() -> DenseInstance:
    """Dense 256x1024 N(0,1/256), 20-sparse +-1 spikes, noise 1e-3, c_tau 1e-2."""
    return dense_instance(256, 1024, 20, seed=120801, amp="pm1", sigma=1e-3, c_tau=1e-2,
                          label="dense_256x1024")


def config_pdct(n: int = 1 << 16) -> DCTInstance:
    """Partial DCT n=2^16, m=n/4, k=floor(n/100) N(0,1), noise 1e-2, c_tau 1e-2."""
    return dct_instance(n, n // 4, n // 100, seed=120802, amp="normal", sigma=1e-2, c_tau=1e-2,
                        label=f"pdct_n{n}")


def config_pdct_hdr(n: int = 1 << 20) -> DCTInstance:
    """Partial DCT n=2^20, m=n/4, k=floor(n/200) +-10^U(0,3), noise 1e-3, c_tau 1e-3."""
    return dct_instance(n, n // 4, n // 200, seed=120803, amp="hdr", sigma=1e-3, c_tau=1e-3,
                        label=f"pdct_hdr_n{n}")


def config_dst(n: int = 1 << 16) -> DCTInstance:
    """Partial DST n=2^16 with the partial-DCT n=2^16 recipe."""
    return dct_instance(n, n // 4, n // 100, seed=120812, amp="normal", sigma=1e-2, c_tau=1e-2,
                        label=f"dst_n{n}", transform="dst")


def config_wht(n: int = 1 << 16) -> DCTInstance:
    """Partial Walsh-Hadamard n=2^16 with the partial-DCT n=2^16 recipe."""
    return dct_instance(n, n // 4, n // 100, seed=120809, amp="normal", sigma=1e-2, c_tau=1e-2,
                        label=f"wht_n{n}", transform="wht")


def config_wht_hdr(n: int = 1 << 20) -> DCTInstance:
    """Partial Walsh-Hadamard n=2^20 with the high-dynamic-range partial-DCT recipe."""
    return dct_instance(n, n // 4, n // 200, seed=120810, amp="hdr", sigma=1e-3, c_tau=1e-3,
                        label=f"wht_hdr_n{n}", transform="wht")


# Section 5.7 (direct solver against PCG): n = 2^5 .. 2^12, m = n/4.
DIRECT_SCALING_NS = tuple(1 << e for e in range(5, 13))


def direct_scaling_instance(n: int, seed: int = 120811) -> DenseInstance:
    """The Section 5.7 comparison problem: Gaussian A (N(0, 1/m), m = n/4),
    k = ceil(m/20) nonzeros at random positions with N(0,1) values,
    noiseless b = A x, tau = 1e-3 (absolute)."""
    m = n // 4
    k = -(-m // 20)
    rng = np.random.default_rng(np.random.PCG64(seed * 100 + int(np.log2(n))))
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x = _sparse_signal(rng, n, k, "normal")
    b = A @ x
    return DenseInstance(A=np.ascontiguousarray(A), b=b, tau=1e-3, x_true=x, seed=seed, label=f"direct_n{n}")


def batched_dense_sizes(batch: int = 256, seed: int = 120804) -> np.ndarray:
    """Signal lengths n_i = 64 * U{16..128} of the batched dense workload."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return 64 * rng.integers(16, 129, size=batch)


def batched_dense_instance(i: int, n: int, seed: int = 120804) -> DenseInstance:
    """Instance i of the batched dense workload: m=n/4, k=floor(n/50) N(0,1)."""
    return dense_instance(n // 4, n, n // 50, seed=seed * 1000 + i, amp="normal",
                          sigma=1e-3, c_tau=1e-2, label=f"batched_dense_{i}")


def config_dct_batch(n: int = 1 << 18, batch: int = 32, seed: int = 120805,
                     sigma: float = 1e-2, c_tau: float = 5e-3, transform: str = "dct") -> DCTInstance:
    """`batch` signals sharing one partial DCT (or Walsh-Hadamard: transform
    "wht") with m=n/4, k=floor(n/100) N(0,1)."""
    dct_apply, dct_apply_t = _APPLY[transform]
    rng = np.random.default_rng(np.random.PCG64(seed))
    m, k = n // 4, n // 100
    rows = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    X = np.zeros((batch, n))
    Bm = np.zeros((batch, m))
    taus = np.zeros(batch)
    for j in range(batch):
        X[j] = _sparse_signal(rng, n, k, "normal")
        e = sigma * rng.standard_normal(m)
        Bm[j] = dct_apply(rows, n, X[j]) + e
        taus[j] = c_tau * np.max(np.abs(dct_apply_t(rows, n, Bm[j])))
    drng = np.random.default_rng(np.random.PCG64(seed + 1))
    direction = drng.standard_normal((batch, m))
    direction /= np.linalg.norm(direction, axis=1, keepdims=True)
    return DCTInstance(n=n, rows=rows, b=Bm, tau=taus, x_true=X, seed=seed,
                       label=f"p{transform}_batch{batch}_n{n}", extra={"fd_direction": direction},
                       transform=transform)


def config_shared_dense(m: int = 2048, n: int = 8192, batch: int = 256, seed: int = 120806,
                        signals=None) -> "SharedDenseInstance":
    """`batch` signals observed through ONE dense Gaussian A (m x n, i.i.d.
    N(0, 1/m)): k = floor(n/50) N(0,1) spikes, noise sigma = 1e-3,
    tau = 1e-2 ||A^T b||_inf per signal.  A comes from PCG64(seed); signal j
    from PCG64(seed * 1000 + j) (support -> amplitudes -> noise), so any
    subset `signals` can be drawn alone."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    A = np.ascontiguousarray(rng.standard_normal((m, n)) / np.sqrt(m))
    idx = list(range(batch)) if signals is None else list(signals)
    k = n // 50
    X = np.zeros((len(idx), n))
    Bm = np.zeros((len(idx), m))
    taus = np.zeros(len(idx))
    for r, j in enumerate(idx):
        srng = np.random.default_rng(np.random.PCG64(seed * 1000 + j))
        X[r] = _sparse_signal(srng, n, k, "normal")
        Bm[r] = A @ X[r] + 1e-3 * srng.standard_normal(m)
        taus[r] = 1e-2 * np.max(np.abs(A.T @ Bm[r]))
    return SharedDenseInstance(A=A, b=Bm, tau=taus, x_true=X, seed=seed, signals=idx,
                               label=f"shared_dense_{batch}_m{m}_n{n}")


@dataclass
class SharedDenseInstance:
    A: np.ndarray          # (m, n), shared by every signal
    b: np.ndarray          # (B, m)
    tau: np.ndarray        # (B,)
    x_true: np.ndarray     # (B, n)
    seed: int
    signals: list
    label: str = ""

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


# --- phase-transition sweep --------------------------------------------------

PHASE_PARAMS = dict(tol=1e-12, tolpcg=1e-6)  # noiseless ranges of the tuning section
PHASE_C_TAU = 1e-6


def phase_transition_grid(n: int = 1024, deltas=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9),
                          rhos=None, trials: int = 10, seed: int = 120807):
    """Noiseless partial-DCT instances over a grid of undersampling
    delta = m/n and sparsity rho = k/m (the average phase-transition
    experiment: m random rows of the orthonormal DCT, k spikes of +-1 at
    random positions, b = A x exactly).  Instance (delta index i, rho index j,
    trial t) draws from PCG64(seed * 10^6 + 10^4 i + 100 j + t).  Returns a
    list of (delta, rho, trial, DCTInstance); tau = 1e-6 ||A^T b||_inf."""
    if rhos is None:
        rhos = tuple(round(0.05 * i, 2) for i in range(1, 20))
    out = []
    for i, d in enumerate(deltas):
        m = max(1, int(round(d * n)))
        for j, r in enumerate(rhos):
            k = max(1, int(round(r * m)))
            for t in range(trials):
                inst = dct_instance(n, m, k, seed=seed * 10 ** 6 + 10 ** 4 * i + 100 * j + t, amp="pm1",
                                    sigma=0.0, c_tau=PHASE_C_TAU, label=f"phase_d{d}_r{r}_t{t}")
                out.append((d, r, t, inst))
    return out
