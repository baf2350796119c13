// Many signals observed through ONE dense matrix A (m x n, row-major):
// the IPMs of all signals advance in lock step, one operator application per
// round, so that the operator becomes two matrix-matrix products with FP64
// MFMA instead of one matrix pass per signal:
//   Y = A D       (m x B; column j = A d_j, minus b_j when signal j asks for
//                  its residual A x - b)
//   T = A^T Y     (n x B; column j = A^T A d_j, or A^T (A x_j - b_j))
// where d_j is the operator input each signal requested in the previous round
// (the PCG direction p_u - p_v, or x = u - v for a residual).  Between the
// products every signal's own IPM (Section 5.1 algorithm) and PCG (Section 4)
// run as a resumable state machine on one workgroup, which consumes its
// columns of Y and T and requests the next product.  Signals that have
// finished keep a zero column (masked); a column group of 64 signals that has
// finished entirely is skipped.  Each signal computes exactly the iterates of
// the single-signal method: the rounds only interleave them.
#pragma once
#include "common.h"
#include "ipm.h"

typedef double double4_t __attribute__((ext_vector_type(4)));

#define LS_TM 128  // output rows of a GEMM work item
#define LS_TN 64   // output columns (signals) of a GEMM work item
#define LS_TK 32   // K chunk staged in LDS per step
#define LS_PAD 2   // LDS row padding (doubles) against bank conflicts
#define LS_SPLIT 4 // split of K = n in the first product (partial sums reduced in order)

// request modes of a signal's column
enum { RQ_NONE = 0, RQ_HAPPLY = 1, RQ_RESID = 2 };
// what the next operator result is for
enum { PH_RES = 0, PH_TRIAL = 1, PH_PCG = 2, PH_DONE = 3 };

struct SigState {
  int phase, corr, k, pcg_it;
  int pcg_total, ncorr, status, pad0;
  long nmat;
  double aP_prev, aD_prev, aP, aD;
  double sigma, mu, mu_t;
  double rhs2, rty, ptp;  // PCG: ||rhs||^2, r^T P^{-1} r, p^T Theta^{-1} p
  double relgap, primal, dual;
};

struct LArgs {
  const InstDesc* inst;  // per-signal offsets (b, x, state) and tau
  int B;        // signals
  long n, m;
  const double* A;     // m x n row-major (lda = n), shared
  const double* b;     // B x m
  double* x;           // B x n output
  double* state;       // B x 4n (may be null)
  DevInfo* info;       // B
  DevParams prm;
  // workspace
  SigState* st;        // B
  int* mode;           // B request modes
  double2* V;          // B x 8 vectors of n pairs: Z S TI X R P DZ DS
  double* D;           // B x n requests
  double* Y;           // B x m
  double* Yp;          // LS_SPLIT x B x m partial products
  double* T;           // B x n
  double* part;        // reduction partials (>= m/8 + 64 doubles)
  double* scal;        // scalars shared by the grid: [0] rho
  int* abort_flag;
  unsigned long long* ctl;
  unsigned long long spin_ticks;
};

// ---------------------------------------------------------------------------
// GEMM work item on FP64 MFMA (v_mfma_f64_16x16x4_f64: lane l holds A[l%16][l/16]
// and B[l/16][l%16]; accumulator element r of lane l is C[l/16 + 4r][l%16],
// as measured on gfx950).
//   C[LS_TM x LS_TN] = sum_{k in [k0, k1)} Aop[i][k] * Bop[k][j]
// Aop is either K-contiguous (a_kmajor = 0: Aop[i][k] = A[(i0+i)*lda + k],
// the first product) or M-contiguous (a_kmajor = 1: Aop[c][k] = A[k*lda + c0+c],
// A^T in the second product).  Bop[k][j] = Bm[(j0+j)*ldb + k] (each signal's
// column contiguous).  Rows past `M` and columns past `N` read zeros.
// Eight waves: wave w owns the 32 x 32 block at rows 32 (w/2), columns
// 32 (w%2), as four 16 x 16 accumulators, so each A and B fragment read from
// LDS feeds two MFMAs.
// ---------------------------------------------------------------------------
struct GemmLDS {
  double a[2][LS_TK][LS_TM + LS_PAD];
  double b[2][LS_TK][LS_TN + LS_PAD];
};

constexpr int LS_EA = LS_TM * LS_TK / MF_THREADS;  // A-tile elements per thread
constexpr int LS_EB = LS_TN * LS_TK / MF_THREADS;  // B-tile elements per thread
static_assert(LS_EA * MF_THREADS == LS_TM * LS_TK && LS_EB * MF_THREADS == LS_TN * LS_TK, "tile split");

// Global loads of one K chunk into registers (zeros outside [0, M) x [0, K)
// and past column N).
__device__ __forceinline__ void gemm_load(const double* __restrict__ A, long lda, int a_kmajor, long i0, long M,
                                          const double* __restrict__ Bm, long ldb, long j0, long N, long k,
                                          long K, double (&ra)[LS_EA], double (&rb)[LS_EB]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < LS_EA; ++e) {
    const int q = t + e * MF_THREADS;
    long gi, gk;
    if (!a_kmajor) {  // LS_TK consecutive k of one row
      gi = i0 + q / LS_TK;
      gk = k + q % LS_TK;
    } else {          // LS_TM consecutive columns of one k
      gk = k + q / LS_TM;
      gi = i0 + q % LS_TM;
    }
    ra[e] = (gi < M && gk < K) ? (a_kmajor ? A[gk * lda + gi] : A[gi * lda + gk]) : 0.0;
  }
#pragma unroll
  for (int e = 0; e < LS_EB; ++e) {  // LS_TK consecutive k of one column
    const int q = t + e * MF_THREADS;
    const long gj = j0 + q / LS_TK, gk = k + q % LS_TK;
    rb[e] = (gj < N && gk < K) ? Bm[gj * ldb + gk] : 0.0;
  }
}

__device__ __forceinline__ void gemm_store_lds(GemmLDS& s, int buf, int a_kmajor, const double (&ra)[LS_EA],
                                               const double (&rb)[LS_EB]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < LS_EA; ++e) {
    const int q = t + e * MF_THREADS;
    if (!a_kmajor) s.a[buf][q % LS_TK][q / LS_TK] = ra[e];
    else s.a[buf][q / LS_TM][q % LS_TM] = ra[e];
  }
#pragma unroll
  for (int e = 0; e < LS_EB; ++e) {
    const int q = t + e * MF_THREADS;
    s.b[buf][q % LS_TK][q / LS_TK] = rb[e];
  }
}

// Accumulates the work item into acc[4] (per wave, see above).
__device__ __forceinline__ void gemm_item(GemmLDS& s, const double* __restrict__ A, long lda, int a_kmajor, long i0,
                                          long M, const double* __restrict__ Bm, long ldb, long j0, long N, long k0,
                                          long k1, double4_t (&acc)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bi = (wave >> 1) * 32, bj = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = double4_t{0, 0, 0, 0};
  double ra[LS_EA], rb[LS_EB];
  gemm_load(A, lda, a_kmajor, i0, M, Bm, ldb, j0, N, k0, k1, ra, rb);
  gemm_store_lds(s, 0, a_kmajor, ra, rb);
  __syncthreads();
  int buf = 0;
  for (long k = k0; k < k1; k += LS_TK) {
    const bool more = k + LS_TK < k1;
    if (more) gemm_load(A, lda, a_kmajor, i0, M, Bm, ldb, j0, N, k + LS_TK, k1, ra, rb);
#pragma unroll
    for (int kk = 0; kk < LS_TK; kk += 4) {
      const double a0 = s.a[buf][kk + lk][bi + li];
      const double a1 = s.a[buf][kk + lk][bi + 16 + li];
      const double b0 = s.b[buf][kk + lk][bj + li];
      const double b1 = s.b[buf][kk + lk][bj + 16 + li];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
    }
    if (more) gemm_store_lds(s, buf ^ 1, a_kmajor, ra, rb);
    __syncthreads();
    buf ^= 1;
  }
}

// Writes the wave's four accumulators: C[(j0 + j) * ldc + i0 + i] for the
// columns in [j0, N) and rows in [i0, M).
__device__ __forceinline__ void gemm_store(double* C, long ldc, long i0, long M, long j0, long N,
                                           const double4_t (&acc)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bi = (wave >> 1) * 32, bj = (wave & 1) * 32;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const long j = j0 + bj + 16 * (h & 1) + (lane & 15);
    if (j >= N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long i = i0 + bi + 16 * (h >> 1) + (lane >> 4) + 4 * r;
      if (i < M) C[j * ldc + i] = acc[h][r];
    }
  }
}

// ---------------------------------------------------------------------------
// Signal phase: one workgroup runs one signal's method between two operator
// applications.  Reductions are per workgroup in a fixed order.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void wg_allreduce(const int (&kinds)[K], double (&v)[K], double* red) {
  __shared__ double bc[MF_MAXK];
  wg_reduce<K>(kinds, v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) bc[j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = bc[j];
  __syncthreads();
}

struct Sig {
  long n, m;
  double tau;
  double2 *Z, *S, *TI, *X, *R, *P, *DZ, *DS;
  const double* t;   // A^T (A d) or A^T (A x - b)
  const double* y;   // A d or A x - b
  const double* b;
  double* d;         // next request
  int* mode;
  double* red;
};

__device__ __forceinline__ Sig make_sig(const LArgs& a, const InstDesc* inst, int j, double* red) {
  Sig g;
  g.n = a.n;
  g.m = a.m;
  g.tau = inst[j].tau;
  double2* v = a.V + (size_t)j * 8 * a.n;
  g.Z = v;
  g.S = v + a.n;
  g.TI = v + 2 * a.n;
  g.X = v + 3 * a.n;
  g.R = v + 4 * a.n;
  g.P = v + 5 * a.n;
  g.DZ = v + 6 * a.n;
  g.DS = v + 7 * a.n;
  g.t = a.T + (size_t)j * a.n;
  g.y = a.Y + (size_t)j * a.m;
  g.b = a.b + inst[j].m_off;
  g.d = a.D + (size_t)j * a.n;
  g.mode = a.mode + j;
  g.red = red;
  return g;
}

// The signal's method from the current phase to its next operator request
// (or to its end).  `st` is the signal's saved state.
__device__ __forceinline__ void sig_advance(const LArgs& a, const InstDesc* inst, int j, SigState& st, Sig& g,
                                            double rho) {
  const DevParams& prm = a.prm;
  const long n = g.n, m = g.m;
  const int tid = threadIdx.x;
  const double tau = g.tau;
  double rr = 0.0;
  int done = 0;
  bool pcg_end = false;

  if (st.phase == PH_RES || st.phase == PH_TRIAL) {
    st.nmat += 2;
    if (st.phase == PH_RES) {
      // gap terms at the current point (Section 5.1; relative gap as in the oracle's reading)
      double v[5] = {0.0, 0.0, -__builtin_inf(), 0.0, 0.0};
      const int kinds[5] = {0, 0, 1, 0, 0};
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i];
        v[0] += z.x + z.y;
        v[1] += z.x * s.x + z.y * s.y;
        v[2] = fmax(v[2], fabs(g.t[i]));
      }
      for (long i = tid; i < m; i += MF_THREADS) {
        const double yy = g.y[i];
        v[3] += yy * yy;
        v[4] += g.b[i] * yy;
      }
      wg_allreduce<5>(kinds, v, g.red);
      const double sumz = v[0], zs = v[1], ginf = v[2], rb2 = v[3], brb = v[4];
      st.mu = zs / (2.0 * (double)n);
      st.primal = tau * sumz + 0.5 * rb2;
      const double th = ginf <= tau ? 1.0 : tau / ginf;
      st.dual = -0.5 * th * th * rb2 - th * brb;
      st.relgap = (st.primal - st.dual) / (1.0 + fabs(st.primal));
      if (!isfinite(st.relgap)) {
        st.status = ST_NONFINITE;
        done = 1;
      } else if (st.relgap <= prm.tol) {
        st.status = ST_CONVERGED;
        done = 1;
      } else if (st.k > prm.maxiters) {
        st.status = ST_MAXITER;
        done = 1;
      }
      if (!done) {
        st.sigma = (st.k != 1 && (st.aP_prev <= prm.alpha_bar || st.aD_prev <= prm.alpha_bar)) ? prm.sigma2
                                                                                               : prm.sigma1;
        // rhs = f_z + Z^{-1} f_s (eqs. (fzfs), (redNewton)), Theta^{-1} = s / z
        double w[3] = {0.0, 0.0, 0.0};
        const int k3[3] = {0, 0, 0};
        const double sm = st.sigma * st.mu;
        for (long i = tid; i < n; i += MF_THREADS) {
          const double2 z = g.Z[i], s = g.S[i];
          const double gi = g.t[i];
          const double2 ti = make_double2(s.x / z.x, s.y / z.y);
          const double ru = (s.x - (tau + gi)) + (sm - z.x * s.x) / z.x;
          const double rv = (s.y - (tau - gi)) + (sm - z.y * s.y) / z.y;
          double yu, yv;
          precond_apply(ti.x, ti.y, rho, ru, rv, yu, yv);
          g.TI[i] = ti;
          g.R[i] = make_double2(ru, rv);
          g.X[i] = make_double2(0.0, 0.0);
          g.P[i] = make_double2(yu, yv);
          g.d[i] = yu - yv;
          w[0] += ru * ru + rv * rv;
          w[1] += ru * yu + rv * yv;
          w[2] += ti.x * yu * yu + ti.y * yv * yv;
        }
        wg_allreduce<3>(k3, w, g.red);
        st.rhs2 = w[0];
        st.rty = w[1];
        st.ptp = w[2];
        st.corr = 0;
        st.pcg_it = 0;
        rr = st.rhs2;
      }
    } else {
      // corrector right-hand side at the trial point (reading: only f_z, f_s
      // and mu move there; Theta and Z^{-1} stay at the current point)
      double v[1] = {0.0};
      const int k1[1] = {0};
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i], dz = g.DZ[i], ds = g.DS[i];
        const double ztu = z.x + st.aP * dz.x, ztv = z.y + st.aP * dz.y;
        const double stu = s.x + st.aD * ds.x, stv = s.y + st.aD * ds.y;
        v[0] += ztu * stu + ztv * stv;
      }
      wg_allreduce<1>(k1, v, g.red);
      st.mu_t = v[0] / (2.0 * (double)n);
      const double sm = prm.sigma3 * st.mu_t;
      double w[3] = {0.0, 0.0, 0.0};
      const int k3[3] = {0, 0, 0};
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i], dz = g.DZ[i], ds = g.DS[i], ti = g.TI[i];
        const double gi = g.t[i];
        const double ztu = z.x + st.aP * dz.x, ztv = z.y + st.aP * dz.y;
        const double stu = s.x + st.aD * ds.x, stv = s.y + st.aD * ds.y;
        const double ru = (stu - (tau + gi)) + (sm - ztu * stu) / z.x;
        const double rv = (stv - (tau - gi)) + (sm - ztv * stv) / z.y;
        double yu, yv;
        precond_apply(ti.x, ti.y, rho, ru, rv, yu, yv);
        g.R[i] = make_double2(ru, rv);
        g.X[i] = make_double2(0.0, 0.0);
        g.P[i] = make_double2(yu, yv);
        g.d[i] = yu - yv;
        w[0] += ru * ru + rv * rv;
        w[1] += ru * yu + rv * yv;
        w[2] += ti.x * yu * yu + ti.y * yv * yv;
      }
      wg_allreduce<3>(k3, w, g.red);
      st.rhs2 = w[0];
      st.rty = w[1];
      st.ptp = w[2];
      st.corr = 1;
      st.pcg_it = 0;
      rr = st.rhs2;
    }
  } else if (st.phase == PH_PCG) {
    // one PCG iteration with t = A^T A d, d = p_u - p_v (Section 4):
    // p^T H p = p^T Theta^{-1} p + ||A d||^2, the latter from the column A d
    st.pcg_it += 1;
    st.pcg_total += 1;
    st.nmat += 2;
    double v[1] = {0.0};
    const int k1[1] = {0};
    for (long i = tid; i < m; i += MF_THREADS) {
      const double yy = g.y[i];
      v[0] += yy * yy;
    }
    wg_allreduce<1>(k1, v, g.red);
    const double pq = st.ptp + v[0];
    if (!(pq > 0.0)) {
      st.status = isfinite(pq) ? ST_PCG_BREAKDOWN : ST_NONFINITE;
      done = 1;
    } else {
      const double alpha = st.rty / pq;
      double w[2] = {0.0, 0.0};
      const int k2[2] = {0, 0};
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 p = g.P[i], ti = g.TI[i], x = g.X[i], r = g.R[i];
        const double t = g.t[i];
        const double2 xn = make_double2(x.x + alpha * p.x, x.y + alpha * p.y);
        const double2 rn = make_double2(r.x - alpha * (ti.x * p.x + t), r.y - alpha * (ti.y * p.y - t));
        g.X[i] = xn;
        g.R[i] = rn;
        double yu, yv;
        precond_apply(ti.x, ti.y, rho, rn.x, rn.y, yu, yv);
        w[0] += rn.x * rn.x + rn.y * rn.y;
        w[1] += rn.x * yu + rn.y * yv;
      }
      wg_allreduce<2>(k2, w, g.red);
      rr = w[0];
      const double rty_new = w[1];
      const double beta = rty_new / st.rty;
      st.rty = rty_new;
      // the new direction (used only if the PCG goes on) and its p^T Theta^{-1} p
      const bool go = isfinite(rr) && !(rr <= prm.tolpcg * prm.tolpcg * st.rhs2) && st.pcg_it != prm.mxiterpcg;
      if (go) {
        double u[1] = {0.0};
        for (long i = tid; i < n; i += MF_THREADS) {
          const double2 p = g.P[i], ti = g.TI[i], r = g.R[i];
          double yu, yv;
          precond_apply(ti.x, ti.y, rho, r.x, r.y, yu, yv);
          const double2 pn = make_double2(yu + beta * p.x, yv + beta * p.y);
          g.P[i] = pn;
          g.d[i] = pn.x - pn.y;
          u[0] += ti.x * pn.x * pn.x + ti.y * pn.y * pn.y;
        }
        wg_allreduce<1>(k1, u, g.red);
        st.ptp = u[0];
      }
    }
  }

  if (!done && st.phase != PH_DONE) {
    // PCG stopping test (before each operator apply)
    if (!isfinite(rr)) {
      st.status = ST_NONFINITE;
      done = 1;
    } else if (rr <= prm.tolpcg * prm.tolpcg * st.rhs2 || st.pcg_it == prm.mxiterpcg) {
      pcg_end = true;
    } else {
      *g.mode = RQ_HAPPLY;  // d already written
      st.phase = PH_PCG;
      __syncthreads();
      return;
    }
  }

  if (!done && pcg_end) {
    // step: ds = f_s / z - Theta^{-1} dz (eq. (redNewtonB)), step lengths
    double v[2] = {__builtin_inf(), __builtin_inf()};
    const int k2[2] = {2, 2};
    if (!st.corr) {
      const double sm = st.sigma * st.mu;
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i], ti = g.TI[i], dz = g.X[i];
        const double2 ds = make_double2((sm - z.x * s.x) / z.x - ti.x * dz.x, (sm - z.y * s.y) / z.y - ti.y * dz.y);
        g.DZ[i] = dz;
        g.DS[i] = ds;
        if (dz.x < 0) v[0] = fmin(v[0], -z.x / dz.x);
        if (dz.y < 0) v[0] = fmin(v[0], -z.y / dz.y);
        if (ds.x < 0) v[1] = fmin(v[1], -s.x / ds.x);
        if (ds.y < 0) v[1] = fmin(v[1], -s.y / ds.y);
      }
    } else {
      const double sm = prm.sigma3 * st.mu_t;
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i], ti = g.TI[i], dzc = g.X[i], dzp = g.DZ[i], dsp = g.DS[i];
        const double ztu = z.x + st.aP * dzp.x, ztv = z.y + st.aP * dzp.y;
        const double stu = s.x + st.aD * dsp.x, stv = s.y + st.aD * dsp.y;
        const double dsu = (sm - ztu * stu) / z.x - ti.x * dzc.x, dsv = (sm - ztv * stv) / z.y - ti.y * dzc.y;
        const double2 dz = make_double2(dzp.x + dzc.x, dzp.y + dzc.y);
        const double2 ds = make_double2(dsp.x + dsu, dsp.y + dsv);
        g.DZ[i] = dz;
        g.DS[i] = ds;
        if (dz.x < 0) v[0] = fmin(v[0], -z.x / dz.x);
        if (dz.y < 0) v[0] = fmin(v[0], -z.y / dz.y);
        if (ds.x < 0) v[1] = fmin(v[1], -s.x / ds.x);
        if (ds.y < 0) v[1] = fmin(v[1], -s.y / ds.y);
      }
    }
    wg_allreduce<2>(k2, v, g.red);
    st.aP = fmin(1.0, prm.eta * v[0]);
    st.aD = fmin(1.0, prm.eta * v[1]);
    if (st.corr) st.ncorr += 1;
    if (!st.corr && (st.aP <= prm.alpha_tilde || st.aD <= prm.alpha_tilde)) {
      // corrector: residual at the trial point
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], dz = g.DZ[i];
        g.d[i] = (z.x + st.aP * dz.x) - (z.y + st.aP * dz.y);
      }
      *g.mode = RQ_RESID;
      st.phase = PH_TRIAL;
      __syncthreads();
      return;
    }
    if (st.aP < prm.step_min && st.aD < prm.step_min) {
      st.status = ST_STEP_UNDERFLOW;
      done = 1;
    } else {
      // update and request the residual at the new point
      for (long i = tid; i < n; i += MF_THREADS) {
        const double2 z = g.Z[i], s = g.S[i], dz = g.DZ[i], ds = g.DS[i];
        const double2 zn = make_double2(z.x + st.aP * dz.x, z.y + st.aP * dz.y);
        g.Z[i] = zn;
        g.S[i] = make_double2(s.x + st.aD * ds.x, s.y + st.aD * ds.y);
        g.d[i] = zn.x - zn.y;
      }
      st.aP_prev = st.aP;
      st.aD_prev = st.aD;
      st.k += 1;
      *g.mode = RQ_RESID;
      st.phase = PH_RES;
      __syncthreads();
      return;
    }
  }

  // the signal ends: x = u - v, the final (z, s), a zero column
  const InstDesc& dsc = inst[j];
  double* xo = a.x + dsc.n_off;
  double2* so = a.state ? reinterpret_cast<double2*>(a.state + 4 * dsc.n_off) : nullptr;
  for (long i = tid; i < n; i += MF_THREADS) {
    const double2 z = g.Z[i];
    xo[i] = z.x - z.y;
    if (so) {
      so[i] = z;
      so[n + i] = g.S[i];
    }
    g.d[i] = 0.0;
  }
  *g.mode = RQ_NONE;
  st.phase = PH_DONE;
  if (tid == 0) {
    DevInfo inf;
    inf.status = st.status;
    inf.ipm_iters = st.k - 1;
    inf.pcg_iters = st.pcg_total;
    inf.correctors = st.ncorr;
    inf.nmat = st.nmat;
    inf.rel_gap = st.relgap;
    inf.mu = st.mu;
    inf.primal_obj = st.primal;
    inf.dual_obj = st.dual;
    inf.rho = rho;
    a.info[j] = inf;
  }
  __syncthreads();
}

// Start of a signal: z = z0, s = s0, request the residual at x = 0.
__device__ __forceinline__ void sig_init(const LArgs& a, const InstDesc* inst, int j, double* red) {
  Sig g = make_sig(a, inst, j, red);
  const double z0 = a.prm.z0, s0 = a.prm.s0;
  for (long i = threadIdx.x; i < g.n; i += MF_THREADS) {
    g.Z[i] = make_double2(z0, z0);
    g.S[i] = make_double2(s0, s0);
    g.d[i] = z0 - z0;
  }
  if (threadIdx.x == 0) {
    SigState st{};
    st.phase = PH_RES;
    st.k = 1;
    st.status = ST_MAXITER;
    st.aP_prev = st.aD_prev = 1.0;
    st.relgap = __builtin_nan("");
    a.st[j] = st;
    *g.mode = RQ_RESID;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The lock-step kernel: one cooperative launch, every workgroup in one team.
// Per round: first product (split over K, partial sums per slice), ordered
// sum of the slices minus b for residual requests, second product, signal
// phase; a team barrier after each.  The loop ends when no signal requests
// a product.
// ---------------------------------------------------------------------------
#define LS_MAX_GROUPS 1024

__global__ void __launch_bounds__(MF_THREADS) k_mfipm_lockstep(LArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_dyn[];
  __shared__ double red[MF_RED_DOUBLES];
  __shared__ int s_act[LS_MAX_GROUPS];
  __shared__ int s_nact;
  GemmLDS& gs = *reinterpret_cast<GemmLDS*>(lds_dyn);
  Team t;
  t.size = gridDim.x;
  t.id = 0;
  t.rank = blockIdx.x;
  t.gen = 0;
  t.abort_flag = a.abort_flag;
  t.spin_ticks = a.spin_ticks;
  t.ctl = a.ctl;
  if (team_init(t)) return;
  const int G = gridDim.x, rank = blockIdx.x, tid = threadIdx.x;
  const long n = a.n, m = a.m;
  const int B = a.B;
  int aborted = 0;
  // rho: Frobenius-closest multiple of I to A^T A, ||A||_F^2 / n (Section 4)
  double rho = a.prm.rho;
  if (!(rho > 0.0)) {
    const int nblk = (int)((m + 7) / 8);
    for (int it = rank; it < nblk; it += G) {
      double s = 0.0;
      const long r0 = (long)it * 8;
      const long r1 = r0 + 8 < m ? r0 + 8 : m;
      for (long r = r0; r < r1; ++r)
        for (long c = tid; c < n; c += MF_THREADS) {
          const double v = a.A[r * n + c];
          s += v * v;
        }
      double v1[1] = {s};
      const int k1[1] = {0};
      wg_reduce<1>(k1, v1, red);
      if (tid == 0) a.part[(long)it * MF_MAXK] = v1[0];
    }
    aborted = team_barrier(t);
    const int k1[1] = {0};
    double r1[1];
    reduce_items<1>(k1, a.part, nblk, r1, red);
    rho = r1[0] / (double)n;
  }
  if (!aborted) {
    for (int j = rank; j < B; j += G) sig_init(a, a.inst, j, red);
    aborted = team_barrier(t);
  }
  const int ngroups = (B + LS_TN - 1) / LS_TN;
  const int mt1 = (int)((m + LS_TM - 1) / LS_TM);
  const int mt2 = (int)((n + LS_TM - 1) / LS_TM);
  const long kslice = ((n + LS_SPLIT - 1) / LS_SPLIT + LS_TK - 1) / LS_TK * LS_TK;
  const long ystride = (long)B * m;
  while (!aborted) {
    // column groups with at least one request (identical in every workgroup)
    if (tid == 0) {
      int na = 0;
      for (int gi = 0; gi < ngroups; ++gi) {
        int any = 0;
        for (int j = gi * LS_TN; j < B && j < (gi + 1) * LS_TN; ++j) any |= ld_flag(a.mode + j) != RQ_NONE;
        if (any) s_act[na++] = gi;
      }
      s_nact = na;
    }
    __syncthreads();
    const int nact = s_nact;
    if (nact == 0) break;
    // first product, per K slice: Yp[s] = A[:, slice] D[slice, :].  Items
    // that read the same tile of A (same rows and slice, another column group)
    // get indices 8 apart, so that they run on the same XCD (workgroups are
    // dealt to the XCDs round robin) and share that tile in its L2.
    const int tiles1 = mt1 * LS_SPLIT;
    const int items1 = (tiles1 + 7) / 8 * 8 * nact;
    for (int q = rank; q < items1; q += G) {
      const int r8 = q >> 3, base = ((r8 / nact) << 3) + (q & 7);
      if (base >= tiles1) continue;
      const int gi = s_act[r8 % nact], sp = base % LS_SPLIT, mt = base / LS_SPLIT;
      const long k0 = sp * kslice, k1 = (k0 + kslice) < n ? (k0 + kslice) : n;
      double4_t acc[4];
      gemm_item(gs, a.A, n, 0, (long)mt * LS_TM, m, a.D, n, (long)gi * LS_TN, B, k0, k1, acc);
      gemm_store(a.Yp + sp * ystride, m, (long)mt * LS_TM, m, (long)gi * LS_TN, B, acc);
    }
    if ((aborted = team_barrier(t))) break;
    // Y = sum of the slices in order, minus b where the residual is requested
    {
      const long per = (long)LS_TN * m;
      const long tot = (long)nact * per;
      for (long e = (long)rank * MF_THREADS + tid; e < tot; e += (long)G * MF_THREADS) {
        const int gi = s_act[e / per];
        const long rem = e % per;
        const long j = (long)gi * LS_TN + rem / m, i = rem % m;
        if (j >= B) continue;
        const long o = j * m + i;
        double y = a.Yp[o];
        for (int sp = 1; sp < LS_SPLIT; ++sp) y += a.Yp[sp * ystride + o];
        if (ld_flag(a.mode + j) == RQ_RESID) y -= a.b[a.inst[j].m_off + i];
        a.Y[o] = y;
      }
    }
    if ((aborted = team_barrier(t))) break;
    // second product: T = A^T Y (same XCD grouping of the items sharing a
    // column block of A)
    const int items2 = (mt2 + 7) / 8 * 8 * nact;
    for (int q = rank; q < items2; q += G) {
      const int r8 = q >> 3, ct = ((r8 / nact) << 3) + (q & 7);
      if (ct >= mt2) continue;
      const int gi = s_act[r8 % nact];
      double4_t acc[4];
      gemm_item(gs, a.A, n, 1, (long)ct * LS_TM, n, a.Y, m, (long)gi * LS_TN, B, 0, m, acc);
      gemm_store(a.T, n, (long)ct * LS_TM, n, (long)gi * LS_TN, B, acc);
    }
    if ((aborted = team_barrier(t))) break;
    // signal phase
    for (int j = rank; j < B; j += G) {
      if (ld_flag(a.mode + j) == RQ_NONE) continue;
      SigState st = a.st[j];
      Sig g = make_sig(a, a.inst, j, red);
      sig_advance(a, a.inst, j, st, g, rho);
      if (tid == 0) a.st[j] = st;
      __syncthreads();
    }
    if ((aborted = team_barrier(t))) break;
  }
  if (aborted) {
    // report the signals that had not finished
    for (int j = rank; j < B; j += G) {
      if (tid == 0 && a.st[j].phase != PH_DONE) {
        DevInfo inf{};
        inf.status = ST_ABORTED;
        inf.rho = rho;
        inf.rel_gap = __builtin_nan("");
        a.info[j] = inf;
      }
    }
  }
}
