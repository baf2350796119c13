// Exact Newton directions for the dense operator: the IPM with its PCG
// replaced by a direct solver (Section 5.7, which factorises the reduced
// Newton system (redNewton) by Cholesky).  The system solved is the n x n
// one behind the Theorem (thm:ne2_prec) of Section 4,
//   M d = r_bar,  M = Theta_bar^{-1} + A^T A,
// whose back-substituted 2n direction is the exact solution of (redNewton).
//
// M is stored row-major, n_pad x n_pad (n_pad = n rounded up to a multiple of
// 64, the padding being the identity), in 64 x 64 tiles of which only the
// lower block triangle is used.  K = A^T A is formed once per solve; each
// IPM iteration forms M = K + diag(Theta_bar^{-1}) and factorises it,
// M = L L^T, by a right-looking blocked Cholesky over the team's workgroups:
// per block column j
//   panel   L_ij = M_ij L_jj^{-T}          for i > j
//   update  M_ik -= L_ij L_kj^T            for j < k <= i
// with the diagonal tile j+1 updated, factorised and inverted in LDS by the
// workgroup of rank 0 during the update phase of column j, so a block column
// costs two team barriers.  Every tile product is a 64 x 64 x 64 FP64 MFMA
// product from LDS.  The inverses of the diagonal tiles are kept, so the
// forward and backward sweeps (L y = r_bar, L^T d = y) are block-column
// sweeps of 64 x 64 matrix-vector products, one team barrier per block.
// The corrector reuses the factorisation (same Theta).
#pragma once
#include "common.h"
#include "op_dense.h"

#define DC_NB 64                // tile size
#define DC_LD (DC_NB + 1)       // LDS pitch of a staged tile (doubles)
#define DC_MAX_N 8192           // largest n of the direct variant
// LDS: two staged tiles (the factorisation uses the first as its tile and
// the second for the pivots and a flag)
#define DC_LDS_BYTES ((size_t)2 * DC_NB * DC_LD * sizeof(double))
static_assert(4 * DC_NB + 1 <= DC_NB * DC_LD, "pivot scratch fits the second staging tile");

typedef double dc_acc_t __attribute__((ext_vector_type(4)));

struct OpDenseDirect : OpDense {
  double* K;   // A^T A, n_pad x n_pad row-major (lower tiles; diagonal tiles full)
  double* M;   // Theta_bar^{-1} + A^T A, overwritten by L (lower tiles)
  double* Li;  // inverses of L's diagonal tiles: T tiles, 64 x 64 row-major
  double* y;   // n_pad: the sweeps' vector; on return the solution d
  double* sX;  // LDS staging
  double* sY;
  long npad;
  int T;
};

__device__ __forceinline__ long dc_npad(long n) { return (n + DC_NB - 1) / DC_NB * DC_NB; }

__device__ __forceinline__ double* dc_tile(double* base, long npad, int I, int J) {
  return base + (long)I * DC_NB * npad + (long)J * DC_NB;
}

// u-th tile of the lower block triangle of an S x S block matrix, rows in
// order: u = i (i + 1) / 2 + k, 0 <= k <= i.
__device__ __forceinline__ void dc_tri_index(int u, int& i, int& k) {
  int r = (int)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= u) ++r;
  while (r * (r + 1) / 2 > u) --r;
  i = r;
  k = u - r * (r + 1) / 2;
}

// Stages the 64 x 64 row-major tile g (pitch ld) transposed: s[k][i] = g[i][k].
__device__ __forceinline__ void dc_stage_t(double* s, const double* g, long ld) {
  for (int e = threadIdx.x; e < DC_NB * DC_NB; e += MF_THREADS) {
    const int i = e >> 6, k = e & 63;
    s[k * DC_LD + i] = g[(long)i * ld + k];
  }
}

// Stages rows [0, rows) and columns [0, cols) of g (pitch ld) as is,
// zero elsewhere: s[k][i] = g[k][i].
__device__ __forceinline__ void dc_stage(double* s, const double* g, long ld, int rows, int cols) {
  for (int e = threadIdx.x; e < DC_NB * DC_NB; e += MF_THREADS) {
    const int k = e >> 6, i = e & 63;
    s[k * DC_LD + i] = (k < rows && i < cols) ? g[(long)k * ld + i] : 0.0;
  }
}

// acc += X Y^T for staged X (sX[k][i] = X[i][k]) and Y (sY[k][j] = Y[j][k]).
// Wave w holds rows 16 (w >> 1) .. +16 and columns 32 (w & 1) .. +32 as two
// 16 x 16 accumulators: acc[h][r] is C[16 (w >> 1) + (lane >> 4) + 4 r]
// [32 (w & 1) + 16 h + (lane & 15)].
__device__ __forceinline__ void dc_mfma(const double* sX, const double* sY, dc_acc_t (&acc)[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int bi = 16 * (wave >> 1), bj = 32 * (wave & 1);
#pragma unroll 4
  for (int kk = 0; kk < DC_NB; kk += 4) {
    const double a = sX[(kk + lk) * DC_LD + bi + li];
    const double b0 = sY[(kk + lk) * DC_LD + bj + li];
    const double b1 = sY[(kk + lk) * DC_LD + bj + 16 + li];
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[1], 0, 0, 0);
  }
}

// (row, column) of accumulator element (h, r) of this lane
__device__ __forceinline__ int dc_row(int r) { return 16 * ((threadIdx.x >> 6) >> 1) + ((threadIdx.x & 63) >> 4) + 4 * r; }
__device__ __forceinline__ int dc_col(int h) { return 32 * ((threadIdx.x >> 6) & 1) + 16 * h + (threadIdx.x & 15); }

// Cholesky of the SPD tile held in LDS (D, pitch DC_LD; lower triangle read)
// by one workgroup: on return D's lower triangle holds L (tile = L L^T), Lg
// (pitch ld) receives L and Lig (64 x 64 row-major) L^{-1}.  piv: 4 x 64 + 1
// doubles of LDS.  Returns nonzero in every thread if a pivot was not
// positive.
__device__ __noinline__ int dc_factor_tile(double* D, double* piv, double* Lg, long ld, double* Lig) {
  double* col = piv;             // two buffers of the current pivot column
  double* dg = piv + 2 * DC_NB;  // square roots of the pivots
  double* rd = piv + 3 * DC_NB;  // their reciprocals
  int* bad = reinterpret_cast<int*>(piv + 4 * DC_NB);
  // Thread (i, p) keeps row i, columns p, p + 8, ..., p + 56 in registers
  // and eliminates them with the unscaled pivot column:
  // D[i][k] -= D[i][c] D[k][c] / D[c][c] for c < k <= i.
  const int ri = threadIdx.x >> 3, rp = threadIdx.x & 7;
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = D[ri * DC_LD + rp + 8 * q];
  if (threadIdx.x == 0) *bad = 0;
#pragma unroll
  for (int c = 0; c < DC_NB; ++c) {
    double* cb = col + (c & 1) * DC_NB;
    if (rp == (c & 7) && ri >= c) cb[ri] = a[c >> 3];  // publish column c (final since step c - 1)
    __syncthreads();
    if (ri > c) {
      const double f = cb[ri] / cb[c];
#pragma unroll
      for (int q = (c + 1) >> 3; q < 8; ++q) {
        const int k = rp + 8 * q;
        if (k > c && k <= ri) a[q] -= f * cb[k];
      }
    }
  }
  // pivots, then L = D / sqrt(pivot) below the diagonal and sqrt(pivot) on it
  if (rp == (ri & 7)) {
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q == (ri >> 3)) d = a[q];
    if (!(d > 0.0)) *bad = 1;
    const double sq = sqrt(d);
    dg[ri] = sq;
    rd[ri] = 1.0 / sq;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int k = rp + 8 * q;
    const double v = k < ri ? a[q] * rd[k] : (k == ri ? dg[k] : 0.0);
    D[ri * DC_LD + k] = v;
    Lg[(long)ri * ld + k] = v;
  }
  __syncthreads();
  // L^{-1}: column j by the 8 lanes (j, p) of one wave; lane p keeps the
  // entries k = p (mod 8) of the column in registers; forward substitution
  // x_i = (delta_ij - sum_{k < i} L[i][k] x_k) / L[i][i].
  {
    const int j = threadIdx.x >> 3, p = threadIdx.x & 7;
    double xr[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xr[q] = 0.0;
#pragma unroll
    for (int i = 0; i < DC_NB; ++i) {
      double part0 = 0.0, part1 = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (8 * q < i) {  // the slot may hold a k < i
          const int k = p + 8 * q;
          if (k < i) {
            if (q & 1) part1 += D[i * DC_LD + k] * xr[q];
            else part0 += D[i * DC_LD + k] * xr[q];
          }
        }
      }
      double part = part0 + part1;
      part += __shfl_xor(part, 1, 64);
      part += __shfl_xor(part, 2, 64);
      part += __shfl_xor(part, 4, 64);
      const double xi = ((i == j ? 1.0 : 0.0) - part) * rd[i];
      if (p == (i & 7)) xr[i >> 3] = xi;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) Lig[(p + 8 * q) * DC_NB + j] = xr[q];
  }
  __syncthreads();
  return *bad;
}

// y_i -= T y_j for the 64 x 64 tile T (pitch ld); one workgroup.
__device__ __forceinline__ void dc_gemv_sub(double* yi, const double* Tg, long ld, const double* yj) {
  const int r = threadIdx.x >> 3, p = threadIdx.x & 7;
  const double* row = Tg + (long)r * ld + 8 * p;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += row[c] * yj[8 * p + c];
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 4, 64);
  if (p == 0) yi[r] -= s;
}

// y_i -= T^T x_j for the 64 x 64 tile T (pitch ld); red: 8 x 64 doubles of LDS.
__device__ __forceinline__ void dc_gemv_t_sub(double* yi, const double* Tg, long ld, const double* xj, double* red) {
  const int c = threadIdx.x & 63, p = threadIdx.x >> 6;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) s += Tg[(long)(8 * p + r) * ld + c] * xj[8 * p + r];
  red[p * DC_NB + c] = s;
  __syncthreads();
  if (threadIdx.x < DC_NB) {
    double t = red[threadIdx.x];
#pragma unroll
    for (int q = 1; q < 8; ++q) t += red[q * DC_NB + threadIdx.x];
    yi[threadIdx.x] -= t;
  }
  __syncthreads();
}

// v <- Li v (trans = 0) or Li^T v (trans = 1) for the block v (64) and the
// 64 x 64 row-major Li; buf: 64 + 8 x 64 doubles of LDS.
__device__ __forceinline__ void dc_tri_apply(double* v, const double* Li, int trans, double* buf) {
  double* vin = buf;
  double* red = buf + DC_NB;
  if (threadIdx.x < DC_NB) vin[threadIdx.x] = v[threadIdx.x];
  __syncthreads();
  const int c = threadIdx.x & 63, p = threadIdx.x >> 6;
  double s = 0.0;
  if (!trans) {
    // out[c] = sum_k Li[c][k] vin[k]: lanes of a wave take one row each
#pragma unroll
    for (int k = 0; k < 8; ++k) s += Li[c * DC_NB + 8 * p + k] * vin[8 * p + k];
  } else {
    // out[c] = sum_k Li[k][c] vin[k]
#pragma unroll
    for (int k = 0; k < 8; ++k) s += Li[(8 * p + k) * DC_NB + c] * vin[8 * p + k];
  }
  red[p * DC_NB + c] = s;
  __syncthreads();
  if (threadIdx.x < DC_NB) {
    double t = red[threadIdx.x];
#pragma unroll
    for (int q = 1; q < 8; ++q) t += red[q * DC_NB + threadIdx.x];
    v[threadIdx.x] = t;
  }
  __syncthreads();
}

// K = A^T A (lower tiles), once per solve.  Also clears the breakdown flag.
__device__ __noinline__ int direct_setup(Ctx& cx, OpDenseDirect& op, int* err) {
  if (cx.t.rank == 0 && threadIdx.x == 0) __hip_atomic_store(err, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int ntile = op.T * (op.T + 1) / 2;
  for (int u = cx.t.rank; u < ntile; u += cx.t.size) {
    int I, J;
    dc_tri_index(u, I, J);
    dc_acc_t acc[2] = {dc_acc_t{0, 0, 0, 0}, dc_acc_t{0, 0, 0, 0}};
    // columns of A in the tile (I, J < T, so at least one each; the padding reads zeros)
    const int ci = (int)min((long)DC_NB, op.n - (long)I * DC_NB);
    const int cj = (int)min((long)DC_NB, op.n - (long)J * DC_NB);
    for (long r0 = 0; r0 < op.m; r0 += DC_NB) {
      const int rows = (int)min((long)DC_NB, op.m - r0);
      // X[i][k] = A[r0 + k][64 I + i], Y[j][k] = A[r0 + k][64 J + j]
      dc_stage(op.sX, op.A + r0 * op.lda + (long)I * DC_NB, op.lda, rows, ci);
      dc_stage(op.sY, op.A + r0 * op.lda + (long)J * DC_NB, op.lda, rows, cj);
      __syncthreads();
      dc_mfma(op.sX, op.sY, acc);
      __syncthreads();
    }
    double* Kt = dc_tile(op.K, op.npad, I, J);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) Kt[(long)dc_row(r) * op.npad + dc_col(h)] = acc[h][r];
  }
  return team_barrier(cx.t) ? ST_ABORTED : 0;
}

// M = K + diag(tb) (identity on the padding) and its Cholesky factorisation.
__device__ __noinline__ int direct_factor(Ctx& cx, OpDenseDirect& op, const double* tb, int* err) {
  const long np = op.npad;
  const int T = op.T;
  double* D = op.sX;
  double* piv = op.sY;
  // form M; rank 0 forms, factorises and inverts the first diagonal tile
  const int ntile = T * (T + 1) / 2;
  for (int u = cx.t.rank; u < ntile; u += cx.t.size) {
    int I, J;
    dc_tri_index(u, I, J);
    const double* Kt = dc_tile(op.K, np, I, J);
    double* Mt = dc_tile(op.M, np, I, J);
    for (int e = threadIdx.x; e < DC_NB * DC_NB; e += MF_THREADS) {
      const int r = e >> 6, c = e & 63;
      double v = Kt[(long)r * np + c];
      if (I == J && r == c) {
        const long g = (long)I * DC_NB + r;
        v += g < op.n ? tb[g] : 1.0;
      }
      if (u == 0) D[r * DC_LD + c] = v;
      else Mt[(long)r * np + c] = v;
    }
    if (u == 0) {
      __syncthreads();
      if (dc_factor_tile(D, piv, op.M, np, op.Li) && threadIdx.x == 0)
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (team_barrier(cx.t)) return ST_ABORTED;
  for (int j = 0; j + 1 < T; ++j) {
    // panel: L_ij = M_ij L_jj^{-T}
    const double* Lij_inv = op.Li + (long)j * DC_NB * DC_NB;
    for (int i = j + 1 + cx.t.rank; i < T; i += cx.t.size) {
      double* Mt = dc_tile(op.M, np, i, j);
      dc_stage_t(op.sX, Mt, np);
      dc_stage_t(op.sY, Lij_inv, DC_NB);
      __syncthreads();
      dc_acc_t acc[2] = {dc_acc_t{0, 0, 0, 0}, dc_acc_t{0, 0, 0, 0}};
      dc_mfma(op.sX, op.sY, acc);
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) Mt[(long)dc_row(r) * np + dc_col(h)] = acc[h][r];
    }
    if (team_barrier(cx.t)) return ST_ABORTED;
    // update: M_ik -= L_ij L_kj^T for j < k <= i; tile (j+1, j+1) first, by
    // rank 0, which then factorises it
    const int S = T - 1 - j;
    const int nupd = S * (S + 1) / 2;
    // rank 0 takes only the diagonal tile (it factorises it afterwards); the
    // other tiles go to the other ranks
    const int ustart = cx.t.size == 1 ? 0 : (cx.t.rank == 0 ? 0 : cx.t.rank);
    const int ustep = cx.t.size == 1 ? 1 : (cx.t.rank == 0 ? nupd : cx.t.size - 1);
    for (int u = ustart; u < nupd; u += ustep) {
      int ii, kk;
      dc_tri_index(u, ii, kk);
      const int i = j + 1 + ii, k = j + 1 + kk;
      dc_stage_t(op.sX, dc_tile(op.M, np, i, j), np);
      dc_stage_t(op.sY, dc_tile(op.M, np, k, j), np);
      __syncthreads();
      dc_acc_t acc[2] = {dc_acc_t{0, 0, 0, 0}, dc_acc_t{0, 0, 0, 0}};
      dc_mfma(op.sX, op.sY, acc);
      __syncthreads();
      double* Mt = dc_tile(op.M, np, i, k);
      if (u == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = dc_row(r), col = dc_col(h);
            D[row * DC_LD + col] = Mt[(long)row * np + col] - acc[h][r];
          }
        __syncthreads();
        if (dc_factor_tile(D, piv, Mt, np, op.Li + (long)(j + 1) * DC_NB * DC_NB) && threadIdx.x == 0)
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const long o = (long)dc_row(r) * np + dc_col(h);
            Mt[o] -= acc[h][r];
          }
      }
    }
    if (team_barrier(cx.t)) return ST_ABORTED;
  }
  return ld_flag(err) ? ST_PCG_BREAKDOWN : 0;
}

// d = M^{-1} r_bar from the factorisation: forward sweep L y = r_bar, then
// backward sweep L^T d = y; the result is left in op.y (n_pad entries).
__device__ __noinline__ int direct_solve(Ctx& cx, OpDenseDirect& op, const double* rb) {
  const long np = op.npad;
  const int T = op.T;
  double* y = op.y;
  double* buf = op.sX;  // 64 + 8 x 64 doubles
  // y = r_bar (zero on the padding); rank 0 starts the forward sweep
  const long nthr = (long)cx.t.size * MF_THREADS;
  for (long g = DC_NB + (long)cx.t.rank * MF_THREADS + threadIdx.x; g < np; g += nthr) y[g] = g < op.n ? rb[g] : 0.0;
  if (cx.t.rank == 0) {
    if (threadIdx.x < DC_NB) y[threadIdx.x] = threadIdx.x < op.n ? rb[threadIdx.x] : 0.0;
    __syncthreads();
    dc_tri_apply(y, op.Li, 0, buf);
    if (T == 1) dc_tri_apply(y, op.Li, 1, buf);
  }
  if (team_barrier(cx.t)) return ST_ABORTED;
  // forward: y_i -= L_ij y_j (i > j); rank 0 finishes block j + 1
  for (int j = 0; j + 1 < T; ++j) {
    for (int i = j + 1 + cx.t.rank; i < T; i += cx.t.size) {
      dc_gemv_sub(y + (long)i * DC_NB, dc_tile(op.M, np, i, j), np, y + (long)j * DC_NB);
      if (i == j + 1) {
        __syncthreads();
        double* Li = op.Li + (long)i * DC_NB * DC_NB;
        dc_tri_apply(y + (long)i * DC_NB, Li, 0, buf);
        if (i == T - 1) dc_tri_apply(y + (long)i * DC_NB, Li, 1, buf);  // starts the backward sweep
      }
    }
    if (team_barrier(cx.t)) return ST_ABORTED;
  }
  // backward: y_i -= L_ji^T d_j (i < j); rank 0 finishes block j - 1
  for (int j = T - 1; j >= 1; --j) {
    for (int q = cx.t.rank; q < j; q += cx.t.size) {
      const int i = j - 1 - q;
      dc_gemv_t_sub(y + (long)i * DC_NB, dc_tile(op.M, np, j, i), np, y + (long)j * DC_NB, buf + DC_NB);
      if (q == 0) dc_tri_apply(y + (long)i * DC_NB, op.Li + (long)i * DC_NB * DC_NB, 1, buf);
    }
    if (team_barrier(cx.t)) return ST_ABORTED;
  }
  return 0;
}
