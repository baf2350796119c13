// Dense operator: explicit row-major m x n matrix A (leading dimension lda).
// The Newton-operator product K d = A^T (A d) and the residual
// A^T (A x - b) are two streaming passes over A, split at a team barrier:
//   pass A: d (from the functor, one value per index) -> D        (index tiles)
//   pass B: y = A D (- b) -> Yv, partial sums of y^2, b.y        (row blocks)
//   pass C: t = A^T Yv -> functor epilogue                        (column blocks)
// Rows are read with all 256 lanes of a workgroup on consecutive columns;
// columns are read by DN_RG row-groups x 64 lanes (512-byte row segments).
#pragma once
#include "common.h"

#define DN_TA 1024   // indices per pass-A item
#define DN_CB 64     // columns per pass-C item
#define DN_RBMAX 16  // max rows per pass-B item
#define DN_RG (MF_THREADS / 64)  // row groups of pass C

enum { DB_HAPPLY = 0, DB_RESID = 1, DB_OUT = 2 };

struct OpDense {
  long n;
  long m;
  long lda;
  const double* __restrict__ A;
  const double* __restrict__ b;
  double* D;
  double* Yv;
  int RB;
  double* lds;  // reduction scratch: >= MF_WAVES * DN_RBMAX + DN_RG * DN_CB doubles

  __device__ int nA() const { return (int)((n + DN_TA - 1) / DN_TA); }
  __device__ int nB() const { return (int)((m + RB - 1) / RB); }
  __device__ int nC() const { return (int)((n + DN_CB - 1) / DN_CB); }

  template <class F>
  __device__ __forceinline__ void passA(int item, F& f) {
    const long base = (long)item * DN_TA;
    constexpr int U = DN_TA / MF_THREADS;
    typename F::In in[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long i = base + threadIdx.x + k * MF_THREADS;
      if (i < n) f.load(i, in[k]);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long i = base + threadIdx.x + k * MF_THREADS;
      if (i < n) D[i] = f.gather(i, in[k]);
    }
  }

  // y_r = A[r,:] . D for the rows of the block; mode RESID subtracts b,
  // mode OUT writes y to `out` instead of Yv.  acc[0] += sum y^2,
  // acc[1] += sum b*y (RESID).  Results valid in thread 0.
  __device__ __forceinline__ void passB(int item, int mode, double (&acc)[2], double* out) {
    const long r0 = (long)item * RB;
    const int nr = (int)((m - r0) < RB ? (m - r0) : RB);
    double s[DN_RBMAX];
#pragma unroll
    for (int r = 0; r < DN_RBMAX; ++r) s[r] = 0.0;
    for (long c = threadIdx.x; c < n; c += MF_THREADS) {
      const double dv = D[c];
#pragma unroll
      for (int r = 0; r < DN_RBMAX; ++r)
        if (r < nr) s[r] += A[(r0 + r) * lda + c] * dv;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < DN_RBMAX; ++r) {
      if (r < nr) {
        const double v = wave_reduce(0, s[r]);
        if (lane == 0) lds[wave * DN_RBMAX + r] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int r = 0; r < nr; ++r) {
        double y = lds[r];
        for (int w = 1; w < MF_WAVES; ++w) y += lds[w * DN_RBMAX + r];
        if (mode == DB_RESID) {
          const double bb = b[r0 + r];
          y -= bb;
          acc[1] += bb * y;
        }
        acc[0] += y * y;
        if (mode == DB_OUT) out[r0 + r] = y;
        else Yv[r0 + r] = y;
      }
    }
    __syncthreads();
  }

  template <class F>
  __device__ __forceinline__ void passC(int item, F& f) {
    const long c0 = (long)item * DN_CB;
    const int col = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const long c = c0 + col;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < n) {
      long i = rg;
      for (; i + 3 * DN_RG < m; i += 4 * DN_RG) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a4[u] += A[(i + DN_RG * u) * lda + c] * Yv[i + DN_RG * u];
      }
      for (; i < m; i += DN_RG) a4[0] += A[i * lda + c] * Yv[i];
    }
    double* red = lds + MF_WAVES * DN_RBMAX;
    red[rg * 64 + col] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    if (rg == 0 && c < n) {
      double t = red[col];
      for (int g = 1; g < DN_RG; ++g) t += red[g * 64 + col];
      typename F::In in;
      f.load(c, in);
      f.scatter(c, t, in);
    }
    __syncthreads();
  }

  // sum of squares of the rows of a block (setup: ||A||_F^2), thread 0
  __device__ __forceinline__ double frob_block(int item) {
    const long r0 = (long)item * RB;
    const int nr = (int)((m - r0) < RB ? (m - r0) : RB);
    double s = 0.0;
    for (int r = 0; r < nr; ++r)
      for (long c = threadIdx.x; c < n; c += MF_THREADS) {
        const double a = A[(r0 + r) * lda + c];
        s += a * a;
      }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_reduce(0, s);
    if (lane == 0) lds[wave] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
      tot = lds[0];
      for (int w = 1; w < MF_WAVES; ++w) tot += lds[w];
    }
    __syncthreads();
    return tot;
  }
};
