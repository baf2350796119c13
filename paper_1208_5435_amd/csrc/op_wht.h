// Partial Walsh-Hadamard operator A = R_m W, W = H_n / sqrt(n), H_n the
// Hadamard matrix in natural (Sylvester) order, R_m keeping m rows; one of
// the fast orthonormal transforms the paper names beside the partial DCT
// (A A^T = I, so rho = m/n as for the DCT).  W is symmetric and orthogonal:
// A^T A d = W M W d and A^T (A x - b) = W (M W x - b~), M the 0/1 mask of the
// kept coefficients, b~ the scattered b.
//
// Four-step split: n = N1 N2, index i = i1 N2 + i2, H_n = H_N1 (x) H_N2, so
// (H_n d)[k1 N2 + k2] = sum_i2 H_N2[k2, i2] sum_i1 H_N1[k1, i1] d[i1 N2 + i2]:
// column transforms of length N1 (pass A; pass C for the way back), then row
// transforms of length N2 (pass B), with no twiddles between the two.  The
// N1 x N2 intermediate lives in HBM in item-major tiles: column block q
// (2^lcb columns) is the contiguous tile [k1][c], so pass A/C items read and
// write whole tiles and a pass-B item (2^lrb consecutive rows) reads
// 2^(lrb+lcb) contiguous doubles from every tile.  Transforms run in LDS as
// in-place radix-4 (and one radix-2) butterfly stages.  The passes follow the
// partial-DCT operator: pass C chains the next gather and its column
// transform, pass B combines the direction's transform by linearity.
#pragma once
#include "common.h"

#define WH_TILE 8192  // doubles in the LDS tile (64 KiB)

// In-place unnormalised Walsh-Hadamard transform of 2^lcount sequences of
// length 2^lL held in LDS, element (s, i) at buf[(s << lss) + (i << lis)]:
// butterflies (a + b, a - b) on pairs at distance h = 1, 2, 4, ... (two
// distances per stage).  Caller synchronises before; the result is visible
// to the whole workgroup on return.
__device__ __forceinline__ void lds_wht(double* buf, int lL, int lcount, int lis, int lss) {
  const int total = 1 << (lL + lcount);
  int lh = 0;
  while (lh < lL) {
    if (lL - lh >= 2) {
      const int lq = lL - 2;  // log2 quads per sequence
      for (int t = threadIdx.x; t < (total >> 2); t += MF_THREADS) {
        int s, j;
        if (lis == 0) {
          s = t >> lq;
          j = t & ((1 << lq) - 1);
        } else {
          // interleaved sequences: neighbouring lanes take neighbouring
          // sequences (adjacent LDS words) rather than quads 2^(lis+2) apart
          s = t & ((1 << lcount) - 1);
          j = t >> lcount;
        }
        const int i0 = ((j >> lh) << (lh + 2)) | (j & ((1 << lh) - 1));
        const int h = 1 << lh;
        double* p0 = buf + (s << lss);
        const int o0 = i0 << lis, o1 = (i0 + h) << lis, o2 = (i0 + 2 * h) << lis, o3 = (i0 + 3 * h) << lis;
        const double e0 = p0[o0], e1 = p0[o1], e2 = p0[o2], e3 = p0[o3];
        const double a = e0 + e1, b = e0 - e1, c = e2 + e3, d = e2 - e3;
        p0[o0] = a + c;
        p0[o1] = b + d;
        p0[o2] = a - c;
        p0[o3] = b - d;
      }
      lh += 2;
    } else {
      const int lp = lL - 1;  // log2 pairs per sequence
      for (int t = threadIdx.x; t < (total >> 1); t += MF_THREADS) {
        int s, j;
        if (lis == 0) {
          s = t >> lp;
          j = t & ((1 << lp) - 1);
        } else {
          s = t & ((1 << lcount) - 1);
          j = t >> lcount;
        }
        const int i0 = ((j >> lh) << (lh + 1)) | (j & ((1 << lh) - 1));
        double* p0 = buf + (s << lss);
        const int o0 = i0 << lis, o1 = (i0 + (1 << lh)) << lis;
        const double e0 = p0[o0], e1 = p0[o1];
        p0[o0] = e0 + e1;
        p0[o1] = e0 - e1;
      }
      lh += 1;
    }
    __syncthreads();
  }
}

// pass-B modes, as for the partial DCT
enum { WB_HAPPLY = 0, WB_RESID = 1, WB_FWDOUT = 2, WB_RESID_STEP = 3, WB_RESID_TRIAL = 4 };

struct OpWht {
  long n;
  long m;
  int l1, l2, N1, N2;
  int lcb;  // log2 columns of a pass-A/C item
  int lrb;  // log2 rows of a pass-B item
  const int* __restrict__ rows;
  const double* __restrict__ b;
  double* Y1;   // column transforms of the operator input (PCG: of the next direction)
  double* Y1p;  // column transforms of the current search direction
  double* Y2;   // row-transformed result before the column transforms back
  double* Yx;   // column transforms of the current x = u - v
  double* Yd;   // column transforms of the step direction
  unsigned char* mask;  // natural coefficient order, n bytes
  double* bt;           // b scattered to its coefficients, n doubles
  double* XS;           // coefficients of a forward product, n doubles
  double* tile;         // LDS
  double scale;         // 1 / sqrt(n)

  __device__ int nA() const { return N2 >> lcb; }
  __device__ int nB() const { return N1 >> lrb; }
  __device__ int nC() const { return N2 >> lcb; }
  __device__ __forceinline__ long coef_pos(long kk) const { return kk; }
  // element (k1, column c of block q) of an intermediate in item-major tiles
  __device__ __forceinline__ long ypos(int q, int k1, int c) const { return ((((long)q << l1) + k1) << lcb) + c; }

  // ---- pass A: gather d (functor) + column transforms -> Y1 ----
  template <class F>
  __device__ __forceinline__ void passA(int q, F& f) {
    const int cb = 1 << lcb, units = N1 << lcb;
    constexpr int U = 4;
    for (int base = 0; base < units; base += MF_THREADS * U) {
      typename F::In in[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) f.load(((long)(u >> lcb) << l2) + ((long)q << lcb) + (u & (cb - 1)), in[k]);
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) tile[u] = f.gather(((long)(u >> lcb) << l2) + ((long)q << lcb) + (u & (cb - 1)), in[k]);
      }
    }
    __syncthreads();
    column_store(q);
  }

  // column transforms of the tile [i1][c] and its store as tile q of Y1
  __device__ __forceinline__ void column_store(int q) {
    lds_wht(tile, l1, lcb, lcb, 0);
    const int units = N1 << lcb;
    double* dst = Y1 + ((long)q << (l1 + lcb));
    for (int u = threadIdx.x; u < units; u += MF_THREADS) dst[u] = tile[u];
    __syncthreads();
  }

  // ---- pass C: Y2 tile -> column transforms -> scatter t (functor) ----
  template <class F>
  __device__ __forceinline__ void passC(int q, F& f) {
    const int cb = 1 << lcb, units = N1 << lcb;
    constexpr int U = 2;
    typename F::In in[U];
    // the functor's first inputs are requested before the transform
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int u = threadIdx.x + k * MF_THREADS;
      if (u < units) f.load(((long)(u >> lcb) << l2) + ((long)q << lcb) + (u & (cb - 1)), in[k]);
    }
    const double* src = Y2 + ((long)q << (l1 + lcb));
    for (int u = threadIdx.x; u < units; u += MF_THREADS) tile[u] = src[u];
    __syncthreads();
    lds_wht(tile, l1, lcb, lcb, 0);
    for (int base = 0; base < units; base += MF_THREADS * U) {
      if (base > 0) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int u = base + threadIdx.x + k * MF_THREADS;
          if (u < units) f.load(((long)(u >> lcb) << l2) + ((long)q << lcb) + (u & (cb - 1)), in[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) {
          const long i = ((long)(u >> lcb) << l2) + ((long)q << lcb) + (u & (cb - 1));
          if constexpr (F::CHAIN) tile[u] = f.scatter(i, tile[u], in[k]);
          else f.scatter(i, tile[u], in[k]);
        }
      }
    }
    __syncthreads();
    if constexpr (F::CHAIN) column_store(q);
  }

  // ---- pass B: rows [r 2^lrb, (r+1) 2^lrb) -> row transforms -> spectral -> back -> Y2 ----
  // acc[0] += sum of squared outputs, acc[1] += sum b~ * output (residual).
  __device__ __forceinline__ void passB(int r, int mode_in, double (&acc)[2], double beta, int first) {
    const int mode = mode_in >= WB_RESID_STEP ? WB_RESID : mode_in;
    const int rb = 1 << lrb, cb = 1 << lcb, k10 = r << lrb;
    const int units = rb << l2;  // rb rows of N2
    const bool lin = mode_in >= WB_RESID_STEP;
    const bool comb = lin || (mode == WB_HAPPLY && !first);
    // loads first (four at a time), then the combination, its store and the tile
    constexpr int EB = 4;
    for (int e0 = 0; e0 < units; e0 += EB * MF_THREADS) {
      double va[EB], vb[EB];
      long gi[EB];
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int u = e0 + threadIdx.x + e * MF_THREADS;
        if (u < units) {
          // u = (q, row, c): contiguous rb x cb block per column block q
          const int q = u >> (lrb + lcb), rr = (u >> lcb) & (rb - 1), c = u & (cb - 1);
          gi[e] = ypos(q, k10 + rr, c);
          va[e] = lin ? Yx[gi[e]] : Y1[gi[e]];
          if (comb) vb[e] = lin ? Yd[gi[e]] : Y1p[gi[e]];
        }
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int u = e0 + threadIdx.x + e * MF_THREADS;
        if (u < units) {
          const int q = u >> (lrb + lcb), rr = (u >> lcb) & (rb - 1), c = u & (cb - 1);
          double v = va[e];
          if (comb) v += beta * vb[e];
          if (mode_in == WB_RESID_STEP || (!lin && mode == WB_RESID)) Yx[gi[e]] = v;
          else if (!lin && mode == WB_HAPPLY) Y1p[gi[e]] = v;
          tile[(rr << l2) + (q << lcb) + c] = v;
        }
      }
    }
    __syncthreads();
    lds_wht(tile, l2, lrb, 0, l2);
    // coefficients of W d, then the spectral step in place
    for (int u = threadIdx.x; u < units; u += MF_THREADS) {
      const long kk = ((long)(k10 + (u >> l2)) << l2) + (u & (N2 - 1));
      const double x = tile[u] * scale;
      if (mode == WB_FWDOUT) {
        XS[kk] = x;
        continue;
      }
      double y = mask[kk] ? x : 0.0;
      if (mode == WB_RESID) {
        const double bb = bt[kk];
        y -= bb;
        acc[1] += bb * y;
      }
      acc[0] += y * y;
      tile[u] = y;
    }
    __syncthreads();
    if (mode == WB_FWDOUT) return;
    lds_wht(tile, l2, lrb, 0, l2);
    for (int u = threadIdx.x; u < units; u += MF_THREADS) {
      const int q = u >> (lrb + lcb), rr = (u >> lcb) & (rb - 1), c = u & (cb - 1);
      Y2[ypos(q, k10 + rr, c)] = tile[(rr << l2) + (q << lcb) + c] * scale;
    }
    __syncthreads();
  }
};
