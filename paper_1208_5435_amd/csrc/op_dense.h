// Dense operator: explicit row-major m x n matrix A (leading dimension lda).
//
// Fused path (n <= DN_FUSED_MAXN): the Newton-operator product
// t = A^T (A d) and the residual A^T (A x - b) read A once:
//   pass A: d (from the functor) -> D                               (index tiles)
//   pass B: each item is a contiguous chunk of rows.  The workgroup holds
//           its columns of d in registers (thread t owns columns t + 512 j),
//           streams the chunk in blocks of DN_FB rows, reduces y_r = A_r . d
//           over the workgroup, and accumulates t_acc += A_blk^T y_blk in
//           registers; one partial t per chunk is written at the end.
//           Partial sums of y^2 (and b.y for the residual).
//   pass C: t = sum over chunks of the partials (fixed order) -> functor
//           epilogue                                                (index tiles)
// Two-pass path (larger n): pass B = row-block GEMV y = A d -> Yv, pass C =
// column-block GEMV^T t = A^T Yv with DN_RG row groups x 64 lanes.
// PCG form: pass C can chain the next gather (F::CHAIN: the functor returns
// the next vector's d value, stored to D), and pass B in HAPPLY mode combines
// d = D (+ beta Dp_prev) on load; chunk 0 stores the combination to Dp_cur
// for the next iteration (two alternating buffers).
#pragma once
#include "common.h"

#define DN_TA 1024   // indices per pass-A / fused pass-C item
#define DN_CB 64     // columns per two-pass pass-C item
#define DN_RBMAX 16  // max rows per two-pass pass-B item
#define DN_RG (MF_THREADS / 64)  // row groups of the two-pass pass C
#define DN_CPT 16                // columns per thread held in registers (fused)
#define DN_FUSED_MAXN (DN_CPT * MF_THREADS)
#define DN_FB 2                  // rows per fused block

// pass-B modes.  RESID reads D (x gathered by a pass A) and keeps it in Dxn
// (chunk 0); RESID_STEP forms Dxc + a Dd by linearity (Dd: the step
// direction's dz_u - dz_v) and keeps it in Dxn; RESID_TRIAL forms it without
// keeping it.  The caller swaps Dxc and Dxn after a kept residual.
enum { DB_HAPPLY = 0, DB_RESID = 1, DB_OUT = 2, DB_RESID_STEP = 3, DB_RESID_TRIAL = 4 };

// 16-byte non-temporal load of a pair of doubles
typedef double dn_pair_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream2(const double2* p) {
  const dn_pair_t v = __builtin_nontemporal_load(reinterpret_cast<const dn_pair_t*>(p));
  return make_double2(v.x, v.y);
}

struct OpDense {
  long n;
  long m;
  long lda;
  const double* __restrict__ A;
  const double* __restrict__ b;
  double* D;
  double* Yv;
  double* Dp_prev;  // PCG: d of the previous search direction (read)
  double* Dp_cur;   // PCG: d of the current search direction (written by item 0)
  double* Dxc;      // current x = u - v (read)
  double* Dxn;      // next x (written by item 0)
  double* Dd;       // step direction dz_u - dz_v
  double* PT;  // fused: partial t, nchunk x n
  int RB;
  int fused;
  int nchunk;      // fused: chunks (pass-B items)
  int chunk_rows;  // fused: rows per chunk (multiple of DN_FB)
  double* lds;     // reduction scratch: >= MF_WAVES * DN_RBMAX + DN_RG * DN_CB doubles
  double2* dsh;    // LDS: the workgroup's d, then its partial t, on the fused path (DN_FUSED_MAXN / 2 pairs each)

  __device__ int nA() const { return (int)((n + DN_TA - 1) / DN_TA); }
  __device__ int nB() const { return fused ? nchunk : (int)((m + RB - 1) / RB); }
  __device__ int nC() const { return (int)((n + DN_CB - 1) / DN_CB); }
  __device__ int nF() const { return (int)((m + 7) / 8); }

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

  // ---- fused pass B over one chunk of rows ----
  // Thread t owns the column pairs p = t + MF_THREADS k, k < CPT/2 (columns 2p, 2p+1,
  // loaded as one 16-byte double2).  Its values of d and its partial t live in
  // registers for CPT <= 8 and in LDS for wider rows (each thread reads back
  // only what it wrote, so no barrier), which keeps the registers for the
  // streamed rows.  acc valid in thread 0: acc[0] += sum y^2,
  // acc[1] += sum b*y (RESID).  Mode OUT writes y to `out` and skips the
  // transposed product.
  template <int CPT>
  __device__ __forceinline__ void passB_fused(int item, int mode_in, double (&acc)[2], double* out, double beta,
                                              int first) {
    const int mode = mode_in >= DB_RESID_STEP ? DB_RESID : mode_in;
    constexpr int KP = CPT / 2;
    const long r_begin = (long)item * chunk_rows;
    const long r_end = (r_begin + chunk_rows) < m ? (r_begin + chunk_rows) : m;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long npair = n >> 1;  // n is even on this path
    constexpr bool INLDS = CPT > 8;
    double2 dreg[INLDS ? 1 : KP], treg[INLDS ? 1 : KP];
    double2* tsh = dsh + DN_FUSED_MAXN / 2;
    auto dv_at = [&](int k) -> double2 { return INLDS ? dsh[tid + k * MF_THREADS] : dreg[INLDS ? 0 : k]; };
    auto t_at = [&](int k) -> double2& { return INLDS ? tsh[tid + k * MF_THREADS] : treg[INLDS ? 0 : k]; };
    const bool lin = mode_in >= DB_RESID_STEP;
    const double2* D2 = reinterpret_cast<const double2*>(lin ? Dxc : D);
    const double2* P2 = reinterpret_cast<const double2*>(lin ? Dd : Dp_prev);
    double2* C2 = reinterpret_cast<double2*>(mode == DB_HAPPLY ? Dp_cur : Dxn);
    const bool comb = mode == DB_HAPPLY ? !first : lin;
    const bool keep = mode == DB_HAPPLY || mode_in == DB_RESID || mode_in == DB_RESID_STEP;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const long p = tid + (long)k * MF_THREADS;
      double2 dv = p < npair ? D2[p] : make_double2(0.0, 0.0);
      if (p < npair) {
        if (comb) {
          const double2 w = P2[p];
          dv = make_double2(dv.x + beta * w.x, dv.y + beta * w.y);
        }
        if (keep && item == 0) C2[p] = dv;
      }
      if (INLDS) dsh[tid + k * MF_THREADS] = dv;
      else dreg[INLDS ? 0 : k] = dv;
      t_at(k) = make_double2(0.0, 0.0);
    }
    double* red = lds;  // [2 parities][MF_WAVES][DN_FB]
    int parity = 0;
    for (long r0 = r_begin; r0 < r_end; r0 += DN_FB) {
      double2 a[DN_FB][KP];
      double s[DN_FB];
#pragma unroll
      for (int r = 0; r < DN_FB; ++r) {
        const bool rv = (r0 + r) < r_end;
        const double2* row = reinterpret_cast<const double2*>(A + (r0 + r) * lda);
        double sr = 0.0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          const long p = tid + (long)k * MF_THREADS;
          // A is streamed once per operator application: a non-temporal
          // load keeps it from displacing the reused vectors in the caches
          a[r][k] = (rv && p < npair) ? ld_stream2(row + p) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          const double2 dv = dv_at(k);
          sr += a[r][k].x * dv.x + a[r][k].y * dv.y;
        }
        s[r] = sr;
      }
#pragma unroll
      for (int r = 0; r < DN_FB; ++r) {
        const double v = wave_reduce(0, s[r]);
        if (lane == 0) red[(parity * MF_WAVES + wave) * DN_FB + r] = v;
      }
      __syncthreads();
      double y[DN_FB];
#pragma unroll
      for (int r = 0; r < DN_FB; ++r) {
        double t = red[(parity * MF_WAVES) * DN_FB + r];
        for (int w = 1; w < MF_WAVES; ++w) t += red[(parity * MF_WAVES + w) * DN_FB + r];
        const bool rv = (r0 + r) < r_end;
        if (rv && mode == DB_RESID) {
          const double bb = b[r0 + r];
          t -= bb;
          if (tid == 0) acc[1] += bb * t;
        }
        if (!rv) t = 0.0;
        if (tid == 0) acc[0] += t * t;
        if (rv && mode == DB_OUT && tid == 0) out[r0 + r] = t;
        y[r] = t;
      }
      parity ^= 1;  // the other half of `red` is written next; no second barrier
      if (mode != DB_OUT) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          double2 t = t_at(k);
#pragma unroll
          for (int r = 0; r < DN_FB; ++r) {
            t.x += a[r][k].x * y[r];
            t.y += a[r][k].y * y[r];
          }
          t_at(k) = t;
        }
      }
    }
    if (mode != DB_OUT) {
      double2* pt = reinterpret_cast<double2*>(PT + (long)item * n);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const long p = tid + (long)k * MF_THREADS;
        if (p < npair) pt[p] = t_at(k);
      }
    }
    __syncthreads();
  }

  // ---- fused pass C: t = sum of chunk partials -> functor ----
  // Items of DN_CB columns; DN_RG groups of 64 lanes split the chunks
  // (group g sums chunks g, g + DN_RG, ...), then lane-column sums of the
  // groups in order feed the functor.
  template <class F>
  __device__ __forceinline__ void passC_fused(int item, F& f) {
    const long c0 = (long)item * DN_CB;
    const int col = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const long c = c0 + col;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < n) {
      int ch = rg;
      for (; ch + 3 * DN_RG < nchunk; ch += 4 * DN_RG) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a4[u] += PT[(long)(ch + DN_RG * u) * n + c];
      }
      for (; ch < nchunk; ch += DN_RG) a4[0] += PT[(long)ch * n + c];
    }
    double* red = lds + MF_WAVES * DN_RBMAX;
    red[rg * 64 + col] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    if (rg == 0 && c < n) {
      double t = red[col];
      for (int g = 1; g < DN_RG; ++g) t += red[g * 64 + col];
      typename F::In in;
      f.load(c, in);
      if constexpr (F::CHAIN) D[c] = f.scatter(c, t, in);
      else f.scatter(c, t, in);
    }
    __syncthreads();
  }

  // ---- two-pass path ----
  // y_r = A[r,:] . D for the rows of the block; mode RESID subtracts b,
  // mode OUT writes y to `out` instead of Yv.  acc[0] += sum y^2,
  // acc[1] += sum b*y (RESID).  Results valid in thread 0.
  __device__ __forceinline__ void passB_rows(int item, int mode_in, double (&acc)[2], double* out, double beta,
                                             int first) {
    const int mode = mode_in >= DB_RESID_STEP ? DB_RESID : mode_in;
    const bool lin = mode_in >= DB_RESID_STEP;
    const double* Din = lin ? Dxc : D;
    const double* Pin = lin ? Dd : Dp_prev;
    double* Cout = mode == DB_HAPPLY ? Dp_cur : Dxn;
    const bool comb = mode == DB_HAPPLY ? !first : lin;
    const bool keep = mode == DB_HAPPLY || mode_in == DB_RESID || mode_in == DB_RESID_STEP;
    const long r0 = (long)item * RB;
    const int nr = (int)((m - r0) < RB ? (m - r0) : RB);
    double s[DN_RBMAX];
#pragma unroll
    for (int r = 0; r < DN_RBMAX; ++r) s[r] = 0.0;
    for (long c = threadIdx.x; c < n; c += MF_THREADS) {
      double dv = Din[c];
      if (comb) dv += beta * Pin[c];
      if (keep && item == 0) Cout[c] = dv;
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
  __device__ __forceinline__ void passC_cols(int item, F& f) {
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
      if constexpr (F::CHAIN) D[c] = f.scatter(c, t, in);
      else f.scatter(c, t, in);
    }
    __syncthreads();
  }

  __device__ __forceinline__ void passB(int item, int mode, double (&acc)[2], double* out, double beta,
                                        int first) {
    if (fused) {
      if (n <= (DN_CPT / 2) * MF_THREADS) passB_fused<DN_CPT / 2>(item, mode, acc, out, beta, first);
      else passB_fused<DN_CPT>(item, mode, acc, out, beta, first);
    } else {
      passB_rows(item, mode, acc, out, beta, first);
    }
  }
  template <class F>
  __device__ __forceinline__ void passC(int item, F& f) {
    if (fused) passC_fused(item, f);
    else passC_cols(item, f);
  }

  // sum of squares of 8 rows (set-up: ||A||_F^2), returned in thread 0
  __device__ __forceinline__ double frob_block(int item) {
    const long r0 = (long)item * 8;
    const int nr = (int)((m - r0) < 8 ? (m - r0) : 8);
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
