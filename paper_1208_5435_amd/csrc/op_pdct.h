// Partial DCT operator A = R_m C (C = orthonormal DCT-II of length n, R_m keeps
// m sampled rows): the product K d = A^T A d = C^T M C d (M = 0/1 mask of the
// kept coefficients) and the residual A^T (A x - b) = C^T (M C x - b~), where
// b~ is b scattered to the kept coefficients.  Orthonormal rows (A A^T = I)
// are the property the paper's preconditioner relies on (Section 2,
// eq. (eq:orthonormality); Section 4, eq. (eq:ne2_P) with rho = m/n).
//
// Transform path (radix-2 FFT staged in LDS; Makhoul's DCT-via-FFT reordering
// and the half-length complex FFT of a real sequence):
//   gather    w_j = d_{4j} + i d_{4j+2},  w_{H-1-j} = d_{4j+3} + i d_{4j+1}
//             (j < n/4, H = n/2), i.e. the even-then-reversed-odd reordering
//             packed two reals per complex;
//   FFT_H     four-step: column FFTs of length N1, twiddle exp(-2 pi i j2 k1/H),
//             row FFTs of length N2 (H = N1 N2);
//   spectral  per pair (k, H-k): split the real-FFT halves, rotate by
//             exp(-i pi k/(2n)), scale -> DCT coefficients X_k, X_{n-k};
//             apply mask / subtract b~; rebuild the Hermitian half-spectrum of
//             the DCT-III input; pack for the inverse half-length FFT;
//   IFFT_H    row inverse FFTs, conjugate twiddle, column inverse FFTs;
//   scatter   the inverse of the gather gives t = C^T (...).
// Passes: A = gather + column FFT (items: pairs of mirrored 4-column blocks),
// B = row FFT + spectral + row IFFT (items: pairs of rows k1, N1-k1),
// C = column IFFT + scatter (items as A).  Complex intermediates live in HBM
// in item-major tiles so that both sides of each exchange are contiguous.
// Pass C can chain the next gather: A and C items cover the same indices, so
// a functor that returns the next vector's d value for each index gets its
// column FFT done in the same pass (written to Y1); pass B can then combine
// Y1 with a stored Y1p by linearity (Y1p <- Y1 + beta Y1p) before the row
// FFTs, so a PCG iteration needs only passes B and C.
#pragma once
#include "common.h"

#define PD_TILE_CPLX 4096  // LDS tile: 4096 complex doubles = 64 KiB
#define PD_EPT (PD_TILE_CPLX / MF_THREADS)  // tile elements per thread
// Tile element a lives at LDS slot a + a / 16: one unused slot after every 16
// elements.  The early Stockham passes write with a stride of R elements
// (R x 16 bytes); unpadded, those lanes fall on the same few LDS banks.
#define PD_PAD_SH 4
#define PD_TILE_LDS (PD_TILE_CPLX + (PD_TILE_CPLX >> PD_PAD_SH))  // LDS slots of the padded tile
__device__ __forceinline__ int tpad(int a) { return a + (a >> PD_PAD_SH); }
// the same for an offset into the tile viewed as doubles (re, im pairs)
__device__ __forceinline__ int tpad_d(int slot) { return (tpad(slot >> 1) << 1) | (slot & 1); }
#ifndef PD_U
#define PD_U 1  // gather/scatter units per thread and batch (2 or more raise the kernel's register spills; measured slower)
#endif
#define PD_MASK_BYTES 8192  // LDS staging of one pass-B item's mask (4 N2 <= 8192)

// ------------------------------- radix kernels --------------------------------
template <int R>
__device__ __forceinline__ void dft_small(cplx (&v)[R], int sign);

template <>
__device__ __forceinline__ void dft_small<2>(cplx (&v)[2], int) {
  cplx a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <>
__device__ __forceinline__ void dft_small<4>(cplx (&v)[4], int sign) {
  cplx a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  cplx a2 = cadd(v[1], v[3]), a3 = cmul_si(csub(v[1], v[3]), sign);
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <>
__device__ __forceinline__ void dft_small<8>(cplx (&v)[8], int sign) {
  cplx e[4] = {v[0], v[2], v[4], v[6]};
  cplx o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4>(e, sign);
  dft_small<4>(o, sign);
  const double h = 0.70710678118654752440;  // sqrt(2)/2
  // o1 *= w8, o2 *= w8^2 = sign*i, o3 *= w8^3, with w8 = exp(sign*i*pi/4)
  o[1] = cmul(o[1], mkc(h, sign * h));
  o[2] = cmul_si(o[2], sign);
  o[3] = cmul(o[3], mkc(-h, sign * h));
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    v[s] = cadd(e[s], o[s]);
    v[s + 4] = csub(e[s], o[s]);
  }
}

// Twiddles and butterfly of one Stockham (self-sorting) radix-R step:
// butterfly b of a sequence at stage Ls takes elements b + r L/R and writes
// (b / Ls) Ls R + (b mod Ls) + r Ls, its inputs rotated by powers of
// w = exp(sign 2 pi i (b mod Ls) / (Ls R)).  All sizes are powers of two and
// passed as log2.  twsh = log2M - log2(Ls R), log2M being the log2 of the
// twiddle resolution of the instance (4 n).
template <int R>
__device__ __forceinline__ void stockham_bfly(cplx (&v)[R], int j, int twsh, int sign, const Twiddle& tw) {
  if (j != 0) {
    const cplx w1 = tw.get(j << twsh, sign);
    cplx w = w1;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul(v[r], w);
      if (r + 1 < R) w = cmul(w, w1);
    }
  }
  dft_small<R>(v, sign);
}

// One radix-R pass over 2^lcount sequences of length 2^lL in LDS, in place,
// spread over the whole workgroup: every thread loads its butterfly inputs,
// the workgroup synchronises, then the outputs are written.  Element (s, i)
// is at buf[tpad((s << lss) + (i << lis))].
template <int R, int LR>
__device__ __forceinline__ void stockham_pass(cplx* buf, int lL, int lLs, int lcount, int lis, int lss, int sign,
                                              const Twiddle& tw, int log2M) {
  constexpr int NB = PD_EPT / R;
  const int lnb = lL - LR;  // log2 butterflies per sequence
  const int nb = 1 << (lnb + lcount);
  const int twsh = log2M - (lLs + LR);
  cplx v[NB][R];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int bt = threadIdx.x + k * MF_THREADS;
    if (bt < nb) {
      int s, b;
      if (lis == 0) {
        s = bt >> lnb;
        b = bt & ((1 << lnb) - 1);
      } else {
        s = bt & ((1 << lcount) - 1);
        b = bt >> lcount;
      }
      const int base = (s << lss) + (b << lis);
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = buf[tpad(base + ((r << lnb) << lis))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int bt = threadIdx.x + k * MF_THREADS;
    if (bt < nb) {
      int s, b;
      if (lis == 0) {
        s = bt >> lnb;
        b = bt & ((1 << lnb) - 1);
      } else {
        s = bt & ((1 << lcount) - 1);
        b = bt >> lcount;
      }
      const int j = b & ((1 << lLs) - 1);
      stockham_bfly<R>(v[k], j, twsh, sign, tw);
      const int ob = (s << lss) + ((((b >> lLs) << (lLs + LR)) + j) << lis);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[tpad(ob + ((r << lLs) << lis))] = v[k][r];
    }
  }
  __syncthreads();
}

// Unnormalised DFT (sign -1) or inverse DFT (sign +1) of 2^lcount sequences
// of length 2^lL held in LDS (element (s, i) at buf[tpad((s << lss) + (i << lis))],
// 2^(lcount + lL) <= 4096).  Caller synchronises before; the result is visible
// to the whole workgroup on return.  Radix 8 while at least three factors of
// two remain, then 4 or 2: the fewest passes (each pass costs two workgroup
// barriers and an LDS round trip, which outweighs idle lanes on small tiles).
// Index arithmetic is shifts and masks only (no integer division).
__device__ __forceinline__ void lds_fft(cplx* buf, int lL, int lcount, int lis, int lss, int sign,
                                        const Twiddle& tw, int log2M) {
  int lg = 0;
  while (lg < lL) {
    const int rem = lL - lg;
    if (rem >= 3) {
      stockham_pass<8, 3>(buf, lL, lg, lcount, lis, lss, sign, tw, log2M);
      lg += 3;
    } else if (rem == 2) {
      stockham_pass<4, 2>(buf, lL, lg, lcount, lis, lss, sign, tw, log2M);
      lg += 2;
    } else {
      stockham_pass<2, 1>(buf, lL, lg, lcount, lis, lss, sign, tw, log2M);
      lg += 1;
    }
  }
}

// pass-B modes.  RESID reads Y1 (x gathered by a pass A) and keeps it as the
// transform of the current x in Yx; RESID_STEP forms Yx + a Yd by linearity
// (Yd: the transform of the step direction) and keeps it; RESID_TRIAL forms
// it without keeping it.
enum { PB_HAPPLY = 0, PB_RESID = 1, PB_FWDOUT = 2, PB_RESID_STEP = 3, PB_RESID_TRIAL = 4 };

struct OpPdct {
  long n;
  long m;
  int H, N1, N2, l1, l2, logn;
  int lcb;  // log2 of the columns of a pass-A/C item: 3 (two mirrored blocks of 4) or 2 (of 2)
  const int* __restrict__ rows;
  const double* __restrict__ b;
  cplx* Y1;
  cplx* Y1p;  // column-FFT data of the current search direction (PCG)
  cplx* Y2;
  cplx* Yx;   // column-FFT data of the current x = u - v
  cplx* Yd;   // column-FFT data of the step direction dz_u - dz_v
  unsigned char* mask;  // spectral layout, n bytes
  double* bt;           // spectral layout, n doubles
  double* XS;           // spectral layout, n doubles (forward output)
  Twiddle tw;
  cplx* tile;          // LDS
  unsigned char* msk;  // LDS: mask of the current pass-B item, rows (k1a, k1b)
  int cur_k1a;
  int wt;  // exchange buffers are written through the L2 (teams of several workgroups)
  double a0, a1;
  // Partial DST-II through the same transform: S d = P C D d with D =
  // diag((-1)^j) and P the index reversal k -> n - 1 - k (the sine rows are
  // the reversed cosine rows of the sign-alternated input; the orthonormal
  // scalings match under the reversal).  flip = 1 applies D on the way in and
  // out and reverses the coefficient indices.
  int flip;
  __device__ __forceinline__ double sgn(long i, double v) const { return (flip && (i & 1)) ? -v : v; }

  // mask value of coefficient owner (k, e), from the LDS copy of the item
  __device__ __forceinline__ double mval(int k, int e) const {
    const int k1 = k & (N1 - 1);
    return (double)msk[(k1 == cur_k1a ? 0 : 2 * N2) + ((k >> l1) << 1) + e];
  }

  __device__ int nA() const { return N2 >> lcb; }
  __device__ int nB() const { return N1 >> 1; }
  __device__ int nC() const { return N2 >> lcb; }
  // tile column c of item q -> column j2 of the N1 x N2 grid
  __device__ __forceinline__ int col_j2(int q, int c) const {
    const int hb = 1 << (lcb - 1);
    return c < hb ? (q << (lcb - 1)) + c : N2 - 1 - (q << (lcb - 1)) - (c - hb);
  }
  __device__ int log2M() const { return logn + 2; }

  // position of coefficient-owner (half index k, e) in the spectral layout
  __device__ __forceinline__ int spos(int k, int e) const {
    return ((((k & (N1 - 1)) << l2) + (k >> l1)) << 1) + e;
  }
  // spectral-layout position of DCT coefficient index kk in [0, n) (of the
  // DST coefficient kk, which is DCT coefficient n - 1 - kk, when flip)
  __device__ __forceinline__ long coef_pos(long kk) const {
    if (flip) kk = n - 1 - kk;
    if (kk == 0) return spos(0, 0);
    if (kk == H) return spos(0, 1);
    if (kk < H) return spos((int)kk, 0);
    return spos((int)(n - kk), 1);
  }

  // An item q holds 2^lcb grid columns: the block of hb = 2^(lcb-1) columns
  // starting at hb q and its mirror image ending at N2 - 1 - hb q, so that
  // w_j and w_{H-1-j} of the gather (mirrored row and column) meet in one
  // item.  Unit u in [0, N1 2^(lcb+1)) -> d index and the tile slot (double
  // offset into the LDS tile viewed as doubles, [row][column][re, im]).
  __device__ __forceinline__ int units() const { return N1 << (lcb + 1); }
  __device__ __forceinline__ void unit_map(int q, int u, long& i, int& slot) const {
    const int hb = 1 << (lcb - 1);
    const int j1 = u >> (lcb + 2), w = u & ((4 << lcb) - 1), seg = w >> (lcb + 1), off = w & ((2 << lcb) - 1);
    const int cc = off >> 2, e = off & 3;
    const int j2 = seg == 0 ? (q << (lcb - 1)) + cc : N2 - hb - (q << (lcb - 1)) + cc;
    const int colA = seg == 0 ? cc : hb + (hb - 1 - cc);
    const int colM = seg == 0 ? hb + cc : hb - 1 - cc;
    i = (long)((((j1 << l2) + j2) << 2) + e);
    if (e == 0) slot = (((j1 << lcb) + colA) << 1);
    else if (e == 2) slot = (((j1 << lcb) + colA) << 1) + 1;
    else if (e == 3) slot = ((((N1 - 1 - j1) << lcb) + colM) << 1);
    else slot = ((((N1 - 1 - j1) << lcb) + colM) << 1) + 1;
  }

  // ---- pass A: gather d (from the functor) + column FFTs + twiddle -> Y1 ----
  template <class F>
  __device__ __forceinline__ void passA(int q, F& f) {
    double* td = reinterpret_cast<double*>(tile);
    const int units = this->units();
    constexpr int U = PD_U;
    for (int base = 0; base < units; base += MF_THREADS * U) {
      typename F::In in[U];
      long idx[U];
      int slot[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) {
          unit_map(q, u, idx[k], slot[k]);
          f.load(idx[k], in[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) td[tpad_d(slot[k])] = sgn(idx[k], f.gather(idx[k], in[k]));
      }
    }
    __syncthreads();
    column_fft_store(q);
  }

  // forward column FFTs of the gathered tile, four-step twiddle, store to Y1
  __device__ __forceinline__ void column_fft_store(int q) {
    lds_fft(tile, l1, lcb, lcb, 0, -1, tw, log2M());
    for (int e = threadIdx.x; e < (N1 << lcb); e += MF_THREADS) {
      const int k1 = e >> lcb, c = e & ((1 << lcb) - 1);
      const int j2 = col_j2(q, c);
      cplx v = tile[tpad(e)];
      v = cmul(v, tw.get((j2 * k1) << 3, -1));
      st_sel(Y1, (q << (l1 + lcb)) + e, v, wt);
    }
    __syncthreads();
  }

  // ---- pass C: Y2 -> column IFFTs -> scatter t to the functor ----
  // (F::CHAIN: the functor returns the next d value of each index, which
  // replaces t in the same tile slot; the tile is then column-FFT'd to Y1.)
  template <class F>
  __device__ __forceinline__ void passC(int q, F& f) {
    const int units = this->units();
    constexpr int U = PD_U;
    // The functor's inputs of the first batch of units are requested before
    // the column IFFTs so that their memory latency overlaps the transform.
    typename F::In in[U];
    long idx[U];
    int slot[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int u = threadIdx.x + k * MF_THREADS;
      if (u < units) {
        unit_map(q, u, idx[k], slot[k]);
        f.load(idx[k], in[k]);
      }
    }
    for (int e = threadIdx.x; e < (N1 << lcb); e += MF_THREADS) tile[tpad(e)] = Y2[(q << (l1 + lcb)) + e];
    __syncthreads();
    lds_fft(tile, l1, lcb, lcb, 0, +1, tw, log2M());
    double* td = reinterpret_cast<double*>(tile);
    for (int base = 0; base < units; base += MF_THREADS * U) {
      if (base > 0) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int u = base + threadIdx.x + k * MF_THREADS;
          if (u < units) {
            unit_map(q, u, idx[k], slot[k]);
            f.load(idx[k], in[k]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int u = base + threadIdx.x + k * MF_THREADS;
        if (u < units) {
          const double t = sgn(idx[k], td[tpad_d(slot[k])]);
          if constexpr (F::CHAIN) td[tpad_d(slot[k])] = sgn(idx[k], f.scatter(idx[k], t, in[k]));
          else f.scatter(idx[k], t, in[k]);
        }
      }
    }
    __syncthreads();
    if constexpr (F::CHAIN) column_fft_store(q);
  }

  // Spectral work for one pair of half-spectrum indices (kA, kB = H - kA).
  // acc[0] += sum of squared outputs, acc[1] += sum b~ * output.
  __device__ __forceinline__ void spectral_pair(int mode, int kA, int pA, int kB, int pB, double (&acc)[2]) {
    const cplx WA = tile[tpad(pA)];
    const double h = 0.70710678118654752440;
    if (kA == 0) {
      // V_0 = Re W0 + Im W0, V_H = Re W0 - Im W0 (both real)
      const double V0 = WA.x + WA.y, VH = WA.x - WA.y;
      double X0 = a0 * V0, XH = a1 * VH * h;
      const int p0 = spos(0, 0), p1 = spos(0, 1);
      if (mode == PB_FWDOUT) {
        XS[p0] = X0;
        XS[p1] = XH;
        return;
      }
      const double m0 = mval(0, 0), m1 = mval(0, 1);
      double Y0 = m0 * X0, YH = m1 * XH;
      if (mode == PB_RESID) {
        const double b0 = bt[p0], b1 = bt[p1];
        Y0 -= b0;
        YH -= b1;
        acc[1] += b0 * Y0 + b1 * YH;
      }
      acc[0] += Y0 * Y0 + YH * YH;
      const double c0 = a0 * Y0, cH = a1 * YH;
      const double H0 = c0, HH = cH * h;
      tile[tpad(pA)] = mkc(H0 + HH, H0 - HH);  // (H0 + HH) + i (H0 - HH)
      return;
    }
    const cplx WB = tile[tpad(pB)];
    // real-FFT split: E = (WA + conj WB)/2, O = (WA - conj WB) / (2i)
    const cplx E = cscale(cadd(WA, cconj(WB)), 0.5);
    const cplx Dd = csub(WA, cconj(WB));
    const cplx O = mkc(0.5 * Dd.y, -0.5 * Dd.x);
    const cplx VA = cadd(E, cmul(tw.get(4 * kA), O));
    const cplx UA = cmul(tw.get(kA), VA);
    const cplx VB = cadd(cconj(E), cmul(tw.get(4 * kB), cconj(O)));
    const cplx UB = cmul(tw.get(kB), VB);
    // coefficients owned: e=0 -> X_k = a1 Re U, e=1 -> X_{n-k} = -a1 Im U
    const int qa0 = spos(kA, 0), qa1 = qa0 + 1, qb0 = spos(kB, 0), qb1 = qb0 + 1;
    double xa0 = a1 * UA.x, xa1 = -a1 * UA.y, xb0 = a1 * UB.x, xb1 = -a1 * UB.y;
    const bool self = (kA == kB);
    if (mode == PB_FWDOUT) {
      XS[qa0] = xa0;
      XS[qa1] = xa1;
      if (!self) {
        XS[qb0] = xb0;
        XS[qb1] = xb1;
      }
      return;
    }
    double ya0 = mval(kA, 0) * xa0, ya1 = mval(kA, 1) * xa1;
    double yb0 = 0, yb1 = 0;
    if (!self) {
      yb0 = mval(kB, 0) * xb0;
      yb1 = mval(kB, 1) * xb1;
    }
    if (mode == PB_RESID) {
      const double ba0 = bt[qa0], ba1 = bt[qa1];
      ya0 -= ba0;
      ya1 -= ba1;
      acc[1] += ba0 * ya0 + ba1 * ya1;
      if (!self) {
        const double bb0 = bt[qb0], bb1 = bt[qb1];
        yb0 -= bb0;
        yb1 -= bb1;
        acc[1] += bb0 * yb0 + bb1 * yb1;
      }
    }
    acc[0] += ya0 * ya0 + ya1 * ya1;
    if (!self) acc[0] += yb0 * yb0 + yb1 * yb1;
    else {
      yb0 = ya0;
      yb1 = ya1;
    }
    // inverse: c = a1 Y; Hk = 1/2 exp(+i pi k/(2n)) (c_k - i c_{n-k})
    const cplx HA = cscale(cmul(cconj(tw.get(kA)), mkc(a1 * ya0, -a1 * ya1)), 0.5);
    const cplx HB = cscale(cmul(cconj(tw.get(kB)), mkc(a1 * yb0, -a1 * yb1)), 0.5);
    // G_k = (H_k + conj H_{H-k}) + i exp(2 pi i k/n) (H_k - conj H_{H-k})
    const cplx GA = cadd(cadd(HA, cconj(HB)), cmul_si(cmul(cconj(tw.get(4 * kA)), csub(HA, cconj(HB))), 1));
    tile[tpad(pA)] = GA;
    if (!self) {
      const cplx GB =
          cadd(cadd(HB, cconj(HA)), cmul_si(cmul(cconj(tw.get(4 * kB)), csub(HB, cconj(HA))), 1));
      tile[tpad(pB)] = GB;
    }
  }

  // ---- pass B: two rows of Y1 -> row FFT -> spectral -> row IFFT -> Y2 ----
  // Mode HAPPLY combines the rows first: Y1p <- Y1 (+ beta Y1p unless first).
  // The residual modes take the rows as described at the mode list (beta = a).
  __device__ __forceinline__ void passB(int r, int mode_in, double (&acc)[2], double beta, int first) {
    const int mode = mode_in >= PB_RESID_STEP ? PB_RESID : mode_in;  // spectral treatment
    const int k1a = r == 0 ? 0 : r;
    const int k1b = r == 0 ? (N1 >> 1) : N1 - r;
    cur_k1a = k1a;
    if (mode != PB_FWDOUT) {
      // the item's mask bytes (two rows of 2 N2) to LDS, as 32-bit words
      const unsigned* ga = reinterpret_cast<const unsigned*>(mask + (k1a << (l2 + 1)));
      const unsigned* gb = reinterpret_cast<const unsigned*>(mask + (k1b << (l2 + 1)));
      unsigned* ml = reinterpret_cast<unsigned*>(msk);
      const int wpr = N2 >> 1;  // 32-bit words per row
      for (int i = threadIdx.x; i < 2 * wpr; i += MF_THREADS) ml[i] = i < wpr ? ga[i] : gb[i - wpr];
    }
    // The thread's loads (up to four elements at a time) are issued before
    // its stores (the rows and the stored combination are different
    // buffers), so that their latencies overlap.
    {
      constexpr int EB = 4;
      const bool lin = mode_in >= PB_RESID_STEP;
      const bool comb = lin || (mode == PB_HAPPLY && !first);
      for (int e0 = 0; e0 < 2 * N2; e0 += EB * MF_THREADS) {
        cplx va[EB], vb[EB];
#pragma unroll
        for (int e = 0; e < EB; ++e) {
          const int u2 = e0 + threadIdx.x + e * MF_THREADS;
          if (u2 < 2 * N2) {
            const int s = u2 >= N2;
            const int u = u2 - s * N2;
            const int gi = ((((u >> lcb) << l1) + (s ? k1b : k1a)) << lcb) + (u & ((1 << lcb) - 1));
            va[e] = lin ? Yx[gi] : Y1[gi];
            if (comb) vb[e] = lin ? Yd[gi] : Y1p[gi];
          }
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
          const int u2 = e0 + threadIdx.x + e * MF_THREADS;
          if (u2 < 2 * N2) {
            const int s = u2 >= N2;
            const int u = u2 - s * N2;
            const int q = u >> lcb, c = u & ((1 << lcb) - 1);
            const int gi = (((q << l1) + (s ? k1b : k1a)) << lcb) + c;
            cplx v = va[e];
            if (comb) v = mkc(v.x + beta * vb[e].x, v.y + beta * vb[e].y);
            if (mode_in == PB_RESID_STEP || (!lin && mode == PB_RESID)) st_sel(Yx, gi, v, wt);
            else if (!lin && mode == PB_HAPPLY) st_sel(Y1p, gi, v, wt);
            tile[tpad(s * N2 + col_j2(q, c))] = v;
          }
        }
      }
    }
    __syncthreads();
    lds_fft(tile, l2, 1, 0, l2, -1, tw, log2M());
    if (r != 0) {
      for (int u = threadIdx.x; u < N2; u += MF_THREADS) {
        const int kA = k1a + (u << l1);
        const int kB = k1b + ((N2 - 1 - u) << l1);
        spectral_pair(mode, kA, u, kB, N2 + (N2 - 1 - u), acc);
      }
    } else {
      for (int u = threadIdx.x; u < N2 + 1; u += MF_THREADS) {
        if (u <= (N2 >> 1)) {
          const int pb = (N2 - u) & (N2 - 1);
          spectral_pair(mode, u << l1, u, pb << l1, pb, acc);
        } else {
          const int v = u - (N2 >> 1) - 1;
          const int kA = (N1 >> 1) + (v << l1);
          const int kB = (N1 >> 1) + ((N2 - 1 - v) << l1);
          spectral_pair(mode, kA, N2 + v, kB, N2 + (N2 - 1 - v), acc);
        }
      }
    }
    __syncthreads();
    if (mode == PB_FWDOUT) return;
    lds_fft(tile, l2, 1, 0, l2, +1, tw, log2M());
    for (int u2 = threadIdx.x; u2 < 2 * N2; u2 += MF_THREADS) {
      const int s = u2 >= N2;
      const int u = u2 - s * N2;
      const int q = u >> lcb, c = u & ((1 << lcb) - 1);
      const int j2 = col_j2(q, c);
      const int k1 = s ? k1b : k1a;
      cplx v = tile[tpad(s * N2 + j2)];
      v = cmul(v, tw.get((j2 * k1) << 3, +1));
      st_sel(Y2, (((q << l1) + k1) << lcb) + c, v, wt);
    }
    __syncthreads();
  }
};
