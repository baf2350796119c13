// Device-side driver of the single-corrector primal-dual matrix-free IPM
// (Section 5.1 algorithm) and of its PCG inner solver (Section 4), written
// once over an operator policy (OpDense; OpPdct, which also serves the DST
// rows; OpWht; OpDenseDirect, whose Newton solves are the Cholesky ones of
// direct.h instead of the PCG).  Per-index data are
// interleaved (u_i, v_i) pairs (double2) so that the 2x2 block structure of
// H and P (Section 4, eqs. (eq:ne2_H), (eq:ne2_P)) is local to one index.
//
// Every pass distributes its items over the workgroups of a team; every
// reduction is first done per item (fixed order inside the workgroup), then
// over items in a fixed order by each workgroup after the team barrier, so
// all workgroups of a team hold bit-identical scalars and take identical
// branch decisions.
#pragma once
#include <type_traits>

#include "common.h"
#include "op_dense.h"
#include "op_pdct.h"
#include "op_wht.h"
#include "direct.h"

// mirror of mfipm_params (host struct) -- same field order and types
struct DevParams {
  double tol;
  int32_t maxiters;
  double tolpcg;
  int32_t mxiterpcg;
  double sigma1, sigma2, sigma3;
  double alpha_bar, alpha_tilde;
  double eta;
  double rho;
  double z0, s0;
  double tolpcg_adj;
  int32_t mxiterpcg_adj;
  double step_min;
  int32_t reduced;
  int32_t direct;
};

struct DevInfo {
  int32_t status, ipm_iters, pcg_iters, correctors;
  int64_t nmat;
  double rel_gap, mu, primal_obj, dual_obj, rho;
};

struct InstDesc {
  long n, m;
  long n_off, m_off, a_off;
  double tau;
};

// per-team workspace (device pointers)
struct TeamWS {
  double2 *X, *R, *P, *TI, *DZ, *DS, *Zs, *Ss;
  double *D, *Yv, *PT, *Dp0, *Dp1, *Dx0, *Dx1, *Dd;
  cplx *Y1, *Y1p, *Y2, *Yx, *Yd;
  unsigned char* mask;
  double *bt, *XS;
  double *partA, *partB, *partC, *partS;
  double *DK, *DM, *DLi, *DY;  // direct variant: A^T A, M / L, diagonal inverses, sweep vector
  unsigned long long* bar;
  int* slot;
  int* err;
};

struct TeamLayout {  // byte offsets inside one team region
  long X, R, P, TI, DZ, DS, Zs, Ss, D, Yv, PT, Dp0, Dp1, Dx0, Dx1, Dd, Y1, Y1p, Y2, Yx, Yd, mask, bt, XS, partA, partB,
      partC, partS, DK, DM, DLi, DY;
  int pt_chunks;  // dense fused path: capacity of PT in chunks
  long stride;
};

struct KArgs {
  const InstDesc* inst;
  const int* order;
  int batch;
  int* queue_head;
  int* abort_flag;
  DevInfo* info;
  const double* A;
  const int* rows;
  int shared_op;
  int op_flip;  // partial DST through the DCT kernel
  const double* b;
  double* x;
  double* state;
  const double* grad_x;
  double* grad_b;
  double* grad_tau;
  DevParams prm;
  char* team_base;
  char* team_ctl;  // MF_CTL_BYTES per team, contiguous
  TeamLayout lay;
  const cplx* tw_lo;
  const cplx* tw_hi;
  int tw_lo_bits;
  int tw_log2n_max;
  int team_size;
  int num_teams;
  int tile_param;
  unsigned long long spin_ticks;
};

__device__ __forceinline__ TeamWS make_ws(const KArgs& a, int team) {
  char* base = a.team_base + (long)team * a.lay.stride;
  TeamWS w;
  w.X = (double2*)(base + a.lay.X);
  w.R = (double2*)(base + a.lay.R);
  w.P = (double2*)(base + a.lay.P);
  w.TI = (double2*)(base + a.lay.TI);
  w.DZ = (double2*)(base + a.lay.DZ);
  w.DS = (double2*)(base + a.lay.DS);
  w.Zs = (double2*)(base + a.lay.Zs);
  w.Ss = (double2*)(base + a.lay.Ss);
  w.D = (double*)(base + a.lay.D);
  w.Yv = (double*)(base + a.lay.Yv);
  w.PT = (double*)(base + a.lay.PT);
  w.Dp0 = (double*)(base + a.lay.Dp0);
  w.Dp1 = (double*)(base + a.lay.Dp1);
  w.Dx0 = (double*)(base + a.lay.Dx0);
  w.Dx1 = (double*)(base + a.lay.Dx1);
  w.Dd = (double*)(base + a.lay.Dd);
  w.Yx = (cplx*)(base + a.lay.Yx);
  w.Yd = (cplx*)(base + a.lay.Yd);
  w.Y1p = (cplx*)(base + a.lay.Y1p);
  w.Y1 = (cplx*)(base + a.lay.Y1);
  w.Y2 = (cplx*)(base + a.lay.Y2);
  w.mask = (unsigned char*)(base + a.lay.mask);
  w.bt = (double*)(base + a.lay.bt);
  w.XS = (double*)(base + a.lay.XS);
  w.partA = (double*)(base + a.lay.partA);
  w.partB = (double*)(base + a.lay.partB);
  w.partC = (double*)(base + a.lay.partC);
  w.partS = (double*)(base + a.lay.partS);
  w.DK = (double*)(base + a.lay.DK);
  w.DM = (double*)(base + a.lay.DM);
  w.DLi = (double*)(base + a.lay.DLi);
  w.DY = (double*)(base + a.lay.DY);
  char* ctl = a.team_ctl + (long)team * MF_CTL_BYTES;
  w.bar = (unsigned long long*)ctl;
  w.slot = (int*)(ctl + MF_CTL_SLOT_BYTES);
  w.err = (int*)(ctl + MF_CTL_ERR_BYTES);
  return w;
}

// ------------------------------------------------------------------------
// Per-index functors.  load() issues the global reads of one index into
// registers; gather()/scatter()/elem() compute, store, accumulate partials.
// ------------------------------------------------------------------------

// PCG pass C (two passes per PCG iteration).  With t = (A^T A d)_i of the
// current direction:
//   y = P^{-1} r (r before the update), p = y + beta p_prev (p = y at the
//   first iteration), q = Theta^{-1} p + [t; -t], x += alpha p, r -= alpha q,
//   store x, r, p; then y' = P^{-1} r (new r) and return d' = y'_u - y'_v,
//   whose column transform the operator prepares for the next iteration.
// Partials: 0 r'^T y', 1 r'^T r', 2 y'^T Theta^{-1} y', 3 y'^T Theta^{-1} p,
// 4 p^T Theta^{-1} p -- the next p^T Theta^{-1} p is
// [2] + 2 beta' [3] + beta'^2 [4] once beta' is known.
struct FPcgC2 {
  static constexpr int K = 5;
  static constexpr bool CHAIN = true;
  struct In {
    double2 p, ti, x, r;
  };
  double2* P;
  double2* TI;
  double2* X;
  double2* R;
  double alpha, beta, rho;
  int first;
  int wt;  // stores write through the L2 (teams of several workgroups)
  double acc[K];
  __device__ void reset() {
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.0;
  }
  __device__ void load(long i, In& in) const {
    if (!first) in.p = P[i];
    in.ti = TI[i];
    in.x = X[i];
    in.r = R[i];
  }
  __device__ double scatter(long i, double t, const In& in) {
    double yu, yv;
    precond_apply(in.ti.x, in.ti.y, rho, in.r.x, in.r.y, yu, yv);
    double2 p;
    if (first) p = make_double2(yu, yv);
    else p = make_double2(yu + beta * in.p.x, yv + beta * in.p.y);
    const double qu = in.ti.x * p.x + t, qv = in.ti.y * p.y - t;
    const double2 x = make_double2(in.x.x + alpha * p.x, in.x.y + alpha * p.y);
    const double2 r = make_double2(in.r.x - alpha * qu, in.r.y - alpha * qv);
    st_sel(X, i, x, wt);
    st_sel(R, i, r, wt);
    st_sel(P, i, p, wt);
    double zu, zv;
    precond_apply(in.ti.x, in.ti.y, rho, r.x, r.y, zu, zv);
    acc[0] += r.x * zu + r.y * zv;
    acc[1] += r.x * r.x + r.y * r.y;
    acc[2] += in.ti.x * zu * zu + in.ti.y * zv * zv;
    acc[3] += in.ti.x * zu * p.x + in.ti.y * zv * p.y;
    acc[4] += in.ti.x * p.x * p.x + in.ti.y * p.y * p.y;
    return zu - zv;
  }
};

// The reduced system (Section 4, Theorem (thm:ne2_prec)): with
// d = dz_u - dz_v the two block rows of (eq:ne2_H) give
// (Theta_bar^{-1} + A^T A) d = Theta_bar^{-1} (Theta_u r_u - Theta_v r_v),
// Theta_bar = Theta_u + Theta_v, preconditioned by Theta_bar^{-1} + rho I.
// In Theta^{-1} entries (tu, tv): Theta_bar^{-1} = tu tv / (tu + tv), the
// right-hand side is (tv r_u - tu r_v) / (tu + tv), and the 2n direction
// follows without an operator product: du = (r_u + r_v + tv d) / (tu + tv),
// dv = du - d.  PCG vectors are n-vectors (x, r, p, Theta_bar^{-1}), the
// operator input is p itself.
struct RedVec {
  double* X;   // PCG solution d
  double* R;   // reduced residual
  double* P;   // direction
  double* TB;  // Theta_bar^{-1}
};
__device__ __forceinline__ RedVec red_vec(const TeamWS& w, long n) {
  RedVec v;
  v.X = reinterpret_cast<double*>(w.X);
  v.TB = v.X + n;
  v.P = reinterpret_cast<double*>(w.P);
  v.R = v.P + n;
  return v;
}
__device__ __forceinline__ double red_tbar(double tu, double tv) { return tu * tv / (tu + tv); }
__device__ __forceinline__ double red_rhs(double tu, double tv, double ru, double rv) {
  return (tv * ru - tu * rv) / (tu + tv);
}
__device__ __forceinline__ double2 red_back(double tu, double tv, double ru, double rv, double d) {
  const double du = (ru + rv + tv * d) / (tu + tv);
  return make_double2(du, du - d);
}

// PCG pass C on the reduced system: as FPcgC2 with n-vectors,
// y = r / (Theta_bar^{-1} + rho), q = Theta_bar^{-1} p + t; returns y'.
struct FPcgRed {
  static constexpr int K = 5;
  static constexpr bool CHAIN = true;
  struct In {
    double p, tb, x, r;
  };
  RedVec v;
  double alpha, beta, rho;
  int first;
  double acc[K];
  __device__ void reset() {
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.0;
  }
  __device__ void load(long i, In& in) const {
    if (!first) in.p = v.P[i];
    in.tb = v.TB[i];
    in.x = v.X[i];
    in.r = v.R[i];
  }
  __device__ double scatter(long i, double t, const In& in) {
    const double y = in.r / (in.tb + rho);
    const double p = first ? y : y + beta * in.p;
    const double q = in.tb * p + t;
    const double x = in.x + alpha * p, r = in.r - alpha * q;
    v.X[i] = x;
    v.R[i] = r;
    v.P[i] = p;
    const double yn = r / (in.tb + rho);
    acc[0] += r * yn;
    acc[1] += r * r;
    acc[2] += in.tb * yn * yn;
    acc[3] += in.tb * yn * p;
    acc[4] += in.tb * p * p;
    return yn;
  }
};

// Residual pass A: bring (z, s) up to date (initial point, pending step) or
// form the trial point of the corrector; d = x = u - v.
// acc0 += 1^T z, acc1 += z^T s.  As an elementwise functor (elem) it serves
// the residual pass B of the later iterations, whose operator input is formed
// by linearity instead.
enum { RA_INIT = 0, RA_STEP = 1, RA_TRIAL = 2, RA_NONE = 3 };
struct FResA {
  static constexpr int K = 2;
  struct In {
    double2 z, s, dz, ds;
  };
  double2* Z;
  double2* S;
  double2* DZ;
  double2* DS;
  double aP, aD, z0, s0;
  int mode;
  double acc[K];
  __device__ void reset() { acc[0] = acc[1] = 0.0; }
  __device__ void load(long i, In& in) const {
    if (mode != RA_INIT) {
      in.z = Z[i];
      in.s = S[i];
    }
    if (mode == RA_STEP || mode == RA_TRIAL) {
      in.dz = DZ[i];
      in.ds = DS[i];
    }
  }
  __device__ double gather(long i, const In& in) {
    double2 z, s;
    if (mode == RA_INIT) {
      z = make_double2(z0, z0);
      s = make_double2(s0, s0);
    } else if (mode == RA_NONE) {
      z = in.z;
      s = in.s;
    } else {
      z = make_double2(in.z.x + aP * in.dz.x, in.z.y + aP * in.dz.y);
      s = make_double2(in.s.x + aD * in.ds.x, in.s.y + aD * in.ds.y);
    }
    if (mode == RA_INIT || mode == RA_STEP) {
      Z[i] = z;
      S[i] = s;
    }
    acc[0] += z.x + z.y;
    acc[1] += z.x * s.x + z.y * s.y;
    return z.x - z.y;
  }
  __device__ void elem(long i, const In& in) { (void)gather(i, in); }
};

// Residual pass C: with g = A^T (A x - b) build the Newton right-hand side
// rhs = f_z + Z^{-1} f_s, f_z = s - [tau + g; tau - g], f_s = sigma mu - z s
// (eqs. (fzfs), (redNewtonA)); store Theta^{-1} = s / z (not at the trial
// point), r = rhs, x = 0.  acc0 = max |g|, acc1 += rhs^T rhs,
// acc2 += rhs^T P^{-1} rhs, acc3 += y^T Theta^{-1} y with y = P^{-1} rhs;
// returns y_u - y_v, the first PCG direction's gather.
template <bool RED>
struct FResCT {
  static constexpr int K = 4;
  static constexpr bool CHAIN = true;
  struct In {
    double2 z, s, dz, ds, ti;
  };
  double2* Z;
  double2* S;
  double2* DZ;
  double2* DS;
  double2* TI;
  double2* R;
  double2* X;
  RedVec v;  // reduced system (RED)
  double tau, sigma, mu, aP, aD, rho;
  int trial;
  double acc[K];
  __device__ void reset() {
    acc[0] = -__builtin_inf();
    acc[1] = acc[2] = acc[3] = 0.0;
  }
  __device__ void load(long i, In& in) const {
    in.z = Z[i];
    in.s = S[i];
    if (trial) {
      in.dz = DZ[i];
      in.ds = DS[i];
      in.ti = TI[i];
    }
  }
  __device__ double scatter(long i, double g, const In& in) {
    double2 zt = in.z, st = in.s, ti;
    if (trial) {
      zt = make_double2(in.z.x + aP * in.dz.x, in.z.y + aP * in.dz.y);
      st = make_double2(in.s.x + aD * in.ds.x, in.s.y + aD * in.ds.y);
      ti = in.ti;
    } else {
      ti = make_double2(in.s.x / in.z.x, in.s.y / in.z.y);
      TI[i] = ti;
    }
    const double fzu = st.x - (tau + g), fzv = st.y - (tau - g);
    const double fsu = sigma * mu - zt.x * st.x, fsv = sigma * mu - zt.y * st.y;
    const double ru = fzu + fsu / in.z.x, rv = fzv + fsv / in.z.y;
    R[i] = make_double2(ru, rv);
    acc[0] = fmax(acc[0], fabs(g));
    if constexpr (RED) {
      // the reduced right-hand side; R keeps the 2n one for the back-substitution
      const double tb = red_tbar(ti.x, ti.y);
      if (!trial) v.TB[i] = tb;
      const double rb = red_rhs(ti.x, ti.y, ru, rv);
      v.R[i] = rb;
      v.X[i] = 0.0;
      const double y = rb / (tb + rho);
      acc[1] += rb * rb;
      acc[2] += rb * y;
      acc[3] += tb * y * y;
      return y;
    } else {
      X[i] = make_double2(0.0, 0.0);
      acc[1] += ru * ru + rv * rv;
      double yu, yv;
      precond_apply(ti.x, ti.y, rho, ru, rv, yu, yv);
      acc[2] += ru * yu + rv * yv;
      acc[3] += ti.x * yu * yu + ti.y * yv * yv;
      return yu - yv;  // first gather of the PCG that follows
    }
  }
};

// Step pass (elementwise).  Predictor: ds = f_s / z - Theta^{-1} dz
// (eq. (redNewtonB)), store DZ, DS.  Corrector: the same at the trial point
// with sigma3, added to the stored predictor direction.  acc0 = min ratio
// over dz < 0 of -z/dz, acc1 likewise for s.  Run as a gather pass, it hands
// dz_u - dz_v to the operator's first stage, whose result (the transform of
// the x-direction) the next residual combines by linearity.
template <bool RED>
struct FStepT {
  static constexpr int K = 2;
  struct In {
    double2 z, s, ti, x, dz, ds;
    double d;
  };
  double2* Z;
  double2* S;
  double2* TI;
  double2* X;  // 2n: the PCG solution; reduced: the 2n right-hand side
  double2* DZ;
  double2* DS;
  const double* Xr;  // reduced: the PCG solution d
  double sigma, mu;      // predictor: sigma, mu; corrector: sigma3, mu~
  double aPp, aDp;       // predictor step sizes (corrector only)
  int corr;
  double acc[K];
  __device__ void reset() { acc[0] = acc[1] = __builtin_inf(); }
  __device__ void load(long i, In& in) const {
    in.z = Z[i];
    in.s = S[i];
    in.ti = TI[i];
    in.x = X[i];
    if constexpr (RED) in.d = Xr[i];
    if (corr) {
      in.dz = DZ[i];
      in.ds = DS[i];
    }
  }
  __device__ double gather(long i, const In& in) {
    // the Newton direction of this solve (2n, or back-substituted from d)
    const double2 sol = RED ? red_back(in.ti.x, in.ti.y, in.x.x, in.x.y, in.d) : in.x;
    double2 dz, ds;
    if (!corr) {
      dz = sol;
      const double fsu = sigma * mu - in.z.x * in.s.x, fsv = sigma * mu - in.z.y * in.s.y;
      ds = make_double2(fsu / in.z.x - in.ti.x * dz.x, fsv / in.z.y - in.ti.y * dz.y);
    } else {
      const double ztu = in.z.x + aPp * in.dz.x, ztv = in.z.y + aPp * in.dz.y;
      const double stu = in.s.x + aDp * in.ds.x, stv = in.s.y + aDp * in.ds.y;
      const double fsu = sigma * mu - ztu * stu, fsv = sigma * mu - ztv * stv;
      const double dsu = fsu / in.z.x - in.ti.x * sol.x, dsv = fsv / in.z.y - in.ti.y * sol.y;
      dz = make_double2(in.dz.x + sol.x, in.dz.y + sol.y);
      ds = make_double2(in.ds.x + dsu, in.ds.y + dsv);
    }
    DZ[i] = dz;
    DS[i] = ds;
    if (dz.x < 0) acc[0] = fmin(acc[0], -in.z.x / dz.x);
    if (dz.y < 0) acc[0] = fmin(acc[0], -in.z.y / dz.y);
    if (ds.x < 0) acc[1] = fmin(acc[1], -in.s.x / ds.x);
    if (ds.y < 0) acc[1] = fmin(acc[1], -in.s.y / ds.y);
    return dz.x - dz.y;
  }
};

// Output pass: x = u - v.
struct FOut {
  static constexpr int K = 1;
  struct In {
    double2 z;
  };
  double2* Z;
  double* x;
  double acc[K];
  __device__ void reset() { acc[0] = 0.0; }
  __device__ void load(long i, In& in) const { in.z = Z[i]; }
  __device__ void elem(long i, const In& in) { x[i] = in.z.x - in.z.y; }
};

// Adjoint set-up (a pass-A functor): Theta^{-1} = s / z at the given state,
// r = rhs = [g; -g], x = 0, and the first PCG gather d = y_u - y_v with
// y = P^{-1} rhs.  acc0 += rhs^T P^{-1} rhs, acc1 += rhs^T rhs,
// acc2 += y^T Theta^{-1} y.
template <bool RED>
struct FBwdInitT {
  static constexpr int K = 3;
  struct In {
    double2 z, s;
    double g;
  };
  const double2* Z;
  const double2* S;
  const double* gx;
  double2* TI;
  double2* R;
  double2* X;
  RedVec v;
  double rho;
  double acc[K];
  __device__ void reset() { acc[0] = acc[1] = acc[2] = 0.0; }
  __device__ void load(long i, In& in) const {
    in.z = Z[i];
    in.s = S[i];
    in.g = gx[i];
  }
  __device__ double gather(long i, const In& in) {
    const double2 ti = make_double2(in.s.x / in.z.x, in.s.y / in.z.y);
    TI[i] = ti;
    const double ru = in.g, rv = -in.g;
    R[i] = make_double2(ru, rv);
    if constexpr (RED) {
      // reduced right-hand side of [g; -g]: (tv g + tu g) / (tu + tv) = g
      const double tb = red_tbar(ti.x, ti.y);
      v.TB[i] = tb;
      const double rb = red_rhs(ti.x, ti.y, ru, rv);
      v.R[i] = rb;
      v.X[i] = 0.0;
      const double y = rb / (tb + rho);
      acc[0] += rb * y;
      acc[1] += rb * rb;
      acc[2] += tb * y * y;
      return y;
    } else {
      X[i] = make_double2(0.0, 0.0);
      double yu, yv;
      precond_apply(ti.x, ti.y, rho, ru, rv, yu, yv);
      acc[0] += ru * yu + rv * yv;
      acc[1] += ru * ru + rv * rv;
      acc[2] += ti.x * yu * yu + ti.y * yv * yv;
      return yu - yv;
    }
  }
};

// Adjoint output gather: d = w_u - w_v; acc0 += 1^T w (reduced: w from the
// back-substitution of [g; -g] with d = the PCG solution).
template <bool RED>
struct FBwdGatherT {
  static constexpr int K = 1;
  struct In {
    double2 w, ti, r;
    double d;
  };
  double2* W;
  const double2* TI;
  const double2* R;
  const double* Xr;
  double acc[K];
  __device__ void reset() { acc[0] = 0.0; }
  __device__ void load(long i, In& in) const {
    if constexpr (RED) {
      in.ti = TI[i];
      in.r = R[i];
      in.d = Xr[i];
    } else {
      in.w = W[i];
    }
  }
  __device__ double gather(long i, const In& in) {
    const double2 w = RED ? red_back(in.ti.x, in.ti.y, in.r.x, in.r.y, in.d) : in.w;
    acc[0] += w.x + w.y;
    return w.x - w.y;
  }
};

// ------------------------------------------------------------------------
// pass runners
// ------------------------------------------------------------------------

template <int K>
__device__ __forceinline__ void kinds_fill(int (&k)[K], int a, int b = 0, int c = 0, int d = 0) {
  const int v[4] = {a, b, c, d};
#pragma unroll
  for (int j = 0; j < K; ++j) k[j] = v[j];
}

template <class F>
__device__ __forceinline__ void finish_item(Ctx& cx, F& f, const int (&kinds)[F::K], double* part, int item) {
  double v[F::K];
#pragma unroll
  for (int j = 0; j < F::K; ++j) v[j] = f.acc[j];
  wg_reduce<F::K>(kinds, v, cx.red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < F::K; ++j) part[(long)item * MF_MAXK + j] = v[j];
  }
}

template <class OP, class F>
__device__ __forceinline__ void run_A(Ctx& cx, OP& op, F& f, const int (&kinds)[F::K], double* part) {
  const int ni = op.nA();
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    f.reset();
    op.passA(it, f);
    finish_item(cx, f, kinds, part, it);
  }
}

template <class OP, class F>
__device__ __forceinline__ void run_C(Ctx& cx, OP& op, F& f, const int (&kinds)[F::K], double* part) {
  const int ni = op.nC();
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    f.reset();
    op.passC(it, f);
    finish_item(cx, f, kinds, part, it);
  }
}

// pass B: two sums (y^2, b.y).  HAPPLY mode combines the direction first
// (beta, first; see the operators).
template <class OP>
__device__ __forceinline__ void run_B(Ctx& cx, OP& op, int mode, double* part, double* out, double beta = 0.0,
                                      int first = 1);

template <>
__device__ __forceinline__ void run_B<OpDense>(Ctx& cx, OpDense& op, int mode, double* part, double* out,
                                               double beta, int first) {
  const int ni = op.nB();
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    double acc[2] = {0.0, 0.0};
    op.passB(it, mode, acc, out, beta, first);
    if (threadIdx.x == 0) {
      part[(long)it * MF_MAXK + 0] = acc[0];
      part[(long)it * MF_MAXK + 1] = acc[1];
    }
  }
}

// transform operators: per-thread partials reduced per item
template <class OP>
__device__ __forceinline__ void run_B_transform(Ctx& cx, OP& op, int mode, double* part, double beta, int first) {
  const int ni = op.nB();
  const int kinds[2] = {0, 0};
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    double acc[2] = {0.0, 0.0};
    op.passB(it, mode, acc, beta, first);
    wg_reduce<2>(kinds, acc, cx.red);
    if (threadIdx.x == 0) {
      part[(long)it * MF_MAXK + 0] = acc[0];
      part[(long)it * MF_MAXK + 1] = acc[1];
    }
  }
}
template <>
__device__ __forceinline__ void run_B<OpPdct>(Ctx& cx, OpPdct& op, int mode, double* part, double*, double beta,
                                              int first) {
  run_B_transform(cx, op, mode, part, beta, first);
}
template <>
__device__ __forceinline__ void run_B<OpWht>(Ctx& cx, OpWht& op, int mode, double* part, double*, double beta,
                                             int first) {
  run_B_transform(cx, op, mode, part, beta, first);
}
template <>
__device__ __forceinline__ void run_B<OpDenseDirect>(Ctx& cx, OpDenseDirect& op, int mode, double* part, double* out,
                                                     double beta, int first) {
  run_B<OpDense>(cx, op, mode, part, out, beta, first);
}

// loads in flight per lane in the reductions over items (see reduce_items)
template <class OP>
__device__ constexpr int red_unroll() {
  return (std::is_same<OP, OpPdct>::value || std::is_same<OP, OpWht>::value) ? 4 : 1;
}

// whether the PCG vector stores write through the L2 (see st_wt)
__device__ __forceinline__ int op_write_through(const OpPdct& op) { return op.wt; }
template <class OP>
__device__ __forceinline__ int op_write_through(const OP&) {
  return 0;
}

// the search-direction buffers of iteration `it` (dense: alternating d of p)
__device__ __forceinline__ void op_direction(OpDense& op, const TeamWS& w, int it) {
  op.Dp_prev = (it & 1) ? w.Dp0 : w.Dp1;
  op.Dp_cur = (it & 1) ? w.Dp1 : w.Dp0;
}
__device__ __forceinline__ void op_direction(OpPdct&, const TeamWS&, int) {}
__device__ __forceinline__ void op_direction(OpWht&, const TeamWS&, int) {}

// The operator's first stage (pass A) writes the transform of the step
// direction instead of the operator input (on = 1), or back (on = 0).
__device__ __forceinline__ void op_step_target(OpDense& op, const TeamWS& w, int on) { op.D = on ? w.Dd : w.D; }
__device__ __forceinline__ void op_step_target(OpPdct& op, const TeamWS& w, int on) { op.Y1 = on ? w.Yd : w.Y1; }
__device__ __forceinline__ void op_step_target(OpWht& op, const TeamWS& w, int on) {
  op.Y1 = reinterpret_cast<double*>(on ? w.Yd : w.Y1);
}
// After a residual pass B that kept x: dense swaps its current / next x.
__device__ __forceinline__ void op_x_advance(OpDense& op) {
  double* t = op.Dxc;
  op.Dxc = op.Dxn;
  op.Dxn = t;
}
__device__ __forceinline__ void op_x_advance(OpPdct&) {}
__device__ __forceinline__ void op_x_advance(OpWht&) {}

// elementwise pass over [0, n), items of 1024 indices
template <class F>
__device__ __forceinline__ void run_E(Ctx& cx, long n, F& f, const int (&kinds)[F::K], double* part) {
  const int ni = (int)((n + 1023) / 1024);
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    f.reset();
    const long base = (long)it * 1024;
    constexpr int U = 1024 / MF_THREADS;
    typename F::In in[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long i = base + threadIdx.x + k * MF_THREADS;
      if (i < n) f.load(i, in[k]);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long i = base + threadIdx.x + k * MF_THREADS;
      if (i < n) f.elem(i, in[k]);
    }
    finish_item(cx, f, kinds, part, it);
  }
}
__device__ __forceinline__ int nE(long n) { return (int)((n + 1023) / 1024); }

// Elementwise work that shares a pass with nb operator items: it goes to the
// workgroups without an operator item when there are any (items of 2^lchunk
// indices, at most one per such workgroup), else to all in items of 1024.
__device__ __forceinline__ void span_E(const Ctx& cx, long n, int nb, int& r0, int& nr, int& lchunk) {
  if (nb < cx.t.size) {
    r0 = nb;
    nr = cx.t.size - nb;
    lchunk = 10;
    while ((((n + (1L << lchunk) - 1) >> lchunk)) > nr) ++lchunk;
  } else {
    r0 = 0;
    nr = cx.t.size;
    lchunk = 10;
  }
}

// elementwise pass over [0, n) in items of 2^lchunk (>= 1024) indices, item j
// taken by team rank r0 + (j mod nr)
template <class F>
__device__ __forceinline__ void run_E_span(Ctx& cx, long n, F& f, const int (&kinds)[F::K], double* part, int r0,
                                           int nr, int lchunk) {
  const int ni = (int)((n + (1L << lchunk) - 1) >> lchunk);
  const int me = cx.t.rank - r0;
  if (me < 0 || me >= nr) return;
  for (int it = me; it < ni; it += nr) {
    f.reset();
    const long end = ((long)(it + 1) << lchunk) < n ? ((long)(it + 1) << lchunk) : n;
    for (long base = (long)it << lchunk; base < end; base += 1024) {
      constexpr int U = 1024 / MF_THREADS;
      typename F::In in[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const long i = base + threadIdx.x + k * MF_THREADS;
        if (i < end) f.load(i, in[k]);
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const long i = base + threadIdx.x + k * MF_THREADS;
        if (i < end) f.elem(i, in[k]);
      }
    }
    finish_item(cx, f, kinds, part, it);
  }
}

// ------------------------------------------------------------------------
// Operator construction and set-up
// ------------------------------------------------------------------------
__device__ __forceinline__ void make_op(OpDense& op, const KArgs& a, const InstDesc& d, const TeamWS& w, char* lds,
                                        int team_size) {
  op.n = d.n;
  op.m = d.m;
  op.lda = d.n;
  op.A = a.A + (a.shared_op ? 0 : d.a_off);
  op.b = a.b ? a.b + d.m_off : nullptr;
  op.D = w.D;
  op.Yv = w.Yv;
  op.PT = w.PT;
  op.Dp_prev = w.Dp1;
  op.Dp_cur = w.Dp0;
  op.Dxc = w.Dx0;
  op.Dxn = w.Dx1;
  op.Dd = w.Dd;
  op.RB = a.tile_param > 0 ? (a.tile_param > DN_RBMAX ? DN_RBMAX : a.tile_param) : 8;
  op.lds = (double*)lds;
  op.dsh = (double2*)(lds + (MF_WAVES * DN_RBMAX + DN_RG * DN_CB) * sizeof(double));
  op.fused = (d.n <= DN_FUSED_MAXN) && ((d.n & 1) == 0) && a.lay.pt_chunks > 0;
  // fused: chunks of whole row blocks, at most one per workgroup of the team
  const long blocks = (d.m + DN_FB - 1) / DN_FB;
  long nc = team_size < a.lay.pt_chunks ? team_size : a.lay.pt_chunks;
  if (nc > blocks) nc = blocks;
  if (nc < 1) nc = 1;
  const long bpc = (blocks + nc - 1) / nc;
  op.chunk_rows = (int)(bpc * DN_FB);
  op.nchunk = (int)((d.m + op.chunk_rows - 1) / op.chunk_rows);
}

// Direct variant: the dense operator for the residuals and steps, plus the
// factorisation's buffers; its LDS staging reuses the dense passes' LDS
// (nothing there outlives a pass).
__device__ __forceinline__ void make_op(OpDenseDirect& op, const KArgs& a, const InstDesc& d, const TeamWS& w,
                                        char* lds, int team_size) {
  make_op(static_cast<OpDense&>(op), a, d, w, lds, team_size);
  op.K = w.DK;
  op.M = w.DM;
  op.Li = w.DLi;
  op.y = w.DY;
  op.sX = reinterpret_cast<double*>(lds);
  op.sY = op.sX + DC_NB * DC_LD;
  op.npad = dc_npad(d.n);
  op.T = (int)(op.npad / DC_NB);
}

__device__ __forceinline__ int ilog2(long v) {
  int l = 0;
  while ((1L << l) < v) ++l;
  return l;
}

__device__ __forceinline__ void make_op(OpPdct& op, const KArgs& a, const InstDesc& d, const TeamWS& w, char* lds,
                                        int team_size) {
  op.n = d.n;
  op.m = d.m;
  op.H = (int)(d.n >> 1);
  op.logn = ilog2(d.n);
  const int lh = op.logn - 1;
  int l1 = lh / 2;
  if (a.tile_param > 0) l1 = a.tile_param;
  if (l1 > 9) l1 = 9;
  if (lh - l1 > 11) l1 = lh - 11;
  if (lh - l1 < 3) l1 = lh - 3;
  op.l1 = l1;
  op.l2 = lh - l1;
  op.N1 = 1 << op.l1;
  op.N2 = 1 << op.l2;
  // narrower pass-A/C items when blocks of 8 columns would leave workgroups idle
  op.lcb = (op.N2 >> 3) < team_size ? 2 : 3;
  op.rows = a.rows + (a.shared_op ? 0 : d.m_off);
  op.b = a.b ? a.b + d.m_off : nullptr;
  op.Y1 = w.Y1;
  op.Y1p = w.Y1p;
  op.Yx = w.Yx;
  op.Yd = w.Yd;
  op.Y2 = w.Y2;
  op.mask = w.mask;
  op.bt = w.bt;
  op.XS = w.XS;
  op.tw.lo = (const cplx*)lds + PD_TILE_LDS;
  op.tw.hi = op.tw.lo + (1 << a.tw_lo_bits);
  op.tw.lo_bits = a.tw_lo_bits;
  op.msk = (unsigned char*)(op.tw.hi + (1 << (a.tw_log2n_max + 2 - a.tw_lo_bits)));
  op.cur_k1a = 0;
  op.tw.scale_shift = a.tw_log2n_max - op.logn;
  op.tile = (cplx*)lds;
  // Write-through pays at large lengths only (measured: it shortens the
  // barriers' L2 write-back at n = 2^18 and 2^20, and costs more than it
  // saves at n = 2^16 and for one-workgroup teams, which skip that write-back).
  op.wt = team_size > 1 && d.n >= (1L << 18);
  op.a0 = sqrt(1.0 / (double)d.n);
  op.a1 = sqrt(2.0 / (double)d.n);
  op.flip = a.op_flip;
}

__device__ __forceinline__ void make_op(OpWht& op, const KArgs& a, const InstDesc& d, const TeamWS& w, char* lds,
                                        int team_size) {
  op.n = d.n;
  op.m = d.m;
  const int ln = ilog2(d.n);
  int l1 = ln / 2;
  if (a.tile_param > 0) l1 = a.tile_param;
  // columns of length <= 2^13 (the LDS tile), rows of length <= 2^12
  if (l1 > 13) l1 = 13;
  if (l1 > ln - 2) l1 = ln - 2;
  if (l1 < 2) l1 = 2;
  if (ln - l1 > 12) l1 = ln - 12;
  op.l1 = l1;
  op.l2 = ln - l1;
  op.N1 = 1 << op.l1;
  op.N2 = 1 << op.l2;
  // widest blocks that fit the 8192-double tile, narrowed while they would
  // leave workgroups of the team idle
  int lcb = 4;
  if (lcb > 13 - op.l1) lcb = 13 - op.l1;
  if (lcb > op.l2) lcb = op.l2;
  while (lcb > 0 && (op.N2 >> lcb) < team_size) --lcb;
  int lrb = 3;
  if (lrb > 13 - op.l2) lrb = 13 - op.l2;
  if (lrb > op.l1) lrb = op.l1;
  while (lrb > 0 && (op.N1 >> lrb) < team_size) --lrb;
  op.lcb = lcb;
  op.lrb = lrb;
  op.rows = a.rows + (a.shared_op ? 0 : d.m_off);
  op.b = a.b ? a.b + d.m_off : nullptr;
  op.Y1 = reinterpret_cast<double*>(w.Y1);
  op.Y1p = reinterpret_cast<double*>(w.Y1p);
  op.Yx = reinterpret_cast<double*>(w.Yx);
  op.Yd = reinterpret_cast<double*>(w.Yd);
  op.Y2 = reinterpret_cast<double*>(w.Y2);
  op.mask = w.mask;
  op.bt = w.bt;
  op.XS = w.XS;
  op.tile = reinterpret_cast<double*>(lds);
  op.scale = 1.0 / sqrt((double)d.n);
}

// Dense set-up: nothing to build.  Returns 0 (ok) or ST_ABORTED.
__device__ __forceinline__ int op_setup(Ctx& cx, OpDense&, const KArgs&, const TeamWS&, int) { return 0; }

// Transform operators' set-up: zero the coefficient mask / b~, then scatter
// the sampled rows (checking they are sorted, distinct and in range).
// with_b = 0 skips b~.
template <class OP>
__device__ __forceinline__ int rows_setup(Ctx& cx, OP& op, const TeamWS& w, int with_b) {
  const long n = op.n;
  const long nthr = (long)cx.t.size * MF_THREADS;
  const long gt = (long)cx.t.rank * MF_THREADS + threadIdx.x;
  if (gt == 0) *w.err = 0;
  for (long i = gt; i < n; i += nthr) {
    w.mask[i] = 0;
    w.bt[i] = 0.0;
  }
  if (team_barrier(cx.t)) return ST_ABORTED;
  int bad = 0;
  for (long i = gt; i < op.m; i += nthr) {
    const long kk = op.rows[i];
    if (kk < 0 || kk >= n || (i > 0 && op.rows[i - 1] >= kk)) {
      bad = 1;
      continue;
    }
    const long p = op.coef_pos(kk);
    w.mask[p] = 1;
    if (with_b) w.bt[p] = op.b[i];
  }
  if (bad) __hip_atomic_store(w.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (team_barrier(cx.t)) return ST_ABORTED;
  if (ld_flag(w.err)) return ST_DEVICE_CHECK;
  return 0;
}

// PDCT set-up: the twiddle tables to LDS, then the rows.
__device__ __forceinline__ int op_setup(Ctx& cx, OpPdct& op, const KArgs& a, const TeamWS& w, int with_b) {
  cplx* lo = const_cast<cplx*>(op.tw.lo);
  cplx* hi = const_cast<cplx*>(op.tw.hi);
  const int nlo = 1 << a.tw_lo_bits;
  const int nhi = 1 << (a.tw_log2n_max + 2 - a.tw_lo_bits);
  for (int e = threadIdx.x; e < nlo; e += MF_THREADS) lo[e] = a.tw_lo[e];
  for (int e = threadIdx.x; e < nhi; e += MF_THREADS) hi[e] = a.tw_hi[e];
  __syncthreads();
  return rows_setup(cx, op, w, with_b);
}
__device__ __forceinline__ int op_setup(Ctx& cx, OpWht& op, const KArgs&, const TeamWS& w, int with_b) {
  return rows_setup(cx, op, w, with_b);
}

// rho: Frobenius-closest scalar to A^T A (Section 4, before eq. (eq:ne2_P)).
__device__ __forceinline__ double op_rho(Ctx& cx, OpDense& op, const TeamWS& w, int& ab) {
  const int ni = op.nF();
  for (int it = cx.t.rank; it < ni; it += cx.t.size) {
    const double s = op.frob_block(it);
    if (threadIdx.x == 0) w.partS[(long)it * MF_MAXK] = s;
  }
  ab = team_barrier(cx.t);
  const int kinds[1] = {0};
  double r[1];
  reduce_items<1>(kinds, w.partS, ni, r, cx.red);
  return r[0] / (double)op.n;
}
__device__ __forceinline__ double op_rho(Ctx&, OpPdct& op, const TeamWS&, int& ab) {
  ab = 0;
  return (double)op.m / (double)op.n;  // orthonormal rows: ||A||_F^2 = m
}
__device__ __forceinline__ double op_rho(Ctx&, OpWht& op, const TeamWS&, int& ab) {
  ab = 0;
  return (double)op.m / (double)op.n;  // orthonormal rows: ||A||_F^2 = m
}

// ------------------------------------------------------------------------
// PCG on (Theta^{-1} + F F^T) x = rhs with the block preconditioner
// (Section 4), two team barriers per iteration.  On entry R = rhs, X = 0,
// TI set, and the operator holds the first gather d(y0) (y0 = P^{-1} rhs)
// from the pass that built rhs; rhs2 = ||rhs||^2, gamma = rhs^T y0,
// yty = y0^T Theta^{-1} y0.  Per iteration:
//   pass B: combine the direction's transform (y + beta p), operator middle
//           stage, partial ||A d||^2 (so p^T H p = p^T Theta^{-1} p + ||A d||^2)
//   pass C: operator last stage, q, x and r updates, next y and its gather,
//           partial dot products for beta and p^T Theta^{-1} p.
// Returns a status (0 = ok); *iters = operator applies.
// ------------------------------------------------------------------------
template <class OP, bool RED>
__device__ __forceinline__ int pcg_run(Ctx& cx, OP& op, const TeamWS& w, double rho, double tol, int maxit,
                                       double rhs2, double gamma, double yty, int* iters, int* capped = nullptr) {
  const int kB[1] = {0};
  const int kC[5] = {0, 0, 0, 0, 0};
  double rr = rhs2, beta = 0.0, ptp = yty;
  int it = 0, status = 0;
  for (;;) {
    if (!isfinite(rr)) {
      status = ST_NONFINITE;
      break;
    }
    if (rr <= tol * tol * rhs2) break;
    if (it == maxit) {
      if (capped) *capped = 1;
      break;
    }
    const int first = (it == 0);
    op_direction(op, w, it);
    run_B<OP>(cx, op, 0, w.partB, nullptr, beta, first);
    if (team_barrier(cx.t)) {
      status = ST_ABORTED;
      break;
    }
    double pB[1];
    reduce_items<1, red_unroll<OP>()>(kB, w.partB, op.nB(), pB, cx.red);
    ++it;
    const double pq = ptp + pB[0];
    if (!(pq > 0.0)) {
      status = isfinite(pq) ? ST_PCG_BREAKDOWN : ST_NONFINITE;
      break;
    }
    if constexpr (RED) {
      FPcgRed fc;
      fc.v = red_vec(w, op.n);
      fc.rho = rho;
      fc.alpha = gamma / pq;
      fc.beta = beta;
      fc.first = first;
      run_C(cx, op, fc, kC, w.partC);
    } else {
      FPcgC2 fc;
      fc.P = w.P;
      fc.TI = w.TI;
      fc.X = w.X;
      fc.R = w.R;
      fc.rho = rho;
      fc.alpha = gamma / pq;
      fc.beta = beta;
      fc.first = first;
      fc.wt = op_write_through(op);
      run_C(cx, op, fc, kC, w.partC);
    }
    if (team_barrier(cx.t)) {
      status = ST_ABORTED;
      break;
    }
    double pC[5];
    reduce_items<5, red_unroll<OP>()>(kC, w.partC, op.nC(), pC, cx.red);
    beta = pC[0] / gamma;
    gamma = pC[0];
    rr = pC[1];
    ptp = pC[2] + 2.0 * beta * pC[3] + beta * beta * pC[4];
  }
  *iters = it;
  return status;
}

// Residual evaluation at the current point (after the pending update given by
// mode/aP/aD) or at the trial point: computes the gap terms and the Newton
// right-hand side for sigma (and mu = z^T s/(2n) at that point).
struct ResOut {
  double sumz, zs, rb2, brb, ginf, rhs2, rty, yty;
  int status;
};

template <class OP, bool RED>
__device__ __forceinline__ ResOut residual_rhs(Ctx& cx, OP& op, const TeamWS& w, double2* Z, double2* S, const DevParams& prm,
                               int mode, double aP, double aD, double tau, double sigma, double sigma3,
                               int trial, double rho) {
  ResOut o;
  o.status = 0;
  FResA fa;
  fa.Z = Z;
  fa.S = S;
  fa.DZ = w.DZ;
  fa.DS = w.DS;
  fa.aP = aP;
  fa.aD = aD;
  fa.z0 = prm.z0;
  fa.s0 = prm.s0;
  fa.mode = mode;
  const int kA[2] = {0, 0};
  const int kb[2] = {0, 0};
  double pA[2], pB[2];
  if (mode == RA_INIT) {
    // set z, s and gather x through pass A; pass B keeps the transform of x
    run_A(cx, op, fa, kA, w.partA);
    if (team_barrier(cx.t)) {
      o.status = ST_ABORTED;
      return o;
    }
    reduce_items<2, red_unroll<OP>()>(kA, w.partA, op.nA(), pA, cx.red);
    run_B<OP>(cx, op, 1, w.partB, nullptr);
    if (team_barrier(cx.t)) {
      o.status = ST_ABORTED;
      return o;
    }
    reduce_items<2, red_unroll<OP>()>(kb, w.partB, op.nB(), pB, cx.red);
    op_x_advance(op);
  } else {
    // The step pass left the transform of the step direction; the operator's
    // input at the new (or trial) point is x + aP dx by linearity, formed in
    // pass B, whose idle workgroups meanwhile apply the step to (z, s) (or
    // form the trial point) and sum 1^T z and z^T s.
    run_B<OP>(cx, op, mode == RA_STEP ? 3 : 4, w.partB, nullptr, aP, 0);
    int r0, nr, lchunk;
    span_E(cx, op.n, op.nB(), r0, nr, lchunk);
    run_E_span(cx, op.n, fa, kA, w.partS, r0, nr, lchunk);
    if (team_barrier(cx.t)) {
      o.status = ST_ABORTED;
      return o;
    }
    reduce_items<2, red_unroll<OP>()>(kb, w.partB, op.nB(), pB, cx.red);
    reduce_items<2, red_unroll<OP>()>(kA, w.partS, (int)((op.n + (1L << lchunk) - 1) >> lchunk), pA, cx.red);
    if (mode == RA_STEP) op_x_advance(op);
  }
  o.sumz = pA[0];
  o.zs = pA[1];
  o.rb2 = pB[0];
  o.brb = pB[1];
  FResCT<RED> fc;
  fc.v = red_vec(w, op.n);
  fc.Z = Z;
  fc.S = S;
  fc.DZ = w.DZ;
  fc.DS = w.DS;
  fc.TI = w.TI;
  fc.R = w.R;
  fc.X = w.X;
  fc.tau = tau;
  fc.sigma = trial ? sigma3 : sigma;
  fc.mu = o.zs / (2.0 * (double)op.n);
  fc.aP = aP;
  fc.aD = aD;
  fc.rho = rho;
  fc.trial = trial;
  const int kC[4] = {1, 0, 0, 0};
  run_C(cx, op, fc, kC, w.partC);
  if (team_barrier(cx.t)) {
    o.status = ST_ABORTED;
    return o;
  }
  double pC[4];
  reduce_items<4, red_unroll<OP>()>(kC, w.partC, op.nC(), pC, cx.red);
  o.ginf = pC[0];
  o.rhs2 = pC[1];
  o.rty = pC[2];
  o.yty = pC[3];
  return o;
}

template <class OP, bool RED>
__device__ __forceinline__ void solve_instance(Ctx& cx, const KArgs& a, int ii, char* lds) {
  const InstDesc d = a.inst[ii];
  const TeamWS w = make_ws(a, cx.t.id);
  const DevParams& prm = a.prm;
  OP op;
  make_op(op, a, d, w, lds, cx.t.size);
  const long n = d.n;
  double2* Z = a.state ? (double2*)(a.state + 4 * d.n_off) : w.Zs;
  double2* S = a.state ? (double2*)(a.state + 4 * d.n_off + 2 * d.n) : w.Ss;
  const double tau = d.tau;

  int status = ST_MAXITER;
  int k = 1, pcg_total = 0, ncorr = 0;
  long nmat = 0;
  double relgap = __builtin_nan(""), mu = 0.0, primal = 0.0, dual = 0.0, rho = prm.rho;
  int st = op_setup(cx, op, a, w, 1);
  if (st) status = st;
  if (!st && !(prm.rho > 0.0)) {
    int ab = 0;
    rho = op_rho(cx, op, w, ab);
    if (ab) st = status = ST_ABORTED;
  }
  constexpr bool DIRECT = std::is_same<OP, OpDenseDirect>::value;
  if constexpr (DIRECT) {
    if (!st) {
      st = direct_setup(cx, op, w.err);
      if (st) status = st;
    }
  }
  if (!st) {
    double aP_prev = 1.0, aD_prev = 1.0, aP = 0.0, aD = 0.0;
    int mode = RA_INIT;
    const int kS[2] = {2, 2};
    for (;;) {
      // sigma for this iteration from the previous step sizes
      const double sigma = (k != 1 && (aP_prev <= prm.alpha_bar || aD_prev <= prm.alpha_bar)) ? prm.sigma2
                                                                                               : prm.sigma1;
      ResOut ro = residual_rhs<OP, RED>(cx, op, w, Z, S, prm, mode, aP, aD, tau, sigma, prm.sigma3, 0, rho);
      nmat += 2;
      if (ro.status) {
        status = ro.status;
        break;
      }
      mu = ro.zs / (2.0 * (double)n);
      primal = tau * ro.sumz + 0.5 * ro.rb2;
      const double theta = ro.ginf <= tau ? 1.0 : tau / ro.ginf;
      dual = -0.5 * theta * theta * ro.rb2 - theta * ro.brb;
      relgap = (primal - dual) / (1.0 + fabs(primal));
      if (!isfinite(relgap)) {
        status = ST_NONFINITE;
        break;
      }
      if (relgap <= prm.tol) {
        status = ST_CONVERGED;
        break;
      }
      if (k > prm.maxiters) {
        status = ST_MAXITER;
        break;
      }
      int its = 0;
      if constexpr (DIRECT) {
        // exact direction: factorise M for this Theta, then the two sweeps
        st = direct_factor(cx, op, red_vec(w, n).TB, w.err);
        if (!st) st = direct_solve(cx, op, red_vec(w, n).R);
      } else {
        st = pcg_run<OP, RED>(cx, op, w, rho, prm.tolpcg, prm.mxiterpcg, ro.rhs2, ro.rty, ro.yty, &its);
      }
      pcg_total += its;
      nmat += 2 * its;
      if (st) {
        status = st;
        break;
      }
      FStepT<RED> fs;
      fs.Z = Z;
      fs.S = S;
      fs.TI = w.TI;
      fs.X = RED ? w.R : w.X;
      if constexpr (DIRECT) fs.Xr = op.y;
      else fs.Xr = red_vec(w, n).X;
      fs.DZ = w.DZ;
      fs.DS = w.DS;
      fs.sigma = sigma;
      fs.mu = mu;
      fs.corr = 0;
      fs.aPp = fs.aDp = 0.0;
      op_step_target(op, w, 1);
      run_A(cx, op, fs, kS, w.partA);
      op_step_target(op, w, 0);
      if (team_barrier(cx.t)) {
        status = ST_ABORTED;
        break;
      }
      double rs[2];
      reduce_items<2, red_unroll<OP>()>(kS, w.partA, op.nA(), rs, cx.red);
      aP = fmin(1.0, prm.eta * rs[0]);
      aD = fmin(1.0, prm.eta * rs[1]);
      if (aP <= prm.alpha_tilde || aD <= prm.alpha_tilde) {
        // corrector: residuals at the trial point with sigma3, same H and P
        ResOut rc = residual_rhs<OP, RED>(cx, op, w, Z, S, prm, RA_TRIAL, aP, aD, tau, sigma, prm.sigma3, 1, rho);
        nmat += 2;
        if (rc.status) {
          status = rc.status;
          break;
        }
        if constexpr (DIRECT) st = direct_solve(cx, op, red_vec(w, n).R);  // same factorisation
        else st = pcg_run<OP, RED>(cx, op, w, rho, prm.tolpcg, prm.mxiterpcg, rc.rhs2, rc.rty, rc.yty, &its);
        pcg_total += its;
        nmat += 2 * its;
        if (st) {
          status = st;
          break;
        }
        fs.sigma = prm.sigma3;
        fs.mu = rc.zs / (2.0 * (double)n);
        fs.corr = 1;
        fs.aPp = aP;
        fs.aDp = aD;
        op_step_target(op, w, 1);
        run_A(cx, op, fs, kS, w.partA);
        op_step_target(op, w, 0);
        if (team_barrier(cx.t)) {
          status = ST_ABORTED;
          break;
        }
        reduce_items<2, red_unroll<OP>()>(kS, w.partA, op.nA(), rs, cx.red);
        aP = fmin(1.0, prm.eta * rs[0]);
        aD = fmin(1.0, prm.eta * rs[1]);
        ++ncorr;
      }
      if (aP < prm.step_min && aD < prm.step_min) {
        status = ST_STEP_UNDERFLOW;
        break;
      }
      mode = RA_STEP;
      aP_prev = aP;
      aD_prev = aD;
      ++k;
    }
    // x = u - v
    FOut fo;
    fo.Z = Z;
    fo.x = a.x + d.n_off;
    const int kO[1] = {0};
    run_E(cx, n, fo, kO, w.partS);
  }
  if (cx.t.rank == 0 && threadIdx.x == 0) {
    DevInfo inf;
    inf.status = status;
    inf.ipm_iters = k - 1;
    inf.pcg_iters = pcg_total;
    inf.correctors = ncorr;
    inf.nmat = nmat;
    inf.rel_gap = relgap;
    inf.mu = mu;
    inf.primal_obj = primal;
    inf.dual_obj = dual;
    inf.rho = rho;
    a.info[ii] = inf;
  }
}

// Forward product y = A d after a pass A that left d in the operator's
// buffers: dense writes y directly; the partial DCT writes the spectral
// coefficients (pass B) and then gathers the sampled rows.
__device__ __forceinline__ void op_forward_out(Ctx& cx, OpDense& op, const TeamWS& w, double* out) {
  run_B<OpDense>(cx, op, DB_OUT, w.partB, out);
}
__device__ __forceinline__ void op_forward_gather(Ctx&, OpDense&, const TeamWS&, double*) {}
__device__ __forceinline__ void op_forward_out(Ctx& cx, OpPdct& op, const TeamWS& w, double*) {
  run_B<OpPdct>(cx, op, PB_FWDOUT, w.partB, nullptr);
}
template <class OP>
__device__ __forceinline__ void forward_gather_rows(Ctx& cx, OP& op, const TeamWS& w, double* out) {
  const long nthr = (long)cx.t.size * MF_THREADS;
  for (long i = (long)cx.t.rank * MF_THREADS + threadIdx.x; i < op.m; i += nthr)
    out[i] = w.XS[op.coef_pos(op.rows[i])];
}
__device__ __forceinline__ void op_forward_gather(Ctx& cx, OpPdct& op, const TeamWS& w, double* out) {
  forward_gather_rows(cx, op, w, out);
}
__device__ __forceinline__ void op_forward_out(Ctx& cx, OpWht& op, const TeamWS& w, double*) {
  run_B<OpWht>(cx, op, WB_FWDOUT, w.partB, nullptr);
}
__device__ __forceinline__ void op_forward_gather(Ctx& cx, OpWht& op, const TeamWS& w, double* out) {
  forward_gather_rows(cx, op, w, out);
}

// Adjoint: (Theta^{-1} + F F^T) w = [g; -g] at the stored state, then
// grad_b = A (w_u - w_v), grad_tau = -1^T w.
template <class OP, bool RED>
__device__ __forceinline__ void backward_instance(Ctx& cx, const KArgs& a, int ii, char* lds) {
  const InstDesc d = a.inst[ii];
  const TeamWS w = make_ws(a, cx.t.id);
  const DevParams& prm = a.prm;
  OP op;
  make_op(op, a, d, w, lds, cx.t.size);
  const long n = d.n;
  const double2* Z = (const double2*)(a.state + 4 * d.n_off);
  const double2* S = (const double2*)(a.state + 4 * d.n_off + 2 * d.n);
  int status = 0, its = 0, capped = 0;
  double rho = prm.rho, gtau = 0.0;
  int st = op_setup(cx, op, a, w, 0);
  if (st) status = st;
  if (!st && !(prm.rho > 0.0)) {
    int ab = 0;
    rho = op_rho(cx, op, w, ab);
    if (ab) st = status = ST_ABORTED;
  }
  if (!st) {
    FBwdInitT<RED> fi;
    fi.v = red_vec(w, n);
    fi.Z = Z;
    fi.S = S;
    fi.gx = a.grad_x + d.n_off;
    fi.TI = w.TI;
    fi.R = w.R;
    fi.X = w.X;
    fi.rho = rho;
    const int kI[3] = {0, 0, 0};
    run_A(cx, op, fi, kI, w.partA);
    if (team_barrier(cx.t)) st = ST_ABORTED;
    double pI[3];
    reduce_items<3, red_unroll<OP>()>(kI, w.partA, op.nA(), pI, cx.red);
    if (!st)
      st = pcg_run<OP, RED>(cx, op, w, rho, prm.tolpcg_adj, prm.mxiterpcg_adj, pI[1], pI[0], pI[2], &its, &capped);
    status = st;
    if (!st) {
      FBwdGatherT<RED> fg;
      fg.W = w.X;
      fg.TI = w.TI;
      fg.R = w.R;
      fg.Xr = red_vec(w, n).X;
      const int kG[1] = {0};
      run_A(cx, op, fg, kG, w.partA);
      if (team_barrier(cx.t)) status = ST_ABORTED;
      double pG[1];
      reduce_items<1, red_unroll<OP>()>(kG, w.partA, op.nA(), pG, cx.red);
      gtau = -pG[0];
      if (!status) {
        op_forward_out(cx, op, w, a.grad_b + d.m_off);
        if (team_barrier(cx.t)) status = ST_ABORTED;
        if (!status) op_forward_gather(cx, op, w, a.grad_b + d.m_off);
      }
      // the adjoint system was not solved to its tolerance: the gradients
      // are those of the last PCG iterate, flagged by the status
      if (!status && capped) status = ST_PCG_MAXITER;
    }
  }
  if (status && status != ST_PCG_MAXITER) {
    // no gradient: NaN in every output of the instance
    const long nthr = (long)cx.t.size * MF_THREADS;
    double* gb = a.grad_b + d.m_off;
    for (long i = (long)cx.t.rank * MF_THREADS + threadIdx.x; i < d.m; i += nthr) gb[i] = __builtin_nan("");
    gtau = __builtin_nan("");
  }
  if (cx.t.rank == 0 && threadIdx.x == 0) {
    a.grad_tau[ii] = gtau;
    DevInfo inf;
    inf.status = status;
    inf.ipm_iters = 0;
    inf.pcg_iters = its;
    inf.correctors = 0;
    inf.nmat = 2L * its + 2;
    inf.rel_gap = 0.0;
    inf.mu = 0.0;
    inf.primal_obj = 0.0;
    inf.dual_obj = 0.0;
    inf.rho = rho;
    a.info[ii] = inf;
  }
}
