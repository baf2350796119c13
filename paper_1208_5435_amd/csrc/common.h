// Shared device-side building blocks of the mfIPM kernels (gfx950, wave64).
// Workgroups are 512 threads (8 waves); reduction scratch in LDS holds
// MF_RED_DOUBLES doubles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MF_THREADS 512
#define MF_WAVES (MF_THREADS / 64)
#define MF_MAXK 6  // partial-sum slots per pass
#define MF_RED_DOUBLES (MF_WAVES * MF_MAXK + MF_MAXK)

// Status / flag values shared with the host driver.
enum {
  ST_CONVERGED = 0,
  ST_MAXITER = 1,
  ST_PCG_BREAKDOWN = 2,
  ST_NONFINITE = 3,
  ST_STEP_UNDERFLOW = 4,
  ST_ABORTED = 5,
  ST_DEVICE_CHECK = 6,
  ST_PCG_MAXITER = 7,  // adjoint only: PCG cap reached before its tolerance
};

struct cplx {
  double x, y;
};

// A store of an 8- or 16-byte element that writes through the XCD's L2 to
// memory (device scope, cache policy sc1), for data that workgroups on other
// XCDs read after the next team barrier: lines written this way are not dirty
// in the L2 when the barrier's release writes the L2 back, which keeps that
// write-back short.  base must be the same for the whole wave (it forms a
// buffer descriptor); idx * sizeof(T) < 2^31.
typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef int mf_v2i __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ void st_wt(T* base, long idx, const T& v) {
  static_assert(sizeof(T) == 16 || sizeof(T) == 8, "8- or 16-byte elements");
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, 0x7fffffff, 0x00020000);
  if constexpr (sizeof(T) == 16)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(mf_v4i, v), r, (int)(idx * 16), 0, 16 /* sc1 */);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(mf_v2i, v), r, (int)(idx * 8), 0, 16 /* sc1 */);
}
// The same or a plain store, as wt says (uniform over the wave).
template <class T>
__device__ __forceinline__ void st_sel(T* base, long idx, const T& v, int wt) {
  if (wt) st_wt(base, idx, v);
  else base[idx] = v;
}

__device__ __forceinline__ cplx mkc(double a, double b) { return cplx{a, b}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cconj(cplx a) { return cplx{a.x, -a.y}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.x * s, a.y * s}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by sign*i (sign = +1 or -1)
__device__ __forceinline__ cplx cmul_si(cplx a, int sign) {
  return sign > 0 ? cplx{-a.y, a.x} : cplx{a.y, -a.x};
}

// Roots of unity T(e) = exp(-2 pi i e / M) from two tables:
// T(e) = hi[e >> lo_bits] * lo[e & (2^lo_bits - 1)].  Tables are built on the
// host in extended precision and copied to LDS once per instance.
// `scale_shift` maps an instance's own resolution (4 n) onto the table
// resolution (4 n_max).
struct Twiddle {
  const cplx* lo;
  const cplx* hi;
  int lo_bits;
  int scale_shift;
  __device__ __forceinline__ cplx get(int e) const {  // e < 2^22
    e <<= scale_shift;
    cplx a = hi[e >> lo_bits];
    cplx b = lo[e & ((1 << lo_bits) - 1)];
    return cmul(a, b);
  }
  // exp(sign * 2 pi i e / M)
  __device__ __forceinline__ cplx get(int e, int sign) const {
    cplx t = get(e);
    return sign < 0 ? t : cconj(t);
  }
};

// ---------------------------------------------------------------------------
// Teams: groups of workgroups that cooperate on one instance.  Every
// workgroup of a team passes the same sequence of barriers because all
// control decisions are taken from identical, deterministically reduced
// values.
//
// The barrier is two-level and follows the chip's cache structure: the
// workgroups of a team that run on one XCD (accelerator complex die, one L2
// each) form a group.  A workgroup waits until its own global stores are
// complete in its XCD's L2 and arrives on its group's counter; the group's
// last arrival writes that L2 back once for the whole group (agent-scope
// release) and arrives on the top counter; the last top arrival publishes the
// generation in a release word on which everyone waits, then acquires
// (invalidating its L2 and L1 view).  One write-back per XCD instead of one
// per workgroup is what makes the release side cheap.
//
// This relies on the hardware, not on the C++/HIP memory model (in which a
// relaxed counter increment does not carry another workgroup's stores): the
// LLVM AMDGPU backend's memory-model description for the GFX942 family
// (AMDGPUUsage, "Memory Model GFX942", which gfx950 follows) implements an
// agent-scope release as "s_waitcnt vmcnt(0)" followed by "buffer_wbl2 sc1",
// and buffer_wbl2 writes back every dirty line of the L2 of the XCD that
// executes it, not only the issuing wave's; an agent-scope acquire is
// "buffer_inv sc1", which invalidates that XCD's L2 and the CU's L1.  Each
// member of a group has its stores complete in the shared L2 (its own
// s_waitcnt) before its arrival is counted, so the last arrival's write-back
// covers them.  Counters only grow
// (targets are generation * count), so nothing is reset between barriers.
// Every wait is bounded in wall-clock time: past the bound a global abort flag
// is raised, later barriers return at once and the solver loops stop, so the
// grid always drains.
//
// Control block layout (unsigned long long words):
//   [0] release word, [16] top counter, [32 + 16 x] counter of the group on
//   XCD x (x < 16), [MF_CTL_REG_WORD + x] registration count of XCD x,
//   [MF_CTL_REG_WORD + 16] registration total.
// ---------------------------------------------------------------------------
#define MF_MAX_XCD 16
#define MF_MAX_TEAM 1024  // largest team (workgroups per instance)
#define MF_CTL_REG_WORD 1296     // registration counters (one-time, after the group counters)
#define MF_CTL_SLOT_BYTES 10240  // byte offset of the queue slot in a team control block
#define MF_CTL_ERR_BYTES 10304   // byte offset of the input-check flag
#define MF_CTL_BYTES 12288       // bytes of one team control block

struct Team {
  int id;
  int rank;
  int size;
  unsigned long long* ctl;
  unsigned long long gen;
  int* abort_flag;
  unsigned long long spin_ticks;  // bound on one wait, in wall-clock ticks
  int xcd;                        // XCD this workgroup runs on
  int gsize;                      // workgroups of the team on that XCD
  int ngroups;                    // XCDs the team occupies
};

__device__ __forceinline__ int ld_flag(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hardware id of the XCD executing this wave (HW_REG_XCC_ID, bits 3:0).
__device__ __forceinline__ int hw_xcd_id() { return __builtin_amdgcn_s_getreg((15 << 11) | 20) & (MF_MAX_XCD - 1); }

// Spins (thread 0) until *p >= target; returns nonzero on abort or timeout.
__device__ __forceinline__ int spin_ge(unsigned long long* p, unsigned long long target, Team& t) {
  const unsigned long long t0 = wall_clock64();
  unsigned iter = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if ((++iter & 255u) == 0) {
      if (ld_flag(t.abort_flag)) return 1;
      if (wall_clock64() - t0 > t.spin_ticks) {
        __hip_atomic_store(t.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 1;
      }
    }
  }
  return 0;
}

// One-time set-up of the barrier groups: every workgroup registers its XCD,
// waits for the whole team, then reads its group's size and the number of
// groups.  The workgroup's rank is then renumbered XCD by XCD (the groups in
// XCD order, each in registration order), so that consecutive work items,
// which touch neighbouring memory, run on workgroups sharing one L2.  Every
// pass keeps its partial sums per item, so results do not depend on this
// numbering.  Returns nonzero if the run was aborted.
__device__ __forceinline__ int team_init(Team& t) {
  __shared__ int s_init[4];
  t.gen = 0;
  t.xcd = hw_xcd_id();
  if (threadIdx.x == 0) {
    unsigned long long* reg = t.ctl + MF_CTL_REG_WORD;
    const unsigned long long pos =
        __hip_atomic_fetch_add(reg + t.xcd, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_fetch_add(reg + MF_MAX_XCD, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ab = spin_ge(reg + MF_MAX_XCD, (unsigned long long)t.size, t);
    int ng = 0, before = 0;
    for (int x = 0; x < MF_MAX_XCD; ++x) {
      const int c = (int)__hip_atomic_load(reg + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ng += c > 0;
      if (x < t.xcd) before += c;
    }
    s_init[0] = ab;
    s_init[1] = (int)__hip_atomic_load(reg + t.xcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_init[2] = ng;
    s_init[3] = before + (int)pos;
  }
  __syncthreads();
  const int ab = s_init[0];
  t.gsize = s_init[1];
  t.ngroups = s_init[2];
  if (!ab) t.rank = s_init[3];
  __syncthreads();
  return ab;
}

// Returns nonzero if the run was aborted.
__device__ __forceinline__ int team_barrier(Team& t) {
  __shared__ int s_abort;
  // Every wave waits until its own global stores are complete in L2 before
  // the workgroup barrier, so the group's write-back below covers them.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  t.gen += 1;
  if (t.size == 1) {
    // A one-workgroup team has nothing to publish: its waves share the CU's
    // L1, which is coherent within the workgroup (no agent-scope release and
    // acquire, so no write-back of the XCD's L2 at every barrier).
    if (threadIdx.x == 0) s_abort = ld_flag(t.abort_flag);
    __syncthreads();
    return s_abort;
  }
  if (threadIdx.x == 0) {
    int ab = ld_flag(t.abort_flag);
    unsigned long long* rel = t.ctl;
    const unsigned long long old =
        __hip_atomic_fetch_add(t.ctl + 32 + 16 * t.xcd, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == t.gen * (unsigned long long)t.gsize) {
      // last of this XCD's group: every member's stores are in this L2
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned long long old2 =
          __hip_atomic_fetch_add(t.ctl + 16, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old2 + 1 == t.gen * (unsigned long long)t.ngroups)
        __hip_atomic_store(rel, t.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!ab) ab = spin_ge(rel, t.gen, t);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_abort = ab;
  }
  __syncthreads();
  return s_abort;
}

// A workgroup's view of its team during one instance.
struct Ctx {
  Team t;
  double* red;  // LDS reduction scratch (MF_RED_DOUBLES doubles)
};

// ---------------------------------------------------------------------------
// Deterministic reductions.  kind: 0 = sum, 1 = max, 2 = min.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rop(int kind, double a, double b) {
  if (kind == 0) return a + b;
  if (kind == 1) return fmax(a, b);
  return fmin(a, b);
}
__device__ __forceinline__ double rid(int kind) {
  return kind == 0 ? 0.0 : (kind == 1 ? -__builtin_inf() : __builtin_inf());
}

__device__ __forceinline__ double wave_reduce(int kind, double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = rop(kind, v, __shfl_xor(v, off, 64));
  return v;
}

// Reduce K per-thread values over the workgroup; thread 0 gets the results in
// out[] (registers of thread 0).  All threads must call.
template <int K>
__device__ __forceinline__ void wg_reduce(const int* kinds, double (&v)[K], double* lds_scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = wave_reduce(kinds[j], v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) lds_scratch[wave * MF_MAXK + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double a = lds_scratch[j];
      for (int w = 1; w < MF_WAVES; ++w) a = rop(kinds[j], a, lds_scratch[w * MF_MAXK + j]);
      v[j] = a;
    }
  }
  __syncthreads();
}

// Reduce per-item partials part[item * MF_MAXK + j] over items [0, nitems) in
// a fixed order; every thread of the workgroup receives the K results.  Lane
// l folds items l, l + 64, l + 128, ... in that order; the loads of RU such
// items are issued together before they are folded.  RU = 4 lets a team of a
// few hundred workgroups pay one memory round trip here instead of one per
// item, at the price of 4 K more live registers in the calling code (the
// operators whose teams are that large take it; the others keep RU = 1).
template <int K, int RU = 1>
__device__ __forceinline__ void reduce_items(const int* kinds, const double* part, int nitems, double (&res)[K],
                                    double* lds_scratch) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double a[K];
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] = rid(kinds[j]);
    for (int it0 = lane; it0 < nitems; it0 += 64 * RU) {
      double v[RU][K];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int it = it0 + 64 * u;
#pragma unroll
        for (int j = 0; j < K; ++j) v[u][j] = it < nitems ? part[(long)it * MF_MAXK + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (it0 + 64 * u < nitems) {
#pragma unroll
          for (int j = 0; j < K; ++j) a[j] = rop(kinds[j], a[j], v[u][j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] = wave_reduce(kinds[j], a[j]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) lds_scratch[MF_WAVES * MF_MAXK + j] = a[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) res[j] = lds_scratch[MF_WAVES * MF_MAXK + j];
  __syncthreads();
}

// The 2x2 block preconditioner of the reduced Newton system,
// P_i = [[tu + rho, -rho], [-rho, tv + rho]] (tu, tv = Theta^{-1} entries);
// returns P_i^{-1} r.
__device__ __forceinline__ void precond_apply(double tu, double tv, double rho, double ru, double rv,
                                              double& yu, double& yv) {
  const double det = tu * tv + rho * (tu + tv);
  yu = ((tv + rho) * ru + rho * rv) / det;
  yv = (rho * ru + (tu + rho) * rv) / det;
}
