// mfipm.hip -- persistent HIP kernels and the C ABI of the matrix-free IPM
// solver for l1-regularised least squares (declared in include/mfipm.h).
//
// One cooperative launch per call.  The grid is split into teams of
// workgroups; each team takes instances from a device queue (host order:
// largest first) and runs the whole IPM of one instance -- residuals, PCG,
// step lengths, corrector, update -- with team barriers between passes.  The
// host only reads the per-instance reports after the kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/mfipm.h"
#include "ipm.h"
#include "lockstep.h"

static_assert(sizeof(DevParams) == sizeof(mfipm_params), "params mirror");
static_assert(sizeof(DevInfo) == sizeof(mfipm_info), "info mirror");
static_assert(DC_LDS_BYTES <= (size_t)DN_FUSED_MAXN * sizeof(double2), "direct staging fits the dense LDS");

// ------------------------------------------------------------------------
// kernels
// ------------------------------------------------------------------------
template <class OP, int BWD, bool RED>
__global__ void __launch_bounds__(MF_THREADS) k_mfipm(KArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_dyn[];
  __shared__ double red[MF_RED_DOUBLES];
  Ctx cx;
  cx.red = red;
  cx.t.size = a.team_size;
  // Teams are interleaved over the grid (workgroup b belongs to team
  // b mod num_teams): the workgroups are dealt to the XCDs round robin, so
  // with a multiple of 8 teams each team runs on one XCD and shares its L2.
  cx.t.id = blockIdx.x % a.num_teams;
  cx.t.rank = blockIdx.x / a.num_teams;
  cx.t.gen = 0;
  cx.t.abort_flag = a.abort_flag;
  cx.t.spin_ticks = a.spin_ticks;
  const TeamWS w = make_ws(a, cx.t.id);
  cx.t.ctl = w.bar;
  if (team_init(cx.t)) return;
  for (;;) {
    // the previous slot value has been read by every workgroup of the team
    if (team_barrier(cx.t)) break;
    if (cx.t.rank == 0 && threadIdx.x == 0) {
      const int q = __hip_atomic_fetch_add(a.queue_head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(w.slot, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (team_barrier(cx.t)) break;
    const int q = ld_flag(w.slot);
    if (q >= a.batch) break;
    const int ii = a.order[q];
    if constexpr (BWD) backward_instance<OP, RED>(cx, a, ii, lds_dyn);
    else solve_instance<OP, RED>(cx, a, ii, lds_dyn);
  }
}

// Clears `words` 64-bit words (control words of a call on the static
// scratch; a kernel rather than a memset node, so a captured call replays it).
__global__ void __launch_bounds__(256) k_zero_words(unsigned long long* p, long words) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (long)gridDim.x * blockDim.x) p[i] = 0ull;
}

// ------------------------------------------------------------------------
// Static device memory of the no-allocation entry point (mfipm_solve_noalloc).
// `scratch` replaces the caller's workspace; `tw_full` holds the roots of
// unity at the largest supported resolution (2^22 = 4 x 2^20: 2^11 low and
// 2^11 high entries), which serve every transform length through the
// resolution shift.  Each device that loads the library holds both until the
// process ends.  In host code these names are host-side stand-ins: only the
// per-device addresses from hipGetSymbolAddress may reach a kernel or a copy.
// ------------------------------------------------------------------------
#define MFIPM_NOALLOC_TW_LOG2 22
#define MFIPM_NOALLOC_TW_LO_BITS 11
static __device__ __align__(256) char scratch[MFIPM_NOALLOC_SCRATCH_BYTES];
static __device__ __align__(256) cplx tw_full[(1 << MFIPM_NOALLOC_TW_LO_BITS) +
                                              (1 << (MFIPM_NOALLOC_TW_LOG2 - MFIPM_NOALLOC_TW_LO_BITS))];

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------
// Kernel kinds: the four operator kinds, and the dense operator with the
// direct (Cholesky) Newton solve.
constexpr int kKindDirect = 4;
constexpr int kKinds = 5;
static_assert(kKindDirect == MFIPM_OP_PDST + 1 && kKinds == kKindDirect + 1, "kernel kinds follow the operator kinds");

struct mfipm_handle {
  mfipm_params prm;
  hipStream_t stream;
  int device;
  int num_cu;
  long long wall_khz;
  int req_wg, req_team, req_tile;
  hipEvent_t ev0, ev1;
  double last_ms;
  int occ[kKinds][2][2];     // [kernel kind][bwd][reduced] max resident workgroups per CU
  int occ_ls;                // the same for the lock-step kernel
  size_t scratch_lane[kKinds][2][2];  // [kernel kind][bwd][reduced] private bytes per lane
  // twiddle tables (device, owned by the handle), one per table resolution
  cplx* tw[32];
  // pinned host staging for the per-call uploads and read-backs
  char* pinned;
  size_t pinned_bytes;
  // this device's static scratch and full twiddle table (device addresses),
  // or null when their set-up failed
  char* na_scratch;
  const cplx* na_tw;
};

// Upper bound on private (scratch) memory of one dispatch: all workgroups of a
// cooperative launch must get their scratch at once.
constexpr size_t kMaxDispatchScratch = (size_t)96 << 20;

namespace {

constexpr size_t kAlign = 256;
// the DCT-II and DST-II rows share one kernel (the DST through a sign flip
// of the input and output and reversed coefficient indices)
inline bool dct_family(int k) { return k == MFIPM_OP_PDCT || k == MFIPM_OP_PDST; }
// Cap on the direct variant's per-team matrices (A^T A and M) of one call.
constexpr size_t kDirectBudget = (size_t)32 << 30;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int check_params(const mfipm_params* p) {
  if (!p) return MFIPM_ERR_INVALID_ARG;
  if (!(p->tol > 0) || p->maxiters < 1 || !(p->tolpcg > 0) || p->mxiterpcg < 1) return MFIPM_ERR_INVALID_ARG;
  if (!(p->eta > 0 && p->eta <= 1) || !(p->z0 > 0) || !(p->s0 > 0)) return MFIPM_ERR_INVALID_ARG;
  if (!(p->tolpcg_adj > 0) || p->mxiterpcg_adj < 1 || !(p->step_min >= 0)) return MFIPM_ERR_INVALID_ARG;
  if (!(p->sigma1 >= 0 && p->sigma1 <= 1 && p->sigma2 >= 0 && p->sigma2 <= 1 && p->sigma3 >= 0 &&
        p->sigma3 <= 1))
    return MFIPM_ERR_INVALID_ARG;
  if (std::isnan(p->rho)) return MFIPM_ERR_INVALID_ARG;
  if (p->reduced != 0 && p->reduced != 1) return MFIPM_ERR_INVALID_ARG;
  if (p->direct != 0 && p->direct != 1) return MFIPM_ERR_INVALID_ARG;
  return MFIPM_OK;
}

inline int ilog2_host(long long v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}
inline bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

// Team region layout for the largest instance of a call.  pt_chunks: chunk
// capacity of the dense fused path's partial-product buffer.
size_t direct_team_bytes(long long n) {
  const size_t np = (size_t)((n + DC_NB - 1) / DC_NB * DC_NB);
  return 2 * align_up(np * np * sizeof(double)) + align_up(np * DC_NB * sizeof(double)) +
         align_up(np * sizeof(double));
}

TeamLayout team_layout(int op_kind, long long n, long long m, int pt_chunks) {
  TeamLayout L{};
  size_t off = 0;
  auto take = [&](long& field, size_t bytes) {
    field = (long)off;
    off += align_up(bytes);
  };
  const size_t v2 = (size_t)n * 2 * sizeof(double);
  take(L.X, v2);
  take(L.R, v2);
  take(L.P, v2);
  take(L.TI, v2);
  take(L.DZ, v2);
  take(L.DS, v2);
  take(L.Zs, v2);
  take(L.Ss, v2);
  L.DK = L.DM = L.DLi = L.DY = 0;
  if (op_kind == kKindDirect) {
    const size_t np = (size_t)((n + DC_NB - 1) / DC_NB * DC_NB);
    take(L.DK, np * np * sizeof(double));
    take(L.DM, np * np * sizeof(double));
    take(L.DLi, np * DC_NB * sizeof(double));
    take(L.DY, np * sizeof(double));
  }
  if (op_kind == MFIPM_OP_DENSE || op_kind == kKindDirect) {
    take(L.D, (size_t)n * sizeof(double));
    take(L.Yv, (size_t)m * sizeof(double));
    L.pt_chunks = n <= DN_FUSED_MAXN ? pt_chunks : 0;
    take(L.PT, (size_t)L.pt_chunks * (size_t)n * sizeof(double));
    take(L.Dp0, (size_t)n * sizeof(double));  // previous/current direction,
    take(L.Dp1, (size_t)n * sizeof(double));  // alternating per PCG iteration
    take(L.Dx0, (size_t)n * sizeof(double));  // current / next x = u - v
    take(L.Dx1, (size_t)n * sizeof(double));
    take(L.Dd, (size_t)n * sizeof(double));   // step direction dz_u - dz_v
    L.Y1 = L.Y1p = L.Y2 = L.Yx = L.Yd = L.mask = L.bt = L.XS = 0;
  } else {
    L.D = L.Yv = L.PT = L.Dp0 = L.Dp1 = L.Dx0 = L.Dx1 = L.Dd = 0;
    L.pt_chunks = 0;
    take(L.Y1, (size_t)n * sizeof(double));  // n/2 complex
    take(L.Y1p, (size_t)n * sizeof(double));  // transform of the direction
    take(L.Yx, (size_t)n * sizeof(double));   // transform of x = u - v
    take(L.Yd, (size_t)n * sizeof(double));   // transform of the step direction
    take(L.Y2, (size_t)n * sizeof(double));
    take(L.mask, (size_t)n);
    take(L.bt, (size_t)n * sizeof(double));
    take(L.XS, (size_t)n * sizeof(double));
  }
  const size_t items = (size_t)(n + m + 64);
  const size_t pb = items * MF_MAXK * sizeof(double);
  take(L.partA, pb);
  take(L.partB, pb);
  take(L.partC, pb);
  take(L.partS, pb);
  L.stride = (long)off;
  return L;
}

// Workspace: [control: global words (256 B) + one block per team]
//            [reports][descriptors + launch order][team regions]
struct GlobalLayout {
  size_t ctl, info, inst, order, teams, total;
  int lo_bits;
  long long hi_count;
};

GlobalLayout global_layout(int op_kind, long long n_max, int batch, int teams, const TeamLayout& tl) {
  GlobalLayout g{};
  size_t off = 0;
  g.ctl = off;
  off += align_up(256 + (size_t)teams * MF_CTL_BYTES);
  g.info = off;
  off += align_up((size_t)batch * sizeof(DevInfo));
  g.inst = off;
  g.order = off + (size_t)batch * sizeof(InstDesc);
  off += align_up((size_t)batch * (sizeof(InstDesc) + sizeof(int)));
  g.lo_bits = 0;
  g.hi_count = 0;
  if (dct_family(op_kind)) {
    const int lm = ilog2_host(n_max) + 2;  // table resolution 4 n_max
    g.lo_bits = (lm + 1) / 2;
    g.hi_count = 1LL << (lm - g.lo_bits);
  }
  g.teams = off;
  off += (size_t)teams * (size_t)tl.stride;
  g.total = off;
  return g;
}

// Chunk capacity of the dense fused path: one chunk per workgroup of a
// single-instance team (up to the resident grid), at most 64 for batches.
int pt_chunks_for(const mfipm_handle* h, int bwd, int batch, long long m_max, int red) {
  const long long blocks = (m_max + DN_FB - 1) / DN_FB;
  const long long gmax = std::max(1, h->occ[MFIPM_OP_DENSE][bwd][red] * h->num_cu);
  const long long cap = batch == 1 ? gmax : 64;
  return (int)std::max(1LL, std::min(blocks, cap));
}

int max_teams_bound(const mfipm_handle* h, int op_kind, int bwd, int batch, int red, long long n_max) {
  const int gmax = std::max(1, h->occ[op_kind][bwd][red] * h->num_cu);
  int bound = std::max(1, std::min(batch, gmax));
  if (op_kind == kKindDirect) {
    const long long cap = (long long)(kDirectBudget / direct_team_bytes(n_max));
    bound = (int)std::max(1LL, std::min<long long>(bound, cap));
  }
  return bound;
}

template <class OP, int BWD, bool RED>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_mfipm<OP, BWD, RED>);
}
template <bool RED>
const void* pick_kernel_r(int op_kind, int bwd) {
  if (op_kind == kKindDirect) return kernel_ptr<OpDenseDirect, 0, true>();  // forward only
  if (op_kind == MFIPM_OP_DENSE) return bwd ? kernel_ptr<OpDense, 1, RED>() : kernel_ptr<OpDense, 0, RED>();
  if (op_kind == MFIPM_OP_WHT) return bwd ? kernel_ptr<OpWht, 1, RED>() : kernel_ptr<OpWht, 0, RED>();
  return bwd ? kernel_ptr<OpPdct, 1, RED>() : kernel_ptr<OpPdct, 0, RED>();
}
const void* pick_kernel(int op_kind, int bwd, int red) {
  return red ? pick_kernel_r<true>(op_kind, bwd) : pick_kernel_r<false>(op_kind, bwd);
}
// Dynamic LDS: dense reduction scratch; partial DCT tile + twiddle tables
// (lo_bits / hi entries of the call, or the largest supported, n = 2^20).
constexpr int kPdctMaxLog2N = 20;
size_t dyn_lds(int op_kind, int lo_bits = -1, long long hi_count = 0) {
  if (op_kind == MFIPM_OP_WHT) return (size_t)WH_TILE * sizeof(double);
  if (op_kind == MFIPM_OP_DENSE || op_kind == kKindDirect)
    return (size_t)(MF_WAVES * DN_RBMAX + DN_RG * DN_CB) * sizeof(double) + DN_FUSED_MAXN * sizeof(double2);
  if (lo_bits < 0) {
    const int lm = kPdctMaxLog2N + 2;
    lo_bits = (lm + 1) / 2;
    hi_count = 1LL << (lm - lo_bits);
  }
  return (size_t)PD_TILE_LDS * sizeof(cplx) + (((size_t)1 << lo_bits) + (size_t)hi_count) * sizeof(cplx) +
         PD_MASK_BYTES;
}

void fill_twiddles(std::vector<cplx>& lo, std::vector<cplx>& hi, int lm, int lo_bits) {
  // T(e) = exp(-2 pi i e / 2^lm) = hi[e >> lo_bits] * lo[e & mask]
  const long double two_pi = 6.283185307179586476925286766559005768L;
  const long double M = (long double)(1LL << lm);
  lo.resize((size_t)1 << lo_bits);
  hi.resize((size_t)1 << (lm - lo_bits));
  for (size_t e = 0; e < lo.size(); ++e) {
    const long double ang = two_pi * (long double)e / M;
    lo[e] = cplx{(double)cosl(ang), (double)-sinl(ang)};
  }
  for (size_t e = 0; e < hi.size(); ++e) {
    const long double ang = two_pi * (long double)(e << lo_bits) / M;
    hi[e] = cplx{(double)cosl(ang), (double)-sinl(ang)};
  }
}

// Device twiddle tables of resolution 2^lm (lo part then hi part), built on
// the host once per resolution and kept by the handle.
const cplx* twiddle_tables(mfipm_handle* h, int lm, int lo_bits) {
  if (lm < 0 || lm >= 32) return nullptr;
  if (h->tw[lm]) return h->tw[lm];
  std::vector<cplx> lo, hi;
  fill_twiddles(lo, hi, lm, lo_bits);
  cplx* d = nullptr;
  if (hipMalloc(&d, (lo.size() + hi.size()) * sizeof(cplx)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, lo.data(), lo.size() * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d + lo.size(), hi.data(), hi.size() * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  h->tw[lm] = d;
  return d;
}

// Items of the widest pass of one instance (used to size a single team).
long long widest_pass(int op_kind, long long n, long long m, int tile) {
  if (op_kind == kKindDirect) {
    // tiles of the lower block triangle (the A^T A product and the first updates)
    const long long T = (n + DC_NB - 1) / DC_NB;
    return std::max(widest_pass(MFIPM_OP_DENSE, n, m, tile), T * (T + 1) / 2);
  }
  if (op_kind == MFIPM_OP_WHT) {
    // items of one column (pass A/C) or one row (pass B); at least one
    // workgroup per 4096 indices
    const int ln = ilog2_host(n);
    const long long N1 = 1LL << (ln / 2), N2 = n / N1;
    return std::max(std::max(N1, N2) / 4, std::max(1LL, n >> 12));
  }
  if (op_kind == MFIPM_OP_DENSE) {
    if (n <= DN_FUSED_MAXN) {
      // about 256 KiB of A per workgroup, at least 32 and at most one block each
      const long long blocks = (m + DN_FB - 1) / DN_FB;
      const long long want = std::max(32LL, (m * n * 8) >> 18);
      return std::max(1LL, std::min(blocks, want));
    }
    const int RB = tile > 0 ? std::min(tile, DN_RBMAX) : 8;
    return std::max((m + RB - 1) / RB, (n + DN_CB - 1) / DN_CB);
  }
  const int lh = ilog2_host(n) - 1;
  int l1 = tile > 0 ? tile : lh / 2;
  l1 = std::min(l1, 9);
  if (lh - l1 > 11) l1 = lh - 11;
  if (lh - l1 < 3) l1 = lh - 3;
  const long long N1 = 1LL << l1, N2 = 1LL << (lh - l1);
  return std::max(N1 / 2, N2 / 8);
}

struct Problem {
  int batch;
  int op_kind;
  int shared_op;
  const int64_t* n_off;
  const int64_t* m_off;
  const int64_t* a_off;
  const double* tau;  // host
  long long n_max, m_max;
};

int validate(const mfipm_handle* h, const Problem& P) {
  if (!h) return MFIPM_ERR_INVALID_ARG;
  if (P.batch < 1 || !P.n_off || !P.m_off) return MFIPM_ERR_INVALID_ARG;
  if (P.op_kind != MFIPM_OP_DENSE && P.op_kind != MFIPM_OP_PDCT && P.op_kind != MFIPM_OP_WHT &&
      P.op_kind != MFIPM_OP_PDST)
    return MFIPM_ERR_INVALID_ARG;
  if (P.op_kind == MFIPM_OP_DENSE && !P.shared_op && !P.a_off) return MFIPM_ERR_INVALID_ARG;
  for (int i = 0; i < P.batch; ++i) {
    const long long n = P.n_off[i + 1] - P.n_off[i];
    const long long m = P.m_off[i + 1] - P.m_off[i];
    if (n < 1 || m < 1 || P.n_off[i] < 0 || P.m_off[i] < 0) return MFIPM_ERR_INVALID_ARG;
    if (P.op_kind != MFIPM_OP_DENSE) {
      if (!is_pow2(n) || n < 64 || n > (1LL << kPdctMaxLog2N) || m > n) return MFIPM_ERR_INVALID_ARG;
    } else if (!P.shared_op && P.a_off[i + 1] - P.a_off[i] != n * m) {
      return MFIPM_ERR_INVALID_ARG;
    }
    if (P.shared_op && i > 0) {
      const long long n0 = P.n_off[1] - P.n_off[0], m0 = P.m_off[1] - P.m_off[0];
      if (n != n0 || m != m0) return MFIPM_ERR_INVALID_ARG;
    }
    if (P.tau && !(P.tau[i] > 0 && std::isfinite(P.tau[i]))) return MFIPM_ERR_INVALID_ARG;
  }
  return MFIPM_OK;
}

// Device addresses of the static scratch and twiddle table, looked up once
// per device (with that device current) and kept for the process.  The
// table is filled at the same time.
constexpr int kMaxDevices = 64;
struct NoallocDevice {
  std::once_flag once;
  int rc = MFIPM_ERR_HIP;
  char* scratch = nullptr;
  cplx* tw = nullptr;
  std::mutex call;  // no-allocation calls on one device run one at a time
};
NoallocDevice g_noalloc[kMaxDevices];

int noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return MFIPM_ERR_HIP;
  NoallocDevice& d = g_noalloc[dev];
  std::call_once(d.once, [&d] {
    void* sp = nullptr;
    void* tp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return;
    if (hipGetSymbolAddress(&tp, HIP_SYMBOL(tw_full)) != hipSuccess || !tp) return;
    std::vector<cplx> lo, hi;
    fill_twiddles(lo, hi, MFIPM_NOALLOC_TW_LOG2, MFIPM_NOALLOC_TW_LO_BITS);
    cplx* t = static_cast<cplx*>(tp);
    if (hipMemcpy(t, lo.data(), lo.size() * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t + lo.size(), hi.data(), hi.size() * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess)
      return;
    d.scratch = static_cast<char*>(sp);
    d.tw = t;
    d.rc = MFIPM_OK;
  });
  return d.rc;
}

#define HIP_TRY(expr)                      \
  do {                                     \
    if ((expr) != hipSuccess) return MFIPM_ERR_HIP; \
  } while (0)

// Where a call's device workspace and host transfers live.  Ordinary calls:
// the caller's workspace, the handle's pinned staging and the handle's
// twiddle tables.  No-allocation calls (tw_fixed set): the device's static
// scratch, a staging buffer on the host stack and the static full-resolution
// twiddle table -- nothing is allocated anywhere in the call.
struct Backing {
  char* ws;
  size_t ws_bytes;
  const cplx* tw_fixed;
};

// Shared launch path of solve (bwd = 0) and backward (bwd = 1).
int launch(mfipm_handle* h, const Problem& P, int bwd, const double* A, const int32_t* rows, const double* b,
           double* x, double* state, const double* grad_x, double* grad_b, double* grad_tau,
           const Backing& bk, mfipm_info* infos) {
  void* ws = bk.ws;
  const size_t ws_bytes = bk.ws_bytes;
  const bool noalloc = bk.tw_fixed != nullptr;
  int rc = validate(h, P);
  if (rc) return rc;
  if (!ws) return MFIPM_ERR_INVALID_ARG;
  if (P.op_kind == MFIPM_OP_DENSE && !A) return MFIPM_ERR_INVALID_ARG;
  if (P.op_kind != MFIPM_OP_DENSE && !rows) return MFIPM_ERR_INVALID_ARG;
  if (!bwd && (!b || !x)) return MFIPM_ERR_INVALID_ARG;
  if (bwd && !state) return MFIPM_ERR_NO_STATE;
  if (bwd && (!grad_x || !grad_b || !grad_tau)) return MFIPM_ERR_INVALID_ARG;

  // kernel kind: the forward solve with direct Newton solves is its own kernel
  int kind = P.op_kind;
  int red = h->prm.reduced;
  if (!bwd && h->prm.direct) {
    if (P.op_kind != MFIPM_OP_DENSE || P.n_max > DC_MAX_N) return MFIPM_ERR_INVALID_ARG;
    kind = kKindDirect;
    red = 1;  // the direct solve works on the n x n system
  }
  // launch shape
  if (h->occ[kind][bwd][red] < 1) return MFIPM_ERR_HIP;
  const int gmax = std::max(1, h->occ[kind][bwd][red] * h->num_cu);
  int team_size, num_teams;
  if (P.batch == 1) {
    long long want = h->req_wg > 0 ? h->req_wg : widest_pass(kind, P.n_max, P.m_max, h->req_tile);
    team_size = (int)std::max(1LL, std::min<long long>(want, gmax));
    num_teams = 1;
  } else {
    if (h->req_team > 0) team_size = std::min(h->req_team, gmax);
    else {
      team_size = std::max(1, gmax / P.batch);
      team_size = 1 << (31 - __builtin_clz((unsigned)team_size));
    }
    const int total = h->req_wg > 0 ? std::min(h->req_wg, gmax) : gmax;
    num_teams = std::max(1, std::min(P.batch, total / team_size));
  }
  if (team_size > MF_MAX_TEAM) team_size = MF_MAX_TEAM;
  const int teams_bound = max_teams_bound(h, kind, bwd, P.batch, red, P.n_max);
  if (num_teams > teams_bound) num_teams = teams_bound;
  // private memory of the whole grid within the dispatch limit: fewer teams,
  // then smaller ones
  const size_t lane_scr = h->scratch_lane[kind][bwd][red];
  if (lane_scr > 0) {
    const long long max_wg = (long long)(kMaxDispatchScratch / (lane_scr * MF_THREADS));
    if (max_wg < 1) return MFIPM_ERR_HIP;
    if ((long long)num_teams * team_size > max_wg) num_teams = (int)std::max(1LL, max_wg / team_size);
    if ((long long)num_teams * team_size > max_wg) team_size = (int)max_wg;
  }
  if (lane_scr * MF_THREADS * (size_t)(num_teams * team_size) > kMaxDispatchScratch) return MFIPM_ERR_HIP;

  const TeamLayout tl = team_layout(kind, P.n_max, P.m_max, pt_chunks_for(h, bwd, P.batch, P.m_max, red));
  GlobalLayout gl = global_layout(kind, P.n_max, P.batch, teams_bound, tl);
  if (ws_bytes < gl.total) return noalloc ? MFIPM_ERR_TOO_LARGE : MFIPM_ERR_WORKSPACE_TOO_SMALL;
  int tw_log2n_max = ilog2_host(P.n_max);
  if (noalloc && dct_family(P.op_kind)) {
    gl.lo_bits = MFIPM_NOALLOC_TW_LO_BITS;
    gl.hi_count = 1LL << (MFIPM_NOALLOC_TW_LOG2 - MFIPM_NOALLOC_TW_LO_BITS);
    tw_log2n_max = MFIPM_NOALLOC_TW_LOG2 - 2;
  }

  char* base = (char*)ws;
  // Staging (the previous call has synchronised): descriptors and the launch
  // order go up in one copy; reports and the abort flag come back into the
  // same buffer.  Pinned and owned by the handle, or on the stack for the
  // no-allocation entry point (single instance).
  const size_t desc_bytes = (size_t)P.batch * (sizeof(InstDesc) + sizeof(int));
  const size_t back_bytes = align_up((size_t)P.batch * sizeof(DevInfo)) + 256;
  const size_t need = std::max(desc_bytes, back_bytes);
  alignas(256) char stack_stage[1024];
  char* stage = stack_stage;
  if (noalloc) {
    if (need > sizeof(stack_stage)) return MFIPM_ERR_INVALID_ARG;
  } else {
    if (h->pinned_bytes < need) {
      if (h->pinned) (void)hipHostFree(h->pinned);
      h->pinned = nullptr;
      h->pinned_bytes = 0;
      if (hipHostMalloc((void**)&h->pinned, need, hipHostMallocDefault) != hipSuccess) return MFIPM_ERR_HIP;
      h->pinned_bytes = need;
    }
    stage = h->pinned;
  }
  char* desc = stage;
  InstDesc* inst = reinterpret_cast<InstDesc*>(desc);
  // launch order: largest instance first, ties by index (the staging buffer
  // holds it after the descriptors; std::sort needs no extra memory)
  int* order = reinterpret_cast<int*>(desc + (size_t)P.batch * sizeof(InstDesc));
  for (int i = 0; i < P.batch; ++i) {
    inst[i].n = P.n_off[i + 1] - P.n_off[i];
    inst[i].m = P.m_off[i + 1] - P.m_off[i];
    inst[i].n_off = P.n_off[i];
    inst[i].m_off = P.m_off[i];
    inst[i].a_off = (P.op_kind == MFIPM_OP_DENSE && !P.shared_op) ? P.a_off[i] : 0;
    inst[i].tau = P.tau ? P.tau[i] : 0.0;
    order[i] = i;
  }
  std::sort(order, order + P.batch, [&](int u, int v) {
    const double cu = (double)inst[u].n * (double)(P.op_kind == MFIPM_OP_DENSE ? inst[u].m : 1);
    const double cv = (double)inst[v].n * (double)(P.op_kind == MFIPM_OP_DENSE ? inst[v].m : 1);
    return cu > cv || (cu == cv && u < v);
  });
  hipStream_t s = h->stream;
  if (hipMemcpyAsync(base + gl.inst, desc, desc_bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return MFIPM_ERR_HIP;
  }
  // From here on the staging buffer may still be read by the copy engine:
  // every return waits for the stream first, so the next call can reuse it.
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(s);
    return code;
  };
  const cplx* tw = nullptr;
  if (dct_family(P.op_kind)) {
    tw = noalloc ? bk.tw_fixed : twiddle_tables(h, tw_log2n_max + 2, gl.lo_bits);
    if (!tw) return fail(MFIPM_ERR_HIP);
  }
  // zero the control words: queue head, abort flag, team barriers and slots
  const size_t ctl_bytes = 256 + (size_t)num_teams * MF_CTL_BYTES;
  if (noalloc) {
    const long words = (long)(ctl_bytes / sizeof(unsigned long long));
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<long>(64, (words + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(base + gl.ctl), words);
    if (hipGetLastError() != hipSuccess) return fail(MFIPM_ERR_HIP);
  } else if (hipMemsetAsync(base + gl.ctl, 0, ctl_bytes, s) != hipSuccess) {
    return fail(MFIPM_ERR_HIP);
  }

  KArgs a{};
  a.inst = (const InstDesc*)(base + gl.inst);
  a.order = (const int*)(base + gl.order);
  a.batch = P.batch;
  a.queue_head = (int*)(base + gl.ctl);
  a.abort_flag = (int*)(base + gl.ctl + 64);
  a.info = (DevInfo*)(base + gl.info);
  a.A = A;
  a.rows = rows;
  a.shared_op = P.shared_op;
  a.op_flip = P.op_kind == MFIPM_OP_PDST ? 1 : 0;
  a.b = b;
  a.x = x;
  a.state = state;
  a.grad_x = grad_x;
  a.grad_b = grad_b;
  a.grad_tau = grad_tau;
  std::memcpy(&a.prm, &h->prm, sizeof(DevParams));
  a.team_base = base + gl.teams;
  a.team_ctl = base + gl.ctl + 256;
  a.lay = tl;
  a.tw_lo = tw;
  a.tw_hi = tw ? tw + ((size_t)1 << gl.lo_bits) : nullptr;
  a.tw_lo_bits = gl.lo_bits;
  a.tw_log2n_max = tw_log2n_max;
  a.team_size = team_size;
  a.num_teams = num_teams;
  a.tile_param = h->req_tile;
  a.spin_ticks = (unsigned long long)h->wall_khz * 1000ull * 5ull;  // 5 s per wait

  void* args[] = {&a};
  const int grid = num_teams * team_size;
  if (hipEventRecord(h->ev0, s) != hipSuccess) return fail(MFIPM_ERR_HIP);
  if (hipLaunchCooperativeKernel(pick_kernel(kind, bwd, red), dim3(grid), dim3(MF_THREADS), args,
                                 (unsigned)dyn_lds(kind, gl.lo_bits, gl.hi_count), s) != hipSuccess)
    return fail(MFIPM_ERR_HIP);
  if (hipEventRecord(h->ev1, s) != hipSuccess) return fail(MFIPM_ERR_HIP);
  const DevInfo* dinf = reinterpret_cast<const DevInfo*>(stage);
  const int* ctl = reinterpret_cast<const int*>(stage + align_up((size_t)P.batch * sizeof(DevInfo)));
  if (hipMemcpyAsync(stage, base + gl.info, sizeof(DevInfo) * P.batch, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync((void*)ctl, base + gl.ctl, 128, hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(MFIPM_ERR_HIP);
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->last_ms = ms;
  rc = MFIPM_OK;
  for (int i = 0; i < P.batch; ++i) {
    if (dinf[i].status == ST_DEVICE_CHECK) rc = MFIPM_ERR_DEVICE_CHECK;
    if (infos) std::memcpy(&infos[i], &dinf[i], sizeof(mfipm_info));
  }
  if (ctl[16] != 0 && rc == MFIPM_OK) rc = MFIPM_ERR_HIP;  // abort flag (offset 64 B)
  return rc;
}

// ---- lock-step path: many signals sharing one dense A ----
// Batches of at least this many signals on one shared dense matrix take the
// lock-step path (unless a team size is requested).
constexpr int kLockstepMinBatch = 8;

struct LsLayout {
  size_t ctl, info, inst, st, mode, V, D, Y, Yp, T, part, total;
};

LsLayout ls_layout(long long n, long long m, int B) {
  LsLayout L{};
  size_t off = 0;
  auto take = [&](size_t& field, size_t bytes) {
    field = off;
    off += align_up(bytes);
  };
  take(L.ctl, 256 + MF_CTL_BYTES);
  take(L.info, (size_t)B * sizeof(DevInfo));
  take(L.inst, (size_t)B * sizeof(InstDesc));
  take(L.st, (size_t)B * sizeof(SigState));
  take(L.mode, (size_t)B * sizeof(int));
  take(L.V, (size_t)B * 8 * (size_t)n * sizeof(double2));
  take(L.D, (size_t)B * (size_t)n * sizeof(double));
  take(L.Y, (size_t)B * (size_t)m * sizeof(double));
  take(L.Yp, (size_t)LS_SPLIT * B * (size_t)m * sizeof(double));
  take(L.T, (size_t)B * (size_t)n * sizeof(double));
  take(L.part, (size_t)((m + 7) / 8 + 64) * MF_MAXK * sizeof(double));
  L.total = off;
  return L;
}

bool use_lockstep(const mfipm_handle* h, int op_kind, int shared_op, int batch) {
  return op_kind == MFIPM_OP_DENSE && shared_op && batch >= kLockstepMinBatch && !h->prm.direct &&
         batch <= LS_MAX_GROUPS * LS_TN && h->req_team <= 0 && !h->prm.reduced;
}

int launch_lockstep(mfipm_handle* h, const Problem& P, const double* A, const double* b, double* x, double* state,
                    void* ws, size_t ws_bytes, mfipm_info* infos) {
  int rc = validate(h, P);
  if (rc) return rc;
  if (!ws || !A || !b || !x) return MFIPM_ERR_INVALID_ARG;
  if (h->occ_ls < 1) return MFIPM_ERR_HIP;
  const int B = P.batch;
  const long long n = P.n_max, m = P.m_max;
  const LsLayout L = ls_layout(n, m, B);
  if (ws_bytes < L.total) return MFIPM_ERR_WORKSPACE_TOO_SMALL;
  const int gmax = h->occ_ls * h->num_cu;
  const int grid = std::max(1, std::min(h->req_wg > 0 ? h->req_wg : h->num_cu, gmax));
  char* base = (char*)ws;
  const size_t desc_bytes = (size_t)B * sizeof(InstDesc);
  const size_t back_bytes = align_up((size_t)B * sizeof(DevInfo)) + 256;
  const size_t need = std::max(desc_bytes, back_bytes);
  if (h->pinned_bytes < need) {
    if (h->pinned) (void)hipHostFree(h->pinned);
    h->pinned = nullptr;
    h->pinned_bytes = 0;
    if (hipHostMalloc((void**)&h->pinned, need, hipHostMallocDefault) != hipSuccess) return MFIPM_ERR_HIP;
    h->pinned_bytes = need;
  }
  InstDesc* inst = reinterpret_cast<InstDesc*>(h->pinned);
  for (int i = 0; i < B; ++i) {
    inst[i].n = P.n_off[i + 1] - P.n_off[i];
    inst[i].m = P.m_off[i + 1] - P.m_off[i];
    inst[i].n_off = P.n_off[i];
    inst[i].m_off = P.m_off[i];
    inst[i].a_off = 0;
    inst[i].tau = P.tau[i];
  }
  hipStream_t s = h->stream;
  if (hipMemcpyAsync(base + L.inst, inst, desc_bytes, hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return MFIPM_ERR_HIP;
  }
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(s);
    return code;
  };
  if (hipMemsetAsync(base + L.ctl, 0, 256 + MF_CTL_BYTES, s) != hipSuccess) return fail(MFIPM_ERR_HIP);
  LArgs a{};
  a.inst = (const InstDesc*)(base + L.inst);
  a.B = B;
  a.n = n;
  a.m = m;
  a.A = A;
  a.b = b;
  a.x = x;
  a.state = state;
  a.info = (DevInfo*)(base + L.info);
  std::memcpy(&a.prm, &h->prm, sizeof(DevParams));
  a.st = (SigState*)(base + L.st);
  a.mode = (int*)(base + L.mode);
  a.V = (double2*)(base + L.V);
  a.D = (double*)(base + L.D);
  a.Y = (double*)(base + L.Y);
  a.Yp = (double*)(base + L.Yp);
  a.T = (double*)(base + L.T);
  a.part = (double*)(base + L.part);
  a.abort_flag = (int*)(base + L.ctl + 64);
  a.ctl = (unsigned long long*)(base + L.ctl + 256);
  a.spin_ticks = (unsigned long long)h->wall_khz * 1000ull * 5ull;
  void* args[] = {&a};
  if (hipEventRecord(h->ev0, s) != hipSuccess) return fail(MFIPM_ERR_HIP);
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_mfipm_lockstep), dim3(grid), dim3(MF_THREADS),
                                 args, (unsigned)sizeof(GemmLDS), s) != hipSuccess)
    return fail(MFIPM_ERR_HIP);
  if (hipEventRecord(h->ev1, s) != hipSuccess) return fail(MFIPM_ERR_HIP);
  const DevInfo* dinf = reinterpret_cast<const DevInfo*>(h->pinned);
  const int* ctl = reinterpret_cast<const int*>(h->pinned + align_up((size_t)B * sizeof(DevInfo)));
  if (hipMemcpyAsync(h->pinned, base + L.info, sizeof(DevInfo) * B, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync((void*)ctl, base + L.ctl, 128, hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(MFIPM_ERR_HIP);
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->last_ms = ms;
  for (int i = 0; i < B; ++i)
    if (infos) std::memcpy(&infos[i], &dinf[i], sizeof(mfipm_info));
  return ctl[16] != 0 ? MFIPM_ERR_HIP : MFIPM_OK;
}

}  // namespace

// ------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------
extern "C" {

int mfipm_params_default(mfipm_params* p) {
  if (!p) return MFIPM_ERR_INVALID_ARG;
  p->tol = 1e-8;
  p->maxiters = 100;
  p->tolpcg = 1e-2;
  p->mxiterpcg = 200;
  p->sigma1 = 0.1;
  p->sigma2 = 0.5;
  p->sigma3 = 0.8;
  p->alpha_bar = 0.5;
  p->alpha_tilde = 0.1;
  p->eta = 0.995;
  p->rho = 0.0;
  p->z0 = 1.0;
  p->s0 = 1.0;
  p->tolpcg_adj = 1e-12;
  p->mxiterpcg_adj = 1000;
  p->step_min = 1e-14;
  p->reduced = 0;
  p->direct = 0;
  return MFIPM_OK;
}

int mfipm_create(mfipm_handle** hp, const mfipm_params* p, void* stream) {
  if (!hp) return MFIPM_ERR_INVALID_ARG;
  *hp = nullptr;
  mfipm_params prm;
  if (p) {
    if (check_params(p)) return MFIPM_ERR_INVALID_ARG;
    prm = *p;
  } else {
    mfipm_params_default(&prm);
  }
  mfipm_handle* h = new (std::nothrow) mfipm_handle();
  if (!h) return MFIPM_ERR_HIP;
  h->prm = prm;
  h->stream = (hipStream_t)stream;
  h->last_ms = -1.0;
  int wclk = 0;
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
      hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, h->device) != hipSuccess) {
    delete h;
    return MFIPM_ERR_HIP;
  }
  h->wall_khz = wclk > 0 ? wclk : 100000;
  for (int op = 0; op < kKinds; ++op)
    for (int bwd = 0; bwd < 2; ++bwd)
      for (int red = 0; red < 2; ++red) {
      int occ = 0;
      const void* k = pick_kernel(op, bwd, red);
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds(op)) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, MF_THREADS, dyn_lds(op)) != hipSuccess) {
        delete h;
        return MFIPM_ERR_HIP;
      }
      h->occ[op][bwd][red] = occ;  // 0: this kernel cannot be resident; calls that need it fail
      hipFuncAttributes fa;
      if (hipFuncGetAttributes(&fa, k) != hipSuccess) {
        delete h;
        return MFIPM_ERR_HIP;
      }
      h->scratch_lane[op][bwd][red] = fa.localSizeBytes;
      }
  {
    const void* k = reinterpret_cast<const void*>(&k_mfipm_lockstep);
    int occ = 0;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(GemmLDS)) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, MF_THREADS, sizeof(GemmLDS)) != hipSuccess) {
      delete h;
      return MFIPM_ERR_HIP;
    }
    h->occ_ls = occ;
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
    delete h;
    return MFIPM_ERR_HIP;
  }
  // the no-allocation entry point's static memory on this device (once per
  // device; a failure only disables that entry point)
  if (noalloc_setup(h->device) == MFIPM_OK) {
    h->na_scratch = g_noalloc[h->device].scratch;
    h->na_tw = g_noalloc[h->device].tw;
  }
  *hp = h;
  return MFIPM_OK;
}

int mfipm_set_params(mfipm_handle* h, const mfipm_params* p) {
  if (!h || check_params(p)) return MFIPM_ERR_INVALID_ARG;
  h->prm = *p;
  return MFIPM_OK;
}

int mfipm_destroy(mfipm_handle* h) {
  if (!h) return MFIPM_OK;
  (void)hipEventDestroy(h->ev0);
  (void)hipEventDestroy(h->ev1);
  for (int i = 0; i < 32; ++i)
    if (h->tw[i]) (void)hipFree(h->tw[i]);
  if (h->pinned) (void)hipHostFree(h->pinned);
  delete h;
  return MFIPM_OK;
}

int mfipm_set_launch(mfipm_handle* h, int32_t workgroups, int32_t team_size, int32_t tile_param) {
  if (!h || workgroups < 0 || team_size < 0 || tile_param < 0) return MFIPM_ERR_INVALID_ARG;
  h->req_wg = workgroups;
  h->req_team = team_size;
  h->req_tile = tile_param;
  return MFIPM_OK;
}

double mfipm_last_kernel_ms(const mfipm_handle* h) { return h ? h->last_ms : -1.0; }

int mfipm_workspace_size(const mfipm_handle* h, int32_t op_kind, int64_t max_n, int64_t max_m, int32_t batch,
                         size_t* bytes) {
  if (!h || !bytes || batch < 1 || max_n < 1 || max_m < 1) return MFIPM_ERR_INVALID_ARG;
  if (op_kind != MFIPM_OP_DENSE && op_kind != MFIPM_OP_PDCT && op_kind != MFIPM_OP_WHT && op_kind != MFIPM_OP_PDST)
    return MFIPM_ERR_INVALID_ARG;
  size_t best = 0;
  for (int bwd = 0; bwd < 2; ++bwd)
    for (int red = 0; red < 2; ++red) {
      const TeamLayout tl = team_layout(op_kind, max_n, max_m, pt_chunks_for(h, bwd, batch, max_m, red));
      const GlobalLayout gl =
          global_layout(op_kind, max_n, batch, max_teams_bound(h, op_kind, bwd, batch, red, max_n), tl);
      best = std::max(best, gl.total);
    }
  if (op_kind == MFIPM_OP_DENSE && h->prm.direct && max_n <= DC_MAX_N) {
    const TeamLayout tl = team_layout(kKindDirect, max_n, max_m, pt_chunks_for(h, 0, batch, max_m, 1));
    const GlobalLayout gl =
        global_layout(kKindDirect, max_n, batch, max_teams_bound(h, kKindDirect, 0, batch, 1, max_n), tl);
    best = std::max(best, gl.total);
  }
  if (op_kind == MFIPM_OP_DENSE && batch >= kLockstepMinBatch) best = std::max(best, ls_layout(max_n, max_m, batch).total);
  *bytes = best;
  return MFIPM_OK;
}

int mfipm_solve(mfipm_handle* h, const mfipm_operator* op, const double* b, double tau, double* x,
                double* state, void* ws, size_t ws_bytes, mfipm_info* info) {
  if (!h || !op) return MFIPM_ERR_INVALID_ARG;
  if (op->op == MFIPM_OP_DENSE && op->lda != op->n) return MFIPM_ERR_INVALID_ARG;
  const int64_t n_off[2] = {0, op->n}, m_off[2] = {0, op->m}, a_off[2] = {0, op->m * op->n};
  Problem P{1, op->op, 1, n_off, m_off, a_off, &tau, op->n, op->m};
  return launch(h, P, 0, op->A, op->rows, b, x, state, nullptr, nullptr, nullptr, Backing{(char*)ws, ws_bytes, nullptr},
                info);
}

int mfipm_solve_noalloc(mfipm_handle* h, const mfipm_operator* op, const double* b, double tau, double* x,
                        double* state, mfipm_info* info) {
  if (!h || !op) return MFIPM_ERR_INVALID_ARG;
  if (op->op == MFIPM_OP_DENSE && op->lda != op->n) return MFIPM_ERR_INVALID_ARG;
  if (!h->na_scratch || !h->na_tw) return MFIPM_ERR_HIP;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) return MFIPM_ERR_INVALID_ARG;
  const int64_t n_off[2] = {0, op->n}, m_off[2] = {0, op->m}, a_off[2] = {0, op->m * op->n};
  Problem P{1, op->op, 1, n_off, m_off, a_off, &tau, op->n, op->m};
  std::lock_guard<std::mutex> lock(g_noalloc[h->device].call);
  return launch(h, P, 0, op->A, op->rows, b, x, state, nullptr, nullptr, nullptr,
                Backing{h->na_scratch, MFIPM_NOALLOC_SCRATCH_BYTES, h->na_tw}, info);
}

int mfipm_solve_batched(mfipm_handle* h, int32_t batch, const int64_t* n_off, const int64_t* m_off,
                        const int64_t* a_off, int32_t op_kind, const double* A_packed, const int32_t* rows_packed,
                        int32_t shared_op, const double* b_packed, const double* tau, double* x_packed,
                        double* state_packed, void* ws, size_t ws_bytes, mfipm_info* infos) {
  if (!h || !n_off || !m_off || !tau || batch < 1) return MFIPM_ERR_INVALID_ARG;
  long long nmax = 0, mmax = 0;
  for (int i = 0; i < batch; ++i) {
    nmax = std::max<long long>(nmax, n_off[i + 1] - n_off[i]);
    mmax = std::max<long long>(mmax, m_off[i + 1] - m_off[i]);
  }
  Problem P{batch, op_kind, shared_op ? 1 : 0, n_off, m_off, a_off, tau, nmax, mmax};
  if (use_lockstep(h, op_kind, shared_op, batch))
    return launch_lockstep(h, P, A_packed, b_packed, x_packed, state_packed, ws, ws_bytes, infos);
  return launch(h, P, 0, A_packed, rows_packed, b_packed, x_packed, state_packed, nullptr, nullptr, nullptr,
                Backing{(char*)ws, ws_bytes, nullptr}, infos);
}

int mfipm_backward(mfipm_handle* h, int32_t batch, const int64_t* n_off, const int64_t* m_off,
                   const int64_t* a_off, int32_t op_kind, const double* A_packed, const int32_t* rows_packed,
                   int32_t shared_op, const double* state_packed, const double* grad_x_packed,
                   double* grad_b_packed, double* grad_tau, void* ws, size_t ws_bytes, mfipm_info* infos) {
  if (!h || !n_off || !m_off || batch < 1) return MFIPM_ERR_INVALID_ARG;
  if (!state_packed) return MFIPM_ERR_NO_STATE;
  long long nmax = 0, mmax = 0;
  for (int i = 0; i < batch; ++i) {
    nmax = std::max<long long>(nmax, n_off[i + 1] - n_off[i]);
    mmax = std::max<long long>(mmax, m_off[i + 1] - m_off[i]);
  }
  Problem P{batch, op_kind, shared_op ? 1 : 0, n_off, m_off, a_off, nullptr, nmax, mmax};
  return launch(h, P, 1, A_packed, rows_packed, nullptr, nullptr, const_cast<double*>(state_packed),
                grad_x_packed, grad_b_packed, grad_tau, Backing{(char*)ws, ws_bytes, nullptr}, infos);
}

const char* mfipm_status_string(int32_t code) {
  switch (code) {
    case MFIPM_ERR_INVALID_ARG: return "invalid argument";
    case MFIPM_ERR_HIP: return "HIP runtime error";
    case MFIPM_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case MFIPM_ERR_NO_STATE: return "no state from a forward solve";
    case MFIPM_ERR_DEVICE_CHECK: return "device-side input check failed";
    case MFIPM_ERR_TOO_LARGE: return "problem too large for the no-allocation scratch";
    case MFIPM_STATUS_CONVERGED: return "converged";
    case MFIPM_STATUS_MAXITER: return "iteration limit";
    case MFIPM_STATUS_PCG_BREAKDOWN: return "PCG breakdown";
    case MFIPM_STATUS_NONFINITE: return "non-finite value";
    case MFIPM_STATUS_STEP_UNDERFLOW: return "step underflow";
    case MFIPM_STATUS_ABORTED: return "aborted (device wait bound exceeded)";
    case MFIPM_STATUS_INPUT_CHECK: return "input check failed";
    case MFIPM_STATUS_PCG_MAXITER: return "adjoint PCG iteration limit";
    default: return "unknown";
  }
}

}  // extern "C"
