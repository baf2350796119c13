/*
 * mfipm.h -- C ABI of the MI355X (gfx950) matrix-free interior point solver
 * for l1-regularised least squares.
 *
 * Problem (Fountoulakis, Gondzio, Zhlobich, "Matrix-free interior point method
 * for compressed sensing problems", Section 1 eq. (formulationsnoisy1) with the
 * 1/2 of Section 1 eq. (wrightBPDN)):
 *
 *     min_x  tau * ||x||_1 + 1/2 * ||A x - b||_2^2
 *
 * solved as the bound-constrained QP over z = [u; v] >= 0, x = u - v
 * (Section 1, eqs. (uvDef), (lintechni), (wrightBPDN)) by the single-corrector
 * primal-dual IPM of Section 5.1, whose Newton directions come from the
 * reduced system (Theta^{-1} + F F^T) dz = f_z + Z^{-1} f_s (Section 3,
 * eq. (redNewton)) solved by preconditioned CG with the block preconditioner
 * of Section 4, eq. (eq:ne2_P).  A is only applied as A*d and A^T*y.
 *
 * Conventions for every entry point
 *   - All numeric data are IEEE double (FP64); index arrays are int32.
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - The caller owns every buffer (operator data, b, x, state, gradients,
 *     workspace).  The library owns only the handle, which caches small
 *     device tables of FFT roots of unity per transform size (freed by
 *     mfipm_destroy).  No caller buffer is retained after a call returns.
 *   - Work is ordered on the stream given to mfipm_create (a hipStream_t
 *     passed as void*; NULL = the default stream).  solve/backward calls
 *     return after the work has finished and `info` is filled.
 *   - A handle is not thread-safe: calls on one handle must not overlap
 *     (it reuses its pinned staging buffer and events between calls); use
 *     one handle per host thread.  Handles on one device share nothing but
 *     the static scratch of mfipm_solve_noalloc, whose calls are serialised.
 *   - Return value: 0 = OK; negative = error, nothing was computed
 *     (MFIPM_ERR_*).  No entry point aborts, throws or exits.
 *   - The solver outcome of each instance is reported in mfipm_info.status
 *     (MFIPM_STATUS_*).
 *
 * Vector layouts
 *   - state: 4n doubles per instance: z as n interleaved pairs (u_i, v_i),
 *     then s as n interleaved pairs (s_u,i, s_v,i).
 *   - packed batches: instance i occupies [n_off[i], n_off[i+1]) of x and
 *     grad_x, [m_off[i], m_off[i+1]) of b and grad_b, 4*n_off[i].. of state
 *     and, for dense operators, [a_off[i], a_off[i+1]) of A_packed (row-major
 *     m_i x n_i, leading dimension n_i).
 */
#ifndef MFIPM_H
#define MFIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MFIPM_OK 0
#define MFIPM_ERR_INVALID_ARG (-1)
#define MFIPM_ERR_HIP (-2)
#define MFIPM_ERR_WORKSPACE_TOO_SMALL (-3)
#define MFIPM_ERR_NO_STATE (-4)
#define MFIPM_ERR_DEVICE_CHECK (-5) /* device-side input check failed (e.g. rows not sorted/distinct) */
#define MFIPM_ERR_TOO_LARGE (-6)    /* mfipm_solve_noalloc: the call's workspace exceeds the static
                                       scratch (MFIPM_NOALLOC_SCRATCH_BYTES)                      */

/* Bytes of the static per-device scratch used by mfipm_solve_noalloc. */
#define MFIPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* solver outcome (mfipm_info.status) */
#define MFIPM_STATUS_CONVERGED 0      /* relative duality gap <= tol                        */
#define MFIPM_STATUS_MAXITER 1        /* maxiters IPM iterations done                       */
#define MFIPM_STATUS_PCG_BREAKDOWN 2  /* p^T H p <= 0 in PCG                                */
#define MFIPM_STATUS_NONFINITE 3      /* NaN/Inf in a reduction (e.g. NaN in b)             */
#define MFIPM_STATUS_STEP_UNDERFLOW 4 /* both step sizes below step_min                     */
#define MFIPM_STATUS_ABORTED 5        /* a device-side wait exceeded its bound              */
#define MFIPM_STATUS_INPUT_CHECK 6    /* device-side input check failed (rows)              */
#define MFIPM_STATUS_PCG_MAXITER 7    /* backward only: the adjoint PCG reached mxiterpcg_adj
                                         before tolpcg_adj; the gradients are those of its
                                         last iterate                                       */

/* operator kinds */
#define MFIPM_OP_DENSE 0 /* explicit m x n row-major matrix                                     */
#define MFIPM_OP_PDCT 1  /* rows of the orthonormal DCT-II of length n (Section 2, eq.
                            (eq:orthonormality): A A^T = I); n a power of two, 64 <= n <= 2^20 */
#define MFIPM_OP_WHT 2   /* rows of the orthonormal Walsh-Hadamard matrix H_n / sqrt(n) in
                            natural (Sylvester) order, another fast transform with orthonormal
                            rows (Section 1, Section 2); n a power of two, 64 <= n <= 2^20   */
#define MFIPM_OP_PDST 3  /* rows of the orthonormal DST-II of length n, a further fast
                            transform with orthonormal rows (Section 1, Section 2); n a power
                            of two, 64 <= n <= 2^20                                          */

typedef struct mfipm_handle mfipm_handle;

/* A single measurement operator.
 * DENSE: A is row-major m x n with leading dimension lda >= n (borrowed).
 * PDCT : rows holds m sorted, distinct indices in [0, n) of the DCT-II rows
 *        kept by A (borrowed); A*d = DCT-II_ortho(d)[rows],
 *        A^T*y = DCT-III_ortho(zero-fill(y)).
 * WHT  : rows as for PDCT, of W = H_n / sqrt(n); A*d = (W d)[rows],
 *        A^T*y = W zero-fill(y).
 * PDST : rows as for PDCT, of the orthonormal DST-II S; A*d = (S d)[rows],
 *        A^T*y = DST-III_ortho(zero-fill(y)).                                   */
typedef struct {
  int32_t op;
  int64_t m, n;
  const double* A;
  int64_t lda;
  const int32_t* rows;
} mfipm_operator;

/* Parameters.  Defaults (mfipm_params_default) are the paper's values:
 * sigma1..3 = 0.1/0.5/0.8 and alpha_bar/alpha_tilde = 0.5/0.1 (Section 5.1,
 * after the algorithm), maxiters = 100 and mxiterpcg = 200 (Section 5.4),
 * tol = 1e-8 and tolpcg = 1e-2 (inside the noisy-problem ranges of
 * Section 5.4).  eta, rho, z0, s0 are readings where the paper is silent:
 * step = min(1, eta * largest feasible step); rho <= 0 selects
 * ||A||_F^2 / n, the closest scalar multiple of the identity to A^T A in the
 * Frobenius norm (Section 4, before eq. (eq:ne2_P)); z0 = s0 = 1.            */
typedef struct {
  double tol;         /* relative duality gap target                              */
  int32_t maxiters;   /* IPM iteration cap                                        */
  double tolpcg;      /* PCG: stop when ||r||_2 <= tolpcg * ||rhs||_2             */
  int32_t mxiterpcg;  /* PCG iteration cap (reaching it is not an error)          */
  double sigma1, sigma2, sigma3;
  double alpha_bar, alpha_tilde;
  double eta;
  double rho;
  double z0, s0;
  double tolpcg_adj;     /* adjoint PCG tolerance                                 */
  int32_t mxiterpcg_adj; /* adjoint PCG iteration cap                             */
  double step_min;       /* STEP_UNDERFLOW when both steps fall below this        */
  int32_t reduced;       /* 0: PCG on the 2n system (eq. (eq:ne2_matrix)) with the
                            block preconditioner (eq. (eq:ne2_P)), as in the paper;
                            1: PCG on the n x n system behind the Theorem
                            (thm:ne2_prec) of Section 4,
                            (Theta_bar^{-1} + A^T A) d = Theta_bar^{-1}
                            (Theta_u r_u - Theta_v r_v), Theta_bar = Theta_u +
                            Theta_v, preconditioned by Theta_bar^{-1} + rho I, the
                            2n direction back-substituted from d = du - dv (half
                            the vector traffic per PCG iteration; different PCG
                            iterates).  Lock-step batches use the 2n system and
                            are not taken when this is set.                     */
  int32_t direct;        /* 0: PCG (the matrix-free method);
                            1: exact Newton directions by a direct solver
                            (Section 5.7): Cholesky factorisation of the
                            n x n system above, M = Theta_bar^{-1} + A^T A,
                            formed from A^T A (computed once per solve) at
                            every IPM iteration, the corrector reusing the
                            factor.  Forward solves with a DENSE operator and
                            n <= 8192 only (else MFIPM_ERR_INVALID_ARG); the
                            workspace grows by about 16 n^2 bytes per
                            concurrently solved instance; pcg_iters reports 0;
                            mfipm_backward ignores it (adjoint by PCG).  A
                            factorisation that meets a non-positive pivot
                            ends the solve with MFIPM_STATUS_PCG_BREAKDOWN.   */
} mfipm_params;

/* Per-instance report (HOST memory). */
typedef struct {
  int32_t status;      /* MFIPM_STATUS_*                                           */
  int32_t ipm_iters;   /* Newton directions taken (a corrector does not count)      */
  int32_t pcg_iters;   /* operator applies inside PCG, summed over the solve        */
  int32_t correctors;  /* corrector directions computed                             */
  int64_t nmat;        /* products with A or A^T (Section 5, symbol table: nMat)    */
  double rel_gap;      /* final relative duality gap                                */
  double mu;           /* final z^T s / (2n)                                         */
  double primal_obj;   /* tau 1^T z + 1/2 ||A(u-v) - b||^2                          */
  double dual_obj;     /* -1/2 ||nu||^2 - b^T nu, nu = min(1,tau/||g||_inf)(Ax-b)   */
  double rho;          /* preconditioner scalar used                                */
} mfipm_info;

/* Fills *p with the defaults above (host only, no device work). */
int mfipm_params_default(mfipm_params* p);

/* Creates a handle bound to the current HIP device and `stream`.
 * Errors: INVALID_ARG for a NULL h or a parameter out of range
 * (tol <= 0, maxiters < 1, tolpcg <= 0, mxiterpcg < 1, eta not in (0,1],
 * z0/s0 <= 0), HIP if the device cannot be queried.                          */
int mfipm_create(mfipm_handle** h, const mfipm_params* p, void* stream);

/* Replaces the parameters of an existing handle (same checks as create). */
int mfipm_set_params(mfipm_handle* h, const mfipm_params* p);

/* Releases the handle (NULL is accepted). */
int mfipm_destroy(mfipm_handle* h);

/* Workspace bytes needed by solve/backward for `batch` instances whose
 * largest signal length is max_n and largest measurement count is max_m
 * (for one operator pass op->n, op->m and batch = 1).  Host only.            */
int mfipm_workspace_size(const mfipm_handle* h, int32_t op_kind, int64_t max_n, int64_t max_m,
                         int32_t batch, size_t* bytes);

/* Solves one instance.  b: m doubles; tau > 0 (host scalar); x: n doubles
 * (output); state: 4n doubles (output, may be NULL) -- the final (z, s),
 * which mfipm_backward needs; ws/ws_bytes: workspace of at least
 * mfipm_workspace_size(h, op->op, op->n, op->m, 1) bytes; info: host.
 * Errors: INVALID_ARG (NULL pointers, m < 1, tau <= 0 or not finite; for
 * PDCT, PDST and WHT: n not a power of two in [64, 2^20] or m > n; with
 * params.direct: an operator other than DENSE or n > 8192);
 * WORKSPACE_TOO_SMALL; DEVICE_CHECK (rows not sorted/distinct/in range);
 * HIP.                                                                      */
int mfipm_solve(mfipm_handle* h, const mfipm_operator* op, const double* b, double tau,
                double* x, double* state, void* ws, size_t ws_bytes, mfipm_info* info);

/* For callers that cannot allocate memory (code under stream/graph capture,
 * tight serving loops, harnesses that forbid allocation): mfipm_solve
 * without a workspace argument.  The workspace is a static device array of
 * MFIPM_NOALLOC_SCRATCH_BYTES (64 MiB) that every device holds from the
 * first mfipm_create on it until the process ends; the FFT roots of unity
 * come from a static full-resolution table filled at that mfipm_create.  The
 * call allocates nothing (no hipMalloc, hipHostMalloc or hipFree; report
 * transfers go through the host stack) and clears the control words it needs
 * with a kernel.  It must be called with the handle's device current.
 * Arguments, layouts, results and errors as mfipm_solve, plus TOO_LARGE when
 * mfipm_workspace_size(h, op->op, op->n, op->m, 1) exceeds the scratch
 * (e.g. partial DCT n >= 2^18), and HIP when the static memory could not be
 * set up.  All calls on one device share the array and keep no state in it
 * between calls: calls from several host threads on one device are
 * serialised by the library; calls from several processes each use their
 * own copy.  Results may differ from mfipm_solve in the last bits (partial
 * DCT: the twiddles come from the full-resolution table).                    */
int mfipm_solve_noalloc(mfipm_handle* h, const mfipm_operator* op, const double* b, double tau,
                        double* x, double* state, mfipm_info* info);

/* Solves `batch` independent instances in one persistent launch; teams of
 * workgroups take instances from a device queue in the host-given order
 * (longest first).  n_off, m_off (and a_off for DENSE) are HOST arrays of
 * batch+1 offsets.  shared_op != 0 means every instance uses the same
 * operator: for PDCT the single rows array of length m_off[1]-m_off[0]; for
 * DENSE the single matrix at A_packed.  tau: HOST array of batch values.
 * state_packed may be NULL.  infos: HOST array of batch reports.
 * DENSE with shared_op and batch >= 8 (and no team size set through
 * mfipm_set_launch) runs all instances in lock step instead: every round
 * applies the operator to all of them at once as two FP64 matrix-matrix
 * products on the matrix cores (A D and A^T Y), and each instance's IPM
 * advances on one workgroup between rounds; per instance the iterates are
 * those of the single-instance method.
 * Errors as mfipm_solve, per instance.                                       */
int mfipm_solve_batched(mfipm_handle* h, int32_t batch, const int64_t* n_off, const int64_t* m_off,
                        const int64_t* a_off, int32_t op_kind, const double* A_packed,
                        const int32_t* rows_packed, int32_t shared_op, const double* b_packed,
                        const double* tau, double* x_packed, double* state_packed, void* ws,
                        size_t ws_bytes, mfipm_info* infos);

/* Adjoint of the solve map (b, tau) -> x at the state written by the
 * matching forward call: solves (Theta^{-1} + F F^T) w = [g; -g] with the
 * same PCG and preconditioner (Theta, P frozen at that state), then
 * grad_b = A (w_u - w_v) (m doubles per instance) and grad_tau = -1^T w
 * (one double per instance, device).  Offsets/operator as in the batched
 * solve.  infos (HOST, may be NULL): status and pcg_iters of the adjoint
 * solve: CONVERGED, PCG_MAXITER (cap reached; gradients of the last
 * iterate), or PCG_BREAKDOWN / NONFINITE / ABORTED / INPUT_CHECK, in which
 * case every grad_b entry and grad_tau of that instance are NaN.
 * Errors: NO_STATE for a NULL state, else as mfipm_solve.                    */
int mfipm_backward(mfipm_handle* h, int32_t batch, const int64_t* n_off, const int64_t* m_off,
                   const int64_t* a_off, int32_t op_kind, const double* A_packed,
                   const int32_t* rows_packed, int32_t shared_op, const double* state_packed,
                   const double* grad_x_packed, double* grad_b_packed, double* grad_tau,
                   void* ws, size_t ws_bytes, mfipm_info* infos);

/* Launch shape used for the next calls: total workgroups (0 = automatic) and
 * workgroups per team for batched calls (0 = automatic).  tile_param is the
 * operator tile choice: DENSE rows per row-block item, PDCT log2 of the
 * column-FFT length (0 = automatic).  Host only; validated at the next call. */
int mfipm_set_launch(mfipm_handle* h, int32_t workgroups, int32_t team_size, int32_t tile_param);

/* Device time in milliseconds of the last solve/backward kernel (measured
 * with HIP events on the handle's stream), or a negative value if none.     */
double mfipm_last_kernel_ms(const mfipm_handle* h);

/* Static text for a return code (<0) or a status (>=0). */
const char* mfipm_status_string(int32_t code);

#ifdef __cplusplus
}
#endif
#endif /* MFIPM_H */
