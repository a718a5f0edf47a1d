/*
 * aao.h - C ABI of libaao.so: the alpha-circulant preconditioned Richardson
 * sweep for the all-at-once collocation system of a linear IVP u' = A u, on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Caklovic, Speck, Frank, "A parallel-in-time collocation method using
 * diagonalization: theory and implementation for linear problems",
 * arXiv 2103.12571.
 *
 *   C u = w,  C = I_L (x) C_coll + E (x) H          (Sec. 2.1, eq. (globalsys))
 *   C_coll = I_MN - dT Q (x) A,  H = H_M (x) I_N     (Sec. 2.1, eq. (Hm))
 *   C_alpha = I_L (x) C_coll + E_alpha (x) H         (Sec. 2.2, eq. (prec))
 *   u <- u + C_alpha^{-1} (w - C u)                  (eq. (Riteration), defect-
 *                                                     correction form)
 *
 * C_alpha^{-1} is applied as in Alg. 1: scale by J^{-1}, DFT over the L steps
 * (Lemma 1), per step the M x M eigenbasis S_l^{-1} of Q G_l^{-1} (Sec. 2.3,
 * eq. (QGL)), L*M decoupled complex-shifted spatial solves
 * (I - dT d_lm A) x2 = x1 (eq. (innerdiag)), then S_l, G_l^{-1}, inverse DFT
 * and J.  Only the L/2+1 non-redundant frequencies are solved: for real data
 * frequency L-j is the complex conjugate of frequency j.
 *
 * Conventions
 *  - Every array argument named *_dev is a DEVICE pointer, owned by the
 *    caller, FP64, contiguous, C order.  u, r, lambda are [B][L][M][N];
 *    u0, g_last, grad_u0 are [B][N]; grad_nu is [B].  n = y*nx + x.
 *  - Host pointers (struct members, alphas, info) are read during the call
 *    only; the library keeps copies of what it needs.
 *  - All device work is enqueued on the stream given to aao_setup (or
 *    aao_set_stream).  Calls that return norms or status synchronise that
 *    stream before returning.
 *  - Device memory: the library allocates only a small table block (per-plan
 *    coefficient tables, a few KB per alpha) and pinned host staging.  All
 *    large scratch (inner-solve vectors, partial sums) lives in a caller-
 *    provided workspace (aao_workspace_size / aao_set_workspace).
 *  - Errors: every call returns an aao_status; AAO_OK is 0, errors are
 *    negative.  No call aborts or throws across the ABI.  On error
 *    aao_last_error() returns a thread-local message.  Argument checks run
 *    before any launch, so an EINVAL/EWORKSPACE/ENODIAG return leaves device
 *    memory untouched.
 *  - A plan is not thread-safe; distinct plans may be used concurrently on
 *    distinct streams.
 */
#ifndef AAO_H
#define AAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aao_plan* aao_plan_t;

typedef enum {
  AAO_OK = 0,
  AAO_EINVAL = -1,      /* invalid argument (sizes, pointers, alpha outside (0,1)) */
  AAO_EHIP = -2,        /* a HIP runtime call failed */
  AAO_ENODIAG = -3,     /* Q G_l^{-1} not (well) diagonalisable for this alpha
                           (Sec. 2.3: eigenvalues coalesce, Examples 1-2) */
  AAO_ENOCONV = -4,     /* aao_solve / adjoint: max_iter sweeps without meeting tol */
  AAO_ESTAGNATE = -5,   /* aao_solve / adjoint: the monitored quantity stopped
                           contracting above tol (Sec. 3.3: consecutive iterates
                           alone can take stagnation for convergence); see
                           aao_solve */
  AAO_EWORKSPACE = -6,  /* no workspace set, or smaller than aao_workspace_size */
  AAO_ENAN = -7,        /* a norm became NaN or Inf */
  AAO_ESTATE = -8       /* call order violated (e.g. sweep before aao_set_u0) */
} aao_status;

enum { AAO_FP64 = 0,   /* every step in FP64 / complex128 */
       AAO_MIXED = 1   /* inner solves stored and computed in complex64; residual,
                          alpha scaling, DFT over L, M x M transforms and the
                          update of u stay FP64 (Theorem 2: round-off grows like
                          alpha^{-(l-1)/L}) */ };

enum { AAO_INNER_COCG = 0,      /* batched COCG: needs A = A^T (complex-symmetric
                                   shifted systems) */
       AAO_INNER_BICGSTAB = 1,  /* batched BiCGStab: any A; systems of at most 4096
                                   points run every iteration in one launch, one
                                   workgroup per system */
       AAO_INNER_FFT = 2        /* spatial-FFT direct solve (exact for periodic
                                   constant-coefficient A); any nx, ny: lengths that are
                                   not powers of two use Bluestein's chirp-z transform
                                   (length P = the power of two >= 2n - 1) */ };

enum { AAO_STOP_LASTSTEP = 0,   /* ||u_L^{k+1} - u_L^k||_inf <= tol (Sec. 3.2, Alg. 2) */
       AAO_STOP_RESIDUAL = 1    /* ||w - C u||_2 / ||w||_2 <= tol */ };

/* A periodic constant-coefficient stencil:
 *   (A v)[x, y] = sum_t coef[t] * v[(x + dx[t]) mod nx, (y + dy[t]) mod ny].
 * ndim 1 uses ny = 1 and ignores dy.  |dx|, |dy| <= 4, ntaps <= 32.
 * dcoef_dnu (nullable) holds dA/dnu with the same taps, used by aao_grad. */
typedef struct {
  int ndim;
  int64_t nx, ny;
  int ntaps;
  const int32_t* dx;
  const int32_t* dy;          /* nullable when ndim == 1 */
  const double* coef;
  const double* dcoef_dnu;    /* nullable */
} aao_stencil;

typedef struct {
  int M;                /* collocation nodes per step, 1..8 */
  const double* nodes;  /* NULL: Radau-right nodes (Sec. 2.1, Sec. 2.3); else M
                           increasing nodes in (0, 1] with nodes[M-1] == 1 */
  int L;                /* steps solved at once; power of two, 1..1024, L * M <= 2048 */
  double dt;            /* step size dT > 0 */
  int batch;            /* B >= 1 independent instances sharing A */
  int precision;        /* AAO_FP64 | AAO_MIXED */
  int inner;            /* AAO_INNER_* */
  double inner_tol;     /* relative residual per shifted system (tau) */
  int inner_maxit;      /* iteration cap per shifted system (Krylov) */
} aao_config;

#define AAO_MAX_HIST 64
typedef struct {
  int iterations;                    /* sweeps performed */
  int converged;                     /* 1 if the stop rule was met */
  double gamma, m0;                  /* Alg. 2 quantities actually used */
  double alpha[AAO_MAX_HIST];        /* alpha_k of sweep k */
  double m[AAO_MAX_HIST];            /* m_k bound of Alg. 2 after sweep k */
  double res_rel[AAO_MAX_HIST];      /* ||w - C u^k||_2 / ||w||_2 before sweep k */
  double dlast_inf[AAO_MAX_HIST];    /* ||u_L^{k+1} - u_L^k||_inf of sweep k */
  double inner_mean[AAO_MAX_HIST];   /* mean Krylov iterations per system, sweep k */
  int inner_max[AAO_MAX_HIST];       /* max Krylov iterations over systems, sweep k */
  int inner_fail[AAO_MAX_HIST];      /* shifted systems of sweep k that stopped without
                                        meeting tau: iteration cap reached or breakdown */
  int inner_fail_total;              /* sum of inner_fail over all sweeps */
} aao_solve_info;

/* Per kernel class: launches, elements processed, event-timed milliseconds and
 * algorithmic bytes moved.  Timing is collected only while enabled by
 * aao_set_timing(plan, 1).  Classes: see aao_kernel_name(). */
#define AAO_NUM_KERNELS 14
typedef struct {
  int64_t launches[AAO_NUM_KERNELS];
  double elements[AAO_NUM_KERNELS];
  double bytes[AAO_NUM_KERNELS];
  double ms[AAO_NUM_KERNELS];
} aao_kernel_stats;

/* Create a plan for the composite collocation problem of Sec. 2.1 with
 * stencil A, nodes/Q, L steps of size dt (eq. (globalsys)).
 * Computes nodes and Q (eq. (collocation)) on the host, uploads the stencil and
 * the DFT twiddles.  hip_stream: a hipStream_t (NULL = default stream).
 * Errors: EINVAL for bad sizes/pointers, COCG with a non-symmetric stencil,
 * FFT inner solve whose transform line (n, or P >= 2n - 1 for Bluestein) times
 * sizeof(complex) exceeds 64 KiB; EHIP. */
aao_status aao_setup(const aao_stencil* A, const aao_config* cfg, void* hip_stream,
                     aao_plan_t* out);

/* Absolute floor of the inner stop inside aao_solve, aao_solve_windows and
 * aao_adjoint_solve.  The paper's iteration (eq. (Riteration) in its
 * right-hand-side form, Alg. 1) gives every shifted system the transform of
 * w + (C_alpha - C) u^k, which is of the size of w, and stops it at the
 * relative tolerance tau (Sec. 5.2 uses GMRES with a relative tolerance; the
 * error model of Sec. 3.3, gamma = L (3 eps + tau) ||w||, rests on it).  In the
 * defect-correction form the right-hand side is the residual, which shrinks
 * sweep by sweep, so a relative stop there asks for far more accuracy than the
 * paper's.  With the floor, system s stops once
 *     ||r_s||_2 <= max(tau ||b_s||_2, tau_w ||x1_s(w)||_2),
 * x1_s(w) being the transform of w that system s would receive (primal: w =
 * 1_M (x) u0 in step 1; adjoint: g_last at the last node of step L; a source
 * is not counted, which only lowers the floor).  Every system still makes at
 * least one iteration.  The error the floor leaves in u is of the order of
 * tau_w ||w|| (Sec. 3.3's round-off model with tau_w in place of tau), so it
 * must sit below the outer stop tolerance.  tau_w = 0: relative stop only;
 * tau_w > 0: that floor in every solve; tau_w < 0 (the default): tau_w =
 * min(tau, tol / 100) with tol the stop tolerance of the solve at hand.  If
 * the monitored quantity makes no progress for two sweeps while the floor is
 * on, the solve tightens it a hundredfold (three times at most, then drops
 * it); AAO_ESTAGNATE is returned only for a stall without the floor.
 * aao_sweep, aao_precond, aao_shifted_solve and aao_solve_gmres always stop
 * relative to their own right-hand sides.
 * EINVAL for a null plan or a non-finite tau_w. */
aao_status aao_set_inner_floor(aao_plan_t plan, double tau_w);

/* Rebind the plan to another stream. */
aao_status aao_set_stream(aao_plan_t plan, void* hip_stream);

/* Bytes of device workspace the plan needs (256-byte aligned pointer). */
aao_status aao_workspace_size(aao_plan_t plan, size_t* bytes);

/* Hand the plan a device workspace of at least aao_workspace_size bytes.  The
 * caller keeps ownership and must keep it alive while the plan uses it. */
aao_status aao_set_workspace(aao_plan_t plan, void* dev_ptr, size_t bytes);

/* Replace the stencil weights of A (ntaps host doubles, same offsets as at
 * setup), e.g. a new diffusion coefficient nu, without re-planning (Sec. 2.1:
 * A enters the sweep only through C_coll = I - dT Q (x) A).  dcoef_dnu
 * (nullable) replaces dA/dnu for aao_grad.  Launches enqueued earlier keep the
 * old weights.  AAO_EINVAL for null or non-finite input, or for weights that
 * make A non-symmetric when the inner solver is COCG (nothing is changed). */
aao_status aao_set_stencil_coef(aao_plan_t plan, const double* coef, const double* dcoef_dnu);

/* Set the initial value u0_dev [B][N]; defines w = (1_M (x) u0, 0, ..., 0)
 * (eq. (globalsys); plus the source term if aao_set_forcing gave one).  The pointer is kept (not copied): u0 must stay
 * valid and unchanged while the plan uses it. */
aao_status aao_set_u0(aao_plan_t plan, const double* u0_dev);

/* Source term of eq. (collocation): b_dev [B][L][M][N] holds b(t) at the
 * collocation times t_{l-1} + tau_m dT of every step (device, caller-owned,
 * kept like u0), so that w_l gains dT (Q (x) I) b_l; NULL removes it.  The
 * transposed (adjoint) system is unaffected.  Recomputes ||w|| if u0 is set;
 * AAO_ENAN if w is not finite (the previous source is kept). */
aao_status aao_set_forcing(aao_plan_t plan, const double* b_dev);

/* Row a1: r = w - C u (eq. (globalsys)), r_dev [B][L][M][N].  res_norm
 * (nullable host out) = ||r||_2 / ||w||_2. */
aao_status aao_residual(aao_plan_t plan, const double* u_dev, double* r_dev, double* res_norm);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): aao_residual
 * with no workspace and no allocation.  Its partial sums and norms live in a
 * fixed 14 KiB device array inside the library (one per GPU, held until the
 * process ends), looked up once per device; the plan needs only aao_setup
 * (host-only), not aao_set_workspace or aao_set_u0.  u0_dev [B][N] defines w
 * as in aao_set_u0 (plus the plan's source, if aao_set_forcing gave one).
 * r_dev [B][L][M][N] receives w - C u; res_norm (nullable host out) =
 * ||r||_2 / ||w||_2, computed by the same kernels in the same order as
 * aao_residual, so both calls give the same bits.  Any problem size fits: at
 * most 1024 partial sums are formed (EINVAL otherwise, never reached).  The
 * plan's device must be current; the call synchronises the plan's stream.  Every call on one GPU shares the array: calls that overlap on one
 * GPU (other threads, other streams) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero (every slot read is
 * written first by the same call).  EINVAL for null arguments, EHIP, ENAN. */
aao_status aao_residual_noalloc(aao_plan_t plan, const double* u0_dev, const double* u_dev, double* r_dev,
                                double* res_norm);

/* Rows a2-a4: delta = C_alpha^{-1} r via Alg. 1's diagonalised steps
 * (Lemma 1; eqs. (s123), (innercoll), (innerdiag), (QGL)).  r_dev and
 * delta_dev are [B][L][M][N]; they may alias.  alpha in (0, 1).
 * Errors: EINVAL, ENODIAG, EWORKSPACE, ESTATE. */
aao_status aao_precond(aao_plan_t plan, const double* r_dev, double* delta_dev, double alpha);

/* One sweep of eq. (Riteration) in defect-correction form on u_dev (in place):
 * u <- u + C_alpha^{-1}(w - C u).  res_rel (nullable host out): relative
 * residual of u BEFORE the sweep; dlast_inf (nullable host out):
 * ||u_L^{new} - u_L^{old}||_inf over all M nodes of the last step. */
aao_status aao_sweep(aao_plan_t plan, double* u_dev, double alpha, double* res_rel,
                     double* dlast_inf);

/* Alg. 2 (or a given alpha list): initialise u = (u0, ..., u0) (Sec. 5),
 * then sweep until the stop rule holds or max_iter sweeps are done.
 * alphas == NULL: adaptive alpha_{k+1} = sqrt(gamma/m_k), m_{k+1} =
 * 2 sqrt(m_k gamma), gamma = L (3 eps + tau) ||w||_inf (Sec. 3.3), clamped to
 * alpha <= 1/2; m0 <= 0 selects m0 = L dT ||A||_inf ||u0||_inf (Sec. 3.3).
 * With AAO_MIXED the same balance is taken for the defect-correction form,
 * whose round-off is relative to the current residual: alpha = min(1/2,
 * sqrt(L (3 eps + tau))) with eps = 2^-24 (eq. (minimeq) on a relative model).
 * alphas != NULL: sweep k uses alphas[min(k, n_alphas-1)].
 * Stopping (Sec. 3.3, Alg. 2): converged when the stop rule holds.  Alg. 2's
 * own loop exit (error model m_k <= tol) counts as converged only if every
 * shifted system of the last sweep met tau (gamma assumes it); otherwise the
 * sweeps go on under the stop rule.  The monitored quantity (the last-step
 * difference, or the relative residual under AAO_STOP_RESIDUAL) must keep
 * improving: when four sweeps in a row leave it above tol and not below 0.99
 * times the smallest value seen so far, the call returns AAO_ESTAGNATE (a
 * slow steady contraction sets a new smallest value every sweep; a round-off
 * plateau does not).
 * Returns ENOCONV when max_iter is reached; info is filled in every case
 * (info->inner_fail counts the shifted systems that missed tau per sweep). */
aao_status aao_solve(aao_plan_t plan, double* u_dev, const double* alphas, int n_alphas,
                     double m0, double tol, int stop_rule, int max_iter, aao_solve_info* info);

/* Moving window (Sec. 5.2): n_windows consecutive blocks of L steps, each
 * solved as by aao_solve (same alphas / m0 / tol / stop rule / max_iter),
 * window k + 1 starting from the last node of window k's last step (copied
 * on the device).  Window 0 starts from the u0 given to aao_set_u0.
 * frc_all (nullable, device): the source of every window, [W][B][L][M][N]
 * at each window's collocation times; NULL keeps the source of
 * aao_set_forcing (if any) for every window.  u_dev ends as the last
 * window's solution.  infos: n_windows entries (host).  Stops at the first
 * window that fails (its status is returned); the plan's u0 and source are
 * restored afterwards. */
aao_status aao_solve_windows(aao_plan_t plan, double* u_dev, int n_windows, const double* frc_all,
                             const double* alphas, int n_alphas, double m0, double tol, int stop_rule,
                             int max_iter, aao_solve_info* infos);

/* Outer Krylov solver in place of the Richardson sweep (the paper points to
 * Krylov acceleration of the alpha-circulant preconditioner, introduction and
 * Sec. 6): flexible GMRES(restart) on C u = w (eq. (globalsys)) with C_alpha
 * (eq. (prec)) as right preconditioner, one Krylov space per instance b.
 * Step k applies C_alpha^{-1} with alphas[min(k, n_alphas-1)]; alphas = NULL
 * uses the fixed alpha = clamp(sqrt(L (3 eps + tau)), 1e-8, 1/2), eps = 2^-53
 * (FP64) or 2^-24 (MIXED): the relative round-off model of mixed precision
 * also fits here, since each preconditioner application is relative to the
 * current Krylov vector.  Gram-Schmidt is classical with one
 * re-orthogonalisation; the small least-squares problems are solved by Givens
 * rotations on the host.  u_dev [B][L][M][N] is overwritten: it starts from
 * u0 at every node.  Stops when max over b of ||w_b - C u_b||_2 / ||w_b||_2
 * <= tol (the true residual, checked at every restart and at the end) or after
 * max_steps preconditioner applications (ENOCONV).
 * work_dev: device scratch of at least aao_gmres_workspace_size bytes, 256-byte
 * aligned, owned by the caller; restart in 1..31. */
typedef struct {
  int steps;                         /* preconditioner applications */
  int cycles;                        /* restart cycles started */
  int converged;                     /* 1 if tol was met */
  double res_rel;                    /* final true max_b ||w_b - C u_b|| / ||w_b|| */
  double alpha[AAO_MAX_HIST];        /* alpha of step k */
  double res_est[AAO_MAX_HIST];      /* least-squares estimate of the relative residual after step k */
  double inner_mean[AAO_MAX_HIST];   /* mean inner iterations per shifted system, step k */
  int inner_max[AAO_MAX_HIST];       /* max inner iterations over systems, step k */
} aao_gmres_info;
aao_status aao_gmres_workspace_size(aao_plan_t plan, int restart, size_t* bytes);
aao_status aao_solve_gmres(aao_plan_t plan, double* u_dev, int restart, const double* alphas, int n_alphas,
                           double tol, int max_steps, void* work_dev, size_t work_bytes, aao_gmres_info* info);

/* Adjoint: solve C^T lambda = g, g = e_{L,M} (x) g_last, by the same
 * alpha-circulant machinery transposed (E_alpha^T = V^{-T} D_alpha V^T, Lemma
 * 1 transposed): per sweep lambda <- lambda + C_alpha^{-T}(g - C^T lambda).
 * g_last_dev [B][N], lambda_dev [B][L][M][N] (output; initialised to zero).
 * Stop rule: ||lambda_1^{k+1} - lambda_1^k||_inf <= tol (the first step carries
 * the largest round-off in the transposed sweep) or max_iter. Alpha rule as
 * in aao_solve with ||g||_inf in gamma. */
aao_status aao_adjoint_solve(aao_plan_t plan, const double* g_last_dev, double* lambda_dev,
                             const double* alphas, int n_alphas, double m0, double tol,
                             int max_iter, aao_solve_info* info);

/* Gradients of J = 1/2 ||u_{L,M} - u_target||^2 given the forward solution
 * u_dev and the adjoint lambda_dev: grad_u0 = sum_m lambda_{1,m} [B][N];
 * grad_nu[b] = dT sum_l lambda_l^T (Q (x) dA/dnu) u_l [B] (needs dcoef_dnu). */
aao_status aao_grad(aao_plan_t plan, const double* u_dev, const double* lambda_dev,
                    double* grad_u0_dev, double* grad_nu_dev);

/* Row a3 alone: solve (I - shift_s A) x_s = b_s for S systems of length N in
 * the plan's inner solver and precision.  shifts: host, 2*S doubles (re, im);
 * b_dev, x_dev: device complex128, [S][N] interleaved (re, im).  S must not
 * exceed B*(L/2+1)*M.  iters (nullable host out, S ints): iterations used. */
aao_status aao_shifted_solve(aao_plan_t plan, int S, const double* shifts, const double* b_dev,
                             double* x_dev, int* iters);

/* Kernel statistics (cumulative since the last reset) and event timing. */
aao_status aao_set_timing(aao_plan_t plan, int on);
aao_status aao_get_stats(aao_plan_t plan, aao_kernel_stats* out);
aao_status aao_reset_stats(aao_plan_t plan);
const char* aao_kernel_name(int kernel_class);

/* Per-alpha host tables for inspection: d_j, r_j (eq. (QGL)) and the
 * eigenvalues d_jm of Q G_j^{-1} for the L/2+1 frequencies j, plus the largest
 * condition number of S_j.  d, r: 2*(L/2+1) doubles; djm: 2*(L/2+1)*M doubles.
 * Any output may be NULL. */
aao_status aao_tables(aao_plan_t plan, double alpha, double* d, double* r, double* djm,
                      double* cond_max);

/* Collocation nodes and Q (row-major M x M) the plan uses. */
aao_status aao_collocation(aao_plan_t plan, double* nodes, double* Q);

const char* aao_last_error(void);
void aao_destroy(aao_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* AAO_H */
