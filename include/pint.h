/*
 * pint.h -- C ABI of the MI355X (gfx950) parallel-in-time BDF-k / CQ-BDF-k
 * solver: one waveform-relaxation (WR) sweep solved by diagonalization in time.
 *
 * Method: S. Wu and Z. Zhou, "A parallel-in-time algorithm for high-order BDF
 * methods for diffusion and subdiffusion equations" (arXiv 2007.13125).
 *
 * Problem (Sec. 1, eqs. heat and fde): d_t^alpha u + A u = f on (0, T],
 * u(0) = v, with 0 < alpha <= 1 (alpha = 1: heat equation; alpha < 1: Caputo
 * subdiffusion), A = A_h the finite-difference Dirichlet Laplacian on a box.
 *
 * Time discretisation (Sec. 2.1 eq. BDF / Table 1; Sec. 3.1 eq. BDF-frac):
 * corrected BDF-k (alpha = 1) or CQ-BDF-k (alpha < 1), k = 1..6, N uniform
 * steps tau = T/N.  The solver returns the trajectory U^1..U^N of that scheme.
 *
 * Iteration (Sec. 2.2 eq. BDF-iter; Sec. 3.2 eq. BDF-frac-iter): each WR
 * sweep solves the kappa-circulant all-at-once system
 *     tau^{-alpha} (B_k(kappa) (x) I) U_m + (I (x) A_h) U_m = F_{m-1}
 * by Algorithm 1 / Algorithm 2: scale time row q by kappa^{q/N}, FFT along
 * time, solve the N/2+1 shifted systems (d_p tau^{-alpha} + A_h) Q_p = H_p
 * (real data => Hermitian spectrum), inverse FFT, scale by kappa^{-q/N}.
 *
 * Conventions for every entry point:
 *  - Array pointers marked DEVICE are HIP device pointers owned by the caller;
 *    the library never frees them.  Pointers marked HOST are host memory.
 *  - Space-time arrays are row-major [time][dof] in FP64, dof index fastest;
 *    dofs are ordered x fastest, then y, then z.
 *  - Nothing is thrown across the ABI.  A negative status is an error and the
 *    outputs are undefined; PINT_NOT_CONVERGED (> 0) is a warning: U holds
 *    the last iterate and the per-sweep norms written so far are valid.
 *  - pint_last_error() returns a thread-local description of the last error.
 *  - A plan is bound to one HIP stream and one device; plans are not
 *    thread-safe.  All work is enqueued on the plan's stream.
 */
#ifndef PINT_H
#define PINT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PINT_OK = 0,
    PINT_NOT_CONVERGED = 1,   /* max_sweeps reached before tol; outputs valid        */
    PINT_E_ARG = -1,          /* invalid argument (message in pint_last_error)       */
    PINT_E_UNSUPPORTED = -2,  /* valid problem outside what the kernels implement    */
    PINT_E_NOMEM = -3,        /* device allocation failed                            */
    PINT_E_HIP = -4,          /* a HIP runtime call failed                           */
    PINT_E_DIVERGED = -5      /* NaN/Inf in an update, or update growth guard fired  */
} pint_status;

enum { PINT_FP64 = 0,         /* every step in FP64                                  */
       PINT_MIXED = 1 };      /* FFTs and shifted solves in complex FP32; residual,
                                 kappa scalings, eigenvalues, update, norms in FP64   */
enum { PINT_RESIDUAL = 0,     /* U_m = U_{m-1} + P^{-1}(G - T U_{m-1}) (default)     */
       PINT_DIRECT = 1 };     /* U_m = P^{-1} F_{m-1}, the paper's literal form;
                                 FP64 only (PINT_MIXED + PINT_DIRECT is rejected with
                                 PINT_E_UNSUPPORTED: an FP32 right-hand side would put
                                 FP32 rounding into the fixed point)                  */
enum { PINT_NORM_INF = 0,     /* stop on max over space-time of |U_m - U_{m-1}|      */
       PINT_NORM_L2_TERMINAL = 1 }; /* stop on the discrete L2 norm at t = T         */
enum { PINT_INIT_V = 0,       /* U_0^n = v for all n (Thm 2.6 / Thm 3.5)             */
       PINT_INIT_ZERO = 1,    /* U_0 = 0 (the start of Tables 2 and 3)               */
       PINT_INIT_USER = 2 };  /* U_0 is the content of U on entry                    */
enum { PINT_SPACE_FD = 0,     /* finite-difference Dirichlet Laplacian A_h (default)  */
       PINT_SPACE_FEM_P1 = 1 }; /* 1D only: Galerkin P1 elements on the uniform mesh,
                                 the discretisation of Sec. 4's experiments: mass
                                 M_h = h/6 tridiag(1,4,1), stiffness K_h = (1/h)
                                 tridiag(-1,2,-1).  The library solves the system
                                 divided by h, Mt d_t^alpha u + A_h u = Ft with
                                 Mt = M_h/h, A_h = K_h/h (the FD matrix), so:
                                 v holds the nodal values of v_h, and f, fder hold
                                 the scaled loads Ft(t_n)_i = (f(t_n), phi_i)/h and
                                 their time derivatives at 0.  The time schemes,
                                 Table 1 corrections and Algorithms 1/2 are those of
                                 the FD case with Mt on the time-derivative terms;
                                 Step 2 solves (tau^{-alpha} d_p Mt + A_h) Q_p = H_p
                                 (exact per sine mode: Mt has eigenvalues
                                 (2 + cos(j pi h))/3).  Stop-test norms as for FD. */

/* Box (0,len_0) x ... with m[i] interior nodes per direction, h_i = len_i/(m_i+1).
 * dim in 1..3; entries beyond dim are ignored. */
typedef struct {
    int dim;
    int m[3];
    double len[3];
} pint_grid;

typedef struct {
    int k;            /* BDF order 1..6                                              */
    double alpha;     /* 0 < alpha <= 1; alpha == 1 selects the heat equation         */
    double T;         /* final time > 0                                               */
    int N;            /* number of time steps; even, k < N <= 2048                    */
    double kappa;     /* WR relaxation parameter, 0 < kappa < 1                       */
    double tol;       /* stop when the chosen update norm is <= tol (> 0)             */
    int max_sweeps;   /* >= 1                                                         */
    int precision;    /* PINT_FP64 | PINT_MIXED                                       */
    int form;         /* PINT_RESIDUAL | PINT_DIRECT                                  */
    int norm;         /* PINT_NORM_INF | PINT_NORM_L2_TERMINAL                        */
    int init;         /* PINT_INIT_V | PINT_INIT_ZERO | PINT_INIT_USER                */
    int space;        /* PINT_SPACE_FD | PINT_SPACE_FEM_P1 (0 = FD)                    */
} pint_params;

typedef struct pint_plan pint_plan;

/* Create a plan: validates the problem, computes the FP64 setup tables on the
 * host (BDF / CQ weights of Sec. 2.1 eq. bdf-gen and Sec. 3.1 eq. delta, the
 * eigenvalues d_p = sum_j kappa^{j/N} omega_j e^{-2 pi i j p/N} of Lemmas
 * diag-heat / diag-frac, kappa^{+-q/N}, sine eigenvalues of A_h, Table 1) and
 * uploads them (the plan owns these small device tables).
 * hip_stream: a hipStream_t (NULL = default stream) of the current device.
 * Grids: any m_i in 1..2047 per axis (sine transforms of length 2(m_i+1);
 * lengths that are not powers of two take Bluestein's chirp-z form).
 * The plan allocates its small tables only; the workspace comes from the
 * caller (pint_plan_set_workspace), so no later call allocates device memory.
 * Errors: PINT_E_ARG (invalid grid/params, NULL plan), PINT_E_UNSUPPORTED
 * (m_i > 2047, N outside the supported powers of two, mixed precision with
 * the direct form), PINT_E_NOMEM, PINT_E_HIP. */
pint_status pint_plan_create(pint_plan **plan, const pint_grid *grid,
                             const pint_params *params, void *hip_stream);

/* Bytes of device workspace one solve needs (spectrum buffer, source
 * corrections, norm partials).  The caller provides it with
 * pint_plan_set_workspace before pint_bind / pint_solve.  0 for a NULL plan
 * and for batch plans (which own their instances' workspaces). */
size_t pint_plan_workspace_bytes(const pint_plan *plan);

/* Hand the plan a caller-owned DEVICE buffer of at least
 * pint_plan_workspace_bytes() bytes, 256-byte aligned.  The plan uses it until
 * destroyed or given another one (the caller keeps ownership and frees it
 * after pint_plan_destroy).  Errors: PINT_E_ARG (NULL, too small, misaligned,
 * batch plan). */
pint_status pint_plan_set_workspace(pint_plan *plan, void *dev_ptr, size_t bytes);

/* Bind the problem data and compute the starting-step source corrections
 * a_n (f(0) - A_h v) + sum_l b_{l,n} tau^l d^l f/dt^l (0), n < k (Sec. 2.1
 * eq. BDF and Table 1; Sec. 3.1 eq. BDF-frac for alpha < 1).
 *   v    DEVICE [M]          initial value
 *   f    DEVICE [N+1][M]     f(t_0) .. f(t_N); NULL means f == 0
 *   fder DEVICE [k-2][M]     d^l f/dt^l (0), l = 1..k-2; NULL means zero
 * The pointers must stay valid while the plan sweeps.  Asynchronous.
 * Errors: PINT_E_ARG (NULL v, no workspace set, batch plan), PINT_E_HIP. */
pint_status pint_bind(pint_plan *plan, const double *v, const double *f, const double *fder);

/* Set U (DEVICE [N][M]) to the initial iterate selected by params.init
 * (INIT_USER leaves it untouched): U_0^n = v as in Thm 2.6 / Thm 3.5, or
 * U_0 = 0 as in the runs of Sec. 4.  Requires pint_bind.  Asynchronous. */
pint_status pint_init_iterate(pint_plan *plan, double *U);

/* Run exactly nsweeps WR sweeps on U (DEVICE [N][M], in/out) with the bound
 * data, asynchronously on the plan's stream, with no host synchronisation.
 * One sweep is one step of the iteration eq. BDF-iter (Sec. 2.2; eq.
 * BDF-frac-iter of Sec. 3.2 for alpha < 1), solved by Algorithm 1 (resp. 2).
 * dev_norms (DEVICE [nsweeps][2], may be NULL) receives per sweep
 * { max |U_m - U_{m-1}|, (h^d sum (U_m^N - U_{m-1}^N)^2)^{1/2} }.
 * Errors: PINT_E_ARG (not bound, NULL U, nsweeps < 0), PINT_E_HIP. */
pint_status pint_sweeps(pint_plan *plan, double *U, int nsweeps, double *dev_norms);

/* Instrumented sweeps for measurement: runs nsweeps sweeps exactly like
 * pint_sweeps, with a HIP event pair recorded on the plan's stream around
 * every kernel launch, then waits for the stream.
 *   ms    HOST [max_slots]: average device milliseconds per sweep of each launch
 *         slot (forward time FFT, each spatial pass, inverse time FFT, norm
 *         reduction, in launch order)
 *   names HOST [max_slots] (may be NULL): slot names, valid until the next call
 *         on this thread
 * Returns the number of slots per sweep (> 0), or a negative pint_status. */
int pint_profile_sweeps(pint_plan *plan, double *U, int nsweeps, double *ms, const char **names,
                        int max_slots);

/* Full solve: bind, initial iterate, then WR sweeps (eq. BDF-iter, Algorithm
 * 1; eq. BDF-frac-iter, Algorithm 2) until the chosen update norm is <= tol
 * (the stopping rule of Sec. 4) or max_sweeps is reached (host-side stop test
 * after every sweep).  Allocates no device memory (the workspace is the
 * caller's).
 *   v, f, fder as in pint_bind; U DEVICE [N][M] (input too for INIT_USER).
 *   upd     HOST [max_sweeps]: the max-norm update per sweep (may be NULL)
 *   upd_l2T HOST [max_sweeps]: the terminal L2_h update per sweep (may be NULL)
 *   sweeps  HOST: number of sweeps performed (may be NULL)
 * Returns PINT_OK, PINT_NOT_CONVERGED, or an error; PINT_E_DIVERGED when an
 * update is NaN/Inf or grows in two consecutive sweeps after the first. */
pint_status pint_solve(pint_plan *plan, const double *v, const double *f, const double *fder,
                       double *U, double *upd, double *upd_l2T, int *sweeps);

/* Windowed solve (the time-window remark that closes Sec. 4's Example 4): the
 * interval (0, nwin T] is cut into nwin windows of the plan's length T and N
 * steps, solved one after another, each by pint_solve's WR sweeps (parallel
 * in time inside the window); window w starts from the last level of window
 * w-1 (from v for w = 0) and the corrected scheme restarts there (its Table 1
 * rows use f and d^l f/dt^l at the window's start).  For alpha < 1 a restart
 * also drops the memory of the earlier windows: the windowed scheme is what is
 * computed.  The space-time state of one window is what must fit the device.
 *   v      DEVICE [M]
 *   f      DEVICE [nwin N + 1][M], f(t_0) .. f(t_{nwin N}); NULL => f == 0
 *   fder   DEVICE [nwin][k-2][M], d^l f/dt^l at each window's start; NULL => 0
 *   U      DEVICE [nwin N][M] out
 *   upd    HOST [nwin][max_sweeps] per-window max-norm updates (may be NULL)
 *   sweeps HOST [nwin] (may be NULL)
 * Returns PINT_OK, PINT_NOT_CONVERGED (some window hit max_sweeps; all windows
 * are solved), or the first error. */
pint_status pint_solve_windows(pint_plan *plan, int nwin, const double *v, const double *f,
                               const double *fder, double *U, double *upd, int *sweeps);

/* The sequential-in-time solver: the corrected BDF-k / CQ-BDF-k scheme of
 * the plan (Sec. 2.1 eq. BDF; Sec. 3.1 eq. BDF-frac; the stepping of the
 * cost paragraph of Sec. 3.2) stepped one level after another, each step one
 * shifted spatial solve (omega_0 tau^{-alpha} + A_h) U^n = rhs_n by the sweep's
 * spatial passes.  This is the trajectory every WR sweep converges to, and
 * the in-GPU baseline of the parallel-in-time method: O(k M N) history work
 * for BDF-k, O(M N^2) for CQ-BDF-k, N dependent steps.  v, f, fder as in
 * pint_bind (DEVICE); U DEVICE [N][M] out.  FP64 plans only
 * (PINT_E_UNSUPPORTED for mixed).  Asynchronous on the plan's stream; uses
 * the plan's workspace.  Errors: PINT_E_ARG (NULL, batch plan, no
 * workspace), PINT_E_HIP. */
pint_status pint_sequential_solve(pint_plan *plan, const double *v, const double *f, const double *fder,
                                  double *U);

/* Semilinear problems d_t^alpha u + A u + g(u) = f, u(0) = v, with the cubic
 * g(u) = c3 u^3 + c1 u (Example 4's Allen-Cahn term for c3 = 1/eps^2,
 * c1 = -1/eps^2), by Algorithm 3 of Sec. 4 (extension to nonlinear problems):
 * the scheme of eq. BDF-CQ-m-r (the plan's k, alpha, N, T, with the Table 1
 * rows carrying f(0) - A_h v - g(v)) is solved by the modified Newton
 * iteration of eq. BDF-CQ-m-r-N, U_l = U_{l-1} + W_l from U_0^n = v, whose
 * linearised system uses the time-averaged Jacobian g'(Ubar_{l-1}) (Ubar the
 * mean of U_{l-1} over the N levels) and is solved by the WR sweeps of eq.
 * BDF-CQ-m-r-N-w from W_{l,0} = 0, each by Algorithm 1/2 with the spatial
 * operator A_h + diag(g'(Ubar)) (PCR/Thomas per frequency), until
 * max |W_{l,m} - W_{l,m-1}| < params.tol or params.max_sweeps sweeps.
 * 1D grids, FP64, residual form (the plan's params; PINT_E_UNSUPPORTED
 * otherwise).  v, f, fder as in pint_bind (DEVICE); U DEVICE [N][M] out.
 *   newton_steps  >= 1: Newton steps at most; stops early once max |W_l| <= newton_tol
 *   inner_sweeps  HOST [newton_steps] (may be NULL): WR sweeps of each step
 *   newton_upd    HOST [newton_steps] (may be NULL): max |W_l| of each step
 *   steps_done    HOST (may be NULL)
 * Returns PINT_OK when max |W_l| <= newton_tol, PINT_NOT_CONVERGED when the
 * step budget (or an inner budget) ran out with valid outputs, PINT_E_DIVERGED
 * on a non-finite update.  The workspace is the plan's (no allocation). */
pint_status pint_nonlinear_solve(pint_plan *plan, double c3, double c1, const double *v, const double *f,
                                 const double *fder, double *U, int newton_steps, double newton_tol,
                                 int *inner_sweeps, double *newton_upd, int *steps_done);

/* pint_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sweeps (same kernels, same results) with the plan's workspace taken
 * from a static device array of the library (64 MiB per device, held until
 * the process ends) instead of the caller's buffer.  Arguments and results as
 * pint_solve; the plan needs no pint_plan_set_workspace, is not autotuned,
 * and is left unbound afterwards (its own workspace, if any, is kept).
 * Allocates nothing: no hipMalloc, no hipFree.  All calls on one device share
 * the one array, so calls that overlap in time on one device (other threads,
 * other streams) race; the array keeps the last call's contents, and every
 * value a call reads from it is written by that call first.
 * Errors: PINT_E_ARG (NULL plan/v/U, batch plan, or a plan whose
 * pint_plan_workspace_bytes exceeds 64 MiB), PINT_E_UNSUPPORTED (device index
 * above 63), PINT_E_HIP (including a failed lookup of the array's address). */
pint_status pint_solve_noalloc(pint_plan *plan, const double *v, const double *f, const double *fder,
                               double *U, double *upd, double *upd_l2T, int *sweeps);

/* Many independent problems in one plan (each instance with its own grid and
 * params; N, k, alpha, precision may all differ).  Every instance is validated
 * as in pint_plan_create and gets its own tables and workspace, which this
 * call allocates (pint_batch_solve allocates nothing).  pint_batch_solve
 * sweeps the 1D instances together: each pass of a sweep (residual, time DFT
 * of general length, a Thomas solve per retained frequency, inverse DFT and
 * update, norms) is one launch over all active instances of a class of
 * (precision, time transform length), and after every sweep one host stop
 * test per instance (the rules of pint_solve) drops the finished ones; the
 * instances of dimension 2 and 3 are solved one after another on the plan's
 * stream through the single-plan path.  count >= 1; grids/params are HOST arrays of count
 * entries.  Errors: as pint_plan_create (the message names the instance). */
pint_status pint_batch_plan_create(pint_plan **plan, int count, const pint_grid *grids,
                                   const pint_params *params, void *hip_stream);

/* Batch solve.  v, f, fder, U: HOST arrays of count DEVICE pointers with the
 * meaning of pint_solve (f and fder entries, or the f/fder arrays themselves,
 * may be NULL).  upd: HOST [count][stride] (may be NULL): instance i writes its
 * max-norm updates to upd[i*stride .. i*stride + sweeps[i]); stride must be
 * at least every instance's max_sweeps (PINT_E_ARG otherwise).  sweeps: HOST
 * [count] (may be NULL).  Each instance stops at its own tol, max_sweeps or
 * divergence.  Returns PINT_OK if every instance converged,
 * PINT_NOT_CONVERGED if one hit max_sweeps, PINT_E_DIVERGED if one diverged
 * (the others still finish). */
pint_status pint_batch_solve(pint_plan *plan, const double *const *v, const double *const *f,
                             const double *const *fder, double *const *U, double *upd, int stride,
                             int *sweeps);

/* Autotuning of the kernels' tile and split choices (the batching row of the
 * method's GPU mapping: FFT radix and tile shapes, PCR/Thomas split).  Four
 * knobs, each 0 = the built-in choice:
 *   [0] forward kernel: BDF-k residual 2D/3D sweeps 0 split (a residual
 *       kernel marching along time, then a time-FFT kernel), 1 march with the
 *       time-FFT tile, 2 one workgroup per tile, 3 half-width wide-tile march
 *       with two workgroups per CU, 4 wide-tile march along the outer axis; CQ
 *       sweeps 0 y-march with radix <= 8 transforms, 1 y-march with radix <= 16,
 *       2 (3, 4) persistent one-tile-at-a-time kernel (a choice that does not
 *       apply to the problem falls back to the next one that does; sweeps whose
 *       time axis is not a power of two have one forward path);
 *   [1] rows per workgroup of the x sine pass: 0 built-in, 1 half as many;
 *   [2] column tile of the y/z passes: 0 built-in, 1 the other width;
 *   [3] 1D grids with 2(m+1) not a power of two: 0 sine solve (Bluestein),
 *       1 PCR/Thomas with the built-in split, 2 PCR/Thomas with more PCR
 *       lanes.  Not tuned (the PCR stage loses accuracy on the near-singular
 *       shifted Laplacians, ~eps (m+1)^2 per sweep); only pinned.
 * Tuning times every value of a knob that launches a different kernel for the
 * problem (reps launches, in three interleaved rounds, best round kept) on the
 * plan's own workspace (the forward kernels read U, nothing writes it), and
 * keeps the fastest; a value other than 0 must be at least 3% faster than the
 * built-in one.  It synchronises the plan's stream.  Results are unchanged up
 * to rounding by the choice.
 *
 * pint_plan_set_autotune: reps > 0 makes pint_solve (pint_batch_solve: every
 * instance) tune once, after binding and the initial iterate, before its first
 * sweep; 0 (the default) keeps the current choices.  Errors: PINT_E_ARG
 * (NULL plan, reps outside 0..1000). */
pint_status pint_plan_set_autotune(pint_plan *plan, int reps);

/* Tune a single plan now.  Requires pint_bind; U: DEVICE [N][M], read only
 * (its values only affect timing); reps in 1..1000.  Errors: PINT_E_ARG (NULL
 * plan or U, not bound, batch plan), PINT_E_HIP. */
pint_status pint_plan_tune(pint_plan *plan, const double *U, int reps);

/* The variants in use: choices HOST [4] (the knobs above).  instance selects a
 * batch member; it must be 0 for a single plan.  Errors: PINT_E_ARG. */
pint_status pint_plan_get_variants(const pint_plan *plan, int instance, int *choices);

/* Pin the variants (choices HOST [4], each within its knob's range), e.g. the
 * result of an earlier tuning run; a pinned plan is not tuned again.
 * Errors: PINT_E_ARG (NULL, out of range, bad instance). */
pint_status pint_plan_set_variants(pint_plan *plan, int instance, const int *choices);

/* Release the plan, its tables and any workspace it allocated itself.
 * Waits for the plan's stream.  NULL is accepted. */
pint_status pint_plan_destroy(pint_plan *plan);

/* Number of space-time unknowns N * M of a plan (sum over a batch). */
long long pint_plan_unknowns(const pint_plan *plan);

const char *pint_status_str(pint_status s);
const char *pint_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PINT_H */
