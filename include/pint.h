/*
 * pint.h — C interface of libpint, a parallel-in-time Newton ODE solver for
 * AMD MI355X (gfx950).
 *
 * Method (Iacob, Razavi, Sarkka, arXiv 2511.01465, Sec. 3.2): the trajectory
 * xi = (x_1..x_T) of the one-step scheme x_n = Phi(x_{n-1}) (classic RK4,
 * eq. explicit-rk) is the root of h(xi) = [x_n - Phi(x_{n-1})]_{n=1..T}
 * (eq. root-finding-problem).  Each Newton iteration (eqs. newton-step,
 * newton-iterates) needs dx_n = J(x_{n-1}) dx_{n-1} - h_n, dx_1 = -h_1
 * (eq. newton-step-recursion), an affine recursion evaluated as a prefix
 * scan (eq. prefix-sum) under the composition of eq. assoc-operator:
 *     (A2, b2) o (A1, b1) = (A2 A1, A2 b1 + b2)   (A1,b1 applied first).
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers unless stated otherwise, owned
 *     by the caller.  The library never allocates or frees caller memory and
 *     allocates no device memory on the solve path: scratch comes from the
 *     caller's workspace `ws` (size from pint_workspace_bytes), 256-byte
 *     aligned.
 *   - Layouts are row-major and packed: a state is d contiguous scalars; a
 *     trajectory of instance b is T_b consecutive states x_1..x_T (x_0 is
 *     NOT stored; it is the x0 input); a batch of trajectories is packed one
 *     instance after the other (CSR by `T_off`).  A matrix is d*d scalars,
 *     row-major.  Scalars are double (PINT_F64) or float (PINT_F32) as
 *     selected by `dtype`; residuals and tolerances are always double.
 *   - Every call is asynchronous on `stream` (0 = the null stream) unless
 *     its comment says otherwise; outputs are valid once the stream has
 *     synchronised.  Calls on one workspace must not overlap.
 *   - Errors are return codes; nothing aborts or throws.  Argument errors
 *     are detected on the host before anything is launched.
 */
#ifndef PINT_H_
#define PINT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pint_stream_t; /* a hipStream_t */

typedef enum {
  PINT_OK = 0,
  PINT_ERR_INVALID_ARG = 1, /* bad argument; nothing was launched          */
  PINT_ERR_DEVICE = 2,      /* a HIP runtime call failed                   */
  PINT_ERR_WORKSPACE = 3,   /* workspace missing or smaller than required  */
  PINT_NOT_CONVERGED = 4,   /* per instance: max_iter reached; last iterate returned */
  PINT_NONFINITE = 5,       /* per instance: a non-finite residual or state stopped Newton */
  PINT_ERR_UNSUPPORTED = 6  /* system / dimension / dtype combination not built */
} pint_status;

typedef enum { PINT_F64 = 0, PINT_F32 = 1 } pint_dtype;

/* Built-in vector fields f(x; theta).  Parameter vectors theta, in order:
 *   LINEAR     f = M x                                  theta = M (d*d, row-major)
 *   LOGISTIC   d=1: f = r x (1 - x/K)                   theta = (r, K)          [Sec. 4.1, eq. logistic]
 *   VDP        d=2: (x, v)' = (v, mu (1-x^2) v - x)     theta = (mu)            [Sec. 4.1, eq. vdp]
 *   CARTPOLE   d=4: (p, th, p', th')                    theta = (g, l, m_c, m_p)[Sec. 4.1, eq. cartpole, with th'^2]
 *   LORENZ63   d=3                                      theta = (sigma, rho, beta)
 *   LORENZ96   d>=4: f_i = (x_{i+1}-x_{i-2}) x_{i-1} - x_i + F   theta = (F)
 *   KURAMOTO   f_i = w_i + K sum_j sin(x_j - x_i)       theta = (K, w_1..w_d)
 *   ROBERTSON  d=3: (-k1 y1 + k3 y2 y3, k1 y1 - k2 y2^2 - k3 y2 y3, k2 y2^2)
 *                                                       theta = (k1, k2, k3)    [Sec. 4.2, eq. robertson]
 */
typedef enum {
  PINT_SYS_LINEAR = 0,
  PINT_SYS_LOGISTIC = 1,
  PINT_SYS_VDP = 2,
  PINT_SYS_CARTPOLE = 3,
  PINT_SYS_LORENZ63 = 4,
  PINT_SYS_LORENZ96 = 5,
  PINT_SYS_KURAMOTO = 6,
  PINT_SYS_ROBERTSON = 7
} pint_system_id;

/* One-step rule x_n = step(x_{n-1}) whose trajectory is solved for.
 *   RK4          classic explicit Runge-Kutta, x_n = Phi(x_{n-1})
 *                (eqs. explicit-ode, explicit-rk); residual
 *                h_n = x_n - Phi(x_{n-1}) (eq. root-finding-problem).
 *   BACKWARD_EULER, TRAPEZOIDAL: the implicit rules x_n = x_{n-1} + g with
 *                g = dt f(x_n) (eq. implicit-euler) or
 *                g = dt/2 (f(x_{n-1}) + f(x_n)) (Sec. 3.4, eq. implicit-ode).
 *                Newton's step is eq. newton-step-implicit-recursion; the
 *                residual the solver tests, reports and returns from
 *                pint_residual is (I - dg/dx_n)^{-1} (x_n - x_{n-1} - g), the
 *                quantity the paper reports for its implicit solver
 *                (Sec. 4.2, Figure 8).  Systems of dimension d <= 4 only
 *                (the batched small solver); others return
 *                PINT_ERR_UNSUPPORTED, as does pint_adjoint. */
typedef enum { PINT_RK4 = 0, PINT_BACKWARD_EULER = 1, PINT_TRAPEZOIDAL = 2 } pint_method;

typedef struct {
  int32_t system;        /* pint_system_id                                      */
  int32_t d;             /* state dimension                                     */
  int32_t n_params;      /* must equal pint_n_params(system, d)                 */
  int32_t params_shared; /* 1: one theta for every instance; 0: [B][n_params]   */
  const void* params;    /* device pointer, solve dtype                         */
  int32_t method;        /* pint_method (0, the RK4 rule, when zero-filled)     */
  int32_t reserved;      /* must be 0                                           */
} pint_system;

typedef struct {
  int32_t dtype;     /* pint_dtype                                               */
  int32_t guess;     /* 0: initial iterate x_n = x0 for all n; 1: traj holds it  */
  int64_t max_iter;  /* maximum Newton updates; <= 0 means T + 1                 */
  int64_t window;    /* 0: the paper's plain Newton over all T steps;            */
                     /* W >= 1: windowed safeguard (see pint_solve_varlen)       */
  double tol;        /* stop when ||h(xi)||_inf < tol (strict)                   */
  double guard;      /* windowed mode: an updated state with |x| > guard (or     */
                     /* non-finite) ends the accepted part of the update         */
  int32_t tile;      /* scan tile / chunk hint; 0 = library default.  For the   */
                     /* cooperative small-d solve (below): steps per workgroup, */
                     /* rounded up to whole chunks of 256; 0 = one chunk        */
  int32_t flags;     /* reserved, must be 0                                      */
  /* Launch shape of the batched small-d solver (d <= 4); results do not
   * depend on them.  Dense dimensions require 0 / 0 / NULL. */
  int32_t block;          /* threads per workgroup: 64, 128 or 256; 0 = 256     */
  int32_t wg_per_cu;      /* persistent workgroups per compute unit, 1..16;     */
                          /* 0 = 4                                              */
  const int64_t* order;   /* device [B]: a permutation of 0..B-1, the order in  */
                          /* which instances are taken from the work queue      */
                          /* (e.g. longest first); entries outside [0, B) are   */
                          /* skipped; NULL = 0, 1, ..., B-1                     */
} pint_options;

/* Bound of the device-side waits of the cooperative solvers (pint_solve of
 * dense dimensions in windowed mode, and of a few long small-d instances in
 * plain mode), in polls of the awaited flag, each followed by the shortest
 * sleep.  When a wait gives up, every workgroup of the instance leaves its
 * Newton loop at its next wait, and the instance's status is
 * PINT_ERR_DEVICE (its result is unreliable).  polls = 0 makes every such
 * wait give up at once, without polling: callers that test the error path
 * force it this way.  Process-wide; applies to launches enqueued after the
 * call; the default is PINT_WAIT_LIMIT_DEFAULT. */
#define PINT_WAIT_LIMIT_DEFAULT 268435456ull
void pint_set_wait_limit(uint64_t polls);

/* Test hook of the decoupled-lookback scans (pint_affine_scan, its
 * no-alloc variant, pint_affine_scan_band and the adjoint's scans): with
 * sleeps > 0, tile t sleeps `sleeps` short intervals before it publishes its
 * aggregate when t % 3 == 1, and before it publishes its inclusive prefix
 * when t % 3 == 2, so that successors meet unpublished and aggregate-only
 * predecessors and take the longer lookback paths.  Results stay correct
 * (up to the rounding of a different composition order); only the timing
 * changes.  Process-wide; applies to launches enqueued after the call;
 * 0 (the default) turns it off.  The lookback's own bounded wait still
 * applies: keep sleeps small (a few hundred at most). */
void pint_set_scan_delay(uint32_t sleeps);

/* The pipelined kernels, on != 0 by default:
 *  - windowed solves of the dense systems (pint_solve of PINT_SYS_LORENZ96
 *    with d = 40, or PINT_SYS_KURAMOTO with d = 64 or 128; window >= 1;
 *    batches of up to as many instances as compute units): the pipelined
 *    solver, in which consecutive Newton updates overlap in time on
 *    separate workgroups (up to 16 per instance; with one, an instance's
 *    updates run in turn, their elements kept on chip); 0 the solver that
 *    applies one update at a time.  Both compute the same iteration (same windows, same accepted
 *    updates, the same states bit for bit).
 *  - pint_adjoint of Lorenz-96: the fused reverse pass, elements built
 *    inside the recursion; 0 the two-kernel path (elements stored per
 *    segment, then the banded scan).  Same recursion, summation order
 *    aside.
 * Process-wide; applies to launches enqueued (and workspace queries made)
 * after the call. */
void pint_set_dense_pipeline(int on);

/* Number of parameters of `system` at dimension d, or -1 if not allowed. */
int pint_n_params(int32_t system, int32_t d);

/* Human-readable name of a status code (static storage). */
const char* pint_status_string(int32_t status);

/* 1 if the (system, d, dtype) combination is compiled into the library. */
int pint_supported(int32_t system, int32_t d, int32_t dtype);

/* Bytes of workspace needed by pint_solve / pint_solve_varlen for B
 * instances with sum T = T_total and max T = T_max. */
size_t pint_workspace_bytes(const pint_system* sys, int64_t B, int64_t T_total,
                            int64_t T_max, const pint_options* opts);

/*
 * pint_solve_varlen — Newton's method on h(xi) = 0 for B independent
 * instances with their own horizons (Sec. 3.2; the per-instance loop,
 * residual test and window logic all run on the device, one persistent
 * launch for the whole batch).
 *
 *   x0      [B][d]            initial states x_0
 *   T_off   [B+1] int64       CSR offsets: instance b owns steps
 *                             T_off[b]..T_off[b+1]-1 of traj; T_off[0] = 0
 *   T_max   host int64        max_b (T_off[b+1]-T_off[b]) (sizes the launch)
 *   traj    [T_off[B]][d]     in: the initial iterate if opts->guess = 1;
 *                             out: the last iterate (x_1..x_T per instance)
 *   iters   [B] int64         Newton updates applied (the paper's K is iters+1)
 *   resid   [B] double        ||h||_inf of the returned iterate
 *   status  [B] int32         PINT_OK / PINT_NOT_CONVERGED / PINT_NONFINITE, or
 *                             PINT_ERR_DEVICE if a cooperative launch's bounded
 *                             device-side wait gave up (result unreliable)
 *
 * Plain mode (window 0): iteration k evaluates h over all steps, stops if
 * ||h||_inf < tol, otherwise applies the full Newton step.  This is the
 * paper's method.  Windowed mode (window W >= 1, also when W >= T_b), a
 * safeguard the paper does not state: with p the first step whose
 * ||h_p||_inf >= tol, the Newton step is computed from dx_{p-1} = 0 (so
 * dx_p = -h_p for RK4) over steps p..min(T_b, p+W-1) only, steps
 * before p are left as they are, and the update is accepted only below the
 * first updated state that is non-finite or exceeds `guard`.  Both modes have
 * the same fixed point (the sequential trajectory).
 * Returns PINT_OK when launched; per-instance outcomes are in `status`.
 */
pint_status pint_solve_varlen(const pint_system* sys, int64_t B, const void* x0,
                              double dt, const int64_t* T_off, int64_t T_max,
                              const pint_options* opts, void* traj,
                              int64_t* iters, double* resid, int32_t* status,
                              void* ws, size_t ws_bytes, pint_stream_t stream);

/* pint_solve — as pint_solve_varlen with every instance of length T
 * (traj is [B][T][d]).  An instance of dense dimension runs on several
 * workgroups at once (cooperative launch with device-side barriers between
 * them).  So does a small-d instance in plain mode (window 0) when the
 * horizon spans at least four chunks of 256 steps and the B * G workgroups
 * fit on the device at once: each workgroup owns a contiguous range of
 * steps, evaluates its elements in registers and exchanges only range
 * compositions and boundary states with the others, one grid barrier per
 * Newton iteration (the workspace from pint_workspace_bytes covers it).
 * Results follow the same plain-mode rules.  Like every entry point, the
 * call only enqueues work. */
pint_status pint_solve(const pint_system* sys, int64_t B, const void* x0,
                       double dt, int64_t T, const pint_options* opts,
                       void* traj, int64_t* iters, double* resid,
                       int32_t* status, void* ws, size_t ws_bytes,
                       pint_stream_t stream);

/*
 * Executable graph of one batched solve (spec batching requirement:
 * thousands of uneven-horizon instances in one persistent launch replayed
 * from a HIP graph).  pint_graph_capture_varlen takes the arguments of
 * pint_solve_varlen, records the launches that call would enqueue (a fill
 * kernel that resets the work queue, then the persistent solver; no memset
 * or memcpy nodes) and instantiates them.  Every pint_graph_launch then
 * repeats that solve on the same buffers, asynchronously on `stream`: the
 * caller updates x0 / params / T_off / traj contents in place between
 * launches, never the pointers or B.  Small dimensions (d <= 4) only;
 * dense dimensions return PINT_ERR_UNSUPPORTED.  The graph owns no caller
 * memory; pint_graph_destroy frees the graph objects only.  Errors: the
 * argument checks of pint_solve_varlen, PINT_ERR_DEVICE if capture or
 * instantiation fails (*out is then NULL).
 */
typedef struct pint_graph_s* pint_graph;
pint_status pint_graph_capture_varlen(const pint_system* sys, int64_t B, const void* x0,
                                      double dt, const int64_t* T_off, int64_t T_max,
                                      const pint_options* opts, void* traj,
                                      int64_t* iters, double* resid, int32_t* status,
                                      void* ws, size_t ws_bytes, pint_graph* out);
pint_status pint_graph_launch(pint_graph graph, pint_stream_t stream);
pint_status pint_graph_destroy(pint_graph graph);

/* pint_seq_integrate — the sequential comparator x_n = Phi(x_{n-1}),
 * n = 1..T_b, for every instance (eq. explicit-ode with classic RK4; for an
 * implicit sys->method each step is solved by Newton's method from
 * x_{n-1} until the correction is within a few ulps of |x_n|, at most 100
 * corrections).  T_off as in pint_solve_varlen; traj [T_off[B]][d] is
 * written. */
pint_status pint_seq_integrate(const pint_system* sys, int64_t B,
                               const void* x0, double dt, const int64_t* T_off,
                               int64_t T_max, int32_t dtype, void* traj,
                               pint_stream_t stream);

/*
 * pint_parareal — Parareal, the method the paper compares against (Sec. 2.2,
 * eqs. parareal-init, fine-integrator, coarse-integrator), for B
 * independent instances split the same way: M windows of S fine steps.  The
 * coarse integrator G is ONE step of sys->method with step size S*dt; the
 * fine integrator F is S steps of size dt.  Initial coarse sweep
 * x_{m+1} = G(x_m) from x_0 = x0; then per iteration the fine sweep
 * F_m = F(x_m) over all windows in parallel, the error
 * R = max_m ||x_{m+1} - F_m||_inf (the paper's R^(k), Sec. 4), a stop when
 * R < opts->tol (strict), else the sequential correction
 * x_{m+1} <- G(x_m new) + F_m - G(x_m old).  The paper takes
 * M = floor(sqrt(N)) and S = floor(N / M) for N steps (the caller chooses).
 *   x0      [B][d]
 *   traj    [B][M*S][d]   out: the dense trajectory of the last fine sweep
 *                         (traj[b][m*S + j] = state after j+1 fine steps of
 *                         window m)
 *   iters   [B] int64     K, the number of fine sweeps (= R evaluations)
 *   resid   [B] double    the last R
 *   status  [B] int32     PINT_OK, PINT_NOT_CONVERGED (max_iter sweeps), or
 *                         PINT_NONFINITE (a non-finite R)
 *   hist    [B][max_iter] double, R of each sweep (entries past K are not
 *                         written), or NULL
 * opts: dtype, tol, max_iter (fine sweeps; <= 0 means M + 1, after which
 * Parareal is exact); every other field must be 0 / NULL (guard is
 * ignored).  Systems of dimension d <= 4 only (PINT_ERR_UNSUPPORTED
 * otherwise).  One workgroup per instance; workspace from
 * pint_parareal_workspace_bytes ((3M + 1) states per instance).  M or S = 0
 * gives K = 0, R = 0, PINT_OK and writes no trajectory.
 */
size_t pint_parareal_workspace_bytes(const pint_system* sys, int64_t B, int64_t M,
                                     int32_t dtype);
pint_status pint_parareal(const pint_system* sys, int64_t B, const void* x0, double dt,
                          int64_t M, int64_t S, const pint_options* opts, void* traj,
                          int64_t* iters, double* resid, int32_t* status, double* hist,
                          void* ws, size_t ws_bytes, pint_stream_t stream);

/* pint_residual — h_n = x_n - Phi(x_{n-1}) for every step of a uniform
 * batch (eq. root-finding-problem; the scaled implicit residual of
 * pint_method for the implicit rules): h [B][T][d] (may be NULL), and
 * hmax [B] (double) the infinity norm per instance (+inf if any entry is
 * non-finite). */
pint_status pint_residual(const pint_system* sys, int64_t B, const void* x0,
                          double dt, int64_t T, int32_t dtype, const void* traj,
                          void* h, double* hmax, pint_stream_t stream);

/* pint_elements — the Newton-step elements of a uniform batch:
 * A [B][T][d][d] with A_n = dPhi/dx at x_n (n = 0..T-1, x_0 = x0) and
 * b [B][T][d] with b_n = -h_{n+1}, so that dx_{n+1} = A_n dx_n + b_n with
 * dx_0 = 0 (eqs. newton-step-recursion, initialization).  For the implicit
 * rules (eq. newton-step-implicit-recursion), with H = I - dg/dx_{n+1} and
 * g = g(x_n, x_{n+1}): A_n = H^{-1} (I + dg/dx_n), b_n = -H^{-1} h_{n+1}. */
pint_status pint_elements(const pint_system* sys, int64_t B, const void* x0,
                          double dt, int64_t T, int32_t dtype,
                          const void* traj, void* A, void* b,
                          pint_stream_t stream);

/* pint_affine_scan — the prefix scan of eq. prefix-sum for affine
 * elements (eq. linear-model): for each of B independent sequences of N
 * elements, z_{n+1} = A_n z_n + b_n from z_0 = z0 (z0 [B][d], or NULL for
 * zero), written as z [B][N][d] (z[n] = z_{n+1}).  A [B][N][d][d],
 * b [B][N][d].  Single-pass decoupled-lookback scan over tiles of `tile`
 * elements (0 = default); workspace from pint_scan_workspace_bytes.
 * Supported d: 1..8, 16, 32, 40, 64, 128.  z must not overlap A, b, z0 or
 * the workspace (the elements are read twice, once per pass).  Returns
 * PINT_OK at once when B or N is 0; PINT_ERR_INVALID_ARG for d < 1,
 * negative sizes or tile, another dtype, or a NULL A, b or z;
 * PINT_ERR_UNSUPPORTED for a d outside the list; PINT_ERR_WORKSPACE when
 * ws is NULL or smaller than the query.  Each tile's wait for its
 * predecessors is bounded (2^24 polls); a wait that gives up sets the 32-bit
 * word at byte offset 4 of ws to nonzero (it is zeroed at the start of every
 * call) and the result is then unreliable: a caller that syncs can read it. */
size_t pint_scan_workspace_bytes(int32_t d, int64_t B, int64_t N, int32_t tile,
                                 int32_t dtype);
pint_status pint_affine_scan(int32_t d, int64_t B, int64_t N, int32_t dtype,
                             const void* A, const void* b, const void* z0,
                             void* z, int32_t tile, void* ws, size_t ws_bytes,
                             pint_stream_t stream);

/*
 * pint_affine_scan_noalloc — pint_affine_scan for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, recursion, outputs and
 * argument checks as pint_affine_scan, without the workspace: the scan's
 * scratch (tile counter, error word, tile flags and payloads, as sized by
 * pint_scan_workspace_bytes) is a fixed device array of
 * PINT_NOALLOC_SCRATCH_BYTES inside the library, one per device, reserved
 * when the library's code is loaded on the device and held until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library call); its first call on a device looks up that
 * device's array address.
 *   err  device uint32, or NULL: receives 0, or 1 if a lookback wait gave up
 *        (the bounded wait of the scan; the result is then unreliable).
 * Returns PINT_ERR_WORKSPACE, before launching anything, when
 * pint_scan_workspace_bytes for these sizes exceeds
 * PINT_NOALLOC_SCRATCH_BYTES (e.g. d = 128 over more than ~120 tiles).
 * Every call on one device shares that device's array: calls that overlap
 * on one device (other streams, other host threads) race and give wrong
 * results.  Calls ordered on one stream are safe: each call first clears
 * what must start at zero, so what an earlier call left there is harmless.
 */
#define PINT_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
pint_status pint_affine_scan_noalloc(int32_t d, int64_t B, int64_t N, int32_t dtype,
                                     const void* A, const void* b, const void* z0, void* z,
                                     int32_t tile, uint32_t* err, pint_stream_t stream);

/* pint_affine_scan_band — pint_affine_scan for elements whose A is
 * cyclically banded: A_n(i, (i + k - boff) mod d) = band_n[i][k] for
 * k < bw, every other entry exactly zero (the RK4 Jacobian of a
 * short-stencil system such as Lorenz-96, eq. lorenz96-model, or its
 * transpose in the adjoint).  Same recursion, output and workspace rules as
 * pint_affine_scan; band [B][N][d][bw] row-major (16-byte aligned for
 * FP64, 8-byte for FP32), b [B][N][d].  The running products of a tile are
 * dense; only the elements are read as bands (d*bw values instead of d*d).
 * Supported shapes: d = 40, bw = 13, boff = 8 (the Lorenz-96 step
 * Jacobian) or 4 (its transpose).  Returns PINT_ERR_UNSUPPORTED for other
 * shapes, PINT_ERR_INVALID_ARG for a misaligned band. */
size_t pint_scan_band_workspace_bytes(int32_t d, int32_t bw, int32_t boff, int64_t B,
                                      int64_t N, int32_t tile, int32_t dtype);
pint_status pint_affine_scan_band(int32_t d, int32_t bw, int32_t boff, int64_t B, int64_t N,
                                  int32_t dtype, const void* band, const void* b,
                                  const void* z0, void* z, int32_t tile, void* ws,
                                  size_t ws_bytes, pint_stream_t stream);

/*
 * pint_adjoint — gradient of a trajectory loss L(x_1..x_T) through the
 * discrete solution map x_n = Phi(x_{n-1}; theta) of a uniform batch:
 *   lambda_T = g_T, lambda_n = g_n + J(x_n)^T lambda_{n+1},
 *   dL/dx0 = J(x_0)^T lambda_1, dL/dtheta = sum_n dPhi/dtheta(x_{n-1})^T lambda_n,
 * i.e. the back substitution H^T lambda = g with the block-bidiagonal H of
 * eq. (jacobian), computed as a reverse-time affine scan over the elements
 * (J_n^T, g_n).
 *   traj      [B][T][d]  the converged forward trajectory
 *   g         [B][T][d]  dL/dx_n
 *   dL_dx0    [B][d]
 *   dL_dtheta [B][n_params] (per instance, also when params_shared = 1;
 *             sum over instances for a shared theta), or NULL
 *   seg       steps per recomputation segment: elements are recomputed from
 *             traj segment by segment (memory seg*d*d per instance); 0 = T
 *             (all elements at once).
 * Lorenz-96 (d = 40) builds each element inside the reverse recursion and
 * stores none (one workgroup per instance): seg is then ignored and the
 * workspace query returns a small constant.  pint_set_dense_pipeline(0)
 * selects the two-kernel path instead (elements of a segment written, then
 * scanned); query the workspace after setting it.  In the fused pass a
 * bounded wait between the workgroup's waves that gives up (not expected)
 * leaves NaN in that instance's outputs.
 */
size_t pint_adjoint_workspace_bytes(const pint_system* sys, int64_t B, int64_t T,
                                    int64_t seg, int32_t dtype);
pint_status pint_adjoint(const pint_system* sys, int64_t B, const void* x0,
                         double dt, int64_t T, int32_t dtype, const void* traj,
                         const void* g, void* dL_dx0, void* dL_dtheta,
                         int64_t seg, void* ws, size_t ws_bytes,
                         pint_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PINT_H_ */
