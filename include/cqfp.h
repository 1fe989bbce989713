/*
 * cqfp.h - C ABI of the MI355X (gfx950) convolution-quadrature solver for the
 * two-state fractional Fokker-Planck system.
 *
 * Method: Sun, Nie & Deng, "Fast algorithms for convolution quadrature of
 * Riemann-Liouville fractional derivative". The problem is the decoupled
 * form (2.1) of system (1.1):
 *   dG1/dt + a D^{1-alpha1} G1 + D^{1-alpha1} A G1 = a D^{1-alpha2} G2,
 *   dG2/dt + a D^{1-alpha2} G2 + D^{1-alpha2} A G2 = a D^{1-alpha1} G1,
 * with a = (1-m)/(2m-1) (m of the transition matrix (1.2)), A = -Laplacian
 * with zero Dirichlet data, discretised in space by the 3-point (1D),
 * 5-point (2D) or 7-point (3D) finite-difference stencil on a uniform grid of
 * interior nodes.
 * Time: backward-Euler CQ, scheme (4.1), or BDF2 (SBD) CQ with the starting
 * correction, scheme (4.7); the CQ history is summed directly (O(N^2)) or by
 * the fast sum-of-geometric-sequences form, schemes (4.3) and (4.8).
 *
 * Conventions for every entry point:
 *  - All arrays are IEEE fp64, contiguous, owned by the caller. "dev" marks a
 *    device pointer on the current HIP device, "host" a host pointer.
 *  - A field G is laid out [2][M]: component 1 then component 2, each with
 *    M = nx*ny*nz nodes, x fastest (node (i,j,k) at index (k*ny + j)*nx + i).
 *  - Device work is enqueued on the caller's hipStream_t (passed as void*;
 *    NULL means the default stream). Entry points that return data to the
 *    host synchronise that stream.
 *  - Entry points never abort and never throw; they return a status code
 *    below. cq_last_error() returns a message for the last failure on the
 *    calling thread.
 */
#ifndef CQFP_H
#define CQFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CQ_OK 0
#define CQ_EINVAL -1      /* an argument is out of range or NULL                */
#define CQ_ESINGULAR -2   /* the implicit step operator is not positive definite */
#define CQ_ENOMEM -3      /* host or device allocation failed                    */
#define CQ_EHIP -4        /* a HIP runtime call failed (or no GPU is present)    */
#define CQ_ETOL -5        /* the fast rule cannot reach fast_tol within np_max   */
#define CQ_ENONFINITE -6  /* G0 holds a NaN or an infinity                       */

/* Grid: Omega = (0,lx) (dim 1), (0,lx)x(0,ly) (dim 2) or (0,lx)x(0,ly)x(0,lz)
 * (dim 3; the problem (1.1) is posed for d = 1, 2, 3); nx, ny, nz interior
 * nodes per direction, h = l/(n+1); A is the 3-, 5- or 7-point
 * finite-difference Laplacian. For dim 1, ny must be 1; for dims 1 and 2,
 * nz must be 0 or 1 (lz is ignored). 3D grids need ny * nz <= 2^20. Nodes are
 * ordered x fastest, then y, then z. */
typedef struct {
    int32_t dim;
    int32_t nx, ny;
    double lx, ly;
    int32_t nz;
    double lz;
} cq_grid;

/* Problem and method parameters (Sections 3-4).
 *  alpha1, alpha2 in (0,1): the CQ orders are beta_k = 1 - alpha_k.
 *  m in [0,1] without 1/2 (m = 0 gives a = -1 as in Tables 3-5; m = 1 gives
 *    a = 0, the decoupled case).
 *  T > 0 and N >= 1: tau = T/N.
 *  scheme: 1 = backward Euler (4.1), 2 = BDF2 with the correction (4.7).
 *  method: 0 = direct history sum, 1 = fast history (3.10) / (3.18).
 *  fast_tol: target relative error of the fast solution against the direct
 *    one (0 selects 1e-8); the node count np is chosen by scanning the weight
 *    errors eps_i of (3.8)/(3.16) unless np > 0 is given.
 *  np: Gauss-Jacobi nodes (BE) or N_{p,2} (BDF2); 0 = choose by the scan.
 *  np1: N_{p,1} for BDF2 (0 selects 16, or the scan's choice below).
 *    ns: N_s for BDF2 (must be >= 3; 0 selects 30 when np is given). With
 *    np = 0 and ns = 0 the BDF2 window is chosen from the weight errors too
 *    (Section 5): N_s in {12,...,32} and N_{p,1} in {8, 12, 16, 24} (unless
 *    np1 > 0), each with its smallest N_{p,2} meeting the tolerance, the
 *    pair of least modelled cost per step (state flops, window flops, state
 *    traffic per block of N_s steps) winning; fp_info reports the choice
 *    (lag = N_s, np1). The batched solver and cq_fast_rule keep 30 and 16.
 *    np_max: scan limit (0 selects 1024). A solver keeps
 *    at most 1024 fast nodes per component (np, or np1 + np for BDF2);
 *    more is CQ_EINVAL.
 *  block_B: direct method, time-block length of the Toeplitz far-field
 *    update (0 = automatic; otherwise 64, 128, 192 or 256). The modal solver
 *    steps in blocks of 64 and takes block_B as the rows of one far-field
 *    pass over the stored levels (0 selects 192, or 256 from 8192 modes): the
 *    pass serves block_B/64 blocks, each later block adding the levels since
 *    the pass on its own.
 *  solver: 0 = nodal: every step assembles the right-hand side on the grid
 *    and solves the coupled system (cyclic reduction in 1D, sine transform
 *    with a 2x2 solve per mode in 2D); 1 = modal: the sine transform is
 *    applied once to G0 and once per read-out, and every mode advances by
 *    its own 2x2 recurrence (same scheme, no per-step global coupling; the
 *    fast form then needs lag <= 64 and at most 1024 nodes per component).
 *  fast_kernel (modal solver, fast method): 0 = the state streamed through
 *    device memory in time blocks (any run, resumable anywhere, the same
 *    levels bit for bit however the run is cut into fp_step calls); 1 = an
 *    fp_step call that takes all N steps from step 0 (fp_solve's) runs them
 *    in one launch of the 16-mode MFMA kernel of fp_solve_batched, the state
 *    in registers (lags 16..33 and <= 608 nodes per component; elsewhere, and
 *    for other calls, 0): the same scheme summed in another order, within
 *    1e-13 relative of 0's; the handle then holds only the final level
 *    (fp_current, fp_get_state at n = N). A whole run keeps 16 modes per
 *    workgroup, so it pays from several thousand modes (two workgroups per
 *    compute unit from 8192). Other values: CQ_EINVAL. */
typedef struct {
    double alpha1, alpha2;
    double m;
    double T;
    int64_t N;
    int32_t scheme;
    int32_t method;
    double fast_tol;
    int32_t np;
    int32_t np1;
    int32_t ns;
    int32_t np_max;
    int32_t block_B;
    int32_t solver;
    int32_t fast_kernel;
} cq_params;

/* What a solver handle chose (filled by fp_info). */
typedef struct {
    int64_t n;            /* steps taken so far                               */
    int64_t N;            /* total steps                                      */
    int32_t np_total;     /* fast nodes per component (N_p, or N_p1 + N_p2)   */
    int32_t lag;          /* first lag covered by the fast rule (2 or N_s)    */
    double max_eps;       /* max_i |eps_i| / d_0 over both components          */
    double theta[2];      /* eigenvalues of the 2x2 step coupling matrix       */
    int32_t block_B;      /* time-block length (direct far field / fast state) */
    int32_t ksplit;       /* direct: K-split of the far-field update           */
    size_t device_bytes;  /* device memory held by the handle                 */
    size_t state_bytes;   /* bytes of fp_get_state                            */
    int32_t np1;          /* BDF2 fast: N_{p,1} (first family), 0 otherwise   */
    int32_t whole_run_kernel; /* 1: a whole-run fp_step takes the MFMA kernel  */
} cq_info;

/* CQ weights d_i, i = 0..n, of order beta: Taylor coefficients of
 * ((1-zeta)/tau)^beta (scheme 1, eqs. (3.3)-(3.4)) or of
 * (((1-zeta) + (1-zeta)^2/2)/tau)^beta (scheme 2, eqs. (3.11)-(3.12)).
 * d_out: host, n+1 doubles. beta in (0,1), tau > 0, n >= 0. Host only. */
int cq_weights(int32_t scheme, double beta, double tau, int64_t n, double* d_out);

/* Fast rule of Section 3: the families of geometric sequences with
 *   d_i ~ sum_j coef_j * ratio_j^(i - lag),   i >= lag,
 * from the Gauss-Jacobi rule of (3.6) (scheme 1, lag = 2) or the two rules
 * of (3.14)-(3.16) with the real-part remark (scheme 2, lag = ns). coef_j
 * folds in the paper's w_j and dbar(lag)(s_j). When np == 0 the node count
 * is the smallest on an internal ladder with max_{lag<=i<=N} |eps_i| <=
 * tol*|d_0|/(10 N); with np > 0 that count is used as given.
 * ratio_out, coef_out: host arrays of capacity `cap`; count_out receives the
 * number of terms (np, or np1 + np2), lag_out the lag, max_eps_out the
 * measured max |eps_i| / |d_0| over lag <= i <= N. Host only.
 * Returns CQ_ETOL if the scan cannot meet tol with np <= np_max and
 * CQ_EINVAL if cap is too small. */
int cq_fast_rule(int32_t scheme, double beta, double tau, int64_t N, double tol,
                 int32_t np, int32_t np1, int32_t ns, int32_t np_max, int32_t cap,
                 double* ratio_out, double* coef_out, int32_t* count_out,
                 int32_t* lag_out, double* max_eps_out);

/* CQ history sum S = sum_{i=1}^{n-1} d_i G^{n-i} (the convolution of
 * (3.8)/(3.17) without the i = 0 term and without G^0, as it enters the
 * schemes (4.1) and (4.7)), with d_i the weights of cq_weights(scheme, beta,
 * tau, .). G_hist: dev [n][M] time-major (level 0 is G^0, unused);
 * S_out: dev [M]. n >= 1, M >= 1 (n = 1 gives zeros). The weights are
 * computed on the host; the sum streams every level once on the device
 * (a weighted sum over levels, split into level slices whose partial sums
 * are added in slice order). Allocates a device workspace (the weights and
 * the partial sums) for the call and frees it; synchronises the stream. */
int cq_history(int32_t scheme, double beta, double tau, const double* G_hist,
               int64_t n, int64_t M, double* S_out, void* hip_stream);

/* The same history sum for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Arguments, layout and result as cq_history; the weights are
 * computed on the device by the same recurrences (so they can differ from
 * cq_history's host weights in the last bits). Calls no hipMalloc, hipFree or
 * other allocating routine: its workspace (the weights and partial sums) is
 * a static device array of 16 MiB that each GPU the library runs on holds
 * until the process ends. Limit: n <= 2^20 levels (CQ_EINVAL beyond); any M.
 * Asynchronous: the work is only enqueued on hip_stream (no synchronisation,
 * no memset). Every call on one GPU shares that GPU's workspace, which keeps
 * the last call's contents: calls whose device work can overlap on one GPU
 * (other streams without ordering, other threads) race and must be
 * serialised by the caller. */
int cq_history_noalloc(int32_t scheme, double beta, double tau, const double* G_hist,
                       int64_t n, int64_t M, double* S_out, void* hip_stream);

/* Create a solver for one problem, starting from G0 (dev [2][M], copied).
 * The handle integrates the decoupled system (2.1) by the scheme prm selects:
 * backward-Euler CQ (4.1) with its fast form (4.3), or BDF2 CQ with the
 * starting correction (4.7) and its fast form (4.8); the history term of
 * each step is the CQ sum (3.8) / (3.17) with the weights of (3.4) / (3.12),
 * and the fast method replaces its far part by the geometric sums of
 * (3.9)-(3.10) / (3.18). Allocates every device buffer the run needs (the full history
 * [N+1][2][M] for method 0; the compressed state [2][np_total][M] and an
 * N_s-level window for method 1). Validates the arguments (CQ_EINVAL,
 * CQ_ENONFINITE; the finiteness check copies G0 to the host and synchronises
 * the stream), checks that the step operator is positive definite
 * (CQ_ESINGULAR) and, for method 1 with np == 0, that the fast rule meets
 * fast_tol (CQ_ETOL). *handle receives the solver; free it with fp_destroy. */
int fp_create(const cq_grid* grid, const cq_params* prm, const double* G0,
              void* hip_stream, void** handle);

/* Advance by nsteps time steps (not beyond N), asynchronously on the
 * handle's stream. Each step n solves the implicit 2x2-block system of
 * (4.1) or (4.7) for G^n (for (4.7), the n = 1 step carries the starting
 * correction) after forming the CQ history of the earlier levels (direct sum,
 * or the fast form (4.3) / (4.8)). Allocates nothing. CQ_EINVAL if
 * n + nsteps > N. */
int fp_step(void* handle, int64_t nsteps);

/* Copy the current solution G^n to G_out (dev [2][M]); *n_out receives n.
 * Asynchronous on the handle's stream. */
int fp_current(void* handle, double* G_out, int64_t* n_out);

/* Report what the handle chose (node counts, block sizes, memory). */
int fp_info(void* handle, cq_info* info);

/* Save / restore the solver state (step index, time levels still needed,
 * compressed history) to / from a host buffer. fp_get_state with dst NULL
 * stores the needed size in *bytes. Restoring into a handle created with the
 * same grid and parameters and then stepping gives the same result as never
 * stopping. Both synchronise the stream. */
int fp_get_state(void* handle, void* dst, size_t* bytes);
int fp_set_state(void* handle, const void* src, size_t bytes);

/* Restart the handle at n = 0 from a new G0 (dev [2][M], copied): clears
 * the compressed history and the level store on the device, reusing every
 * device buffer (no device allocation). G0 is first checked for NaN and
 * infinity (CQ_ENONFINITE): that check copies it into a temporary host
 * buffer and synchronises the handle's stream; the restart itself is then
 * enqueued asynchronously on that stream. */
int fp_reset(void* handle, const double* G0);

/* Release a handle and all its device memory. NULL is accepted. */
int fp_destroy(void* handle);

/* One-call solve of (2.1) by the scheme prm selects ((4.1)/(4.3) or
 * (4.7)/(4.8), as fp_create): create, take all N steps, write G^N to GN
 * (dev [2][M]), destroy. Errors as fp_create. Synchronises the stream. */
int fp_solve(const cq_grid* grid, const cq_params* prm, const double* G0, double* GN,
             void* hip_stream);

/* Gradient of a loss of the final state (extension, not in the paper): the
 * discrete adjoint of the scheme of (4.1)/(4.3) or (4.7)/(4.8) that fp_solve
 * runs with the same grid and parameters (direct or fast; modal solver,
 * solver = 1, required). Given gN = dl/dG^N (dev [2][M]) it writes
 *   gG0  (dev [2][M])   dl/dG^0,
 *   grad (host [3])     dl/dalpha_1, dl/dalpha_2, dl/dm,
 *   GN   (dev [2][M])   G^N, or NULL.
 * With mu^n the multipliers of the step equations c G^n - E^n + Dm X^n = 0
 * (Dm = [[a+A, -a], [-a, a+A]], X^n the CQ sums of the scheme), they solve
 * the transposed steps backwards in time: (cI + W_0 Dm) mu^n = [n=N] gN
 * + (time-difference terms of mu^{n+1}, mu^{n+2}) - sum_{i>=1} W_i Dm
 * mu^{n+i}, the same CQ recurrence with the same weights (fast or direct)
 * run in reversed time on psi = Dm mu. Parameter gradients contract mu with
 * d/dtheta of the step equations; for alpha_k the weights' beta-derivative
 * is exact for the direct scheme; for the fast scheme beyond its lag the
 * rule's factor tau^-beta is differentiated exactly and the rest by a
 * fourth-order difference in beta of the rebuilt Gauss-Jacobi rule (below
 * 1e-11 relative). The alpha contraction sum_n psi^n . sum_l dw_{n-l} g^l
 * runs in the frequency domain for N <= 4096 (steps in blocks of up to 256,
 * one 512-point FFT per block, mode and component, and the block pairs
 * contracted with the spectra of the weight windows between them), else as
 * Toeplitz products; setting the environment variable CQFP_BETA_TOEPLITZ
 * (not "0") when the handle is made selects the Toeplitz form at any N. The
 * forward trajectory, its history sums and the adjoint (psi, mu) are kept in
 * device memory (4 (N+1) 2M doubles) when they fit in the free memory;
 * otherwise the fast method recomputes the forward from saved states (see
 * cq_adjoint_opts; the alpha contraction then runs as Toeplitz products) and
 * the direct method returns CQ_ENOMEM. Device work runs on hip_stream; the
 * call synchronises it. Errors as fp_create, plus CQ_EINVAL for solver != 1 or
 * a fast window (ns) above 32. */
int fp_adjoint(const cq_grid* grid, const cq_params* prm, const double* G0, const double* gN,
               double* gG0, double* grad, double* GN, void* hip_stream);

/* The same in two parts, for many gradients at one grid and parameter set:
 * fp_adjoint_create does the host set-up (weights, rules and their
 * beta-derivatives) and allocates the device arrays once; every
 * fp_adjoint_run then only enqueues device work on the handle's stream (and
 * synchronises it to return grad). Arguments and errors as fp_adjoint. The
 * handle is released by fp_destroy; the stepping calls (fp_step, ...)
 * reject it with CQ_EINVAL. */
int fp_adjoint_create(const cq_grid* grid, const cq_params* prm, void* hip_stream, void** handle);

/* Memory form of a gradient handle (extension). The forward trajectory, its
 * history sums and the adjoint fill 4 (N+1) 2M doubles when kept whole. For
 * the fast method the forward can instead be recomputed from saved states:
 * the steps are cut into segments (whole chunks of the gradient reductions,
 * a multiple of the fast form's state block); a saved state is the fast
 * state H and the last L levels at a segment start; a binomial (revolve)
 * schedule, optimal for the number of states that fit, chooses where the
 * forward advances and saves, and every segment is recomputed once more with
 * its levels and history sums in a segment buffer while the adjoint takes
 * the segment's steps (psi = Dm mu is kept whole: (N+1) 2M doubles). The
 * gradient is the same computation: G^N, dl/dG0 and dl/dm equal the kept
 * form's bit for bit; the alpha contraction, summed as Toeplitz products
 * segment by segment, agrees to rounding (relative 1e-10).
 *  max_device_bytes: the handle's budget (0: the free device memory).
 *  mode: 0 automatic (keep whole if it fits the budget, else checkpointed
 *    for the fast method, else CQ_ENOMEM), 1 keep whole, 2 checkpointed
 *    (fast method only; CQ_EINVAL otherwise).
 *  segment_steps, slots: checkpointed form's segment length (rounded up to
 *    whole chunks) and number of saved states; 0 chooses the pair with the
 *    fewest recomputed forward steps that fits the budget.
 *  forward_kernel: the kept-whole fast sweeps. 0 automatic (2 where it
 *    applies from 8192 modes), 1 the streamed state (the kernels of fp_step: the gradient
 *    then equals the checkpointed form's as stated above), 2 the forward
 *    and the adjoint sweep each in one launch of the batched 16-mode MFMA
 *    kernel over all N steps, levels, history sums and multipliers written
 *    as they go (lags 16..32, <= 512 nodes per component; elsewhere 1;
 *    up to 448 nodes it also writes the levels as the d/dalpha block DFTs'
 *    time series, 2 x N x 2M more values where the budget holds them): the
 *    same schemes summed in another order: G^N, dl/dG0 and dl/dm agree with
 *    1's to 1e-12 relative, dl/dalpha_k to 1e-11 (their contraction cancels
 *    across modes). Other values: CQ_EINVAL. */
typedef struct {
    size_t max_device_bytes;
    int32_t mode;
    int32_t segment_steps;
    int32_t slots;
    int32_t forward_kernel;
} cq_adjoint_opts;

/* What a gradient handle chose. */
typedef struct {
    int32_t mode;           /* 1 kept whole, 2 checkpointed                 */
    int64_t segment_steps;  /* steps per segment (N when kept whole)        */
    int32_t segments;
    int32_t slots;          /* saved forward states (0 when kept whole)     */
    int64_t forward_steps;  /* forward steps per gradient (N when kept whole) */
    size_t device_bytes;    /* device memory held by the handle             */
    int32_t forward_kernel; /* 1 streamed state, 2 16-mode MFMA (see opts)  */
} cq_adjoint_info;

/* fp_adjoint_create with a memory form (opts NULL: automatic). */
int fp_adjoint_create_opts(const cq_grid* grid, const cq_params* prm, const cq_adjoint_opts* opts,
                           void* hip_stream, void** handle);
int fp_adjoint_info(void* handle, cq_adjoint_info* info);
int fp_adjoint_run(void* handle, const double* G0, const double* gN, double* gG0, double* grad,
                   double* GN);

/* Batched fast solves (extension): `count` independent problems (own grid,
 * orders, m, T, N, scheme; method must be 1, the fast form) solved by the
 * modal solver in one captured HIP graph. Every problem's sine modes are
 * work items of one persistent kernel per register class (problems grouped
 * by nodes per lane), each mode running its problem's whole time loop, so
 * problems of uneven size share the GPU without a barrier between them.
 * Three kernels: the per-step one (64 or 32 lanes per mode, each step sums
 * the state over the lanes), the time-blocked one (one wave per mode;
 * the state advances over a block of L steps at a time, the lag of the
 * exact-weight window, before the block's steps are solved; needs every lag
 * <= 32 and <= 768 nodes per component) and the 16-mode MFMA one (a
 * workgroup per 16 modes of a problem: over blocks of 16 steps the state
 * advance and its sums are FP64 matrix-core products over the modes; needs
 * lags 16..33 and <= 608 nodes per component). G0[i], GN[i]: dev [2][M_i]
 * (caller-owned, distinct). autotune: 1 times the candidates for every
 * class on a short run and keeps the fastest (cached for the process);
 * 0 takes the 16-mode MFMA kernel where it applies, else the time-blocked
 * one where it applies, else 64 lanes per mode; 2, 3 and 4 take the
 * time-blocked, the 16-mode MFMA and the per-step (64 lanes) kernel where
 * each applies (elsewhere the time-blocked one or 64 lanes per mode); other
 * values are CQ_EINVAL. The caller's stream is
 * waited on before the solve and the call returns when every GN[i] is
 * written. Temporary device buffers are allocated and freed inside.
 * report (may be NULL) receives the classes and timings. */
typedef struct {
    int32_t problems;
    int64_t modes;            /* sum of M_i                                   */
    int32_t classes;          /* register classes launched (<= 8 reported)   */
    int32_t class_npl64[8];   /* nodes per lane at 64 lanes of each class    */
    int32_t class_lanes[8];   /* lanes per mode chosen for each class        */
    int32_t class_problems[8];
    int32_t class_blocked[8]; /* 1 time-blocked, 2 16-mode MFMA, 0 per-step */
    double setup_s;           /* host set-up and forward transforms          */
    double autotune_s;        /* tile timing (0 when cached or disabled)     */
    double run_s;             /* the graph: time loops and inverse transforms */
} cq_batch_report;

int fp_solve_batched(int32_t count, const cq_grid* grids, const cq_params* params,
                     const double* const* G0, double* const* GN, void* hip_stream,
                     int32_t autotune, cq_batch_report* report);

/* Kernel timing (opt-in). While enabled, every kernel launch of the library
 * is bracketed by a pair of HIP events on the stream it runs on. The kernels
 * are grouped by kind: 0 fast history, 1 direct near field, 2 Toeplitz far
 * field (FP64 MFMA), 3 1D right-hand side + PCR solve, 4 2D right-hand side,
 * 5 DST GEMM (forward/inverse and per-mode solve), 6 standalone history
 * reduction, 7 modal fast steps, 8 modal direct near field + solve,
 * 9 batched modal fast time loops, 10 sum of the far field's K-split
 * partials, 11 time-series transposes of the adjoint, 12 the adjoint's
 * spectral d/dbeta contraction (FFT per column and dot). cq_prof_read
 * synchronises the recorded events and returns, for one kind, the launch
 * count and the summed duration in milliseconds.
 * cq_prof_enable(1) also clears earlier records. Not thread safe. */
int cq_prof_enable(int32_t on);
int cq_prof_read(int32_t kind, int64_t* launches, double* total_ms);

/* Message describing the last failure on this thread ("" if none). */
const char* cq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CQFP_H */
