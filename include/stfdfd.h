/*
 * stfdfd.h - C ABI of the MI355X (gfx950) overlapping-PML source-transfer FDFD solver.
 *
 * Method: arXiv 2509.20801, "Parallel overlapping-domain decomposition FDFD for
 * large-scale complex nanostructures modeling".  The library solves the 2D TM
 * FDFD system A e = b (Sec. 2.1, Eqs. (2)-(4)) with the stretched-coordinate PML
 * of Sec. 2.2 (Eqs. (9)-(13)) by flexible GMRES in FP64, right-preconditioned by
 * one source-transfer round over overlapping PML-terminated subdomains
 * (Sec. 2.3, Eqs. (14)-(21), Algorithm 1) whose local systems are factored by a
 * nested-dissection multifrontal LU (Sec. 2.4, Eqs. (22)-(23)).
 *
 * Conventions used by every call:
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - Node arrays are row-major [ny][nx], x fastest: node (i, j) is element j*nx + i,
 *     at position x = i*dx, y = j*dy.
 *   - The cell permittivity map is row-major [ny+1][nx+1]; cell (c, d) is the dual
 *     cell whose corners are nodes (c-1..c, d-1..d).  The node permittivity is the
 *     mean of its four cells (Eq. (3)).
 *   - Pointers marked "host or device" are read as device pointers when the call's
 *     on_device argument is nonzero, else as host pointers.  Device pointers must
 *     be accessible from the context's device; work on them is ordered on the
 *     context's stream.  The caller owns every buffer it passes; the library
 *     never retains a caller pointer after the call returns.
 *   - Every call returns a status and never aborts, exits or throws; the message
 *     of the last failing call on a context is returned by stf_last_error().
 *   - One context per host thread.  Calls on one context are not thread safe.
 */
#ifndef STFDFD_H
#define STFDFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stf_ctx_s*     stf_ctx;      /* device, stream, symbolic cache, timers */
typedef struct stf_problem_s* stf_problem;  /* one assembled problem: operator, partition, factors */

typedef enum {
  STF_OK = 0,
  STF_EINVAL = 1,   /* invalid argument (sizes, NaN/Inf input, partition too fine, ...) */
  STF_ENOMEM = 2,   /* device or host allocation failed */
  STF_EDEVICE = 3,  /* HIP runtime error */
  STF_ESTATE = 4,   /* call out of order (e.g. solve before factor) */
  STF_EPIVOT = 5,   /* a tiny pivot was perturbed during factorisation; results are valid
                       (FGMRES absorbs the perturbation) */
  STF_ENOCONV = 6,  /* max_iter reached above tol; x holds the last iterate */
  STF_ENAN = 7      /* non-finite residual during the solve */
} stf_status;

/* Precision of the subdomain fronts and sweeps.  FGMRES, the global stencil,
 * the Arnoldi process and the solution update are always FP64. */
enum { STF_C128 = 0, STF_C64 = 1 };

/* Initial guess.  STF_X0_LEARNED: the context's network (stf_ctx_set_nn)
 * predicts the field on overlapping tiles of the physical interior and the
 * blended prediction is the guess, unless its FP64 residual is not below |b|
 * (then the zero guess is used instead; see stf_solve_info.used_learned). */
enum { STF_X0_ZERO = 0, STF_X0_USER = 1, STF_X0_LEARNED = 2 };

/* Order of the source transfer inside one preconditioner application.
 * STF_ORDER_ADDITIVE is the paper's Jacobi round (Algorithm 1: every subdomain
 * solves with the previous round's data, Eq. (21) sums the local fields).  The
 * others visit the subdomains in stages, as the sweeping source-transfer
 * methods the paper builds on (Sec. 1) do: each stage solves its subdomains
 * with the residual left by the stages before it and adds their full local
 * fields,  z = 0;  for every stage: z += sum_{k in stage} P_k A_k^{-1} R_k^I (v - A z).
 *   STF_ORDER_ROWS       subdomain rows ky = 0 .. py-1, then back down to 0;
 *   STF_ORDER_ROWS_COLS  rows up and down, then columns kx = 0 .. px-1 and back;
 *   STF_ORDER_DIAGONAL   the anti-diagonals kx + ky rising and falling, then the
 *                        diagonals kx + (py-1-ky) rising and falling (four
 *                        corner-to-corner directions);
 *   STF_ORDER_CHECKER    two colours: the subdomains with kx + ky even, then
 *                        those with kx + ky odd (no stage holds two edge
 *                        neighbours).
 * The sweeping orders read the factors once per stage a subdomain belongs to
 * (2-4 times) but carry waves across many subdomains, so FGMRES needs far
 * fewer iterations where waves cross many subdomains.  The two-colour order
 * reads every factor once, like the Jacobi round, in two half-size stages. */
enum { STF_ORDER_ADDITIVE = 0, STF_ORDER_ROWS = 1, STF_ORDER_ROWS_COLS = 2, STF_ORDER_DIAGONAL = 3,
       STF_ORDER_CHECKER = 4 };

/* Problem description (Sec. 2.1-2.3).  Global PML sides are ordered x-, x+, y-, y+.
 * The interior [pml[0], nx-pml[1]) x [pml[2], ny-pml[3]) is split into px x py
 * blocks as evenly as possible (earlier blocks take the remainder); edge blocks
 * also own the global PML on their side.  Each block is extended on every side
 * facing a neighbour by overlap + local_pml nodes: `overlap` unstretched cells
 * then a local PML of `local_pml` cells (Eqs. (10)-(13) with local_pml_order and
 * local_pml_R).  Requires every interior block side >= overlap + local_pml + 1,
 * and, with three or more blocks along an axis, >= 2 (overlap + local_pml), so
 * that no node lies in more than two blocks' extended domains per axis. */
typedef struct {
  int32_t nx, ny;            /* nodes, global PML included (each >= 3) */
  double  dx, dy;            /* grid steps (> 0) */
  double  k0;                /* free-space wavenumber 2*pi/lambda in the same unit (> 0) */
  int32_t pml[4];            /* global PML cells per side (>= 0) */
  int32_t pml_order;         /* m of Eqs. (11)-(12) (>= 0) */
  double  pml_R;             /* R(0) of Eq. (13), 0 < R < 1 */
  int32_t px, py;            /* subdomain grid (>= 1 each) */
  int32_t overlap;           /* unstretched overlap cells before the local PML (>= 0) */
  int32_t local_pml;         /* local PML cells (>= 1 when px*py > 1) */
  int32_t local_pml_order;
  double  local_pml_R;
  int32_t front_prec;        /* STF_C128 or STF_C64 */
  int32_t leaf_size;         /* largest leaf box (nodes) of the nested dissection; 0 = 32 */
} stf_params;

typedef struct {
  double  tol;        /* stop when |b - A x|_2 <= tol |b|_2 (FP64 true residual) */
  int32_t restart;    /* FGMRES cycle length m (1..200) */
  int32_t max_iter;   /* total inner iterations (>= 1) */
  int32_t x0_mode;    /* STF_X0_ZERO, STF_X0_USER (x holds the guess on entry) or STF_X0_LEARNED */
  int32_t rounds;     /* source-transfer rounds per preconditioner application (0 or 1 = one
                         round z = B v; r > 1 adds r-1 stationary corrections
                         z += B (v - A z), i.e. r Jacobi rounds of Algorithm 1; <= 8) */
  int32_t debug_fault; /* test hook of the tiny-pivot path (Eq. (22) with pivoting): 0 = off;
                          1 = before iterating, factor the problem again with one planted
                          fault, the first pivot column of one front of tree level 1
                          zeroed on its fully summed rows, so that the pivot is replaced
                          by its perturbation (multipliers then grow like 1/tau, which
                          limits the attainable accuracy).  The solve then returns
                          STF_EPIVOT when every right-hand side converged (info.status
                          stays STF_OK).  The factors keep the fault until the next
                          stf_factor. */
  int32_t order;      /* STF_ORDER_*: order of the source transfer in the preconditioner
                         (rounds > 1 only with STF_ORDER_ADDITIVE) */
} stf_solve_opts;

typedef struct {
  int32_t iters;          /* inner FGMRES iterations performed */
  int32_t restarts;       /* completed cycles */
  int32_t status;         /* stf_status of this right-hand side */
  int32_t history_len;    /* entries written to history */
  double  relres_true;    /* FP64 |b - A x| / |b| at exit */
  double  relres_x0;      /* FP64 |b - A x0| / |b| (for STF_X0_LEARNED: of the network's
                             guess, before the fallback) */
  double* history;        /* caller-owned host buffer (may be NULL): relative residual
                             estimate after every iteration, true residual at x0 first */
  int32_t history_cap;    /* capacity of history */
  int32_t used_learned;   /* STF_X0_LEARNED: 1 if the network's guess was kept, 0 after fallback */
  /* Phase timers (device time, HIP events on the context stream, ms). */
  double  t_factor_ms;    /* the problem's most recent factorisation */
  double  t_solve_ms;     /* this call's solve of the group of right-hand sides swept with this
                             one (initial residuals to the last true residual) */
  double  t_nn_ms;        /* the network's guess for this right-hand side (STF_X0_LEARNED) */
} stf_solve_info;

/* Sizes and work counts of a plan. */
typedef struct {
  int64_t ndof;             /* nx*ny */
  int32_t nsub;             /* px*py */
  int32_t nshapes;          /* distinct subdomain shapes (symbolic plans) */
  int64_t local_dof;        /* sum of subdomain node counts */
  int64_t nfronts;          /* fronts over all subdomains */
  int32_t max_front;        /* largest front order m = p + q */
  int32_t max_depth;        /* deepest tree level (root = 0) */
  int64_t factor_entries;   /* sum over fronts of p*p + 2*p*q (entries the sweeps read) */
  int64_t front_entries;    /* sum over fronts of m*m (the working blocks; the library keeps
                               only two tree levels' worth, the even depths in one arena and
                               the odd in another, each sized for its largest level) */
  double  lu_flops;         /* real flops of the partial LUs: 8 * sum_k (m-k)^2, k = 1..p */
  int64_t device_bytes;     /* device memory held by the problem (0 from stf_plan_query) */
} stf_plan_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to order
 * all work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a
 * stream of the library's own.  */
stf_status  stf_ctx_create(int device, void* hip_stream, stf_ctx* out);
void        stf_ctx_destroy(stf_ctx ctx);                 /* NULL-safe */
const char* stf_last_error(stf_ctx ctx);                  /* never NULL */

/* Per-kernel timing with HIP events on the context stream.  While enabled,
 * every launch of the listed kernel classes is bracketed by two events. */
enum {
  STF_K_ASSEMBLE = 0, STF_K_STENCIL = 1, STF_K_FRONT_ASM = 2, STF_K_FRONT_LU = 3,
  STF_K_SWEEP_FWD = 4, STF_K_SWEEP_BWD = 5, STF_K_SCATTER = 6, STF_K_ARNOLDI = 7,
  STF_K_UPDATE = 8, STF_K_NN = 9, STF_K_COUNT = 10
};
stf_status  stf_ctx_set_timing(stf_ctx ctx, int enable);  /* all classes; enabling resets the counters */
/* Timing restricted to the classes whose bits (1 << STF_K_*) are set in mask (0 = off);
 * resets the counters.  Fewer bracketed launches perturb the timed region less. */
stf_status  stf_ctx_set_timing_mask(stf_ctx ctx, uint32_t mask);
/* Synchronises the stream, then reports the summed duration (ms) and launch count
 * of kernel class `cls` since timing was enabled. */
stf_status  stf_ctx_kernel_stats(stf_ctx ctx, int cls, double* total_ms, int64_t* launches);

/* ---- problem ------------------------------------------------------------ */

/* Host-only: validate `prm` and compute the partition and the nested-dissection
 * plan statistics without touching a device. */
stf_status  stf_plan_query(const stf_params* prm, stf_plan_info* out);

/* Host-only test hook: the 1D coupling coefficients of subdomain k's local
 * operator (Sec. 2.3 with the stretch of Eqs. (10)-(13)).  cw[t], ce[t] (t < local
 * nx) couple local node column t to t-1 and t+1; cs[u], cn[u] (u < local ny) in y.
 * Each is an interleaved complex array; dims receives {ox0, oy0, nxl, nyl,
 * ix0, ix1, iy0, iy1} (global node ranges of Omega_k and I_k).  Any output
 * pointer may be NULL; non-NULL arrays must hold the local size. */
stf_status  stf_debug_local_axes(const stf_params* prm, int32_t k, int32_t* dims,
                                 double* cw, double* ce, double* cs, double* cn);

/* "Assemble from eps(x,y), omega, PML profile and subdomain partition" (Sec. 2.1-2.3,
 * Algorithm 1 preprocessing): validates prm, builds the global and local stretch
 * arrays, the partition and the symbolic plans (cached per subdomain shape in
 * the context), allocates the device state and assembles the node permittivity.
 * eps_cells: (ny+1)*(nx+1) complex, host or device.  */
stf_status  stf_problem_create(stf_ctx ctx, const stf_params* prm, const double* eps_cells,
                               int on_device, stf_problem* out);
/* Re-assemble with a new permittivity map of the same shape (invalidates factors). */
stf_status  stf_assemble(stf_problem pb, const double* eps_cells, int on_device);
/* Numeric multifrontal LU of every subdomain operator (Eq. (22)); returns
 * STF_EPIVOT if a pivot was perturbed. */
stf_status  stf_factor(stf_problem pb);
/* Solve A x = b for nrhs right-hand sides (FGMRES, FP64, right-preconditioned by
 * one source-transfer round).  b, x: nrhs*ny*nx complex, host or device.
 * info: array of nrhs (may be NULL).  Returns the worst per-RHS status. */
stf_status  stf_solve(stf_problem pb, int32_t nrhs, const double* b, double* x, int on_device,
                      const stf_solve_opts* opts, stf_solve_info* info);
/* stf_factor then stf_solve in one call (Eq. (22), then the solve phase), with
 * the same arguments as stf_solve.  With STF_X0_LEARNED and device arrays the
 * network's guesses (which need only the permittivity and b) are computed on a
 * second stream of the context while the factorisation runs, and the solve
 * waits for them: the network's memory-bound kernels share the GPU with the
 * factorisation's leaf levels and fill what its top tree levels leave idle.  The results equal those of the two separate
 * calls.  Returns STF_EPIVOT if a pivot was perturbed and the solve itself
 * succeeded, else the solve's status. */
stf_status  stf_factor_solve(stf_problem pb, int32_t nrhs, const double* b, double* x, int on_device,
                             const stf_solve_opts* opts, stf_solve_info* info);
/* Stop rules of the stationary iteration: the FP64 true relative residual
 * |b - A x| / |b| <= tol, or Eq. (20): the summed 2-norms of the subdomains'
 * local fields on their overlapping regions (Omega_k outside I_k, the fields
 * E^F that the round transfers) fall below tol times the same sum after the
 * initial local solves (Eq. (20) with its TOL taken relative to that scale). */
enum { STF_STOP_RESIDUAL = 0, STF_STOP_OVERLAP = 1 };

/* Algorithm 1 as the paper runs it: a stationary iteration of source-transfer
 * rounds (Sec. 2.3).  x_0 = B b (the initial local solves, Eq. (14)), then
 * x <- x + B (b - A x) (the transferred sources of Eqs. (18)-(19) solved
 * locally and summed as in Eq. (21)), until the stop rule `stop` (STF_STOP_*)
 * holds or max_rounds rounds after x_0 (0 <= max_rounds <= 100000).  b, x:
 * ny*nx complex, host or device (on_device).  hist, hist_energy (host, each
 * may be NULL): max_rounds + 1 doubles, the relative residual, resp. the
 * overlap energy of Eq. (20), of x_0 and of every round taken.  *rounds_out
 * (may be NULL): rounds taken after x_0.  Returns STF_ENOCONV when the rule
 * was not met (x, the histories, *rounds_out still written), STF_ENAN on a
 * non-finite value, STF_ESTATE before stf_factor. */
stf_status  stf_stationary_solve(stf_problem pb, const double* b, double* x, int on_device,
                                 double tol, int32_t max_rounds, int32_t stop, double* hist,
                                 double* hist_energy, int32_t* rounds_out);
/* Time-averaged power through a grid line, the line integral
 * U = 1/2 int_l Re(E x H*) of Sec. 3.2 for E = E_z z, with H from Faraday's law
 * (exp(+j w t), w mu = k0, fields normalised so that eta0 = 1):
 * H_x = (j/k0) dE_z/dy, H_y = -(j/k0) dE_z/dx, E_z on the line the mean of the
 * two node rows, the derivative their difference over the step.  axis 1: the
 * line between node rows index and index + 1 (0 <= index < ny - 1), nodes x in
 * [lo, hi) (0 <= lo <= hi <= nx), power towards +y; axis 0: between node
 * columns index and index + 1, nodes y in [lo, hi), power towards +x.  The
 * line should lie outside the PML (the step is the grid step there).  e: ny*nx
 * complex field, host or device (on_device); *out (host): the power. */
stf_status  stf_line_flux(stf_problem pb, const double* e, int on_device, int32_t axis,
                          int32_t index, int32_t lo, int32_t hi, double* out);
/* Radar cross section (2D scattering width) by the near-to-far-field transform,
 * the quantity the paper compares with the Mie series (Sec. 3.1, Fig. 5a).  e:
 * the SCATTERED field (ny*nx complex, host or device), e.g. the solution of the
 * scattered-field source of Eq. (7), for a unit incident wave.  The contour is
 * the rectangle through the half-node lines x = (box[0] + 1/2) dx,
 * (box[1] + 1/2) dx, y = (box[2] + 1/2) dy, (box[3] + 1/2) dy (0 <= box[0] <
 * box[1] < nx - 1, likewise y); it must enclose every scatterer and source and
 * lie outside the PML.  With u the mean of the two node lines an edge
 * separates and du/dn their difference over the step (outward), F(phi) =
 * sum [du/dn - j k0 (rhat . n) u] exp(j k0 rhat . r) dl by the midpoint rule
 * (Green's representation with the outgoing Hankel function, exp(+j w t)), and
 * sigma(phi) = |F|^2 / (4 k0), phi measured from +x.  phis: nang angles (host);
 * sigma: nang doubles (host); F: 2 nang doubles (host, interleaved, may be NULL). */
stf_status  stf_rcs(stf_problem pb, const double* e, int on_device, const int32_t* box, int32_t nang,
                    const double* phis, double* sigma, double* F);
/* y = A x with the global FP64 operator (Eqs. (2), (9)).  x, y: ny*nx complex. */
stf_status  stf_apply(stf_problem pb, const double* x, double* y, int on_device);
/* One source-transfer round z = sum_k P_k A_k^{-1} R_k^I v (Eqs. (14), (21)):
 * restriction to each subdomain's own box, local multifrontal solve
 * (Eq. (23)), and the sum of the full local fields.  v, z: ny*nx complex. */
stf_status  stf_precond_apply(stf_problem pb, const double* v, double* z, int on_device);
/* The same round for nrhs vectors (v, z: nrhs*ny*nx complex), swept up to four
 * at a time with one read of the factors; each result equals that of
 * stf_precond_apply on its own vector. */
stf_status  stf_precond_apply_batch(stf_problem pb, int32_t nrhs, const double* v, double* z,
                                    int on_device);
/* One application of the preconditioner in a given order (STF_ORDER_*; the
 * additive order is stf_precond_apply): v, z: ny*nx complex, host or device. */
stf_status  stf_sweep_apply(stf_problem pb, int32_t order, const double* v, double* z,
                            int on_device);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the round of
 * stf_precond_apply on device buffers, allocating nothing.  v, z: ny*nx complex,
 * DEVICE pointers (caller-owned, ordered on the context stream; the call returns
 * after enqueueing, without synchronising).  The round's workspace (front
 * vectors and local fields, fully written before they are read) lives in a
 * static per-device array of 128 MiB that the library holds until the process
 * ends: problems whose workspace exceeds it (about 1.2M DoF with complex128
 * fronts, 2.3M with complex64 at 8 x 8 subdomains) are rejected with STF_EINVAL
 * before anything is launched.  Every call on one device shares that array, so
 * calls whose work overlaps on one device (several streams or host threads)
 * race.  STF_ESTATE before stf_factor.  No event timing is recorded. */
stf_status  stf_precond_apply_noalloc(stf_problem pb, const double* v, double* z);
/* Batched solve (Algorithm 1's parallel loop over subdomains, extended over
 * problems): factor the nprob problems together, one launch per elimination-tree
 * level over the fronts of all of them (Eq. (22)), then solve all their right-hand
 * sides by FGMRES in lockstep, every kernel launch covering every (problem,
 * right-hand side) system, one source-transfer round per preconditioner
 * application (Eqs. (14)-(21)); each system keeps its own Krylov basis and stops
 * on its own FP64 true residual (convergence is tracked on the device, the host
 * looks once per FGMRES cycle, and a cycle is replayed as one HIP graph).
 * probs: nprob distinct assembled problems of this context with the same
 * front_prec; nrhs[p] >= 1; b[p], x[p]: nrhs[p]*ny_p*nx_p complex each, all host
 * or all device (on_device); x[p] holds the guesses for STF_X0_USER.
 * opts: as stf_solve with restart <= 32, rounds <= 1, debug_fault = 0 (any order;
 * a staged order runs stage t of every problem in the same launches).
 * info: NULL, or nprob pointers (each NULL or an array of nrhs[p] infos).
 * The factors live in a state cached on the context and reused while the same
 * problems (and assemblies) are passed; every call factors again (a problem's
 * own stf_factor state is neither needed nor touched).  Each system's result
 * satisfies its tolerance like a solo solve; kernel variants are chosen per
 * batched level, so results agree with solo solves to the tolerance, not bit
 * for bit.  Returns the worst per-system status, or STF_EPIVOT when all
 * converged after a perturbed pivot. */
stf_status  stf_batch_solve(stf_ctx ctx, int32_t nprob, const stf_problem* probs,
                            const int32_t* nrhs, const double* const* b, double* const* x,
                            int on_device, const stf_solve_opts* opts, stf_solve_info* const* info);
stf_status  stf_problem_info(stf_problem pb, stf_plan_info* out);
void        stf_problem_destroy(stf_problem pb);          /* NULL-safe */

/* ---- autotuner ------------------------------------------------------------
 * Not part of the method: a search over the launch shapes of the per-level
 * kernels of Eq. (22)'s multifrontal factorisation and of the source-transfer
 * round's forward and backward sweeps (Eqs. (18)-(19)), which change how the
 * work is spread over the GPU, not what is computed (results agree to rounding).
 * A level's signature is (operation, front precision, right-hand sides per
 * sweep, fronts in the level, largest front order m, largest separator p).
 *
 * stf_autotune times every candidate shape of every level (HIP events, `reps`
 * passes of 1..100, the fastest pass counting) for the problems given: one
 * problem (its own fronts), or nprob > 1 problems as the set that
 * stf_batch_solve builds for the same problems in the same order.  what: a
 * sum of 1 (the factorisation), 2 (the additive round's sweeps with nrhs
 * (1..4) right-hand sides), 4, 8, 16, 32 (the subtree choice of the staged
 * orders rows, rows + columns, diagonal, two colours: whole applications timed
 * level by level and with subtree sweeps in every stage, operation 3 + order
 * below).  The fastest shape per level signature is kept in the context
 * and used by every later factorisation and round on it whose levels have
 * that signature (solo, batched, staged or allocation-free); other levels keep
 * the built-in rule.  Needs assembled problems of this context with one front
 * precision (STF_ESTATE otherwise); leaves them factored (the factorisation
 * is run again with the chosen shapes; a perturbed pivot is not reported
 * here).  Contents of the round's workspaces are overwritten.  With the
 * sweeps, it then times whole rounds' sweeps level by level against subtree
 * sweeps (the deep levels swept 1, 2, 4 or 8 subtrees per workgroup, each
 * root depth that fits) and keeps the fastest for the set's signature
 * (operation 3 in the entries below).  report: NULL or filled with the levels timed, how many
 * changed from the built-in shape, the summed level times with the built-in
 * and with the chosen shapes (ms), the chosen subtree root depth (-1: level
 * by level, or no sweeps tuned) and the sweeps' time with the built-in and
 * with the chosen subtree choice (ms). */
typedef struct {
  int32_t levels;
  int32_t changed;
  double  ms_default;
  double  ms_tuned;
  int32_t fuse_depth;
  double  ms_round_default;
  double  ms_round_tuned;
} stf_tune_report;
stf_status  stf_autotune(stf_ctx ctx, int32_t nprob, const stf_problem* probs, int32_t nrhs,
                         int32_t what, int32_t reps, stf_tune_report* report);
/* Test hook: sets, without timing, the entry of every level of the given
 * problems (as stf_autotune selects them) to the level's candidate shape
 * `index` (>= 0; the last candidate where a level has fewer; 0 is the
 * built-in shape), and with the sweeps (what & 2, and the staged orders'
 * bits 4, 8, 16, 32) the subtree choice of the set to its option `index` (0 level
 * by level, the built-in choice, then each root depth and subtrees per
 * workgroup that fit).  *max_candidates (may be NULL) receives the largest
 * candidate count over the levels, so that index = 0 .. max - 1 visits every
 * candidate; every one must give the same results to rounding. */
stf_status  stf_tune_pick(stf_ctx ctx, int32_t nprob, const stf_problem* probs, int32_t nrhs,
                          int32_t what, int32_t index, int32_t* max_candidates);
/* Host-only check of the launch-shape rules on a problem's plan (no device):
 * the levels of the plan (tree depths over all subdomains), the number of
 * candidate shapes over all levels and operations, and how many built-in or
 * candidate shapes fail the validity rules (0 expected).  The device limits
 * are those of the current device when one is present, else gfx950's (160 KiB
 * of LDS per workgroup, 256 compute units). */
stf_status  stf_debug_level_shapes(const stf_params* prm, int32_t nrhs, int32_t* nlevels,
                                   int32_t* ncandidates, int32_t* invalid);
/* The context's tuned shapes as a text file for this device architecture
 * (first line: "stfdfd-tune 1 <arch> <entries>", then one entry per line), and
 * back: a file for another architecture, or malformed, is STF_EINVAL and
 * changes nothing; loaded entries replace those of the same signature.  An
 * entry whose shape cannot run its level is ignored at launch. */
stf_status  stf_tune_save(stf_ctx ctx, const char* path);
stf_status  stf_tune_load(stf_ctx ctx, const char* path);
stf_status  stf_tune_clear(stf_ctx ctx);
/* Number of entries (-1 for a NULL ctx), and entry i (0-based, in signature
 * order): key = {op (0 factorisation, 1 forward sweep, 2 backward sweep),
 * bytes per complex entry, nrhs (0 for the factorisation), fronts in the
 * level, max m, max p}; shape = {kind, nb or kp, ntf or ntl, parts};
 * ms = {chosen, built-in}.  Operation 3 (the subtree choice of a set): key =
 * {3, bytes, nrhs, fronts of the set, deepest level, subdomains}, shape =
 * {1, root depth or -1 (level by level), subtrees per workgroup (1, 2, 4, 8),
 * 0}; operations 4, 5, 6, 7: the same for the stages of the orders rows,
 * rows + columns, diagonal, two colours.  Any output pointer may be NULL. */
int32_t     stf_tune_count(stf_ctx ctx);
stf_status  stf_tune_entry(stf_ctx ctx, int32_t i, int32_t* key, int32_t* shape, double* ms);

/* ---- learned warm start -------------------------------------------------
 * A spectral neural operator on n x n tiles: pointwise lift of the cin
 * input features to W channels, L layers h <- act(K h + W_l h + c_l) with the
 * spectral convolution K h = Finv(R . Ftrunc(h)) over the modes kx in [0, M),
 * ky in [-M, M) (complex weights R per mode and channel pair), GELU (tanh
 * form) after every layer but the last, and a pointwise projection to the
 * real and imaginary part of the field.  Features of a tile:
 * ((Re eps_node - 1) / 4, Re b, Im b).  Parameters form one flat FP32 vector:
 * P_w (W, cin), P_b (W), per layer Re R (W, W, 2M, M), Im R, W_l (W, W),
 * c_l (W), then Q_w (2, W), Q_b (2).  The library keeps that vector as an FP32
 * master copy (get/set_params, the Adam step) and computes with the master
 * copy rounded to BF16 (round to nearest, ties to even: the weights), refreshed
 * after every change; activations, transforms and every sum are FP32 (the
 * transforms on the FP32 matrix cores), and gradients are taken at the BF16
 * weights.  Training minimises the mean over tiles of |y - t|^2 / |t|^2 with
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the master copy.
 * Tensors are planar [tile][channel][y][x], x fastest. */
typedef struct stf_nn_s* stf_nn;
typedef struct {
  int32_t n;          /* tile side in nodes (2M <= n) */
  int32_t width;      /* W: 4, 8, 16 or 32 */
  int32_t modes;      /* M (1 <= M <= 22, 2M <= n) */
  int32_t layers;     /* L >= 1 */
  int32_t cin;        /* input features: 3 */
  int32_t max_batch;  /* largest number of tiles per call */
} stf_nn_config;

int64_t     stf_nn_param_count(const stf_nn_config* cfg);       /* -1 if cfg is invalid */
/* params: host array of stf_nn_param_count floats (copied). */
stf_status  stf_nn_create(stf_ctx ctx, const stf_nn_config* cfg, const float* params, stf_nn* out);
void        stf_nn_destroy(stf_nn nn);                          /* NULL-safe */
stf_status  stf_nn_get_params(stf_nn nn, float* params);        /* host, param_count floats */
stf_status  stf_nn_set_params(stf_nn nn, const float* params);  /* host; resets the Adam moments */
/* y (batch, 2, n, n) = network(f (batch, cin, n, n)); device pointers. */
stf_status  stf_nn_forward(stf_nn nn, int32_t batch, const float* f, float* y);
/* Loss and gradient of the loss for one batch (device f, t (batch, 2, n, n));
 * grad: host array of param_count floats, or NULL. */
stf_status  stf_nn_loss_grad(stf_nn nn, int32_t batch, const float* f, const float* t,
                             double* loss, float* grad);
/* loss_grad followed by one Adam step with learning rate lr; step counts from 1. */
stf_status  stf_nn_train_step(stf_nn nn, int32_t batch, const float* f, const float* t, double lr,
                              int32_t step, double* loss);
/* Network used by STF_X0_LEARNED solves on this context (NULL detaches; not owned). */
stf_status  stf_ctx_set_nn(stf_ctx ctx, stf_nn nn);
/* The blended guess for source b on problem pb: tiles of side n at stride n/2
 * over the physical interior (last tile flush with the far edge), weights
 * sin^2(pi (i + 1/2) / n) per axis held at 1 on the outer half of edge tiles,
 * divided by the summed weights; 0 in the global PML.  b, x0: ny*nx complex.
 * Needs an assembled problem whose interior is at least n x n. */
stf_status  stf_nn_initial_guess(stf_problem pb, stf_nn nn, const double* b, double* x0,
                                 int on_device);
/* Training data of problem pb on the same tiles (device pointers): features
 * f (ntiles, cin, n, n) of source b, and the field x as t (ntiles, 2, n, n)
 * (real, imaginary).  f or t may be NULL; *ntiles receives the tile count
 * (call with f = t = NULL to size the buffers). */
stf_status  stf_nn_tile_data(stf_problem pb, stf_nn nn, const double* b, const double* x, float* f,
                             float* t, int32_t* ntiles);

#ifdef __cplusplus
}
#endif
#endif /* STFDFD_H */
