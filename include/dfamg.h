/*
 * dfamg.h - C ABI of the MI355X subdomain-deflated local-AMG Krylov solver.
 *
 * The method is the one of Demidov & Rossi, "Subdomain deflation combined
 * with local AMG" (arXiv:1710.03940):
 *   - the solution is split as x = y + Z lambda with Z the subdomain
 *     deflation basis (section "Subdomain deflation", eq. (2));
 *   - a Krylov method solves the deflated system P(A y) = P(b) with the
 *     projector P = I - A Z E^{-1} Z^T, E = Z^T A Z (eqs. (3)-(7)), applied
 *     matrix-free as t1 = Z^T r, t2 = E^{-1} t1, r* = r - (AZ) t2 with AZ and
 *     E formed explicitly (section "Implementation", projector equation);
 *   - the preconditioner is block AMG without overlap: one smoothed-
 *     aggregation V-cycle per subdomain, built on the square diagonal block
 *     of A (section "Implementation");
 *   - lambda = E^{-1} Z^T (b - A y) recovers x (eqs. (4)-(5));
 *   - alternatively (solver FGMRES), the deflation with an exact or inexact
 *     E^{-1} preconditions A x = b itself, combined multiplicatively with the
 *     block AMG, inside restarted flexible GMRES (section "On precision of
 *     the coarse system solution").
 * Usage follows Listing 1: setup once from a CRS matrix and parameters, then
 * solve(rhs, x) with x as the initial guess, returning iterations and the
 * relative residual.
 *
 * Conventions for every entry point:
 *   - every function returns a dfamg_status; no C++ exception crosses the ABI;
 *   - on failure a message is available from dfamg_last_error(handle) (or
 *     dfamg_last_error(NULL) when no handle exists yet);
 *   - host pointers are read during the call only; the caller keeps
 *     ownership;
 *   - device pointers (rhs, x of the solve calls) are HIP device memory on the
 *     device that was current at setup, borrowed for the duration of the call;
 *   - a handle is not thread-safe; all of its GPU work is ordered on the
 *     stream given at setup.
 */
#ifndef DFAMG_H
#define DFAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DFAMG_OK = 0,
    DFAMG_EINVAL = 1,      /* malformed input or parameters (nothing changed) */
    DFAMG_ENOMEM = 2,      /* host or device allocation failed               */
    DFAMG_ESINGULAR = 3,   /* E or a coarsest-level block is not invertible,
                              or a local deflation block is rank deficient    */
    DFAMG_ENOCONV = 4,     /* maxiter reached; outputs hold the last iterate  */
    DFAMG_EBREAKDOWN = 5,  /* BiCGStab(2): a scalar it divides by (rho,
                              (r~, v), omega, sigma) became exactly zero;
                              FGMRES: a zero diagonal of the rotated
                              Hessenberg matrix (x holds the iterate formed
                              from the steps before it)                      */
    DFAMG_ENAN = 6,        /* a non-finite value appeared in the iteration    */
    DFAMG_EHIP = 7,        /* a HIP runtime call failed                       */
    DFAMG_ENOGPU = 8       /* no usable gfx950 device                         */
} dfamg_status;

enum { DFAMG_SOLVER_CG = 0, DFAMG_SOLVER_BICGSTAB = 1, DFAMG_SOLVER_BICGSTAB2 = 2, DFAMG_SOLVER_FGMRES = 3 };
/* Coarse solve t2 = E_hat t1 of the FGMRES path (section "On precision of
 * the coarse system solution"): EXACT applies E^{-1} in FP64; FP32 applies
 * E^{-1} rounded to single precision, in single precision; CG runs
 * Jacobi-preconditioned CG on E from zero until ||t1 - E t2|| <= coarse_rtol
 * ||t1|| or coarse_maxiter steps (E must be symmetric with a positive
 * diagonal), so the preconditioner changes from one application to the next.
 * The projected solvers (CG, BiCGStab, BiCGStab(2)) always use EXACT: the
 * deflated system is only equivalent to A x = b when E is solved exactly. */
enum { DFAMG_COARSE_EXACT = 0, DFAMG_COARSE_FP32 = 1, DFAMG_COARSE_CG = 2 };
enum { DFAMG_PREC_FP64 = 0, DFAMG_PREC_MIXED = 1 };
/* Smoother of the V-cycle: SPAI-0 (m_i = a_ii / sum_j a_ij^2), damped
 * Jacobi, or block SPAI-0 for point-block matrices (block_size b: per node
 * the b x b block M_i = A_ii^T (A_(i,:) A_(i,:)^T)^{-1} minimising
 * ||I - M A||_F over block-diagonal M; with b = 1 it is SPAI-0). */
enum { DFAMG_SMOOTHER_SPAI0 = 0, DFAMG_SMOOTHER_JACOBI = 1, DFAMG_SMOOTHER_BLOCK_SPAI0 = 2 };
/* Sparse layouts: SELL slices, CSR (several lanes per row), CSR staged from
 * per-tile gather lists, BSR4: 4 x 4 dense blocks with one column index per
 * block, for point-block matrices (block_size 4, the velocity-pressure nodes
 * of the Navier-Stokes problem; explicit zeros of a block are stored), and
 * COLUMN_TILED: the restriction operators split by column tiles of the
 * finer vector (each tile staged once in LDS, one partial sum per row
 * segment, the partials added per row in tile order), every other operator
 * in SELL. */
enum { DFAMG_FORMAT_AUTO = 0, DFAMG_FORMAT_CSR = 1, DFAMG_FORMAT_SELL = 2, DFAMG_FORMAT_CSR_GATHER = 3,
       DFAMG_FORMAT_BSR4 = 4, DFAMG_FORMAT_COLUMN_TILED = 5 };
/* Preconditioner M: the block-local SA-AMG V-cycle, none (M = I), or the
 * purely local SPAI-0 diagonal m_i = a_ii / sum_j a_ij^2 (the velocity-block
 * preconditioner of the Schur pressure correction, section "Navier-Stokes
 * problem"). */
enum { DFAMG_PRECOND_AMG = 0, DFAMG_PRECOND_NONE = 1, DFAMG_PRECOND_SPAI0 = 2 };

typedef struct {
    int32_t solver;         /* DFAMG_SOLVER_*; CG needs a symmetric A; one
                               BiCGStab(2) iteration is one cycle of two BiCG
                               steps and the minimal-residual step (four
                               operator products).  FGMRES solves A x = b
                               itself (no deflated system, no recovery) with
                               restarted flexible GMRES, preconditioned by
                               B(v) = Z E_hat Z^T v + M^{-1}(v - AZ E_hat Z^T v):
                               the deflation combined multiplicatively with
                               the block AMG M; one iteration is one Arnoldi
                               step                                           */
    int32_t maxiter;        /* iteration limit (default 1000)                  */
    double  rtol;           /* stop when ||r_k|| <= rtol ||b|| (default 1e-8)  */
    int32_t precision;      /* DFAMG_PREC_FP64: whole path FP64; MIXED: AMG
                               hierarchy, smoother and V-cycle vectors FP32,
                               Krylov vectors, dots and deflation FP64        */
    int32_t smoother;       /* DFAMG_SMOOTHER_SPAI0 (default), _JACOBI or
                               _BLOCK_SPAI0                                   */
    double  jacobi_omega;   /* damped Jacobi damping (default 0.8, Listing 1)  */
    int32_t coarse_enough;  /* stop coarsening at <= this many unknowns (500)  */
    double  eps_strong;     /* strength threshold on level 0 (0.08), halved
                               on every coarser level                          */
    int32_t max_levels;     /* hierarchy depth limit (20)                      */
    int32_t block_size;     /* 1 (scalar) or 2..8 (point blocks, interleaved)  */
    int32_t precond;        /* DFAMG_PRECOND_AMG (default), _NONE (M = I) or
                               _SPAI0 (diagonal)                              */
    int32_t spmv_format;    /* DFAMG_FORMAT_*: AUTO lets the setup autotuner
                               time the candidates on the device (BSR4 among
                               them when block_size is 4); CSR_GATHER
                               restricts the multigrid operators to CSR that
                               stages each tile's distinct input columns in
                               LDS (a gather list; unstaged CSR where the list
                               exceeds 64 KiB), the outer operator to CSR;
                               BSR4 (block_size 4 only) stores every operator
                               in 4 x 4 blocks; COLUMN_TILED stores the
                               restrictions (the fused operator B with one
                               pre-smoothing sweep) in column tiles of 512
                               unknowns and the rest in SELL, untimed     */
    int32_t autotune;       /* 1 (default): time the candidate layouts of every
                               matrix at setup and keep the fastest; 0: one
                               fixed layout (SELL, one row per lane, natural
                               order, 32-bit columns; CSR with 8 lanes when
                               spmv_format = CSR, and with gather lists for
                               the multigrid operators when CSR_GATHER), so
                               that two handles built
                               from the same subdomains sum every dot product
                               in the same order (bitwise-equal results).
                               Environment: DFAMG_TUNE_CACHE names a file that
                               records the chosen layouts by matrix structure
                               across processes (read, then appended to);
                               DFAMG_TUNE_VERIFY (any value) applies every
                               candidate once to a varied input and fails the
                               setup with DFAMG_EINVAL, the message naming both
                               layouts, if one differs from the operator's
                               first candidate beyond rounding               */
    int32_t graph_iters;    /* Krylov iterations per captured HIP graph;
                               0 launches kernels directly (default 16)       */
    int32_t host_threads;   /* setup worker threads, 0 = hardware concurrency  */
    int32_t verbose;        /* 1 prints setup/solve phase times to stderr,
                               2 also every autotuning candidate's time       */
    int32_t profile;        /* 1 records HIP events around the outer SpMV and
                               the level-0 restriction (DFAMG_KERNEL_SPMV and
                               _PRESMOOTH0) of the Krylov iterations of the
                               first captured graph of every solve (every
                               iteration with direct launches or FGMRES;
                               later chunks replay a graph without event
                               nodes), 2 around every kernel span of every
                               iteration (inside the captured graph as well);
                               averages in dfamg_stats                        */
    int32_t restart;        /* FGMRES: Arnoldi steps per cycle, 1..64 (30);
                               one captured graph runs one cycle              */
    int32_t coarse_solve;   /* DFAMG_COARSE_*; FP32 and CG need solver = FGMRES */
    double  coarse_rtol;    /* COARSE_CG: relative residual target (1e-2)    */
    int32_t coarse_maxiter; /* COARSE_CG: step limit per coarse solve (100)  */
    int32_t flexible_cg;    /* CG only: 0 (default) beta = rho'/rho; 1 the
                               flexible (Polak-Ribiere) beta
                               (r', s' - s) / rho, equal in exact arithmetic
                               for a fixed preconditioner and robust when the
                               preconditioner varies (costs one more vector
                               read per iteration)                           */
    int32_t npre;           /* V-cycle pre-smoothing sweeps, 0..4 (1); with a
                               value other than 1 the level operators keep
                               the pre-smoothing, residual and restriction
                               as separate steps                              */
    int32_t npost;          /* V-cycle post-smoothing sweeps, 1..4 (1).  The
                               paper's runs use V(1,1); CG needs npre = npost
                               for a symmetric preconditioner.  The block
                               SPAI-0 smoother supports V(1,1) only           */
    int32_t setup_device;   /* 0 (default): the smoothed-aggregation
                               hierarchies are built on the host; 1: on the
                               current GPU (strength, aggregation, smoothed
                               prolongator, Galerkin products), equal to the
                               host's bit for bit; block_size 1 and a
                               diagonal smoother (SPAI-0, damped Jacobi) only */
} dfamg_params;

/* Fill *p with the defaults listed above. */
void dfamg_params_default(dfamg_params *p);

typedef struct dfamg_handle_s *dfamg_handle;

/*
 * Build the solver on the current HIP device.
 *   n          number of unknowns (rows of the square matrix), n >= 1
 *   row_ptr    host, n+1 entries, 0-based CRS row pointers, monotone,
 *              row_ptr[0] == 0
 *   col        host, row_ptr[n] column indices in [0, n); no duplicates
 *              within a row (any order)
 *   val        host, row_ptr[n] finite FP64 values
 *   part       host, n subdomain ids in [0, nsub); every subdomain non-empty;
 *              with block_size b > 1 all b unknowns of a node (rows
 *              b*k .. b*k+b-1) share one subdomain
 *   nsub       number of subdomains (>= 1)
 *   ndv        deflation vectors per subdomain (0..8); 0 disables deflation
 *   Z          host, n x ndv row-major FP64: row i holds the ndv local
 *              deflation vectors of subdomain part[i] at unknown i (sections
 *              "Constant deflation", "Linear deflation"); may be NULL if
 *              ndv == 0
 *   stream     hipStream_t for all work of this handle (NULL = null stream)
 *   out        receives the handle
 * Errors: EINVAL (validation, before any device work), ESINGULAR (E, a
 * coarsest block or a local Z block not invertible / of full rank, with the
 * subdomain named in the message), ENOMEM, EHIP, ENOGPU.
 */
dfamg_status dfamg_setup(const dfamg_params *prm, int64_t n,
                         const int64_t *row_ptr, const int32_t *col,
                         const double *val, const int32_t *part, int32_t nsub,
                         int32_t ndv, const double *Z, void *stream,
                         dfamg_handle *out);

/*
 * Batched setup: nsys independent systems concatenated into one
 * block-diagonal matrix.  sys_row_off (host, nsys+1 entries) gives the row
 * range of every system; no matrix entry may couple two systems; subdomain
 * ids are global across the batch and each subdomain lies inside one system.
 * Every system gets its own deflation operator E, its own Krylov scalars and
 * its own convergence test; all of them advance together in the same
 * kernel launches.  Other arguments as in dfamg_setup.
 */
dfamg_status dfamg_setup_batched(const dfamg_params *prm, int32_t nsys,
                                 const int64_t *sys_row_off, int64_t n,
                                 const int64_t *row_ptr, const int32_t *col,
                                 const double *val, const int32_t *part,
                                 int32_t nsub, int32_t ndv, const double *Z,
                                 void *stream, dfamg_handle *out);

/*
 * Setup of the Schur pressure-correction solver for a velocity-pressure
 * system [K G; D S] (section "Navier-Stokes problem"): restarted flexible
 * GMRES on A x = b (prm->solver must be DFAMG_SOLVER_FGMRES; restart, rtol,
 * maxiter from prm; the paper runs FGMRES(50)) preconditioned by
 *   1. u^ ~ K^{-1} r_u,  2. p ~ S^^{-1} (r_p - D u^),  3. u ~ K^{-1} (r_u - G p)
 * with S^ = S - D diag(K)^{-1} G formed on the host.  The K solves are
 * FGMRES(5) with the local SPAI-0 preconditioner to 1e-3 (at most 5 steps);
 * the pressure solves are FGMRES(20) to 1e-2 (at most 20 steps) on S^,
 * preconditioned by the subdomain deflation (exact E^{-1}) combined with the
 * block-local AMG of S^ (precision, smoother, coarse_enough and eps_strong
 * from prm): the settings of the paper's JSON listing.  Every inner solve
 * starts from zero; one reaching its step limit returns its last iterate.
 *   pmask   host, n flags: nonzero marks a pressure unknown; the velocity
 *           and pressure unknowns are numbered in ascending index order
 *   part    host, one subdomain id in [0, nsub) per pressure unknown
 *   Z       host, (number of pressure unknowns) x ndv row-major deflation
 *           vectors of the pressure block (as in dfamg_setup)
 * Other arguments as in dfamg_setup.  The handle is solved with dfamg_solve;
 * dfamg_apply and the batched calls reject it.  Errors as dfamg_setup, and
 * EINVAL when a block is empty or a diagonal entry of K is zero.
 */
dfamg_status dfamg_setup_schur(const dfamg_params *prm, int64_t n,
                               const int64_t *row_ptr, const int32_t *col,
                               const double *val, const int32_t *pmask,
                               const int32_t *part, int32_t nsub, int32_t ndv,
                               const double *Z, void *stream, dfamg_handle *out);

/*
 * Solve A x = b (single-system handle).
 *   rhs       device, n FP64 values (not modified)
 *   x         device, n FP64 values: initial guess on entry, solution on exit
 *   iters     host out: Krylov iterations performed
 *   relres    host out: ||r_k|| / ||b|| of the recurrence residual at exit
 *   relres_true host out: ||b - A x|| / ||b|| recomputed in FP64 at exit
 *   history   host out (may be NULL): relative residual of iterations
 *             0..iters, at most history_cap values written
 * Returns after the stream has been synchronised.  b == 0 gives x = 0,
 * iters = 0.  ENOCONV when maxiter is reached (x holds the recovered last
 * iterate).  ENAN when a non-finite value appears.
 */
dfamg_status dfamg_solve(dfamg_handle h, const double *rhs, double *x,
                         int32_t *iters, double *relres, double *relres_true,
                         double *history, int32_t history_cap);

/*
 * Batched solve: rhs and x are the concatenated device vectors; iters,
 * relres_true and status are host arrays of nsys entries (status may be
 * NULL).  Returns DFAMG_OK when every system converged, else the first
 * non-OK per-system status.
 */
dfamg_status dfamg_solve_batched(dfamg_handle h, const double *rhs, double *x,
                                 int32_t *iters, double *relres_true,
                                 int32_t *status);

/* Single operators of the method on device vectors in the caller's
 * (original) ordering, for checking them one at a time. */
enum {
    DFAMG_OP_SPMV = 0,      /* out = A in                                     */
    DFAMG_OP_PROJECT = 1,   /* out = P in = in - AZ E^{-1} Z^T in             */
    DFAMG_OP_PRECOND = 2,   /* out = M^{-1} in (one V-cycle per subdomain)    */
    DFAMG_OP_RECOVER = 3    /* out = in + Z E^{-1} Z^T (b - A in), b = the
                               right-hand side of the last solve             */
};
dfamg_status dfamg_apply(dfamg_handle h, int32_t op, const double *in,
                         double *out);

typedef struct {
    int64_t n, nnz;
    int32_t nsys, nsub, ndv, m_total;
    int32_t nlevels_max;              /* deepest hierarchy over subdomains   */
    int64_t level_rows[20];           /* packed unknowns per level           */
    int64_t level_nnz[20];            /* packed nnz(A_l) per level           */
    int64_t level_p_nnz[20];          /* packed nnz(P_l) per level           */
    int32_t format_outer;             /* chosen DFAMG_FORMAT_* for A         */
    int32_t format_level[20];         /* chosen format for A_l               */
    int32_t lanes_level[20];          /* lanes per row for CSR formats       */
    double  setup_host_s;             /* host setup (hierarchy, AZ, E) time  */
    double  setup_device_s;           /* uploads, E inversion, tuning time   */
    double  solve_s;                  /* wall time of the last solve call    */
    int64_t device_bytes;             /* device memory owned by the handle   */
    double  bytes_per_iter;           /* algorithmic HBM bytes per Krylov
                                         iteration (whole batch) of CG,
                                         BiCGStab and FGMRES; 0 for
                                         BiCGStab(2)                          */
    /* Per-kernel profile (params.profile = 1), indexed by DFAMG_KERNEL_*:
       launches timed, total milliseconds and algorithmic bytes per launch. */
    int64_t kernel_calls[16];
    double  kernel_ms[16];
    double  kernel_bytes[16];
    int32_t profile_in_graph;         /* 1: events were replayed inside the
                                         captured graphs; 0: the profiled
                                         solves launched kernels directly   */
    char    layouts[1024];            /* text: the layout the autotuner chose
                                         for every matrix, NUL-terminated    */
    double  outer_layout_bytes;       /* bytes one outer-operator launch
                                         moves in its chosen layout (stored
                                         entries incl. padding and index
                                         width, couplings, vectors, Z as
                                         stored); the algorithmic figure is
                                         kernel_bytes[DFAMG_KERNEL_SPMV]     */
    int64_t coarse_iters;             /* COARSE_CG: CG steps of all coarse
                                         solves of the last solve call (sum
                                         over systems)                        */
    int64_t schur_inner_iters[2];     /* Schur handle: iterations of the
                                         velocity and of the pressure inner
                                         solves in the last solve call        */
    double  setup_hierarchy_s;        /* hierarchy construction time (part of
                                         setup_host_s)                        */
    int32_t setup_hierarchy_device;   /* 1: hierarchies built on the GPU      */
} dfamg_stats;

/* Kernel ids of the profile: the outer SpMV with its fused (p,q) and Z^T q
 * epilogue, the per-system projection reduction (t1 sums, t2 = E^{-1} t1,
 * alpha), the fused deflation-correction / Krylov update, the stopping test,
 * the level-0 V-cycle kernels, everything on coarser levels (including the
 * coarsest direct solves) as one span, and the (r,s) / direction update;
 * the coarser span is also split into the level-1 downward step (pre-
 * smoothing residual and restriction), the level-1 upward step
 * (prolongation and post-smoothing) and everything deeper (levels >= 2 and
 * all coarsest direct solves).
 * When level 0 applies the pre-smoothing sweep, the residual and the
 * restriction as one operator (chosen at setup when it is faster), that
 * kernel is PRESMOOTH0 and RESTRICT0 records no launches. */
enum {
    DFAMG_KERNEL_SPMV = 0, DFAMG_KERNEL_PROJECT = 1, DFAMG_KERNEL_UPDATE = 2,
    DFAMG_KERNEL_TEST = 3, DFAMG_KERNEL_PRESMOOTH0 = 4, DFAMG_KERNEL_RESTRICT0 = 5,
    DFAMG_KERNEL_COARSER = 6, DFAMG_KERNEL_PROLONG0 = 7, DFAMG_KERNEL_POSTSMOOTH0 = 8,
    DFAMG_KERNEL_DIRECTION = 9, DFAMG_KERNEL_RESTRICT1 = 10, DFAMG_KERNEL_DEEP = 11,
    DFAMG_KERNEL_UP1 = 12, DFAMG_KERNEL_COUNT = 13
};

dfamg_status dfamg_get_stats(dfamg_handle h, dfamg_stats *out);

/* Release every resource of the handle (NULL is accepted). */
dfamg_status dfamg_destroy(dfamg_handle h);

/* Last error message of the handle, or of the calling thread's last failed
 * setup when h is NULL.  The pointer stays valid until the next call. */
const char *dfamg_last_error(dfamg_handle h);

/*
 * Inspection of the setup: the same validation, permutation, hierarchy, AZ
 * and E construction that dfamg_setup performs, kept on the host so that it
 * can be compared with other implementations.  No device is touched, except
 * that with setup_device = 1 the hierarchies are built on the current GPU.
 */
typedef struct dfamg_plan_s *dfamg_plan;

dfamg_status dfamg_plan_create(const dfamg_params *prm, int32_t nsys,
                               const int64_t *sys_row_off, int64_t n,
                               const int64_t *row_ptr, const int32_t *col,
                               const double *val, const int32_t *part,
                               int32_t nsub, int32_t ndv, const double *Z,
                               dfamg_plan *out);

/* Level sizes of subdomain `sub` (user id): writes up to cap entries into
 * rows[l], nnz[l] (A_l) and p_nnz[l] (P_l, 0 on the coarsest), omega[l]
 * (0 on the coarsest); *nlevels receives the hierarchy depth. */
dfamg_status dfamg_plan_levels(dfamg_plan p, int32_t sub, int32_t cap,
                               int32_t *nlevels, int64_t *rows, int64_t *nnz,
                               int64_t *p_nnz, double *omega);

/* Aggregate ids (-1 = in no aggregate) of level `level` of subdomain `sub`,
 * in the subdomain's local order (ascending original index); *count gets the
 * number of nodes; at most cap ids written. */
dfamg_status dfamg_plan_aggregates(dfamg_plan p, int32_t sub, int32_t level,
                                   int64_t cap, int32_t *agg, int64_t *count);

/* CRS of matrix `which` (0 = A_l, 1 = P_l, 2 = B_l = R_l (I - A_l diag(m_l)),
 * the operator the solve applies for pre-smoothing from a zero guess,
 * residual and restriction together (empty with the block smoother),
 * 3 = the smoother M_l as a matrix: diagonal, or block diagonal for block
 * SPAI-0) of level `level` of subdomain `sub` in local numbering; pass NULL
 * arrays to query sizes only. */
dfamg_status dfamg_plan_level_matrix(dfamg_plan p, int32_t sub, int32_t level,
                                     int32_t which, int64_t *nrows,
                                     int64_t *ncols, int64_t *nnz,
                                     int64_t *row_ptr, int32_t *col,
                                     double *val);

/* E of system `sys` as a dense m x m row-major array (m = ndv * subdomains of
 * the system, columns ordered by user subdomain id then vector). */
dfamg_status dfamg_plan_coarse_operator(dfamg_plan p, int32_t sys, int32_t *m,
                                        double *E, int64_t cap);

dfamg_status dfamg_plan_destroy(dfamg_plan p);

/*
 * E^{-1} of system `sys` as the handle holds it on the device (the inverse
 * the projection applies), copied to the host buffer Einv (row-major m x m,
 * same ordering as dfamg_plan_coarse_operator); pass NULL to query m only.
 * EINVAL when cap < m * m or sys is out of range.
 */
dfamg_status dfamg_coarse_inverse(dfamg_handle h, int32_t sys, int32_t *m,
                                  double *Einv, int64_t cap);

/*
 * E = Z^T A Z of system `sys` assembled on the device from the handle's own
 * operator and deflation vectors (one operator product per column, the
 * operator's Z^T epilogue giving the column; the setup forms E this way for
 * coarse operators of 1024 or more unknowns), copied to the host buffer E
 * (row-major m x m, ordering as dfamg_plan_coarse_operator); NULL E queries
 * m.  Uses the handle's work vectors: not concurrent with a solve.
 */
dfamg_status dfamg_coarse_operator(dfamg_handle h, int32_t sys, int32_t *m, double *E,
                                   int64_t cap);

/*
 * Dense FP64 inverse of the host row-major n x n matrix a into out (host),
 * computed on the current device by one of the two eliminations the setup
 * uses for E (Gauss-Jordan, partial pivoting, first row of largest |a_ik|):
 * method 0, column panels of 64 with GEMM updates (rocBLAS on the FP64 matrix
 * cores), the form used for coarse operators of 1024 or more unknowns;
 * method 1, one pivot per step over the whole matrix, used for smaller
 * ones and the coarsest AMG blocks.  1 <= n <= 4096.  ESINGULAR when a pivot
 * column is exactly zero.  Synchronous.
 */
dfamg_status dfamg_dense_inverse(const double *a, int32_t n, int32_t method,
                                 double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * unblocked inverse of dfamg_dense_inverse (method 1) on device memory,
 * with no allocation by the library.  Its working storage (the augmented
 * n x 2n matrix, the pivot column and the job record, 4 MiB at the limit)
 * is one static array per GPU, which the process holds until it ends.
 *   a       device, n x n row-major FP64 (not modified)
 *   n       1 <= n <= DFAMG_NOALLOC_MAX_N; larger n is rejected (EINVAL)
 *   out     device, n x n row-major FP64: the inverse, bitwise equal to
 *           what dfamg_dense_inverse(a, n, 1, out) returns
 *   stream  hipStream_t for the work (NULL = null stream); the call
 *           synchronises it before returning
 * ESINGULAR when a pivot column is exactly zero (out unspecified).  Every
 * call starts from a freshly written workspace, but all calls on one GPU
 * share it: calls that overlap on the same GPU (from several threads, or on
 * several streams) race and give wrong results.
 */
#define DFAMG_NOALLOC_MAX_N 512
dfamg_status dfamg_dense_inverse_noalloc(const double *a, int32_t n, double *out,
                                         void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DFAMG_H */
