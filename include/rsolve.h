/*
 * rsolve.h -- C ABI of an MI355X (gfx950) block-ILU0-preconditioned BiCGStab
 * solver for BCSR matrices with 3x3 FP64 blocks.
 *
 * Problem statement followed (Qiu et al., "An Evaluation and Comparison of
 * GPU Hardware and Solver Libraries for Accelerating the OPM Flow Reservoir
 * Simulator"):
 *   - a matrix handed over as three arrays, nonzero blocks, row pointers and
 *     column indices, blocks stored row-major one after another, vectors as
 *     one contiguous array of 3 values per block row (Section "OPM Flow");
 *   - a sparsity pattern analysed once and reused while the values change
 *     every solve; rows reordered by level scheduling or graph colouring, or
 *     kept in natural order (Section "ILU0" of the implementation chapter);
 *   - ILU0 decomposition (Algorithm 2) and application (equations 3-4);
 *   - BiCGStab with a relative residual reduction (default 1e-2) and an
 *     iteration limit (default 200) (Section "Bicgstab solver");
 *   - a solver that may fail without being fatal, so the caller can fall
 *     back to another solver (Section "Fallback");
 *   - a check for zeros on the diagonal (runtime breakdown in Section
 *     "Profiling").
 *
 * Conventions for every entry point:
 *   - Return value: RS_OK (0), a positive non-fatal solver outcome, or a
 *     negative error.  Nothing is thrown across the ABI; nothing exits.
 *     rsolve_last_error() gives a text for the last error of the calling
 *     thread.
 *   - Pointers marked "mem" live where the `mem` argument says: RS_MEM_HOST
 *     or RS_MEM_DEVICE (device memory of the current HIP device).  They are
 *     borrowed for the duration of the call; device sources must stay valid
 *     until `stream` has passed the call's work.  The library never frees
 *     caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *     return a status read from the device (factor, solve) synchronise it.
 *   - Handles own every device buffer they allocate.  A handle must not be
 *     used from two host threads at once.
 *   - Block size is 3; indices are int32; values FP64, block-row-major.
 *   - Vectors `b`, `x`, `v`, `z`, `y` are in the caller's (original) row
 *     order; the internal reordering is applied and undone inside the calls.
 */
#ifndef RSOLVE_H
#define RSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_bcsr *bcsr_t;
typedef struct rs_ilu0 *ilu0_t;

enum rs_status {
    RS_OK = 0,
    RS_NOT_CONVERGED = 1,   /* iteration limit reached; x holds the last iterate */
    RS_BREAKDOWN = 2,       /* rho, (rhat,v), (t,t) or omega became zero */
    RS_PENDING = 3,         /* server_poll: the request has not finished yet */
    RS_INVALID_ARG = -1,
    RS_UNSUPPORTED_BLOCK_SIZE = -2,
    RS_BAD_PATTERN = -3,    /* row pointers not monotone, columns unsorted, duplicate or out of range */
    RS_MISSING_DIAGONAL = -4,
    RS_ZERO_PIVOT = -5,     /* a diagonal block of U is singular or not finite */
    RS_NON_FINITE = -6,     /* NaN or Inf reached a reduction */
    RS_OUT_OF_MEMORY = -7,  /* device allocation failed or a budget was exceeded */
    RS_HIP_ERROR = -8,
    RS_PATTERN_MISMATCH = -9, /* an ilu0_t used with a matrix of another pattern */
    RS_NOT_FACTORED = -10   /* solve or apply before a successful ilu0_factor */
};

/* Row orderings of Section "ILU0": the caller's order (sequential ILU), level
 * scheduling (a row's level is one more than its lower neighbours' deepest),
 * or graph colouring by DSatur (Brelaz 1979: the uncoloured row whose
 * neighbours hold the most distinct colours next, ties to more neighbours,
 * then to the lower index; each takes the lowest free colour).  Rows are
 * sorted stably by level or colour.
 * RS_ORDER_RCM_LEVEL_SET: level scheduling after a reverse Cuthill-McKee
 * renumbering (Cuthill and McKee 1969), the level-reducing reordering that
 * the paper's comparison of level sets and graph colouring calls for on
 * patterns whose non-neighbour connections chain distant rows.  On the
 * symmetrised graph (i ~ j when either block is stored): each breadth-first
 * search starts at the unnumbered row with the fewest neighbours (lowest
 * index on a tie); a row taken from the queue appends its unnumbered
 * neighbours by increasing neighbour count (lower index on a tie); the
 * sequence is reversed (position n-1-k for the k-th row numbered).  A
 * row's level is one more than the deepest level of its neighbours at
 * lower positions (0 if none); rows are sorted by (level, position). */
enum rs_ordering { RS_ORDER_NATURAL = 0, RS_ORDER_LEVEL_SET = 1, RS_ORDER_GRAPH_COLOUR = 2,
                   RS_ORDER_RCM_LEVEL_SET = 3 };
enum rs_precision { RS_PREC_FP64 = 0, RS_PREC_FP32_FACTORS = 1 };
enum rs_mem { RS_MEM_HOST = 0, RS_MEM_DEVICE = 1 };

/* Execution options of an ilu0_t (ilu0_set_option).  They change how the
 * work is launched.  The factor's and the sweeps' arithmetic never changes;
 * SpMV shapes and reduction modes change only the summation order of the
 * dot products fused into the SpMVs (the last bits of alpha and omega). */
enum rs_option {
    RS_OPT_SWEEP_TILES = 0,  /* 1: one launch per triangular sweep, row tiles wait only on the
                                tiles they depend on; 0: one launch per level.  Default: 0 for
                                graph colouring (few wide levels), 1 otherwise */
    RS_OPT_SWEEP_GRID = 1,   /* workgroups of a single-launch sweep (default 1024) */
    RS_OPT_POLL_CHUNK = 2,   /* BiCGStab iterations queued between host polls of convergence (default 1) */
    RS_OPT_USE_GRAPH = 3,    /* 1 (default): an iteration is captured once as a HIP graph and replayed.
                                A capture is invalidated by device-synchronising calls (hipFree,
                                synchronous copies) made meanwhile by other threads: set 0 when
                                solving from several threads */
    RS_OPT_PREDICT_POLL = 4, /* 1 (default): the first poll comes after as many iterations as the
                                last converged solve on this handle needed, at most 50
                                (iterations queued past convergence return at once); solves that
                                end without converging leave the prediction unchanged */
    RS_OPT_SPMV_VARIANT = 5, /* launch shape of the SpMVs: 0..8 = {4, 2, 1} waves per workgroup
                                with blocks staged in LDS, then the same three reading directly,
                                then the same three staged in LDS with non-temporal loads */
    RS_OPT_SWEEP_VARIANT = 6, /* launch shape of the one-launch-per-level sweeps (same encoding) */
    RS_OPT_REDUCE_SPLIT = 7, /* dot products fused into the SpMVs: 0 (default) = each workgroup
                                joins a ticket tree inside the SpMV; 1 = each wave only stores
                                its partial and a one-workgroup kernel adds them; 2 = each wave
                                stores its partial and every workgroup of the next vector kernel
                                adds them (few partials: small systems) */
    RS_OPT_SPIN_LIMIT = 8,   /* polls before a single-launch sweep's dependency wait gives up
                                (default 4194304, >= 0).  A wait that gives up lets its tile go
                                on, so the launch still ends; the solve then returns RS_HIP_ERROR
                                and the handle's sweep counters and tile flags are reset, so the
                                next call starts clean.  A small value forces that error path
                                (for tests of the recovery) */
    RS_OPT_FUSE_SPMV = 9,    /* 1 (default): where the rows without lower blocks are the first rows
                                of the analysed order (at least a quarter of them) and share one
                                upper level (graph colouring of a grid: the first colour),
                                BiCGStab's upper launch of those rows reads each of their rows
                                of A' once for the sweep and for their rows of the SpMV that
                                follows (their U rows equal their rows of A'); the SpMV then
                                covers the other rows.  Same z; v and t of those rows add the
                                diagonal's term last, and the dot products' summation order
                                changes: the solve agrees with the unfused one to rounding.
                                With separate wells (bcsr_set_wells), the well terms of those
                                rows, which need the whole product's x, are subtracted after
                                the SpMV by a small launch that also corrects the dot products.
                                Used with per-level sweeps and reduction split 0; 0: never */
    RS_OPT_FUSED_ROWS = 10,  /* read only (ilu0_get_option): how many rows the analysed pattern
                                lets RS_OPT_FUSE_SPMV fuse (0: none) */
    RS_OPT_Y_INPUT = 11,     /* 1 (default): where the analysed pattern allows it (RS_OPT_Y_INPUT_PATTERN),
                                a preconditioner application stores no intermediate y = L^-1 v.
                                The rows without lower blocks have y = v, so the launches read
                                their v directly and their lower launch is left out (BiCGStab's
                                first application keeps one vector launch that updates p on
                                those rows); every other row finishes in the lower launch.  Used
                                with per-level sweeps when the upper launch of those rows reads
                                A' (FP64 factors, or the RS_OPT_FUSE_SPMV iteration).  The same
                                bits either way; 0: always store y */
    RS_OPT_Y_INPUT_PATTERN = 12, /* read only: 1 when the analysed pattern has two lower levels,
                                the first being the RS_OPT_FUSED_ROWS rows, and none of the other
                                rows holds an upper block (graph colouring of a bipartite
                                pattern such as a 7-point grid) */
    RS_OPT_FACTOR_ASYNC = 13, /* 0 (default): ilu0_factor waits for the factorisation and returns its
                                status.  1: ilu0_factor only queues it on its stream and returns
                                RS_OK (bad_row untouched); a singular pivot then shows as
                                RS_ZERO_PIVOT in the statuses of the next solve, and
                                ilu0_factor_status waits for it and gives what the waiting call
                                would have returned.  A solve or application on another stream
                                must wait for the factorisation's stream first. */
    RS_OPT_LOWER_PARTS = 14  /* 1 (default): with FP64 factors, in BiCGStab's fused iteration on a
                                pattern of RS_OPT_Y_INPUT_PATTERN, the SpMV v = A phat also forms,
                                from the same FP64 blocks, the sums sum_k A'_ik inv(U_kk) r_k and
                                sum_k A'_ik inv(U_kk) v_k of each row with lower blocks (its lower
                                blocks are L_ik = A'_ik inv(U_kk) on such a pattern); the
                                iteration's second application then forms sum_k L_ik s_k as their
                                combination for s = r - alpha v instead of reading L again (not
                                with separate wells).  The
                                same mathematics (Algorithm 2, equations 3-4), other rounding: the
                                solves agree with the option off to rounding; 0: off */
};

/* Per-system outcome of bicgstab_solve and gmres_solve. */
typedef struct {
    int32_t status;            /* rs_status of this system */
    int32_t half_steps;        /* BiCGStab: 2i-1 when stopping at the half step of iteration i, 2i at
                                  its end; GMRES: Arnoldi steps */
    double r0_norm;            /* ||b||_2 (x0 = 0) */
    double final_norm;         /* recursively updated residual norm at the stop */
    double true_rel_residual;  /* ||b - A x||_2 / ||b||_2 with the caller's A, FP64 */
    double factor_ms;          /* device time of the ILU0 factorisation the solve used (HIP events
                                  around its launches on the stream of that ilu0_factor call;
                                  whole batch) */
    double solve_ms;           /* device time of this solve call on its stream, from the first
                                  kernel (permutation of b, initial residual) to the end of the
                                  true residual (HIP events; whole batch; host gaps between
                                  polls included) */
} solve_info;

/* bcsr_create -- validate a BCSR pattern and copy pattern and values to the
 * device.  Section "OPM Flow" (three arrays, contiguous nonzeros that must be
 * checked) and the zero-diagonal check of Section "Profiling".
 *   n_brows, nnzb : block rows and stored blocks (n_brows >= 0)
 *   block_size    : must be 3, else RS_UNSUPPORTED_BLOCK_SIZE
 *   batch         : number of same-pattern systems (>= 1)
 *   row_ptr[n+1], col_idx[nnzb] (mem): columns ascending and unique per row,
 *                   every row has its diagonal block
 *   vals (mem)    : batch * nnzb * 9 doubles, system-major, may be NULL
 *                   (values set later with bcsr_set_values)
 *   out           : receives the handle; bad_row (host, may be NULL)
 *                   receives the offending row on a pattern error.
 * The pattern is copied on `stream`, which is synchronised before return
 * (values, when given, stay stream-ordered as in bcsr_set_values).
 * Errors: RS_INVALID_ARG, RS_UNSUPPORTED_BLOCK_SIZE, RS_BAD_PATTERN,
 * RS_MISSING_DIAGONAL, RS_OUT_OF_MEMORY, RS_HIP_ERROR. */
int bcsr_create(int32_t n_brows, int32_t nnzb, int32_t block_size, int32_t batch, const int32_t *row_ptr,
                const int32_t *col_idx, const double *vals, int32_t mem, void *stream, bcsr_t *out,
                int32_t *bad_row);

/* bcsr_set_values -- replace the values of systems [first_sys, first_sys +
 * n_sys) (vals: n_sys * nnzb * 9 doubles, mem).  The pattern is unchanged,
 * as between Newton steps.  Stream-ordered; no synchronisation. */
int bcsr_set_values(bcsr_t A, const double *vals, int32_t first_sys, int32_t n_sys, int32_t mem, void *stream);

/* bcsr_get_dims -- n_brows, nnzb, batch of a handle (host outputs, any may be NULL). */
int bcsr_get_dims(bcsr_t A, int32_t *n_brows, int32_t *nnzb, int32_t *batch);

/* bcsr_spmv -- y = A x for systems [first_sys, first_sys + n_sys), FP64,
 * caller order (x, y: n_sys * n_brows * 3 doubles, mem).  Section "Sparse
 * Matrix-Vector multiplication". */
int bcsr_spmv(bcsr_t A, const double *x, double *y, int32_t first_sys, int32_t n_sys, int32_t mem, void *stream);

/* bcsr_set_option -- RS_OPT_SPMV_VARIANT of bcsr_spmv (other options are
 * RS_INVALID_ARG). */
int bcsr_set_option(bcsr_t A, int32_t option, int32_t value);

/* bcsr_set_wells -- standard wells kept separate, Section "Well
 * Contributions" (Algorithm 5), with the block shapes Section "OPM Flow"
 * gives for black oil (B, C: 4x3 blocks; D: 4x4): from now on every product with A (the
 * solver's SpMVs, the true residual, bcsr_spmv) is y = A x - sum over wells
 * w of C_w^T D_w^-1 B_w x.  The ILU0 preconditioner stays that of A.
 *   n_wells          : wells (0 removes them)
 *   well_ptr[n_wells+1], perf_row[n_perf] (host): the perforations of well w
 *                      are [well_ptr[w], well_ptr[w+1]); perf_row gives each
 *                      perforation's block row (n_perf = well_ptr[n_wells])
 *   B, C (mem)       : batch * n_perf 4x3 blocks, row-major (one block row
 *                      per well, a block per perforated cell)
 *   Dinv (mem)       : batch * n_wells 4x4 blocks, the inverse of each well's
 *                      diagonal block (the paper stores the inverse)
 * Copies everything; synchronises `stream`.  Errors: RS_INVALID_ARG
 * (well_ptr not starting at 0 or decreasing, a row out of range),
 * RS_OUT_OF_MEMORY, RS_HIP_ERROR. */
int bcsr_set_wells(bcsr_t A, int32_t n_wells, const int32_t *well_ptr, const int32_t *perf_row, const double *B,
                   const double *C, const double *Dinv, int32_t mem, void *stream);

/* bcsr_destroy -- free the handle (NULL is accepted). */
int bcsr_destroy(bcsr_t A);

/* ilu0_analyse -- host analysis of A's pattern (integer work, once per
 * pattern): the ordering (RS_ORDER_*), the reordered pattern, lower and
 * upper sweep schedules and the factor update lists; all copied to the
 * device (complete on return, usable from any stream).  Section "ILU0" of
 * the implementation chapter.  Errors: RS_INVALID_ARG (ordering not an
 * rs_ordering), RS_OUT_OF_MEMORY, RS_HIP_ERROR. */
int ilu0_analyse(bcsr_t A, int32_t ordering, ilu0_t *out);

/* ilu0_analyse_jacobi -- as ilu0_analyse for the Block-Jacobi-ILU0
 * preconditioner of Section "Block-Jacobi-ILU0": part (host, n_brows ints)
 * assigns every row a partition id; the ordering, sweep schedules and ILU0
 * use only the blocks joining rows of one partition (the Jacobi matrix),
 * while the SpMV and the true residual keep all of A.  The Jacobi matrix's
 * blocks are gathered from A at every ilu0_factor (the paper's copy
 * indexes), so values change freely between factorisations.
 * Errors: RS_INVALID_ARG (part NULL), RS_OUT_OF_MEMORY, RS_HIP_ERROR. */
int ilu0_analyse_jacobi(bcsr_t A, int32_t ordering, const int32_t *part, ilu0_t *out);

/* bcsr_partition -- host-only partitioner for ilu0_analyse_jacobi: n_parts
 * partitions of near-equal size (sizes differ by at most one), each grown
 * from the first unassigned row in natural order by repeatedly taking the
 * unassigned row most strongly coupled to it.  Coupling = sum of |weights|
 * (host, one per stored block, e.g. transmissibilities; NULL: all 1) of the
 * blocks joining the row to the partition, so strongly coupled cells stay
 * together (the paper partitions by transmissibility).  part: host output,
 * n_brows ints in [0, n_parts).  Errors: RS_INVALID_ARG, RS_BAD_PATTERN,
 * RS_MISSING_DIAGONAL. */
int bcsr_partition(int32_t n_brows, int32_t nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                   const double *weights, int32_t n_parts, int32_t *part);

/* ilu0_analyse_shared -- a further preconditioner handle for A, whose
 * pattern must equal the one `like` was analysed for (RS_PATTERN_MISMATCH
 * otherwise): it shares like's analysis (ordering, schedules, their device
 * copy; reference-counted, so `like` may be destroyed first) and has its own
 * factors, workspace and default options.  No host analysis runs.  Reads
 * only immutable parts of `like`, so `like` may be in use on another thread. */
int ilu0_analyse_shared(bcsr_t A, ilu0_t like, ilu0_t *out);

/* ilu0_get_schedule -- the reordering of Section "ILU0" of the
 * implementation chapter, as analysed: perm[new] = old (host, n_brows ints,
 * may be NULL), the permutation P of b' = P b and A' = P A P^T;
 * *n_sets = number of levels (LS, RCM then LS), colours (GC) or one per row
 * (natural order); set_ptr (host, n_sets + 1 ints, may be NULL) = the start
 * of each level/colour in the new order (natural: i).  Rows of one set have
 * no dependency on each other, so one launch per set may process them
 * together.  Host only; errors: RS_INVALID_ARG. */
int ilu0_get_schedule(ilu0_t M, int32_t *perm, int32_t *n_sets, int32_t *set_ptr);

/* ilu0_get_sweep_levels -- number of levels of the lower and upper sweep
 * schedules the device executes (host outputs, may be NULL). */
int ilu0_get_sweep_levels(ilu0_t M, int32_t *n_lower, int32_t *n_upper);

/* ilu0_set_option / ilu0_get_option -- read or change an rs_option of the
 * handle.  RS_INVALID_ARG for an unknown option or a value out of range. */
int ilu0_set_option(ilu0_t M, int32_t option, int32_t value);
int ilu0_get_option(ilu0_t M, int32_t option, int32_t *value);

/* Outcome of ilu0_autotune. */
typedef struct {
    int32_t spmv_variant, sweep_variant, sweep_tiles, sweep_grid; /* chosen rs_option values */
    double us_per_solve;   /* mean time of one bicgstab_solve call with them (0 when cached) */
    int32_t candidates;    /* configurations timed (0 when taken from the cache) */
    int32_t from_cache;    /* 1 when read from the cache file */
    int32_t reduce_split;  /* chosen RS_OPT_REDUCE_SPLIT */
} rs_tune_result;

/* ilu0_autotune -- pick the launch configuration of a factored handle by
 * timing it: every one-launch-per-level sweep shape, the single-launch sweep
 * with several grid sizes, then every SpMV shape with the best sweep, then
 * the split reduction with the best of those, each
 * over `reps` (>= 1) bicgstab_solve calls on right-hand sides b (batch *
 * n_brows * 3 doubles, mem) at `reduction`.  The fastest is applied with
 * ilu0_set_option.  When the environment variable RSOLVE_TUNE_CACHE names a
 * file, results are looked up there first and appended after a search,
 * keyed by the problem shape (n, nnzb, batch, ordering, precision, sweep
 * levels) and the device.  Configurations change launch shapes only; a
 * different SpMV shape reorders the partial sums of the fused dot products
 * (results agree to rounding; each configuration is deterministic).
 * Synchronises `stream`. */
int ilu0_autotune(ilu0_t M, bcsr_t A, const double *b, int32_t mem, double reduction, int32_t reps, void *stream,
                  rs_tune_result *out);

/* ilu0_factor -- block ILU0 (Algorithm 2) of every system of A in the
 * analysed order, levels ascending.  precision RS_PREC_FP64 keeps FP64
 * factors; RS_PREC_FP32_FACTORS computes them in FP64 and stores them
 * rounded to FP32 for the sweeps.  bad_row (host, batch ints, may be NULL)
 * receives, per system, the original index of the first singular pivot
 * block or -1.  Returns RS_ZERO_PIVOT if any system failed.  Synchronises
 * `stream` (unless RS_OPT_FACTOR_ASYNC is set: then stream-ordered). */
int ilu0_factor(ilu0_t M, bcsr_t A, int32_t precision, void *stream, int32_t *bad_row);

/* ilu0_factor_status -- the status and bad_row (as ilu0_factor) of the
 * handle's last factorisation; waits for it when it was queued with
 * RS_OPT_FACTOR_ASYNC (the pivot test of Algorithm 2's inverse, as
 * ilu0_factor).  RS_NOT_FACTORED before any factorisation. */
int ilu0_factor_status(ilu0_t M, int32_t *bad_row);

/* ilu0_get_factors -- copy system `sys`'s factors to host, in the reordered
 * pattern (rows in new order, columns renumbered and ascending, as P A P^T):
 * lu (nnzb * 9 doubles) holds L below the diagonal and U above it, zero
 * elsewhere (the diagonal, and blocks outside a Jacobi matrix); dinv
 * (n_brows * 9) holds inv(U_ii) in new row order.  FP32 factors are returned
 * widened.  Synchronous (waits for the whole device). */
int ilu0_get_factors(ilu0_t M, int32_t sys, double *lu, double *dinv);

/* ilu0_apply -- z = U^{-1} L^{-1} v for systems [first_sys, first_sys +
 * n_sys) in caller order (equations 3-4).  Stream-ordered. */
int ilu0_apply(ilu0_t M, const double *v, double *z, int32_t first_sys, int32_t n_sys, int32_t mem,
               void *stream);

/* ilu0_apply_noalloc -- ilu0_apply for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same results bit for bit,
 * with v and z device pointers (caller order, n_sys * n_brows * 3 doubles,
 * caller-owned) and every intermediate (the new-order input and output, the
 * lower sweep's y, the single-launch sweeps' tile flags and counters) in a
 * fixed workspace of RS_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  Calls no hipMalloc, hipFree
 * or allocating library routine.  n_sys systems of n_brows block rows need
 * about 72 * n_brows * n_sys bytes (3 vectors) plus 8 bytes per sweep tile:
 * up to about 1.1M block rows for one system; larger calls return
 * RS_OUT_OF_MEMORY with the sizes in rsolve_last_error().  Every call on a
 * GPU shares that GPU's workspace, whatever the handle: calls that overlap
 * on one GPU (two streams, two host threads) race and must be ordered by
 * the caller.  Stream-ordered; with single-launch sweeps on
 * (RS_OPT_SWEEP_TILES) it also synchronises `stream` to read the sweeps'
 * error word (RS_HIP_ERROR when a dependency wait gave up), so only the
 * per-level sweeps may be captured in a graph.  Errors as ilu0_apply. */
#define RS_NOALLOC_SCRATCH_BYTES (80u << 20)
int ilu0_apply_noalloc(ilu0_t M, const double *v, double *z, int32_t first_sys, int32_t n_sys, void *stream);

/* bicgstab_solve -- BiCGStab (Section "Bicgstab solver": the Krylov solver
 * of the simulator, relative residual reduction 1e-2 and 200 iterations by
 * default) right-preconditioned by the factors of the last ilu0_factor
 * (equations 3-4), for every system of A (b, x: batch * n_brows * 3
 * doubles, mem, caller's row order) with x0 = 0.  Each iteration tests the
 * recursively updated residual's 2-norm after its half step (on s) and its
 * full step (on r) against reduction * ||b||; max_iter full iterations at
 * most.  A failed solve is not fatal (Section "Fallback"): x holds the last
 * iterate and the status says why, so the caller may switch solvers.
 * info (host, batch entries, may be NULL) receives each system's outcome,
 * including the true FP64 residual ||b - A x|| / ||b|| and the device times
 * of the factorisation and the solve.  Returns the worst status over the
 * systems (errors first, then RS_BREAKDOWN, RS_NOT_CONVERGED, RS_OK).
 * Statuses: RS_BREAKDOWN when rho, (rhat,v), (t,t) or omega is exactly zero
 * (after omega = 0, x keeps its half-step update); RS_NON_FINITE when a
 * reduction is NaN or Inf; RS_ZERO_PIVOT for a system whose factorisation
 * failed; errors RS_INVALID_ARG (reduction < 0, max_iter < 0, NULL
 * vectors), RS_NOT_FACTORED, RS_PATTERN_MISMATCH, RS_OUT_OF_MEMORY,
 * RS_HIP_ERROR.  Synchronises `stream`. */
int bicgstab_solve(ilu0_t M, bcsr_t A, const double *b, double *x, double reduction, int32_t max_iter,
                   int32_t mem, void *stream, solve_info *info);

/* gmres_solve -- right-preconditioned restarted GMRES(restart) for every
 * system of A, the simulator's alternative Krylov solver (Section "OPM
 * Flow"), on the same factors, sweeps and SpMV as bicgstab_solve.  x0 = 0;
 * each cycle builds an orthonormal basis of up to `restart` (1..32) Krylov
 * vectors of A M^-1 (classical Gram-Schmidt applied twice) and minimises the
 * residual over it with Givens rotations; the residual estimate is tested
 * after every Arnoldi step against reduction * ||b||, and a cycle that ends
 * without meeting it restarts from the explicit residual b - A x.  max_iter
 * counts Arnoldi steps (one preconditioner application and one product with
 * A each); info[i].half_steps receives the steps taken and final_norm the
 * last residual estimate (or explicit residual norm after a restart).
 * A breakdown of the basis (h_{j+1,j} = 0) zeroes the estimate, so it
 * ends the solve as converged.
 * Standard wells set on A (bcsr_set_wells) enter every product with A, as
 * in bicgstab_solve.  b, x: batch * n_brows * 3 doubles (mem).  Workspace:
 * restart basis vectors per system, allocated on first use and kept by the
 * handle.  Errors: RS_INVALID_ARG, RS_NOT_FACTORED, RS_PATTERN_MISMATCH,
 * RS_OUT_OF_MEMORY, RS_HIP_ERROR.
 * Returns the worst status over the systems, as bicgstab_solve (never
 * RS_BREAKDOWN).  Synchronises `stream`. */
int gmres_solve(ilu0_t M, bcsr_t A, const double *b, double *x, int32_t restart, double reduction,
                int32_t max_iter, int32_t mem, void *stream, solve_info *info);

/* ilu0_destroy -- free the handle (NULL is accepted). */
int ilu0_destroy(ilu0_t M);

/* ilu0_analyse_host -- the host analysis alone, without a device: validates
 * the pattern and writes perm[new] = old (n ints) and the number of
 * levels/colours.  Same orderings as ilu0_analyse. */
int ilu0_analyse_host(int32_t n_brows, const int32_t *row_ptr, const int32_t *col_idx, int32_t ordering,
                      int32_t *perm, int32_t *n_sets, int32_t *bad_row);

/* rsolve_profile_enable -- time classes of kernel work with HIP events
 * recorded on the launch stream (bit c of mask enables class c:
 * 0 = one ILU0 factorisation, 1 = one lower sweep (all its level
 * launches), 2 = one upper sweep, 3 = one v = A phat launch, 4 = one
 * vector-update launch, 5 = one t = A shat launch (and GMRES's products
 * with A), 6 = one GMRES Gram-Schmidt launch, 7 = one preconditioner
 * application (both sweeps)).  Single-kernel units record dispatch events
 * (the kernel's own start and end); with graphs on, a timed sweep or
 * application replays as a graph segment of its own between two events.
 * Algorithmic bytes per unit (nL, nU: blocks of L and U; N rows; tb = 8
 * for FP64 factors, 4 for FP32): factorisation 148 nnzb; lower sweep
 * (9 tb + 4) nL + 52 N; upper sweep (9 tb + 4)(nU + N) + 48 N (inv(U_ii)
 * with U); application the sum of both; v = A phat and t = A shat 76 nnzb
 * + 52 N; vector updates the vectors they read and write.  The fused work
 * a kernel also does (the p update in the first lower sweep, the dot
 * product in the SpMV) is not counted.
 * Resets the counters.  Process-wide, not thread-safe; 0 disables. */
int rsolve_profile_enable(int32_t mask);

/* rsolve_profile_set_mask -- change the timed classes without clearing the
 * counters (e.g. to time a sample of the solves).  Process-wide. */
int rsolve_profile_set_mask(int32_t mask);

/* rsolve_profile_get -- accumulated device milliseconds, units timed and
 * algorithmic bytes moved (the bytes the method must read and write, not
 * cache traffic) of class `cls` since the last enable (host outputs, may be
 * NULL).  Waits for pending events. */
int rsolve_profile_get(int32_t cls, double *ms, int64_t *units, double *bytes);

/* ------------------------------------------------------------- serving
 * A request server for streams of solves of mixed sizes (one system each).
 * Requests name a registered pattern; they wait in arrival order and are
 * admitted as soon as a worker slot is free and a resident instance of the
 * pattern is idle, or the device footprint of a new instance fits in the
 * memory budget.  Each slot runs on its own HIP stream, so admitted requests
 * overlap on the device.  An instance (matrix + preconditioner handles,
 * factors, Krylov workspace) stays resident after its request, so a later
 * request of the same pattern only uploads values, factors and solves; all
 * instances of a pattern share one analysis (ilu0_analyse_shared).  When the
 * head of the queue does not fit, idle instances are freed, least recently
 * used first.  Each request is factored (`precision`) and solved exactly as
 * ilu0_factor / bicgstab_solve would, so results do not depend on the mix;
 * with `autotune`, the first request of a pattern runs ilu0_autotune on its
 * instance, and every other request of that pattern waits (in its slot)
 * until the tuning has ended and then runs with the tuned configuration, so
 * all results of a pattern come from one launch configuration. */
typedef struct rs_server *server_t;

typedef struct {
    size_t hbm_budget_bytes;  /* device bytes all resident instances may hold together */
    int32_t max_slots;        /* requests processed at once (1..64) */
    int32_t ordering;         /* RS_ORDER_* for every pattern */
    int32_t precision;        /* RS_PREC_* for every request */
    int32_t autotune;         /* 1: ilu0_autotune once per pattern */
} server_config;

typedef struct {
    double queue_ms;    /* submission to admission */
    double analyse_ms;  /* instance creation: handles, analysis or its reuse, allocation (0 when resident) */
    double factor_ms;   /* value upload and queueing the ILU0 factorisation (waiting for it on the
                           first request of a pattern with autotune; its device time is in the
                           request's solve_info.factor_ms) */
    double tune_ms;     /* autotuning (first instance of a pattern) */
    double solve_ms;    /* BiCGStab, true residual, result copy */
    double total_ms;    /* submission to completion */
    int32_t slot;
    int32_t resident;   /* 1: ran on an instance that was already resident */
} server_timing;

typedef struct {
    int64_t queued, running, completed;
    int64_t instances;      /* resident instances now */
    int64_t created, evicted, analyses;
    size_t reserved_bytes, peak_reserved_bytes;   /* the budget's account of footprints */
    size_t device_used_bytes;   /* hipMemGetInfo total - free now (the whole process and device) */
    size_t device_total_bytes;  /* hipMemGetInfo total */
} server_stats;

/* server_create -- start max_slots worker threads on the current device.
 * Errors: RS_INVALID_ARG, RS_HIP_ERROR. */
int server_create(const server_config *cfg, server_t *out);

/* server_request_bytes -- the device footprint an instance of this shape
 * reserves against the budget (the shared analysis is counted once per
 * pattern, in addition, as server_analysis_bytes). */
int server_request_bytes(int32_t n_brows, int32_t nnzb, int32_t precision, size_t *bytes);
int server_analysis_bytes(int32_t n_brows, int32_t nnzb, size_t *bytes);

/* server_add_pattern -- register a pattern (host row_ptr / col_idx, copied
 * and validated as bcsr_create does) and return its id; an identical
 * pattern registered again gets the same id.  Errors: RS_INVALID_ARG,
 * RS_BAD_PATTERN, RS_MISSING_DIAGONAL (bad_row set when not NULL),
 * RS_OUT_OF_MEMORY when one instance of it exceeds the budget. */
int server_add_pattern(server_t S, int32_t n_brows, int32_t nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                       int32_t *pattern, int32_t *bad_row);

/* server_submit -- queue one solve (batch 1) of a registered pattern:
 * vals (nnzb*9), b (n*3) and x (n*3, the result) in `mem`, borrowed until
 * server_poll/server_wait reports completion.  Returns a ticket. */
int server_submit(server_t S, int32_t pattern, const double *vals, const double *b, double *x, double reduction,
                  int32_t max_iter, int32_t mem, int64_t *ticket);

/* server_poll -- RS_PENDING while the request runs or waits; otherwise its
 * status (as bicgstab_solve would return), with info and timing (may be
 * NULL); the ticket is then released. */
int server_poll(server_t S, int64_t ticket, solve_info *info, server_timing *timing);

/* server_wait -- as server_poll, blocking until the request completes. */
int server_wait(server_t S, int64_t ticket, solve_info *info, server_timing *timing);

int server_get_stats(server_t S, server_stats *out);

/* server_destroy -- finish queued and running requests, stop the slots,
 * free every instance and pattern (NULL accepted). */
int server_destroy(server_t S);

const char *rsolve_status_string(int status);
const char *rsolve_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
