/*
 * rp.h -- C ABI of librp, reachability probabilities of discrete-time Markov
 * chains on AMD Instinct MI355X (gfx950).
 *
 * Method (Cormie-Bowins, "A Comparison of Sequential and GPU Implementations
 * of Iterative Methods to Compute Reachability Probabilities", GRAPHITE 2012):
 *   * Section 2.2: partition the states into S_{=0} (cannot reach the goal
 *     set GS), S_{=1} (reach GS with probability one) and S_? by searches on
 *     the underlying digraph (edge s -> s' iff P(s,s') > 0).
 *   * Section 2.3: on S_? the probabilities x solve (I - A) x = b with
 *     A = P restricted to S_? x S_? and b_s = P(s, S_{=1}).
 *   * Section 3.1 / 3.2: solve that system with the Jacobi method or with
 *     un-preconditioned BiCGStab.
 *
 * Conventions for every entry point
 *   * All array arguments marked "device" are caller-owned device buffers on
 *     the context's device.  They are read (or written) only during the call;
 *     every call returns after its work on the context's stream is complete.
 *   * Arrays marked "host" are ordinary host memory.
 *   * Return value: RP_OK (0) or one of the RP_ERR_* codes below.  No C++
 *     exception crosses this boundary.  rp_last_error() gives a message for
 *     the last failing call on a context.
 *   * Several independent chains ("instances") can be packed block-diagonally
 *     in one rp_chain; they are partitioned and solved together, each with its
 *     own convergence test, and per-instance results are reported.
 */
#ifndef RP_H
#define RP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
#define RP_OK 0
#define RP_ERR_INVALID_ARG 1   /* null pointer, bad size or bad option        */
#define RP_ERR_BAD_CHAIN 2     /* input is not a valid Markov chain (see msg) */
#define RP_ERR_NOT_CONVERGED 3 /* iteration cap hit; or the FP64 residual
                                  stopped falling (three refinement steps
                                  without halving it: tol is below what
                                  FP64 can certify); or, under
                                  RP_STOP_DELTA, the stopping measure did not
                                  halve its best value for max(65,536, the
                                  iterations it took to reach it) iterations
                                  (tol below the rounding floor); x and info
                                  still valid                                */
#define RP_ERR_BREAKDOWN 4     /* BiCGStab breakdown (q.r, q.v or omega = 0)  */
#define RP_ERR_NONFINITE 5     /* NaN or Inf appeared during the iteration    */
#define RP_ERR_OOM 6           /* device allocation failed                    */
#define RP_ERR_HIP 7           /* HIP runtime error                           */
#define RP_ERR_TOO_LARGE 8     /* sizes beyond 32-bit row / column indices    */

/* ---- state classes written by rp_precompute (Section 2.2) ----------------- */
#define RP_S0 0 /* probability 0 */
#define RP_S1 1 /* probability 1 */
#define RP_SQ 2 /* undecided: solved by the iterative methods */

/* ---- rp_precompute flags ---------------------------------------------------- */
/* Take S_{=1} = GS (skip the second search).  S_? = S \ (S_{=0} u GS) and
 * b = P(s, GS), the literal form of Section 2.3; gives the same x.            */
#define RP_PROB0_ONLY 1u

/* ---- stopping rules ------------------------------------------------------- */
/* Paper's rule: Jacobi stops after the first sweep with max|x' - x| < tol;
 * BiCGStab stops once every |s_i| <= tol (the test inside the CUDA kernel of
 * Section 5.2).  Requires precision RP_FP64.                                  */
#define RP_STOP_DELTA 0
/* Certified: stop when ||T||_inf * ||b - (I-A)x||_inf <= tol, where
 * T = (I-A)^{-1} 1 is bounded once per system (I - A is a nonsingular
 * M-matrix on S_?, so this bounds max|x - x*|).  The residual is recomputed
 * in FP64 from the FP64 matrix.                                               */
#define RP_STOP_CERTIFIED 1
/* Stop when the FP64 residual ||b - (I-A)x||_inf <= tol.                     */
#define RP_STOP_RESIDUAL 2

/* ---- arithmetic ------------------------------------------------------------- */
#define RP_FP64 0         /* FP64 values and vectors throughout                 */
#define RP_FP32_REFINED 1 /* FP32 values/vectors in the inner sweeps, inside an
                             FP64 iterative-refinement loop (FP64 residual,
                             FP64 solution, FP64 dot-product scalars)          */

/* ---- kernel layout (rp_opts.tiling) ----------------------------------------- */
#define RP_TILING_AUTO 0
#define RP_TILING_OFF 1

/* ---- data types ---------------------------------------------------------- */
typedef struct rp_chain {
    int32_t num_instances;            /* K >= 1                                  */
    const int64_t *inst_state_offset; /* host, K+1: [0] = 0, [K] = n, strictly
                                         increasing; instance k owns states
                                         [off[k], off[k+1])                     */
    int64_t n;                        /* total number of states, 1 <= n < 2^31  */
    int64_t nnz;                      /* stored transitions, 0 <= nnz < 2^31    */
    const int32_t *row_ptr;           /* device, n+1, row_ptr[0] = 0,
                                         row_ptr[n] = nnz (compressed row
                                         storage, Section 4)                     */
    const int32_t *col;               /* device, nnz: target state; strictly
                                         ascending within a row and inside the
                                         row's own instance                      */
    const double *val;                /* device, nnz: P(s, s') in [0, 1]; every
                                         row sums to 1 (within rowsum_tol)        */
} rp_chain;

typedef struct rp_opts {
    double tol;          /* stopping tolerance (meaning set by `stop`)          */
    int32_t stop;        /* RP_STOP_*                                            */
    int32_t precision;   /* RP_FP64 or RP_FP32_REFINED                           */
    int64_t max_iter;    /* cap on inner iterations (sweeps / BiCGStab steps)
                            summed over refinements, per instance               */
    double inner_tol;    /* inside refinement, each inner solve reduces the
                            residual by min(inner_tol, what the final tolerance
                            still needs), but not below the rounding floor of
                            the inner precision (default 1e-2: the inner sweeps
                            slow down near that floor, so looser steps need
                            fewer sweeps in total)                              */
    int32_t max_refine;  /* cap on refinement corrections (default 60)          */
    int32_t chunk;       /* most iterations launched between two host checks
                            (default 32; the first checks of an inner solve
                            come after 4, 8, 16, ... iterations; tiled
                            BiCGStab checks at least every 8 steps)            */
    int32_t schedule;    /* row layout of the tiled sparse products:
                            1,2,...,64: that many lanes sum each row;
                            0: sliced rows -- each tile's rows sorted by length
                            in slices of 64, one lane per row;
                            RP_SCHEDULE_SEGSCAN (-2): see below;
                            -1 (default): tuned -- sliced rows and the lane
                            counts from the mean row length and its two
                            neighbours are timed on a few sweeps the first
                            time a system of that shape is solved on the
                            context, and the choice is kept.  The iterates
                            differ only in the rounding order inside a row
                            (none for 0 and 1: one lane sums a row in order) */
    int32_t tiling;      /* RP_TILING_AUTO (default): row tiles that keep a
                            window of the iterate in on-chip memory;
                            RP_TILING_OFF: row chunks reading every operand
                            from device memory (same results up to rounding
                            order)                                             */
    const double *x0;    /* device, n (full state vector) or NULL: starting
                            point on S_? (default zero)                         */
    int32_t update;      /* Jacobi only (BiCGStab: RP_ERR_INVALID_ARG unless
                            RP_UPDATE_TWO_BUFFER):
                            RP_UPDATE_TWO_BUFFER (default): x_{m+1} from x_m
                            held apart, the Jacobi iteration of Section 3.1;
                            RP_UPDATE_IN_PLACE: each sweep overwrites the
                            iterate row by row and every row sum reads the
                            neighbour values present at that moment (the
                            single-vector update of the Section 5.1 kernel:
                            asynchronous, Gauss-Seidel-like within a block;
                            same fixed point, sweep counts depend on timing).
                            Either way the certified and residual stops test
                            the FP64 residual of the returned iterate.  Runs
                            on row chunks read from device memory.           */
    int32_t graph;       /* 1: tiled Jacobi sweeps (inner solves of refinement)
                            run as replays of one captured HIP graph per
                            batch of `chunk` sweeps (an even count): the
                            sweeps, the check of the last one and the status
                            publication, with sweep numbers kept on the
                            device; same iterates and counts as 0 (default,
                            one launch per sweep).  The graph is captured on
                            a private stream of the context and replayed on
                            the context's stream.                            */
} rp_opts;

/* opts.schedule value (Jacobi only): row sums by a backward segmented scan
 * over the stored entries, one thread per entry (the entry-parallel sparse
 * product the paper cites for Jacobi on GPUs, Section 8), on row chunks read
 * from device memory.  Same iteration; sums in scan (tree) order.           */
#define RP_SCHEDULE_SEGSCAN (-2)
#define RP_UPDATE_TWO_BUFFER 0
#define RP_UPDATE_IN_PLACE   1

typedef struct rp_solve_info {  /* one per instance */
    int64_t iterations;   /* inner iterations performed                        */
    int64_t refinements;  /* FP64 residual evaluations (refinement steps)      */
    double final_delta;   /* last stopping measure of the inner iteration      */
    double residual_inf;  /* ||b - (I-A)x||_inf in FP64 at the returned x      */
    double error_bound;   /* certified bound on max|x - x*|, or -1 if no bound
                             of ||(I-A)^{-1}1|| has been computed              */
    int32_t status;       /* RP_OK or RP_ERR_* for this instance               */
    int32_t lanes;        /* layout the tiled sparse products used: lanes per
                             row, or 0 for sliced rows                         */
    int32_t panels;       /* sliced rows only: column panels the instance's
                             iterate was staged in (its block is too large for
                             one LDS window and has no band), 0 otherwise     */
    int32_t reserved;     /* 0                                                 */
} rp_solve_info;

typedef struct rp_context rp_context;
typedef struct rp_system rp_system;

/* ---- lifecycle -------------------------------------------------------------- */
/* Create a context bound to `device` and the HIP stream `stream` (a
 * hipStream_t; NULL means the default stream).  The stream is borrowed.       */
int rp_context_create(rp_context **ctx_out, int device, void *stream);
/* Destroy every system of the context first: their device blocks go back to
 * a cache the context owns (reused by later systems, freed here).           */
int rp_context_destroy(rp_context *ctx);
/* Message for the last failing call on `ctx` ("" if none).  Owned by ctx.     */
const char *rp_last_error(const rp_context *ctx);
/* Fill `opts` with defaults: tol 1e-10, RP_STOP_CERTIFIED, RP_FP64,
 * max_iter 10^7, inner_tol 1e-2, max_refine 60, chunk 32, schedule -1.        */
void rp_opts_default(rp_opts *opts);

/* ---- graph precomputation (Sections 2.2, 2.3) --------------------------------
 * Validates the chain (row sums within rowsum_tol * max(1, row length); a
 * non-positive rowsum_tol means 1e-12), computes the classes by two backward
 * searches (the second one never passes through a goal state, which is
 * absorbing for "eventually GS"), and builds the reduced system over S_? in
 * FP64 plus an FP32 copy.
 *   goal_mask  device, n bytes: non-zero marks a goal state.
 *   flags      0 or RP_PROB0_ONLY.
 *   class_out  device, n bytes, or NULL: RP_S0 / RP_S1 / RP_SQ per state.
 *   sys_out    receives a library-owned system; free with rp_system_destroy.
 * The chain arrays are copied as needed; the caller may free them after the
 * call.  Errors: RP_ERR_INVALID_ARG, RP_ERR_BAD_CHAIN (message names the first
 * bad row and the reason), RP_ERR_TOO_LARGE, RP_ERR_OOM, RP_ERR_HIP.          */
int rp_precompute(rp_context *ctx, const rp_chain *chain,
                  const uint8_t *goal_mask, uint32_t flags, double rowsum_tol,
                  uint8_t *class_out, rp_system **sys_out);
int rp_system_destroy(rp_system *sys);

/* ---- general systems (the experiments of Section 6) --------------------------
 * A library-owned system for A x = b with A square (compressed row storage,
 * columns strictly ascending, the diagonal stored and nonzero), solved by
 * the same rp_jacobi / rp_bicgstab / rp_solve_rhs: Jacobi splits A into its
 * diagonal and the rest (Section 3.1), BiCGStab uses A itself (Section 3.2).
 * Independent systems can be packed block-diagonally (inst_row_offset as
 * rp_chain's inst_state_offset).  The solvers' x_out is x (n entries).  A
 * certified stop needs every row strictly diagonally dominant and then uses
 * Varah's bound ||A^{-1}||_inf <= 1 / min_i (|a_ii| - sum_{j!=i} |a_ij|) in
 * place of ||(I-A)^{-1} 1|| (otherwise RP_ERR_INVALID_ARG; RP_STOP_RESIDUAL
 * and RP_STOP_DELTA need no bound).  rp_adjoint does not apply.
 *   row_ptr, col, val  device (n+1, nnz, nnz); rhs device, n doubles.
 * Errors: RP_ERR_INVALID_ARG, RP_ERR_BAD_CHAIN (first bad row and reason),
 * RP_ERR_TOO_LARGE, RP_ERR_OOM, RP_ERR_HIP.                                    */
int rp_matrix_system(rp_context *ctx, int32_t num_instances,
                     const int64_t *inst_row_offset, int64_t n, int64_t nnz,
                     const int32_t *row_ptr, const int32_t *col,
                     const double *val, const double *rhs, rp_system **sys_out);

/* ---- state classes without allocation ------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * validation and the two backward searches of rp_precompute, writing only
 * the classes (RP_S0 / RP_S1 / RP_SQ, bit-identical to rp_precompute's
 * class_out) and building no system.  Calls no allocating routine: its
 * working memory is a fixed device array of the library, one per GPU, held
 * until the process ends and sized for RP_NOALLOC_MAX_STATES states.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (from
 * several threads or streams) race and must be serialised by the caller.
 *   chain, goal_mask, flags, rowsum_tol  as for rp_precompute.
 *   class_out  device, n bytes (required).
 * Errors: as rp_precompute; RP_ERR_TOO_LARGE when n > RP_NOALLOC_MAX_STATES. */
#define RP_NOALLOC_MAX_STATES 8388608
int rp_classify_noalloc(rp_context *ctx, const rp_chain *chain,
                        const uint8_t *goal_mask, uint32_t flags,
                        double rowsum_tol, uint8_t *class_out);

/* Sizes of a system: instances, total states, total |S_?| and total number of
 * off-diagonal entries of A over all instances.  Any pointer may be NULL.     */
int rp_system_sizes(const rp_system *sys, int64_t *num_instances,
                    int64_t *n_states, int64_t *n_undecided,
                    int64_t *nnz_offdiag);
/* Per-instance |S_?| (host, K entries).                                       */
int rp_system_instance_sizes(const rp_system *sys, int64_t *nq_out);
/* Copy of the reduced system in compact form (rows of S_? in ascending state
 * order, instance after instance), for inspection and tests.
 *   row_ptr  device, n_undecided+1 (int32)   col device, nnz_offdiag (int32,
 *   compact row index)  val device, nnz_offdiag   diag device, n_undecided
 *   (1 - P(s,s))   rhs device, n_undecided (b)   any may be NULL.            */
int rp_system_export(rp_context *ctx, const rp_system *sys, int32_t *row_ptr,
                     int32_t *col, double *val, double *diag, double *rhs);

/* ---- solvers (Sections 3.1, 3.2) ---------------------------------------------
 * Solve (I - A) x = b on S_? of every instance.
 *   x_out  device, n doubles: the full probability vector (0 on S_{=0}, 1 on
 *          S_{=1}, the solution on S_?).
 *   info   host, K entries (may be NULL).
 * Returns the worst per-instance status: RP_OK, RP_ERR_NOT_CONVERGED,
 * RP_ERR_BREAKDOWN or RP_ERR_NONFINITE (x_out and info are written in every
 * one of these cases), or an argument / runtime error (nothing written).      */
int rp_jacobi(rp_context *ctx, rp_system *sys, const rp_opts *opts,
              double *x_out, rp_solve_info *info);
int rp_bicgstab(rp_context *ctx, rp_system *sys, const rp_opts *opts,
                double *x_out, rp_solve_info *info);

/* ---- the reduced system with another right-hand side ----------------------------
 * Solve (I - A) y = c on S_? (the system of Section 2.3 with b replaced by a
 * caller vector) with the Jacobi method (method 0) or BiCGStab (method 1)
 * under `opts` (tolerances are absolute, as for the solvers; opts.x0 is a
 * starting point on S_?).  With c = b this is rp_jacobi / rp_bicgstab; with
 * c = 1 on S_?, y is the expected number of steps spent in S_? before
 * absorption; with c = b - (I - A) x^ (a residual) y is the correction of x^,
 * obtained in its own precision rather than rounded into x^ + y (used for
 * finite differences of the solution).
 *   rhs    device, n doubles (full state vector; entries outside S_? unused).
 *   y_out  device, n doubles: y on S_?, 0 on S_{=0} and S_{=1}.
 * Returns as for the solvers.                                                  */
int rp_solve_rhs(rp_context *ctx, rp_system *sys, int method, const double *rhs,
                 const rp_opts *opts, double *y_out, rp_solve_info *info);

/* ---- adjoint and gradient ------------------------------------------------------
 * For a loss L(x) with seed = dL/dx (device, n doubles; e.g. the unit vector
 * of an initial state for d x_init), solve (I - A)^T lambda = seed on S_? with
 * the Jacobi method (method 0) or BiCGStab (method 1) under `opts`, then form
 * dL/dP(s, s') = lambda_s * x_{s'} for every stored transition of a row in S_?
 * (x = 1 on S_{=1}, 0 on S_{=0}); rows outside S_? get 0.  The partition is
 * held fixed (a derivative on P's sparsity pattern).  The first adjoint on a
 * system builds the transposed reduced matrix (a stable sort of the entries
 * by column) and keeps it with the system: 18 bytes per off-diagonal entry
 * of A and 4 per row, plus about 24 bytes per entry of temporary device
 * memory during the build.
 *   x            device, n: the solution returned by rp_jacobi / rp_bicgstab.
 *   lambda_out   device, n (may be NULL): lambda on S_?, 0 elsewhere.
 *   grad_val_out device, nnz (may be NULL): aligned with the chain's val.
 * Returns as for the solvers.                                                 */
int rp_adjoint(rp_context *ctx, rp_system *sys, int method, const double *x,
               const double *seed, const rp_opts *opts, double *lambda_out,
               double *grad_val_out, rp_solve_info *info);

/* ---- strongly connected components of S_? (Section 8) ---------------------------
 * The decomposition the paper proposes as future work: split S_? into the
 * strongly connected components of A's graph (an edge s -> s' for every
 * stored A(s,s') > 0; self-loops join nothing) and solve them in reverse
 * topological order, a component with one state by substitution.
 *   label_out  device, n int32 (may be NULL): per state of S_?, the smallest
 *              state index of its component; -1 on S_{=0} and S_{=1}.
 *   level_out  device, n int32 (may be NULL): per state of S_?, its
 *              component's level: 0 when no edge leaves the component, else
 *              1 + the largest level an edge leads to; -1 outside S_?.
 *              Solving the levels in increasing order respects every
 *              dependency.
 *   info       host (may be NULL): counts below.
 * Markov-chain systems only (rp_matrix_system systems: RP_ERR_INVALID_ARG).
 * Components never cross instances.                                          */
typedef struct rp_scc_info {
    int64_t components;        /* components of S_? over all instances          */
    int64_t cyclic_components; /* components of more than one state             */
    int64_t largest;           /* states of the largest component               */
    int32_t levels;            /* levels 0 .. levels-1                           */
    int32_t rounds;            /* decomposition rounds (coloring + search)       */
    /* rp_scc_solve only (0 from rp_scc):                                         */
    int32_t substitution_levels; /* levels with one-state components: one
                                    substitution pass over those states        */
    int32_t jacobi_levels;     /* levels with larger components: in-place
                                  Jacobi sweeps over the states of those      */
    int64_t substitution_rows; /* states solved by substitution                  */
    int64_t jacobi_rows;       /* states solved by Jacobi sweeps                 */
    int64_t jacobi_sweeps;     /* sweeps summed over the Jacobi levels           */
} rp_scc_info;
int rp_scc(rp_context *ctx, rp_system *sys, int32_t *label_out,
           int32_t *level_out, rp_scc_info *info);
/* Solve by components, level by level in FP64: in each level the states of
 * one-state components take one substitution pass, then the states of the
 * larger components take in-place Jacobi sweeps until their largest change
 * is below opts.tol / 100 (at most opts.max_iter).  The lower levels are final
 * when a level starts, so each level's equations hold with the values below
 * it.  The result then starts the ordinary refinement under opts (stop,
 * precision, tolerance), which certifies or polishes it as rp_jacobi would
 * (usually with no or few further sweeps).
 *   x_out, info  as for rp_jacobi;  scc_info  host (may be NULL).
 * opts.update and opts.schedule are ignored for the level phase.             */
int rp_scc_solve(rp_context *ctx, rp_system *sys, const rp_opts *opts,
                 double *x_out, rp_solve_info *info, rp_scc_info *scc_info);

/* ---- measurement hook ------------------------------------------------------------
 * Not part of the method: kernel timing for benchmarks.  While enabled, each
 * batch of iteration launches between two host checks (opts.chunk
 * iterations) is bracketed by one pair of HIP events on the context's stream,
 * and the algorithmic bytes of the work those launches did are added up from
 * the per-instance iteration counts (Jacobi sweep: (4+w) z + (4+4w) n per
 * instance-iteration, w = 8 for FP64, 4 for FP32, z = off-diagonal entries of
 * A, n = |S_?|; a whole BiCGStab step, both sparse products and the vector
 * updates: 2(4+w) z + (8+21w) n; FP64 residual: 12 z + 36 n, one event pair
 * per launch).  Where the iteration needs a separate finishing launch per
 * iteration (systems too large for the LDS-staged kernels) the sparse-product
 * launches are timed one by one.  "launches" counts iterations for the
 * batched ids.  rp_profile_enable resets the totals.                          */
#define RP_PROF_JACOBI_FP64 0
#define RP_PROF_JACOBI_FP32 1
#define RP_PROF_SPMV_FP64 2
#define RP_PROF_SPMV_FP32 3
#define RP_PROF_VECTOR_FP64 4
#define RP_PROF_VECTOR_FP32 5
#define RP_PROF_RESIDUAL_FP64 6
#define RP_PROF_BICGSTAB_FP64 7
#define RP_PROF_BICGSTAB_FP32 8
/* the sweeps a tiled Jacobi solve runs resident once only a few small
 * instances still run (counted apart from the tiled sweeps above) */
#define RP_PROF_JACOBI_TAIL_FP64 9
#define RP_PROF_JACOBI_TAIL_FP32 10
#define RP_PROF_NKERNELS 11
int rp_profile_enable(rp_context *ctx, int enable);
/* Totals since the last rp_profile_enable: launches, summed event time (ms)
 * and algorithmic bytes.  Any output pointer may be NULL.                     */
int rp_profile_read(rp_context *ctx, int kernel, int64_t *launches,
                    double *total_ms, double *alg_bytes);

#ifdef __cplusplus
}
#endif

#endif /* RP_H */
