/*
 * stc.h -- C ABI of the structure-adaptive tile Cholesky library (libstc.so)
 * for AMD Instinct MI355X (gfx950), FP64 throughout.
 *
 * The operation is the numerical phase of the fixed-grid tile Cholesky of
 * arXiv 2609.29765: a sparsity pattern is analysed once (ordering, symbolic
 * factor, tile classification, static task list; Sec. 3, Sec. 5.1-5.2), then
 * its factor L with P A P^T = L L^T is computed many times for new values by
 * replaying one static POTRF/SYRK/GEMM/TRSM tile schedule (Algorithm 1), the
 * factor staying resident on the device where the log-determinant and solves
 * consume it (Sec. 6.7).  The split of a once-per-pattern analysis from a
 * repeated factorization is the interface the paper states (Sec. 6.6).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success; negative for usage errors (STC_ERR_*);
 *     STC_NOT_SPD (positive) when a factorization met a pivot that is not
 *     positive and finite.  No C++ exception crosses this boundary.  After a
 *     non-zero return, stc_last_error() holds a message (thread-local).
 *   - Host pointers are marked (host); device pointers (device).  Device
 *     pointers must address memory of the device that was current when the
 *     handle was bound.
 *   - The caller owns every device buffer (workspace, values, right-hand
 *     sides, outputs) and every stream.  The library allocates no device
 *     memory: stc_workspace_bytes() says how much the caller must provide.
 *     The one exception is the static per-device array (32 MiB) that
 *     stc_solve_noalloc uses in place of workspace scratch.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Calls taking a stream are asynchronous with respect to the host.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef STC_H
#define STC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define STC_OK 0
#define STC_ERR_ARG (-1)     /* a null pointer, a size out of range, a bad option */
#define STC_ERR_PATTERN (-2) /* input pattern not a valid lower CSC (see stc_analyse) */
#define STC_ERR_STATE (-3)   /* wrong call order (e.g. logdet before factorize)    */
#define STC_ERR_ALLOC (-4)   /* host allocation failed or workspace too small      */
#define STC_ERR_HIP (-5)     /* a HIP runtime call failed                          */
#define STC_ERR_SCHEDULE (-6) /* stc_check_schedule found a conflicting pair of kernels */
#define STC_NOT_SPD 1        /* numerical: a pivot was not positive and finite     */

/* orderings (Sec. 3): the paper runs several fill-reducing heuristics and scores
   them; this library offers its own deterministic NATURAL, RCM and level-
   structure nested dissection, and AUTO scoring of the three */
#define STC_ORD_NATURAL 0
#define STC_ORD_RCM 1
#define STC_ORD_ND 2
#define STC_ORD_AUTO 3
#define STC_ORD_GIVEN 4

/* storage mode: AUTO follows the selector (Sec. 5.1); DENSE stores every
   non-empty tile in full; SEMISPARSE keeps only active rows (Sec. 4.1) */
#define STC_MODE_AUTO 0
#define STC_MODE_DENSE 1
#define STC_MODE_SEMISPARSE 2

/* routes reported by the selector (Sec. 5.1); SUPERNODAL is reported and the
   factorization then runs on the active-column tiles */
#define STC_ROUTE_DENSE 0
#define STC_ROUTE_SEMISPARSE 1
#define STC_ROUTE_SUPERNODAL 2

/* task opcodes of Algorithm 1 */
#define STC_OP_POTRF 1
#define STC_OP_SYRK 2
#define STC_OP_TRSM 3
#define STC_OP_GEMM 4

typedef struct stc_handle stc_handle;

typedef struct {
  int32_t nb;            /* tile size n_b: 32, 64, 128 or 256; 0 = automatic:
                            64, or, when the pattern takes the dense route at
                            64 (mode AUTO: Sec. 5.1's selector; or mode
                            DENSE), 256 from n = 2048 and 128 from n = 512     */
  int32_t mode;          /* STC_MODE_*                                           */
  int32_t ordering;      /* STC_ORD_*                                            */
  const int32_t* perm;   /* (host) perm[new] = old, read when ordering == GIVEN  */
  int32_t wg_slots;      /* schedule: concurrent update work-groups the per-
                            level split of long update chains (deterministic
                            split-K) is balanced for, and the early-group
                            work above which a level's last groups get a
                            launch of their own; 0 = 448 for n_b >= 128 and
                            896 for smaller tiles (the best of sweeps on
                            MI355X).  Changes timing only.                     */
  int32_t align;         /* tile grid: 0 = the uniform n_b grid of Sec. 4.1,
                            except for patterns the selector routes
                            supernodal (mode AUTO), whose grid is aligned at
                            n_b (Sec. 5.4: their tiles follow the fill);
                            > 0 = a grid aligned to the elimination tree of
                            P A P^T: every subtree of at least `align` columns
                            whose columns are consecutive starts on a tile
                            boundary, the tile before it padded with identity
                            rows (tiles then follow the tree, as the supernodal
                            tiles of Sec. 5.4 follow the supernodes, and
                            independent subtrees no longer share a tile).  The
                            features, the route and the factor's values are
                            those of the uniform grid; tiles, tasks and the
                            schedule follow the aligned grid.                  */
  int32_t max_split;     /* schedule: most work-groups one update task's K
                            stream is split over (1-64; 0 = 64)               */
  int32_t fold_pct;      /* schedule: weight, in percent of the measured cost,
                            that the split's cost model gives to folding one
                            partial slot (0 = 100).  Both change timing only. */
  int32_t batch;         /* schedule: value sets factorized together (0 or 1:
                            one).  B > 1 value sets of one pattern already
                            fill the device B times over, so each set's split
                            is balanced for max(16, wg_slots / B) work-groups
                            (wg_slots or its default).  Changes timing only;
                            any batch size can still be bound.                 */
} stc_opts;

/* Analyse a sparsity pattern once (Sec. 3, Sec. 5.1-5.2).
   n       order of the symmetric matrix A, 1 <= n < 2^31.
   colptr  (host) int64[n+1], rowind (host) int32[colptr[n]]: the LOWER
           triangle of A in CSC form, original numbering, rows ascending within
           each column, the diagonal present and first, no duplicates.  Input
           values passed later to stc_factorize follow this entry order.
   opts    (host) may be NULL (automatic tile size, AUTO mode, AUTO ordering).
   out     (host) receives a new handle; the library copies the pattern.
   Errors: STC_ERR_PATTERN for an invalid pattern, STC_ERR_ARG for bad
   options.  The handle owns only host memory until stc_bind is called. */
int stc_analyse(int64_t n, const int64_t* colptr, const int32_t* rowind, const stc_opts* opts,
                stc_handle** out);

/* Device workspace needed to bind with `batch` value sets (batch >= 1):
   device metadata, `batch` tile stores, and scratch for logdet, solve and the
   logdet adjoint.  bytes (host) receives the size. */
int stc_workspace_bytes(const stc_handle* h, int32_t batch, size_t* bytes);

/* Bind a caller-owned device workspace of at least stc_workspace_bytes(batch)
   bytes, aligned to 256 bytes, on the current device.  Uploads the metadata
   (synchronously) and captures the factorization schedule as a HIP graph.
   The workspace must stay allocated while the handle uses it; binding again
   (new buffer or new batch) replaces the previous binding. */
int stc_bind(stc_handle* h, void* d_workspace, size_t bytes, int32_t batch, void* stream);

/* Factorize one value set (Sec. 5.2-5.3): d_values (device) double[nnz] in
   the analysed CSC entry order.  The factor stays in the workspace.  Pivot
   failures are recorded on the device: read them with stc_info. */
int stc_factorize(stc_handle* h, const double* d_values, void* stream);

/* Factorize B same-pattern value sets in one graph launch and write their
   log-determinants.  d_values (device) double[B][nnz]; d_logdet (device)
   double[B]; d_info (device) int32[B], 0 or the 1-based permuted column of the
   first failing pivot of that member (its logdet is then NaN).  Requires
   1 <= B <= the batch the handle was bound with. */
int stc_factorize_batched(stc_handle* h, const double* d_values, int32_t B, double* d_logdet,
                          int32_t* d_info, void* stream);

/* log det A = 2 sum_i log L_ii of the last single factorization, written to
   d_out (device) double[1]; NaN if that factorization failed. */
int stc_logdet(stc_handle* h, double* d_out, void* stream);

/* Solve A X = B in place with the last single factorization (Sec. 6.7: the
   factor stays on the device and is reused): d_b (device) double[n * nrhs],
   column-major, original numbering, 1 <= nrhs <= 64.  Forward and backward
   block sweeps over the factor's tiles, level by level, for up to 8 columns
   at a time (the factor is read once per group): the products of the tiles
   a level's solved blocks unlock are subtracted from the blocks those tiles
   feed, each fed block (or chunk of it) by one work item in a fixed tile
   order, so results are reproducible bit for bit; the work item of a block
   of the next level then solves its diagonal block in the same launch.  The
   sweeps for each group are captured in a graph on first use.  When that
   factorization failed (stc_info != 0) every entry of d_b is set to NaN. */
int stc_solve(stc_handle* h, double* d_b, int32_t nrhs, void* stream);

/* Solve A_b X_b = B_b in place for value sets b = 0..B-1 of the last batched
   factorization (1 <= B <= the B of that call; member 0 is also the last
   single factorization): d_b (device) double[B][n * nrhs], value set b's
   right-hand sides column-major at d_b + b n nrhs, original numbering,
   1 <= nrhs <= 8.  The same level sweeps as stc_solve, each launch covering
   every value set (grid.y = value set), captured in a graph per (B, nrhs
   group) on first use.  A value set whose factorization failed gets NaN.
   STC_ERR_STATE before a batched factorization of at least B value sets. */
int stc_solve_batched(stc_handle* h, double* d_b, int32_t B, int32_t nrhs, void* stream);

/* For callers that cannot allocate device memory or instantiate graphs while
   they run (code under HIP graph capture, tight serving loops, harnesses
   that forbid allocation): stc_solve with the same arguments, results and
   error codes, except that the permuted right-hand sides its sweeps work on
   live in a static device array of the library (32 MiB, one per device,
   held until the process ends; its address is looked up by stc_bind) instead
   of the workspace, and the sweeps are launched kernel by kernel instead of
   from a captured graph.  The call allocates nothing: no hipMalloc, hipFree,
   graph instantiation or allocating library routine.  Limit: padded order
   (N_T * n_b) * nrhs <= 4,194,304 doubles, else STC_ERR_ARG before any
   launch.  Every call on one device shares that array, and each call
   rewrites all of it that it reads, so no state carries over between calls;
   calls that overlap in time on one device (different streams, host
   threads) race on it and must be serialized by the caller. */
int stc_solve_noalloc(stc_handle* h, double* d_b, int32_t nrhs, void* stream);

/* Reverse mode of logdet through the last single factorization: given the
   scalar cotangent d_gbar (device) double[1], writes d_grad_values (device)
   double[nnz] in the analysed CSC entry order, the symmetric matrix being
   parameterised by its lower triangle: gbar * 2 (A^-1)_ij off the diagonal and
   gbar * (A^-1)_ii on it.  For this cotangent the adjoint of the tile Cholesky
   restricted to the pattern of L is the selected inverse Z = A^-1 on that
   pattern (the selected inversion that consumes the resident factor, Sec.
   6.7), computed on the device by the blocked Takahashi recurrence over the
   tile DAG in reverse order (one graph launch; long tasks of a level are
   split over several work-groups and their partial results added after the
   level in a fixed order, so the result is reproducible bit for bit), from
   the factor and the 32 x 32 diagonal-block inverses the factorization left
   in the workspace.  Writes
   NaN everywhere when that factorization failed (stc_info != 0).  Overwrites
   the workspace's selected-inverse scratch; the factor is left intact. */
int stc_logdet_backward(stc_handle* h, const double* d_gbar, double* d_grad_values, void* stream);

/* Selected inversion of the last single factorization (Sec. 6.7: the
   resident factor serves selected inversion, whose diagonal gives the
   posterior marginal variances of a Gaussian field with precision A).
   Computes Z = (P A P^T)^-1 on the pattern of L on the device -- the
   blocked Takahashi recurrence over the tile DAG in reverse, the same sweep
   as stc_logdet_backward, into the workspace's selected-inverse scratch --
   and, when d_diag (device) double[n] is not NULL, writes diag(A^-1) to it
   in original numbering.  NaN throughout when that factorization failed.
   The factor is left intact; the scratch holds Z until the next
   factorization (read it with stc_get_selinv). */
int stc_selinv(stc_handle* h, double* d_diag, void* stream);

/* Copy Z = (P A P^T)^-1 on the pattern of L, as left by the last stc_selinv
   or stc_logdet_backward of the current factorization, to h_Zx (host)
   double[nnz(L)] in stc_get_L_pattern order (permuted numbering);
   synchronizes the stream.  STC_ERR_STATE if no selected inverse of the
   current factorization is held.  NaN throughout when it failed. */
int stc_get_selinv(stc_handle* h, double* h_Zx, void* stream);

/* Status of the last single factorization; synchronizes the bound stream.
   info (host) receives 0 or the 1-based permuted column of the first pivot
   that was not positive and finite. */
int stc_info(stc_handle* h, int32_t* info);

/* Symbolic exports (host copies, for inspection and bit-exact checks).
   sizes (host) int64[16]: n, nnz(tril A), nnz(L), nb, N_T, non-empty
   off-diagonal tiles, total stored active rows, tasks, mode (1 dense,
   2 semisparse), route, dense rows set aside, ordering used, active tiles
   (off-diagonal + N_T), tile-store doubles per value set, levels, kernel
   launches of the forward and backward sweeps of one solve group. */
int stc_get_sizes(const stc_handle* h, int64_t* sizes);
/* features (host) double[3]: fill ratio phi, mean occupancy rho, skew sigma */
int stc_get_features(const stc_handle* h, double* features);
int stc_get_perm(const stc_handle* h, int32_t* perm);     /* int32[n], perm[new] = old */
int stc_get_etree(const stc_handle* h, int32_t* parent);  /* int32[n], -1 for roots    */
int stc_get_L_pattern(const stc_handle* h, int64_t* colptr, int32_t* rowind); /* permuted */
/* tiles in order k ascending then m ascending: m, k, stored rows, pattern rows,
   contiguous flag, row offsets int64[ntiles+1], rows (local to block m), kd[N_T] */
int stc_get_tiles(const stc_handle* h, int32_t* m, int32_t* k, int32_t* cnt, int32_t* true_cnt,
                  int8_t* contig, int64_t* roff, int32_t* rows, int32_t* kd);
int stc_get_tasks(const stc_handle* h, int32_t* tasks); /* int32[ntasks][4]: op, m, k, n */
/* grid position of every column of P A P^T (int64[n], ascending); tile t
   covers positions [t n_b, (t+1) n_b), positions no column takes are padding.
   The identity on the uniform grid.  *align (if not null) receives the
   grid's stc_opts.align (0 for the uniform grid). */
int stc_get_grid_positions(const stc_handle* h, int64_t* pos, int64_t* align);

/* Copy the last single factor to the host, in stc_get_L_pattern order
   (h_Lx double[nnz(L)]); synchronizes the stream. */
int stc_get_factor(stc_handle* h, double* h_Lx, void* stream);

/* Copy the factor of value set `member` (0 <= member < the bound batch) of
   the last batched factorization to the host, in stc_get_L_pattern order
   (h_Lx double[nnz(L)]); member 0 is also the last single factorization.
   Synchronizes the stream. */
int stc_get_batch_factor(stc_handle* h, int32_t member, double* h_Lx, void* stream);

/* Static work of one factorization with this plan (host) double[10]:
   [0] tile-algorithmic flops of the SYRK+GEMM updates: sum |R_kn|^2 n_b over
       SYRK tasks + sum 2 |R_mn| |R_kn| n_b over GEMM tasks (Algorithm 1's
       tasks on the stored active rows, Sec. 5.2); [1] POTRF flops sum h^3/3;
   [2] TRSM flops sum |R_mk| n_b^2; [3] their total; [4] exact Cholesky flops
   sum_j c_j^2 (c_j = entries of column j of L); [5] update bytes: operand
   rows read per task plus every output tile read and written once; [6] value
   load bytes: 16 per input entry (value and its load entry) plus 8 per
   stored double (the store written once); [7] levels;
   [8] flops of stc_logdet_backward (tile products of the selected-inverse
   recurrence, 2 per multiply-add); [9] its levels after the diagonal-tile
   inverses: one contraction launch each, followed by a launch that folds the
   partial results where the level's long tasks were split. */
int stc_get_work(const stc_handle* h, double* work);

/* Shape of the replayed schedule (host, no device work), stats (host)
   int64[5]: [0] update tasks whose K stream is split over several
   work-groups (deterministic split-K: parts after the first leave partial
   sums that the tile's next update folds in a fixed order); [1] doubles of
   partial-sum slot memory per value set; [2] levels whose last-group updates
   have a kernel of their own; [3] kernels (graph nodes) of one
   factorization; [4] doubles the slots would take without sharing memory
   (slots share memory where the kernel graph orders the fold of one before
   the write of the next).  All are set by the plan alone (the pattern, n_b,
   mode and the schedule options). */
int stc_get_plan_stats(const stc_handle* h, int64_t* stats);

/* Host check of the factorization schedule, no device work.  The
   factorization replays a graph with one node per non-empty POTRF, update
   and TRSM kernel of a level, whose edges stand for the waits Algorithm 2
   performs on its progress matrix (Sec. 5.3).  This re-derives from the plan
   the data each kernel reads and writes (tiles, diagonal tiles with their
   32 x 32 inverses, split-K partial slots) and verifies that the kernels of
   one level touch disjoint data, that every edge points to an earlier node,
   and that every two kernels that both touch one object, at least one of
   them writing it, are ordered by a path of edges.  Partial slots are
   checked as ranges of the slot memory, which slots share: every two kernels
   whose slot ranges overlap, one of them writing, are ordered, no kernel
   writes a slot range that it also reads, and every range lies inside the
   slot memory.  stats (host) int64[5] receives: nodes, edges, pairs of
   kernels the graph leaves unordered (and that may therefore overlap), data
   objects (tiles), pairs of kernels ordered because they share slot memory.
   Returns 0, STC_ERR_ARG for a null argument, or STC_ERR_SCHEDULE with
   stc_last_error naming the pair. */
int stc_check_schedule(const stc_handle* h, int64_t* stats);

/* Host check of the solve's work items (Sec. 6.7: the sweeps over the
   resident factor), no device work.  Per sweep it replays the launches in
   order, the items of one launch taken as concurrent, and verifies that every
   block is solved by exactly one step item, only after every tile that feeds
   it has been applied; that every tile is applied exactly once (whole, or as
   one of each of its row / column chunks) and only after a launch that
   solved its source block; and that no two items of a launch write the same
   rows.  stats (host) int64[4] receives, over both sweeps: launches, step
   items, panel items, launches holding both kinds.  Returns 0,
   STC_ERR_ARG for a null argument, or STC_ERR_SCHEDULE with stc_last_error
   naming the violation. */
int stc_check_solve_schedule(const stc_handle* h, int64_t* stats);

/* Host check of the reverse-mode plan (stc_logdet_backward, stc_selinv), no
   device work.  Its levels run in order: the diagonal-tile inverses G_k,
   then one contraction launch per level, each followed by a launch that folds
   the partial results of the level's split tasks.  Verified: every term of
   the recurrence belongs to exactly one task and contracts over 1..n_b
   entries (the contraction kernel streams a task's terms and reads a term's
   first chunk during the previous term's last); every tile a level reads (Z,
   M = L_mk G_k, G_k) was written at an earlier level; every Z and M tile is
   written by one task of one level (the diagonal Z_kk accumulating once into
   H_k); partial slots lie in the slot scratch and the slots of one level are
   disjoint; each fold adds, to a tile its level wrote, slots that the level's
   parts wrote.  stats (host) int64[5]: levels, tasks, tile reads checked,
   folds, partial slots.  Returns 0, STC_ERR_ARG for a null argument, or
   STC_ERR_SCHEDULE with stc_last_error naming the violation. */
int stc_check_backward(const stc_handle* h, int64_t* stats);

/* Measurement helper: one factorization of d_values (device) double[nnz]
   with the same kernels as stc_factorize, launched one by one instead of from
   the graph, with a HIP event pair around each launch on `stream`;
   synchronizes the stream.  kind_ms (host) double[5], kind_launches (host)
   int64[5] and kind_flops (host) double[5] receive total kernel milliseconds,
   launch counts and tile-algorithmic flops (the stc_get_work [3] terms of the
   tasks each launch runs) for: [0] value load (fill + scatter, no flops);
   [1] POTRF; [2] updates with 128 x 128 blocks; [3] updates with 64 x 64
   blocks only; [4] TRSM.  In the graph the kernels of one level run
   concurrently; here they run one after the other.  Leaves the factor
   resident like stc_factorize. */
int stc_profile_factorize(stc_handle* h, const double* d_values, void* stream, double* kind_ms,
                          int64_t* kind_launches, double* kind_flops);

/* Measurement helper: FP64 matrix-core (MFMA 16x16x4) issue rate of the
   current device in TFLOP/s, from a kernel that keeps 16 independent
   accumulators per wave in registers and touches no memory in its loop
   (8 work-groups of 4 waves per compute unit).  tflops (host) double[1]. */
int stc_fp64_mfma_peak(void* stream, double* tflops);

/* Persist the analysis of a handle (Sec. 6.6, Table 6: the analysis is the
   one-off cost that many factorizations amortize) so that another process
   can skip it.  stc_save writes the symbolic analysis, the factorization
   and solve plans and the reverse-mode plan to the file at path (host,
   NUL-terminated; overwritten); nothing device-side is saved.  stc_load reads
   such a file into a new unbound handle (*out), which then behaves exactly
   like the one saved: every export and every result is identical.  The
   file is for the same library build on the same kind of host: it carries
   a magic, a format version, the host's type sizes and a checksum, and
   stc_load returns STC_ERR_ARG for a file that does not match them or is
   truncated or corrupted, STC_ERR_ALLOC when host memory runs out. */
int stc_save(const stc_handle* h, const char* path);
int stc_load(const char* path, stc_handle** out);

void stc_destroy(stc_handle* h);
const char* stc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STC_H */
