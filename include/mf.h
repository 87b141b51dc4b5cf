/*
 * mf.h -- C ABI of libmf: Foata-level multifrontal LU of FEM systems on one MI355X (gfx950).
 *
 * The problem is stated as in the paper: a set of element matrices plus mesh connectivity
 * (the fronts at the leaves of the elimination tree are the element matrices, Sec. 2.4), and a
 * right-hand side (the multifrontal driver of Table 2 takes the FEM input and the load vector).
 *
 * Conventions shared by every entry point
 *   - Every call returns int: MF_OK (0) on success, a negative MF_E* code on failure.  After a
 *     failure, mf_last_error() returns a thread-local, NUL-terminated message.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory on the
 *     current device (e.g. from torch tensors).  The caller owns every buffer it passes; the
 *     plan copies what it keeps.  All matrices are row-major, FP64 unless stated otherwise.
 *   - Device work is enqueued on `hip_stream` (a hipStream_t, NULL = the null stream).
 *   - A plan must not be used from two threads at the same time.
 *   - Batches: n_mesh > 1 meshes are solved together.  Nodes and elements are concatenated in
 *     mesh order; global node id = mesh node id + sum of n_nodes of the preceding meshes, and
 *     the same for elements.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MF_OK = 0,
  MF_EINVAL = -1,       /* invalid argument (sizes, ids, pointers, unsupported combination) */
  MF_ENOMEM = -2,       /* host or device allocation failed */
  MF_EZERO_PIVOT = -3,  /* zero or non-finite pivot during factorization (no pivoting) */
  MF_EHIP = -4,         /* a HIP runtime call failed (message names it) */
  MF_ENOCONV = -5,      /* iterative refinement did not reach the tolerance */
  MF_ESTATE = -6        /* call out of order, e.g. solve before a successful factor */
};

/* Arithmetic of the Schur-complement update C22 -= L21 U12 (Sec. 2.2) on the tiled path.  The
 * pivot-block LU, the triangular solves and everything else always run in FP64. */
enum { MF_FP64 = 0, MF_SCHUR_FP32 = 1, MF_SCHUR_BF16 = 2 };

typedef struct mf_plan mf_plan;   /* opaque: host analysis, device plan, factor storage */

/* One structured or unstructured mesh of tensor-product elements.
 *   dim       2 or 3
 *   npe       nodes per element: (p+1)^dim for Q_p Lagrange elements, p = 1, 2, 3 (the
 *             linear, quadratic and cubic bases of Sec. 5); equal for all meshes of a batch
 *   n_nodes   nodes of this mesh; ids 0..n_nodes-1, every node used by some element
 *   n_elem    elements of this mesh (>= 1)
 *   conn      host [n_elem][npe] node ids in the element's local order; the element matrices
 *             passed to mf_factor / mf_refine use the same order (the tree depends only on
 *             which nodes an element has, not on their order)
 *   elem_ijk  host [n_elem][dim] integer element coordinates, pairwise distinct; they drive the
 *             nested-dissection bisection of the elimination tree.  NULL: connectivity only,
 *             the tree of Table 3 (element fronts sorted by lowest node id, joined in adjacent
 *             pairs round after round, an odd last front carried to the next round)        */
typedef struct {
  int32_t dim, npe;
  int64_t n_nodes, n_elem;
  const int32_t *conn;
  const int32_t *elem_ijk;
} mf_mesh;

typedef struct {
  int64_t n;                 /* unknowns (sum of n_nodes) */
  int64_t n_elem;            /* elements (sum of n_elem) */
  int64_t n_fronts;          /* fronts (2 n_elem - n_mesh) */
  int64_t sum_m;             /* sum of front widths: length of front_idx */
  int64_t sum_mk;            /* sum of m*k: length of the L (and of the U) export buffer */
  int64_t store_doubles;     /* device factor storage, doubles (sum of m^2) */
  int32_t n_mesh, dim, npe;
  int32_t height;            /* Foata classes are 0..height */
  int32_t max_m, max_k;
  double factor_flops;       /* sum over pivots of (r-1) + 2 (r-1)^2, r = m - p */
  double solve_flops_per_rhs;/* sum over pivots of 1 + 4 (r-1) (forward + backward) */
  double sum_cb2;            /* extend-add entries: sum over fronts of (m-k)^2 */
} mf_info;

/* Builds the elimination tree of the batch (host work only; no GPU needed).
 * Tree (Sec. 2.4, Table 3): recursive coordinate bisection of each mesh's element index box --
 * split the axis with the most elements (ties: lowest axis) at lo + floor(len/2), lower half
 * first -- down to single elements; fronts numbered in post-order, mesh after mesh.
 * Pivots of a front are the nodes whose elements all lie in it and in neither child (the front
 * that owns them alone, Table 2); its contribution block (CB) is the rest of its children's
 * CBs (a leaf: of its element's nodes).  Index list: pivots ascending, then CB ascending
 * (pivots first, Sec. 3.2).  Foata class (Sec. 3.3) = height above the leaves.
 * meshes: host array of n_mesh descriptors (read only during the call).
 * out: receives a new plan; release it with mf_destroy.  The plan replays its per-class launch
 * sequences as captured hipGraphs unless the environment holds MF_GRAPHS=0 when it is created.
 * Errors: MF_EINVAL (bad sizes, ids out of range, duplicate elem_ijk, unused node), MF_ENOMEM. */
int mf_analyse(int32_t n_mesh, const mf_mesh *meshes, mf_plan **out);

/* Sizes and operation counts of an analysed plan: fronts, Foata classes (Sec. 3.3) and the
 * flop counts of the task alphabet of Sec. 3 (per pivot of a front, Table 2's division,
 * multiplication and subtraction tasks; per pivot and right-hand side, the solve's).
 * out: host, filled on success.  Errors: MF_EINVAL (null argument). */
int mf_plan_info(const mf_plan *plan, mf_info *out);

/* Copies the tree to host buffers sized from mf_info (any pointer may be NULL to skip it):
 *   parent[n_fronts] (-1 at a root), level[n_fronts], front_ptr[n_fronts+1] (offsets into
 *   front_idx), front_idx[sum_m] (global node ids), npiv[n_fronts],
 *   leaf_elem[n_fronts] (global element id of a leaf, -1 for internal fronts). */
int mf_plan_export_tree(const mf_plan *plan, int32_t *parent, int32_t *level, int64_t *front_ptr,
                        int32_t *front_idx, int32_t *npiv, int64_t *leaf_elem);

/* Scalar-task trace of the factorization and its Foata classes (Sec. 3, Sec. 3.3), a host
 * analysis for tiny meshes (at most 4096 unknowns and 5e7 tasks).  The tasks: division T1 per
 * pivot and later entry of its row, multiplication T2 and subtraction T3 per pivot and pair of
 * later front entries, assertion T4 per global entry; the dependencies J1..J4, subtractions into
 * one entry ordered by their pivots' elimination order.  out receives the task counts, the
 * number of Foata classes (every task in the earliest class after its predecessors), how many
 * of them hold a single task type, the number of classes of the 4-periodic schedule (every task
 * in the earliest such class congruent to its type: T4 1, T1 2, T2 3, T3 0 mod 4), and whether
 * the front classes (tree heights) order every dependency between two fronts' tasks.
 * hist (host, may be NULL) receives hist[c * 4 + t] = tasks of type t (T1, T2, T3, T4) in
 * Foata class c, for c < cap / 4; needed (may be NULL) the entries it takes, 4 (classes + 1).
 * Errors: MF_EINVAL (null plan, mesh too large). */
typedef struct {
  int64_t tasks[4];
  int32_t fnf_classes, fnf_single_type_classes, typed_classes, levels_order_dependencies;
} mf_trace_info;

int mf_task_trace(const mf_plan *plan, mf_trace_info *out, int64_t *hist, int64_t cap,
                  int64_t *needed);

/* Schedule tuning of an analysed plan (set by mf_autotune, or by hand; defaults otherwise).
 *   small_max_m  fronts of width <= small_max_m are assembled, eliminated and stored by one
 *                workgroup with the front resident in LDS; wider fronts take the tiled path
 *                (assembly, panel LU of nb pivots at a time, MFMA Schur GEMM).  It is clipped
 *                to what fits in one workgroup's LDS on the device.  0 keeps the current value.
 *   nb           panel width of the tiled path's separate panel launches: 16, 32 or 64.
 *                0 keeps the current value.  (The persistent route always uses 32.)
 *   fused_max_m  tiled fronts of width <= fused_max_m run all their panels (32 pivots each) in
 *                one workgroup, leaving only the Schur GEMM to a separate launch; wider fronts
 *                use one launch per panel step.  Clipped to 576; -1 disables the fused route;
 *                0 keeps the current value.  (Not used by the persistent route.)
 *   tile         output tile edge of the MFMA GEMMs: 32 or 64.  0 keeps the current value.
 *   persistent   1: the tiled fronts of a Foata class run in one persistent launch whose
 *                workgroups take the class's extend-add strips, panel chunks, update tiles
 *                and Schur tiles in order and wait on per-front progress counters;
 *                -1: one launch per kind of work and per panel step (the default); 0 keeps it.
 * The values apply to every class (a per-class schedule chosen by mf_autotune is dropped).
 * Invalidates a previous factorization.  Errors: MF_EINVAL. */
int mf_set_tuning(mf_plan *plan, int32_t small_max_m, int32_t nb, int32_t fused_max_m,
                  int32_t tile, int32_t persistent);

/* Per-class schedule: params (host) holds n_class = height + 1 rows of five values, one row per
 * Foata class in order -- small_max_m (>= 1), nb (16, 32, 64), fused_max_m (0 = off, clipped to
 * 576), tile (32, 64), persistent (0, 1), each meaning what it does in mf_set_tuning, for the
 * fronts of that class only.  n_class = 0 drops a per-class schedule (mf_set_tuning's values
 * then apply to every class).  This is the form mf_autotune chooses ("classes" of its report).
 * Invalidates a previous factorization.  Errors: MF_EINVAL (wrong class count, bad value). */
int mf_set_class_tuning(mf_plan *plan, int32_t n_class, const int32_t *params);

/* Bottom-subtree launches (Sec. 3.3's class barrier kept inside a workgroup): the leading
 * Foata classes whose fronts all take the one-wave-per-front routes (the tiny factor route,
 * fronts up to 32 wide; the wave solves, up to 64) run as one launch of the factorization and
 * one of each sweep instead of one per class.  The fronts of those classes split into units --
 * a front whose parent lies above the fused classes, with all its descendants -- and one
 * workgroup takes a unit class by class with a workgroup barrier between classes; the results
 * are identical to the per-class launches.  max_classes: at most this many classes (-1: as many
 * as the routes allow, 0 or 1: off, the default); min_units: the most classes that still give
 * at least this many units are fused (default 2048, so that the launch fills the chip; >= 1).
 * The factorization and the solves choose separately.  Off by default: a unit's classes run
 * one after another inside its workgroup with fewer fronts per class than waves near its root,
 * while the per-class launches keep every wave busy -- on the 2D and 3D trees measured the
 * per-class launches are faster.  Takes effect at the next device call; invalidates a previous
 * factorization.  Errors: MF_EINVAL. */
int mf_set_subtree_launch(mf_plan *plan, int32_t max_classes, int64_t min_units);

/* The bottom-subtree launches in use (uploads the plan's schedule first, see mf_factor):
 * out (host, 4 values) = classes fused and units of the factorization, then of the solves
 * (0 classes: per-class launches).  Errors: MF_EINVAL, MF_EHIP. */
int mf_subtree_launch_info(mf_plan *plan, int64_t *out);

/* Chunked triangle solves (no transposition): a class whose widest front has at least
 * min_pivots pivots solves its fronts' pivot triangles in launches of 128 pivots, one workgroup
 * per 128-row tile of the rows each chunk updates (every workgroup solving the chunk's own
 * triangle from its diagonal-block inverses), instead of one workgroup walking each front's
 * whole triangle; its contribution rows take the rectangular launches.  The same solution up to
 * rounding.  min_pivots: 0 = off; default 512.  Takes effect at the next device call (the
 * factorization is kept).  Errors: MF_EINVAL. */
int mf_set_chunked_solve(mf_plan *plan, int32_t min_pivots);

/* Autotuner: factors elem_mats (device, as in mf_factor) under each candidate schedule that the
 * workload's front widths make relevant -- persistent class launches on/off, GEMM tile 64/32,
 * fused route on/off, panel width 32/64, LDS limit 128/64 -- timing `reps` factorizations of
 * each as a whole (host clock, median) and each Foata class's launches on their own (device
 * events on the launch stream, mean).  Every class then takes the candidate under which its
 * launches were fastest; the per-class schedule is kept if the whole factorization under it is
 * faster than under the best single candidate, else that candidate is kept for every class.
 * Leaves the plan factored with the kept schedule.  report (host, cap bytes, may be NULL)
 * receives a NUL-terminated JSON summary {"candidates": [{..., "ms", "class_ms": [...]}],
 * "chosen": {"mode": "per_class" | "global", "ms", ..., "classes": [...]}}; needed (may be NULL)
 * its size.  Synchronizes hip_stream.  Errors: as mf_factor, MF_EINVAL. */
int mf_autotune(mf_plan *plan, const double *elem_mats, int32_t precision, int32_t reps,
                void *hip_stream, char *report, int64_t cap, int64_t *needed);

/* Numerical factorization (Table 2 over Foata classes, Sec. 3.3): for every class in order, all
 * its fronts extend-add their children's contribution blocks (a leaf takes its element
 * matrix), partially LU-eliminate their k pivots with the pivot row scaled by the pivot
 * (U unit upper, L carrying the pivots), and apply the Schur update to their CB.
 * elem_mats: device [n_elem][npe][npe] FP64.  precision: MF_FP64 / MF_SCHUR_FP32 / MF_SCHUR_BF16.
 * Synchronizes `hip_stream` to read back the pivot status.
 * Errors: MF_EZERO_PIVOT (the plan then holds no valid factor; see mf_last_error for the front
 * and pivot), MF_EINVAL, MF_ENOMEM, MF_EHIP. */
int mf_factor(mf_plan *plan, const double *elem_mats, int32_t precision, void *hip_stream);

/* Solves A x = b (transpose = 0) or A^T x = b (transpose = 1) with the stored factors:
 * forward substitution leaves -> root, backward substitution root -> leaves (Sec. 1.1).
 * b, x: device [n][nrhs] FP64 (may alias).  Asynchronous on hip_stream.
 * Errors: MF_ESTATE (no valid factor), MF_EINVAL, MF_ENOMEM, MF_EHIP. */
int mf_solve(mf_plan *plan, const double *b, double *x, int32_t nrhs, int32_t transpose,
             void *hip_stream);

/* Largest scratch of mf_solve_noalloc, in doubles (64 MiB): the sum of contribution-block
 * widths of the plan (plus the chunked triangle solves' rows) times nrhs must not exceed it (the
 * 256 x 256 Q1 grid: 901,042 x 8 RHS). */
#define MF_NOALLOC_SCRATCH_DOUBLES 8388608

/* mf_solve for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and results as mf_solve,
 * launched eagerly on hip_stream, with no hipMalloc, hipFree or other allocation in the call.
 * Its only workspace, the per-front contribution blocks of the right-hand sides and the pivot
 * rows of the chunked triangle solves ((sum of CB widths + the widest chunked class's pivots)
 * x nrhs doubles), lives in a static device array of MF_NOALLOC_SCRATCH_DOUBLES doubles
 * that each GPU holds until the process ends; its device address is looked up once per device
 * (on the first call with that device current).  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (two streams, two threads, two plans) race: order them.  The
 * plan must already be factored (mf_factor allocates what the solve reads), and the plan's
 * device must be current.  b, x: device [n][nrhs] FP64 (may alias).  Asynchronous.
 * Errors: MF_EINVAL (nrhs too large for the scratch, bad arguments), MF_ESTATE (no valid
 * factor), MF_EHIP. */
int mf_solve_noalloc(mf_plan *plan, const double *b, double *x, int32_t nrhs, int32_t transpose,
                     void *hip_stream);

/* r = b - A x with A applied element by element (A = sum_e P_e^T K_e P_e, the FEM operator
 * whose element matrices are the leaves of Sec. 2.4), FP64.  Not a step of the paper's method:
 * the check of the solve that the refinement below uses.
 * elem_mats device [n_elem][npe][npe]; x, b, r device [n][nrhs].  Asynchronous. */
int mf_residual(mf_plan *plan, const double *elem_mats, const double *x, const double *b,
                double *r, int32_t nrhs, void *hip_stream);

/* Iterative refinement in FP64 around the solve of Sec. 1.1 (not in the paper; it restores
 * FP64 accuracy when the Schur updates of Sec. 2.2 ran in FP32 or BF16, MF_SCHUR_*):
 * x = solve(b); repeat r = b - A x, x += solve(r) until
 * max_r ||r_r||_2 / ||b_r||_2 <= tol or max_it corrections were applied.
 * elem_mats, b, x as above; its (host, may be NULL) receives the number of corrections and
 * relres (host, may be NULL) the final relative residual.  Synchronizes hip_stream once per
 * iteration.  Errors: MF_ENOCONV (tolerance not met; x holds the last iterate), MF_ESTATE,
 * MF_EINVAL, MF_ENOMEM, MF_EHIP. */
int mf_refine(mf_plan *plan, const double *elem_mats, const double *b, double *x,
              int32_t nrhs, double tol, int32_t max_it, int32_t *its, double *relres,
              void *hip_stream);

/* Refinement by GMRES in FP64, preconditioned by the stored factors (GMRES-IR): x = solve(b);
 * then restarted cycles of right-preconditioned GMRES on A x = b (one Krylov basis of at most
 * `restart` vectors per right-hand side, classical Gram-Schmidt applied twice, Givens
 * rotations on the host), each Arnoldi step one solve with the stored factors and one
 * element-by-element FP64 product with A; every cycle ends with the true FP64 residual, and the
 * iteration stops once max_r ||b_r - A x_r||_2 / ||b_r||_2 <= tol.  For factors whose Schur
 * updates ran in BF16 or FP32 (mf_factor with MF_SCHUR_BF16 / MF_SCHUR_FP32), where plain
 * refinement (mf_refine) converges slowly.  max_it bounds the Arnoldi steps; its (host, may be
 * NULL) receives the steps taken, relres (host, may be NULL) the final relative residual.
 * elem_mats, b, x as in mf_refine (b and x must not alias).  Synchronizes hip_stream several
 * times per step.  Errors: MF_ENOCONV (x holds the last iterate), MF_ESTATE, MF_EINVAL
 * (restart outside 1..64), MF_ENOMEM, MF_EHIP. */
int mf_refine_gmres(mf_plan *plan, const double *elem_mats, const double *b, double *x,
                    int32_t nrhs, double tol, int32_t max_it, int32_t restart, int32_t *its,
                    double *relres, void *hip_stream);

/* mf_factor followed by mf_refine in one call, with the forward substitution of the first
 * solve overlapped with the factorization: class l of the forward sweep depends only on classes
 * <= l of the factorization (the elimination tree orders it, Sec. 2.4 / Sec. 3.3), so it runs
 * on a second stream of the plan while the upper classes are still being factored; the
 * backward sweep and the refinement loop follow on hip_stream.  The same kernels in the same
 * per-class order as mf_factor then mf_refine, so x and the factors are identical to theirs.
 * Launched eagerly (not as a captured graph), so that the two streams overlap.
 * Arguments and errors: those of mf_factor and mf_refine (MF_EZERO_PIVOT leaves no valid
 * factor and x unspecified).  Synchronizes hip_stream at least twice. */
int mf_factor_refine(mf_plan *plan, const double *elem_mats, int32_t precision, const double *b,
                     double *x, int32_t nrhs, double tol, int32_t max_it, int32_t *its,
                     double *relres, void *hip_stream);

/* Adjoint element gradient: gK[e][a][b] = -sum_r lam[conn_e[a]][r] * u[conn_e[b]][r], the
 * derivative of a loss through A = sum_e P_e^T K_e P_e given lam = A^{-T} dL/du.
 * lam, u device [n][nrhs]; gK device [n_elem][npe][npe].  Asynchronous. */
int mf_elem_grad(mf_plan *plan, const double *lam, const double *u, int32_t nrhs,
                 double *gK, void *hip_stream);

/* Copies the factors of every front (Table 2's compute_front: the division tasks scale the
 * pivot row, so U is unit upper and L carries the pivots, Sec. 3) to host buffers sized from
 * mf_info, front after front in id order:
 *   L: for each front an m x k row-major block, L[i][p] for i >= p (pivots on the diagonal),
 *      zeros above;
 *   U: for each front a k x m row-major block, U[p][p] = 1, U[p][j] for j > p, zeros left.
 * Synchronous.  Errors: MF_ESTATE (no valid factor), MF_EINVAL, MF_EHIP. */
int mf_export_factors(const mf_plan *plan, double *L, double *U);

/* Per-launch timing (tracing).  enable = 1 clears the counters and starts bracketing every
 * kernel launch the plan issues with HIP events on the launch stream (captured graphs are not
 * used while it is on); enable = 0 stops it.  Errors: MF_EINVAL. */
int mf_profile(mf_plan *plan, int32_t enable);

/* Writes a NUL-terminated JSON summary of the timed launches into buf (cap bytes, may be
 * NULL): {"kernels": [{"name", "launches", "ms" (summed event time), "bytes", "flops"}]},
 * where bytes and flops are the algorithmic HBM traffic and operation count of those launches.
 * needed (may be NULL) receives the size required.  Waits for the recorded events.
 * Errors: MF_EINVAL, MF_EHIP. */
int mf_profile_report(mf_plan *plan, char *buf, int64_t cap, int64_t *needed);

/* Releases the plan and all its device memory (NULL is ignored). */
void mf_destroy(mf_plan *plan);

/* Message of the last failed call on this thread ("" if none). */
const char *mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
