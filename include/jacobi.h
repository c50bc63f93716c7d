/*
 * jacobi.h -- C ABI of the MI355X (gfx950) over-decomposed Jacobi library.
 *
 * The library runs the data-parallel core of the Jacobi3D proxy application
 * of the paper (Section 4.3, Proxy Application: Jacobi3D): a synchronous
 * 5-point (2D) or 7-point (3D) Jacobi sweep over a grid that is
 * over-decomposed (Section 4.4, Over-decomposition) into many cuboid blocks,
 * each stored with a one-cell face halo that is refreshed from the neighbour
 * blocks, plus an FP64 L2 residual taken every few sweeps.
 *
 * Problem (the paper names the Jacobi method only; this is the reading used):
 *   -Laplace(u) = f on the unit square/cube, Dirichlet values on the ring of
 *   nodes around the interior, h = 1/(n+1), b = h^2 f.
 *   2D update   u'[c] = ((u[W] + u[E]) + (u[S] + u[N]) + b[c]) * 1/4
 *   3D update   u'[c] = (((u[W] + u[E]) + (u[S] + u[N])) + (u[B] + u[F]) + b[c]) * fl(1/6)
 *   evaluated exactly in this order, IEEE round-to-nearest, no FMA, no flush
 *   to zero; Laplace (no source) drops "+ b[c]".  The ring never changes.
 *   residual    sqrt(sum over the interior of (b - (2d u - s))^2), all in FP64
 *               from the state widened to FP64 (s = the neighbour sum above).
 *
 * Arrays crossing the boundary (all device pointers unless noted):
 *   full state  (n_x+2)(n_y+2)[(n_z+2)] values of the handle's dtype, x
 *               fastest, ring included: node (i, j[, k]) at
 *               ((k * (n_y+2)) + j) * (n_x+2) + i, with 0 and n+1 the ring.
 *   source f    n_x n_y [n_z] interior values of the handle's dtype, x fastest.
 *
 * Memory and streams: the library never allocates device memory.  The caller
 * supplies one device workspace of jacobi_workspace_bytes() bytes (typically a
 * torch tensor) that holds both state buffers, the blocked source and the
 * reduction scratch; it must stay allocated until jacobi_destroy returns.
 * Every operation is enqueued on the handle's HIP stream in call order and is
 * asynchronous unless documented otherwise; input/output pointers must stay
 * valid until the stream reaches the operation.
 *
 * Errors: every function returns JACOBI_OK (0) or a negative status and never
 * throws.  Argument checks run before any HIP call.  The text of the last
 * error on the calling thread is available from jacobi_last_error().
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jacobi_s *jacobi_t; /* opaque handle (host object) */

enum jacobi_dtype { JACOBI_F32 = 0, JACOBI_F64 = 1 };

enum jacobi_status {
    JACOBI_OK = 0,
    JACOBI_E_INVAL = -1,       /* bad argument (sizes, pointers, dtype, ranges)   */
    JACOBI_E_NOMEM = -2,       /* workspace too small or host allocation failed    */
    JACOBI_E_HIP = -3,         /* a HIP runtime call failed (text in last_error)   */
    JACOBI_E_STATE = -4,       /* call not valid in the handle's state             */
    JACOBI_E_UNSUPPORTED = -5  /* valid request this build does not implement      */
};

/* Tuning flags for jacobi_set_tuning. */
enum jacobi_flags {
    /* Sweep each block from its own storage after an explicit halo exchange
     * before every sweep (pack -> copy -> unpack between blocks in HBM), the
     * step order of Section 4.3.  Temporal depth is forced to 1.  Without the
     * flag the sweep reads face neighbours' cells directly from their blocks
     * (the exchange fused into the sweep's loads) and may do several sweeps
     * per pass. */
    JACOBI_FLAG_EXPLICIT_HALO = 1,
    /* Store pass outputs with the non-temporal hint (not kept in the caches).
     * A pure performance choice; results are identical either way. */
    JACOBI_FLAG_NT_STORES = 2,
    /* Accepted and ignored: the 2D passes now choose how far ahead they load
     * by their depth (two rows at depths up to 13, one row beyond and in the
     * adjoint pass).  Kept so that callers that set it keep working. */
    JACOBI_FLAG_DEEP_PREFETCH = 4,
    /* With JACOBI_FLAG_EXPLICIT_HALO (required): cut the blocks into up to 4
     * slabs of block layers along the slowest axis and overlap each slab's
     * face sends (on a second stream the library owns, default priority)
     * with the sweep of the next slab -- the over-decomposition of Section
     * 4.4, one piece's halo transfer hidden under another piece's kernel.
     * Results are identical to the explicit-halo schedule. */
    JACOBI_FLAG_OVERLAP = 8
};

/* ---------------------------------------------------------------- set-up */

/* Device bytes the handle needs for this problem.
 * Implements: the decomposition of the domain into cuboid blocks (Section
 * 4.3, and more blocks than processing elements in Section 4.4); the sizes
 * and the 32-byte x granularity are this library's choice.
 *   ndim    2 or 3
 *   grid    interior nodes per axis, x first (ndim values, each >= 1)
 *   blocks  blocks per axis, x first (ndim values, 1 <= blocks <= grid);
 *           the block extent along x is ceil(n/B) rounded up to 32 bytes of
 *           elements, along y and z ceil(n/B); the last block on an axis takes
 *           the remainder and must not be empty (JACOBI_E_INVAL otherwise).
 *   dtype   JACOBI_F32 or JACOBI_F64 (arithmetic and storage type of the sweep)
 *   bytes   out: workspace size.  JACOBI_E_INVAL on overflow. */
int jacobi_workspace_bytes(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                           size_t *bytes);

/* Implements: Section 4.3's cuboid decomposition, as block storage in one
 * device workspace.
 * Create a handle over a caller-owned device workspace (256-byte aligned,
 * >= jacobi_workspace_bytes).  stream: hipStream_t to enqueue on, or NULL for
 * the null stream.  The handle starts without a state (JACOBI_E_STATE from
 * sweep/residual until jacobi_set_state) and without a source (Laplace). */
int jacobi_create(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                  void *workspace, size_t workspace_bytes, void *stream, jacobi_t *out);

/* Implements: Section 4.3's per-iteration face exchange between cuboids and
 * Section 4.4's over-decomposition in their communication-avoiding form
 * (deep-halo block storage; the exchange pattern is the paper's, its depth
 * this library's choice).  Every block stores a frame of H nodes around its
 * interior (faces, edges and corners); each pass first refreshes every
 * frame from the blocks owning those nodes (one exchange launch), then runs
 * up to H sweeps of every block from that block's own storage alone (one
 * launch over all blocks), so blocks exchange data once per H sweeps.
 *   ndim, grid, blocks, dtype  as for jacobi_workspace_bytes
 *   halo    requested frame depth H, 1 <= H <= 64; it is stored rounded up
 *           to the next value with (H - 1) a multiple of 16 bytes of
 *           elements (FP32: 1, 5, 9, 13, ...; FP64: 1, 3, 5, ...; see
 *           jacobi_get_halo), which must not exceed the extent of any block
 *           on an axis with more than one block (JACOBI_E_INVAL otherwise)
 *   bytes   out: workspace size.  JACOBI_E_INVAL on overflow. */
int jacobi_deep_workspace_bytes(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                                int halo, size_t *bytes);

/* Implements: as jacobi_deep_workspace_bytes.  Create a handle over a
 * caller-owned workspace of jacobi_deep_workspace_bytes bytes (256-byte
 * aligned, device memory).  The handle supports every call a jacobi_create
 * handle does, with identical results (bit for bit); jacobi_sweep and
 * jacobi_solve run deep-halo passes of up to min(t_depth, stored H) sweeps
 * (the residual, when asked for, is a pass of its own), and
 * JACOBI_FLAG_EXPLICIT_HALO still selects the one-cell exchange before every
 * sweep. */
int jacobi_deep_create(int ndim, const int64_t *grid, const int64_t *blocks, int dtype, int halo,
                       void *workspace, size_t workspace_bytes, void *stream, jacobi_t *out);

/* Not in the paper (a query).  Stored frame depth of a deep-halo handle, 0
 * for a jacobi_create handle.  JACOBI_E_INVAL for a NULL pointer. */
int jacobi_get_halo(jacobi_t h, int *halo);

/* Library plumbing (no passage).  Wait for the handle's stream, then free
 * the host object.  NULL is a no-op.  The workspace stays the caller's. */
int jacobi_destroy(jacobi_t h);

/* Library plumbing (no passage).  Rebind the handle to another stream
 * (hipStream_t; NULL = null stream); later calls enqueue there. */
int jacobi_set_stream(jacobi_t h, void *stream);

/* Implements: Section 4.3's cuboid blocks, reported.  Block geometry per
 * axis x first: blocks and block extent (3 host int64 values each, unused
 * axes 1).  JACOBI_E_INVAL if either pointer is NULL. */
int jacobi_get_layout(jacobi_t h, int64_t *blocks3, int64_t *extent3);

/* ------------------------------------------------------- data in and out */

/* Implements: Section 4.3, the domain decomposed into cuboids, each with its
 * face halos.  Scatter a full state (ring + interior, layout above) into the
 * blocks of both state buffers and fill every block's halo.  u: device,
 * handle dtype, read when the stream reaches the call.  JACOBI_E_INVAL if u
 * is NULL. */
int jacobi_set_state(jacobi_t h, const void *u);

/* Implements: the inverse of the Section 4.3 decomposition.  Gather the
 * current state (ring + interior) into u (device, handle dtype, caller-owned).
 * JACOBI_E_STATE before jacobi_set_state. */
int jacobi_get_state(jacobi_t h, void *u);

/* Not in the paper (its proxy states no equation): the right-hand side of
 * the Poisson reading -Laplace(u) = f.
 * Set the scaled source b = fl_T(h2 * f) blockwise, with the product formed in
 * FP64 and rounded once to the handle dtype T.  f: device interior array of
 * the handle dtype, or NULL for the Laplace equation (b = 0).  h2 > 0, finite. */
int jacobi_set_source(jacobi_t h, const void *f, double h2);

/* ------------------------------------------------------------- hot path */

/* Implements: Section 4.3, packing each block's face data, moving it to the
 * face neighbour and unpacking it into that block's halo (in HBM here).
 * Refresh every internal face halo of the current state buffer from the face
 * neighbour's edge cells (pack, copy, unpack in HBM; one launch for all faces
 * of all blocks).  Domain-edge halos keep the boundary values.  Idempotent. */
int jacobi_halo_exchange(jacobi_t h);

/* Implements: Section 4.3, the Jacobi update run for a fixed number of
 * iterations once the halos are in (the exchange is fused into the pass
 * kernels' loads, or run explicitly with JACOBI_FLAG_EXPLICIT_HALO).
 * Run n_iter >= 0 synchronous sweeps (0 is a no-op).  The sweeps are grouped
 * into passes of up to the tuned temporal depth; every pass reads the current
 * buffer and writes the other.  Halos are valid when the last pass ends. */
int jacobi_sweep(jacobi_t h, int64_t n_iter);

/* Not in the paper (its proxy runs a fixed iteration count): the FP64 L2
 * residual of the Poisson reading, the step whose cancellation needs FP64.
 * FP64 residual of the current state, written to the device double *res_dev
 * (stream-ordered, no synchronisation, deterministic summation order). */
int jacobi_residual_async(jacobi_t h, double *res_dev);

/* Not in the paper (as jacobi_residual_async).  Same value, copied to the
 * host double *res_host; synchronises the stream. */
int jacobi_residual(jacobi_t h, double *res_host);

/* Implements: Section 4.3's iteration loop, with the residual check (not in
 * the paper) every R sweeps.
 * Sweep n_iter times, taking the residual of the states after 0, R, 2R, ...
 * sweeps and after the last sweep: res_dev receives
 * ceil(n_iter / R) + 1 device doubles (R = check_every >= 1).  Stream-ordered,
 * no host synchronisation. */
int jacobi_solve(jacobi_t h, int64_t n_iter, int64_t check_every, double *res_dev);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as jacobi_create over a workspace, then jacobi_set_source(f, h2),
 * jacobi_set_state(u0), jacobi_solve(n_iter, check_every, res_dev) and
 * jacobi_get_state(u_out), with the library's default schedule, but without
 * a handle or a workspace: the library's own device scratch array (a fixed
 * JACOBI_NOALLOC_MAX_BYTES bytes per GPU, reserved when the library first
 * runs on that GPU and held until the process ends) stands in for the
 * workspace.  Allocates nothing (no hipMalloc, hipFree or allocating library
 * call); the first call on a device looks up that device's copy of the array.
 *   ndim, grid, blocks, dtype  as for jacobi_workspace_bytes; a problem whose
 *           workspace would exceed JACOBI_NOALLOC_MAX_BYTES is refused with
 *           JACOBI_E_NOMEM (about 2048^2 FP32 in 4x4 blocks fits)
 *   u0      device full state (ring + interior), handle-dtype layout above
 *   f, h2   device interior source and h^2 (f NULL: Laplace, h2 ignored)
 *   u_out   device full state receiving u after n_iter sweeps (may be u0)
 *   res_dev ceil(n_iter / check_every) + 1 device doubles, as jacobi_solve
 *   stream  hipStream_t or NULL; asynchronous, stream-ordered.
 * Results are bit-identical to the handle path with the same blocks.  Every
 * call on a GPU uses that GPU's one scratch array: calls that overlap on one
 * GPU (two streams or two threads) race and give wrong results; the array
 * keeps the last call's contents, which no later call reads before writing. */
#define JACOBI_NOALLOC_MAX_BYTES (64u << 20)
int jacobi_solve_noalloc(int ndim, const int64_t *grid, const int64_t *blocks, int dtype,
                         const void *u0, const void *f, double h2, int64_t n_iter,
                         int64_t check_every, void *u_out, double *res_dev, void *stream);

/* Not in the paper (performance only; Section 4.4's over-decomposition is
 * the JACOBI_FLAG_OVERLAP schedule).  The paper's interface has no knobs;
 * the three here are the ones the kernels have: depth (sweeps per pass),
 * rows (the tile height of the 2D pass / z segment of the 3D pass, which
 * fixes the tile width too) and flags (schedule forms).  Tile width is not a
 * separate knob: a lane handles 16 bytes of a row and a wave 64 lanes.
 * Choose the sweep schedule.  t_depth: sweeps per pass (temporal blocking,
 * 1..jacobi_max_depth(); 0 = library default; a depth without a compiled
 * kernel is run as passes of the nearest smaller compiled depths).
 * rows (0 = default): rows per interior tile of the 2D pass (>= 8; tiles
 * that reach the grid's boundary ring get fewer rows, derived from this
 * height, because they run a slower edge step), z planes per work item of
 * the 3D pass (>= 8), or, with JACOBI_FLAG_EXPLICIT_HALO on a 2D grid, rows
 * per work item of the block-local sweep (>= 1).
 * flags: jacobi_flags.  JACOBI_E_INVAL for values out of range.
 * Bit-neutral: every choice gives the same results. */
int jacobi_set_tuning(jacobi_t h, int t_depth, int rows, int flags);
int jacobi_get_tuning(jacobi_t h, int *t_depth, int *rows, int *flags);

/* Not in the paper.  Largest temporal depth this build supports for the
 * ndim/dtype (JACOBI_E_INVAL for unknown ones). */
int jacobi_max_depth(int ndim, int dtype);

/* --------------------------------------------------------------- batched */
/*
 * Not in the paper: the batched form of the method (the paper runs one
 * domain).  Each grid is decomposed and swept as in Section 4.3.
 * Many independent 2D Poisson grids of uneven sizes solved together: every
 * pass is one launch over the tiles of all grids that are still active, the
 * FP64 residual of each grid is folded into the first pass of each check
 * interval, and the relative-residual stop test runs on the GPU, so one
 * interval (its passes, counters and tests) is captured once as a hipGraph
 * and replayed.  Stop rule per grid (a reading; the paper runs a fixed
 * iteration count): residuals are checked on the states after 0, R, 2R, ...
 * sweeps and after max_sweeps; a grid stops, converged, at the first checked
 * k > 0 with res_k / res_0 <= rel_tol, converged at 0 sweeps if res_0 == 0,
 * diverged if a residual is not finite, otherwise at max_sweeps.  A stopped
 * grid keeps the state it was checked on.
 */
typedef struct jacobi_batch_s *jacobi_batch_t; /* opaque handle */

enum jacobi_batch_status {
    JACOBI_RUNNING = 0,
    JACOBI_CONVERGED = 1,
    JACOBI_MAX_SWEEPS = 2,
    JACOBI_DIVERGED = 3
};

/* Batched form (not in the paper); Section 4.3's decomposition per grid.
 * Workspace for `count` grids; grids: count pairs (n_x, n_y) of interior
 * sizes (host array); block: target block side (>= 8; blocks per axis =
 * ceil(n / block), reduced if the last block would be empty).  dtype as for
 * jacobi_create. */
int jacobi_batch_workspace_bytes(int count, const int64_t *grids, int64_t block, int dtype,
                                 size_t *bytes);

/* Batched form (not in the paper); Section 4.3's block storage per grid.
 * Create a batch over a caller-owned device workspace (256-byte aligned).
 * stream: hipStream_t; hipGraph capture needs a non-NULL stream (with NULL
 * the intervals are launched one kernel at a time). */
int jacobi_batch_create(int count, const int64_t *grids, int64_t block, int dtype,
                        void *workspace, size_t workspace_bytes, void *stream,
                        jacobi_batch_t *out);

/* Library plumbing.  Wait for the stream, release graphs and host memory.
 * NULL is a no-op. */
int jacobi_batch_destroy(jacobi_batch_t b);

/* Implements: Section 4.3's scatter into cuboids, per grid.  JACOBI_E_INVAL
 * for a bad index, NULL pointers or a bad h2.
 * Set grid i: u full state (ring + interior) and f interior source, both
 * device arrays of the batch dtype in the single-grid layout; b = fl(h2 f).
 * Every grid must be set before a solve. */
int jacobi_batch_set_grid(jacobi_batch_t b, int i, const void *u, const void *f, double h2);

/* Implements: the inverse of Section 4.3's decomposition, per grid.
 * JACOBI_E_STATE for a grid never set.  Gather grid i's final state (the state its stop test was taken on) into u. */
int jacobi_batch_get_grid(jacobi_batch_t b, int i, void *u);

/* Not in the paper (performance only).  Schedule: temporal depth (0 = default), tile rows (0 = default, else >= 8),
 * use_graph (replay captured check intervals). */
int jacobi_batch_set_tuning(jacobi_batch_t b, int t_depth, int rows, int use_graph);
int jacobi_batch_get_tuning(jacobi_batch_t b, int *t_depth, int *rows, int *use_graph);

/* Not in the paper (the batched form's autotuner).  Time candidate depths and
 * tile heights on one check interval of
 * check_every sweeps and keep the fastest (all are bit-identical).  Uses the
 * grids' buffers as scratch: every grid must be set again afterwards.
 * Synchronises the stream.  Outputs may be NULL. */
int jacobi_batch_autotune(jacobi_batch_t b, int64_t check_every, int *t_depth, int *rows);

/* Implements: Section 4.3's iteration loop over every grid at once, with the
 * stop rule above (not in the paper).  JACOBI_E_STATE if a grid is not set.
 * Solve every grid with the stop rule above.  Host outputs (count entries
 * each, may be NULL): sweeps of the final state, its relative residual, and
 * the jacobi_batch_status.  Synchronises the stream. */
int jacobi_batch_solve(jacobi_batch_t b, double rel_tol, int64_t max_sweeps, int64_t check_every,
                       int64_t *sweeps, double *rel, int *status);

/* --------------------------------------------------------------- adjoint */
/*
 * Not in the paper: the differentiable form of the Section 4.3 sweep.
 * Reverse-mode derivative through K 2D sweeps.  One sweep is the affine map
 * u_k = w (S u_{k-1} + B g + b), w = 1/4, with S the neighbour sum over the
 * interior (zero ring, symmetric) and B moving each ring value into its one
 * adjacent interior node.  Given lam_K = dL/du_K, the adjoint runs
 *     for k = K .. 1:  Gb += w lam_k;   lam_{k-1} = w S lam_k   (zero ring)
 * and yields dL/db = Gb, dL/df = h^2 Gb, dL/du_0 = lam_0 and, for each
 * non-corner ring node q, dL/dg_q = Gb[p(q)] (p(q) its adjacent interior
 * node; corners 0).  The lam sweep is the 5-point sweep with a zero ring and
 * no source; Gb is accumulated in FP64 in the order k = K, K-1, ..., 1.
 * 2D only (JACOBI_E_UNSUPPORTED for 3D handles).
 */

/* Forward K >= 0 sweeps from the current state (as jacobi_sweep), saving a
 * checkpoint every C >= 1 sweeps: ckpt (device, caller-owned, or NULL for
 * none) receives ceil(K / C) full states of the handle dtype back to back,
 * the states after 0, C, 2C, ... sweeps (k < K).  Afterwards the handle holds
 * u_K.  The checkpoints are restart points of the forward run; the adjoint
 * below does not read them (the sweep is affine, so the lam recurrence needs
 * no forward state).  JACOBI_E_STATE before jacobi_set_state. */
int jacobi_forward_ckpt(jacobi_t h, int64_t K, int64_t C, void *ckpt);

/* Gradients of a loss L(u_K) after K sweeps with respect to the source and
 * the whole initial state, in one call; the adjoint sweeps run in segments of
 * C >= 1 (any C gives the same bits).
 *   dL_duK  device full state of the handle dtype: dL/du_K at every node,
 *           ring included (the sweeps copy the ring, so the ring of u_K is
 *           g and its gradient passes to g unchanged)
 *   h2      h^2 > 0 of the forward run (b = h2 f)
 *   dL_df   device FP64 interior array (n_y x n_x, x fastest): dL/df.  Also
 *           the accumulator during the run.
 *   dL_dU0  device FP64 full array ((n_y+2) x (n_x+2)), distinct from
 *           dL_df: interior = dL/du_0 = lam_0; non-corner ring node q =
 *           dL_duK[q] + Gb[p(q)]; corner = dL_duK[corner].
 * Runs on the handle's stream, no synchronisation.  Uses the handle's state
 * buffers: afterwards the state is lam_0 with a zero ring.  2D only
 * (JACOBI_E_UNSUPPORTED otherwise); JACOBI_E_INVAL for NULL pointers, K < 0,
 * C < 1, a bad h2 or dL_df == dL_dU0. */
int jacobi_adjoint(jacobi_t h, int64_t K, int64_t C, const void *dL_duK, double h2,
                   double *dL_df, double *dL_dU0);

/* The same run in three calls, for callers that drive the segments
 * themselves.  Start an adjoint run: the handle's state becomes lam (device
 * full state array of the handle dtype whose interior holds dL/du_K; its
 * ring is read as zero), and grad_b (device FP64 interior array, n_y x n_x, x fastest,
 * caller-owned) is zeroed and becomes the accumulator.  grad_b must stay
 * valid until jacobi_adjoint_end. */
int jacobi_adjoint_begin(jacobi_t h, const void *lam, double *grad_b);

/* n_iter >= 0 adjoint sweeps (backward through n_iter forward sweeps),
 * grouped into passes like jacobi_sweep.  Segments may be issued in any
 * chunking (checkpointing): results do not depend on it.  Afterwards
 * jacobi_get_state returns lam with a zero ring. */
int jacobi_adjoint_sweep(jacobi_t h, int64_t n_iter);

/* Finish: grad_f (device FP64 interior array, may be NULL, may alias
 * grad_b) = h2 * grad_b; grad_ring (device FP64 full (n_y+2) x (n_x+2) array,
 * may be NULL) = the part of dL/dg that flows through the sweeps, Gb[p(q)],
 * on non-corner ring nodes, 0 on corners and interior.  A loss that also
 * reads the ring of u_K adds its gradient there itself (jacobi_adjoint
 * does). */
int jacobi_adjoint_end(jacobi_t h, double h2, double *grad_f, double *grad_ring);

/* ------------------------------------------------------------ profiling */

/* Not in the paper (measurement).  Start (enable != 0) or stop recording a pair of HIP events on the handle's
 * stream around every sweep-kernel launch (the pass kernels of jacobi_sweep
 * and jacobi_solve).  Enabling discards earlier records.  Recording adds no
 * device work besides the event markers. */
int jacobi_profile(jacobi_t h, int enable);

/* Not in the paper (measurement).  Summarise the records: launches of passes of `depth` sweeps (0 = all
 * launches).  Outputs: summed kernel time in milliseconds, number of
 * launches, cell updates performed (interior cells times sweeps) and
 * algorithmic HBM bytes (per pass: one read of the state and the source and
 * one write of the state per interior cell).  Synchronises the stream.  Any
 * output pointer may be NULL. */
int jacobi_profile_read(jacobi_t h, int depth, double *ms, int64_t *launches,
                        double *cell_updates, double *alg_bytes);

/* Not in the paper (performance only).  Pick the sweep schedule by timing.  Runs jacobi_sweep(n_sweeps) on the
 * handle's own buffers for each candidate temporal depth and tile height
 * (plus the explicit-halo schedule) and keeps the fastest; every candidate
 * computes identical results, so the choice never changes any output.
 * with_source: time the Poisson (1) or Laplace (0) kernels.  The buffers'
 * contents are used as scratch: the handle is left without a state
 * (JACOBI_E_STATE until jacobi_set_state).  Synchronises the stream.
 * If the environment variable JACOBI_TUNE_CACHE names a file, results are
 * looked up in and appended to it (one line per problem shape).
 * Outputs (may be NULL): the chosen depth, rows and flags. */
int jacobi_autotune(jacobi_t h, int64_t n_sweeps, int with_source, int *t_depth, int *rows,
                    int *flags);

/* --------------------------------------------------------------- errors */
/* Library plumbing.  Static text of a status; the last error's message on
 * the calling thread (valid until that thread's next failing call). */
const char *jacobi_strerror(int status);
const char *jacobi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_H */
