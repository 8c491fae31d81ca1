/*
 * trid.h -- C ABI of the MI355X (gfx950) batched tridiagonal solver library.
 *
 * The operation is the one posed in arxiv 2201.03950 ("High Throughput
 * Multidimensional Tridiagonal Systems Solvers on FPGAs"):
 *   - eqs. (1)-(2): a_i u_{i-1} + b_i u_i + c_i u_{i+1} = d_i, i = 0..N-1, with
 *     a_0 = c_{N-1} = 0;
 *   - Section II-B: many such systems lie along the x, y or z lines of a 2D/3D
 *     mesh whose coefficients are given per grid point, stored column-major
 *     (x contiguous); the systems along one axis are solved together;
 *   - Section III: batched Thomas (Alg. 1) per line, and for long or contiguous
 *     lines the tiled modified Thomas of eq. (7) whose reduced system is solved
 *     by PCR (Alg. 2) -- the "Thomas-PCR" hybrid;
 *   - Section IV-A, Alg. 3: the ADI heat-diffusion step, whose right-hand side
 *     comes from an explicit stencil and whose coefficients are generated
 *     inside the solver (the Tridslv(x-dim / y-dim / z-dim) calls).
 *
 * Conventions shared by every entry point
 *   Mesh:     `ndim` in 1..3 extents `dims[0..ndim)`, dims[0] fastest, and
 *             `batch` independent meshes stored one after another (batch
 *             outermost).  Point (i, j, k) of mesh m is element
 *             ((m*nz + k)*ny + j)*nx + i.  Lines of axis `axis` have length
 *             dims[axis] and element stride prod(dims[0..axis)).
 *   Memory:   every data pointer is a DEVICE pointer owned by the caller; the
 *             library never frees or retains it past the call.  `dims` and
 *             `offsets_host` are HOST pointers read during the call.
 *   Rows:     a at the first row and c at the last row of every line are
 *             ignored (treated as 0), as eq. (1) requires; their storage must
 *             still exist.  There is no pivoting and no singularity check
 *             (Alg. 1): the result is defined for diagonally dominant systems;
 *             otherwise inf/NaN propagate.
 *   Streams:  work is enqueued on the handle's stream (trid_set_stream;
 *             default: the null stream) and returns before it completes.
 *   Errors:   every call returns TRID_OK (0) or a TRID_ERR_* code and never
 *             throws or aborts.  Arguments are validated on the host before any
 *             HIP call; a failing call leaves its outputs untouched unless the
 *             failure is TRID_ERR_HIP from an already-launched kernel.
 *             trid_last_error() returns the text of the handle's last error.
 *   Threads:  one handle per host thread; a handle may be used with any
 *             stream of the device that was current when it was first used.
 *             A handle's calls share its workspace, work counters and
 *             schedules, so they never overlap: when trid_set_stream switches
 *             to another stream, work enqueued there afterwards waits for the
 *             work already enqueued on the previous stream (not across a graph
 *             capture: a caller capturing a graph keeps one stream per handle,
 *             or uses one handle per stream).
 *   Caches:   captured graphs and uneven-batch schedules are cached per handle
 *             and keyed on the device pointers; each cache keeps a bounded
 *             number of entries and evicts the least recently used one
 *             (trid_cache_report).
 */
#ifndef TRID_H
#define TRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct trid_handle_s *trid_handle_t;
typedef void *trid_stream_t; /* a hipStream_t; NULL is the null stream */

/* (the two sentinels give the enum the range of int, so an out-of-range
 * value a caller passes is still a value of the type, which the entry points
 * reject with TRID_ERR_ARG) */
typedef enum { TRID_F32 = 0, TRID_F64 = 1, TRID_DTYPE_MIN_ = -0x7fffffff - 1, TRID_DTYPE_MAX_ = 0x7fffffff } trid_dtype_t;

/* precision of a solve: plain FP64, plain FP32, or FP32 bulk solves with one
 * FP64 residual and refinement sweep */
typedef enum {
    TRID_PREC_F64 = 0,
    TRID_PREC_F32 = 1,
    TRID_PREC_F32_REFINE64 = 2,
    TRID_PREC_MIN_ = -0x7fffffff - 1, /* range sentinels, as for trid_dtype_t */
    TRID_PREC_MAX_ = 0x7fffffff
} trid_prec_t;

enum {
    TRID_OK = 0,
    TRID_ERR_ARG = 1,         /* invalid argument (null pointer, bad dims/axis/dtype, ...) */
    TRID_ERR_ALLOC = 2,       /* device or host allocation failed */
    TRID_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
    TRID_ERR_UNSUPPORTED = 4  /* valid but not supported (e.g. a line longer than the limit) */
};

/* flags of trid_adi_step */
#define TRID_ADI_GRAPH 1u /* capture the nsteps launches in a hipGraph once and replay it */
#define TRID_ADI_STREAM 2u /* 2D: always run the per-step kernels, never the LDS-resident loop */

/* Longest line a single-workgroup tile plan handles (rows). */
#define TRID_MAX_LINE 8192

/* Longest contiguous line (axis 0, i.e. the line is the fastest-varying
 * index) the batched solves accept: longer than TRID_MAX_LINE, such a line is
 * cut into chunks of 2048 rows, one workgroup each, coupled through a reduced
 * system of two rows per chunk (the tiling of Section III-B one level up). */
#define TRID_MAX_LONG_LINE 8388608

/* ---------------------------------------------------------------- handle -- */

/* Create a handle.  Allocates host memory only; device state (workspace,
 * graphs) is created on first use on the device current at that time.
 * Errors: TRID_ERR_ARG if h is NULL, TRID_ERR_ALLOC. */
int trid_create(trid_handle_t *h);

/* Destroy a handle: synchronises its stream, frees its workspace, plans and
 * graphs.  NULL is accepted (no-op). */
int trid_destroy(trid_handle_t h);

/* Select the stream later calls enqueue on (NULL = null stream).  If the
 * handle has enqueued work on the previous stream, the new stream is made to
 * wait for it (an event), unless either stream is capturing a graph.
 * Errors: TRID_ERR_ARG (NULL handle), TRID_ERR_HIP. */
int trid_set_stream(trid_handle_t h, trid_stream_t stream);

/* Text of the handle's last error ("" if none); valid until the next call on h.
 * With h == NULL, the text of the last trid_create failure. */
const char *trid_last_error(trid_handle_t h);

/* Library ABI version (major*10000 + minor*100 + patch). */
int trid_version(void);

/* Force the tile plan of later line solves on this handle: M rows per tile
 * (8, 16 or 32) and L lines per workgroup (a power of two); 0 restores the
 * automatic choice.  Every plan computes the same solution up to rounding
 * (Section III-B: the tile split only changes the reduced system); this knob
 * exists for tuning and for tests that vary the plan.
 * Errors: TRID_ERR_ARG for other values. */
int trid_set_tile(trid_handle_t h, int M, int L);

/* Per-kernel timing with HIP events (for measurement tools).  With on != 0,
 * every kernel this handle launches outside graph capture has its start and
 * end stamped into two events by its dispatch (work replayed from a graph,
 * such as an uneven batch with several launches, is bracketed by two events
 * recorded on the stream instead; an uneven batch of one persistent launch
 * then runs directly, not from its captured graph); on = 0 stops it.  Either
 * call first waits for pending events and clears the accumulated totals.
 * trid_timing_read waits for pending events, then writes NUL-terminated JSON
 * text {"kernel": [launch count, total milliseconds], ...} into buf (len bytes).
 * Errors: TRID_ERR_ARG (NULL handle or buffer, buffer too small), TRID_ERR_HIP. */
int trid_timing_enable(trid_handle_t h, int on);
int trid_timing_read(trid_handle_t h, char *buf, int64_t len);

/* Thin out the per-kernel timing: only launches named `name` (a name that
 * trid_timing_read reports, such as "adi_z_update"; NULL or "" = every name),
 * and of each timed name only every `every`-th launch (the first after this
 * call, then every `every`-th).  The other launches run without events, which
 * cost a few microseconds of dispatch time each; with name NULL and every = k,
 * a loop of steps is stamped in every k-th step.  (NULL, 1) times every launch
 * again.  Like trid_timing_enable, it first waits for pending events and
 * clears the totals; it does not switch timing on or off.
 * Errors: TRID_ERR_ARG (NULL handle, name over 200 characters, every < 1),
 * TRID_ERR_HIP. */
int trid_timing_select(trid_handle_t h, const char *name, int every);

/* ------------------------------------------------------- batched solves -- */

/* Solve every line of `axis` of `batch` meshes: A x = d with per-point
 * coefficient arrays a (sub), b (diagonal), c (super) of dtype dt, in the
 * mesh layout (eqs. (1)-(2), Section II-B).  d is IN/OUT: the right-hand side
 * on entry, the solution on return.  a, b, c are read only.
 * Lines of axis 0 may be up to TRID_MAX_LONG_LINE rows long; those longer
 * than TRID_MAX_LINE take the chunked solve (three launches, a workspace of
 * 10 * lines * ceil(n / 2048) values owned by the handle).
 * Errors: TRID_ERR_ARG (null pointer, ndim not in 1..3, axis not in
 * 0..ndim-1, a dim < 1, batch < 1, bad dtype), TRID_ERR_UNSUPPORTED (line
 * length > TRID_MAX_LINE along axis > 0, or > TRID_MAX_LONG_LINE), TRID_ERR_ALLOC,
 * TRID_ERR_HIP. */
int trid_gtsv_batched(trid_handle_t h, trid_dtype_t dt, const void *a, const void *b,
                      const void *c, void *d, int ndim, const int64_t *dims, int axis,
                      int64_t batch);

/* As trid_gtsv_batched with the same (a, b, c) on every row, generated inside
 * the kernel (the fused coefficient generation of Section IV-A); the scalars
 * are rounded to dt.  Only d is read and written. */
int trid_gtsv_batched_const(trid_handle_t h, trid_dtype_t dt, double a, double b, double c,
                            void *d, int ndim, const int64_t *dims, int axis, int64_t batch);

/* As trid_gtsv_batched with rows generated from a per-point array s (dtype dt):
 * a_i = c_i = -s_i, b_i = 1 + 2 s_i (the implicit diffusion operator of Alg. 3
 * with a spatially varying diffusion number). */
int trid_gtsv_batched_s(trid_handle_t h, trid_dtype_t dt, const void *s, void *d, int ndim,
                        const int64_t *dims, int axis, int64_t batch);

/* FP32 bulk solve with one FP64 refinement sweep: with A the matrix of the
 * FP32 coefficient arrays a, b, c (exactly representable, the matrix of
 * record), computes x32 = solve32(A, fp32(d)), r = d - A x32 in FP64,
 * delta = solve32(A, fp32(r)), x = x32 + delta in FP64.  d has dtype d_dt
 * (FP32 or FP64) and is read only; x (FP64) receives the result and may not
 * alias d.  Same layout and errors as trid_gtsv_batched; contiguous lines
 * longer than TRID_MAX_LINE run the refinement as passes around the chunked
 * FP32 solve (FP64 residual pass, FP32 correction solve, FP64 sum) with a
 * workspace of two FP32 mesh-sized arrays owned by the handle. */
int trid_gtsv_batched_refine(trid_handle_t h, trid_dtype_t d_dt, const float *a, const float *b,
                             const float *c, const void *d, double *x, int ndim,
                             const int64_t *dims, int axis, int64_t batch);

/* As trid_gtsv_batched_refine with rows a = c = -s, b = 1 + 2 s from FP32 s. */
int trid_gtsv_batched_s_refine(trid_handle_t h, trid_dtype_t d_dt, const float *s, const void *d,
                               double *x, int ndim, const int64_t *dims, int axis,
                               int64_t batch);

/* ------------------------------------------------------------ uneven batch -- */

/* `nsys` systems of different lengths packed back to back: system k occupies
 * rows [offsets[k], offsets[k+1]) of a, b, c, d and x (Section III-B's tiled
 * solver handles the long ones).  offsets_host is a HOST int64 array of
 * nsys+1 non-decreasing entries with offsets[0] = 0 and every length in
 * 1..TRID_MAX_LONG_LINE.  Systems of up to TRID_MAX_LINE rows are tiled inside
 * one workgroup; longer ones are cut into chunks of 2048 rows coupled through
 * a reduced system of two rows per chunk (the chunked solve of
 * trid_gtsv_batched, one system after the other after the persistent launch;
 * with F32_REFINE64 as passes: FP32 chunked solve, FP64 residual, FP32 chunked
 * correction solve, FP64 sum).  Precision p selects the arithmetic:
 *   TRID_PREC_F64:          a, b, c, d, x are double;
 *   TRID_PREC_F32:          a, b, c, d, x are float;
 *   TRID_PREC_F32_REFINE64: a, b, c are float, d and x are double.
 * d is read only; x receives the solution (x may equal d for F64 and F32).
 * All systems are solved by ONE persistent launch that pulls work items,
 * longest first, from a device counter.  The schedule (work list, tile plan
 * per length class) is built on the first call for a given offsets content
 * and cached in the handle; with the environment variable TRID_AUTOTUNE=1 the
 * tile plan is chosen by timing candidates on this call's data: the
 * TRID_AUTOTUNE_TOP (default 3; 0 = all) plans that the performance model
 * (its uneven-batch part: per work item, rows, tile sweep and reduced solve)
 * ranks fastest.  The timed runs write x, or, when x is d, a workspace array
 * of the handle, so an in-place solve still returns A^{-1} d.
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED, TRID_ERR_ALLOC, TRID_ERR_HIP. */
int trid_gtsv_varlen(trid_handle_t h, trid_prec_t p, const void *a, const void *b, const void *c,
                     const void *d, void *x, const int64_t *offsets_host, int64_t nsys);

/* As trid_gtsv_varlen with the offsets in DEVICE memory (int64[nsys + 1]).
 * The schedule is built on the host, so the call copies the offsets to the
 * host after the work already enqueued on the handle's stream and waits for
 * that copy (the call synchronises the stream once; it cannot be captured
 * into a graph).  Then as trid_gtsv_varlen.
 * Errors: as trid_gtsv_varlen. */
int trid_gtsv_varlen_dev(trid_handle_t h, trid_prec_t p, const void *a, const void *b, const void *c,
                         const void *d, void *x, const int64_t *offsets_dev, int64_t nsys);

/* ------------------------------------------------------------------- ADI -- */

/* `nsteps` ADI heat-diffusion steps (Alg. 3) in place on u, in the Douglas
 * delta form:  d = 2 s L u  (L: 7-point Laplacian in 3D, 5-point in 2D, zero
 * outside the mesh), then d <- X^{-1} d, d <- Y^{-1} d (, d <- Z^{-1} d) with
 * rows (-s, 1 + 2s, -s) along each axis, then u += d.  s is a per-point
 * array of dtype dt, or NULL for the constant s0.  ndim is 2 or 3.  One step
 * is three fused kernels in 3D (stencil + x solve; y solve; z solve + update)
 * and two in 2D.  The d workspace (one mesh-sized array) is owned by the
 * handle.  With TRID_ADI_GRAPH the launches of all nsteps are captured once
 * into a hipGraph keyed on (u, s, s0, dims, batch, nsteps, dt) and replayed.
 * 2D meshes of at most 128 points per line whose u, d (and s) fit one
 * workgroup's LDS run instead as ONE launch with each mesh resident in LDS
 * for all nsteps (u read and written once; the on-chip pipeline and unrolled
 * time loop of the 2D application, Section V); TRID_ADI_STREAM forces the
 * per-step kernels.  Both compute the same steps up to rounding.
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED, TRID_ERR_ALLOC, TRID_ERR_HIP. */
int trid_adi_step(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, double s0, int ndim,
                  const int64_t *dims, int64_t batch, int nsteps, unsigned flags);

/* Size of the device array that trid_adi_step_noalloc uses as its workspace
 * (one mesh-sized array of the step's dtype must fit). */
#define TRID_NOALLOC_SCRATCH_BYTES (64u << 20)

/* trid_adi_step for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same steps with the same kernels, but the d workspace is a statically sized
 * device array of TRID_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends, instead of the handle's allocated
 * workspace; the call makes no hipMalloc / hipFree and records no events.
 * Meshes whose d array (points x dtype size) exceeds that size are
 * TRID_ERR_UNSUPPORTED; 2D meshes that take the LDS-resident loop need no
 * workspace at all.  flags: 0 or TRID_ADI_STREAM (TRID_ADI_GRAPH is
 * TRID_ERR_ARG: instantiating a graph allocates; a caller may capture this
 * call into its own graph instead).  Every call on one GPU, from any handle or
 * thread, uses that GPU's one array: calls that overlap in time on one GPU
 * race and give wrong results; serialise them (one stream, or events).
 * Nothing in the array needs to start at zero: each step writes it before
 * reading it.  Errors: as trid_adi_step. */
int trid_adi_step_noalloc(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, double s0, int ndim,
                          const int64_t *dims, int64_t batch, int nsteps, unsigned flags);

/* `nsteps` Hundsdorfer-Verwer ADI steps of u_t = a u_xx + b u_yy + c u_xy in
 * place on u: the synthetic stand-in for the call structure of the SLV
 * application (Alg. 4, Section V): explicit predictor stencils alternating
 * with line solves along x and y.  u, a, b, c are device arrays of dtype dt
 * and shape (batch, ny, nx), x contiguous (dims = {nx, ny}); a, b, c are the
 * per-point coefficients (read only; u must not overlap them), with unit
 * spacing and zero values outside the mesh.
 * With F1 = a D_xx, F2 = b D_yy, F0 = c D_xy (D_xy the 4-point cross stencil
 * over 4) and F = F0 + F1 + F2, one step of size tau is
 *   Y0 = U + tau F(U)
 *   (I - theta tau A1) Y1 = Y0 - theta tau F1(U)
 *   (I - theta tau A2) Y2 = Y1 - theta tau F2(U)
 *   W0 = Y0 + tau/2 (F(Y2) - F(U))
 *   (I - theta tau A1) W1 = W0 - theta tau F1(Y2)
 *   (I - theta tau A2) U  = W1 - theta tau F2(Y2)
 * with A1 = a D_xx and A2 = b D_yy, so the implicit systems are the s form
 * (-s, 1 + 2 s, -s) with s = theta tau a (x lines) or theta tau b (y lines).
 * Meshes of at most 128 points per line whose three work arrays (u and two
 * stage arrays) fit one workgroup's LDS run all nsteps as ONE launch, each
 * mesh resident in LDS and every predictor fused into the line solve after
 * it (the fused on-chip modules of the SLV design, Section V); a, b, c are
 * read from memory as the phases need them.  Other meshes, or flags =
 * TRID_ADI_STREAM, take per-step kernels: four predictor launches and four
 * batched line solves per step, with four mesh-sized work arrays owned by
 * the handle.  Both compute the same steps up to rounding.  tau >= 0 and
 * theta > 0, both finite; nsteps >= 0 (0 is a no-op); lines up to
 * TRID_MAX_LINE rows along each axis; flags is 0 or TRID_ADI_STREAM.
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED, TRID_ERR_ALLOC, TRID_ERR_HIP. */
int trid_hv_step(trid_handle_t h, trid_dtype_t dt, void *u, const void *a, const void *b,
                 const void *c, double tau, double theta, const int64_t *dims, int64_t batch,
                 int nsteps, unsigned flags);

/* ------------------------------------------------------------- adjoints -- */

/* Reverse mode of x = A^{-1} d along `axis` (arrays form).  x is the forward
 * solution.  g is IN/OUT: dL/dx on entry, dL/dd = lambda = A^{-T} g on return.
 * ga, gb, gc (written, not accumulated) receive dL/da = -lambda_i x_{i-1},
 * dL/db = -lambda_i x_i, dL/dc = -lambda_i x_{i+1}; the entries of the ignored
 * a_0 and c_{N-1} are written as 0.  Same layout and errors as
 * trid_gtsv_batched; contiguous lines longer than TRID_MAX_LINE write the rows
 * of A^T into a handle workspace (three mesh-sized arrays) and take the
 * chunked solve, then the gradients pointwise. */
int trid_gtsv_batched_adjoint(trid_handle_t h, trid_dtype_t dt, const void *a, const void *b,
                              const void *c, const void *x, void *g, void *ga, void *gb, void *gc,
                              int ndim, const int64_t *dims, int axis, int64_t batch);

/* Reverse mode of x = A(s)^{-1} d with rows (-s, 1 + 2 s, -s): g IN/OUT as
 * above, and gs += lambda_i (x_{i-1} - 2 x_i + x_{i+1}) (zero outside the
 * line), i.e. dL/ds of this solve is ACCUMULATED into gs. */
int trid_gtsv_batched_s_adjoint(trid_handle_t h, trid_dtype_t dt, const void *s, const void *x,
                                void *g, void *gs, int ndim, const int64_t *dims, int axis,
                                int64_t batch);

/* One ADI step (trid_adi_step, one step, no graph) in reverse: given the
 * checkpoint u_t (the field before the step) and u_bar = dL/du_{t+1},
 * recomputes the step's intermediates from u_t, overwrites u_bar with
 * dL/du_t and ACCUMULATES dL/ds of this step into s_bar.  s is the per-point
 * diffusion number (dtype dt), or NULL for the constant s0 (finite); with a
 * constant s0, s_bar receives the per-point derivative dL/ds_i at s = s0
 * everywhere, whose sum over the mesh is dL/ds0.  s_bar may be NULL when the
 * s gradient is not wanted.  Workspace is owned by the handle.
 * Errors: TRID_ERR_ARG (NULL u_t or u_bar, ndim not 2 or 3, non-finite s0,
 * ...), TRID_ERR_UNSUPPORTED, TRID_ERR_ALLOC, TRID_ERR_HIP. */
int trid_adi_step_adjoint(trid_handle_t h, trid_dtype_t dt, const void *u_t, const void *s, double s0,
                          void *u_bar, void *s_bar, int ndim, const int64_t *dims, int64_t batch);

/* One ADI step with per-point s (as trid_adi_step, one step, no graph) that
 * KEEPS its intermediates for the reverse pass instead of discarding them:
 *   w1 = X^{-1} (2 s L u),  w2 = Y^{-1} w1,  (3D) w3 = Z^{-1} w2,
 * then u += w3 (3D) or u += w2 (2D) (Alg. 3, Douglas delta form).  w1, w2, w3
 * are caller-owned device arrays of the mesh's size and type, distinct from u
 * and from each other; w3 is ignored (may be NULL) in 2D.  The kept step costs
 * one extra mesh-sized write (the last solve also stores its solution) and
 * lets trid_adi_step_adjoint_kept skip the recomputation.  Errors as
 * trid_adi_step; aliasing arrays are TRID_ERR_ARG. */
int trid_adi_step_keep(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, int ndim,
                       const int64_t *dims, int64_t batch, void *w1, void *w2, void *w3);

/* Reverse of one kept step: as trid_adi_step_adjoint, with the intermediates
 * w1, w2, (3D) w3 written by trid_adi_step_keep for the step that started from
 * u_t, so nothing is recomputed.  u_bar is overwritten with dL/du_t; dL/ds is
 * ACCUMULATED into s_bar.  Workspace (one mesh-sized array) is owned by the
 * handle. */
int trid_adi_step_adjoint_kept(trid_handle_t h, trid_dtype_t dt, const void *u_t, const void *s,
                               const void *w1, const void *w2, const void *w3, void *u_bar,
                               void *s_bar, int ndim, const int64_t *dims, int64_t batch);

/* ----------------------------------------------------- performance model -- */

#define TRID_FORM_ARRAYS 0 /* rows from per-point a, b, c (trid_gtsv_batched) */
#define TRID_FORM_S 1      /* rows (-s, 1 + 2 s, -s) (trid_gtsv_batched_s) */

/* Predicted kernel duration, in microseconds, of the batched solve that
 * trid_gtsv_batched (form TRID_FORM_ARRAYS) or trid_gtsv_batched_s
 * (TRID_FORM_S) would launch for this geometry, with the tile plan it would
 * choose (honouring trid_set_tile).  The model is the GPU counterpart of the
 * paper's analytic latency model (Section III's per-call clock-cycle counts,
 * applied to the applications in Section IV, which reports its predictions
 * within 15% of measured runtimes): a fixed
 * launch cost plus the larger of (bytes moved / streaming bandwidth of the
 * access pattern) and (workgroup rounds x one workgroup's memory round trips,
 * tile sweep and reduced-solve levels).  If json is not NULL, up to len bytes
 * of a JSON object describing the plan and the model's terms are written.
 * Host computation only (no HIP call, no GPU needed).  Lines longer than
 * TRID_MAX_LINE are TRID_ERR_UNSUPPORTED.
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED. */
int trid_model_gtsv(trid_handle_t h, trid_dtype_t dt, int form, int ndim, const int64_t *dims,
                    int axis, int64_t batch, double *us, char *json, size_t len);

/* Predicted GPU time, in microseconds, of trid_adi_step (Alg. 3; dims, batch,
 * dtype and flags as there, per_point_s != 0 for a per-point s array) over
 * nsteps steps: the sum over the call's kernels of the model of
 * trid_model_gtsv, extended to the fused stencil + x kernels and the
 * constant-row line kernels (bytes over the streaming rate of the kernel's
 * class, or its workgroup rounds times a per-round latency, whichever is
 * larger) and to the LDS-resident 2D time loop (rounds of meshes times a load
 * and store cost plus each step's points over the workgroup's threads) -- the
 * counterpart of the paper's per-application predictions (Section IV-A,
 * applied there to the ADI solver).  Only TRID_ADI_STREAM of flags changes the
 * prediction (graph replay changes launch overhead, not kernel time).  If json
 * is not NULL, up to len bytes of {"us": total, "kernels": [{"name", "class",
 * "us", "launches", "bytes", "rounds", "units"}, ...]} are written (units: a
 * resident loop's mesh points per thread and step), kernel names as
 * trid_timing_read reports them.  Host computation only (no HIP call).
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED (no kernel plan for the mesh). */
int trid_model_adi(trid_handle_t h, trid_dtype_t dt, int ndim, const int64_t *dims, int64_t batch, int per_point_s,
                   int nsteps, unsigned flags, double *us, char *json, size_t len);

/* The same prediction for trid_hv_step (the SLV stand-in of Alg. 4's call
 * structure, Section IV-B): the resident loop, or per step four predictor
 * stencils and four s-form line solves (with TRID_ADI_STREAM, or when the mesh
 * does not fit one workgroup's LDS).  dims = {nx, ny}.  json as for
 * trid_model_adi.  Host computation only.
 * Errors: TRID_ERR_ARG, TRID_ERR_UNSUPPORTED. */
int trid_model_hv(trid_handle_t h, trid_dtype_t dt, const int64_t *dims, int64_t batch, int nsteps, unsigned flags,
                  double *us, char *json, size_t len);

/* The most recent autotuning run of trid_gtsv_varlen (TRID_AUTOTUNE=1) as a
 * JSON array, best predicted first: per plan its tile rows M, tiles per work
 * item NT, reduced solve ("pcr" / "thomas"), split flag, the persistent
 * workgroups of its launch (blocks; blocks_small for the short systems of a
 * split plan), the model's predicted time pred_us and the measured time
 * meas_us (-1 for plans the tuner did not time).  With TRID_AUTOTUNE_TOP=k
 * (default 3) the tuner times only the k plans the model ranks best; k = 0
 * times every plan.  An empty array if no tuning has run.
 * Errors: TRID_ERR_ARG (NULL buffer or too small). */
int trid_autotune_report(trid_handle_t h, char *buf, size_t len);

/* The handle's caches as JSON text: {"adi_graphs": n, "adi_graph_cap": n,
 * "varlen_schedules": n, "varlen_schedule_cap": n, "varlen_graphs": n,
 * "varlen_graph_cap": n} -- captured ADI runs, uneven-batch schedules, and
 * captured uneven-batch launches (summed over schedules; the cap is per
 * schedule).  Host only.  Errors: TRID_ERR_ARG (NULL buffer or too small). */
int trid_cache_report(trid_handle_t h, char *buf, size_t len);

/* The LDS layout of the resident 2D loops (trid_adi_step on small 2D meshes,
 * hv != 0: trid_hv_step) for meshes of nx x ny points: out[0..9] = tile rows
 * M, tiles per x line, tiles per y line, row pitch, skew added per block of M
 * rows, pad element after every M points of a row (0/1), elements per array,
 * HV coefficient arrays staged in LDS (0: none, 1: b, 2: a, b, c), threads
 * per workgroup, LDS bytes per workgroup.  Point (y, x) of every array sits at
 * y * pitch + (y / M) * skew + x + pad * (x / M) of that array; the arrays
 * follow one another (u, then d (, s) or the HV stage arrays).  force_M = 0
 * gives the automatic tile size; 8, 10, 12 or 14 forces one.  Host only (a
 * layout query for tests and tools).  Errors: TRID_ERR_ARG (NULL out, len <
 * 10, bad dtype or tile size), TRID_ERR_UNSUPPORTED (no layout fits). */
int trid_resident_layout(trid_handle_t h, trid_dtype_t dt, int64_t nx, int64_t ny, int hv, int per_point_s,
                         int force_M, int64_t *out, int len);

/* ------------------------------------------------------------ plan cache -- */

/* Load / save the tile-plan cache (JSON text: one entry per tuned key, each
 * with the gfx architecture it was tuned on).  Unknown keys are ignored on
 * load; a missing file on load is TRID_ERR_ARG.  With the environment variable
 * TRID_PLAN_CACHE set to a path, trid_create loads that file when it exists and
 * trid_destroy writes the handle's plans back to it.
 *
 * Testing aid: with TRID_FAIL_ALLOC set, every workspace allocation of the
 * library fails with TRID_ERR_ALLOC before any HIP call. */
int trid_plan_load(trid_handle_t h, const char *path);
int trid_plan_save(trid_handle_t h, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* TRID_H */
