/*
 * lbm.h -- C ABI of the MinxEnt-LBM stream-and-collide library for AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the MinxEnt lattice Boltzmann method of T. L. Wilson,
 * M. Pugh and F. Dawson, "Stabilization of the Lattice Boltzmann Method Using
 * Information Theory" (arXiv:1801.03863): every fluid node replaces the BGK
 * relaxation by one Newton-Raphson step that minimises the Kullback-Leibler
 * divergence from the lattice weights subject to mass, momentum and relaxed
 * stress constraints (Sec. IV.C-D), followed by streaming (Sec. II.A).
 *
 * Conventions shared by every entry point
 *  - Return value: LBM_OK (0) or a negative error code (LBM_E*).  A failed
 *    call leaves no partial object behind; lbm_last_error() gives a message.
 *  - Host arrays of macroscopic fields are row-major [y][x] (x fastest), one
 *    double per node, nx*ny values (nx for D1Q3).  Batched calls take the
 *    instances' arrays concatenated in instance order.
 *  - D2Q9 populations are ordered rest, E, N, W, S, NE, NW, SW, SE: the
 *    column order of the moment matrix T of Sec. IV.D (Table I lists the
 *    same set with the rest velocity last).  D1Q3: rest, +1, -1.
 *  - Device memory handed in by the caller stays owned by the caller; the
 *    library never frees it.  A NULL workspace makes the library allocate
 *    (and later free) its own.
 *  - hip_stream is a hipStream_t passed as void*; NULL means the default
 *    stream.  All device work of a context is ordered on that stream.
 *  - A context is not thread-safe: calls on one context must not overlap.
 *  - Instability (a negative or non-finite post-collision population at a
 *    fluid node, Sec. IV.G) is not an error return: it sets a sticky status
 *    bit read by lbm_status(), so lbm_step() stays asynchronous.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2

/* Error codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)   /* bad argument or parameter combination */
#define LBM_ENOMEM (-2)   /* device or host allocation failed, or workspace too small */
#define LBM_EHIP (-3)     /* a HIP runtime call failed; see lbm_last_error() */
#define LBM_ENODEV (-4)   /* no usable gfx950 device */

/* Lattices: D1Q3 and D2Q9 (Table I). */
enum { LBM_D1Q3 = 1, LBM_D2Q9 = 2 };

/* Collision rule of fluid nodes.  MINXENT4 is the paper's MinxEnt with five
 * constraints and four free moments (Sec. IV.C-D); MINXENT2 adds the two
 * constraints C5, C7 relaxed with tau2 (two free moments).  SRT is the BGK
 * rule of Sec. II.B.1.  TRT and MRT are the comparator rules of Sec. II.B.2
 * with the relaxation rates of Table III (tau2 as for MINXENT2).  On D1Q3
 * every rule is SRT: with mass, momentum and the relaxed second moment fixed
 * no moment is left to minimise over. */
enum { LBM_MINXENT4 = 0, LBM_MINXENT2 = 1, LBM_SRT = 2, LBM_TRT = 3, LBM_MRT = 4 };

/* Boundary kinds (Sec. IV.E): full-way bounce-back walls and an equilibrium
 * moving wall.
 *   PERIODIC: every axis wraps, every node is fluid.
 *   TUBE:     walls at x = 0 and x = nx-1; y wraps (D2Q9).
 *   CAVITY:   walls at x = 0, x = nx-1, y = 0; the top row y = ny-1,
 *             corners included, is a lid held at the equilibrium of
 *             (rho0, (u_lid, 0)).  D1Q3: walls at both ends.
 *   BOX:      walls on every side. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_TUBE = 1, LBM_BC_CAVITY = 2, LBM_BC_BOX = 3 };

/* Storage / arithmetic forms.
 *   FP64:          populations stored and computed in double.
 *   FP32_NEWTON64: populations stored in float, every node computed in
 *                  double (moments, logarithms, Newton step, correction);
 *                  reciprocal refinements and log series stop about 2^-42
 *                  relative, four orders below the float storage rounding.
 *   FP32:          stored and computed in float (the four logarithms of the
 *                  gradient are taken of products of population ratios that
 *                  are each close to one).
 *   FP16DEV:       stored as binary16 deviations (f_i - W_i rho0) * 2^k,
 *                  computed in float as FP32.  The reference density rho0
 *                  is per instance; a deviation beyond 65504 * 2^-k overflows
 *                  to inf and sets UNSTABLE. */
enum { LBM_FP64 = 0, LBM_FP32_NEWTON64 = 1, LBM_FP32 = 2, LBM_FP16DEV = 3 };

typedef struct lbm_params {
    int32_t lattice;    /* LBM_D1Q3 or LBM_D2Q9 */
    int32_t collision;  /* LBM_MINXENT4, LBM_MINXENT2, LBM_SRT, LBM_TRT or LBM_MRT */
    int32_t bc;         /* LBM_BC_* */
    int32_t precision;  /* LBM_FP64, LBM_FP32_NEWTON64, LBM_FP32, LBM_FP16DEV */
    int32_t nx, ny;     /* nodes per axis, boundary nodes included; ny = 1 for D1Q3 */
    int32_t fp16_exp;   /* FP16DEV scale exponent k (0 selects 14: |f_i - W_i rho0| < 4); ignored otherwise */
    int32_t reserved;   /* must be 0 */
    double tau;         /* relaxation time, > 1/2; nu = (2 tau - 1)/6 (Sec. IV.C) */
    double tau2;        /* MINXENT2, TRT, MRT; <= 0 selects (8 tau - 1)/(2 tau - 1) (Sec. IV.C) */
    double u_lid;       /* lid x-velocity for LBM_BC_CAVITY */
    double rho0;        /* lid density, and the FP16DEV reference density */
} lbm_params_t;

typedef struct lbm_status {
    uint32_t flags;      /* bit 0: UNSTABLE, bit 1: GUARDED (some node skipped its Newton step) */
    int32_t reserved;
    int64_t first_step;  /* step (0-based) of the first UNSTABLE event, -1 if none */
    int64_t first_node;  /* the smallest node index x + y*nx unstable at first_step, -1 if none;
                            for lbm_status() over a batch, in the instances' concatenated node
                            order.  Steps beyond 2^32 - 1 are recorded as 2^32 - 1. */
    int64_t guarded;     /* node-steps that kept their Newton start point: a start population
                            <= 0 or not finite, or (FP64 arithmetic) a product of the nine
                            below the smallest normal double */
} lbm_status_t;

typedef struct lbm_ctx lbm_ctx_t;

/* Bytes of device workspace a context for p needs: the two population
 * buffers (2 * b * plane stride * bytes per stored population, the plane
 * stride as lbm_set_plane_pad states it).  Returns LBM_EINVAL for invalid
 * parameters, among them a lattice of 2^30 nodes or more, or a D2Q9 lattice
 * whose padded rows hold 2^31 elements or more. */
int lbm_workspace_bytes(const lbm_params_t *p, size_t *bytes);

/* Create a context and set every node to the polynomial equilibrium of the
 * given fields (Sec. IV.E, initial state); lid nodes start at the lid
 * equilibrium.  rho, ux, uy: host arrays, nx*ny doubles each (uy ignored and
 * may be NULL for D1Q3); read only during the call.  dev_workspace: caller
 * device memory of ws_bytes >= lbm_workspace_bytes(), 256-byte aligned
 * (LBM_EINVAL otherwise), or NULL.  On success
 * *out holds the new context; the device state is ready when the stream
 * reaches this point. */
int lbm_init(const lbm_params_t *p, const double *rho, const double *ux, const double *uy,
             void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_ctx_t **out);

/* Workspace bytes for a batch of n independent instances (each with its own
 * size, tau, tau2, u_lid).  All instances share lattice, collision, bc and
 * precision. */
int lbm_workspace_bytes_batch(const lbm_params_t *p, int32_t n, size_t *bytes);

/* Create a batched context: n instances advanced together by one launch per
 * time step.  p: n parameter records; fields concatenated in instance order. */
int lbm_init_batch(const lbm_params_t *p, int32_t n, const double *rho, const double *ux,
                   const double *uy, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                   lbm_ctx_t **out);

/* Enqueue nsteps time steps on the context's stream and return without
 * waiting.  One step is the cycle of Sec. II.A: every node applies its role
 * (fluid collision, bounce-back wall, equilibrium lid; Sec. IV.E), then the
 * post-collision populations stream to the neighbours.  nsteps >= 0. */
int lbm_step(lbm_ctx_t *ctx, int64_t nsteps);

/* Per-instance step counts of a batch: instance i takes no step once the
 * context has completed stop_steps[i] steps (counted from its creation, as
 * lbm_info reports them); from then on its state is carried over unchanged
 * and lbm_moments returns it as it was after that step.  A negative entry,
 * or stop_steps == NULL, removes the limits.  n must equal the number of
 * instances.  Works with graph replay, the LDS-resident shape and shapes
 * that take several steps per launch (a limit inside a launch ends that
 * instance's steps there).  LBM_EINVAL for a single-lattice context.
 * Synchronises. */
int lbm_set_batch_steps(lbm_ctx_t *ctx, const int64_t *stop_steps, int32_t n);

/* Replay time steps from a captured HIP graph of `chunk` steps (chunk >= 1;
 * 0 turns graph replay off).  lbm_step() then enqueues nsteps / chunk graph
 * launches plus the remainder as plain launches.  Results are bitwise equal
 * to plain launches. */
int lbm_set_graph_chunk(lbm_ctx_t *ctx, int32_t chunk);

/* Time the candidate launch shapes of the fused kernel on this context's own
 * buffers (the state is left unchanged) and keep the fastest: every shape
 * is timed, then the eight fastest again with longer trials taken in turn
 * over six rounds.
 * Candidates produce bitwise identical results.  If cache_path is not NULL
 * the choice is read from / appended to that text file, keyed by a hash of
 * the kernel sources, device, lattice, precision, collision, boundary and
 * size.  *chosen (may be NULL) receives the index of the chosen shape.
 * A single lattice whose planes hold at least 1 MiB also has its plane pad
 * tuned (see lbm_set_plane_pad) together with the two fastest shapes, and
 * the fastest (shape, pad) pair is kept; the cache line then carries the
 * pad too.  Synchronises.  For a batch, shapes with another tile
 * size rebuild the tile tables (a device allocation). */
int lbm_autotune(lbm_ctx_t *ctx, const char *cache_path, int32_t *chosen);

/* Plane pad of a single lattice whose planes hold at least 1 MiB.  The b
 * population planes of a buffer follow each other at a stride of
 * round_up(ny * pitch, 64) elements plus pad_bytes, where a D2Q9 row takes
 * pitch = nx rounded up to whole 128-byte lines (its padding is never read)
 * and a D1Q3 lattice is one row of nx; the workspace is sized for the
 * largest pad (8192 bytes), and contexts start at 2048.  A stride that is a
 * large power of two starts all planes at the same memory-channel offset, and
 * which pad avoids that best depends on the size, so the autotuner measures
 * it.  pad_bytes: a multiple of 256 in [0, 8192].  The state moves to the
 * new layout (the other buffer becomes current); results are bitwise the
 * same.  LBM_EINVAL for a batch, a lattice with smaller planes, or a bad pad.
 * Synchronises. */
int lbm_set_plane_pad(lbm_ctx_t *ctx, int32_t pad_bytes);

/* Layout of instance 0: the plane stride in elements and the plane pad in
 * bytes (-1 for a context that takes none); either pointer may be NULL. */
int lbm_get_layout(const lbm_ctx_t *ctx, int64_t *plane_stride, int32_t *pad_bytes);

/* Force a launch shape by index (0 = default); LBM_EINVAL if out of range.
 * For a batch, a shape with another tile size rebuilds the tile tables (a
 * device allocation). */
int lbm_set_variant(lbm_ctx_t *ctx, int32_t variant);

/* Number of launch shapes (for lbm_set_variant) and a short description. */
int lbm_variant_count(const lbm_ctx_t *ctx);
const char *lbm_variant_name(const lbm_ctx_t *ctx, int32_t variant);

/* Steps one launch of a shape takes at most: 1; 2 for the temporally blocked
 * D2Q9 shapes (MinxEnt4, single lattices and batches), which compute one
 * step into on-chip memory and the next from there; 16, 32, 64 or 256 for
 * the D1Q3 shapes that keep 1024-node segments on chip for that many steps.
 * HBM then sees one read and one write of every population per launch.
 * Results are bitwise equal to single steps, status records included;
 * lbm_step() and graph chunks run a remainder as a launch of fewer steps,
 * and a batch instance's step limit can end its steps inside a launch.  0 if
 * ctx is NULL or variant out of range. */
int lbm_variant_steps(const lbm_ctx_t *ctx, int32_t variant);

/* Write rho, ux, uy of the current state (Sec. II.A moments of the
 * populations every node holds before its next collision) into host arrays
 * of nx*ny doubles (concatenated over instances for a batch); any pointer may
 * be NULL.  Synchronises the stream. */
int lbm_moments(lbm_ctx_t *ctx, double *rho, double *ux, double *uy);

/* Copy the current populations (the pre-collision state of every node) to
 * host memory: b planes of nodes doubles each (instance-concatenated for a
 * batch).  Slots fed from outside the lattice on boundary nodes hold
 * unspecified values.  Synchronises. */
int lbm_get_populations(lbm_ctx_t *ctx, double *f);

/* Replace the state with host populations in the layout lbm_get_populations
 * returns (checkpoint restore); resets nothing else.  Synchronises. */
int lbm_set_populations(lbm_ctx_t *ctx, const double *f);

/* Status of instance 0 (or the OR/sum over all instances of a batch).
 * Synchronises. */
int lbm_status(lbm_ctx_t *ctx, lbm_status_t *out);

/* Per-instance status of a batch (n records).  Synchronises. */
int lbm_status_batch(lbm_ctx_t *ctx, lbm_status_t *out, int32_t n);

/* Clear the status of every instance (stream-ordered). */
int lbm_reset_status(lbm_ctx_t *ctx);

/* Steps taken so far, nodes per step, and algorithmic HBM bytes per step
 * (every stored population read once and written once). */
int lbm_info(const lbm_ctx_t *ctx, int64_t *steps_done, int64_t *nodes, int64_t *bytes_per_step);

/* Destroy a context; NULL-safe; never frees caller memory.  Synchronises. */
void lbm_free(lbm_ctx_t *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): run one
 * single lattice from initial fields to final fields with no allocation of
 * any kind.  The two population buffers and the status record live in a
 * fixed device array of LBM_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.
 *   p:             one parameter record, as for lbm_init (no batches).
 *   rho, ux, uy:   DEVICE arrays of nx*ny doubles, the initial fields; uy is
 *                  ignored and may be NULL for D1Q3.  Every node starts at the
 *                  polynomial equilibrium of its fields, lid nodes at the lid
 *                  equilibrium (the state lbm_init sets).
 *   nsteps:        steps to run (>= 0), in the one-step launch shape 0.
 *   rho_out, ux_out, uy_out: DEVICE arrays of nx*ny doubles receiving the
 *                  moments of the final state, as lbm_moments writes them;
 *                  any may be NULL; they may alias the inputs.
 *   status:        HOST record of the run's status, or NULL.  If not NULL the
 *                  call waits for the stream; otherwise it only enqueues work.
 *   hip_stream:    hipStream_t as void*, NULL for the default stream.
 * Results are bitwise those of lbm_init + lbm_step + lbm_moments with the
 * same parameters.  A lattice needing more than LBM_NOALLOC_SCRATCH_BYTES
 * (256 + 2 * b * round_up(ny * pitch, 64) * bytes per population, each
 * buffer rounded up to 256 bytes; pitch as in lbm_set_plane_pad) is rejected
 * with LBM_EINVAL before any work is enqueued.  Every call on one GPU shares
 * that GPU's array and leaves its state there: calls that overlap on one GPU
 * (two streams, or two threads) race and must be serialised by the caller. */
#define LBM_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbm_run_noalloc(const lbm_params_t *p, const double *rho, const double *ux, const double *uy,
                    int64_t nsteps, double *rho_out, double *ux_out, double *uy_out,
                    lbm_status_t *status, void *hip_stream);

/* Plain device-to-device copy kernel of `bytes` bytes (multiple of 16; 0 is a
 * no-op) on hip_stream: a reference for achievable HBM bandwidth.  Each thread
 * moves four 16-byte vectors with non-temporal loads and stores.  dst and src
 * are device pointers that must not overlap. */
int lbm_copy_kernel(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Message of the last error on this thread, and the text of an error code. */
const char *lbm_last_error(void);
const char *lbm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
