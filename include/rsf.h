/*
 * rsf.h -- C ABI of the MI355X (gfx950) RSF level-set evolution library.
 *
 * The library evolves a level-set function phi over a 3D image I by the
 * region-scalable fitting (RSF) model in the form of Niger et al., arXiv
 * 2404.02813: explicit time steps phi <- phi + dt * E (Sec. 2, Eq. 1) with
 *
 *   E = mu * R(phi) + delta_eps(phi) * (nu * kappa - (lambda1 e1 - lambda2 e2))
 *
 * (Sec. 3, final energy), where
 *   H_eps(u) = 1/2 (1 + (2/pi) atan(u/eps)),  delta_eps = H_eps'      (Sec. 3)
 *   f1 = K*(H I) / K*H,  f2 = K*((1-H) I) / K*(1-H)    (Sec. 3, local_intensity)
 *   e_i = I^2 (K*1) - 2 I (K*f_i) + K*(f_i^2)          (fitting energies of the
 *                                                        RSF model, Sec. 3 force)
 *   kappa = div(grad phi / sqrt(|grad phi|^2 + eta))   (Sec. 2.2 smoothing)
 *   R = lap(phi) + div(D(|grad phi|) grad phi)         (Sec. 2.1 regulariser)
 * K is the Gaussian of Sec. 3 sampled on the grid, truncated at R = ceil(3
 * sigma) voxels per axis and normalised to unit sum; convolutions use zero
 * padding.  Differences are central, the Laplacian 7-point, ghost values by
 * reflection about the boundary voxel.  Sign convention: H weights phi > 0,
 * so f1 is the fit of the phi > 0 region.
 *
 * Conventions for every entry point:
 *   - Arrays are dense [nz][ny][nx] with x fastest.  Pointers named "device"
 *     are HIP device pointers on the context's device; the library never
 *     frees or retains them beyond the call's stream work.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously; device faults surface at the next synchronising call.
 *   - Every entry validates its arguments before enqueuing anything and leaves
 *     its outputs untouched on a validation error.  No C++ exception crosses
 *     the ABI.  rsf_last_error() describes the last failure on a context.
 *   - A context is not thread-safe: use one per host thread.  Calls on one
 *     context may use different streams: a call that uses the context's own
 *     workspace first makes its stream wait (on the device) for the end of
 *     the previous such call.  A caller-supplied workspace is the caller's
 *     to order.
 *   - Every xy plane is at most 2^28 voxels (nx * ny <= 268435456): kernels
 *     address a slice with 32-bit offsets.  Larger planes give
 *     RSF_ERR_INVALID_ARG.
 */
#ifndef RSF_H
#define RSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsf_context rsf_context;

typedef enum {
    RSF_NOT_READY = 1,          /* rsf_server_poll / _wait: request not done yet */
    RSF_OK = 0,
    RSF_ERR_INVALID_ARG = -1,
    RSF_ERR_OUT_OF_MEMORY = -2,
    RSF_ERR_DEVICE = -3,
    RSF_ERR_NONFINITE = -4,
    RSF_ERR_BUDGET = -5,
    RSF_ERR_INTERNAL = -6
} rsf_status;

/* Element types.  The image may be RSF_F32 or RSF_U16 (normalised on the
 * device to u / 65535); the intermediate fields (the convolved fields and
 * K*I) may be stored as RSF_F32, RSF_F16 or RSF_BF16.  Arithmetic and phi
 * are always FP32; the convergence sums FP64.  Combinations other than
 * (F32 image, F32 storage) are built for ceil(3 sigma) in 4..12. */
typedef enum {
    RSF_F32 = 0,
    RSF_F16 = 1,
    RSF_BF16 = 2,
    RSF_U16 = 3
} rsf_dtype;

/* Distance-regulariser reading (Sec. 2.1).  The paper names "forward and
 * backward (FAB) diffusion" and prints a garbled single-well formula:
 *   RSF_REG_DOUBLE_WELL (default): D(s) = sin(2 pi s)/(2 pi s) - 1 for
 *       s <= 1, -1/s for s > 1 (the double-well potential of distance-
 *       regularised level sets, whose diffusion is forward-and-backward);
 *   RSF_REG_SINGLE_WELL: D = -1/sqrt(s^2 + eta), i.e. R = lap(phi) - kappa.
 *       Backward diffusion where |grad phi| < 1 makes this reading amplify
 *       rounding; it is provided for comparison. */
typedef enum {
    RSF_REG_DOUBLE_WELL = 0,
    RSF_REG_SINGLE_WELL = 1
} rsf_regulariser;

/* Data force.
 *   RSF_FORCE_RSF (default): lambda1 e1 - lambda2 e2 with the fitting
 *       energies e_i = I^2 (K*1) - 2 I (K*f_i) + K*(f_i^2) of the RSF model
 *       the paper builds on, the same sigma for the fits and the force;
 *       two Gaussian stages per iteration.
 *   RSF_FORCE_PAPER: the expansion of Sec. 4.2 (voxel level parallelism),
 *       F+- = K2*I^2 - 2 r+- K2*I + r+-^2 with K2 the Gaussian of scale
 *       sigma2, and lambda1 F+ - lambda2 F-.  With sigma2 = 0 (every 3D run
 *       of the paper, Sec. 5) K2 is the identity and F+- = (I - r+-)^2: one
 *       Gaussian stage per iteration.  With sigma2 > 0, K2*I and K2*I^2 are
 *       computed once per evolution and need two more workspace fields
 *       (size the workspace with rsf_workspace_bytes_params).  r+ = f1,
 *       r- = f2. */
typedef enum {
    RSF_FORCE_RSF = 0,
    RSF_FORCE_PAPER = 1
} rsf_force;

/* Parameters of one evolution (Sec. 2-3 notation: alpha = nu, beta carried
 * by lambda1 = lambda2, mu weighs the regulariser). */
typedef struct {
    float sigma;      /* Gaussian scale, voxels; R = ceil(3 sigma) <= 16     */
    float lambda1;    /* weight of e1 (phi > 0 region)                        */
    float lambda2;    /* weight of e2 (phi < 0 region)                        */
    float nu;         /* curvature (smoothing) weight, >= 0                   */
    float mu;         /* regulariser weight, >= 0                             */
    float dt;         /* time step, > 0                                       */
    float eps;        /* Heaviside / Dirac width, > 0                         */
    float eta;        /* floor inside |grad phi| of the normal; <= 0 -> 1e-10 */
    int regulariser;  /* rsf_regulariser                                      */
    int storage;      /* rsf_dtype of the intermediate fields (F32/F16/BF16)  */
    int force;        /* rsf_force                                            */
    float sigma2;     /* scale of the force kernel for RSF_FORCE_PAPER (0 =
                         the identity, the value of the paper's 3D runs);
                         ceil(3 sigma2) <= 16, and 4..12 for the FP16/BF16/
                         uint16 type combinations                            */
} rsf_params;

/* Results of the last evolution on a context. */
typedef struct {
    int iters_requested;
    int iters_run;        /* < iters_requested only when tol stopped it early */
    double last_sum_abs;  /* sum |phi_{n+1} - phi_n| of the last iteration run */
} rsf_stats;

/* Create a context bound to HIP device `device_ordinal`.  *out is NULL on
 * failure. */
rsf_status rsf_create(rsf_context **out, int device_ordinal);

/* Destroy a context and the device memory it owns.  NULL is a no-op. */
void rsf_destroy(rsf_context *ctx);

/* Text of the last error on `ctx` ("" if none; a static message if ctx is
 * NULL).  Valid until the next call on the context. */
const char *rsf_last_error(const rsf_context *ctx);

/* Bytes of device workspace an evolution of an nx*ny*nz volume over `iters`
 * iterations needs with intermediate fields of type `storage`: five fields of
 * that type, one float field, small tables (24 B/voxel at RSF_F32, 14 B/voxel
 * at RSF_F16/RSF_BF16).  0 for invalid arguments. */
size_t rsf_workspace_bytes(int64_t nx, int64_t ny, int64_t nz, int iters, int storage);

/* Evolve phi in place for `iters` iterations of Eq. (1) with the default
 * (double-well) regulariser, eta = 1e-10 and FP32 storage.
 *   volume : device, const, nx*ny*nz elements of `volume_dtype` (RSF_F32 or
 *            RSF_U16; the image I)
 *   phi    : device, nx*ny*nz floats; phi_0 on entry, phi_iters on return
 *   nx,ny,nz >= 3; sigma > 0 with ceil(3 sigma) <= 16; eps > 0; dt > 0;
 *   nu, mu >= 0; lambda1, lambda2 finite; iters >= 0 (0 is a no-op).
 * The workspace is allocated by the context (grown on demand, kept). */
rsf_status rsf_evolve(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                      int64_t nx, int64_t ny, int64_t nz,
                      float sigma, float lambda1, float lambda2, float nu, float mu,
                      float dt, float eps, int iters, void *stream);

/* As rsf_evolve with explicit parameters and options.
 *   params    : host, read during the call only.
 *   tol       : > 0 stops early (on the device) once sum|dphi| / voxels < tol;
 *               the remaining iterations leave phi unchanged.  0 = fixed count.
 *   workspace : device buffer of >= rsf_workspace_bytes(...) bytes owned by the
 *               caller, or NULL to use the context's own allocation.
 * The per-iteration sums are kept on the device; rsf_get_stats() reads them. */
rsf_status rsf_evolve_ex(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                         int64_t nx, int64_t ny, int64_t nz, const rsf_params *params,
                         int iters, double tol, void *workspace, size_t workspace_bytes,
                         void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  As
 * rsf_evolve_ex with the context's workspace, but that workspace is a fixed
 * device array of RSF_NOALLOC_MAX_BYTES per GPU, created with the library's
 * code object on that device and held until the process ends, and the tile
 * table is written by a kernel from its argument: the call allocates no
 * device or pinned host memory (no hipMalloc, hipFree or hipHostMalloc, no
 * events; rsf_profile_enable is ignored for it).  The caller passes the
 * image and phi as in rsf_evolve_ex.
 *   RSF_ERR_INVALID_ARG when rsf_workspace_bytes_params(nx, ny, nz, iters,
 *   params) exceeds RSF_NOALLOC_MAX_BYTES (e.g. 128^3 voxels with FP32
 *   storage fit, 192^3 with FP16 storage fit), phi untouched.
 * Every call on one GPU, from any context or stream, shares that GPU's array,
 * which keeps the last call's contents (each call's set-up clears what must
 * start at zero): calls that overlap on one GPU race, and the caller must
 * order them.  rsf_get_stats() reads the last call's sums from the array
 * until the next such call. */
#define RSF_NOALLOC_MAX_BYTES ((size_t)128 << 20)
rsf_status rsf_evolve_noalloc(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                              int64_t nx, int64_t ny, int64_t nz, const rsf_params *params,
                              int iters, double tol, void *stream);

/* One volume of a batch (device pointers, as in rsf_evolve). */
typedef struct {
    const void *volume;   /* image I, nx*ny*nz elements of the batch's volume dtype */
    float *phi;           /* phi_0 on entry, phi_iters on return                    */
    int64_t nx, ny, nz;   /* each >= 3                                              */
} rsf_tile;

/* Bytes of device workspace rsf_evolve_batch needs for these tiles. */
size_t rsf_batch_workspace_bytes(const rsf_tile *tiles, int n_tiles, int iters, int storage);

/* As rsf_workspace_bytes / rsf_batch_workspace_bytes, but for the full
 * parameter set: counts the two extra fields the Sec. 4.2 force needs when
 * sigma2 > 0.  0 for invalid parameters or dims. */
size_t rsf_workspace_bytes_params(int64_t nx, int64_t ny, int64_t nz, int iters,
                                  const rsf_params *params);
size_t rsf_batch_workspace_bytes_params(const rsf_tile *tiles, int n_tiles, int iters,
                                        const rsf_params *params);

/* Evolve every tile of a batch by `iters` iterations with shared parameters
 * (the sub-volume parallelism of Sec. 4.1: tiles are independent problems,
 * each with its own boundary; a tile's result does not depend on the rest of
 * the batch).  Every pass is one launch over all tiles, however uneven their
 * shapes; tiles may differ in size but share sigma, the volume dtype and the
 * storage type.  tiles: host array, read during the call; other arguments as
 * in rsf_evolve_ex (tol applies per tile).  rsf_get_tile_stats() reads the
 * per-tile statistics afterwards. */
rsf_status rsf_evolve_batch(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                            int volume_dtype, const rsf_params *params, int iters, double tol,
                            void *workspace, size_t workspace_bytes, void *stream);

/* Autotuner.  Times `trial_iters` iterations of these tiles (on copies of
 * their phi; the caller's buffers are not modified) for candidate workgroup
 * splits of each pass (row chunks of the xy passes, z chunks of the z and
 * update passes), one pass at a time with the passes separate, and keeps the
 * fastest split per tile shape and radius in the context.  Then, where the
 * force and radius allow the fused update (rsf_set_fusion), it times that
 * schedule against the separate passes and keeps the faster for this set of
 * tile shapes.  Later evolutions of the same shapes use both.
 *   chosen : NULL or int64_t[4]: the xy, z and update workgroup targets, and
 *            1 if the fused update was chosen (else 0).
 * phi after an evolution is bitwise independent of the split and schedule;
 * the FP64 sums of |dphi| are grouped per update workgroup, so they may
 * differ in the last bits.  Synchronises `stream`; allocates a scratch copy
 * of phi for the duration of the call (rsf_autotune_ex takes it from the
 * caller); invalidates the statistics of the last evolution. */
rsf_status rsf_autotune(rsf_context *ctx, const rsf_tile *tiles, int n_tiles, int volume_dtype,
                        const rsf_params *params, int trial_iters, int64_t *chosen,
                        void *stream);

/* Device bytes of rsf_autotune_ex's workspace for these tiles: the copies of
 * their phi (each rounded up to 256 bytes) and the batch workspace of the
 * largest trial any candidate split can need (trial_iters + 1 iterations).
 * Depends on the context's workgroup targets.  0 for invalid arguments. */
size_t rsf_autotune_workspace_bytes(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                                    const rsf_params *params, int trial_iters);

/* rsf_autotune with the phi copies and every trial's batch workspace in the
 * caller's workspace (device, 256-byte aligned, at least
 * rsf_autotune_workspace_bytes(...) bytes; NULL allocates as rsf_autotune
 * does, the trials then using the context's own workspace), so that the call
 * allocates no device memory.  RSF_ERR_INVALID_ARG for a workspace that is
 * too small or misaligned, before anything runs.  The choices and the
 * statistics of the last evolution follow rsf_autotune, except that the
 * context's own workspace and its statistics are left alone. */
rsf_status rsf_autotune_ex(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                           int volume_dtype, const rsf_params *params, int trial_iters,
                           int64_t *chosen, void *workspace, size_t workspace_bytes,
                           void *stream);

/* Workgroup targets of a whole batch (xy waves, z-pass workgroups, update-
 * pass workgroups) from which untuned splits are derived, each tile taking
 * its share of the batch's voxels; 0 keeps the built-in value (16384, 2048,
 * 1024).  rsf_autotune starts its search from these and reports the targets
 * it chose in chosen[0..2].  Results do not depend on them. */
rsf_status rsf_set_split_targets(rsf_context *ctx, int64_t xy_waves, int64_t z_blocks,
                                 int64_t u_blocks);

/* Forget all autotuned splits and schedules of the context. */
void rsf_autotune_reset(rsf_context *ctx);

/* Statistics of tile `tile` of the last evolution (tile 0 for rsf_evolve). */
rsf_status rsf_get_tile_stats(rsf_context *ctx, int tile, rsf_stats *out, double *s_hist,
                              int cap);

/* Synchronise the stream of the last evolution and report its statistics.
 * s_hist (host, may be NULL) receives up to `cap` per-iteration sums
 * sum|phi_{n+1} - phi_n| in double (the convergence reduction). */
rsf_status rsf_get_stats(rsf_context *ctx, rsf_stats *out, double *s_hist, int cap);

/* Volume-level driver (Sec. 4.1, volume level parallelism).  Splits the
 * volume into sub-volumes whose cores cut each axis into near-equal parts of
 * at most `block` voxels, extends each core by a curtain of `curtain`
 * voxels (0: ceil(3 max(sigma, sigma2))) on every side shared with a
 * neighbour, evolves the sub-volumes independently (each from its slice of
 * phi, `iters` iterations, in batches of at most `budget_bytes` of copies
 * and workspace; 0 = all at once), and merges them into phi by linear
 * interpolation across each 2*curtain-wide overlap: along an axis the
 * weight of a sub-volume ramps linearly from 1/(4C) to 1 - 1/(4C) across
 * the overlap and its neighbour's weight is the complement; corners take the
 * product of the per-axis weights, so the weights of all sub-volumes sum to
 * one.  With a single sub-volume the result is rsf_evolve_ex's.
 * Every core must be at least 2 * curtain long (RSF_ERR_INVALID_ARG);
 * a sub-volume larger than the budget gives RSF_ERR_BUDGET.  Allocates an
 * FP32 merge buffer of the volume's size and the sub-volume copies for the
 * duration of the call (rsf_evolve_volume_ex takes them from the caller);
 * synchronises `stream`; phi is untouched on a validation error.
 * Tolerance-based stopping and statistics are not offered here. */
rsf_status rsf_evolve_volume(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                             int64_t nx, int64_t ny, int64_t nz, int64_t block, int64_t curtain,
                             const rsf_params *params, int iters, size_t budget_bytes,
                             void *stream);

/* Device bytes rsf_evolve_volume_ex needs for these arguments on this
 * context (its split targets size the batch workspace): the FP32 merge
 * buffer, the sub-volume copies of the largest group and that group's batch
 * workspace.  0 for invalid arguments. */
size_t rsf_volume_workspace_bytes(rsf_context *ctx, int volume_dtype, int64_t nx, int64_t ny,
                                  int64_t nz, int64_t block, int64_t curtain,
                                  const rsf_params *params, int iters, size_t budget_bytes);

/* rsf_evolve_volume with every device buffer in the caller's workspace
 * (device, 256-byte aligned, at least rsf_volume_workspace_bytes(...) bytes;
 * NULL allocates as rsf_evolve_volume does), so that the caller owns all the
 * device memory the call uses.  RSF_ERR_INVALID_ARG for a workspace that is
 * too small or misaligned, phi untouched.  The result is bitwise
 * rsf_evolve_volume's. */
rsf_status rsf_evolve_volume_ex(rsf_context *ctx, const void *volume, int volume_dtype,
                                float *phi, int64_t nx, int64_t ny, int64_t nz, int64_t block,
                                int64_t curtain, const rsf_params *params, int iters,
                                size_t budget_bytes, void *workspace, size_t workspace_bytes,
                                void *stream);

/* ------------------------------------------------------------------------
 * Initialisation (Sec. 4.3): seed points from blob detection by the
 * determinant of the Hessian in each z slice, then phi0 from the distance to
 * the nearest seed by fast sweeping.
 * ---------------------------------------------------------------------- */

/* Seed mask (device, nx*ny*nz bytes, 1 at seeds).  Each z slice is smoothed
 * by the sampled, unit-sum 2D Gaussian of scale sigma_b (zero padding); the
 * in-slice Hessian of the result comes from central second differences
 * (reflection about the boundary voxel).  A voxel is a seed when its
 * determinant exceeds `threshold` (in [0, 1)) times the largest determinant
 * of the volume, the trace is negative (a bright blob) and the determinant
 * is a maximum of the 3x3 in-slice neighbourhood (strictly above the
 * neighbours earlier in raster order, at least the later ones).  *n_seeds
 * (host, may be NULL) receives the count; synchronises `stream`.  volume:
 * RSF_F32 or RSF_U16.  Allocates scratch for the call (rsf_seeds_ex takes it
 * from the caller). */
rsf_status rsf_seeds(rsf_context *ctx, const void *volume, int volume_dtype, int64_t nx,
                     int64_t ny, int64_t nz, float sigma_b, float threshold, unsigned char *mask,
                     int64_t *n_seeds, void *stream);

/* Device bytes of rsf_seeds_ex's workspace for an nx*ny*nz volume: the
 * distance field and three smoothing / Hessian fields (4n bytes each) and
 * two per-block reduction arrays, each piece rounded up to 256 bytes.  0 for
 * invalid dimensions. */
size_t rsf_seeds_workspace_bytes(int64_t nx, int64_t ny, int64_t nz);

/* rsf_seeds with its scratch in the caller's workspace (device, 256-byte
 * aligned, at least rsf_seeds_workspace_bytes(nx, ny, nz) bytes; NULL
 * allocates as rsf_seeds does).  RSF_ERR_INVALID_ARG for a workspace that is
 * too small or misaligned (mask untouched).  The result is bitwise
 * rsf_seeds's; calls that share one workspace must not overlap. */
rsf_status rsf_seeds_ex(rsf_context *ctx, const void *volume, int volume_dtype, int64_t nx,
                        int64_t ny, int64_t nz, float sigma_b, float threshold,
                        unsigned char *mask, int64_t *n_seeds, void *workspace,
                        size_t workspace_bytes, void *stream);

/* Fast sweeping (Zhao 2005) in place: u (device floats) holds 0 at the
 * seeds and a large value (1e30) elsewhere; `rounds` repetitions of the
 * eight Gauss-Seidel sweep orderings of the Godunov upwind discretisation of
 * |grad u| = 1 on the unit grid.  Each sweep runs over hyperplanes of
 * 32x8x8 blocks (each block swept in LDS along its own hyperplanes), which
 * gives the same updates as the sequential sweep.  One round reaches
 * the discrete solution for a single seed; several seeds can need a second
 * (first-round differences of order 1e-4). */
rsf_status rsf_fast_sweep(rsf_context *ctx, float *u, int64_t nx, int64_t ny, int64_t nz,
                          int rounds, void *stream);

/* phi0 = offset - (distance to the nearest seed): seeds as rsf_seeds, the
 * distance as rsf_fast_sweep.  With offset 0 the seeds lie on the zero level
 * and the vessels around them grow into phi > 0 (the region H weights).
 * RSF_ERR_INVALID_ARG if no seed is found (phi untouched).  Synchronises
 * `stream`; allocates scratch for the call (rsf_init_phi_ex takes it from
 * the caller). */
rsf_status rsf_init_phi(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                        int64_t nx, int64_t ny, int64_t nz, float sigma_b, float threshold,
                        float offset, int rounds, int64_t *n_seeds, void *stream);

/* Device bytes of rsf_init_phi_ex's workspace for an nx*ny*nz volume: the
 * seed mask (n bytes), the distance field and three smoothing / Hessian
 * fields (4n bytes each) and two per-block reduction arrays, each piece
 * rounded up to 256 bytes.  0 for invalid dimensions. */
size_t rsf_init_workspace_bytes(int64_t nx, int64_t ny, int64_t nz);

/* rsf_init_phi with its scratch in the caller's workspace (device, 256-byte
 * aligned, at least rsf_init_workspace_bytes(nx, ny, nz) bytes; NULL
 * allocates as rsf_init_phi does).  RSF_ERR_INVALID_ARG for a workspace that
 * is too small or misaligned (phi untouched).  The result is bitwise
 * rsf_init_phi's; calls that share one workspace must not overlap. */
rsf_status rsf_init_phi_ex(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                           int64_t nx, int64_t ny, int64_t nz, float sigma_b, float threshold,
                           float offset, int rounds, int64_t *n_seeds, void *workspace,
                           size_t workspace_bytes, void *stream);

/* One zero-padded Gaussian convolution out = K * in (Sec. 3 kernel), the
 * separable passes the evolution uses.  in, out: device floats, distinct;
 * every dimension >= 3. */
rsf_status rsf_gauss3d(rsf_context *ctx, const float *in, float *out,
                       int64_t nx, int64_t ny, int64_t nz, float sigma, void *stream);

/* Intermediate fields of ONE iteration from (volume, phi), for parity checks.
 * Each non-NULL pointer is a device buffer of nx*ny*nz floats that receives:
 *   H = H_eps(phi), f1, f2 (region fits), Fd = lambda1 e1 - lambda2 e2,
 *   kappa, lap (7-point Laplacian), R (regulariser), E (the update rate)
 * and phi_next = phi + dt E.  phi is not modified. */
typedef struct {
    float *H, *f1, *f2, *Fd, *kappa, *lap, *R, *E, *phi_next;
} rsf_probe_fields;

rsf_status rsf_probe(rsf_context *ctx, const void *volume, int volume_dtype, const float *phi,
                     int64_t nx, int64_t ny, int64_t nz, const rsf_params *params,
                     const rsf_probe_fields *fields, void *stream);

/* Per-pass timing with HIP events recorded around every launch on the
 * caller's stream (tracing support; the paper profiles per kernel in
 * Table 1).  Passes of one iteration: */
typedef enum {
    RSF_PASS_SETUP = 0,        /* edge tables of K*1 and K*I, once per call   */
    RSF_PASS_Z_HEAVISIDE = 1,  /* z Gaussian of (H I, H)                      */
    RSF_PASS_XY_FITS = 2,      /* xy Gaussian + region fits -> g1, g2         */
    RSF_PASS_XY_FORCE = 3,     /* xy Gaussian of (g1, g2)                     */
    RSF_PASS_Z_UPDATE = 4,     /* z Gaussian + force, curvature, update       */
    RSF_PASS_REDUCE = 5,       /* FP64 sum |dphi|                             */
    /* initialisation (Sec. 4.3) */
    RSF_PASS_INIT_SMOOTH = 6,  /* x or y pass of the slice Gaussian           */
    RSF_PASS_INIT_HESSIAN = 7, /* determinant and trace, and their maximum    */
    RSF_PASS_INIT_SELECT = 8,  /* seed selection, initial distance field      */
    RSF_PASS_INIT_SWEEP = 9,   /* one hyperplane of blocks of a fast sweep    */
    RSF_PASS_INIT_OFFSET = 10, /* phi0 = offset - distance                    */
    RSF_PASS_COUNT = 11
} rsf_pass;

typedef struct {
    int launches[RSF_PASS_COUNT];
    double ms[RSF_PASS_COUNT];      /* summed event time per pass */
} rsf_profile;

/* The update also forms the next iteration's stage-1 z Gaussian (Sec. 3
 * fits) from the phi it has just written, so that pass is not launched again
 * (on != 0, the default).  Applies to single volumes and batches alike when
 * the RSF force's radius ceil(3 sigma) is at most 12 with RSF_F16 storage, 9
 * with RSF_F32 or RSF_BF16 storage and an RSF_F32 image, 8 with a uint16
 * image (any radius for the Sec. 4.2 force); every tile's update then marches
 * its whole z extent.  Results are bitwise the same either way; off runs the
 * passes separately.  Affects later rsf_evolve* calls on this context. */
rsf_status rsf_set_fusion(rsf_context *ctx, int on);

/* Iterations replayed from a captured HIP graph (on != 0, the default): with
 * at least 8 iterations and per-pass timing off, rsf_evolve, rsf_evolve_ex
 * and rsf_evolve_batch capture one group of 16 iterations' launches (kernel
 * launches only) and replay it on the caller's stream; the rest of the count
 * launches directly.  A later call whose launches are the same replays the
 * kept graph without capturing again.  Results are bitwise the same either
 * way; off launches every iteration directly. */
rsf_status rsf_set_graphs(rsf_context *ctx, int on);

/* Measurement aid: one launch of a streaming kernel with a pass's read/write
 * mix, for the achievable HBM bandwidth the passes are compared against.
 *   in  : device, n_read (1..4) float fields of n floats each, contiguous
 *         (field k at in + k n); 16-byte aligned
 *   out : device, n_write (1..3) float fields of n floats, likewise;
 *         out_j[i] = j + sum_k in_k[i]
 *   n   : floats per field, a positive multiple of 4
 * Enqueued on `stream` on the current device; RSF_ERR_INVALID_ARG for bad
 * arguments, RSF_ERR_DEVICE if the launch fails. */
rsf_status rsf_stream_probe(const float *in, int n_read, float *out, int n_write, int64_t n,
                            void *stream);

/* Start (on != 0) or stop recording events on later launches. */
rsf_status rsf_profile_enable(rsf_context *ctx, int on);

/* Wait for the recorded launches, return their totals and clear them. */
rsf_status rsf_profile_read(rsf_context *ctx, rsf_profile *out);

/* Injected allocation failures, for tests of the error paths.  spec
 * "alloc_fail:N" or "alloc_fail:N:K" (N, K >= 1, K = 1 if omitted): from
 * this call on, the library counts every device and pinned host allocation
 * it attempts (all contexts and servers of the process), and attempts
 * N .. N+K-1 fail as out of memory (RSF_ERR_OUT_OF_MEMORY from the call that
 * made them) without allocating.  NULL, "" or "off" disarms.  The same spec
 * in the environment variable RSF_FAULT arms it when the library is loaded;
 * a malformed RSF_FAULT makes rsf_create return RSF_ERR_INVALID_ARG.
 * RSF_ERR_INVALID_ARG for a malformed spec (the current state is kept). */
rsf_status rsf_set_fault(const char *spec);

/* Allocation attempts counted since the fault was armed; -1 when disarmed. */
int64_t rsf_fault_allocations(void);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of independent tiles.
 *
 * The paper evolves a large volume as independent sub-volumes, each with a
 * curtain (halo) sized by the Gaussian scale (Sec. 4.1, volume level
 * parallelism).  A server evolves such tiles as requests arrive: a worker
 * thread admits requests in arrival order while the sum of the admitted
 * requests' workspaces (rsf_workspace_bytes_params) stays within the HBM budget and
 * a resident slot is free, then advances every resident tile by up to
 * `chunk_iters` iterations per scheduling chunk.  Tiles with equal
 * parameters, image type and storage type (in particular equal sigma) share
 * each launch; tiles join and leave the batch at chunk boundaries, each with
 * its own iteration count, so requests that arrive while others run overlap
 * with them on the device.  A tile's result is bitwise the one rsf_evolve_ex
 * gives for it alone.
 *
 * Workspaces come from a device arena that grows in segments up to the
 * budget and is kept until the server is destroyed.  One server per device;
 * its functions may be called from any host thread.
 * ---------------------------------------------------------------------- */
typedef struct rsf_server rsf_server;

/* Which resident tiles run in a chunk when batch_voxels caps the batch:
 * RSF_ORDER_ARRIVAL takes them oldest first, RSF_ORDER_SHORTEST by least
 * remaining work (iterations left times voxels), ties by arrival.  The rest
 * wait, resident, for a later chunk. */
typedef enum {
    RSF_ORDER_ARRIVAL = 0,
    RSF_ORDER_SHORTEST = 1
} rsf_order;

typedef struct {
    int device;            /* HIP device ordinal                               */
    size_t budget_bytes;   /* HBM for request workspaces (admission limit)     */
    size_t segment_bytes;  /* arena growth step; 0 = 8 GiB                     */
    int chunk_iters;       /* iterations per scheduling chunk; 0 = 4           */
    int max_resident;      /* most tiles resident at once; 0 = 256 (<= 4096)  */
    int64_t batch_voxels;  /* run tiles (in `order`) until their voxels reach
                              this per chunk; 0 = every resident tile runs    */
    int order;             /* rsf_order                                        */
    int64_t split_targets[3]; /* as rsf_set_split_targets; 0 = built-in       */
    int separate_passes;   /* 0: a group whose force and radius allow it runs
                              the update fused with the next stage-1 z pass
                              (one stage-1 pass per chunk); 1: every pass
                              separately.  Bitwise the same results.         */
} rsf_server_config;

typedef struct {
    const void *volume;    /* device image [nz][ny][nx], volume_dtype         */
    float *phi;            /* device phi0 on entry, phi_iters when done        */
    int64_t nx, ny, nz;
    int volume_dtype;      /* RSF_F32 or RSF_U16                               */
    rsf_params params;     /* sigma ... storage, as for rsf_evolve_ex          */
    int iters;             /* >= 0                                             */
    double tol;            /* early stop as for rsf_evolve_ex (0 = never)      */
} rsf_request;

typedef struct {
    int status;            /* RSF_OK, or the error that ended the request     */
    int iters_run;
    double last_sum_abs;   /* sum |dphi| of the last iteration run            */
    double t_submit;       /* host monotonic clock (CLOCK_MONOTONIC), seconds */
    double t_admit;
    double t_done;         /* when the worker saw the result complete         */
    size_t workspace_bytes;
} rsf_result;

typedef struct {
    uint64_t submitted, completed;
    int pending, resident, peak_resident;
    size_t bytes_in_use, peak_bytes, bytes_reserved;
    uint64_t chunks;       /* scheduling chunks launched                      */
    double voxel_iters;    /* voxel-iterations of completed requests          */
} rsf_server_stats;

/* Create a server.  Validates the configuration; allocates streams, events
 * and pinned staging, not the arena (that grows as requests are admitted). */
rsf_status rsf_server_create(rsf_server **out, const rsf_server_config *cfg);

/* Queue a request; *ticket identifies it.  Validation as for rsf_evolve_ex
 * (RSF_ERR_INVALID_ARG); a request whose workspace alone exceeds the budget
 * is refused with RSF_ERR_BUDGET.  The volume and phi must be ready on the
 * device (the server's stream does not wait for the caller's streams) and
 * must stay allocated and untouched until the request is done. */
rsf_status rsf_server_submit(rsf_server *srv, const rsf_request *req, uint64_t *ticket);

/* Result of a request: RSF_OK and *out filled when done (the server no
 * longer references its buffers), RSF_NOT_READY while queued or running,
 * RSF_ERR_INVALID_ARG for an unknown ticket.  A result is kept until read
 * by poll or wait, then forgotten. */
rsf_status rsf_server_poll(rsf_server *srv, uint64_t ticket, rsf_result *out);

/* As poll, but blocks up to timeout_s seconds (< 0: no limit). */
rsf_status rsf_server_wait(rsf_server *srv, uint64_t ticket, double timeout_s, rsf_result *out);

/* Block until every request submitted so far is done. */
rsf_status rsf_server_drain(rsf_server *srv);

rsf_status rsf_server_get_stats(rsf_server *srv, rsf_server_stats *out);

/* Last error of the server (validation, or the device error that failed its
 * requests). */
const char *rsf_server_last_error(const rsf_server *srv);

/* Drain, stop the worker and free the server.  NULL is a no-op. */
void rsf_server_destroy(rsf_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* RSF_H */
