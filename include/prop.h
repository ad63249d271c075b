/*
 * prop.h -- C ABI of the MI355X (gfx950) finite-difference wave propagators.
 *
 * Two explicit time-stepped propagators, each with its exact discrete adjoint:
 *
 *   PROP_TTI      pseudo-acoustic tilted transverse isotropy: coupled fields
 *                 p, q and self-adjoint rotated second derivatives built from
 *                 m = 1/vp^2, Thomsen epsilon, delta, tilt theta, azimuth phi
 *                 (the paper's anisotropic wave-equation section, Eq. "rot"
 *                 and the rotated-derivative listing), leapfrog in time.
 *   PROP_ELASTIC  isotropic velocity-stress on a staggered grid with Lame
 *                 parameters and density (Eq. "elas1" and the elastic listing),
 *                 velocities first, then stresses from the new velocities.
 *
 * The calls follow the paper's problem statement (Eq. "acou" and the Grid /
 * Function / TimeFunction / SparseTimeFunction listings): a model on a grid,
 * a source wavelet at off-grid points, receiver traces at off-grid points,
 * a space order and a time order.
 *
 * Conventions
 *   - Arrays of grid values are FP32, shape (nz, ny, nx), x fastest (C order).
 *     2D grids use ndim = 2, ny = 1 and the axes x and z.
 *   - Coordinates are metres; point (i, j, k) sits at origin + (i hx, j hy, k hz);
 *     z is depth.  Point coordinates are given as (x, z) in 2D, (x, y, z) in 3D.
 *   - Values outside the grid are zero for every field and every intermediate
 *     (truncation); the absorbing layer of nbl points lies inside the shape.
 *   - Step n = 0..nt-1 uses wavelet sample n (time n dt) and produces trace
 *     sample n from the new state (time (n+1) dt).
 *   - Pointers marked DEVICE are HIP device pointers; HOST pointers are read
 *     during the call only.  The caller owns everything it passes in; the
 *     handle owns its internal wavefields, checkpoints and tables.  Model
 *     arrays are referenced, not copied: keep them alive and unchanged until
 *     prop_set_model or prop_destroy.
 *   - All GPU work is enqueued on the stream given at creation (a hipStream_t,
 *     NULL = default stream); the calls return after enqueueing, except where
 *     a result must come back to the host (prop_dot_f64, error checks of the
 *     instability watchdog).
 *   - Every call returns PROP_OK (0) or a negative error code; no C++
 *     exception crosses the ABI.  prop_last_error() gives a message for the
 *     last failure on the calling thread.
 *   - Calls on one handle must not overlap (one handle = one set of wavefields).
 */
#ifndef PROP_H
#define PROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PROP_OK         0
#define PROP_EINVAL    (-1)  /* bad argument: shape, order, null pointer, point outside the grid */
#define PROP_ENOMEM    (-2)  /* device allocation failed */
#define PROP_EHIP      (-3)  /* HIP runtime error (message includes hipGetErrorString) */
#define PROP_EUNSTABLE (-4)  /* dt above the stability bound, epsilon < delta, or NaN/Inf detected */
#define PROP_ESTATE    (-5)  /* call not valid in the handle's current state */

typedef struct prop_s *prop_t;

typedef enum { PROP_TTI = 1, PROP_ELASTIC = 2 } prop_kind;

/* Storage type of gradient checkpoints (each snapshot has a power-of-two scale). */
typedef enum { PROP_CKPT_F32 = 0, PROP_CKPT_F16 = 1, PROP_CKPT_BF16 = 2 } prop_ckpt_dtype;

/* Discretised domain (the paper's Grid listing plus space/time order). */
typedef struct {
    int32_t ndim;         /* 2 (x, z) or 3 (x, y, z) */
    int64_t shape[3];     /* nx, ny, nz; ny = 1 when ndim = 2 */
    double  spacing[3];   /* hx, hy, hz in metres */
    double  origin[3];    /* metres */
    int32_t space_order;  /* even, 2..16: accuracy order of every first derivative */
    int32_t time_order;   /* 2 for PROP_TTI (leapfrog), 1 for PROP_ELASTIC (first-order system) */
    int32_t nbl;          /* absorbing-layer width in points, inside the shape, per face */
    double  dt;           /* time step in seconds; must not exceed prop_cfl_dt() */
    int32_t nt;           /* number of time steps */
    double  v_ref;        /* m/s: reference velocity of the absorbing-layer profile */
    int32_t free_surface; /* 0 = absorbing layer on every face; 1 = free surface on the top face
                             (small z; PROP_ELASTIC only, nbl >= space_order / 2): that face has no
                             absorbing layer, its nbl rows are vacuum (lambda = mu = 0, the given
                             density kept) and the surface is the normal-stress plane of row nbl.
                             Shot windows must then start at z index 0; the gradient is zero for vp
                             and vs in the vacuum rows.  (The paper names a free surface as an
                             equation on a sub-domain, the elastic section; the vacuum form keeps
                             the step, its transpose and its gradient unchanged in form.)
                             2 = free surface by the method of images (PROP_ELASTIC only, nbl >=
                             space_order - 2, a fluid (vs = 0) on rows nbl .. nbl + space_order / 2,
                             else PROP_EINVAL from prop_create / prop_set_model): as 1, and after
                             every step the normal stresses of the surface row nbl are set to zero
                             and the nbl rows above it take odd copies of tau_zz (about that row) and
                             of tau_xz, tau_yz (about the same plane); their density mirrors the
                             rows below (the input density of those rows is not used; the gradient
                             there is zero and flows to the mirrored rows).  In a fluid this is the
                             method of images exactly. */
} prop_grid;

/* Model parameters, DEVICE, dense (nz, ny, nx) over the whole grid.
 *   PROP_TTI:     p[0] = m = 1/vp^2 (s^2/m^2), p[1] = epsilon, p[2] = delta,
 *                 p[3] = theta (tilt from vertical, rad), p[4] = phi (azimuth, rad; ignored in 2D).
 *                 Requires epsilon >= delta everywhere (otherwise the system is unstable).
 *   PROP_ELASTIC: p[0] = vp (m/s), p[1] = vs (m/s), p[2] = rho (kg/m^3); p[3], p[4] unused.
 *                 lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2, buoyancy = 1/rho. */
typedef struct {
    const float *p[5];
} prop_model;

/* One shot (one source experiment).
 * The shot runs on a window of the grid: win_origin = index of its first node, win_shape = its
 * size (all zero = the whole grid).  The absorbing layer lies inside the window.  Coordinates are
 * absolute (grid frame) and must lie inside the window.
 * Sources: nsrc points, src_xyz HOST nsrc x ndim, src_wavelet DEVICE nt x nsrc (time-major).
 *   TTI: the same wavelet drives p and q.  Elastic: explosive source added to the three normal
 *   stresses.
 * Receivers: nrec points, rec_xyz HOST nrec x ndim.  TTI records p.  Elastic: rec_kind HOST
 *   (NULL = all 0): 0 = pressure, the trace txx + tyy + tzz at nodes; 1 = vz on its staggered grid. */
typedef struct {
    int64_t win_origin[3];
    int64_t win_shape[3];
    int32_t nsrc;
    const float *src_xyz;
    const float *src_wavelet;
    int32_t nrec;
    const float *rec_xyz;
    const int32_t *rec_kind;
} prop_shot;

/* Create a propagator for a grid and a model.  Validates the grid (even space order 2..16,
 * time order 2 for TTI / 1 for elastic, at least 2 points per active axis, positive spacing and
 * dt; a shot window needs at least 2 nbl + 2 points per active axis), computes the derived coefficients on the device (TTI: 1+2eps, sqrt(1+2delta),
 * symmetry axis; elastic: lambda, mu, buoyancy) and checks dt against the stability bound for
 * the model's largest velocity (PROP_EUNSTABLE).  stream is a hipStream_t (NULL = default).
 * On success *out owns device memory until prop_destroy. */
int prop_create(prop_t *out, prop_kind kind, const prop_grid *grid, const prop_model *model,
                void *stream);

/* Largest stable dt for a model whose largest velocity is vmax (TTI: vertical vp; elastic: vp)
 * and largest epsilon eps_max (TTI only).
 *   TTI:     dt <= 2 / (vmax sqrt((1 + 2 eps_max) S_D sum_a 1/h_a^2)), S_D = max_k (sum_j 2 a_j sin(jk))^2
 *   elastic: dt <= h_min / (vmax sqrt(ndim) sum_j |c_j|)
 * Returns a negative value for an invalid grid. */
double prop_cfl_dt(prop_kind kind, const prop_grid *grid, double vmax, double eps_max);

/* Replace the model (same grid); validates like prop_create.  Invalidates the checkpoints that a
 * saving prop_forward left on the handle (the model arrays may have new values). */
int prop_set_model(prop_t h, const prop_model *model);

/* Forward modelling of one shot: rec_out DEVICE nt x nrec receives the traces (row n is recorded
 * from the new level f^{n+1}).
 * TTI: a f^{n+1} = b f^n - c f^{n-1} + C (H0 p^n, Hz q^n) + P_s^T s^n for f in (p, q), with
 * a = m/dt^2 + eta/(2 dt), b = 2 m/dt^2, c = m/dt^2 - eta/(2 dt), eta the damping of the absorbing
 * layer, C = [[1+2 eps, sqrt(1+2 delta)], [sqrt(1+2 delta), 1]].
 * Elastic: the staggered velocity-stress scheme of the elastic section.
 * save_ckpt = 0: modelling only.  save_ckpt = n >= 1: the run also keeps, on the handle, the forward
 * checkpoints that prop_gradient / prop_image with n_ckpt = n and this ckpt_dtype would store (TTI:
 * n = 1 keeps the whole run in ckpt_dtype; elastic: ckpt_dtype must be PROP_CKPT_F32), so that a
 * gradient or image of the same shot under the same model skips its own forward sweep (the usual
 * FWI iteration: modelling, residual, gradient).  The traces are the same as with save_ckpt = 0.
 * The saved checkpoints stay valid until prop_set_model, the next saving prop_forward, or a gradient,
 * image or batched call that stores checkpoints of its own; prop_adjoint and plain forward calls
 * keep them.  ckpt_dtype is ignored when save_ckpt = 0. */
int prop_forward(prop_t h, const prop_shot *shot, float *rec_out, int32_t save_ckpt, prop_ckpt_dtype ckpt_dtype);

/* Exact transpose of prop_forward for the same shot (traces -> wavelet):
 * rec_in DEVICE nt x nrec, src_out DEVICE nt x nsrc (overwritten). */
int prop_adjoint(prop_t h, const prop_shot *shot, const float *rec_in, float *src_out);

/* Gradient of J = 1/2 sum_n ||d^n - d_obs^n||^2 over the shot's window.
 * PROP_ELASTIC: with respect to (vp, vs, rho); grad_m DEVICE receives three window-shaped dense
 * fields in that order; FP32 checkpoints of the nine fields every ceil(N / n_ckpt) steps
 * (ckpt_dtype must be PROP_CKPT_F32); the stored forward velocities of each segment give the
 * strains and the force of the adjoint-state imaging condition.
 * PROP_TTI: with respect to m over the shot's
 * window, given residual = d - d_obs (DEVICE nt x nrec): a forward run that stores n_ckpt evenly
 * spaced checkpoints of (p, q) at two time levels in ckpt_dtype with a power-of-two scale per
 * snapshot, then, segment by segment in reverse, an FP32 recomputation from the checkpoint and the
 * adjoint run with the imaging condition
 *     g = -(1/dt^2) sum_k sum_{f in p,q} f^k (y^k - 2 y^{k+1} + y^{k+2}).
 * The per-step levels f^k of the segment being processed are kept in FP32.
 * grad_m DEVICE, window-shaped dense (nz, ny, nx), overwritten.  n_ckpt >= 1; n_ckpt = 1 stores
 * the whole forward wavefield instead (one segment, no checkpoint), in ckpt_dtype (FP32, or
 * FP16/BF16 with a power-of-two scale per x-row), and takes two sweeps (forward with storage,
 * adjoint) instead of three: N x 2 fields x 4 B (FP32) or 2 B (FP16/BF16) per point of device
 * memory.
 * Checkpoint reuse (both kinds): when the last saving prop_forward ran this shot (same window, the
 * same source points and the same wavelet array, left unchanged) under the current model with
 * save_ckpt = n_ckpt and the same ckpt_dtype, its checkpoints are used and the forward sweep is
 * skipped (with n_ckpt = 1 only the adjoint sweep remains).  n_ckpt = 0 asks for exactly that reuse,
 * whatever n and dtype the forward saved with, and returns PROP_ESTATE when the handle holds no valid
 * checkpoints of this shot (none saved, or invalidated since; see prop_forward). */
int prop_gradient(prop_t h, const prop_shot *shot, const float *residual, float *grad_m,
                  int32_t n_ckpt, prop_ckpt_dtype ckpt_dtype);

/* TTI only.  Zero-lag cross-correlation image of one shot (reverse-time migration imaging
 * condition; the paper images with the adjoint-state gradient summed over shots, in its 3D
 * imaging section, and this condition is the conventional alternative):
 *     I = sum_{k=1}^{N} sum_{f in p,q} f^k y_f^k,
 * f the forward state driven by the shot's wavelet, y the adjoint state driven by rec_in (DEVICE
 * nt x nrec, e.g. recorded data) through the receivers.  Same checkpointing as prop_gradient;
 * image DEVICE window-shaped dense, overwritten. */
int prop_image(prop_t h, const prop_shot *shot, const float *rec_in, float *image, int32_t n_ckpt,
               prop_ckpt_dtype ckpt_dtype);

/* Many shots at once (TTI): all shots step in lockstep on their own windows; every stencil launch
 * covers the tiles of all shots of a group.  Shots are processed in groups that fit the device
 * memory.  rec_out[i] DEVICE nt x nrec_i. */
int prop_forward_batched(prop_t h, int32_t nshot, const prop_shot *shots, float *const *rec_out);

/* Batched gradient: per shot as prop_gradient, accumulated in FP64 into grad_global (DEVICE,
 * whole-grid dense (nz, ny, nx) doubles; NOT zeroed: the call adds), in shot order. */
int prop_gradient_batched(prop_t h, int32_t nshot, const prop_shot *shots,
                          const float *const *residual, double *grad_global, int32_t n_ckpt,
                          prop_ckpt_dtype ckpt_dtype);

/* Batched image: per shot as prop_image, accumulated in FP64 into image_global (DEVICE, whole-grid
 * dense doubles; the call adds), in shot order (the multi-shot image is the sum of the shot images). */
int prop_image_batched(prop_t h, int32_t nshot, const prop_shot *shots, const float *const *rec_in,
                       double *image_global, int32_t n_ckpt, prop_ckpt_dtype ckpt_dtype);

/* Copy a final wavefield of the last forward or adjoint call into out (DEVICE, window-shaped
 * dense).  TTI: 0 = p^N, 1 = q^N, 2 = p^{N-1}, 3 = q^{N-1} after prop_forward; after
 * prop_adjoint 0, 1 = y_p^1, y_q^1.  Elastic: 0..2 = vx, vy, vz; 3..8 = txx, tyy, tzz, txy, txz, tyz. */
int prop_read_state(prop_t h, int32_t field, float *out);

/* Kernel timing: when enabled, every stencil launch is bracketed by HIP events on the handle's
 * stream.  prop_kernel_time returns, for kernel class k (0 = the TTI gradient/mix pass, 1 = the
 * TTI divergence/update pass, 2 = elastic velocity pass, 3 = elastic stress pass, 4 = the fused
 * elastic step), the summed milliseconds and the number of launches since the last reset, and
 * names the class. */
int prop_set_timing(prop_t h, int32_t enable);
int prop_kernel_time(prop_t h, int32_t kclass, double *ms, int64_t *launches, const char **name);

/* Run-time options of a handle; they apply to the calls that follow.  They change how the work is
 * launched.  GRAPH, AUTOTUNE, TILE1/2, ZC, ZC2, XCD and BATCH_MB leave every result bitwise unchanged:
 * each point is computed by the same arithmetic whatever the tiling or launch mode.  SCHEME selects
 * another arrangement of the same operators: schemes 0 and 3 give bitwise equal results, and the
 * others agree with them to FP32 rounding (sums formed in another order).
 *   PROP_OPT_GRAPH     0/1 (default 0): record each run of time steps between two host checks
 *                      (the non-finite watchdog every 500 steps; each gradient segment) in a HIP
 *                      graph and launch it as one unit.  Ignored while kernel timing is on.
 *   PROP_OPT_AUTOTUNE  0/1 (default 0): TTI only; on the first call for a set of window shapes
 *                      and a direction, time both tile variants of each stencil pass at three
 *                      z-chunk lengths and keep the fastest (cached on the handle).
 *   PROP_OPT_TILE1/2   0 or 1 (default 1): tile variant of TTI pass 1 / pass 2 when not
 *                      autotuning (0: 64 x 8 threads, 1: 64 x 16 threads; the fused pass uses
 *                      TILE2 and a 64 x 16 tile either way, 0: 512 threads of two rows,
 *                      1: 1024 threads of one row).  Elastic handles on 3D grids read TILE1 for
 *                      the velocity pass (default 0) and TILE2 for the stress pass and the
 *                      gradient's imaging condition (default 1), 0: 64 x 8 tiles, 1: 64 x 16.
 *                      Traces, states and adjoint traces are bitwise the same either way; the
 *                      elastic gradient may differ at rounding level (1e-7) with TILE2.
 *   PROP_OPT_ZC        z-chunk length in planes when not autotuning, 0 = automatic (default).
 *   PROP_OPT_ZC2       z-chunk of TTI pass 2 when not autotuning, 0 = that of pass 1 (default);
 *                      elastic: z-chunk of the stress pass, 0 = that of the velocity pass.
 *   PROP_OPT_XCD       0/1 (default 0): deal the tiles over the 8 XCDs in contiguous ranges.
 *   PROP_OPT_EL_FUSED  0/1 (default 0): elastic prop_forward on 3D grids up to space order 8 runs
 *                      one fused velocity-stress launch a step (kernel class 4) instead of the
 *                      velocity and stress passes (classes 2 and 3): the same expressions, so the
 *                      same bits, and fewer HBM bytes, but slower on this chip (its register and
 *                      LDS budget allows only 32 x 16 tiles and half the waves per CU).  The
 *                      adjoint and the gradient always run the two passes.
 *   PROP_OPT_BATCH_MB  device-memory budget of the batched shot-group planner in MiB,
 *                      0 = 85 % of the free memory (default).
 *   PROP_OPT_SCHEME    TTI step scheme: 0 = two passes, pass 1 stores the six components of
 *                      (I - n n^T) grad p and n n^T grad q (value 1 is not used: PROP_EINVAL);
 *                      2 = one fused pass, the projections stay on chip (space order <= 12 and x-y
 *                      planes below 4 GiB, else PROP_EINVAL; kernel class 1 then times the fused
 *                      pass and class 0 is unused); 3 = two passes, pass 1 stores the three
 *                      components of (I - n n^T) grad p and the scalar n . grad q, and pass 2
 *                      re-forms n n^T grad q from it and the axis (bitwise equal to 0, 8 bytes
 *                      a point fewer); 4 = two fused single-field passes, h = H0 p (or H0 w_p)
 *                      into a temporary, then Hz q (or Hz w_q) and the update (space order <= 12
 *                      and x-y planes below 4 GiB; bitwise equal to 2; kernel classes 0 and 1).
 *                      Default: 2 up to space order 8, 4 up to 12 (3 when the planes are 4 GiB or
 *                      more), 0 above.
 * Read-only (prop_get_option): PROP_INFO_TILE1/2 and PROP_INFO_ZC1/2, the variant and z-chunk
 * used by the last TTI call; PROP_INFO_GRAPHS, graphs launched since create; PROP_INFO_GROUPS,
 * shot groups of the last batched call.  Unknown options give PROP_EINVAL. */
enum {
    PROP_OPT_GRAPH = 1,
    PROP_OPT_AUTOTUNE = 2,
    PROP_OPT_TILE1 = 3,
    PROP_OPT_TILE2 = 4,
    PROP_OPT_ZC = 5,
    PROP_OPT_XCD = 6,
    PROP_OPT_BATCH_MB = 7,
    PROP_OPT_SCHEME = 8,
    PROP_OPT_ZC2 = 9,
    PROP_OPT_EL_FUSED = 10,
    PROP_INFO_TILE1 = 101,
    PROP_INFO_TILE2 = 102,
    PROP_INFO_ZC1 = 103,
    PROP_INFO_ZC2 = 104,
    PROP_INFO_GRAPHS = 105,
    PROP_INFO_GROUPS = 106
};
int prop_set_option(prop_t h, int32_t option, int64_t value);
int prop_get_option(prop_t h, int32_t option, int64_t *value);

/* Checkpoint codec (the packing used by prop_gradient), exposed for testing:
 * encode n FP32 values (DEVICE) with scale s = 2^ceil(log2 max|f|) (1 for all-zero input) into
 * codes (DEVICE: n uint16 for F16/BF16, round to nearest even; n floats for F32, s = 1), writing s
 * to *scale_dev (DEVICE float).  decode: f = s * code. */
int prop_ckpt_encode(const float *f, int64_t n, prop_ckpt_dtype dtype, void *codes, float *scale_dev,
                     void *stream);
int prop_ckpt_decode(const void *codes, const float *scale_dev, int64_t n, prop_ckpt_dtype dtype,
                     float *f, void *stream);

/* Row codecs of the gradient's stores, exposed for testing.  Fields are dense (nz, ny, nx) FP32
 * arrays (DEVICE); every x-row (fixed y, z) gets its own power-of-two scale s = 2^k,
 * k = ceil(log2 max|row|) clamped to [-126, 127] (1 for an all-zero row), and its values f * (1/s)
 * (an exact FP32 product) round to nearest even FP16 (dtype F16) or BF16 (dtype BF16).
 *   pair = 1: the checkpoint pair of one field at two time levels: a = cur, b = cur - prev (the FP32
 *             difference; the time derivative it carries is much smaller than either level);
 *   pair = 0: two independent fields a = cur, b = prev (the per-step store of p and q when the
 *             gradient keeps the whole run).
 * codes_a, codes_b DEVICE nz*ny*nx uint16; scale_a, scale_b DEVICE nz*ny floats.  Requires
 * 1 <= ny, nz <= 65535 and 1 <= nx <= 2^31 - 1 (PROP_EINVAL otherwise).  Enqueued on stream. */
int prop_ckpt_encode_rows(const float *cur, const float *prev, int64_t nx, int64_t ny, int64_t nz, int32_t pair,
                          prop_ckpt_dtype dtype, uint16_t *codes_a, uint16_t *codes_b, float *scale_a,
                          float *scale_b, void *stream);
/* Inverse of the pair codec: cur = s_a a, prev = cur - s_b b (FP32), dense (nz, ny, nx) DEVICE. */
int prop_ckpt_decode_rows(const uint16_t *codes_a, const uint16_t *codes_b, const float *scale_a,
                          const float *scale_b, int64_t nx, int64_t ny, int64_t nz, prop_ckpt_dtype dtype,
                          float *cur, float *prev, void *stream);

/* FP64 inner product of two FP32 device vectors (deterministic order); blocks until done. */
int prop_dot_f64(const float *a, const float *b, int64_t n, double *result, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): prop_dot_f64 without any allocation.  Same arguments, kernels and
 * result (bitwise) as prop_dot_f64, which allocates its partial sums per call.  The scratch is a
 * static device array of 1025 doubles per device (the partial sums of the kernels' fixed grid of
 * 1024 blocks and the result), held until the process ends; its size does not depend on n, and a
 * build whose kernels would need more fails with PROP_EINVAL.  Every call on a device uses that
 * device's array: calls that overlap on one device (several threads or streams) race.  stream must
 * belong to the current device.  Blocks until the result is on the host. */
int prop_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *result, void *stream);

int prop_destroy(prop_t h);

/* Message of the last error on the calling thread ("" if none). */
const char *prop_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PROP_H */
