// Per-shot job descriptors and host-side launch entry points of the propagator kernels.
#pragma once
#include "common.h"

#include <hip/hip_fp16.h>

// One TTI shot window.  cur/prev wavefields ping-pong between p[0]/p[1] (and q) with the step
// parity: the new level overwrites the level two steps back.
struct TTIJob {
    Win w;
    float *p[2], *q[2];           // wavefields (state layout)
    float *wmix[2][2];            // adjoint only: w = C y of the newest level (components p, q), the
                                  // input of pass 1; double-buffered with the step parity (pass 1
                                  // reads wmix[par], pass 2 writes wmix[par ^ 1]) because the fused
                                  // and split passes read w on tile halos while they write the new w
    float *t[3], *s[3];           // pass-1 outputs (state layout): six-field scheme: the vectors
                                  // (I - n n^T) grad u and n n^T grad v; four-field scheme: t as
                                  // six-field, s[0] = n . grad v; split scheme: t[0] = h = H0 u
    const float *m, *A, *B;       // m, 1 + 2 eps, sqrt(1 + 2 delta) (model layout)
    const float *nx, *ny;         // symmetry axis (model layout); n_z = sqrt(1 - n_x^2 - n_y^2) >= 0
    const float *ex, *ey, *ez;    // absorbing layer: eta/(2 dt) per window axis
    float *grad;                  // imaging-condition accumulator (state layout) or null
    int image;                    // imaging condition: 0 = gradient w.r.t. m, 1 = zero-lag cross-correlation
    float *seg;                   // segment store (FP32): per step 2 fields (p then q) of seg_field elems
    int64_t seg_field;            // elements of one stored field (= plane pitch * nz)
    int seg_dtype;                // segment store type: 0 FP32 (seg), 1 FP16 / 2 BF16 (seg16, segsc)
    uint16_t *seg16;              // 16-bit store: per step 2 fields of seg16_field codes, dense (nz, ny, nx)
    float *segsc;                 // ... and 2 x segsc_field power-of-two scales, one per x-row
    int64_t seg16_field, segsc_field;
};

__device__ __forceinline__ float code16_to_f32(uint16_t c, int dtype)
{
    return dtype == 1 ? __half2float(__ushort_as_half(c)) : __uint_as_float((unsigned)c << 16);
}

// The stored forward levels (p, q) of segment step s at window point (x, y, z), state index si.
__device__ __forceinline__ void seg_load(const TTIJob &J, int s, int x, int y, int z, int64_t si, float &fp, float &fq)
{
    if (J.seg_dtype == 0) {
        const float *sp = J.seg + (int64_t)s * 2 * J.seg_field;
        fp = gld(sp, si);
        fq = gld(sp, J.seg_field + si);
    } else {
        typedef __attribute__((address_space(1))) const uint16_t gu16;
        const int64_t r = (int64_t)z * J.w.ny + y, di = r * J.w.nx + x;
        const gu16 *c = (const gu16 *)(J.seg16 + (int64_t)s * 2 * J.seg16_field);
        const float *sc = J.segsc + (int64_t)s * 2 * J.segsc_field;
        fp = gld(sc, r) * code16_to_f32(c[di], J.seg_dtype);
        fq = gld(sc, J.segsc_field + r) * code16_to_f32(c[J.seg16_field + di], J.seg_dtype);
    }
}

// One elastic shot window (fields in state layout; parameters in model layout).
struct ElJob {
    Win w;
    float *v[3];                  // vx, vy, vz
    float *vo[3];                 // forward velocity pass: where v+ goes (v itself for a step in place)
    float *t[6];                  // txx, tyy, tzz, txy, txz, tyz
    float *aux[6];                // adjoint: stiffness-weighted stresses sigma = C (g tau~)
    float *u[3];                  // adjoint: buoyancy-weighted velocities u = bbar (g v~)
    const float *lam, *mu, *b;    // lambda, mu, buoyancy
    const float *gx, *gy, *gz;    // absorbing layer: exp(-kappa_a dt) per window axis
};

// The fused elastic step (3D): reads the state (vi, ti) and writes the next state (vo, to); the two
// sets must not overlap.
struct ElFusedJob {
    Win w;
    const float *vi[3], *ti[6];   // v and tau of the step's start (state layout)
    float *vo[3], *to[6];         // v+ and tau+ (state layout)
    const float *lam, *mu, *b;    // lambda, mu, buoyancy (model layout)
    const float *gx, *gy, *gz;    // absorbing layer: exp(-kappa_a dt) per window axis
};

// Elastic gradient: the imaging condition of one adjoint step, and the final spread to the nodes.
struct ElGradJob {
    Win w;
    const float *vn1[3];          // forward velocities after the step (stored), v^{n+1}
    const float *vn0[3];          // forward velocities before the step, v^n
    const float *tt[6];           // adjoint stresses after the step (receiver residuals injected)
    const float *vt[3];           // adjoint velocities after the transposed velocity update, g v~''
    const float *b;               // buoyancy (model layout)
    const float *gx, *gy, *gz;    // absorbing layer factors per window axis
    float *acc[8];                // accumulators: lambda, mu (normal part) at nodes; mubar at the xy,
                                  // xz, yz shear positions; bbar at the x, y, z velocity positions
};

enum { K2_FWD = 0, K2_FWD_STORE = 1, K2_ADJ = 2, K2_ADJ_IC = 3 };
// Schemes of the TTI step: two passes with six-field temporaries, one fused pass (projections
// kept on chip), two passes with four temporaries: t and the scalar n . grad v, from which pass 2
// re-forms s = n (n . grad v), or two fused single-field passes (h = H0 u, then Hz v and the
// update; one temporary, h).  (Value 1 is not used.)
enum { TTI_SIX = 0, TTI_FUSED = 2, TTI_FOUR = 3, TTI_SPLIT = 4 };

// shape: tile-shape variant of the pass; tti_tile_rows gives its tile height.
void launch_tti_pass1(int R, int scheme, int shape, bool adjoint, const TTIJob *jobs, const Tile *tiles, int ntiles,
                      int zc, int par, const Weights &W, hipStream_t st);
void launch_tti_pass2(int R, int scheme, int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles,
                      int zc, int par, const Weights &W, float idt2, int seg_step, hipStream_t st);
// The fused scheme runs only the second launch (pass 1 is a no-op).
int tti_tile_rows(int R, int scheme, int pass, int shape);
int tti_fused_max_radius();
// The split scheme: part 0 = pass A (h = H0 u, written to t[0]), part 1 = pass B (Hz v, update).
int tti_split_max_radius();
void launch_tti_split(int R, int part, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, float idt2, int seg_step, hipStream_t st);
void launch_tti_fused(int R, int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, float idt2, int seg_step, hipStream_t st);

enum { EL_FWD = 0, EL_ADJ = 1 };
// The fused elastic step supports space orders up to 2 * el_fused_max_radius() on 3D windows; its
// tiles are EF_TX x EF_TY (one block of EF_TX * EF_TY threads per CU: 256 registers a lane).
#define EF_TX 32
#define EF_TY 16
int el_fused_max_radius();
void launch_el_fused(int R, const ElFusedJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt,
                     hipStream_t st);
// by: tile rows of the launch (el_tile_rows); the tiles must have been made with that height.
void launch_el_vel(int R, int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc,
                   const Weights &W, float dt, hipStream_t st);
void launch_el_stress(int R, int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc,
                      const Weights &W, float dt, hipStream_t st);
void launch_el_grad_ic(int R, int by, const ElGradJob *job, const Tile *tiles, int ntiles, int zc, const Weights &W,
                       float dt, hipStream_t st);
// Spread the accumulators to the nodes (transpose of the half-node averages) and convert to
// (vp, vs, rho): out = three dense window fields.  Rows z < nvac are vacuum (lambda = mu = 0 there,
// independent of vp, vs and rho).
// nvac: vacuum rows above a free surface (their lambda, mu are fixed); nimg: the surface row of an
// image free surface (0: none), whose image rows copy the buoyancy of the rows below.
void launch_el_grad_finish(const ElGradJob *job, const Win &w, int ndim, int nvac, int nimg, const float *vp,
                           const float *vs,
                           const float *rho, float *out, hipStream_t st);
int el_tile_rows(int R, int ndim);
