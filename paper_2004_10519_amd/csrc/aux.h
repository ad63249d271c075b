// Host-side entry points of the auxiliary kernels (sparse operators, codec, reductions).
#pragma once
#include "common.h"

// Node-wise injection plan (compressed rows): row r adds sum_{e in [ptr[r], ptr[r+1])} w[e] data[col[e]]
// to the state node node[r].  TTI rows also carry the model index of the node and its damping term
// eta/(2dt), so the kernel can divide by a = m/dt^2 + eta/(2dt).
struct Csr {
    int nrows;
    const int64_t *node;
    const int64_t *mnode;
    const float *e;
    const int *ptr;
    const int *col;
    const float *w;
};

// Multilinear gather plan: point o reads nc corners idx[o*nc + c] with weights w[o*nc + c] and
// writes output column pos[o].
struct Gather {
    int n, nc;
    const int64_t *idx;
    const float *w;
    const int *pos;
};

// Shot-group plans: every row/point carries the index of its shot in the group's job table.
struct BCsr {
    int nrows;
    const int *shot;
    const int64_t *node;
    const int64_t *mnode;
    const float *e;
    const int *ptr;
    const int *col;
    const float *w;
};
struct BGather {
    int n, nc;
    const int *shot;
    const int64_t *idx;
    const float *w;
    const int *pos;
};
struct TTIJob;
// TTI source injection into p, q of the new level (and its segment copy when seg_step >= 0);
// data[shot] is that shot's wavelet array (nt x npt[shot]).
void aux_tti_src(const BCsr &c, const TTIJob *jobs, int par, const float *const *data, const int *npt, int n,
                 float idt2, int seg_step, hipStream_t st);
// TTI adjoint receiver injection into y_p (+ w = C y, + imaging condition when ic != 0).
void aux_tti_rec_adj(const BCsr &c, const TTIJob *jobs, int par, const float *const *data, const int *npt, int n,
                     float idt2, int ic, int seg_step, hipStream_t st);
// TTI gather: mode 0 = p of the new level (traces), 1 = y_p + y_q of the new level (source adjoint).
void aux_tti_gather(const BGather &g, const TTIJob *jobs, int par, int mode, float *const *out, const int *npt, int n,
                    hipStream_t st);

void aux_tti_inject(const Csr &c, const float *data, float idt2, const float *m, float *d0, float *d1, float *d2,
                    float *d3, hipStream_t st);
void aux_tti_inject_adj(const Csr &c, const float *data, float idt2, const float *m, const float *A, const float *B,
                        float *yp, float *wp, float *wq, float *grad, const float *fpk, hipStream_t st);
void aux_el_inject(const Csr &c, const float *data, float scale, float *d0, float *d1, float *d2, hipStream_t st);
// Elastic adjoint: sigma_ii = lambda tr(g tau~) + 2 mu g tau~_ii at the plan's nodes (after an injection
// into tau~_ii there); g = gx[x] gy[y] gz[z] of the window, lambda and mu at the plan's model nodes.
void aux_el_remix(const Csr &c, const Win &w, const float *gx, const float *gy, const float *gz, const float *lam,
                  const float *mu, const float *t0, const float *t1, const float *t2, float *a0, float *a1, float *a2,
                  hipStream_t st);
// Free surface by the method of images: the forward fill of the surface row ks and the rows above
// it (tyz NULL in 2D; tyy is formed in 2D too), and its transpose on the adjoint stresses followed by sigma = C (g tau~)
// on rows 0 .. 2 ks.
struct ElImage {
    float *t[6];                  // adjoint stresses tau~ (state layout)
    float *s[6];                  // sigma = C (g tau~) (state layout)
    const float *lam, *mu;        // model layout
    const float *gx, *gy, *gz;    // absorbing factors per window axis
};
void aux_el_image_fill(const Win &w, int ks, float *txx, float *tyy, float *tzz, float *txz, float *tyz,
                       hipStream_t st);
void aux_el_image_fold(const Win &w, int ks, int ndim, const ElImage &J, hipStream_t st);
void aux_gather(const Gather &g, const float *f0, const float *f1, const float *f2, float scale, float *out,
                hipStream_t st);
void aux_fill(float *p, int64_t n, float v, hipStream_t st);
void aux_fill_u32(unsigned *p, int n, unsigned v, hipStream_t st);
void aux_absmax(const float *f, int64_t n, unsigned *out, hipStream_t st);
void aux_encode(const float *f, int64_t n, const unsigned *maxbits, int dtype, uint16_t *codes, float *scale_out,
                hipStream_t st);
void aux_decode(const uint16_t *codes, const float *scale, int64_t n, int dtype, float *f, hipStream_t st);
void aux_absmax_win(const float *f, const Win &w, unsigned *out, hipStream_t st);
void aux_encode_win(const float *f, const Win &w, const unsigned *maxbits, int dtype, void *codes, float *scale_out,
                    hipStream_t st);
void aux_decode_win(const void *codes, const float *scale, const Win &w, int dtype, float *f, hipStream_t st);
// Gradient checkpoint codec (FP16 = 1 / BF16 = 2): a = cur, b = cur - prev, per-x-row power-of-two
// scales; ca, cb: dense window codes; sca, scb: ny*nz scales each.
void aux_ckpt_pair_encode(const float *cur, const float *prev, const Win &w, int dtype, uint16_t *ca, uint16_t *cb,
                          float *sca, float *scb, hipStream_t st);
void aux_ckpt_pair_decode(const uint16_t *ca, const uint16_t *cb, const float *sca, const float *scb, const Win &w,
                          int dtype, float *cur, float *prev, hipStream_t st);
// 16-bit segment store of one step: p, q rounded to FP16 (dtype 1) / BF16 (dtype 2) with per-x-row
// power-of-two scales; codes dense (nz, ny, nx).
void aux_encode_rows2(const float *p, const float *q, const Win &w, int dtype, uint16_t *cp, uint16_t *cq, float *sp,
                      float *sq, hipStream_t st);
void aux_dot_f64(const float *a, const float *b, int64_t n, double *part, double *out, hipStream_t st);
int aux_dot_blocks();
void aux_tti_prep(const float *m, const float *eps, const float *dl, const float *th, const float *ph, int64_t n,
                  int ndim, float *A, float *B, float *nx, float *ny, unsigned *stats, hipStream_t st);
// Elastic parameters (lambda, mu, b) from (vp, vs, rho); stats[2] gets flag 4 when vs > 0 on a plane
// row in [fluid_lo, fluid_hi) (rows of `plane` points).
void aux_el_prep(const float *vp, const float *vs, const float *rho, int64_t n, float *lam, float *mu, float *b,
                 unsigned *stats, int64_t plane, int fluid_lo, int fluid_hi, hipStream_t st);
void aux_nonfinite_win(const float *f, const Win &w, unsigned *flag, hipStream_t st);
void aux_copy_out(const float *src, const Win &w, float *dst, hipStream_t st);
void aux_accum_f64(const float *src, const Win &w, double *dst, hipStream_t st);
