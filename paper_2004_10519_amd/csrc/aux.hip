// Sparse source/receiver operators, checkpoint codec, reductions and model preprocessing (gfx950).
#include "aux.h"
#include "jobs.h"

#include <hip/hip_fp16.h>

#include <math.h>

namespace {

constexpr int BS = 256;

__device__ __forceinline__ float csr_row_value(const Csr &c, int r, const float *data)
{
    float v = 0.f;
    for (int e = c.ptr[r]; e < c.ptr[r + 1]; ++e) v += c.w[e] * data[c.col[e]];
    return v;
}

// TTI injection of sum_e w_e data[col_e] into up to four fields at node r, divided by
// a = m/dt^2 + eta/(2dt) at the node (the source term enters a f+ = ... + P^T s).
__global__ void k_tti_inject(Csr c, const float *__restrict__ data, float idt2, const float *__restrict__ m,
                             float *d0, float *d1, float *d2, float *d3)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const float a = m[c.mnode[r]] * idt2 + c.e[r];
    const float v = csr_row_value(c, r, data) / a;
    const int64_t n = c.node[r];
    if (d0) d0[n] += v;
    if (d1) d1[n] += v;
    if (d2) d2[n] += v;
    if (d3) d3[n] += v;
}

// Adjoint receiver injection into y_p (node-wise gather, deterministic); keeps w = C y in step
// (w_p += (1+2eps) v, w_q += sqrt(1+2delta) v) and adds the imaging condition's share of the
// injected increment: g -= (1/dt^2) f_p^k * increment.
__global__ void k_tti_inject_adj(Csr c, const float *__restrict__ data, float idt2, const float *__restrict__ m,
                                 const float *__restrict__ A, const float *__restrict__ B, float *yp, float *wp,
                                 float *wq, float *grad, const float *__restrict__ fpk)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const int64_t mn = c.mnode[r];
    const float a = m[mn] * idt2 + c.e[r];
    const float v = csr_row_value(c, r, data) / a;
    const int64_t n = c.node[r];
    yp[n] += v;
    wp[n] += A[mn] * v;
    wq[n] += B[mn] * v;
    if (grad) grad[n] -= idt2 * fpk[n] * v;
}

// Elastic injection: d_i[node] += scale * sum_e w_e data[col_e].
__global__ void k_el_inject(Csr c, const float *__restrict__ data, float scale, float *d0, float *d1, float *d2)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const float v = scale * csr_row_value(c, r, data);
    const int64_t n = c.node[r];
    if (d0) d0[n] += v;
    if (d1) d1[n] += v;
    if (d2) d2[n] += v;
}

// Elastic adjoint: the diagonal of sigma = C (g tau~) at the nodes of an injection plan, recomputed
// from tau~ after receiver residuals were added there (the stress pass formed sigma from tau~ before
// the injection; the shear components are not injected).  Same arithmetic as the stress pass.
__global__ void k_el_remix(Csr c, Win w, const float *__restrict__ gx, const float *__restrict__ gy,
                           const float *__restrict__ gz, const float *__restrict__ lam, const float *__restrict__ mu,
                           const float *t0, const float *t1, const float *t2, float *a0, float *a1, float *a2)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const int64_t si = c.node[r], mi = c.mnode[r];
    const int z = (int)(si / w.sy);
    const int64_t rem = si - (int64_t)z * w.sy;
    const int y = (int)(rem / w.sx), x = (int)(rem - (int64_t)y * w.sx);
    const float g = gx[x] * gy[y] * gz[z];
    const float s0 = g * t0[si], s1 = g * t1[si], s2 = g * t2[si];
    const float lt = lam[mi] * (s0 + s1 + s2), m2 = 2.f * mu[mi];
    a0[si] = lt + m2 * s0;
    a1[si] = lt + m2 * s1;
    a2[si] = lt + m2 * s2;
}

// Free surface by the method of images (surface node row ks, a fluid): after a forward step the
// surface row's normal stresses are zero (txx, tyy, tzz) and the rows above take odd copies of the
// tractions, tzz[ks - k] = -tzz[ks + k], and for txz, tyz, whose storage row i holds the half row
// i + 1/2, tc[ks - k] = -tc[ks + k - 1] (k = 1 .. ks).  One thread per (x, y, k); k = 0 clears the
// surface row.  Rows read (> ks for tzz, >= ks for txz, tyz) and rows written (< ks, and row ks by
// k = 0 only) are disjoint.
__global__ void k_el_image_fill(Win w, int ks, float *txx, float *tyy, float *tzz, float *txz, float *tyz)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
    if (x >= w.nx) return;
    if (k == 0) {
        const int64_t s0 = sidx(w, x, y, ks);
        txx[s0] = 0.f;
        if (tyy) tyy[s0] = 0.f;
        tzz[s0] = 0.f;
        return;
    }
    const int64_t lo = sidx(w, x, y, ks - k);
    tzz[lo] = -tzz[sidx(w, x, y, ks + k)];
    txz[lo] = -txz[sidx(w, x, y, ks + k - 1)];
    if (tyz) tyz[lo] = -tyz[sidx(w, x, y, ks + k - 1)];
}

// Transpose of k_el_image_fill on the adjoint stresses tau~ (one thread per (x, y, k), like the
// fill): each image row hands its value, negated, to the row it copies and is cleared (k >= 1);
// k = 0 clears the normal stresses of row ks.  Every thread touches its own rows.
__global__ void k_el_image_fold(Win w, int ks, int ndim, ElImage J)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
    if (x >= w.nx) return;
    float *const tzz = J.t[2], *const txz = J.t[4], *const tyz = J.t[5];
    if (k == 0) {
        const int64_t s0 = sidx(w, x, y, ks);
        J.t[0][s0] = 0.f;
        J.t[1][s0] = 0.f;
        tzz[s0] = 0.f;
        return;
    }
    const int64_t lo = sidx(w, x, y, ks - k), hz = sidx(w, x, y, ks + k), hs = sidx(w, x, y, ks + k - 1);
    tzz[hz] -= tzz[lo];
    tzz[lo] = 0.f;
    txz[hs] -= txz[lo];
    txz[lo] = 0.f;
    if (ndim == 3) {
        tyz[hs] -= tyz[lo];
        tyz[lo] = 0.f;
    }
}

// sigma = C (g tau~) of the rows the fold touched (z = 0 .. 2 ks; one thread per point), with the
// expressions of the transposed stress pass's epilogue, for the transposed velocity pass.
__global__ void k_el_image_sigma(Win w, int ndim, ElImage J)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= w.nx || z >= w.nz) return;
    const int64_t si = sidx(w, x, y, z), mi = midx(w, x, y, z);
    const int64_t ox = x + 1 < w.nx ? 1 : 0, oy = y + 1 < w.ny ? w.mx : 0, oz = z + 1 < w.nz ? w.my : 0;
    const float g = J.gx[x] * J.gy[y] * J.gz[z];
    const float s0 = g * J.t[0][si], s1 = g * J.t[1][si], s2 = g * J.t[2][si];
    const float lam = J.lam[mi], mu0 = J.mu[mi];
    const float lt = lam * (s0 + s1 + s2), m2 = 2.f * mu0;
    J.s[0][si] = lt + m2 * s0;
    J.s[1][si] = lt + m2 * s1;
    J.s[2][si] = lt + m2 * s2;
    const float mx_ = J.mu[mi + ox], mz_ = J.mu[mi + oz];
    const float mxz = 0.25f * (mu0 + mx_ + mz_ + J.mu[mi + ox + oz]);
    J.s[4][si] = mxz * (g * J.t[4][si]);
    if (ndim == 3) {
        const float my_ = J.mu[mi + oy];
        const float myz = 0.25f * (mu0 + my_ + mz_ + J.mu[mi + oy + oz]);
        J.s[5][si] = myz * (g * J.t[5][si]);
    }
}

// Multilinear gather: out[pos_o] = scale * sum_c w_oc (f0 + f1 + f2)[idx_oc].  One point per lane.
// Multilinear gathers run one corner per lane: the nc = 2^d lanes of a point (a power of two that
// divides the wavefront) each load one corner value times its weight, and a butterfly of lane shuffles
// within the group sums them in a fixed order (every lane takes part in the shuffles, so lanes past
// the last point carry zeros instead of returning early); the group's first lane writes the result.
__device__ __forceinline__ float group_sum(float v, int nc)
{
    for (int o = nc >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ void k_gather(Gather g, const float *__restrict__ f0, const float *__restrict__ f1,
                         const float *__restrict__ f2, float scale, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t o = t / g.nc;
    const bool on = o < g.n;
    float s = 0.f;
    if (on) {
        const int64_t i = g.idx[t];
        float v = f0[i];
        if (f1) v += f1[i];
        if (f2) v += f2[i];
        s = g.w[t] * v;
    }
    s = group_sum(s, g.nc);
    if (on && t % g.nc == 0) out[g.pos[o]] = scale * s;
}

__device__ __forceinline__ float bcsr_row_value(const BCsr &c, int r, const float *data)
{
    float v = 0.f;
    for (int e = c.ptr[r]; e < c.ptr[r + 1]; ++e) v += c.w[e] * data[c.col[e]];
    return v;
}

__global__ void k_tti_src(BCsr c, const TTIJob *__restrict__ jobs, int par, const float *const *__restrict__ data,
                          const int *__restrict__ npt, int n, float idt2, int seg_step)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const int sh = c.shot[r];
    const TTIJob &J = jobs[sh];
    const float a = J.m[c.mnode[r]] * idt2 + c.e[r];
    const float v = bcsr_row_value(c, r, data[sh] + (int64_t)n * npt[sh]) / a;
    const int64_t nd = c.node[r];
    J.p[par ^ 1][nd] += v;
    J.q[par ^ 1][nd] += v;
    if (seg_step >= 0 && J.seg_dtype == 0) {   // (a 16-bit store is encoded after the injection)
        float *sp = J.seg + (int64_t)seg_step * 2 * J.seg_field;
        sp[nd] += v;
        sp[J.seg_field + nd] += v;
    }
}

__global__ void k_tti_rec_adj(BCsr c, const TTIJob *__restrict__ jobs, int par, const float *const *__restrict__ data,
                              const int *__restrict__ npt, int n, float idt2, int ic, int seg_step)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= c.nrows) return;
    const int sh = c.shot[r];
    const TTIJob &J = jobs[sh];
    const int64_t mn = c.mnode[r];
    const float a = J.m[mn] * idt2 + c.e[r];
    const float v = bcsr_row_value(c, r, data[sh] + (int64_t)n * npt[sh]) / a;
    const int64_t nd = c.node[r];
    J.p[par ^ 1][nd] += v;
    J.wmix[par ^ 1][0][nd] += J.A[mn] * v;
    J.wmix[par ^ 1][1][nd] += J.B[mn] * v;
    if (ic) {   // the injected share of y^k in the imaging condition (f_p^k times it)
        const int64_t z = nd / J.w.sy, rem = nd - z * J.w.sy, y = rem / J.w.sx, x = rem - y * J.w.sx;
        float fp, fq;
        seg_load(J, seg_step, (int)x, (int)y, (int)z, nd, fp, fq);
        if (J.image) J.grad[nd] += fp * v;
        else J.grad[nd] -= idt2 * fp * v;
    }
}

__global__ void k_tti_gather(BGather g, const TTIJob *__restrict__ jobs, int par, int mode, float *const *__restrict__ out,
                             const int *__restrict__ npt, int n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t o = t / g.nc;
    const bool on = o < g.n;
    float s = 0.f;
    int sh = 0;
    if (on) {
        sh = g.shot[o];
        const TTIJob &J = jobs[sh];
        const int64_t i = g.idx[t];
        const float v = mode == 0 ? J.p[par ^ 1][i] : J.p[par ^ 1][i] + J.q[par ^ 1][i];
        s = g.w[t] * v;
    }
    s = group_sum(s, g.nc);
    if (on && t % g.nc == 0) out[sh][(int64_t)n * npt[sh] + g.pos[o]] = s;
}

__global__ void k_fill(float *p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(unsigned *p, int n, unsigned v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// max |f| as ordered bits (non-negative floats order like their bit patterns; NaN sorts above Inf).
__global__ void k_absmax(const float *__restrict__ f, int64_t n, unsigned *out)
{
    __shared__ unsigned sm[BS];
    unsigned mx = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, __float_as_uint(f[i]) & 0x7fffffffu);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sm[0]);
}

// Power-of-two scale s = 2^k, k = ceil(log2 max|f|) clamped to FP32's normal exponents [-126, 127]
// (1 for an all-zero field), built from the exponent bits so that 1/s is exact and finite even
// when the maximum is subnormal.
__device__ __forceinline__ float pow2_scale(unsigned maxbits)
{
    if (maxbits == 0) return 1.0f;
    const int eb = (int)((maxbits >> 23) & 0xffu);
    const unsigned mb = maxbits & 0x7fffffu;
    int k = eb == 0 ? -126 : eb - 127 + (mb != 0u ? 1 : 0);
    k = max(-126, min(k, 127));
    return __uint_as_float((unsigned)(k + 127) << 23);
}

// Round-to-nearest-even FP32 -> BF16 by the rounding-bias method.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    const unsigned bias = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

__global__ void k_encode(const float *__restrict__ f, int64_t n, const unsigned *__restrict__ maxbits, int dtype,
                         uint16_t *__restrict__ codes, float *__restrict__ scale_out)
{
    const float s = pow2_scale(*maxbits);
    const float rs = 1.0f / s;   // exact: power of two
    if (blockIdx.x == 0 && threadIdx.x == 0 && scale_out) *scale_out = s;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = f[i] * rs;
        codes[i] = dtype == 1 ? __half_as_ushort(__float2half_rn(x)) : f32_to_bf16_rne(x);
    }
}

__global__ void k_decode(const uint16_t *__restrict__ codes, const float *__restrict__ scale, int64_t n, int dtype,
                         float *__restrict__ f)
{
    const float s = *scale;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t c = codes[i];
        const float x = dtype == 1 ? __half2float(__ushort_as_half(c)) : __uint_as_float((unsigned)c << 16);
        f[i] = s * x;
    }
}

// Window-strided codec: encode/decode one state-layout field of a window.
__global__ void k_absmax_win(const float *__restrict__ f, Win w, unsigned *out)
{
    __shared__ unsigned sm[BS];
    unsigned mx = 0;
    const int y = blockIdx.y, z = blockIdx.z;
    for (int x = threadIdx.x; x < w.nx; x += BS) mx = max(mx, __float_as_uint(f[sidx(w, x, y, z)]) & 0x7fffffffu);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sm[0]);
}

__global__ void k_encode_win(const float *__restrict__ f, Win w, const unsigned *__restrict__ maxbits, int dtype,
                             void *__restrict__ codes, float *__restrict__ scale_out)
{
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t row = ((int64_t)z * w.ny + y) * w.nx;   // codes are dense per window
    if (dtype == 0) {
        float *o = (float *)codes;
        for (int x = threadIdx.x; x < w.nx; x += BS) o[row + x] = f[sidx(w, x, y, z)];
        if (blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *scale_out = 1.0f;
        return;
    }
    const float s = pow2_scale(*maxbits);
    const float rs = 1.0f / s;
    if (blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *scale_out = s;
    uint16_t *o = (uint16_t *)codes;
    for (int x = threadIdx.x; x < w.nx; x += BS) {
        const float v = f[sidx(w, x, y, z)] * rs;
        o[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(v)) : f32_to_bf16_rne(v);
    }
}

__global__ void k_decode_win(const void *__restrict__ codes, const float *__restrict__ scale, Win w, int dtype,
                             float *__restrict__ f)
{
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t row = ((int64_t)z * w.ny + y) * w.nx;
    const float s = *scale;
    for (int x = threadIdx.x; x < w.nx; x += BS) {
        float v;
        if (dtype == 0) v = ((const float *)codes)[row + x];
        else {
            const uint16_t c = ((const uint16_t *)codes)[row + x];
            v = s * (dtype == 1 ? __half2float(__ushort_as_half(c)) : __uint_as_float((unsigned)c << 16));
        }
        f[sidx(w, x, y, z)] = v;
    }
}

// Checkpoint codec of the gradient: for a field pair (current level c, previous level c-1) store
// a = f^c and b = f^c - f^{c-1} (the level difference keeps the time derivative accurate), each
// rounded to nearest-even FP16/BF16 with its own power-of-two scale per x-row.  One block per row:
// reduce the two row maxima in LDS, then encode.
__global__ void k_encode_pair_rows(const float *__restrict__ cur, const float *__restrict__ prev, Win w, int dtype,
                                   uint16_t *__restrict__ ca, uint16_t *__restrict__ cb, float *__restrict__ sca,
                                   float *__restrict__ scb)
{
    __shared__ unsigned sa[BS], sb[BS];
    const int y = blockIdx.y, z = blockIdx.z;
    unsigned xa = 0, xb = 0;
    for (int x = threadIdx.x; x < w.nx; x += BS) {
        const int64_t i = sidx(w, x, y, z);
        const float c = cur[i];
        xa = max(xa, __float_as_uint(c) & 0x7fffffffu);
        xb = max(xb, __float_as_uint(c - prev[i]) & 0x7fffffffu);
    }
    sa[threadIdx.x] = xa;
    sb[threadIdx.x] = xb;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sa[threadIdx.x] = max(sa[threadIdx.x], sa[threadIdx.x + s]);
            sb[threadIdx.x] = max(sb[threadIdx.x], sb[threadIdx.x + s]);
        }
        __syncthreads();
    }
    const float s1 = pow2_scale(sa[0]), s2 = pow2_scale(sb[0]);
    const float r1 = 1.0f / s1, r2 = 1.0f / s2;
    const int64_t r = (int64_t)z * w.ny + y;
    if (threadIdx.x == 0) {
        sca[r] = s1;
        scb[r] = s2;
    }
    const int64_t row = r * w.nx;
    for (int x = threadIdx.x; x < w.nx; x += BS) {
        const int64_t i = sidx(w, x, y, z);
        const float c = cur[i], d = c - prev[i];
        const float va = c * r1, vb = d * r2;
        ca[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(va)) : f32_to_bf16_rne(va);
        cb[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(vb)) : f32_to_bf16_rne(vb);
    }
}

// 16-bit segment store of one time step: p and q each rounded to nearest-even FP16/BF16 with a
// power-of-two scale per x-row.  One wavefront per row: the row's values stay in registers between
// the two row maxima (reduced across the wavefront with lane shuffles) and the encode; rows longer
// than 64 KR points re-read the rest.
template <int KR>
__global__ void k_encode_rows2(const float *__restrict__ p, const float *__restrict__ q, Win w, int dtype,
                               uint16_t *__restrict__ cp, uint16_t *__restrict__ cq, float *__restrict__ sp,
                               float *__restrict__ sq)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (r >= (int64_t)w.ny * w.nz) return;   // whole wavefronts
    const int z = (int)(r / w.ny), y = (int)(r - (int64_t)z * w.ny);
    const int64_t base = sidx(w, 0, y, z);
    float vp[KR], vq[KR];
    unsigned xa = 0, xb = 0;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int x = lane + 64 * k;
        vp[k] = x < w.nx ? p[base + x] : 0.f;
        vq[k] = x < w.nx ? q[base + x] : 0.f;
        xa = max(xa, __float_as_uint(vp[k]) & 0x7fffffffu);
        xb = max(xb, __float_as_uint(vq[k]) & 0x7fffffffu);
    }
    for (int x = lane + 64 * KR; x < w.nx; x += 64) {
        xa = max(xa, __float_as_uint(p[base + x]) & 0x7fffffffu);
        xb = max(xb, __float_as_uint(q[base + x]) & 0x7fffffffu);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        xa = max(xa, (unsigned)__shfl_xor((int)xa, o));
        xb = max(xb, (unsigned)__shfl_xor((int)xb, o));
    }
    const float s1 = pow2_scale(xa), s2 = pow2_scale(xb);
    const float r1 = 1.0f / s1, r2 = 1.0f / s2;
    if (lane == 0) {
        sp[r] = s1;
        sq[r] = s2;
    }
    const int64_t row = r * w.nx;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int x = lane + 64 * k;
        if (x < w.nx) {
            const float va = vp[k] * r1, vb = vq[k] * r2;
            cp[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(va)) : f32_to_bf16_rne(va);
            cq[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(vb)) : f32_to_bf16_rne(vb);
        }
    }
    for (int x = lane + 64 * KR; x < w.nx; x += 64) {
        const float va = p[base + x] * r1, vb = q[base + x] * r2;
        cp[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(va)) : f32_to_bf16_rne(va);
        cq[row + x] = dtype == 1 ? __half_as_ushort(__float2half_rn(vb)) : f32_to_bf16_rne(vb);
    }
}

__global__ void k_decode_pair_rows(const uint16_t *__restrict__ ca, const uint16_t *__restrict__ cb,
                                   const float *__restrict__ sca, const float *__restrict__ scb, Win w, int dtype,
                                   float *__restrict__ cur, float *__restrict__ prev)
{
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t r = (int64_t)z * w.ny + y;
    const float s1 = sca[r], s2 = scb[r];
    const int64_t row = r * w.nx;
    for (int x = threadIdx.x; x < w.nx; x += BS) {
        const uint16_t a = ca[row + x], b = cb[row + x];
        const float va = dtype == 1 ? __half2float(__ushort_as_half(a)) : __uint_as_float((unsigned)a << 16);
        const float vb = dtype == 1 ? __half2float(__ushort_as_half(b)) : __uint_as_float((unsigned)b << 16);
        const int64_t i = sidx(w, x, y, z);
        const float c = s1 * va;
        cur[i] = c;
        prev[i] = c - s2 * vb;
    }
}

// Deterministic FP64 dot product: fixed grid, per-thread strided partial sums, fixed-order tree.
constexpr int DOT_BLOCKS = 1024;
__global__ void k_dot_partial(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                              double *__restrict__ part)
{
    __shared__ double sm[BS];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)DOT_BLOCKS * BS)
        s += (double)a[i] * (double)b[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int k = BS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_dot_final(const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sm[BS];
    double s = 0.0;
    for (int i = threadIdx.x; i < DOT_BLOCKS; i += BS) s += part[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int k = BS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0];
}

// TTI coefficients: A = 1 + 2 eps, B = sqrt(1 + 2 delta), symmetry axis n from tilt/azimuth;
// statistics: max 1/sqrt(m) (bits), max eps (bits), flags (bit 0: m <= 0 or non-finite,
// bit 1: eps < delta).
__global__ void k_tti_prep(const float *__restrict__ m, const float *__restrict__ eps, const float *__restrict__ dl,
                           const float *__restrict__ th, const float *__restrict__ ph, int64_t n, int ndim,
                           float *A, float *B, float *nx, float *ny, unsigned *stats)
{
    unsigned vmax = 0, emax = 0, flags = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float e = eps[i], d = dl[i], t = th[i], p = ndim == 3 ? ph[i] : 0.f, mm = m[i];
        A[i] = 1.f + 2.f * e;
        B[i] = sqrtf(1.f + 2.f * d);
        float st, ct, sp, cp;
        sincosf(t, &st, &ct);
        sincosf(p, &sp, &cp);
        // the axis is stored as (n_x, n_y) of the unit vector with n_z >= 0 (n and -n give the same
        // operators); the kernels re-form n_z = sqrt(1 - n_x^2 - n_y^2)
        const float sg = ct < 0.f ? -1.f : 1.f;
        nx[i] = sg * (st * cp);
        ny[i] = ndim == 3 ? sg * (st * sp) : 0.f;
        if (!(mm > 0.f) || !isfinite(mm) || !isfinite(e) || !isfinite(d) || !isfinite(t) || !isfinite(p)) flags |= 1u;
        else vmax = max(vmax, __float_as_uint(1.0f / sqrtf(mm)));
        if (e < d - 1e-6f) flags |= 2u;
        if (e > 0.f) emax = max(emax, __float_as_uint(e));
    }
    atomicMax(&stats[0], vmax);
    atomicMax(&stats[1], emax);
    atomicOr(&stats[2], flags);
}

// Elastic coefficients: lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2, b = 1/rho; stats: max vp (bits),
// flags (bit 0: rho <= 0, vp <= 0, vs < 0 or non-finite; bit 1: lambda < 0).
// flags: 1 invalid value, 2 negative lambda, 4 vs > 0 on the plane rows [fluid_lo, fluid_hi) that
// must be fluid (the image free surface)
__global__ void k_el_prep(const float *__restrict__ vp, const float *__restrict__ vs, const float *__restrict__ rho,
                          int64_t n, float *lam, float *mu, float *b, unsigned *stats, int64_t plane, int fluid_lo,
                          int fluid_hi)
{
    unsigned vmax = 0, flags = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float p = vp[i], s = vs[i], r = rho[i];
        lam[i] = r * (p * p - 2.f * s * s);
        mu[i] = r * s * s;
        b[i] = 1.f / r;
        if (!(r > 0.f) || !(p > 0.f) || !(s >= 0.f) || !isfinite(p) || !isfinite(s) || !isfinite(r)) flags |= 1u;
        else vmax = max(vmax, __float_as_uint(p));
        if (p * p < 2.f * s * s) flags |= 2u;
        const int64_t z = i / plane;
        if (z >= fluid_lo && z < fluid_hi && s != 0.f) flags |= 4u;
    }
    atomicMax(&stats[0], vmax);
    atomicOr(&stats[2], flags);
}

__global__ void k_nonfinite_win(const float *__restrict__ f, Win w, unsigned *flag)
{
    const int y = blockIdx.y, z = blockIdx.z;
    bool bad = false;
    for (int x = threadIdx.x; x < w.nx; x += BS) bad |= !isfinite(f[sidx(w, x, y, z)]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ void k_copy_out(const float *__restrict__ src, Win w, float *__restrict__ dst)
{
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t row = ((int64_t)z * w.ny + y) * w.nx;
    for (int x = threadIdx.x; x < w.nx; x += BS) dst[row + x] = src[sidx(w, x, y, z)];
}

__global__ void k_accum_f64(const float *__restrict__ src, Win w, double *__restrict__ dst)
{
    const int y = blockIdx.y, z = blockIdx.z;
    for (int x = threadIdx.x; x < w.nx; x += BS) dst[midx(w, x, y, z)] += (double)src[sidx(w, x, y, z)];
}

inline unsigned nblocks(int64_t n, int cap = 8192)
{
    int64_t b = (n + BS - 1) / BS;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

void aux_tti_src(const BCsr &c, const TTIJob *jobs, int par, const float *const *data, const int *npt, int n,
                 float idt2, int seg_step, hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_tti_src, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, jobs, par, data, npt, n, idt2,
                       seg_step);
}

void aux_tti_rec_adj(const BCsr &c, const TTIJob *jobs, int par, const float *const *data, const int *npt, int n,
                     float idt2, int ic, int seg_step, hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_tti_rec_adj, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, jobs, par, data, npt, n, idt2,
                       ic, seg_step);
}

void aux_tti_gather(const BGather &g, const TTIJob *jobs, int par, int mode, float *const *out, const int *npt, int n,
                    hipStream_t st)
{
    if (g.n <= 0) return;
    const int64_t lanes = (int64_t)g.n * g.nc;
    hipLaunchKernelGGL(k_tti_gather, dim3((unsigned)((lanes + BS - 1) / BS)), dim3(BS), 0, st, g, jobs, par, mode, out,
                       npt, n);
}

void aux_tti_inject(const Csr &c, const float *data, float idt2, const float *m, float *d0, float *d1, float *d2,
                    float *d3, hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_tti_inject, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, data, idt2, m, d0, d1, d2, d3);
}

void aux_tti_inject_adj(const Csr &c, const float *data, float idt2, const float *m, const float *A, const float *B,
                        float *yp, float *wp, float *wq, float *grad, const float *fpk, hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_tti_inject_adj, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, data, idt2, m, A, B, yp, wp,
                       wq, grad, fpk);
}

void aux_el_inject(const Csr &c, const float *data, float scale, float *d0, float *d1, float *d2, hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_el_inject, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, data, scale, d0, d1, d2);
}

void aux_el_remix(const Csr &c, const Win &w, const float *gx, const float *gy, const float *gz, const float *lam,
                  const float *mu, const float *t0, const float *t1, const float *t2, float *a0, float *a1, float *a2,
                  hipStream_t st)
{
    if (c.nrows <= 0) return;
    hipLaunchKernelGGL(k_el_remix, dim3((c.nrows + BS - 1) / BS), dim3(BS), 0, st, c, w, gx, gy, gz, lam, mu, t0, t1,
                       t2, a0, a1, a2);
}

void aux_el_image_fill(const Win &w, int ks, float *txx, float *tyy, float *tzz, float *txz, float *tyz,
                       hipStream_t st)
{
    if (ks <= 0) return;
    hipLaunchKernelGGL(k_el_image_fill, dim3((w.nx + BS - 1) / BS, w.ny, ks + 1), dim3(BS), 0, st, w, ks, txx, tyy,
                       tzz, txz, tyz);
}

void aux_el_image_fold(const Win &w, int ks, int ndim, const ElImage &J, hipStream_t st)
{
    if (ks <= 0) return;
    hipLaunchKernelGGL(k_el_image_fold, dim3((w.nx + BS - 1) / BS, w.ny, ks + 1), dim3(BS), 0, st, w, ks, ndim, J);
    hipLaunchKernelGGL(k_el_image_sigma, dim3((w.nx + BS - 1) / BS, w.ny, std::min(2 * ks + 1, w.nz)), dim3(BS), 0,
                       st, w, ndim, J);
}

void aux_gather(const Gather &g, const float *f0, const float *f1, const float *f2, float scale, float *out,
                hipStream_t st)
{
    if (g.n <= 0) return;
    const int64_t lanes = (int64_t)g.n * g.nc;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((lanes + BS - 1) / BS)), dim3(BS), 0, st, g, f0, f1, f2, scale, out);
}

void aux_fill(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(BS), 0, st, p, n, v);
}

void aux_fill_u32(unsigned *p, int n, unsigned v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3((n + BS - 1) / BS), dim3(BS), 0, st, p, n, v);
}

void aux_absmax(const float *f, int64_t n, unsigned *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_absmax, dim3(nblocks(n)), dim3(BS), 0, st, f, n, out);
}

void aux_encode(const float *f, int64_t n, const unsigned *maxbits, int dtype, uint16_t *codes, float *scale_out,
                hipStream_t st)
{
    hipLaunchKernelGGL(k_encode, dim3(nblocks(n)), dim3(BS), 0, st, f, n, maxbits, dtype, codes, scale_out);
}

void aux_decode(const uint16_t *codes, const float *scale, int64_t n, int dtype, float *f, hipStream_t st)
{
    hipLaunchKernelGGL(k_decode, dim3(nblocks(n)), dim3(BS), 0, st, codes, scale, n, dtype, f);
}

void aux_absmax_win(const float *f, const Win &w, unsigned *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_absmax_win, dim3(1, w.ny, w.nz), dim3(BS), 0, st, f, w, out);
}

void aux_encode_win(const float *f, const Win &w, const unsigned *maxbits, int dtype, void *codes, float *scale_out,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_encode_win, dim3(1, w.ny, w.nz), dim3(BS), 0, st, f, w, maxbits, dtype, codes, scale_out);
}

void aux_decode_win(const void *codes, const float *scale, const Win &w, int dtype, float *f, hipStream_t st)
{
    hipLaunchKernelGGL(k_decode_win, dim3(1, w.ny, w.nz), dim3(BS), 0, st, codes, scale, w, dtype, f);
}

void aux_ckpt_pair_encode(const float *cur, const float *prev, const Win &w, int dtype, uint16_t *ca, uint16_t *cb,
                          float *sca, float *scb, hipStream_t st)
{
    hipLaunchKernelGGL(k_encode_pair_rows, dim3(1, w.ny, w.nz), dim3(BS), 0, st, cur, prev, w, dtype, ca, cb, sca, scb);
}

void aux_encode_rows2(const float *p, const float *q, const Win &w, int dtype, uint16_t *cp, uint16_t *cq, float *sp,
                      float *sq, hipStream_t st)
{
    const int64_t rows = (int64_t)w.ny * w.nz, per = BS / 64;
    hipLaunchKernelGGL(k_encode_rows2<8>, dim3((unsigned)((rows + per - 1) / per)), dim3(BS), 0, st, p, q, w, dtype, cp,
                       cq, sp, sq);
}

void aux_ckpt_pair_decode(const uint16_t *ca, const uint16_t *cb, const float *sca, const float *scb, const Win &w,
                          int dtype, float *cur, float *prev, hipStream_t st)
{
    hipLaunchKernelGGL(k_decode_pair_rows, dim3(1, w.ny, w.nz), dim3(BS), 0, st, ca, cb, sca, scb, w, dtype, cur,
                       prev);
}

void aux_dot_f64(const float *a, const float *b, int64_t n, double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(BS), 0, st, a, b, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(BS), 0, st, part, out);
}

int aux_dot_blocks() { return DOT_BLOCKS; }

void aux_tti_prep(const float *m, const float *eps, const float *dl, const float *th, const float *ph, int64_t n,
                  int ndim, float *A, float *B, float *nx, float *ny, unsigned *stats, hipStream_t st)
{
    hipLaunchKernelGGL(k_tti_prep, dim3(nblocks(n)), dim3(BS), 0, st, m, eps, dl, th, ph, n, ndim, A, B, nx, ny,
                       stats);
}

void aux_el_prep(const float *vp, const float *vs, const float *rho, int64_t n, float *lam, float *mu, float *b,
                 unsigned *stats, int64_t plane, int fluid_lo, int fluid_hi, hipStream_t st)
{
    hipLaunchKernelGGL(k_el_prep, dim3(nblocks(n)), dim3(BS), 0, st, vp, vs, rho, n, lam, mu, b, stats, plane,
                       fluid_lo, fluid_hi);
}

void aux_nonfinite_win(const float *f, const Win &w, unsigned *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_nonfinite_win, dim3(1, w.ny, w.nz), dim3(BS), 0, st, f, w, flag);
}

void aux_copy_out(const float *src, const Win &w, float *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_out, dim3(1, w.ny, w.nz), dim3(BS), 0, st, src, w, dst);
}

void aux_accum_f64(const float *src, const Win &w, double *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_accum_f64, dim3(1, w.ny, w.nz), dim3(BS), 0, st, src, w, dst);
}
