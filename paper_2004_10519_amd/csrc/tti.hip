// Pseudo-acoustic TTI stencil kernels (gfx950).
//
// The rotated operators of the TTI section (G = D_i^T D_i with the tilt/azimuth factors inside
// the second, transposed derivative pass) are evaluated in the algebraically identical projector
// form: because the rotated axes are orthonormal at every point,
//     H0 f = -(G_xbar + G_ybar) f = div_D((I - n n^T) grad_D f),   Hz f = -G_zbar f = div_D(n n^T grad_D f)
// with n the symmetry axis and grad_D, div_D built from the same truncated centred first
// derivative D (D^T = -D).  One time step is two passes over the grid:
//   pass 1: t = (I - n n^T) grad p,  s = n (n . grad q)            (forward)
//           the same on w = C y (mix first, the transpose order)   (adjoint)
//   pass 2: H0 = div t, Hz = div s; forward L = C (H0, Hz), adjoint L = (H0, Hz);
//           a f+ = b f - c f- + L,  a = m/dt^2 + eta/(2dt), b = 2m/dt^2, c = m/dt^2 - eta/(2dt),
//           with C = [[1+2eps, sqrt(1+2delta)], [sqrt(1+2delta), 1]].
#include "jobs.h"

namespace {

template <int R, int NY, bool ADJ>
__global__ __launch_bounds__(PROP_NT) void tti_pass1(const TTIJob *__restrict__ jobs,
                                                    const Tile *__restrict__ tiles, int zc, int par,
                                                    Weights W)
{
    constexpr int TY = PROP_BY * NY, Q = 2 * R + 1;
    using P = Plane<R, TY>;
    __shared__ float Lp[P::SIZE], Lq[P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    const float *__restrict__ fp = J.p[par];
    const float *__restrict__ fq = J.q[par];

    auto load2 = [&](int x, int y, int z, float &a, float &b) {
        if (in_win(w, x, y, z)) {
            const int64_t i = sidx(w, x, y, z);
            const float yp = fp[i], yq = fq[i];
            if (ADJ) {
                const int64_t mi = midx(w, x, y, z);
                const float A = J.A[mi], B = J.B[mi];
                a = A * yp + B * yq;
                b = B * yp + yq;
            } else {
                a = yp;
                b = yq;
            }
        } else {
            a = 0.f;
            b = 0.f;
        }
    };

    float qp[NY][Q], qq[NY][Q];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) load2(gx, y0 + ty * NY + r, z0 - R + s - 1, qp[r][s], qq[r][s]);

    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qp[r][s] = qp[r][s + 1];
                qq[r][s] = qq[r][s + 1];
            }
            load2(gx, y0 + ty * NY + r, z + R, qp[r][Q - 1], qq[r][Q - 1]);
            Lp[P::at(ty * NY + r, tx)] = qp[r][R];
            Lq[P::at(ty * NY + r, tx)] = qq[r][R];
        }
        // halo of both fields in one pass over the halo points
        for (int i = tid; i < 2 * R * TY; i += PROP_NT) {
            int row = i / (2 * R), c = i - row * (2 * R);
            int xx = c < R ? c - R : PROP_TX + c - R;
            float a, b;
            load2(x0 + xx, y0 + row, z, a, b);
            Lp[P::at(row, xx)] = a;
            Lq[P::at(row, xx)] = b;
        }
        for (int i = tid; i < 2 * R * PROP_TX; i += PROP_NT) {
            int rr = i / PROP_TX, xx = i - rr * PROP_TX;
            int yy = rr < R ? rr - R : TY + rr - R;
            float a, b;
            load2(x0 + xx, y0 + yy, z, a, b);
            Lp[P::at(yy, xx)] = a;
            Lq[P::at(yy, xx)] = b;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            if (gx < w.nx && y < w.ny) {
                const int li = P::at(ty * NY + r, tx);
                const float dpx = dc_lds_x<R>(Lp, li, W.wx), dpy = dc_lds_y<R, P::LX>(Lp, li, W.wy);
                const float dqx = dc_lds_x<R>(Lq, li, W.wx), dqy = dc_lds_y<R, P::LX>(Lq, li, W.wy);
                const float dpz = dc_q<R>(qp[r], W.wz), dqz = dc_q<R>(qq[r], W.wz);
                const int64_t mi = midx(w, gx, y, z);
                const float n0 = J.nx[mi], n1 = J.ny[mi], n2 = J.nz[mi];
                const float wp = n0 * dpx + n1 * dpy + n2 * dpz;
                const float wq = n0 * dqx + n1 * dqy + n2 * dqz;
                const int64_t si = sidx(w, gx, y, z);
                J.t[0][si] = dpx - n0 * wp;
                J.t[1][si] = dpy - n1 * wp;
                J.t[2][si] = dpz - n2 * wp;
                J.s[0][si] = n0 * wq;
                J.s[1][si] = n1 * wq;
                J.s[2][si] = n2 * wq;
            }
        }
        __syncthreads();
    }
}

template <int R, int NY, int MODE>
__global__ __launch_bounds__(PROP_NT) void tti_pass2(const TTIJob *__restrict__ jobs,
                                                    const Tile *__restrict__ tiles, int zc, int par,
                                                    Weights W, float idt2, int seg_step)
{
    constexpr int TY = PROP_BY * NY, Q = 2 * R + 1;
    constexpr bool ADJ = (MODE == K2_ADJ || MODE == K2_ADJ_IC);
    using P = Plane<R, TY>;
    __shared__ float Ltx[P::SIZE], Lty[P::SIZE], Lsx[P::SIZE], Lsy[P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    const float *__restrict__ T0 = J.t[0];
    const float *__restrict__ T1 = J.t[1];
    const float *__restrict__ T2 = J.t[2];
    const float *__restrict__ S0 = J.s[0];
    const float *__restrict__ S1 = J.s[1];
    const float *__restrict__ S2 = J.s[2];
    const float *__restrict__ pc = J.p[par];
    const float *__restrict__ qc = J.q[par];
    float *__restrict__ pn = J.p[par ^ 1];   // holds the previous level, receives the new one
    float *__restrict__ qn = J.q[par ^ 1];

    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? f[sidx(w, x, y, z)] : 0.f;
    };

    float qt[NY][Q], qs[NY][Q];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) {
            qt[r][s] = ld(T2, gx, y0 + ty * NY + r, z0 - R + s - 1);
            qs[r][s] = ld(S2, gx, y0 + ty * NY + r, z0 - R + s - 1);
        }

    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qt[r][s] = qt[r][s + 1];
                qs[r][s] = qs[r][s + 1];
            }
            qt[r][Q - 1] = ld(T2, gx, y, z + R);
            qs[r][Q - 1] = ld(S2, gx, y, z + R);
            const int li = P::at(ty * NY + r, tx);
            Ltx[li] = ld(T0, gx, y, z);
            Lty[li] = ld(T1, gx, y, z);
            Lsx[li] = ld(S0, gx, y, z);
            Lsy[li] = ld(S1, gx, y, z);
        }
        for (int i = tid; i < 2 * R * TY; i += PROP_NT) {
            int row = i / (2 * R), c = i - row * (2 * R);
            int xx = c < R ? c - R : PROP_TX + c - R;
            Ltx[P::at(row, xx)] = ld(T0, x0 + xx, y0 + row, z);
            Lsx[P::at(row, xx)] = ld(S0, x0 + xx, y0 + row, z);
        }
        for (int i = tid; i < 2 * R * PROP_TX; i += PROP_NT) {
            int rr = i / PROP_TX, xx = i - rr * PROP_TX;
            int yy = rr < R ? rr - R : TY + rr - R;
            Lty[P::at(yy, xx)] = ld(T1, x0 + xx, y0 + yy, z);
            Lsy[P::at(yy, xx)] = ld(S1, x0 + xx, y0 + yy, z);
        }
        __syncthreads();
        const float ezv = J.ez[z];
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            if (gx < w.nx && y < w.ny) {
                const int li = P::at(ty * NY + r, tx);
                const float h0 = dc_lds_x<R>(Ltx, li, W.wx) + dc_lds_y<R, P::LX>(Lty, li, W.wy) +
                                 dc_q<R>(qt[r], W.wz);
                const float hz = dc_lds_x<R>(Lsx, li, W.wx) + dc_lds_y<R, P::LX>(Lsy, li, W.wy) +
                                 dc_q<R>(qs[r], W.wz);
                const int64_t mi = midx(w, gx, y, z);
                const int64_t si = sidx(w, gx, y, z);
                float Lp, Lq;
                if (ADJ) {
                    Lp = h0;
                    Lq = hz;
                } else {
                    const float A = J.A[mi], B = J.B[mi];
                    Lp = A * h0 + B * hz;
                    Lq = B * h0 + hz;
                }
                const float mm = J.m[mi] * idt2;
                const float e = J.ex[gx] + J.ey[y] + ezv;
                const float ra = 1.0f / (mm + e);
                const float cc = mm - e;
                const float p0 = pc[si], q0 = qc[si], p1 = pn[si], q1 = qn[si];
                const float np_ = (2.f * mm * p0 - cc * p1 + Lp) * ra;
                const float nq_ = (2.f * mm * q0 - cc * q1 + Lq) * ra;
                pn[si] = np_;
                qn[si] = nq_;
                if (MODE == K2_FWD_STORE) {
                    float *sp = J.seg + (int64_t)seg_step * 2 * J.seg_field;
                    sp[si] = np_;
                    sp[J.seg_field + si] = nq_;
                }
                if (MODE == K2_ADJ_IC) {
                    const float *sp = J.seg + (int64_t)seg_step * 2 * J.seg_field;
                    const float fpk = sp[si], fqk = sp[J.seg_field + si];
                    J.grad[si] -= idt2 * (fpk * (np_ - 2.f * p0 + p1) + fqk * (nq_ - 2.f * q0 + q1));
                }
            }
        }
        __syncthreads();
    }
}

template <int R>
constexpr int ny_of()
{
    return R <= 6 ? 4 : 2;
}

template <int R>
void p1_dispatch(bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                 const Weights &W, hipStream_t st)
{
    constexpr int NY = ny_of<R>();
    dim3 blk(PROP_TX, PROP_BY), grd(ntiles);
    if (adj) hipLaunchKernelGGL((tti_pass1<R, NY, true>), grd, blk, 0, st, jobs, tiles, zc, par, W);
    else     hipLaunchKernelGGL((tti_pass1<R, NY, false>), grd, blk, 0, st, jobs, tiles, zc, par, W);
}

template <int R>
void p2_dispatch(int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                 const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    constexpr int NY = ny_of<R>();
    dim3 blk(PROP_TX, PROP_BY), grd(ntiles);
    switch (mode) {
    case K2_FWD:
        hipLaunchKernelGGL((tti_pass2<R, NY, K2_FWD>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    case K2_FWD_STORE:
        hipLaunchKernelGGL((tti_pass2<R, NY, K2_FWD_STORE>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    case K2_ADJ:
        hipLaunchKernelGGL((tti_pass2<R, NY, K2_ADJ>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    default:
        hipLaunchKernelGGL((tti_pass2<R, NY, K2_ADJ_IC>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    }
}

}  // namespace

int tti_rows_per_thread(int R)
{
    return R <= 6 ? 4 : 2;
}

void launch_tti_pass1(int R, bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, hipStream_t st)
{
    switch (R) {
    case 1: p1_dispatch<1>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 2: p1_dispatch<2>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 3: p1_dispatch<3>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 4: p1_dispatch<4>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 5: p1_dispatch<5>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 6: p1_dispatch<6>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    case 7: p1_dispatch<7>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    default: p1_dispatch<8>(adj, jobs, tiles, ntiles, zc, par, W, st); break;
    }
}

void launch_tti_pass2(int R, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    switch (R) {
    case 1: p2_dispatch<1>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 2: p2_dispatch<2>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 3: p2_dispatch<3>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 4: p2_dispatch<4>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 5: p2_dispatch<5>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 6: p2_dispatch<6>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 7: p2_dispatch<7>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    default: p2_dispatch<8>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    }
}
