// Pseudo-acoustic TTI stencil kernels (gfx950).
//
// The rotated operators of the TTI section (G = D_i^T D_i with the tilt/azimuth factors inside
// the second, transposed derivative pass) are evaluated in the algebraically identical projector
// form: because the rotated axes are orthonormal at every point,
//     H0 f = -(G_xbar + G_ybar) f = div_D((I - n n^T) grad_D f),   Hz f = -G_zbar f = div_D(n n^T grad_D f)
// with n the symmetry axis and grad_D, div_D built from the same truncated centred first
// derivative D (D^T = -D).  One time step is two passes over the grid:
//   pass 1: t = (I - n n^T) grad u,  s = n (n . grad v)
//           forward: (u, v) = (p, q); adjoint: (u, v) = w = C y (mix first, the transpose order)
//           (four-field scheme: s is stored as the scalar n . grad v and re-formed in pass 2 from
//           it and the axis, which pass 2 reads; the products are the same, so is every bit)
//   pass 2: H0 = div t, Hz = div s; forward L = C (H0, Hz), adjoint L = (H0, Hz);
//           a f+ = b f - c f- + L,  a = m/dt^2 + eta/(2dt), b = 2m/dt^2, c = m/dt^2 - eta/(2dt),
//           with C = [[1+2eps, sqrt(1+2delta)], [sqrt(1+2delta), 1]]; the adjoint pass also writes
//           w = C y+ for the next pass 1.
//
// Both passes run the pipelined 2.5D z-march: while plane z is computed from LDS (x and y
// derivatives) and from the register queues (z derivatives), the global loads of plane z+1
// are already in flight into registers; LDS is double-buffered so one barrier per plane suffices.
#include "jobs.h"

namespace {

// Tile shapes (threads in y x rows per thread) selectable per pass at run time:
//   pass 1: 0 -> 8 x 2 (TY 16),  1 -> 16 x 2 (TY 32);   pass 2: 0 -> 8 x 1 (TY 8),  1 -> 16 x 1 (TY 16)
// Rows per thread drop to 1 for the widest stencils to keep the register queues in budget.
template <int R> constexpr int ny1_of() { return R <= 6 ? 2 : 1; }

// SCH: TTI_SIX (t and s), TTI_FOUR (t and n . grad v)
template <int R, int NY, int BY, bool ADJ, int SCH>
__global__ __launch_bounds__(PROP_TX * BY) void tti_pass1(const TTIJob *__restrict__ jobs,
                                                       const Tile *__restrict__ tiles, int zc, int par, Weights W)
{
    constexpr int TY = BY * NY, Q = 2 * R + 1, NT = PROP_TX * BY;
    using P = Plane<R, TY>;
    using H = Halo<R, TY, NT>;
    __shared__ float Lp[2][P::SIZE], Lq[2][P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    const float *__restrict__ U = ADJ ? J.wmix[par][0] : J.p[par];
    const float *__restrict__ V = ADJ ? J.wmix[par][1] : J.q[par];
    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? gld(f, sidx(w, x, y, z)) : 0.f;
    };

    float qu[NY][Q], qv[NY][Q];                       // z queues of u and v
    float nu[NY], nv[NY];                             // prefetched plane z+R of the queues
    float hxu[H::NXH], hxv[H::NXH], hyu[H::NYH], hyv[H::NYH];   // prefetched halos of plane z
    // before the first shift, slot s holds plane z0 - R + s - 1 (s = 1 .. 2R)
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) {
            qu[r][s] = ld(U, gx, y0 + ty * NY + r, z0 - R + s - 1);
            qv[r][s] = ld(V, gx, y0 + ty * NY + r, z0 - R + s - 1);
        }
    auto fetch = [&](int z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            nu[r] = ld(U, gx, y0 + ty * NY + r, z + R);
            nv[r] = ld(V, gx, y0 + ty * NY + r, z + R);
        }
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NXI) H::xitem(i, yy, xx);
            hxu[k] = i < H::NXI ? ld(U, x0 + xx, y0 + yy, z) : 0.f;
            hxv[k] = i < H::NXI ? ld(V, x0 + xx, y0 + yy, z) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < H::NYH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NYI) H::yitem(i, yy, xx);
            hyu[k] = i < H::NYI ? ld(U, x0 + xx, y0 + yy, z) : 0.f;
            hyv[k] = i < H::NYI ? ld(V, x0 + xx, y0 + yy, z) : 0.f;
        }
    };
    fetch(z0);
    int b = 0;
    for (int z = z0; z < z1; ++z) {
        float *lu = Lp[b], *lv = Lq[b];
#pragma unroll
        for (int r = 0; r < NY; ++r) {
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qu[r][s] = qu[r][s + 1];
                qv[r][s] = qv[r][s + 1];
            }
            qu[r][Q - 1] = nu[r];
            qv[r][Q - 1] = nv[r];
            lu[P::at(ty * NY + r, tx)] = qu[r][R];
            lv[P::at(ty * NY + r, tx)] = qv[r][R];
        }
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NXI) {
                int yy, xx;
                H::xitem(i, yy, xx);
                lu[P::at(yy, xx)] = hxu[k];
                lv[P::at(yy, xx)] = hxv[k];
            }
        }
#pragma unroll
        for (int k = 0; k < H::NYH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NYI) {
                int yy, xx;
                H::yitem(i, yy, xx);
                lu[P::at(yy, xx)] = hyu[k];
                lv[P::at(yy, xx)] = hyv[k];
            }
        }
        __syncthreads();
        // per-point symmetry axis of plane z first, then the prefetch of plane z+1
        float n0[NY], n1[NY], n2[NY];
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            const bool in = gx < w.nx && y < w.ny;
            const int64_t mi = midx(w, in ? gx : 0, in ? y : 0, z);
            n0[r] = gld(J.nx, mi);
            n1[r] = gld(J.ny, mi);
            n2[r] = axis_z(n0[r], n1[r]);
        }
        if (z + 1 < z1) fetch(z + 1);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            const int li = P::at(ty * NY + r, tx);
            const float dpx = dc_lds_x<R>(lu, li, W.wx), dpy = dc_lds_y<R, P::LX>(lu, li, W.wy);
            const float dqx = dc_lds_x<R>(lv, li, W.wx), dqy = dc_lds_y<R, P::LX>(lv, li, W.wy);
            const float dpz = dc_q<R>(qu[r], W.wz), dqz = dc_q<R>(qv[r], W.wz);
            if (gx < w.nx && y < w.ny) {
                const float wp = n0[r] * dpx + n1[r] * dpy + n2[r] * dpz;
                const float wq = n0[r] * dqx + n1[r] * dqy + n2[r] * dqz;
                const int64_t si = sidx(w, gx, y, z);
                gst(J.t[0], si, dpx - n0[r] * wp);
                gst(J.t[1], si, dpy - n1[r] * wp);
                gst(J.t[2], si, dpz - n2[r] * wp);
                if (SCH == TTI_FOUR) {
                    gst(J.s[0], si, wq);
                } else {
                    gst(J.s[0], si, n0[r] * wq);
                    gst(J.s[1], si, n1[r] * wq);
                    gst(J.s[2], si, n2[r] * wq);
                }
            }
        }
        b ^= 1;
    }
}

// FOUR: pass 1 stored t and the scalar wq = n . grad v (in s[0]); s = n wq is formed here, at the
// front plane for the z queue and the centre plane, and at the halo points, from wq and the axis.
// The centre products of the own columns are formed at the front and wait R planes in a delay
// ring in LDS, private to the thread (plane z in slot z mod (R + 1)); registers are the limit here.
template <int R, int NY, int BY, int MODE, bool FOUR>
__global__ __launch_bounds__(PROP_TX * BY) void tti_pass2(const TTIJob *__restrict__ jobs,
                                                       const Tile *__restrict__ tiles, int zc, int par, Weights W,
                                                       float idt2, int seg_step)
{
    constexpr int TY = BY * NY, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool ADJ = (MODE == K2_ADJ || MODE == K2_ADJ_IC);
    using P = Plane<R, TY>;
    using H = Halo<R, TY, NT>;
    constexpr int ND = FOUR ? (R + 1) * NY * NT : 1;
    __shared__ float Ltx[2][P::SIZE], Lty[2][P::SIZE], Lsx[2][P::SIZE], Lsy[2][P::SIZE];
    __shared__ float Dsx[ND], Dsy[ND];

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    // delay-ring slot of plane z, row r of this thread
    auto dslot = [&](int z, int r) { return ((((z % (R + 1)) + (R + 1)) % (R + 1)) * NY + r) * NT + tid; };
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
        return in_win(w, x, y, z) ? gld(f, sidx(w, x, y, z)) : 0.f;
    };
    auto ldm = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? gld(f, midx(w, x, y, z)) : 0.f;
    };
    const float *__restrict__ AX = J.nx;
    const float *__restrict__ AY = J.ny;

    float qt[NY][Q], qs[NY][Q];
    float nt[NY], ns[NY], itx[NY], ity[NY], isx[NY], isy[NY];
    float hxt[H::NXH], hxs[H::NXH], hyt[H::NYH], hys[H::NYH], hxn[H::NXH], hyn[H::NYH];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) {
            const int y = y0 + ty * NY + r, zz = z0 - R + s - 1;
            qt[r][s] = ld(T2, gx, y, zz);
            if (FOUR) {
                const float wq = ld(S0, gx, y, zz), ax = ldm(AX, gx, y, zz), ay = ldm(AY, gx, y, zz);
                qs[r][s] = axis_z(ax, ay) * wq;
                if (s > R) {   // planes z0 .. z0 + R - 1, centres of the first R planes
                    Dsx[dslot(zz, r)] = ax * wq;
                    Dsy[dslot(zz, r)] = ay * wq;
                }
            } else {
                qs[r][s] = ld(S2, gx, y, zz);
            }
        }
    auto fetch = [&](int z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            nt[r] = ld(T2, gx, y, z + R);
            itx[r] = ld(T0, gx, y, z);
            ity[r] = ld(T1, gx, y, z);
            if (FOUR) {   // wq and the axis of the front plane
                ns[r] = ld(S0, gx, y, z + R);
                isx[r] = ldm(AX, gx, y, z + R);
                isy[r] = ldm(AY, gx, y, z + R);
            } else {
                ns[r] = ld(S2, gx, y, z + R);
                isx[r] = ld(S0, gx, y, z);
                isy[r] = ld(S1, gx, y, z);
            }
        }
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NXI) H::xitem(i, yy, xx);
            hxt[k] = i < H::NXI ? ld(T0, x0 + xx, y0 + yy, z) : 0.f;
            hxs[k] = i < H::NXI ? ld(S0, x0 + xx, y0 + yy, z) : 0.f;
            hxn[k] = FOUR && i < H::NXI ? ldm(AX, x0 + xx, y0 + yy, z) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < H::NYH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NYI) H::yitem(i, yy, xx);
            hyt[k] = i < H::NYI ? ld(T1, x0 + xx, y0 + yy, z) : 0.f;
            hys[k] = i < H::NYI ? ld(FOUR ? S0 : S1, x0 + xx, y0 + yy, z) : 0.f;
            hyn[k] = FOUR && i < H::NYI ? ldm(AY, x0 + xx, y0 + yy, z) : 0.f;
        }
    };
    float nvp0[NY], nvq0[NY], nvp1[NY], nvq1[NY], nvm[NY], nvA[NY], nvB[NY], nfpk[NY], nfqk[NY], nvg[NY];
    auto pload = [&](int z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            const bool in = gx < w.nx && y < w.ny;
            const int64_t si = sidx(w, in ? gx : 0, in ? y : 0, z);
            const int64_t mi = midx(w, in ? gx : 0, in ? y : 0, z);
            nvp0[r] = gld(pc, si);
            nvq0[r] = gld(qc, si);
            nvp1[r] = gld(pn, si);
            nvq1[r] = gld(qn, si);
            nvm[r] = gld(J.m, mi);
            nvA[r] = gld(J.A, mi);
            nvB[r] = gld(J.B, mi);
            nfpk[r] = nfqk[r] = nvg[r] = 0.f;
            if (MODE == K2_ADJ_IC) {
                seg_load(J, seg_step, in ? gx : 0, in ? y : 0, z, si, nfpk[r], nfqk[r]);
                nvg[r] = gld(J.grad, si);
            }
        }
    };
    pload(z0);
    fetch(z0);
    int b = 0;
    for (int z = z0; z < z1; ++z) {
        float *ltx = Ltx[b], *lty = Lty[b], *lsx = Lsx[b], *lsy = Lsy[b];
#pragma unroll
        for (int r = 0; r < NY; ++r) {
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qt[r][s] = qt[r][s + 1];
                qs[r][s] = qs[r][s + 1];
            }
            qt[r][Q - 1] = nt[r];
            const int li = P::at(ty * NY + r, tx);
            ltx[li] = itx[r];
            lty[li] = ity[r];
            if (FOUR) {
                // plane z + R enters the slot of plane z - 1, which the previous plane consumed
                qs[r][Q - 1] = axis_z(isx[r], isy[r]) * ns[r];
                Dsx[dslot(z + R, r)] = isx[r] * ns[r];
                Dsy[dslot(z + R, r)] = isy[r] * ns[r];
                lsx[li] = Dsx[dslot(z, r)];
                lsy[li] = Dsy[dslot(z, r)];
            } else {
                qs[r][Q - 1] = ns[r];
                lsx[li] = isx[r];
                lsy[li] = isy[r];
            }
        }
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NXI) {
                int yy, xx;
                H::xitem(i, yy, xx);
                ltx[P::at(yy, xx)] = hxt[k];
                lsx[P::at(yy, xx)] = FOUR ? hxn[k] * hxs[k] : hxs[k];
            }
        }
#pragma unroll
        for (int k = 0; k < H::NYH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NYI) {
                int yy, xx;
                H::yitem(i, yy, xx);
                lty[P::at(yy, xx)] = hyt[k];
                lsy[P::at(yy, xx)] = FOUR ? hyn[k] * hys[k] : hys[k];
            }
        }
        __syncthreads();
        // per-point values of plane z were loaded one plane earlier; those of plane z+1 are issued
        // before the prefetch of plane z+1, so that waiting for them next time does not wait for it
        float vp0[NY], vq0[NY], vp1[NY], vq1[NY], vm[NY], vA[NY], vB[NY], fpk[NY], fqk[NY], vg[NY];
        const float ezv = gld(J.ez, z);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            vp0[r] = nvp0[r];
            vq0[r] = nvq0[r];
            vp1[r] = nvp1[r];
            vq1[r] = nvq1[r];
            vm[r] = nvm[r] * idt2 + 0.f;
            vA[r] = nvA[r];
            vB[r] = nvB[r];
            fpk[r] = nfpk[r];
            fqk[r] = nfqk[r];
            vg[r] = nvg[r];
        }
        if (z + 1 < z1) {
            pload(z + 1);
            fetch(z + 1);
        }
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            const int li = P::at(ty * NY + r, tx);
            const float h0 = dc_lds_x<R>(ltx, li, W.wx) + dc_lds_y<R, P::LX>(lty, li, W.wy) + dc_q<R>(qt[r], W.wz);
            const float hz = dc_lds_x<R>(lsx, li, W.wx) + dc_lds_y<R, P::LX>(lsy, li, W.wy) + dc_q<R>(qs[r], W.wz);
            if (gx < w.nx && y < w.ny) {
                const int64_t si = sidx(w, gx, y, z);
                float Lp, Lq;
                if (ADJ) {
                    Lp = h0;
                    Lq = hz;
                } else {
                    Lp = vA[r] * h0 + vB[r] * hz;
                    Lq = vB[r] * h0 + hz;
                }
                const float mm = vm[r];
                const float e = gld(J.ex, gx) + gld(J.ey, y) + ezv;
                const float ra = 1.0f / (mm + e);
                const float cc = mm - e;
                const float np_ = (2.f * mm * vp0[r] - cc * vp1[r] + Lp) * ra;
                const float nq_ = (2.f * mm * vq0[r] - cc * vq1[r] + Lq) * ra;
                gst(pn, si, np_);
                gst(qn, si, nq_);
                if (ADJ) {
                    gst(J.wmix[par ^ 1][0], si, vA[r] * np_ + vB[r] * nq_);
                    gst(J.wmix[par ^ 1][1], si, vB[r] * np_ + nq_);
                }
                if (MODE == K2_FWD_STORE && J.seg_dtype == 0) {
                    float *sp = J.seg + (int64_t)seg_step * 2 * J.seg_field;
                    gst(sp, si, np_);
                    gst(sp, J.seg_field + si, nq_);
                }
                if (MODE == K2_ADJ_IC)
                    gst(J.grad, si, J.image ? vg[r] + (fpk[r] * np_ + fqk[r] * nq_)
                                            : vg[r] - idt2 * (fpk[r] * (np_ - 2.f * vp0[r] + vp1[r]) +
                                                              fqk[r] * (nq_ - 2.f * vq0[r] + vq1[r])));
            }
        }
        b ^= 1;
    }
}

template <int R, int BY, int SCH>
void p1_launch(bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par, const Weights &W,
               hipStream_t st)
{
    constexpr int NY = ny1_of<R>();
    dim3 blk(PROP_TX, BY), grd(ntiles);
    if (adj) hipLaunchKernelGGL((tti_pass1<R, NY, BY, true, SCH>), grd, blk, 0, st, jobs, tiles, zc, par, W);
    else     hipLaunchKernelGGL((tti_pass1<R, NY, BY, false, SCH>), grd, blk, 0, st, jobs, tiles, zc, par, W);
}

template <int R, int SCH>
void p1_shape(int shape, bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
              const Weights &W, hipStream_t st)
{
    if (shape == 1) p1_launch<R, 16, SCH>(adj, jobs, tiles, ntiles, zc, par, W, st);
    else            p1_launch<R, 8, SCH>(adj, jobs, tiles, ntiles, zc, par, W, st);
}

template <int R>
void p1_dispatch(int scheme, int shape, bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                 const Weights &W, hipStream_t st)
{
    if (scheme == TTI_FOUR) p1_shape<R, TTI_FOUR>(shape, adj, jobs, tiles, ntiles, zc, par, W, st);
    else                    p1_shape<R, TTI_SIX>(shape, adj, jobs, tiles, ntiles, zc, par, W, st);
}

template <int R, int BY, bool FOUR>
void p2_launch(int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par, const Weights &W,
               float idt2, int seg_step, hipStream_t st)
{
    dim3 blk(PROP_TX, BY), grd(ntiles);
    switch (mode) {
    case K2_FWD:
        hipLaunchKernelGGL((tti_pass2<R, 1, BY, K2_FWD, FOUR>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    case K2_FWD_STORE:
        hipLaunchKernelGGL((tti_pass2<R, 1, BY, K2_FWD_STORE, FOUR>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    case K2_ADJ:
        hipLaunchKernelGGL((tti_pass2<R, 1, BY, K2_ADJ, FOUR>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    default:
        hipLaunchKernelGGL((tti_pass2<R, 1, BY, K2_ADJ_IC, FOUR>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    }
}

template <int R>
void p2_dispatch(int scheme, int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                 const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    if (scheme == TTI_FOUR) {
        if (shape == 1) p2_launch<R, 16, true>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
        else            p2_launch<R, 8, true>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
    } else {
        if (shape == 1) p2_launch<R, 16, false>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
        else            p2_launch<R, 8, false>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
    }
}

}  // namespace

int tti_tile_rows(int R, int scheme, int pass, int shape)
{
    if (scheme == TTI_FUSED || scheme == TTI_SPLIT) return 16;
    const int by = shape == 1 ? 16 : 8;
    return pass == 1 ? by * (R <= 6 ? 2 : 1) : by;
}

#define R_SWITCH(FN, ...)                   \
    switch (R) {                            \
    case 1: FN<1>(__VA_ARGS__); break;      \
    case 2: FN<2>(__VA_ARGS__); break;      \
    case 3: FN<3>(__VA_ARGS__); break;      \
    case 4: FN<4>(__VA_ARGS__); break;      \
    case 5: FN<5>(__VA_ARGS__); break;      \
    case 6: FN<6>(__VA_ARGS__); break;      \
    case 7: FN<7>(__VA_ARGS__); break;      \
    default: FN<8>(__VA_ARGS__); break;     \
    }

void launch_tti_pass1(int R, int scheme, int shape, bool adj, const TTIJob *jobs, const Tile *tiles, int ntiles,
                      int zc, int par, const Weights &W, hipStream_t st)
{
    if (scheme == TTI_FUSED) return;
    if (scheme == TTI_SPLIT)
        return launch_tti_split(R, 0, adj ? K2_ADJ : K2_FWD, jobs, tiles, ntiles, zc, par, W, 0.f, 0, st);
    R_SWITCH(p1_dispatch, scheme, shape, adj, jobs, tiles, ntiles, zc, par, W, st)
}

void launch_tti_pass2(int R, int scheme, int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles,
                      int zc, int par, const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    if (scheme == TTI_FUSED) return launch_tti_fused(R, shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
    if (scheme == TTI_SPLIT) return launch_tti_split(R, 1, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
    R_SWITCH(p2_dispatch, scheme, shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st)
}
