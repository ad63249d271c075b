// Single-pass TTI step (gfx950).
//
// Same operators and update as the two-pass kernels (projector form of the rotated TTI operators,
// TTI section):  t = (I - n n^T) grad u,  s = n (n . grad v),  H0 = div t,  Hz = div s,
//   a f+ = b f - c f- + L,  forward L = C (H0, Hz) with (u, v) = (p, q); adjoint L = (H0, Hz) with
//   (u, v) = w = C y, and the new w = C y+ written for the next step.
// Here the projections never leave the chip: one launch per time step reads u, v, the previous
// level, m, A, B and the axis once and writes the new level once (44 B per point forward, against
// 40 + 60 B for the two passes).
//
// A block owns a TX x TY tile and the output planes [z0, z1).  It marches a front plane zf from
// z0 - R to z1 + R - 1; per front plane:
//  1. register queues of u and v over planes zf - R .. zf + R advance by one plane, for the tile's
//     own columns and for the columns of its R-wide halo (x halo beside the tile rows, y halo
//     beside the tile columns); plane zf is staged in LDS over the tile, the halo, a second R-wide
//     ring and the R x R corners (everything the x and y derivatives on the halo touch);
//  2. t and s of plane zf are formed on the tile (all components) and on the halo (x components on
//     the x halo, y components on the y halo); the x and y components go to LDS, the z components
//     of the own columns are scattered with the derivative weights into per-column accumulators of
//     planes zf - R .. zf + R (a plane's z derivative is summed as its neighbours are formed);
//  3. the x-y part of div t, div s of plane zf joins its accumulator; the accumulators of plane
//     zf - R are then complete and that plane is updated.
// Every intermediate is zero outside the window, as in the two-pass kernels.  Two barriers per
// plane; the loads of the next plane are in flight during the compute.
#include "jobs.h"

namespace {

// Item lists of a TX x TY tile (coordinates relative to the tile origin).
//   halo: the R-wide x halo (tile rows, columns [-R, 0) and [TX, TX + R)), then the R-wide y halo
//         (tile columns, rows [-R, 0) and [TY, TY + R)); these columns carry z queues.
//   ring: what the x and y derivatives on the halo need beyond it, on plane zf only: x strips
//         (tile rows, columns [-2R, -R) and [TX + R, TX + 2R)), y strips (tile columns, rows
//         [-2R, -R) and [TY + R, TY + 2R)) and the four R x R corners diagonal to the tile corners.
template <int R, int TY>
struct FusedItems {
    static constexpr int NXI = 2 * R * TY, NYI = 2 * R * PROP_TX, NHI = NXI + NYI;
    static constexpr int NOX = 2 * R * TY, NOY = 2 * R * PROP_TX, NOC = 4 * R * R, NOI = NOX + NOY + NOC;
    // returns true for an x-halo item
    __device__ static __forceinline__ bool halo(int i, int &yy, int &xx)
    {
        if (i < NXI) {
            const int row = i / (2 * R), c = i - row * (2 * R);
            yy = row;
            xx = c < R ? c - R : PROP_TX + c - R;
            return true;
        }
        i -= NXI;
        const int rr = i / PROP_TX;
        xx = i - rr * PROP_TX;
        yy = rr < R ? rr - R : TY + rr - R;
        return false;
    }
    __device__ static __forceinline__ void ring(int i, int &yy, int &xx)
    {
        if (i < NOX) {
            const int row = i / (2 * R), c = i - row * (2 * R);
            yy = row;
            xx = c < R ? c - 2 * R : PROP_TX + c;
            return;
        }
        i -= NOX;
        if (i < NOY) {
            const int rr = i / PROP_TX;
            xx = i - rr * PROP_TX;
            yy = rr < R ? rr - 2 * R : TY + rr;
            return;
        }
        i -= NOY;
        const int qd = i / (R * R), k = i - qd * (R * R), cy = k / R, cx = k - cy * R;
        xx = (qd & 1) ? PROP_TX + cx : cx - R;
        yy = (qd & 2) ? TY + cy : cy - R;
    }
};


template <int R, int BY, int NY, int MODE>
__global__ __launch_bounds__(PROP_TX * BY) void tti_fused(const TTIJob *__restrict__ jobs,
                                                       const Tile *__restrict__ tiles, int zc, int par, Weights W,
                                                       float idt2, int seg_step)
{
    constexpr int TY = BY * NY, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool ADJ = (MODE == K2_ADJ || MODE == K2_ADJ_IC);
    using UP = Plane<2 * R, TY>;
    using XP = XPlane<R, TY>;
    using YP = YPlane<R, TY>;
    using IT = FusedItems<R, TY>;
    constexpr int NH = (IT::NHI + NT - 1) / NT, NO = (IT::NOI + NT - 1) / NT;
    __shared__ float Lu[UP::SIZE], Lv[UP::SIZE], Lt0[XP::SIZE], Ls0[XP::SIZE], Lt1[YP::SIZE], Ls1[YP::SIZE];
    __shared__ float Hu[Q * IT::NHI], Hv[Q * IT::NHI];   // z queues of the halo columns: plane z in slot z mod Q

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    const float *U = ADJ ? J.wmix[par][0] : J.p[par];
    const float *V = ADJ ? J.wmix[par][1] : J.q[par];
    // the job fields the march uses, read once before it (the loop's stores could alias the job table,
    // which would otherwise make the compiler reload them on every plane)
    const float *const Pc = J.p[par], *const Qc = J.q[par];
    float *const Pn = J.p[par ^ 1], *const Qn = J.q[par ^ 1];
    float *const Wn0 = ADJ ? J.wmix[par ^ 1][0] : nullptr, *const Wn1 = ADJ ? J.wmix[par ^ 1][1] : nullptr;
    const float *const Mm = J.m, *const MA = J.A, *const MB = J.B, *const Nx = J.nx, *const Ny = J.ny;
    const float *const Ez = J.ez;
    float *const Grad = J.grad;
    const int image = J.image;
    float *const SegP = (MODE == K2_FWD_STORE && J.seg_dtype == 0) ? J.seg + (int64_t)seg_step * 2 * J.seg_field : nullptr;
    float *const SegQ = SegP ? SegP + J.seg_field : nullptr;
    auto sp = [&](const float *f, int z) { return (gcchar *)(f + (int64_t)z * w.sy); };
    auto mp = [&](const float *f, int z) { return (gcchar *)(f + w.moff + (int64_t)z * w.my); };
    auto spw = [&](float *f, int z) { return (gchar *)(f + (int64_t)z * w.sy); };
    auto zok = [&](int z) { return (unsigned)z < (unsigned)w.nz; };
    auto slot = [](int z) { return ((z % Q) + Q) % Q; };

    // own columns: in-plane validity, byte offsets in state and model planes (0 when outside)
    bool ok[NY];
    uint32_t os[NY], om[NY];
    float exy[NY];
#pragma unroll
    for (int r = 0; r < NY; ++r) {
        const int y = y0 + ty * NY + r;
        ok[r] = gx < w.nx && y < w.ny;
        os[r] = ok[r] ? 4u * (uint32_t)(y * w.sx + gx) : 0u;
        om[r] = ok[r] ? 4u * (uint32_t)(y * w.mx + gx) : 0u;
        exy[r] = ok[r] ? gld(J.ex, gx) + gld(J.ey, y) : 0.f;
    }
    // halo items of this thread (slots past the list or outside the window plane load nothing)
    int hyy[NH], hxx[NH];
    bool hok[NH], hisx[NH];
    uint32_t hs[NH], hm[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const int i = tid + k * NT;
        int yy = 0, xx = 0;
        bool isx = false;
        if (i < IT::NHI) isx = IT::halo(i, yy, xx);
        const int x = x0 + xx, y = y0 + yy;
        hyy[k] = yy;
        hxx[k] = xx;
        hisx[k] = isx;
        hok[k] = i < IT::NHI && x >= 0 && y >= 0 && x < w.nx && y < w.ny;
        hs[k] = hok[k] ? 4u * (uint32_t)(y * w.sx + x) : 0u;
        hm[k] = hok[k] ? 4u * (uint32_t)(y * w.mx + x) : 0u;
    }
    // ring items
    bool rok[NO];
    uint32_t rs[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int i = tid + k * NT;
        int yy = 0, xx = 0;
        if (i < IT::NOI) IT::ring(i, yy, xx);
        const int x = x0 + xx, y = y0 + yy;
        rok[k] = i < IT::NOI && x >= 0 && y >= 0 && x < w.nx && y < w.ny;
        rs[k] = rok[k] ? 4u * (uint32_t)(y * w.sx + x) : 0u;
    }

    const int zs = z0 - R, ze = z1 + R;
    float qu[NY][Q], qv[NY][Q];                 // own columns: u, v over planes zf - R .. zf + R
    float at[NY][Q], as[NY][Q];                 // own columns: div t, div s of planes zf - R .. zf + R
    // before the first shift, own queue slot s holds plane zs - R + s - 1 (s = 1 .. 2R); the halo
    // ring holds planes zs - R .. zs + R - 1
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const int z = zs - R + s - 1;
        const bool zv = s >= 1 && zok(z);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            qu[r][s] = zv && ok[r] ? ldo(sp(U, z), os[r]) : 0.f;
            qv[r][s] = zv && ok[r] ? ldo(sp(V, z), os[r]) : 0.f;
            at[r][s] = as[r][s] = 0.f;
        }
    }
#pragma unroll
    for (int k = 0; k < NH; ++k)
        if (tid + k * NT < IT::NHI) {
            const int i = tid + k * NT;
            for (int z = zs - R; z < zs + R; ++z) {
                const bool v = zok(z) && hok[k];
                Hu[slot(z) * IT::NHI + i] = v ? ldo(sp(U, z), hs[k]) : 0.f;
                Hv[slot(z) * IT::NHI + i] = v ? ldo(sp(V, z), hs[k]) : 0.f;
            }
        }

    float nu[NY], nv[NY], on0[NY], on1[NY];     // next front zf: own u, v of plane zf + R; own axis of plane zf
    float hu[NH], hv[NH], hn0[NH], hn1[NH];     // ... the same for the halo items
    float ou[NO], ov[NO];                       // ... ring u, v of plane zf
    auto fetch = [&](int zf) {
        const bool za = zok(zf + R), zb = zok(zf);
        uint32_t fos[NY], fom[NY], fhs[NH], fhm[NH], frs[NO];
#pragma unroll
        for (int r = 0; r < NY; ++r) fos[r] = fresh(os[r]), fom[r] = fresh(om[r]);
#pragma unroll
        for (int k = 0; k < NH; ++k) fhs[k] = fresh(hs[k]), fhm[k] = fresh(hm[k]);
#pragma unroll
        for (int k = 0; k < NO; ++k) frs[k] = fresh(rs[k]);
        gcchar *bu = sp(U, zf + R), *bv = sp(V, zf + R), *cu = sp(U, zf), *cv = sp(V, zf);
        gcchar *bn0 = mp(Nx, zf), *bn1 = mp(Ny, zf);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            nu[r] = nv[r] = on0[r] = on1[r] = 0.f;
            if (za) {
                nu[r] = ldo(bu, fos[r]);
                nv[r] = ldo(bv, fos[r]);
            }
            if (zb) {
                on0[r] = ldo(bn0, fom[r]);
                on1[r] = ldo(bn1, fom[r]);
            }
        }
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            hu[k] = hv[k] = hn0[k] = hn1[k] = 0.f;
            if (za) {
                hu[k] = ldo(bu, fhs[k]);
                hv[k] = ldo(bv, fhs[k]);
            }
            if (zb) {
                hn0[k] = ldo(bn0, fhm[k]);
                hn1[k] = ldo(bn1, fhm[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            ou[k] = ov[k] = 0.f;
            if (zb) {
                ou[k] = ldo(cu, frs[k]);
                ov[k] = ldo(cv, frs[k]);
            }
        }
    };
    // update operands: current plane (v*) and next plane (nv*)
    float vp0[NY], vq0[NY], vp1[NY], vq1[NY], vm[NY], vA[NY], vB[NY], fpk[NY], fqk[NY], vg[NY];
    float nvp0[NY], nvq0[NY], nvp1[NY], nvq1[NY], nvm[NY], nvA[NY], nvB[NY];
    auto load_upd = [&](int zo) {
        const bool v = zo >= z0 && zo < z1;   // block-uniform
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const uint32_t uos = fresh(os[r]), uom = fresh(om[r]);
            nvp0[r] = nvq0[r] = nvp1[r] = nvq1[r] = nvm[r] = nvA[r] = nvB[r] = 0.f;
            if (v) {
                if (ADJ) {
                    nvp0[r] = ldo(sp(Pc, zo), uos);
                    nvq0[r] = ldo(sp(Qc, zo), uos);
                }
                nvp1[r] = ldo(sp(Pn, zo), uos);
                nvq1[r] = ldo(sp(Qn, zo), uos);
                nvm[r] = ldo(mp(Mm, zo), uom);
                nvA[r] = ldo(mp(MA, zo), uom);
                nvB[r] = ldo(mp(MB, zo), uom);
            }
        }
    };
    load_upd(zs - R);
    fetch(zs);
    for (int zf = zs; zf < ze; ++zf) {
        // 1. advance the queues (plane zf + R enters) and stage plane zf
        const int s0 = slot(zf - R);   // ring slot of plane zf - R; plane zf - R + j is in slot s0 + j (mod Q)
#pragma unroll
        for (int r = 0; r < NY; ++r) {
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qu[r][s] = qu[r][s + 1];
                qv[r][s] = qv[r][s + 1];
            }
            qu[r][Q - 1] = ok[r] ? nu[r] : 0.f;
            qv[r][Q - 1] = ok[r] ? nv[r] : 0.f;
            Lu[UP::at(ty * NY + r, tx)] = qu[r][R];
            Lv[UP::at(ty * NY + r, tx)] = qv[r][R];
        }
        {
            const int sl = s0 == 0 ? Q - 1 : s0 - 1;   // plane zf + R takes the slot of plane zf - R - 1
            const int sc = s0 + R >= Q ? s0 + R - Q : s0 + R;
#pragma unroll
            for (int k = 0; k < NH; ++k)
                if (tid + k * NT < IT::NHI) {
                    const int i = tid + k * NT;
                    Hu[sl * IT::NHI + i] = hok[k] ? hu[k] : 0.f;
                    Hv[sl * IT::NHI + i] = hok[k] ? hv[k] : 0.f;
                    Lu[UP::at(hyy[k], hxx[k])] = Hu[sc * IT::NHI + i];
                    Lv[UP::at(hyy[k], hxx[k])] = Hv[sc * IT::NHI + i];
                }
        }
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int i = tid + k * NT;
            if (i < IT::NOI) {
                int yy, xx;
                IT::ring(i, yy, xx);
                Lu[UP::at(yy, xx)] = rok[k] ? ou[k] : 0.f;
                Lv[UP::at(yy, xx)] = rok[k] ? ov[k] : 0.f;
            }
        }
        float a0[NY], a1[NY], b0[NH], b1[NH];
#pragma unroll
        for (int r = 0; r < NY; ++r) a0[r] = on0[r], a1[r] = on1[r];
#pragma unroll
        for (int k = 0; k < NH; ++k) b0[k] = hn0[k], b1[k] = hn1[k];
        __syncthreads();

        // plane zo = zf - R is updated in this iteration with the operands loaded one plane earlier;
        // the operands of plane zo + 1 are issued before the next plane's prefetch, so that the
        // wait for them in the next iteration does not wait for that prefetch as well
        const int zo = zf - R;
        const bool out = zo >= z0;
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            vp0[r] = ADJ ? nvp0[r] : qu[r][0];
            vq0[r] = ADJ ? nvq0[r] : qv[r][0];
            vp1[r] = nvp1[r];
            vq1[r] = nvq1[r];
            vm[r] = nvm[r];
            vA[r] = nvA[r];
            vB[r] = nvB[r];
        }
        // imaging-condition operands of plane zo: issued here, before the loads of the next planes
        // (a plane ahead they would cost three more registers than this mode has)
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            fpk[r] = fqk[r] = vg[r] = 0.f;
            if (MODE == K2_ADJ_IC && out) {
                const int y = ok[r] ? y0 + ty * NY + r : 0, x = ok[r] ? gx : 0;
                seg_load(J, seg_step, x, y, zo, sidx(w, x, y, zo), fpk[r], fqk[r]);
                vg[r] = ldo(sp(Grad, zo), fresh(os[r]));
            }
        }
        load_upd(zo + 1);
        if (zf + 1 < ze) fetch(zf + 1);

        // 2. t and s of plane zf: own columns (all components), halo (x or y components)
        const bool zin = zok(zf);
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int row = ty * NY + r;
            const int li = UP::at(row, tx);
            const float dux = dc_lds_x<R>(Lu, li, W.wx), duy = dc_lds_y<R, UP::LX>(Lu, li, W.wy);
            const float dvx = dc_lds_x<R>(Lv, li, W.wx), dvy = dc_lds_y<R, UP::LX>(Lv, li, W.wy);
            const float duz = dc_q<R>(qu[r], W.wz), dvz = dc_q<R>(qv[r], W.wz);
            const float n2 = axis_z(a0[r], a1[r]);
            const float wu = a0[r] * dux + a1[r] * duy + n2 * duz;
            const float wv = a0[r] * dvx + a1[r] * dvy + n2 * dvz;
            const bool in = zin && ok[r];
            Lt0[XP::at(row, tx)] = in ? dux - a0[r] * wu : 0.f;
            Ls0[XP::at(row, tx)] = in ? a0[r] * wv : 0.f;
            Lt1[YP::at(row, tx)] = in ? duy - a1[r] * wu : 0.f;
            Ls1[YP::at(row, tx)] = in ? a1[r] * wv : 0.f;
            const float tz = in ? duz - n2 * wu : 0.f, sz = in ? n2 * wv : 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                at[r][R - j] = __builtin_fmaf(W.wz[j - 1], tz, at[r][R - j]);
                at[r][R + j] = __builtin_fmaf(-W.wz[j - 1], tz, at[r][R + j]);
                as[r][R - j] = __builtin_fmaf(W.wz[j - 1], sz, as[r][R - j]);
                as[r][R + j] = __builtin_fmaf(-W.wz[j - 1], sz, as[r][R + j]);
            }
        }
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const int i = tid + k * NT;
            if (i >= IT::NHI) continue;
            const int li = UP::at(hyy[k], hxx[k]);
            const float dux = dc_lds_x<R>(Lu, li, W.wx), duy = dc_lds_y<R, UP::LX>(Lu, li, W.wy);
            const float dvx = dc_lds_x<R>(Lv, li, W.wx), dvy = dc_lds_y<R, UP::LX>(Lv, li, W.wy);
            float duz = 0.f, dvz = 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                int sP = s0 + R + j, sM = s0 + R - j;
                sP = sP >= Q ? sP - Q : sP;
                sM = sM >= Q ? sM - Q : sM;
                duz += W.wz[j - 1] * (Hu[sP * IT::NHI + i] - Hu[sM * IT::NHI + i]);
                dvz += W.wz[j - 1] * (Hv[sP * IT::NHI + i] - Hv[sM * IT::NHI + i]);
            }
            const float n2 = axis_z(b0[k], b1[k]);
            const float wu = b0[k] * dux + b1[k] * duy + n2 * duz;
            const float wv = b0[k] * dvx + b1[k] * dvy + n2 * dvz;
            const bool in = zin && hok[k];
            if (hisx[k]) {
                Lt0[XP::at(hyy[k], hxx[k])] = in ? dux - b0[k] * wu : 0.f;
                Ls0[XP::at(hyy[k], hxx[k])] = in ? b0[k] * wv : 0.f;
            } else {
                Lt1[YP::at(hyy[k], hxx[k])] = in ? duy - b1[k] * wu : 0.f;
                Ls1[YP::at(hyy[k], hxx[k])] = in ? b1[k] * wv : 0.f;
            }
        }
        __syncthreads();

        // 3. x-y divergence of plane zf; update of plane zo
        const float ezo = out ? gld(Ez, zo) : 0.f;
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int row = ty * NY + r;
            at[r][R] += dc_lds_x<R>(Lt0, XP::at(row, tx), W.wx) + dc_lds_y<R, PROP_TX>(Lt1, YP::at(row, tx), W.wy);
            as[r][R] += dc_lds_x<R>(Ls0, XP::at(row, tx), W.wx) + dc_lds_y<R, PROP_TX>(Ls1, YP::at(row, tx), W.wy);
            if (out && ok[r]) {
                const uint32_t uos = fresh(os[r]);
                const float h0 = at[r][0], hz = as[r][0];
                float Lp, Lq;
                if (ADJ) {
                    Lp = h0;
                    Lq = hz;
                } else {
                    Lp = vA[r] * h0 + vB[r] * hz;
                    Lq = vB[r] * h0 + hz;
                }
                const float mm = vm[r] * idt2 + 0.f;
                const float e = exy[r] + ezo;
                const float ra = 1.0f / (mm + e);
                const float cc = mm - e;
                const float np_ = (2.f * mm * vp0[r] - cc * vp1[r] + Lp) * ra;
                const float nq_ = (2.f * mm * vq0[r] - cc * vq1[r] + Lq) * ra;
                sto(spw(Pn, zo), uos, np_);
                sto(spw(Qn, zo), uos, nq_);
                if (ADJ) {
                    sto(spw(Wn0, zo), uos, vA[r] * np_ + vB[r] * nq_);
                    sto(spw(Wn1, zo), uos, vB[r] * np_ + nq_);
                }
                if (MODE == K2_FWD_STORE && SegP) {
                    sto(spw(SegP, zo), uos, np_);
                    sto(spw(SegQ, zo), uos, nq_);
                }
                if (MODE == K2_ADJ_IC)
                    sto(spw(Grad, zo), uos,
                        image ? vg[r] + (fpk[r] * np_ + fqk[r] * nq_)
                                : vg[r] - idt2 * (fpk[r] * (np_ - 2.f * vp0[r] + vp1[r]) +
                                                  fqk[r] * (nq_ - 2.f * vq0[r] + vq1[r])));
            }
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                at[r][s] = at[r][s + 1];
                as[r][s] = as[r][s + 1];
            }
            at[r][Q - 1] = as[r][Q - 1] = 0.f;
        }
    }
}

template <int R, int BY, int NY>
void pf_launch(int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par, const Weights &W,
               float idt2, int seg_step, hipStream_t st)
{
    dim3 blk(PROP_TX, BY), grd(ntiles);
    switch (mode) {
    case K2_FWD:
        hipLaunchKernelGGL((tti_fused<R, BY, NY, K2_FWD>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    case K2_FWD_STORE:
        hipLaunchKernelGGL((tti_fused<R, BY, NY, K2_FWD_STORE>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    case K2_ADJ:
        hipLaunchKernelGGL((tti_fused<R, BY, NY, K2_ADJ>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    default:
        hipLaunchKernelGGL((tti_fused<R, BY, NY, K2_ADJ_IC>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2,
                           seg_step);
        break;
    }
}

// Tile variants, both 64 x 16: 1 (the default) = 1024 threads of one row each, 0 = 512 threads of
// two rows each.  (A 64 x 32 tile would halve the y-halo work per point, but two rows of queues and
// accumulators per thread exceed the 128 registers a thread of a 1024-thread block may hold.)
// Space orders up to 12 (R <= 6): beyond that the halo queues outgrow the LDS of a CU.
template <int R>
void pf_dispatch(int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                 const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    if (shape == 1) pf_launch<R, 16, 1>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
    else            pf_launch<R, 8, 2>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);
}

}  // namespace

int tti_fused_max_radius() { return 6; }

void launch_tti_fused(int R, int shape, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, float idt2, int seg_step, hipStream_t st)
{
    switch (R) {
    case 1: pf_dispatch<1>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 2: pf_dispatch<2>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 3: pf_dispatch<3>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 4: pf_dispatch<4>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 5: pf_dispatch<5>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    case 6: pf_dispatch<6>(shape, mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st); break;
    default: break;   // rejected when the scheme is selected
    }
}
