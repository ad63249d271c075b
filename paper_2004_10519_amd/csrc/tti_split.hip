// Split single-field TTI step (gfx950): the operators of the fused pass, one field per launch.
//
// The rotated TTI operators in projector form (TTI section, Eq. "rot"): H0 u = div((I - n n^T) grad u)
// needs only u and Hz v = div(n (n . grad v)) needs only v.  The step therefore runs as two fused
// single-field passes instead of one two-field pass:
//   pass A: h = H0 u                    (read u and the axis, write h: 16 B per point)
//   pass B: Hz v, then the update       (read v, the axis, h, f and f- of p and q, m, A, B;
//           forward L = C (h, Hz v),     write p+, q+: 48 B per point; the adjoint reads and writes
//           adjoint L = (h, Hz v)        the w = C y pair as well)
// with (u, v) = (p, q) forward and w = C y adjoint.  Each pass has half the registers and LDS of the
// two-field pass, so the wide stencils (space order 12) keep every queue on chip without spilling.
// Both passes form their projections and divergences with the same expressions, in the same order,
// as the two-field pass, so h and Hz v are the same floats and the step gives the same bits.
//
// A block owns a TX x TY tile and the output planes [z0, z1) and marches a front plane zf from
// z0 - R to z1 + R - 1, as the two-field pass does: plane zf enters the z queues (own columns and
// the R-wide halo columns; a thread owns at most one halo column, whose queue it keeps in
// registers), plane zf is staged in LDS over the tile, the halo, a second R-wide ring and the
// corners; the projected gradient of plane zf is formed on the tile (all components) and on the
// halo (its x or y component); the z components are scattered into per-column accumulators of
// planes zf - R .. zf + R; plane zf - R is then complete.  The LDS planes are double-buffered, so a
// plane needs one barrier (pass A; pass B keeps a second one): the x-y divergence of plane zf - 1
// (read from the other buffer) joins its accumulator right after the barrier of plane zf, before
// plane zf's z components are scattered, which keeps every accumulator's order of additions that of
// the two-field pass.
#include "jobs.h"

#include <type_traits>

namespace {

// f(integral_constant<int, K>) for K = B .. E-1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int R, int TY>
struct SplitItems {
    static constexpr int NXI = 2 * R * TY, NYI = 2 * R * PROP_TX, NHI = NXI + NYI;
    static constexpr int NOX = 2 * R * TY, NOY = 2 * R * PROP_TX, NOC = 4 * R * R, NOI = NOX + NOY + NOC;
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


// PART 0: pass A (h = H0 u into J.t[0]).  PART 1: pass B (Hz v and the update), MODE as K2_*.
template <int R, int PART, int MODE>
__global__ __launch_bounds__(PROP_TX * 16) void tti_split(const TTIJob *__restrict__ jobs,
                                                         const Tile *__restrict__ tiles, int zc, int par, Weights W,
                                                         float idt2, int seg_step)
{
    constexpr int BY = 16, TY = 16, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool ADJ = (MODE == K2_ADJ || MODE == K2_ADJ_IC);
    using UP = Plane<2 * R, TY>;
    using XP = XPlane<R, TY>;
    using YP = YPlane<R, TY>;
    using IT = SplitItems<R, TY>;
    static_assert(IT::NHI <= NT, "one halo column per thread");
    constexpr int NO = (IT::NOI + NT - 1) / NT;
    // Double-buffered LDS (one barrier a plane) in pass A; pass B keeps single buffers and a second
    // barrier, since the deferred divergence adds registers that its update operands need.
    constexpr bool DB = PART == 0;
    constexpr int NB = DB ? 2 : 1;
    __shared__ float Lu[NB * UP::SIZE], Lt0[NB * XP::SIZE], Lt1[NB * YP::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const TTIJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    // the field of this pass and the job fields the march uses, read once before it
    const float *const U = PART == 0 ? (ADJ ? J.wmix[par][0] : J.p[par]) : (ADJ ? J.wmix[par][1] : J.q[par]);
    float *const Hb = J.t[0];
    const float *const Pc = J.p[par], *const Qc = J.q[par];
    float *const Pn = J.p[par ^ 1], *const Qn = J.q[par ^ 1];
    float *const Wn0 = ADJ ? J.wmix[par ^ 1][0] : nullptr, *const Wn1 = ADJ ? J.wmix[par ^ 1][1] : nullptr;
    const float *const Mm = J.m, *const MA = J.A, *const MB = J.B, *const Nx = J.nx, *const Ny = J.ny;
    const float *const Ez = J.ez;
    float *const Grad = J.grad;
    const int image = J.image;
    float *const SegP = (PART == 1 && MODE == K2_FWD_STORE && J.seg_dtype == 0)
                            ? J.seg + (int64_t)seg_step * 2 * J.seg_field : nullptr;
    float *const SegQ = SegP ? SegP + J.seg_field : nullptr;
    auto sp = [&](const float *f, int z) { return (gcchar *)(f + (int64_t)z * w.sy); };
    auto mp = [&](const float *f, int z) { return (gcchar *)(f + w.moff + (int64_t)z * w.my); };
    auto spw = [&](float *f, int z) { return (gchar *)(f + (int64_t)z * w.sy); };
    auto zok = [&](int z) { return (unsigned)z < (unsigned)w.nz; };

    // own column
    const bool ok = gx < w.nx && gy < w.ny;
    const uint32_t os = ok ? 4u * (uint32_t)(gy * w.sx + gx) : 0u;
    const uint32_t om = ok ? 4u * (uint32_t)(gy * w.mx + gx) : 0u;
    const float exy = ok ? gld(J.ex, gx) + gld(J.ey, gy) : 0.f;
    // halo column of this thread (if any)
    int hyy = 0, hxx = 0;
    const bool hitem = tid < IT::NHI;
    const bool hisx = hitem ? IT::halo(tid, hyy, hxx) : false;
    const bool hok = hitem && x0 + hxx >= 0 && y0 + hyy >= 0 && x0 + hxx < w.nx && y0 + hyy < w.ny;
    const uint32_t hs = hok ? 4u * (uint32_t)((y0 + hyy) * w.sx + x0 + hxx) : 0u;
    const uint32_t hm = hok ? 4u * (uint32_t)((y0 + hyy) * w.mx + x0 + hxx) : 0u;
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
    float qu[Q], hq[Q], at[Q];   // own u, halo-column u over planes zf - R .. zf + R; accumulators
    // before the first shift, slot s holds plane zs - R + s - 1 (s = 1 .. 2R)
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const int z = zs - R + s - 1;
        const bool zv = s >= 1 && zok(z);
        qu[s] = zv && ok ? ldo(sp(U, z), os) : 0.f;
        hq[s] = zv && hok ? ldo(sp(U, z), hs) : 0.f;
        at[s] = 0.f;
    }

    // next front zf: own u of plane zf + R, own axis of plane zf; halo; ring u of plane zf.  Pass A keeps
    // two sets, alternating with the plane, so a prefetch never overwrites operands still in use.
    float nu[NB], on0[NB], on1[NB], hu[NB], hn0[NB], hn1[NB], ou[NB][NO];
    auto fetch = [&](int zf, int f) {
        const bool za = zok(zf + R), zb = zok(zf);
        const uint32_t fos = fresh(os), fom = fresh(om), fhs = fresh(hs), fhm = fresh(hm);
        uint32_t frs[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) frs[k] = fresh(rs[k]);
        gcchar *bu = sp(U, zf + R), *cu = sp(U, zf);
        gcchar *bn0 = mp(Nx, zf), *bn1 = mp(Ny, zf);
        nu[f] = on0[f] = on1[f] = hu[f] = hn0[f] = hn1[f] = 0.f;
        if (za) {
            nu[f] = ldo(bu, fos);
            hu[f] = ldo(bu, fhs);
        }
        if (zb) {
            on0[f] = ldo(bn0, fom);
            on1[f] = ldo(bn1, fom);
            hn0[f] = ldo(bn0, fhm);
            hn1[f] = ldo(bn1, fhm);
        }
#pragma unroll
        for (int k = 0; k < NO; ++k) ou[f][k] = zb ? ldo(cu, frs[k]) : 0.f;
    };
    // update operands (pass B): current plane (v*) and next plane (nv*)
    float vp0 = 0.f, vq0 = 0.f, vp1 = 0.f, vq1 = 0.f, vm = 0.f, vA = 0.f, vB = 0.f, vh = 0.f;
    float nvp0 = 0.f, nvq0 = 0.f, nvp1 = 0.f, nvq1 = 0.f, nvm = 0.f, nvA = 0.f, nvB = 0.f, nvh = 0.f;
    auto load_upd = [&](int zo) {
        if (PART == 0) return;
        const bool v = zo >= z0 && zo < z1;   // block-uniform
        const uint32_t uos = fresh(os), uom = fresh(om);
        nvp0 = nvq0 = nvp1 = nvq1 = nvm = nvA = nvB = nvh = 0.f;
        if (v) {
            nvp0 = ldo(sp(Pc, zo), uos);
            if (ADJ) nvq0 = ldo(sp(Qc, zo), uos);
            nvp1 = ldo(sp(Pn, zo), uos);
            nvq1 = ldo(sp(Qn, zo), uos);
            nvm = ldo(mp(Mm, zo), uom);
            nvA = ldo(mp(MA, zo), uom);
            nvB = ldo(mp(MB, zo), uom);
            nvh = ldo(sp(Hb, zo), uos);
        }
    };
    load_upd(zs - R);
    fetch(zs, 0);
    // The march is unrolled by Q planes (2Q in pass A, so that its LDS buffer and prefetch set follow the
    // parity of K): in unrolled step K the three queues are rotated by K slots, so that advancing them
    // costs no register moves.  Logical slot s of the own and halo u queues (after plane zf + R has
    // entered) is register (s + K + 1) mod Q; accumulator slot s is register (s + K) mod Q.
    constexpr int UNR = NB * Q;
    for (int zb = zs; zb < ze; zb += UNR) {
        static_for<0, UNR>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const int zf = zb + K;
            if (zf >= ze) return;   // block-uniform
            auto U_ = [&](int s_) -> float & { return qu[(s_ + K + 1) % Q]; };
            auto H_ = [&](int s_) -> float & { return hq[(s_ + K + 1) % Q]; };
            auto A_ = [&](int s_) -> float & { return at[(s_ + K) % Q]; };
            // LDS buffers of plane zf (b) and of plane zf - 1 (b ^ 1)
            constexpr int b = DB ? K & 1 : 0, F = b;
            float *const Lub = Lu + b * UP::SIZE;
            float *const Lt0b = Lt0 + b * XP::SIZE, *const Lt1b = Lt1 + b * YP::SIZE;
            const float *const Lt0o = Lt0 + (b ^ 1) * XP::SIZE, *const Lt1o = Lt1 + (b ^ 1) * YP::SIZE;
            // 1. plane zf + R enters the queues (into the register of the plane that left); stage plane zf
            U_(Q - 1) = ok ? nu[F] : 0.f;
            H_(Q - 1) = hok ? hu[F] : 0.f;
            Lub[UP::at(ty, tx)] = U_(R);
            if (hitem) Lub[UP::at(hyy, hxx)] = H_(R);
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                const int i = tid + k * NT;
                if (i < IT::NOI) {
                    int yy, xx;
                    IT::ring(i, yy, xx);
                    Lub[UP::at(yy, xx)] = rok[k] ? ou[F][k] : 0.f;
                }
            }
            const float a0 = on0[F], a1 = on1[F], b0 = hn0[F], b1 = hn1[F];
            __syncthreads();

            // x-y divergence of plane zf - 1 (its x and y components were written before this barrier)
            if (DB && zf > zs)
                A_(R - 1) += dc_lds_x<R>(Lt0o, XP::at(ty, tx), W.wx) + dc_lds_y<R, PROP_TX>(Lt1o, YP::at(ty, tx), W.wy);

            // plane zo = zf - R is updated in this step with the operands loaded one plane earlier
            const int zo = zf - R;
            const bool out = zo >= z0;
            if (PART == 1) {
                vp0 = nvp0;
                vq0 = ADJ ? nvq0 : U_(0);
                vp1 = nvp1;
                vq1 = nvq1;
                vm = nvm;
                vA = nvA;
                vB = nvB;
                vh = nvh;
            }
            float fpk = 0.f, fqk = 0.f, vg = 0.f;
            if (PART == 1 && MODE == K2_ADJ_IC && out) {
                const int y = ok ? gy : 0, x = ok ? gx : 0;
                seg_load(J, seg_step, x, y, zo, sidx(w, x, y, zo), fpk, fqk);
                vg = ldo(sp(Grad, zo), fresh(os));
            }
            load_upd(zo + 1);
            if (zf + 1 < ze) fetch(zf + 1, F ^ (NB - 1));

            // 2. projected gradient of plane zf: own column (all components), halo column (x or y component)
            const bool zin = zok(zf);
            {
                const int li = UP::at(ty, tx);
                const float dux = dc_lds_x<R>(Lub, li, W.wx), duy = dc_lds_y<R, UP::LX>(Lub, li, W.wy);
                float duz = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) duz += W.wz[j - 1] * (U_(R + j) - U_(R - j));
                const float n2 = axis_z(a0, a1);
                const float wu = a0 * dux + a1 * duy + n2 * duz;
                const bool in = zin && ok;
                float tz;
                if (PART == 0) {
                    Lt0b[XP::at(ty, tx)] = in ? dux - a0 * wu : 0.f;
                    Lt1b[YP::at(ty, tx)] = in ? duy - a1 * wu : 0.f;
                    tz = in ? duz - n2 * wu : 0.f;
                } else {
                    Lt0b[XP::at(ty, tx)] = in ? a0 * wu : 0.f;
                    Lt1b[YP::at(ty, tx)] = in ? a1 * wu : 0.f;
                    tz = in ? n2 * wu : 0.f;
                }
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    A_(R - j) = __builtin_fmaf(W.wz[j - 1], tz, A_(R - j));
                    A_(R + j) = __builtin_fmaf(-W.wz[j - 1], tz, A_(R + j));
                }
            }
            if (hitem) {
                const int li = UP::at(hyy, hxx);
                const float dux = dc_lds_x<R>(Lub, li, W.wx), duy = dc_lds_y<R, UP::LX>(Lub, li, W.wy);
                float duz = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) duz += W.wz[j - 1] * (H_(R + j) - H_(R - j));
                const float n2 = axis_z(b0, b1);
                const float wu = b0 * dux + b1 * duy + n2 * duz;
                const bool in = zin && hok;
                if (hisx) Lt0b[XP::at(hyy, hxx)] = in ? (PART == 0 ? dux - b0 * wu : b0 * wu) : 0.f;
                else      Lt1b[YP::at(hyy, hxx)] = in ? (PART == 0 ? duy - b1 * wu : b1 * wu) : 0.f;
            }

            if (!DB) {
                // x-y divergence of plane zf
                __syncthreads();
                A_(R) += dc_lds_x<R>(Lt0, XP::at(ty, tx), W.wx) + dc_lds_y<R, PROP_TX>(Lt1, YP::at(ty, tx), W.wy);
            }

            // 3. plane zo complete (its x-y divergence has joined its accumulator)
            if (out && ok) {
                const uint32_t uos = fresh(os);
                if (PART == 0) {
                    sto(spw(Hb, zo), uos, A_(0));
                } else {
                    const float ezo = gld(Ez, zo);
                    const float h0 = vh, hz = A_(0);
                    float Lp, Lq;
                    if (ADJ) {
                        Lp = h0;
                        Lq = hz;
                    } else {
                        Lp = vA * h0 + vB * hz;
                        Lq = vB * h0 + hz;
                    }
                    const float mm = vm * idt2 + 0.f;
                    const float e = exy + ezo;
                    const float ra = 1.0f / (mm + e);
                    const float cc = mm - e;
                    const float np_ = (2.f * mm * vp0 - cc * vp1 + Lp) * ra;
                    const float nq_ = (2.f * mm * vq0 - cc * vq1 + Lq) * ra;
                    sto(spw(Pn, zo), uos, np_);
                    sto(spw(Qn, zo), uos, nq_);
                    if (ADJ) {
                        sto(spw(Wn0, zo), uos, vA * np_ + vB * nq_);
                        sto(spw(Wn1, zo), uos, vB * np_ + nq_);
                    }
                    if (MODE == K2_FWD_STORE && SegP) {
                        sto(spw(SegP, zo), uos, np_);
                        sto(spw(SegQ, zo), uos, nq_);
                    }
                    if (MODE == K2_ADJ_IC)
                        sto(spw(Grad, zo), uos,
                            image ? vg + (fpk * np_ + fqk * nq_)
                                  : vg - idt2 * (fpk * (np_ - 2.f * vp0 + vp1) + fqk * (nq_ - 2.f * vq0 + vq1)));
                }
            }
            A_(0) = 0.f;   // the register of the completed plane becomes the newest accumulator slot
        });
    }
}

template <int R, int PART>
void sp_launch(int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par, const Weights &W,
               float idt2, int seg_step, hipStream_t st)
{
    dim3 blk(PROP_TX, 16), grd(ntiles);
    if (PART == 0) {
        // pass A does not depend on the mode beyond the direction (which field is u)
        if (mode == K2_ADJ || mode == K2_ADJ_IC)
            hipLaunchKernelGGL((tti_split<R, 0, K2_ADJ>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        else
            hipLaunchKernelGGL((tti_split<R, 0, K2_FWD>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        return;
    }
    switch (mode) {
    case K2_FWD:
        hipLaunchKernelGGL((tti_split<R, 1, K2_FWD>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    case K2_FWD_STORE:
        hipLaunchKernelGGL((tti_split<R, 1, K2_FWD_STORE>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    case K2_ADJ:
        hipLaunchKernelGGL((tti_split<R, 1, K2_ADJ>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    default:
        hipLaunchKernelGGL((tti_split<R, 1, K2_ADJ_IC>), grd, blk, 0, st, jobs, tiles, zc, par, W, idt2, seg_step);
        break;
    }
}

}  // namespace

int tti_split_max_radius() { return 6; }

void launch_tti_split(int R, int part, int mode, const TTIJob *jobs, const Tile *tiles, int ntiles, int zc, int par,
                      const Weights &W, float idt2, int seg_step, hipStream_t st)
{
#define SP_CASE(RR)                                                                                  \
    case RR:                                                                                         \
        if (part == 0) sp_launch<RR, 0>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);  \
        else sp_launch<RR, 1>(mode, jobs, tiles, ntiles, zc, par, W, idt2, seg_step, st);            \
        break;
    switch (R) {
        SP_CASE(1)
        SP_CASE(2)
        SP_CASE(3)
        SP_CASE(4)
        SP_CASE(5)
        SP_CASE(6)
    default: break;   // rejected when the scheme is selected
    }
#undef SP_CASE
}
