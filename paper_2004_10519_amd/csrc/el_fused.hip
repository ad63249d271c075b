// Fused velocity-stress step of the isotropic elastic system on a staggered grid (3D, gfx950).
//
// One launch per time step does what the velocity pass and the stress pass do in two (the elastic
// listing: velocities from the stresses, then stresses from the new velocities):
//   v+   = g (v + dt bbar (D_tau tau))
//   tau+ = g (tau + dt C E v+)
// reading v, tau and the parameters once and writing v+ and tau+ once (84 bytes a point against 120
// for the two passes).  The state is double-buffered: a step reads one buffer set and writes the
// other, because a block recomputes v+ on an R-wide ring around its tile from the old stresses of
// its neighbours' tiles, which must not change under it.
//
// A block owns an EF_TX x EF_TY (32 x 16) tile and the output planes [z0, z1) and marches a front
// plane zf from z0 - R to z1 + R - 1.  Per front plane:
//   1. the old stresses of plane zf are staged in LDS over the tile and a 2R ring (x and y
//      derivatives of the velocity update); tau_zz, tau_xz, tau_yz also enter z queues (registers
//      for the tile's own columns, LDS for the ring's columns);
//   2. v+ of plane zf is formed on the tile and its R-wide ring (not the corners), with the same
//      expressions as the velocity pass; the tile's own v+ is stored (planes inside the chunk),
//      all of it goes to an LDS plane, and the own v+ enters z queues;
//   3. the stress update of plane zf - R: its z derivatives from the v+ queues, its x and y
//      derivatives formed R planes earlier from the LDS plane of v+ and held in a register delay
//      line; the sums are those of the stress pass, term for term.
// The march is unrolled by 2R planes, so the queues (length 2R) and the delay line (length R)
// rotate by register index.  v+ is recomputed on 2R planes beyond each chunk (the stress of the
// chunk's end planes needs them), so chunks are long.
#include "jobs.h"

#include <type_traits>

namespace {

template <int B, int E, class F>
__device__ __forceinline__ void ef_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        ef_for<B + 1, E>(f);
    }
}

template <int R>
struct EFGeom {
    static constexpr int TX = EF_TX, TY = EF_TY, NT = TX * TY;
    // stress planes: tile with a 2R ring
    static constexpr int LT = TX + 4 * R, HT = TY + 4 * R, ST = LT * HT;
    // velocity plane: tile with an R ring (the corners are not used)
    static constexpr int LV = TX + 2 * R, HV = TY + 2 * R, SV = LV * HV;
    // buoyancy plane: [-R, TX + R] x [-R, TY + R]
    static constexpr int LB = TX + 2 * R + 1, HB = TY + 2 * R + 1, SB = LB * HB;
    // ring points of the velocity update: x ring (2R columns beside the tile rows), y ring
    static constexpr int NXI = 2 * R * TY, NH = NXI + 2 * R * TX;
    // the rest of the stress planes: rows beyond the velocity ring, the corners of the velocity
    // ring and its outer 2R-wide band, the outer columns beside the tile rows
    static constexpr int RA = 2 * R * LT, RB = 2 * R * 4 * R, RC = TY * 2 * R, NRI = RA + RB + RC;
    static constexpr int NO = (NRI + NT - 1) / NT;   // outer points per thread
    static_assert(NH <= NT, "one ring point per thread");
    __device__ static __forceinline__ int at_t(int yy, int xx) { return (yy + 2 * R) * LT + xx + 2 * R; }
    __device__ static __forceinline__ int at_v(int yy, int xx) { return (yy + R) * LV + xx + R; }
    __device__ static __forceinline__ int at_b(int yy, int xx) { return (yy + R) * LB + xx + R; }
    __device__ static __forceinline__ void halo(int i, int &yy, int &xx)
    {
        if (i < NXI) {
            const int row = i / (2 * R), c = i - row * (2 * R);
            yy = row;
            xx = c < R ? c - R : TX + c - R;
            return;
        }
        i -= NXI;
        const int rr = i / TX;
        xx = i - rr * TX;
        yy = rr < R ? rr - R : TY + rr - R;
    }
    __device__ static __forceinline__ void outer(int i, int &yy, int &xx)
    {
        if (i < RA) {
            const int r = i / LT, c = i - r * LT;
            yy = r < R ? r - 2 * R : TY + r;   // rows [-2R, -R) and [TY + R, TY + 2R)
            xx = c - 2 * R;
            return;
        }
        i -= RA;
        if (i < RB) {
            const int r = i / (4 * R), c = i - r * (4 * R);
            yy = r < R ? r - R : TY + r - R;   // rows [-R, 0) and [TY, TY + R)
            xx = c < 2 * R ? c - 2 * R : TX + c - 2 * R;
            return;
        }
        i -= RB;
        const int r = i / (2 * R), c = i - r * (2 * R);
        yy = r;
        xx = c < R ? c - 2 * R : TX + R + c - R;   // columns [-2R, -R) and [TX + R, TX + 2R)
    }
};


template <int R>
__global__ __launch_bounds__(EF_TX * EF_TY) void el_fused(const ElFusedJob *__restrict__ jobs,
                                                        const Tile *__restrict__ tiles, int zc, Weights W, float dt)
{
    using G = EFGeom<R>;
    constexpr int TX = G::TX, TY = G::TY, NT = G::NT, U = 2 * R;
    __shared__ float Lt[5][G::ST];            // old txx, tyy, txy, txz, tyz of plane zf
    __shared__ float Lv[3][G::SV];            // new vx, vy, vz of plane zf
    __shared__ float Lb[G::SB];               // buoyancy of plane zf (clamped at the window's far edges)
    __shared__ float Hq[3][U][G::NH];         // ring columns' z queues: tzz, txz, tyz

    const Tile tl = tiles[blockIdx.x];
    const ElFusedJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    auto sp = [&](const float *f, int z) { return (gcchar *)(f + (int64_t)z * w.sy); };
    auto mp = [&](const float *f, int z) { return (gcchar *)(f + w.moff + (int64_t)z * w.my); };
    auto spw = [&](float *f, int z) { return (gchar *)(f + (int64_t)z * w.sy); };
    auto zok = [&](int z) { return (unsigned)z < (unsigned)w.nz; };
    const float *const Txx = J.ti[0], *const Tyy = J.ti[1], *const Tzz = J.ti[2];
    const float *const Txy = J.ti[3], *const Txz = J.ti[4], *const Tyz = J.ti[5];
    const float *const Bm = J.b, *const Lm = J.lam, *const Mm = J.mu;

    // own column
    const bool ok = gx < w.nx && gy < w.ny;
    const uint32_t os = ok ? 4u * (uint32_t)(gy * w.sx + gx) : 0u;
    const uint32_t om = ok ? 4u * (uint32_t)(gy * w.mx + gx) : 0u;
    const uint32_t dmx = gx + 1 < w.nx ? 4u : 0u, dmy = gy + 1 < w.ny ? 4u * (uint32_t)w.mx : 0u;
    const float gxy = ok ? gld(J.gx, gx) * gld(J.gy, gy) : 0.f;
    // ring column of the velocity update (if any)
    int hyy = 0, hxx = 0;
    const bool hitem = tid < G::NH;
    if (hitem) G::halo(tid, hyy, hxx);
    const int hX = x0 + hxx, hY = y0 + hyy;
    const bool hok = hitem && hX >= 0 && hY >= 0 && hX < w.nx && hY < w.ny;
    const uint32_t hs = hok ? 4u * (uint32_t)(hY * w.sx + hX) : 0u;
    const float hgxy = hok ? gld(J.gx, hX) * gld(J.gy, hY) : 0.f;
    // outer points of the stress planes (NO per thread); their buoyancy feeds the plane
    // [-R, TX + R] x [-R, TY + R]
    constexpr int NO = G::NO;
    int ryy[NO], rxx[NO];
    bool ritem[NO], rok[NO], rbin[NO];
    uint32_t rs[NO], rbm[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int i = tid + k * NT;
        ryy[k] = rxx[k] = 0;
        ritem[k] = i < G::NRI;
        if (ritem[k]) G::outer(i, ryy[k], rxx[k]);
        const int rX = x0 + rxx[k], rY = y0 + ryy[k];
        rok[k] = ritem[k] && rX >= 0 && rY >= 0 && rX < w.nx && rY < w.ny;
        rs[k] = rok[k] ? 4u * (uint32_t)(rY * w.sx + rX) : 0u;
        rbin[k] = ritem[k] && rxx[k] >= -R && rxx[k] <= TX + R && ryy[k] >= -R && ryy[k] <= TY + R && rX >= 0 &&
                  rY >= 0;
        rbm[k] = rbin[k] ? 4u * (uint32_t)(min(rY, w.ny - 1) * w.mx + min(rX, w.nx - 1)) : 0u;
    }
    // buoyancy of the own and ring columns in the plane (clamped beyond the far edges)
    const bool obin = gx <= w.nx && gy <= w.ny;   // the columns whose buoyancy a velocity update reads
    const uint32_t obm = 4u * (uint32_t)(min(gy, w.ny - 1) * w.mx + min(gx, w.nx - 1));
    const bool hbin = hitem && hX >= 0 && hY >= 0;
    const uint32_t hbm = hbin ? 4u * (uint32_t)(min(hY, w.ny - 1) * w.mx + min(hX, w.nx - 1)) : 0u;

    const int zs0 = z0 - R, ze = z1 + R;
    // own z queues (register index = (logical slot + K) mod 2R in unrolled step K):
    //   qzz slot s: plane zf - R + 1 + s;  qxz, qyz slot s: plane zf - R + s
    //   vx, vy slot s: plane zf - 2R + 1 + s (after v+ of zf entered);  vz slot s: plane zf - 2R + s
    //   (before v+ of zf entered);  delay line slot s: in-plane stress terms of plane zf - R + s
    float qzz[U], qxz[U], qyz[U], qvx[U], qvy[U], qvz[U];
    float dxx[R], dyy[R], dxy[R], dxz[R], dyz[R];
#pragma unroll
    for (int s = 0; s < U; ++s) {
        qzz[s] = qxz[s] = qyz[s] = 0.f;
        qvx[s] = qvy[s] = qvz[s] = 0.f;
    }
#pragma unroll
    for (int s = 0; s < R; ++s) dxx[s] = dyy[s] = dxy[s] = dxz[s] = dyz[s] = 0.f;
    // fill: slots 0 .. 2R-2 for the first front zs0 (register index = slot at K = 0)
#pragma unroll
    for (int s = 0; s < U - 1; ++s) {
        const int za = zs0 - R + 1 + s, zb = zs0 - R + s;
        qzz[s] = ok && zok(za) ? ldo(sp(Tzz, za), os) : 0.f;
        qxz[s] = ok && zok(zb) ? ldo(sp(Txz, zb), os) : 0.f;
        qyz[s] = ok && zok(zb) ? ldo(sp(Tyz, zb), os) : 0.f;
        if (hitem) {
            Hq[0][s][tid] = hok && zok(za) ? ldo(sp(Tzz, za), hs) : 0.f;
            Hq[1][s][tid] = hok && zok(zb) ? ldo(sp(Txz, zb), hs) : 0.f;
            Hq[2][s][tid] = hok && zok(zb) ? ldo(sp(Tyz, zb), hs) : 0.f;
        }
    }

    // prefetched operands of the next front zf: z-queue fronts (tzz of zf + R, txz and tyz of
    // zf + R - 1), the in-plane stresses of zf, buoyancy (own and ring: of zf + 1; outer: of zf)
    float nzz, nxz, nyz, nxx, nyy, nxy, nb;
    float hzz, hxz, hyz, hxx_, hyy_, hxy, hb;
    float rxx_[NO], ryy_[NO], rxy[NO], rxz[NO], ryz[NO], rb[NO];
    auto fetch = [&](int zf) {
        const bool za = zok(zf + R), zb = zok(zf + R - 1), zc0 = zok(zf);
        const int zbn = min(zf + 1, w.nz - 1);
        const uint32_t fos = fresh(os), fhs = fresh(hs);
        nzz = ok && za ? ldo(sp(Tzz, zf + R), fos) : 0.f;
        nxz = ok && zb ? ldo(sp(Txz, zf + R - 1), fos) : 0.f;
        nyz = ok && zb ? ldo(sp(Tyz, zf + R - 1), fos) : 0.f;
        nxx = ok && zc0 ? ldo(sp(Txx, zf), fos) : 0.f;
        nyy = ok && zc0 ? ldo(sp(Tyy, zf), fos) : 0.f;
        nxy = ok && zc0 ? ldo(sp(Txy, zf), fos) : 0.f;
        nb = zf + 1 >= 0 ? ldo(mp(Bm, zbn), fresh(obm)) : 0.f;
        hzz = hok && za ? ldo(sp(Tzz, zf + R), fhs) : 0.f;
        hxz = hok && zb ? ldo(sp(Txz, zf + R - 1), fhs) : 0.f;
        hyz = hok && zb ? ldo(sp(Tyz, zf + R - 1), fhs) : 0.f;
        hxx_ = hok && zc0 ? ldo(sp(Txx, zf), fhs) : 0.f;
        hyy_ = hok && zc0 ? ldo(sp(Tyy, zf), fhs) : 0.f;
        hxy = hok && zc0 ? ldo(sp(Txy, zf), fhs) : 0.f;
        hb = hbin && zf + 1 >= 0 ? ldo(mp(Bm, zbn), fresh(hbm)) : 0.f;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const uint32_t frs = fresh(rs[k]);
            rxx_[k] = rok[k] && zc0 ? ldo(sp(Txx, zf), frs) : 0.f;
            ryy_[k] = rok[k] && zc0 ? ldo(sp(Tyy, zf), frs) : 0.f;
            rxy[k] = rok[k] && zc0 ? ldo(sp(Txy, zf), frs) : 0.f;
            rxz[k] = rok[k] && zc0 ? ldo(sp(Txz, zf), frs) : 0.f;
            ryz[k] = rok[k] && zc0 ? ldo(sp(Tyz, zf), frs) : 0.f;
            rb[k] = rbin[k] && zc0 ? ldo(mp(Bm, zf), fresh(rbm[k])) : 0.f;
        }
    };
    // buoyancy of plane zf at the own and ring columns (the first front's is loaded here)
    float ob = zok(zs0) && obin ? ldo(mp(Bm, zs0), obm) : 0.f;
    float hb0 = hbin && zok(zs0) ? ldo(mp(Bm, zs0), hbm) : 0.f;
    fetch(zs0);

    for (int zb = zs0; zb < ze; zb += U) {
        ef_for<0, U>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const int zf = zb + K;
            if (zf >= ze) return;   // block-uniform
            auto QZZ = [&](int s) -> float & { return qzz[(s + K) % U]; };
            auto QXZ = [&](int s) -> float & { return qxz[(s + K) % U]; };
            auto QYZ = [&](int s) -> float & { return qyz[(s + K) % U]; };
            auto VX = [&](int s) -> float & { return qvx[(s + K) % U]; };
            auto VY = [&](int s) -> float & { return qvy[(s + K) % U]; };
            auto VZ = [&](int s) -> float & { return qvz[(s + K) % U]; };
            constexpr int KD = K % R;
            auto DXX = [&](int s) -> float & { return dxx[(s + KD) % R]; };
            auto DYY = [&](int s) -> float & { return dyy[(s + KD) % R]; };
            auto DXY = [&](int s) -> float & { return dxy[(s + KD) % R]; };
            auto DXZ = [&](int s) -> float & { return dxz[(s + KD) % R]; };
            auto DYZ = [&](int s) -> float & { return dyz[(s + KD) % R]; };
            const int hq_front = (U - 1 + K) % U;   // ring queue register of the entering planes
            const bool zin = zok(zf);

            // 1. queue fronts enter; stage the old stresses and the buoyancy of plane zf
            QZZ(U - 1) = nzz;
            QXZ(U - 1) = nxz;
            QYZ(U - 1) = nyz;
            {
                const int li = G::at_t(ty, tx);
                Lt[0][li] = nxx;
                Lt[1][li] = nyy;
                Lt[2][li] = nxy;
                Lt[3][li] = QXZ(R);
                Lt[4][li] = QYZ(R);
                Lb[G::at_b(ty, tx)] = ob;
            }
            if (hitem) {
                Hq[0][hq_front][tid] = hzz;
                Hq[1][hq_front][tid] = hxz;
                Hq[2][hq_front][tid] = hyz;
                const int li = G::at_t(hyy, hxx);
                Lt[0][li] = hxx_;
                Lt[1][li] = hyy_;
                Lt[2][li] = hxy;
                Lt[3][li] = Hq[1][(R + K) % U][tid];
                Lt[4][li] = Hq[2][(R + K) % U][tid];
                Lb[G::at_b(hyy, hxx)] = hb0;
            }
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                if (ritem[k]) {
                    const int li = G::at_t(ryy[k], rxx[k]);
                    Lt[0][li] = rxx_[k];
                    Lt[1][li] = ryy_[k];
                    Lt[2][li] = rxy[k];
                    Lt[3][li] = rxz[k];
                    Lt[4][li] = ryz[k];
                    if (rxx[k] >= -R && rxx[k] <= TX + R && ryy[k] >= -R && ryy[k] <= TY + R)
                        Lb[G::at_b(ryy[k], rxx[k])] = rb[k];
                }
            }
            const float obz = nb, hbz = hb;   // buoyancy of plane zf + 1 (clamped)
            __syncthreads();

            // 2. operands of this plane's velocity update, then the next front's prefetch
            const uint32_t vos = fresh(os), vhs = fresh(hs);
            const float v0 = ok && zin ? ldo(sp(J.vi[0], zf), vos) : 0.f;
            const float v1 = ok && zin ? ldo(sp(J.vi[1], zf), vos) : 0.f;
            const float v2 = ok && zin ? ldo(sp(J.vi[2], zf), vos) : 0.f;
            const float hv0 = hok && zin ? ldo(sp(J.vi[0], zf), vhs) : 0.f;
            const float hv1 = hok && zin ? ldo(sp(J.vi[1], zf), vhs) : 0.f;
            const float hv2 = hok && zin ? ldo(sp(J.vi[2], zf), vhs) : 0.f;
            const float gz = zin ? gld(J.gz, zf) : 0.f;
            if (zf + 1 < ze) fetch(zf + 1);

            // 3. v+ of plane zf: own column (z derivatives from the register queues) and ring
            //    column (from the LDS queues), with the velocity pass's expressions
            float vn0 = 0.f, vn1 = 0.f, vn2 = 0.f;
            {
                const int li = G::at_t(ty, tx), lb = G::at_b(ty, tx);
                float szx = 0.f, szy = 0.f, szz = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    szx += W.wz[j - 1] * (QXZ(R + j - 1) - QXZ(R - j));
                    szy += W.wz[j - 1] * (QYZ(R + j - 1) - QYZ(R - j));
                    szz += W.wz[j - 1] * (QZZ(R - 1 + j) - QZZ(R - j));
                }
                const float fx = ds_lds<R, true>(Lt[0], li, 1, W.wx) + ds_lds<R, false>(Lt[2], li, G::LT, W.wy) + szx;
                const float fy = ds_lds<R, false>(Lt[2], li, 1, W.wx) + ds_lds<R, true>(Lt[1], li, G::LT, W.wy) + szy;
                const float fz = ds_lds<R, false>(Lt[3], li, 1, W.wx) + ds_lds<R, false>(Lt[4], li, G::LT, W.wy) + szz;
                if (ok && zin) {
                    const float b0 = Lb[lb], bxn = Lb[lb + 1], byn = Lb[lb + G::LB];
                    const float g = gxy * gz;
                    vn0 = g * (v0 + dt * (0.5f * (b0 + bxn)) * fx);
                    vn1 = g * (v1 + dt * (0.5f * (b0 + byn)) * fy);
                    vn2 = g * (v2 + dt * (0.5f * (b0 + obz)) * fz);
                    if (zf >= z0 && zf < z1) {
                        const uint32_t uos = fresh(os);
                        sto(spw(J.vo[0], zf), uos, vn0);
                        sto(spw(J.vo[1], zf), uos, vn1);
                        sto(spw(J.vo[2], zf), uos, vn2);
                    }
                }
                const int lv = G::at_v(ty, tx);
                Lv[0][lv] = vn0;
                Lv[1][lv] = vn1;
                Lv[2][lv] = vn2;
            }
            if (hitem) {
                const int li = G::at_t(hyy, hxx), lb = G::at_b(hyy, hxx);
                float szx = 0.f, szy = 0.f, szz = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    szx += W.wz[j - 1] * (Hq[1][(R + j - 1 + K) % U][tid] - Hq[1][(R - j + K) % U][tid]);
                    szy += W.wz[j - 1] * (Hq[2][(R + j - 1 + K) % U][tid] - Hq[2][(R - j + K) % U][tid]);
                    szz += W.wz[j - 1] * (Hq[0][(R - 1 + j + K) % U][tid] - Hq[0][(R - j + K) % U][tid]);
                }
                const float fx = ds_lds<R, true>(Lt[0], li, 1, W.wx) + ds_lds<R, false>(Lt[2], li, G::LT, W.wy) + szx;
                const float fy = ds_lds<R, false>(Lt[2], li, 1, W.wx) + ds_lds<R, true>(Lt[1], li, G::LT, W.wy) + szy;
                const float fz = ds_lds<R, false>(Lt[3], li, 1, W.wx) + ds_lds<R, false>(Lt[4], li, G::LT, W.wy) + szz;
                float a0 = 0.f, a1 = 0.f, a2 = 0.f;
                if (hok && zin) {
                    const float b0 = Lb[lb], bxn = Lb[lb + 1], byn = Lb[lb + G::LB];
                    const float g = hgxy * gz;
                    a0 = g * (hv0 + dt * (0.5f * (b0 + bxn)) * fx);
                    a1 = g * (hv1 + dt * (0.5f * (b0 + byn)) * fy);
                    a2 = g * (hv2 + dt * (0.5f * (b0 + hbz)) * fz);
                }
                const int lv = G::at_v(hyy, hxx);
                Lv[0][lv] = a0;
                Lv[1][lv] = a1;
                Lv[2][lv] = a2;
            }
            VX(U - 1) = vn0;
            VY(U - 1) = vn1;
            ob = obz;
            hb0 = hbz;
            __syncthreads();

            // 4. stress update of plane zs = zf - R (z terms from the v+ queues, x-y terms from the
            //    delay line), with the stress pass's expressions
            const int zs = zf - R;
            if (zs >= z0 && ok) {
                const uint32_t tos = fresh(os), tom = fresh(om);
                const uint32_t tomx = tom + dmx, tomy = tom + dmy, tomxy = tomx + dmy;
                const int64_t oz = zs + 1 < w.nz ? w.my : 0;
                float t[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) t[c] = ldo(sp(J.ti[c], zs), tos);
                gcchar *ml = mp(Lm, zs), *mu_ = mp(Mm, zs), *muz = mp(Mm, zs) + 4 * oz;
                const float lam = ldo(ml, tom);
                const float mu0 = ldo(mu_, tom);
                const float mx_ = ldo(mu_, tomx), mz_ = ldo(muz, tom), my_ = ldo(mu_, tomy);
                const float mxz = 0.25f * (mu0 + mx_ + mz_ + ldo(muz, tomx));
                const float mxy = 0.25f * (mu0 + mx_ + my_ + ldo(mu_, tomxy));
                const float myz = 0.25f * (mu0 + my_ + mz_ + ldo(muz, tomy));
                const float g = gxy * gld(J.gz, zs);
                float ezz = 0.f, gxz_z = 0.f, gyz_z = 0.f;
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    ezz += W.wz[j - 1] * (VZ(R + j - 1) - VZ(R - j));
                    gxz_z += W.wz[j - 1] * (VX(R + j - 1) - VX(R - j));
                    gyz_z += W.wz[j - 1] * (VY(R + j - 1) - VY(R - j));
                }
                const float exx = DXX(0), eyy = DYY(0), gxy_ = DXY(0);
                const float gxz = gxz_z + DXZ(0), gyz = gyz_z + DYZ(0);
                const float lt = lam * (exx + eyy + ezz), m2 = 2.f * mu0;
                const uint32_t uos = fresh(os);
                sto(spw(J.to[0], zs), uos, g * (t[0] + dt * (lt + m2 * exx)));
                sto(spw(J.to[1], zs), uos, g * (t[1] + dt * (lt + m2 * eyy)));
                sto(spw(J.to[2], zs), uos, g * (t[2] + dt * (lt + m2 * ezz)));
                sto(spw(J.to[3], zs), uos, g * (t[3] + dt * mxy * gxy_));
                sto(spw(J.to[4], zs), uos, g * (t[4] + dt * mxz * gxz));
                sto(spw(J.to[5], zs), uos, g * (t[5] + dt * myz * gyz));
            }
            VZ(0) = vn2;   // the register of plane zf - 2R now holds v+_z of zf
            // 5. x-y terms of the stress update of plane zf from the LDS plane of v+
            {
                const int lv = G::at_v(ty, tx);
                DXX(0) = ds_lds<R, false>(Lv[0], lv, 1, W.wx);
                DYY(0) = ds_lds<R, false>(Lv[1], lv, G::LV, W.wy);
                DXY(0) = ds_lds<R, true>(Lv[0], lv, G::LV, W.wy) + ds_lds<R, true>(Lv[1], lv, 1, W.wx);
                DXZ(0) = ds_lds<R, true>(Lv[2], lv, 1, W.wx);
                DYZ(0) = ds_lds<R, true>(Lv[2], lv, G::LV, W.wy);
            }
        });
    }
}

template <int R>
void ef_launch(const ElFusedJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt, hipStream_t st)
{
    hipLaunchKernelGGL((el_fused<R>), dim3(ntiles), dim3(EF_TX, EF_TY), 0, st, jobs, tiles, zc, W, dt);
}

}  // namespace

int el_fused_max_radius() { return 4; }

void launch_el_fused(int R, const ElFusedJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt,
                     hipStream_t st)
{
    switch (R) {
    case 1: ef_launch<1>(jobs, tiles, ntiles, zc, W, dt, st); break;
    case 2: ef_launch<2>(jobs, tiles, ntiles, zc, W, dt, st); break;
    case 3: ef_launch<3>(jobs, tiles, ntiles, zc, W, dt, st); break;
    case 4: ef_launch<4>(jobs, tiles, ntiles, zc, W, dt, st); break;
    default: break;   // rejected when the path is selected
    }
}
