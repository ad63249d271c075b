// Isotropic elastic velocity-stress kernels on a staggered grid (gfx950).
//
// Field positions (storage index i holds the listed position):
//   txx, tyy, tzz (i, j, k)   vx (i+1/2, j, k)   vy (i, j+1/2, k)   vz (i, j, k+1/2)
//   txy (i+1/2, j+1/2, k)     txz (i+1/2, j, k+1/2)                tyz (i, j+1/2, k+1/2)
// Staggered derivatives: D+ (node -> half node) and D- (half node -> node), with (D+)^T = -D-
// under truncation.  Half-node parameters are arithmetic means of the neighbouring nodes,
// clamped at the last index of the window.
//
// Forward step (the elastic listing: velocities first, then stresses from the new velocities,
// both multiplied by the absorbing factor g):
//   v   <- g (v + dt bbar (D_tau tau))
//   tau <- g (tau + dt C E v)
// Adjoint step (exact transpose, applied in reverse): with sigma = C (g tau~) and u = bbar (g v~)
//   v~ <- g (v~ + dt E^T sigma);   then   tau~ <- g tau~ + dt D_tau^T u,
// where E^T = -(the D_tau pattern) and D_tau^T = -(the E pattern), so the adjoint reuses the two
// forward stencil kernels on the pointwise-weighted fields with a minus sign.  Two launches a
// step: el_vel updates v~ from sigma and forms u in its epilogue; el_stress applies g to tau~ while
// it adds dt D_tau^T u, and forms sigma of the new tau~ for the next step in its epilogue (the
// diagonal components are recomputed at the receiver-injection nodes after the injection).
#include "jobs.h"

namespace {

// Tile rows (= threads in y, one row each): 16 on 3D grids (the launchers also take 8); 2D grids
// (ny = 1) use one row, so a block is a single wavefront and no y-halo work is done (its y
// derivatives are zero).
constexpr int EBY = 16;
// 64 x 8 tiles (512 threads) are built for three blocks a CU, 6 waves a SIMD (at most 80 VGPRs) up
// to space order 8; beyond it their registers would spill, and they take what they need.
constexpr int EL_NARROW_WAVES = 6;

// Velocity pass.  Fields read: F[0..5] = (xx, yy, zz, xy, xz, yz) stresses (forward: tau;
// adjoint: sigma).  LDS: xx (x-halo), yy (y-halo), xy (x and y), xz (x), yz (y);
// register queues: zz, xz, yz.  Pipelined like the TTI passes: the loads of plane z+1 are in
// flight while plane z is computed; LDS is double-buffered.
// 2D (SKIPY): v_y, tau_xy and tau_yz start at zero, have no source and stay exactly zero (their
// only drivers are y derivatives and each other), and so do their adjoint counterparts (v~_y,
// u_y, tau~_xy, tau~_yz, sigma_xy, sigma_yz: no receiver injects into them); the 2D passes neither
// load nor store them, and the fields keep the zeros they were filled with.  tau_yy is still
// formed (it is part of the final state), but in 2D nothing reads it back: its y derivative is
// zero.
// Per-lane byte offsets within a plane for the imaging-condition kernel: the own column (state and
// model layouts, with the +x and +y neighbours of the buoyancy average, clamped at the far faces)
// and the x- and y-halo items, with whether each lies in the window; and the column's absorbing
// factor g_x g_y.
template <int R, int TY, int NT>
struct ElCols {
    using H = Halo<R, TY, NT>;
    uint32_t os, om, omx, omy;
    uint32_t hxo[H::NXH], hyo[H::NYH];
    bool hxok[H::NXH], hyok[H::NYH];
    float gxy;
    template <class Job>
    __device__ __forceinline__ ElCols(const Win &w, int x0, int y0, int gx, int gy, bool own, int tid, bool two_d,
                                      const Job &J)
    {
        const int cx = own ? gx : 0, cy = own ? gy : 0;
        os = 4u * (uint32_t)(cy * w.sx + cx);
        om = 4u * (uint32_t)(cy * w.mx + cx);
        omx = om + (gx + 1 < w.nx ? 4u : 0u);
        omy = om + (gy + 1 < w.ny ? 4u * (uint32_t)w.mx : 0u);
        gxy = gld(J.gx, cx) * gld(J.gy, cy);
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NXI) H::xitem(i, yy, xx);
            const int x = x0 + xx, y = y0 + yy;
            hxok[k] = i < H::NXI && (unsigned)x < (unsigned)w.nx && (unsigned)y < (unsigned)w.ny;
            hxo[k] = hxok[k] ? 4u * (uint32_t)(y * w.sx + x) : 0u;
        }
#pragma unroll
        for (int k = 0; k < H::NYH; ++k) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NYI) H::yitem(i, yy, xx);
            const int x = x0 + xx, y = y0 + yy;
            hyok[k] = !two_d && i < H::NYI && (unsigned)x < (unsigned)w.nx && (unsigned)y < (unsigned)w.ny;
            hyo[k] = hyok[k] ? 4u * (uint32_t)(y * w.sx + x) : 0u;
        }
    }
};

template <int R, int MODE, int BY>
__global__ __launch_bounds__(PROP_TX * BY) __attribute__((amdgpu_waves_per_eu(BY == 8 && R <= 4 ? EL_NARROW_WAVES : 1))) void el_vel(const ElJob *__restrict__ jobs,
                                                       const Tile *__restrict__ tiles, int zc, Weights W, float dt)
{
    constexpr int TY = BY, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool TWO_D = BY == 1;
    constexpr bool SKIPY = TWO_D;
    using P = Plane<R, TY>;
    using H = Halo<R, TY, NT>;
    constexpr int LX = P::LX;
    __shared__ float Lxx[2][P::SIZE], Lyy[2][P::SIZE], Lxy[2][P::SIZE], Lxz[2][P::SIZE], Lyz[2][P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const ElJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < w.nx && gy < w.ny;
    float *const *F = (MODE == EL_FWD) ? J.t : J.aux;
    const float *__restrict__ Fxx = F[0];
    const float *__restrict__ Fyy = F[1];
    const float *__restrict__ Fzz = F[2];
    const float *__restrict__ Fxy = F[3];
    const float *__restrict__ Fxz = F[4];
    const float *__restrict__ Fyz = F[5];
    // 2D one-row tiles address every load by a 64-bit index; 3D tiles by a uniform plane base plus
    // a fixed 32-bit lane offset (fewer registers: 3D measured faster, 2D slower that way).
    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? gld(f, sidx(w, x, y, z)) : 0.f;
    };
    const ElCols<R, TY, NT> cols(w, x0, y0, gx, gy, own, tid, TWO_D, J);
    auto sp = [&](const float *f, int zz) { return (gcchar *)(f + (int64_t)zz * w.sy); };
    auto zok = [&](int zz) { return (unsigned)zz < (unsigned)w.nz; };
    // own column / halo item k of plane z, zero outside the window
    auto ld_own = [&](const float *f, int zz) -> float {
        if constexpr (TWO_D) return ld(f, gx, gy, zz);
        else return own && zok(zz) ? ldo(sp(f, zz), fresh(cols.os)) : 0.f;
    };
    auto ld_hx = [&](const float *f, int k, int zz) -> float {
        if constexpr (TWO_D) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NXI) H::xitem(i, yy, xx);
            return i < H::NXI ? ld(f, x0 + xx, y0 + yy, zz) : 0.f;
        } else {
            return cols.hxok[k] && zok(zz) ? ldo(sp(f, zz), fresh(cols.hxo[k])) : 0.f;
        }
    };
    auto ld_hy = [&](const float *f, int k, int zz) -> float {
        return cols.hyok[k] && zok(zz) ? ldo(sp(f, zz), fresh(cols.hyo[k])) : 0.f;
    };

    float qzz[Q], qxz[Q], qyz[Q];
    float nzz, nxz, nyz, ixx, iyy, ixy;
    float hxx[H::NXH], hxy_x[H::NXH], hxz[H::NXH], hyy[H::NYH], hxy_y[H::NYH], hyz[H::NYH];
#pragma unroll
    for (int s = 1; s < Q; ++s) {
        const int z = z0 - R + s - 1;
        qzz[s] = ld_own(Fzz, z);
        qxz[s] = ld_own(Fxz, z);
        qyz[s] = SKIPY ? 0.f : ld_own(Fyz, z);
    }
    auto fetch = [&](int z) {
        nzz = ld_own(Fzz, z + R);
        nxz = ld_own(Fxz, z + R);
        nyz = SKIPY ? 0.f : ld_own(Fyz, z + R);
        ixx = ld_own(Fxx, z);
        iyy = TWO_D ? 0.f : ld_own(Fyy, z);   // read only by the y derivative
        ixy = SKIPY ? 0.f : ld_own(Fxy, z);
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            hxx[k] = ld_hx(Fxx, k, z);
            hxy_x[k] = SKIPY ? 0.f : ld_hx(Fxy, k, z);
            hxz[k] = ld_hx(Fxz, k, z);
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            hyy[k] = ld_hy(Fyy, k, z);
            hxy_y[k] = ld_hy(Fxy, k, z);
            hyz[k] = ld_hy(Fyz, k, z);
        }
    };
    fetch(z0);
    // 3D: b of plane z, carried from the previous plane's plane-z+1 load (the same address)
    float c_b0 = 0.f;
    if constexpr (!TWO_D) c_b0 = ldo((gcchar *)(J.b + w.moff + (int64_t)z0 * w.my), cols.om);
    int b = 0;
    for (int z = z0; z < z1; ++z) {
        float *lxx = Lxx[b], *lyy = Lyy[b], *lxy = Lxy[b], *lxz = Lxz[b], *lyz = Lyz[b];
#pragma unroll
        for (int s = 0; s < Q - 1; ++s) {
            qzz[s] = qzz[s + 1];
            qxz[s] = qxz[s + 1];
            qyz[s] = qyz[s + 1];
        }
        qzz[Q - 1] = nzz;
        qxz[Q - 1] = nxz;
        qyz[Q - 1] = nyz;
        const int li = P::at(ty, tx);
        lxx[li] = ixx;
        if (!TWO_D) lyy[li] = iyy;
        if (!SKIPY) lxy[li] = ixy;
        lxz[li] = qxz[R];
        if (!TWO_D) lyz[li] = qyz[R];
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NXI) {
                int yy, xx;
                H::xitem(i, yy, xx);
                lxx[P::at(yy, xx)] = hxx[k];
                if (!SKIPY) lxy[P::at(yy, xx)] = hxy_x[k];
                lxz[P::at(yy, xx)] = hxz[k];
            }
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            const int i = tid + k * NT;
            if (i < H::NYI) {
                int yy, xx;
                H::yitem(i, yy, xx);
                lyy[P::at(yy, xx)] = hyy[k];
                lxy[P::at(yy, xx)] = hxy_y[k];
                lyz[P::at(yy, xx)] = hyz[k];
            }
        }
        __syncthreads();
        // per-point values of plane z, then the prefetch of plane z+1
        if constexpr (TWO_D) {
            const int64_t si = sidx(w, own ? gx : 0, own ? gy : 0, z);
            const int64_t mi = midx(w, own ? gx : 0, own ? gy : 0, z);
            const float v0 = gld(J.v[0], si), v1 = SKIPY ? 0.f : gld(J.v[1], si), v2 = gld(J.v[2], si);
            const float b0 = gld(J.b, mi);
            const float bxn = gld(J.b, mi + (gx + 1 < w.nx ? 1 : 0));
            const float byn = SKIPY ? 0.f : gld(J.b, mi + (gy + 1 < w.ny ? w.mx : 0));
            const float bzn = gld(J.b, mi + (z + 1 < w.nz ? w.my : 0));
            const float g = gld(J.gx, own ? gx : 0) * gld(J.gy, own ? gy : 0) * gld(J.gz, z);
            if (z + 1 < z1) fetch(z + 1);
            const float fx = ds_lds<R, true>(lxx, li, 1, W.wx) + (TWO_D ? 0.f : ds_lds<R, false>(lxy, li, LX, W.wy)) +
                             ds_q<R, false>(qxz, W.wz);
            const float fy = SKIPY ? 0.f
                                   : ds_lds<R, false>(lxy, li, 1, W.wx) +
                                         (TWO_D ? 0.f : ds_lds<R, true>(lyy, li, LX, W.wy)) + ds_q<R, false>(qyz, W.wz);
            const float fz = ds_lds<R, false>(lxz, li, 1, W.wx) + (TWO_D ? 0.f : ds_lds<R, false>(lyz, li, LX, W.wy)) +
                             ds_q<R, true>(qzz, W.wz);
            if (own) {
                if (MODE == EL_FWD) {
                    gst(J.vo[0], si, g * (v0 + dt * (0.5f * (b0 + bxn)) * fx));
                    if (!SKIPY) gst(J.vo[1], si, g * (v1 + dt * (0.5f * (b0 + byn)) * fy));
                    gst(J.vo[2], si, g * (v2 + dt * (0.5f * (b0 + bzn)) * fz));
                } else {
                    const float a0 = v0 - dt * fx, a1 = v1 - dt * fy, a2 = v2 - dt * fz;
                    const float c0 = g * a0, c1 = g * a1, c2 = g * a2;
                    gst(J.v[0], si, c0);
                    if (!SKIPY) gst(J.v[1], si, c1);
                    gst(J.v[2], si, c2);
                    gst(J.u[0], si, (0.5f * (b0 + bxn)) * c0);
                    if (!SKIPY) gst(J.u[1], si, (0.5f * (b0 + byn)) * c1);
                    gst(J.u[2], si, (0.5f * (b0 + bzn)) * c2);
                }
            }
        } else {
            auto spw = [&](float *f, int zz) { return (gchar *)(f + (int64_t)zz * w.sy); };
            auto mp = [&](const float *f, int zz) { return (gcchar *)(f + w.moff + (int64_t)zz * w.my); };
            const uint32_t fos = fresh(cols.os), fom = fresh(cols.om);
            const float v0 = ldo(sp(J.v[0], z), fos), v1 = ldo(sp(J.v[1], z), fos);
            const float v2 = ldo(sp(J.v[2], z), fos);
            gcchar *const bz = mp(J.b, z);
            const float b0 = c_b0;
            const float bxn = ldo(bz, fresh(cols.omx));
            const float byn = ldo(bz, fresh(cols.omy));
            const float bzn = ldo(mp(J.b, z + 1 < w.nz ? z + 1 : z), fom);
            c_b0 = bzn;
            const float g = cols.gxy * gld(J.gz, z);
            if (z + 1 < z1) fetch(z + 1);
            const float fx = ds_lds<R, true>(lxx, li, 1, W.wx) + ds_lds<R, false>(lxy, li, LX, W.wy) +
                             ds_q<R, false>(qxz, W.wz);
            const float fy = ds_lds<R, false>(lxy, li, 1, W.wx) + ds_lds<R, true>(lyy, li, LX, W.wy) +
                             ds_q<R, false>(qyz, W.wz);
            const float fz = ds_lds<R, false>(lxz, li, 1, W.wx) + ds_lds<R, false>(lyz, li, LX, W.wy) +
                             ds_q<R, true>(qzz, W.wz);
            if (own) {
                const uint32_t sos = fresh(cols.os);
                if (MODE == EL_FWD) {
                    sto(spw(J.vo[0], z), sos, g * (v0 + dt * (0.5f * (b0 + bxn)) * fx));
                    sto(spw(J.vo[1], z), sos, g * (v1 + dt * (0.5f * (b0 + byn)) * fy));
                    sto(spw(J.vo[2], z), sos, g * (v2 + dt * (0.5f * (b0 + bzn)) * fz));
                } else {
                    const float a0 = v0 - dt * fx, a1 = v1 - dt * fy, a2 = v2 - dt * fz;
                    const float c0 = g * a0, c1 = g * a1, c2 = g * a2;
                    sto(spw(J.v[0], z), sos, c0);
                    sto(spw(J.v[1], z), sos, c1);
                    sto(spw(J.v[2], z), sos, c2);
                    sto(spw(J.u[0], z), sos, (0.5f * (b0 + bxn)) * c0);
                    sto(spw(J.u[1], z), sos, (0.5f * (b0 + byn)) * c1);
                    sto(spw(J.u[2], z), sos, (0.5f * (b0 + bzn)) * c2);
                }
            }
        }
        b ^= 1;
    }
}

// Stress pass.  Fields read: V[0..2] (forward: v; adjoint: u = bbar g v~), each staged in LDS
// with x and y halos and queued in z.
template <int R, int MODE, int BY>
__global__ __launch_bounds__(PROP_TX * BY) __attribute__((amdgpu_waves_per_eu(BY == 8 && R <= 4 ? EL_NARROW_WAVES : 1))) void el_stress(const ElJob *__restrict__ jobs,
                                                          const Tile *__restrict__ tiles, int zc, Weights W, float dt)
{
    constexpr int TY = BY, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool TWO_D = BY == 1;
    constexpr bool SKIPY = TWO_D;   // 2D: v_y, tau_xy, tau_yz (and their adjoints) stay zero
    using P = Plane<R, TY>;
    using H = Halo<R, TY, NT>;
    constexpr int LX = P::LX;
    __shared__ float Lx[2][P::SIZE], Ly[2][P::SIZE], Lz[2][P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const ElJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < w.nx && gy < w.ny;
    float *const *V = (MODE == EL_FWD) ? J.v : J.u;
    const float *__restrict__ Vx = V[0];
    const float *__restrict__ Vy = V[1];
    const float *__restrict__ Vz = V[2];
    // addressing as in the velocity pass: 64-bit indices in 2D, plane base + lane offset in 3D
    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? gld(f, sidx(w, x, y, z)) : 0.f;
    };
    const ElCols<R, TY, NT> cols(w, x0, y0, gx, gy, own, tid, TWO_D, J);
    auto sp = [&](const float *f, int zz) { return (gcchar *)(f + (int64_t)zz * w.sy); };
    auto zok = [&](int zz) { return (unsigned)zz < (unsigned)w.nz; };
    auto ld_own = [&](const float *f, int zz) -> float {
        if constexpr (TWO_D) return ld(f, gx, gy, zz);
        else return own && zok(zz) ? ldo(sp(f, zz), fresh(cols.os)) : 0.f;
    };
    auto ld_hx = [&](const float *f, int k, int zz) -> float {
        if constexpr (TWO_D) {
            const int i = tid + k * NT;
            int yy = 0, xx = 0;
            if (i < H::NXI) H::xitem(i, yy, xx);
            return i < H::NXI ? ld(f, x0 + xx, y0 + yy, zz) : 0.f;
        } else {
            return cols.hxok[k] && zok(zz) ? ldo(sp(f, zz), fresh(cols.hxo[k])) : 0.f;
        }
    };
    auto ld_hy = [&](const float *f, int k, int zz) -> float {
        return cols.hyok[k] && zok(zz) ? ldo(sp(f, zz), fresh(cols.hyo[k])) : 0.f;
    };

    float qx[Q], qy[Q], qz[Q];
    float nx_, ny_, nz_;
    float hx[3][H::NXH], hy[3][H::NYH];
#pragma unroll
    for (int s = 1; s < Q; ++s) {
        const int z = z0 - R + s - 1;
        qx[s] = ld_own(Vx, z);
        qy[s] = SKIPY ? 0.f : ld_own(Vy, z);
        qz[s] = ld_own(Vz, z);
    }
    auto fetch = [&](int z) {
        nx_ = ld_own(Vx, z + R);
        ny_ = SKIPY ? 0.f : ld_own(Vy, z + R);
        nz_ = ld_own(Vz, z + R);
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            hx[0][k] = ld_hx(Vx, k, z);
            hx[1][k] = SKIPY ? 0.f : ld_hx(Vy, k, z);
            hx[2][k] = ld_hx(Vz, k, z);
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            hy[0][k] = ld_hy(Vx, k, z);
            hy[1][k] = ld_hy(Vy, k, z);
            hy[2][k] = ld_hy(Vz, k, z);
        }
    };
    fetch(z0);
    // 3D: mu at the own column, its +x and +y neighbours of plane z, carried from the previous plane's
    // plane-z+1 loads (the same addresses, so the same values)
    float c_mu0 = 0.f, c_mx = 0.f, c_my = 0.f;
    if constexpr (!TWO_D) {
        gcchar *const mz0 = (gcchar *)(J.mu + w.moff + (int64_t)z0 * w.my);
        c_mu0 = ldo(mz0, cols.om);
        c_mx = ldo(mz0, cols.omx);
        c_my = ldo(mz0, cols.omy);
    }
    int b = 0;
    for (int z = z0; z < z1; ++z) {
        float *lx = Lx[b], *ly = Ly[b], *lz = Lz[b];
#pragma unroll
        for (int s = 0; s < Q - 1; ++s) {
            qx[s] = qx[s + 1];
            qy[s] = qy[s + 1];
            qz[s] = qz[s + 1];
        }
        qx[Q - 1] = nx_;
        qy[Q - 1] = ny_;
        qz[Q - 1] = nz_;
        const int li = P::at(ty, tx);
        lx[li] = qx[R];
        if (!SKIPY) ly[li] = qy[R];
        lz[li] = qz[R];
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NXI) {
                int yy, xx;
                H::xitem(i, yy, xx);
                lx[P::at(yy, xx)] = hx[0][k];
                if (!SKIPY) ly[P::at(yy, xx)] = hx[1][k];
                lz[P::at(yy, xx)] = hx[2][k];
            }
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            const int i = tid + k * NT;
            if (i < H::NYI) {
                int yy, xx;
                H::yitem(i, yy, xx);
                lx[P::at(yy, xx)] = hy[0][k];
                ly[P::at(yy, xx)] = hy[1][k];
                lz[P::at(yy, xx)] = hy[2][k];
            }
        }
        __syncthreads();
        if constexpr (TWO_D) {
            const int64_t si = sidx(w, own ? gx : 0, own ? gy : 0, z);
            const int64_t mi = midx(w, own ? gx : 0, own ? gy : 0, z);
            float t[6];
    #pragma unroll
            for (int c = 0; c < 6; ++c) t[c] = SKIPY && (c == 3 || c == 5) ? 0.f : gld(J.t[c], si);
            float lam = 0.f, mu0 = 0.f, mxy = 0.f, mxz = 0.f, myz = 0.f;
            const float g = gld(J.gx, own ? gx : 0) * gld(J.gy, own ? gy : 0) * gld(J.gz, z);
            {   // (the adjoint needs them for sigma of the new tau~)
                const int64_t ox = gx + 1 < w.nx ? 1 : 0, oy = gy + 1 < w.ny ? w.mx : 0, oz = z + 1 < w.nz ? w.my : 0;
                lam = gld(J.lam, mi);
                mu0 = gld(J.mu, mi);
                const float mx_ = gld(J.mu, mi + ox), mz_ = gld(J.mu, mi + oz);
                mxz = 0.25f * (mu0 + mx_ + mz_ + gld(J.mu, mi + ox + oz));
                if (!SKIPY) {
                    const float my_ = gld(J.mu, mi + oy);
                    mxy = 0.25f * (mu0 + mx_ + my_ + gld(J.mu, mi + ox + oy));
                    myz = 0.25f * (mu0 + my_ + mz_ + gld(J.mu, mi + oy + oz));
                }
            }
            if (z + 1 < z1) fetch(z + 1);
            const float exx = ds_lds<R, false>(lx, li, 1, W.wx);
            const float eyy = (TWO_D ? 0.f : ds_lds<R, false>(ly, li, LX, W.wy));
            const float ezz = ds_q<R, false>(qz, W.wz);
            const float gxy =
                SKIPY ? 0.f : (TWO_D ? 0.f : ds_lds<R, true>(lx, li, LX, W.wy)) + ds_lds<R, true>(ly, li, 1, W.wx);
            const float gxz = ds_q<R, true>(qx, W.wz) + ds_lds<R, true>(lz, li, 1, W.wx);
            const float gyz = SKIPY ? 0.f : ds_q<R, true>(qy, W.wz) + (TWO_D ? 0.f : ds_lds<R, true>(lz, li, LX, W.wy));
            if (own) {
                if (MODE == EL_FWD) {
                    const float lt = lam * (exx + eyy + ezz), m2 = 2.f * mu0;
                    gst(J.t[0], si, g * (t[0] + dt * (lt + m2 * exx)));
                    gst(J.t[1], si, g * (t[1] + dt * (lt + m2 * eyy)));
                    gst(J.t[2], si, g * (t[2] + dt * (lt + m2 * ezz)));
                    if (!SKIPY) gst(J.t[3], si, g * (t[3] + dt * mxy * gxy));
                    gst(J.t[4], si, g * (t[4] + dt * mxz * gxz));
                    if (!SKIPY) gst(J.t[5], si, g * (t[5] + dt * myz * gyz));
                } else {
                    float tg[6], tn[6];
    #pragma unroll
                    for (int c = 0; c < 6; ++c) tg[c] = g * t[c];
                    tn[0] = tg[0] - dt * exx;
                    tn[1] = tg[1] - dt * eyy;
                    tn[2] = tg[2] - dt * ezz;
                    tn[3] = tg[3] - dt * gxy;
                    tn[4] = tg[4] - dt * gxz;
                    tn[5] = tg[5] - dt * gyz;
    #pragma unroll
                    for (int c = 0; c < 6; ++c)
                        if (!(SKIPY && (c == 3 || c == 5))) gst(J.t[c], si, tn[c]);
                    // sigma = C (g tau~) of the new tau~, which the velocity pass of the next (earlier)
                    // step reads; where that step injects receiver residuals into tau~, el_remix
                    // recomputes the diagonal components after the injection
                    float sg[6];
    #pragma unroll
                    for (int c = 0; c < 6; ++c) sg[c] = g * tn[c];
                    const float lt = lam * (sg[0] + sg[1] + sg[2]), m2 = 2.f * mu0;
                    gst(J.aux[0], si, lt + m2 * sg[0]);
                    gst(J.aux[1], si, lt + m2 * sg[1]);
                    gst(J.aux[2], si, lt + m2 * sg[2]);
                    if (!SKIPY) gst(J.aux[3], si, mxy * sg[3]);
                    gst(J.aux[4], si, mxz * sg[4]);
                    if (!SKIPY) gst(J.aux[5], si, myz * sg[5]);
                }
            }
        } else {
            auto spw = [&](float *f, int zz) { return (gchar *)(f + (int64_t)zz * w.sy); };
            auto mp = [&](const float *f, int zz) { return (gcchar *)(f + w.moff + (int64_t)zz * w.my); };
            const uint32_t fos = fresh(cols.os), fom = fresh(cols.om);
            float t[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) t[c] = ldo(sp(J.t[c], z), fos);
            const float g = cols.gxy * gld(J.gz, z);
            gcchar *const m0 = mp(J.mu, z), *const m1 = mp(J.mu, z + 1 < w.nz ? z + 1 : z);
            const uint32_t omx = fresh(cols.omx), omy = fresh(cols.omy), omxy = omx + omy - fom;
            const float lam = ldo(mp(J.lam, z), fom);
            const float mu0 = c_mu0, mx_ = c_mx, my_ = c_my;
            const float mz_ = ldo(m1, fom), mxz1 = ldo(m1, omx), myz1 = ldo(m1, omy);
            c_mu0 = mz_;
            c_mx = mxz1;
            c_my = myz1;
            const float mxz = 0.25f * (mu0 + mx_ + mz_ + mxz1);
            const float mxy = 0.25f * (mu0 + mx_ + my_ + ldo(m0, omxy));
            const float myz = 0.25f * (mu0 + my_ + mz_ + myz1);
            if (z + 1 < z1) fetch(z + 1);
            const float exx = ds_lds<R, false>(lx, li, 1, W.wx);
            const float eyy = ds_lds<R, false>(ly, li, LX, W.wy);
            const float ezz = ds_q<R, false>(qz, W.wz);
            const float gxy = ds_lds<R, true>(lx, li, LX, W.wy) + ds_lds<R, true>(ly, li, 1, W.wx);
            const float gxz = ds_q<R, true>(qx, W.wz) + ds_lds<R, true>(lz, li, 1, W.wx);
            const float gyz = ds_q<R, true>(qy, W.wz) + ds_lds<R, true>(lz, li, LX, W.wy);
            if (own) {
                const uint32_t sos = fresh(cols.os);
                if (MODE == EL_FWD) {
                    const float lt = lam * (exx + eyy + ezz), m2 = 2.f * mu0;
                    sto(spw(J.t[0], z), sos, g * (t[0] + dt * (lt + m2 * exx)));
                    sto(spw(J.t[1], z), sos, g * (t[1] + dt * (lt + m2 * eyy)));
                    sto(spw(J.t[2], z), sos, g * (t[2] + dt * (lt + m2 * ezz)));
                    sto(spw(J.t[3], z), sos, g * (t[3] + dt * mxy * gxy));
                    sto(spw(J.t[4], z), sos, g * (t[4] + dt * mxz * gxz));
                    sto(spw(J.t[5], z), sos, g * (t[5] + dt * myz * gyz));
                } else {
                    float tg[6], tn[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) tg[c] = g * t[c];
                    tn[0] = tg[0] - dt * exx;
                    tn[1] = tg[1] - dt * eyy;
                    tn[2] = tg[2] - dt * ezz;
                    tn[3] = tg[3] - dt * gxy;
                    tn[4] = tg[4] - dt * gxz;
                    tn[5] = tg[5] - dt * gyz;
#pragma unroll
                    for (int c = 0; c < 6; ++c) sto(spw(J.t[c], z), sos, tn[c]);
                    float sg[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) sg[c] = g * tn[c];
                    const float lt = lam * (sg[0] + sg[1] + sg[2]), m2 = 2.f * mu0;
                    sto(spw(J.aux[0], z), sos, lt + m2 * sg[0]);
                    sto(spw(J.aux[1], z), sos, lt + m2 * sg[1]);
                    sto(spw(J.aux[2], z), sos, lt + m2 * sg[2]);
                    sto(spw(J.aux[3], z), sos, mxy * sg[3]);
                    sto(spw(J.aux[4], z), sos, mxz * sg[4]);
                    sto(spw(J.aux[5], z), sos, myz * sg[5]);
                }
            }
        }
        b ^= 1;
    }
}

// Imaging condition of the elastic gradient for one adjoint step (after the transposed velocity
// update, before the transposed stress update).  The strains of the stored forward velocities
// v^{n+1} are formed exactly as in the forward stress pass (LDS planes with x and y halos, z
// queues); then, per storage point,
//   acc_lambda += dt g tr(tau~) tr(E v),  acc_mu += 2 dt g sum_a tau~_aa (E v)_aa,
//   acc_s      += dt g tau~_s (E v)_s for the shear components s (at their staggered positions),
//   acc_b,c    += v~_c dt (D_tau tau^n)_c = v~_c (v^{n+1}_c - g v^n_c) / (g bbar_c)
// (the velocity update v^{n+1} = g (v^n + dt bbar D_tau tau^n) gives the force from two stored
// velocity levels).
template <int R, int BY>
__global__ __launch_bounds__(PROP_TX * BY) void el_grad_ic(const ElGradJob *__restrict__ jobs,
                                                           const Tile *__restrict__ tiles, int zc, Weights W, float dt)
{
    constexpr int TY = BY, Q = 2 * R + 1, NT = PROP_TX * BY;
    constexpr bool TWO_D = BY == 1;
    using P = Plane<R, TY>;
    using H = Halo<R, TY, NT>;
    constexpr int LX = P::LX;
    __shared__ float Lx[2][P::SIZE], Ly[2][P::SIZE], Lz[2][P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const ElGradJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < w.nx && gy < w.ny;
    const float *__restrict__ Vx = J.vn1[0];
    const float *__restrict__ Vy = J.vn1[1];
    const float *__restrict__ Vz = J.vn1[2];
    // addressing: uniform plane bases and per-lane byte offsets within a plane (own column, halo items)
    auto sp = [&](const float *f, int zz) { return (gcchar *)(f + (int64_t)zz * w.sy); };
    auto spw = [&](float *f, int zz) { return (gchar *)(f + (int64_t)zz * w.sy); };
    auto mp = [&](const float *f, int zz) { return (gcchar *)(f + w.moff + (int64_t)zz * w.my); };
    auto zok = [&](int zz) { return (unsigned)zz < (unsigned)w.nz; };
    const ElCols<R, TY, NT> cols(w, x0, y0, gx, gy, own, tid, TWO_D, J);
    const uint32_t os = cols.os, om = cols.om, omx = cols.omx, omy = cols.omy;

    float qx[Q], qy[Q], qz[Q];
    float nx_, ny_, nz_;
    float hx[3][H::NXH], hy[3][H::NYH];
#pragma unroll
    for (int s = 1; s < Q; ++s) {
        const int z = z0 - R + s - 1;
        const bool v = own && zok(z);
        qx[s] = v ? ldo(sp(Vx, z), os) : 0.f;
        qy[s] = v ? ldo(sp(Vy, z), os) : 0.f;
        qz[s] = v ? ldo(sp(Vz, z), os) : 0.f;
    }
    auto fetch = [&](int z) {
        const bool va = own && zok(z + R), vz = zok(z);
        const uint32_t fos = fresh(os);
        nx_ = va ? ldo(sp(Vx, z + R), fos) : 0.f;
        ny_ = va ? ldo(sp(Vy, z + R), fos) : 0.f;
        nz_ = va ? ldo(sp(Vz, z + R), fos) : 0.f;
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const bool v = vz && cols.hxok[k];
            const uint32_t o = fresh(cols.hxo[k]);
            hx[0][k] = v ? ldo(sp(Vx, z), o) : 0.f;
            hx[1][k] = v ? ldo(sp(Vy, z), o) : 0.f;
            hx[2][k] = v ? ldo(sp(Vz, z), o) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            const bool v = vz && cols.hyok[k];
            const uint32_t o = fresh(cols.hyo[k]);
            hy[0][k] = v ? ldo(sp(Vx, z), o) : 0.f;
            hy[1][k] = v ? ldo(sp(Vy, z), o) : 0.f;
            hy[2][k] = v ? ldo(sp(Vz, z), o) : 0.f;
        }
    };
    fetch(z0);
    // per-point operands, loaded a plane ahead: tau~, v~, v^n, buoyancy at the node and its +x, +y, +z
    // neighbours (clamped at the window's far faces)
    float pt_t[6], pt_vt[3], pt_v0[3], pt_b[4];
    // (after the first plane, b at the node is the previous plane's +z neighbour, already loaded: the
    // same address, so the same value)
    auto load_pt = [&](int z, bool carry) {
        const uint32_t fos = fresh(os), fom = fresh(om);
#pragma unroll
        for (int c = 0; c < 6; ++c) pt_t[c] = ldo(sp(J.tt[c], z), fos);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pt_vt[c] = ldo(sp(J.vt[c], z), fos);
            pt_v0[c] = ldo(sp(J.vn0[c], z), fos);
        }
        gcchar *const bz = mp(J.b, z);
        pt_b[0] = carry ? pt_b[3] : ldo(bz, fom);
        pt_b[1] = ldo(bz, fresh(omx));
        pt_b[2] = ldo(bz, fresh(omy));
        pt_b[3] = ldo(mp(J.b, z + 1 < w.nz ? z + 1 : z), fom);
    };
    load_pt(z0, false);
    int b = 0;
    for (int z = z0; z < z1; ++z) {
        float *lx = Lx[b], *ly = Ly[b], *lz = Lz[b];
#pragma unroll
        for (int s = 0; s < Q - 1; ++s) {
            qx[s] = qx[s + 1];
            qy[s] = qy[s + 1];
            qz[s] = qz[s + 1];
        }
        qx[Q - 1] = nx_;
        qy[Q - 1] = ny_;
        qz[Q - 1] = nz_;
        const int li = P::at(ty, tx);
        lx[li] = qx[R];
        ly[li] = qy[R];
        lz[li] = qz[R];
#pragma unroll
        for (int k = 0; k < H::NXH; ++k) {
            const int i = tid + k * NT;
            if (i < H::NXI) {
                int yy, xx;
                H::xitem(i, yy, xx);
                lx[P::at(yy, xx)] = hx[0][k];
                ly[P::at(yy, xx)] = hx[1][k];
                lz[P::at(yy, xx)] = hx[2][k];
            }
        }
#pragma unroll
        for (int k = 0; k < (TWO_D ? 0 : H::NYH); ++k) {
            const int i = tid + k * NT;
            if (i < H::NYI) {
                int yy, xx;
                H::yitem(i, yy, xx);
                lx[P::at(yy, xx)] = hy[0][k];
                ly[P::at(yy, xx)] = hy[1][k];
                lz[P::at(yy, xx)] = hy[2][k];
            }
        }
        __syncthreads();
        float t[6], vt[3], v0[3];
#pragma unroll
        for (int c = 0; c < 6; ++c) t[c] = pt_t[c];
#pragma unroll
        for (int c = 0; c < 3; ++c) vt[c] = pt_vt[c], v0[c] = pt_v0[c];
        const float b0 = pt_b[0], bxn = pt_b[1], byn = pt_b[2], bzn = pt_b[3];
        const float g = cols.gxy * gld(J.gz, z);
        const float v1[3] = {qx[R], qy[R], qz[R]};
        if (z + 1 < z1) {
            load_pt(z + 1, true);
            fetch(z + 1);
        }
        const float exx = ds_lds<R, false>(lx, li, 1, W.wx);
        const float eyy = (TWO_D ? 0.f : ds_lds<R, false>(ly, li, LX, W.wy));
        const float ezz = ds_q<R, false>(qz, W.wz);
        const float gxy = (TWO_D ? 0.f : ds_lds<R, true>(lx, li, LX, W.wy)) + ds_lds<R, true>(ly, li, 1, W.wx);
        const float gxz = ds_q<R, true>(qx, W.wz) + ds_lds<R, true>(lz, li, 1, W.wx);
        const float gyz = ds_q<R, true>(qy, W.wz) + (TWO_D ? 0.f : ds_lds<R, true>(lz, li, LX, W.wy));
        if (own) {
            const float gdt = g * dt;
            const float bb[3] = {0.5f * (b0 + bxn), 0.5f * (b0 + byn), 0.5f * (b0 + bzn)};
            const uint32_t aos = fresh(os);
            auto acc_add = [&](int c, float d) { sto(spw(J.acc[c], z), aos, ldo(sp(J.acc[c], z), aos) + d); };
            acc_add(0, gdt * (t[0] + t[1] + t[2]) * (exx + eyy + ezz));
            acc_add(1, 2.f * gdt * (t[0] * exx + t[1] * eyy + t[2] * ezz));
            acc_add(2, gdt * t[3] * gxy);
            acc_add(3, gdt * t[4] * gxz);
            acc_add(4, gdt * t[5] * gyz);
#pragma unroll
            for (int c = 0; c < 3; ++c) acc_add(5 + c, vt[c] * (v1[c] - g * v0[c]) / (g * bb[c]));
        }
        b ^= 1;
    }
}

// Transpose of the half-node averages, gathered at each node, and the chain rule to (vp, vs, rho):
// a position p enters the average at nodes p and min(p + 1, n - 1) along each averaged axis, so a
// node i collects from p = i - 1 (weight 1) and p = i (weight 1 + [i = n - 1]), times 1/2 per axis.
__device__ __forceinline__ float spread_w(int p, int i, int n) { return (p == i ? 1.f : 0.f) + (min(p + 1, n - 1) == i ? 1.f : 0.f); }

__global__ void el_grad_finish(const ElGradJob *__restrict__ jobs, int ndim, int nvac, int nimg,
                               const float *__restrict__ vp, const float *__restrict__ vs,
                               const float *__restrict__ rho, float *__restrict__ out)
{
    const ElGradJob &J = jobs[0];
    const Win w = J.w;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= w.nx) return;
    const int n[3] = {w.nx, w.ny, w.nz};
    const int c3[3] = {x, y, z};
    auto at = [&](const float *f, int px, int py, int pz) { return gld(f, sidx(w, px, py, pz)); };
    const int64_t si = sidx(w, x, y, z);
    float gl = gld(J.acc[0], si);
    float gm = gld(J.acc[1], si);
    // shear positions: (x, y) for xy, (x, z) for xz, (y, z) for yz
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int k = 0; k < 3; ++k) {
        const int a1 = pairs[k][0], a2 = pairs[k][1];
        if (ndim == 2 && (a1 == 1 || a2 == 1)) continue;
        for (int d1 = -1; d1 <= 0; ++d1) {
            const int p1 = c3[a1] + d1;
            if (p1 < 0) continue;
            for (int d2 = -1; d2 <= 0; ++d2) {
                const int p2 = c3[a2] + d2;
                if (p2 < 0) continue;
                int p[3] = {x, y, z};
                p[a1] = p1;
                p[a2] = p2;
                const float wgt = 0.25f * spread_w(p1, c3[a1], n[a1]) * spread_w(p2, c3[a2], n[a2]);
                gm += wgt * at(J.acc[2 + k], p[0], p[1], p[2]);
            }
        }
    }
    // buoyancy sensitivity of node (x, y, zz): the shares of the two-node means it enters
    auto gb_at = [&](int zz) {
        const int cz[3] = {x, y, zz};
        float acc = 0.f;
        for (int a = 0; a < 3; ++a) {
            if (ndim == 2 && a == 1) continue;
            for (int d = -1; d <= 0; ++d) {
                const int pa = cz[a] + d;
                if (pa < 0) continue;
                int p[3] = {x, y, zz};
                p[a] = pa;
                acc += 0.5f * spread_w(pa, cz[a], n[a]) * at(J.acc[5 + a], p[0], p[1], p[2]);
            }
        }
        return acc;
    };
    float gb = gb_at(z);
    if (z < nvac) {   // vacuum: lambda and mu are fixed at zero; only the buoyancy depends on rho
        gl = 0.f;
        gm = 0.f;
    }
    if (nimg > 0) {   // image rows above the surface row nimg copy the buoyancy of the rows below
        if (z < nimg) gb = 0.f;
        else if (z > nimg && z <= 2 * nimg) gb += gb_at(2 * nimg - z);
    }
    const int64_t mi = midx(w, x, y, z);
    const float a = gld(vp, mi), s = gld(vs, mi), r = gld(rho, mi);
    const int64_t o = ((int64_t)z * w.ny + y) * w.nx + x, np_ = (int64_t)w.nx * w.ny * w.nz;
    gst(out, o, 2.f * r * a * gl);
    gst(out, np_ + o, 2.f * r * s * (gm - 2.f * gl));
    gst(out, 2 * np_ + o, (a * a - 2.f * s * s) * gl + s * s * gm - gb / (r * r));
}

template <int R, int BY>
void vel_launch(int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt,
                hipStream_t st)
{
    dim3 blk(PROP_TX, BY), grd(ntiles);
    if (mode == EL_FWD) hipLaunchKernelGGL((el_vel<R, EL_FWD, BY>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
    else                hipLaunchKernelGGL((el_vel<R, EL_ADJ, BY>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
}

template <int R>
void vel_dispatch(int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W,
                  float dt, hipStream_t st)
{
    if (by == 1)      vel_launch<R, 1>(mode, jobs, tiles, ntiles, zc, W, dt, st);
    else if (by == 8) vel_launch<R, 8>(mode, jobs, tiles, ntiles, zc, W, dt, st);
    else              vel_launch<R, EBY>(mode, jobs, tiles, ntiles, zc, W, dt, st);
}

template <int R, int BY>
void stress_launch(int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt,
                   hipStream_t st)
{
    dim3 blk(PROP_TX, BY), grd(ntiles);
    if (mode == EL_FWD) hipLaunchKernelGGL((el_stress<R, EL_FWD, BY>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
    else                hipLaunchKernelGGL((el_stress<R, EL_ADJ, BY>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
}

template <int R>
void stress_dispatch(int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W,
                     float dt, hipStream_t st)
{
    if (by == 1)      stress_launch<R, 1>(mode, jobs, tiles, ntiles, zc, W, dt, st);
    else if (by == 8) stress_launch<R, 8>(mode, jobs, tiles, ntiles, zc, W, dt, st);
    else              stress_launch<R, EBY>(mode, jobs, tiles, ntiles, zc, W, dt, st);
}

}  // namespace

int el_tile_rows(int R, int ndim)
{
    (void)R;
    return ndim == 2 ? 1 : EBY;
}

#define EL_SWITCH(FN, ...)                                  \
    switch (R) {                                            \
    case 1: FN<1>(__VA_ARGS__); break;                      \
    case 2: FN<2>(__VA_ARGS__); break;                      \
    case 3: FN<3>(__VA_ARGS__); break;                      \
    case 4: FN<4>(__VA_ARGS__); break;                      \
    case 5: FN<5>(__VA_ARGS__); break;                      \
    case 6: FN<6>(__VA_ARGS__); break;                      \
    case 7: FN<7>(__VA_ARGS__); break;                      \
    default: FN<8>(__VA_ARGS__); break;                     \
    }

void launch_el_vel(int R, int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc,
                   const Weights &W, float dt, hipStream_t st)
{
    EL_SWITCH(vel_dispatch, by, mode, jobs, tiles, ntiles, zc, W, dt, st)
}

void launch_el_stress(int R, int by, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc,
                      const Weights &W, float dt, hipStream_t st)
{
    EL_SWITCH(stress_dispatch, by, mode, jobs, tiles, ntiles, zc, W, dt, st)
}


template <int R>
void gic_dispatch(int by, const ElGradJob *job, const Tile *tiles, int ntiles, int zc, const Weights &W, float dt,
                  hipStream_t st)
{
    if (by == 1) hipLaunchKernelGGL((el_grad_ic<R, 1>), dim3(ntiles), dim3(PROP_TX, 1), 0, st, job, tiles, zc, W, dt);
    else if (by == 8)
        hipLaunchKernelGGL((el_grad_ic<R, 8>), dim3(ntiles), dim3(PROP_TX, 8), 0, st, job, tiles, zc, W, dt);
    else hipLaunchKernelGGL((el_grad_ic<R, EBY>), dim3(ntiles), dim3(PROP_TX, EBY), 0, st, job, tiles, zc, W, dt);
}

void launch_el_grad_ic(int R, int by, const ElGradJob *job, const Tile *tiles, int ntiles, int zc, const Weights &W,
                       float dt, hipStream_t st)
{
    EL_SWITCH(gic_dispatch, by, job, tiles, ntiles, zc, W, dt, st)
}

void launch_el_grad_finish(const ElGradJob *job, const Win &w, int ndim, int nvac, int nimg, const float *vp,
                           const float *vs, const float *rho, float *out, hipStream_t st)
{
    dim3 blk(256), grd((w.nx + 255) / 256, w.ny, w.nz);
    hipLaunchKernelGGL(el_grad_finish, grd, blk, 0, st, job, ndim, nvac, nimg, vp, vs, rho, out);
}
