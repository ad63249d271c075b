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
//   v~ += dt E^T sigma, tau~ <- g tau~;   then   tau~ += dt D_tau^T u, v~ <- g v~,
// where E^T = -(the D_tau pattern) and D_tau^T = -(the E pattern), so the adjoint reuses the two
// forward stencil kernels on the pointwise-weighted fields with a minus sign.
#include "jobs.h"

namespace {

template <int R>
constexpr int el_ny()
{
    return R <= 4 ? 2 : 1;
}

// Velocity pass.  Fields read: F[0..5] = (xx, yy, zz, xy, xz, yz) stresses (forward: tau;
// adjoint: sigma).  LDS: xx (x-halo), yy (y-halo), xy (x and y), xz (x), yz (y);
// queues: zz, xz, yz.
template <int R, int NY, int MODE>
__global__ __launch_bounds__(PROP_NT) void el_vel(const ElJob *__restrict__ jobs, const Tile *__restrict__ tiles,
                                                 int zc, Weights W, float dt)
{
    constexpr int TY = PROP_BY * NY, Q = 2 * R + 1;
    using P = Plane<R, TY>;
    constexpr int LX = P::LX;
    __shared__ float Lxx[P::SIZE], Lyy[P::SIZE], Lxy[P::SIZE], Lxz[P::SIZE], Lyz[P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const ElJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    float *const *F = (MODE == EL_FWD) ? J.t : J.aux;
    const float *__restrict__ Fxx = F[0];
    const float *__restrict__ Fyy = F[1];
    const float *__restrict__ Fzz = F[2];
    const float *__restrict__ Fxy = F[3];
    const float *__restrict__ Fxz = F[4];
    const float *__restrict__ Fyz = F[5];

    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? f[sidx(w, x, y, z)] : 0.f;
    };

    float qzz[NY][Q], qxz[NY][Q], qyz[NY][Q];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) {
            const int y = y0 + ty * NY + r, z = z0 - R + s - 1;
            qzz[r][s] = ld(Fzz, gx, y, z);
            qxz[r][s] = ld(Fxz, gx, y, z);
            qyz[r][s] = ld(Fyz, gx, y, z);
        }

    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qzz[r][s] = qzz[r][s + 1];
                qxz[r][s] = qxz[r][s + 1];
                qyz[r][s] = qyz[r][s + 1];
            }
            qzz[r][Q - 1] = ld(Fzz, gx, y, z + R);
            qxz[r][Q - 1] = ld(Fxz, gx, y, z + R);
            qyz[r][Q - 1] = ld(Fyz, gx, y, z + R);
            const int li = P::at(ty * NY + r, tx);
            Lxx[li] = ld(Fxx, gx, y, z);
            Lyy[li] = ld(Fyy, gx, y, z);
            Lxy[li] = ld(Fxy, gx, y, z);
            Lxz[li] = qxz[r][R];
            Lyz[li] = qyz[r][R];
        }
        for (int i = tid; i < 2 * R * TY; i += PROP_NT) {
            int row = i / (2 * R), c = i - row * (2 * R);
            int xx = c < R ? c - R : PROP_TX + c - R;
            const int li = P::at(row, xx);
            Lxx[li] = ld(Fxx, x0 + xx, y0 + row, z);
            Lxy[li] = ld(Fxy, x0 + xx, y0 + row, z);
            Lxz[li] = ld(Fxz, x0 + xx, y0 + row, z);
        }
        for (int i = tid; i < 2 * R * PROP_TX; i += PROP_NT) {
            int rr = i / PROP_TX, xx = i - rr * PROP_TX;
            int yy = rr < R ? rr - R : TY + rr - R;
            const int li = P::at(yy, xx);
            Lyy[li] = ld(Fyy, x0 + xx, y0 + yy, z);
            Lxy[li] = ld(Fxy, x0 + xx, y0 + yy, z);
            Lyz[li] = ld(Fyz, x0 + xx, y0 + yy, z);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            if (gx < w.nx && y < w.ny) {
                const int li = P::at(ty * NY + r, tx);
                const float fx = ds_lds<R, true>(Lxx, li, 1, W.wx) + ds_lds<R, false>(Lxy, li, LX, W.wy) +
                                 ds_q<R, false>(qxz[r], W.wz);
                const float fy = ds_lds<R, false>(Lxy, li, 1, W.wx) + ds_lds<R, true>(Lyy, li, LX, W.wy) +
                                 ds_q<R, false>(qyz[r], W.wz);
                const float fz = ds_lds<R, false>(Lxz, li, 1, W.wx) + ds_lds<R, false>(Lyz, li, LX, W.wy) +
                                 ds_q<R, true>(qzz[r], W.wz);
                const int64_t si = sidx(w, gx, y, z);
                if (MODE == EL_FWD) {
                    const float g = J.gx[gx] * J.gy[y] * J.gz[z];
                    const int64_t mi = midx(w, gx, y, z);
                    const float b0 = J.b[mi];
                    const float bx = 0.5f * (b0 + J.b[mi + (gx + 1 < w.nx ? 1 : 0)]);
                    const float by = 0.5f * (b0 + J.b[mi + (y + 1 < w.ny ? w.mx : 0)]);
                    const float bz = 0.5f * (b0 + J.b[mi + (z + 1 < w.nz ? w.my : 0)]);
                    J.v[0][si] = g * (J.v[0][si] + dt * bx * fx);
                    J.v[1][si] = g * (J.v[1][si] + dt * by * fy);
                    J.v[2][si] = g * (J.v[2][si] + dt * bz * fz);
                } else {
                    J.v[0][si] -= dt * fx;
                    J.v[1][si] -= dt * fy;
                    J.v[2][si] -= dt * fz;
                }
            }
        }
        __syncthreads();
    }
}

// Stress pass.  Fields read: V[0..2] (forward: v; adjoint: u = bbar g v~), each staged in LDS
// with x and y halos and queued in z.
template <int R, int NY, int MODE>
__global__ __launch_bounds__(PROP_NT) void el_stress(const ElJob *__restrict__ jobs, const Tile *__restrict__ tiles,
                                                    int zc, Weights W, float dt)
{
    constexpr int TY = PROP_BY * NY, Q = 2 * R + 1;
    using P = Plane<R, TY>;
    constexpr int LX = P::LX;
    __shared__ float Lx[P::SIZE], Ly[P::SIZE], Lz[P::SIZE];

    const Tile tl = tiles[blockIdx.x];
    const ElJob &J = jobs[tl.job];
    const Win w = J.w;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * PROP_TX + tx;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = min(z0 + zc, w.nz);
    const int gx = x0 + tx;
    float *const *V = (MODE == EL_FWD) ? J.v : J.aux;
    const float *__restrict__ Vx = V[0];
    const float *__restrict__ Vy = V[1];
    const float *__restrict__ Vz = V[2];

    auto ld = [&](const float *f, int x, int y, int z) -> float {
        return in_win(w, x, y, z) ? f[sidx(w, x, y, z)] : 0.f;
    };

    float qx[NY][Q], qy[NY][Q], qz[NY][Q];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int s = 1; s < Q; ++s) {
            const int y = y0 + ty * NY + r, z = z0 - R + s - 1;
            qx[r][s] = ld(Vx, gx, y, z);
            qy[r][s] = ld(Vy, gx, y, z);
            qz[r][s] = ld(Vz, gx, y, z);
        }

    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
#pragma unroll
            for (int s = 0; s < Q - 1; ++s) {
                qx[r][s] = qx[r][s + 1];
                qy[r][s] = qy[r][s + 1];
                qz[r][s] = qz[r][s + 1];
            }
            qx[r][Q - 1] = ld(Vx, gx, y, z + R);
            qy[r][Q - 1] = ld(Vy, gx, y, z + R);
            qz[r][Q - 1] = ld(Vz, gx, y, z + R);
            const int li = P::at(ty * NY + r, tx);
            Lx[li] = qx[r][R];
            Ly[li] = qy[r][R];
            Lz[li] = qz[r][R];
        }
        for (int i = tid; i < 2 * R * TY; i += PROP_NT) {
            int row = i / (2 * R), c = i - row * (2 * R);
            int xx = c < R ? c - R : PROP_TX + c - R;
            const int li = P::at(row, xx);
            Lx[li] = ld(Vx, x0 + xx, y0 + row, z);
            Ly[li] = ld(Vy, x0 + xx, y0 + row, z);
            Lz[li] = ld(Vz, x0 + xx, y0 + row, z);
        }
        for (int i = tid; i < 2 * R * PROP_TX; i += PROP_NT) {
            int rr = i / PROP_TX, xx = i - rr * PROP_TX;
            int yy = rr < R ? rr - R : TY + rr - R;
            const int li = P::at(yy, xx);
            Lx[li] = ld(Vx, x0 + xx, y0 + yy, z);
            Ly[li] = ld(Vy, x0 + xx, y0 + yy, z);
            Lz[li] = ld(Vz, x0 + xx, y0 + yy, z);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NY; ++r) {
            const int y = y0 + ty * NY + r;
            if (gx < w.nx && y < w.ny) {
                const int li = P::at(ty * NY + r, tx);
                const float exx = ds_lds<R, false>(Lx, li, 1, W.wx);
                const float eyy = ds_lds<R, false>(Ly, li, LX, W.wy);
                const float ezz = ds_q<R, false>(qz[r], W.wz);
                const float gxy = ds_lds<R, true>(Lx, li, LX, W.wy) + ds_lds<R, true>(Ly, li, 1, W.wx);
                const float gxz = ds_q<R, true>(qx[r], W.wz) + ds_lds<R, true>(Lz, li, 1, W.wx);
                const float gyz = ds_q<R, true>(qy[r], W.wz) + ds_lds<R, true>(Lz, li, LX, W.wy);
                const int64_t si = sidx(w, gx, y, z);
                if (MODE == EL_FWD) {
                    const float g = J.gx[gx] * J.gy[y] * J.gz[z];
                    const int64_t mi = midx(w, gx, y, z);
                    const int64_t ox = gx + 1 < w.nx ? 1 : 0, oy = y + 1 < w.ny ? w.mx : 0,
                                  oz = z + 1 < w.nz ? w.my : 0;
                    const float lam = J.lam[mi], mu0 = J.mu[mi];
                    const float mxy = 0.25f * (mu0 + J.mu[mi + ox] + J.mu[mi + oy] + J.mu[mi + ox + oy]);
                    const float mxz = 0.25f * (mu0 + J.mu[mi + ox] + J.mu[mi + oz] + J.mu[mi + ox + oz]);
                    const float myz = 0.25f * (mu0 + J.mu[mi + oy] + J.mu[mi + oz] + J.mu[mi + oy + oz]);
                    const float lt = lam * (exx + eyy + ezz), m2 = 2.f * mu0;
                    J.t[0][si] = g * (J.t[0][si] + dt * (lt + m2 * exx));
                    J.t[1][si] = g * (J.t[1][si] + dt * (lt + m2 * eyy));
                    J.t[2][si] = g * (J.t[2][si] + dt * (lt + m2 * ezz));
                    J.t[3][si] = g * (J.t[3][si] + dt * mxy * gxy);
                    J.t[4][si] = g * (J.t[4][si] + dt * mxz * gxz);
                    J.t[5][si] = g * (J.t[5][si] + dt * myz * gyz);
                } else {
                    J.t[0][si] -= dt * exx;
                    J.t[1][si] -= dt * eyy;
                    J.t[2][si] -= dt * ezz;
                    J.t[3][si] -= dt * gxy;
                    J.t[4][si] -= dt * gxz;
                    J.t[5][si] -= dt * gyz;
                }
            }
        }
        __syncthreads();
    }
}

// sigma = C (g tau~) into aux[0..5]; tau~ <- g tau~.
__global__ void el_mix_stress(const ElJob *__restrict__ jobs)
{
    const ElJob &J = jobs[0];
    const Win w = J.w;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= w.nx) return;
    const int64_t si = sidx(w, x, y, z), mi = midx(w, x, y, z);
    const float g = J.gx[x] * J.gy[y] * J.gz[z];
    float t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        t[c] = g * J.t[c][si];
        J.t[c][si] = t[c];
    }
    const int64_t ox = x + 1 < w.nx ? 1 : 0, oy = y + 1 < w.ny ? w.mx : 0, oz = z + 1 < w.nz ? w.my : 0;
    const float lam = J.lam[mi], mu0 = J.mu[mi];
    const float lt = lam * (t[0] + t[1] + t[2]), m2 = 2.f * mu0;
    J.aux[0][si] = lt + m2 * t[0];
    J.aux[1][si] = lt + m2 * t[1];
    J.aux[2][si] = lt + m2 * t[2];
    J.aux[3][si] = 0.25f * (mu0 + J.mu[mi + ox] + J.mu[mi + oy] + J.mu[mi + ox + oy]) * t[3];
    J.aux[4][si] = 0.25f * (mu0 + J.mu[mi + ox] + J.mu[mi + oz] + J.mu[mi + ox + oz]) * t[4];
    J.aux[5][si] = 0.25f * (mu0 + J.mu[mi + oy] + J.mu[mi + oz] + J.mu[mi + oy + oz]) * t[5];
}

// u = bbar (g v~) into aux[0..2]; v~ <- g v~.
__global__ void el_mix_vel(const ElJob *__restrict__ jobs)
{
    const ElJob &J = jobs[0];
    const Win w = J.w;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= w.nx) return;
    const int64_t si = sidx(w, x, y, z), mi = midx(w, x, y, z);
    const float g = J.gx[x] * J.gy[y] * J.gz[z];
    const float b0 = J.b[mi];
    const float bx = 0.5f * (b0 + J.b[mi + (x + 1 < w.nx ? 1 : 0)]);
    const float by = 0.5f * (b0 + J.b[mi + (y + 1 < w.ny ? w.mx : 0)]);
    const float bz = 0.5f * (b0 + J.b[mi + (z + 1 < w.nz ? w.my : 0)]);
    const float v0 = g * J.v[0][si], v1 = g * J.v[1][si], v2 = g * J.v[2][si];
    J.v[0][si] = v0;
    J.v[1][si] = v1;
    J.v[2][si] = v2;
    J.aux[0][si] = bx * v0;
    J.aux[1][si] = by * v1;
    J.aux[2][si] = bz * v2;
}

template <int R>
void vel_dispatch(int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W,
                  float dt, hipStream_t st)
{
    constexpr int NY = el_ny<R>();
    dim3 blk(PROP_TX, PROP_BY), grd(ntiles);
    if (mode == EL_FWD) hipLaunchKernelGGL((el_vel<R, NY, EL_FWD>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
    else                hipLaunchKernelGGL((el_vel<R, NY, EL_ADJ>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
}

template <int R>
void stress_dispatch(int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W,
                     float dt, hipStream_t st)
{
    constexpr int NY = el_ny<R>();
    dim3 blk(PROP_TX, PROP_BY), grd(ntiles);
    if (mode == EL_FWD) hipLaunchKernelGGL((el_stress<R, NY, EL_FWD>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
    else                hipLaunchKernelGGL((el_stress<R, NY, EL_ADJ>), grd, blk, 0, st, jobs, tiles, zc, W, dt);
}

}  // namespace

int el_rows_per_thread(int R)
{
    return R <= 4 ? 2 : 1;
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

void launch_el_vel(int R, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc, const Weights &W,
                   float dt, hipStream_t st)
{
    EL_SWITCH(vel_dispatch, mode, jobs, tiles, ntiles, zc, W, dt, st)
}

void launch_el_stress(int R, int mode, const ElJob *jobs, const Tile *tiles, int ntiles, int zc,
                      const Weights &W, float dt, hipStream_t st)
{
    EL_SWITCH(stress_dispatch, mode, jobs, tiles, ntiles, zc, W, dt, st)
}

void launch_el_mix_stress(const ElJob *jobs, int, const Win &w0, hipStream_t st, int64_t)
{
    dim3 blk(256), grd((w0.nx + 255) / 256, w0.ny, w0.nz);
    hipLaunchKernelGGL(el_mix_stress, grd, blk, 0, st, jobs);
}

void launch_el_mix_vel(const ElJob *jobs, int, const Win &w0, hipStream_t st, int64_t)
{
    dim3 blk(256), grd((w0.nx + 255) / 256, w0.ny, w0.nz);
    hipLaunchKernelGGL(el_mix_vel, grd, blk, 0, st, jobs);
}
