// Shared device-side definitions of the propagator kernels (gfx950, wave64).
//
// Layout: every field is a dense (nz, ny, nx) array with x fastest.  Wavefields live in
// "state" arrays of one shot window (row pitch sx, plane pitch sy); model coefficients live
// in whole-grid arrays addressed through the window's offset.
//
// Stencil engine ("2.5D z-march"): a block owns a TX x TY tile of the x-y plane and marches
// through a chunk of z-planes.  For every plane it stages the fields whose x or y derivatives
// are needed into LDS (tile plus an R-wide halo in x and/or y), while the fields whose z
// derivatives are needed sit in per-thread register queues of 2R+1 planes that rotate as the
// block advances.  Each thread owns one x column of NY consecutive rows; a wavefront spans the
// 64 x positions of a row, so every global access of a wavefront is one contiguous run of x.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PROP_TX 64      // tile width in x = wavefront width
#define PROP_BY 8       // threads per block in y (block = 512 threads = 8 wavefronts)
#define PROP_NT (PROP_TX * PROP_BY)

struct Win {
    int nx, ny, nz;       // window shape
    int64_t sx, sy;       // state strides: row, plane (elements)
    int64_t mx, my;       // model strides: row, plane (elements)
    int64_t moff;         // model index of the window's first node
};

// First-derivative weights per axis, already divided by the spacing of that axis.
struct Weights {
    float wx[8], wy[8], wz[8];
};

// Global-address-space views of device pointers.  Pointers read from a job table in memory are
// otherwise treated as generic (flat) pointers; flat loads also count against the LDS wait counter,
// which would make every LDS wait in the compute phase wait for the next plane's prefetch as well.
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ float gld(const float *p, int64_t i) { return ((const gfloat *)p)[i]; }
__device__ __forceinline__ void gst(float *p, int64_t i, float v) { ((gfloat *)p)[i] = v; }

// Third component of the unit symmetry axis from the other two (the axis is stored with nz >= 0;
// n and -n give the same operators).  The hardware square root (within 1 ulp) rather than the
// correctly rounded sqrtf, whose fix-up costs about a dozen more VALU instructions: the stencil
// passes form n_z at every point of every plane, twice where halo columns are recomputed.
__device__ __forceinline__ float axis_z(float n0, float n1)
{
    return __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - n0 * n0 - n1 * n1));
}

__device__ __forceinline__ bool in_win(const Win &w, int x, int y, int z)
{
    return (unsigned)x < (unsigned)w.nx && (unsigned)y < (unsigned)w.ny && (unsigned)z < (unsigned)w.nz;
}
__device__ __forceinline__ int64_t sidx(const Win &w, int x, int y, int z)
{
    return (int64_t)z * w.sy + (int64_t)y * w.sx + x;
}
__device__ __forceinline__ int64_t midx(const Win &w, int x, int y, int z)
{
    return w.moff + (int64_t)z * w.my + (int64_t)y * w.mx + x;
}

// Plane addressing of the z-marching kernels: a load or store names a uniform plane base (64-bit,
// scalar registers) and a per-lane 32-bit byte offset within the plane that stays fixed through the
// march.
typedef __attribute__((address_space(1))) const char gcchar;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ float ldo(gcchar *plane, uint32_t off) { return *(const gfloat *)(plane + off); }
__device__ __forceinline__ void sto(gchar *plane, uint32_t off, float v) { *(gfloat *)(plane + off) = v; }
// Re-define an offset inside the loop body (no instruction of its own): keeps it a 32-bit register
// that the loads add to their scalar base, instead of a widened 64-bit copy per field hoisted out of
// the loop.
__device__ __forceinline__ uint32_t fresh(uint32_t o)
{
    asm volatile("" : "+v"(o));
    return o;
}

// LDS plane of a tile with an R-wide halo on every side (corners unused).
template <int R, int TY>
struct Plane {
    static constexpr int LX = PROP_TX + 2 * R;
    static constexpr int LY = TY + 2 * R;
    static constexpr int SIZE = LX * LY;
    __device__ static __forceinline__ int at(int yy, int xx) { return (yy + R) * LX + xx + R; }
};

// LDS planes of the x and y components of a vector field for its divergence: the x component on
// the tile rows with an R-wide x-halo, the y component on the tile columns with an R-wide y-halo.
template <int R, int TY>
struct XPlane {
    static constexpr int LX = PROP_TX + 2 * R;
    static constexpr int SIZE = LX * TY;
    __device__ static __forceinline__ int at(int yy, int xx) { return yy * LX + xx + R; }
};
template <int R, int TY>
struct YPlane {
    static constexpr int SIZE = PROP_TX * (TY + 2 * R);
    __device__ static __forceinline__ int at(int yy, int xx) { return (yy + R) * PROP_TX + xx; }
};

// Stage the halo of one plane into LDS.  `get(x, y)` returns the (window-local) value at
// (x, y) of the current plane, zero outside the window.  HX: x-halo rows [0, TY), columns
// [-R, 0) and [TX, TX+R); HY: y-halo rows [-R, 0) and [TY, TY+R), columns [0, TX).
template <int R, int TY, bool HX, bool HY, class Get>
__device__ __forceinline__ void stage_halo(float *lds, int tid, int x0, int y0, Get get)
{
    using P = Plane<R, TY>;
    if (HX) {
        for (int i = tid; i < 2 * R * TY; i += PROP_NT) {
            int row = i / (2 * R), c = i - row * (2 * R);
            int xx = c < R ? c - R : PROP_TX + c - R;
            lds[P::at(row, xx)] = get(x0 + xx, y0 + row);
        }
    }
    if (HY) {
        for (int i = tid; i < 2 * R * PROP_TX; i += PROP_NT) {
            int rr = i / PROP_TX, xx = i - rr * PROP_TX;
            int yy = rr < R ? rr - R : TY + rr - R;
            lds[P::at(yy, xx)] = get(x0 + xx, y0 + yy);
        }
    }
}

// Centred first derivative: sum_j w_j (f[+j] - f[-j]).
template <int R>
__device__ __forceinline__ float dc_lds_x(const float *L, int i, const float *w)
{
    float s = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) s += w[j - 1] * (L[i + j] - L[i - j]);
    return s;
}
template <int R, int LX>
__device__ __forceinline__ float dc_lds_y(const float *L, int i, const float *w)
{
    float s = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) s += w[j - 1] * (L[i + j * LX] - L[i - j * LX]);
    return s;
}
template <int R>
__device__ __forceinline__ float dc_q(const float *q, const float *w)
{
    float s = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) s += w[j - 1] * (q[R + j] - q[R - j]);
    return s;
}

// Staggered derivatives at storage index i:
//   plus : sum_j c_j (f[i+j]   - f[i+1-j])   (node -> half node)
//   minus: sum_j c_j (f[i+j-1] - f[i-j])     (half node -> node)
// `st` = stride between neighbours along the axis in the array addressed by `L`.
template <int R, bool PLUS>
__device__ __forceinline__ float ds_lds(const float *L, int i, int st, const float *w)
{
    float s = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        if (PLUS) s += w[j - 1] * (L[i + j * st] - L[i + (1 - j) * st]);
        else      s += w[j - 1] * (L[i + (j - 1) * st] - L[i - j * st]);
    }
    return s;
}
template <int R, bool PLUS>
__device__ __forceinline__ float ds_q(const float *q, const float *w)
{
    float s = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        if (PLUS) s += w[j - 1] * (q[R + j] - q[R + 1 - j]);
        else      s += w[j - 1] * (q[R + j - 1] - q[R - j]);
    }
    return s;
}

// Halo items of a tile plane and their assignment to the threads of a block: x-halo items are
// the 2R columns beside the tile on each of its TY rows, y-halo items the 2R rows above and below
// it on its TX columns.  Thread tid handles items tid, tid + NT, ... of each list.
template <int R, int TY, int NT = PROP_NT>
struct Halo {
    static constexpr int NXI = 2 * R * TY, NYI = 2 * R * PROP_TX;
    static constexpr int NXH = (NXI + NT - 1) / NT, NYH = (NYI + NT - 1) / NT;
    __device__ static __forceinline__ void xitem(int i, int &yy, int &xx)
    {
        const int row = i / (2 * R), c = i - row * (2 * R);
        yy = row;
        xx = c < R ? c - R : PROP_TX + c - R;
    }
    __device__ static __forceinline__ void yitem(int i, int &yy, int &xx)
    {
        const int rr = i / PROP_TX;
        xx = i - rr * PROP_TX;
        yy = rr < R ? rr - R : TY + rr - R;
    }
};

// Tile descriptor of one block: job (shot) index and tile origin.
struct Tile {
    int job, x0, y0, z0;
};
