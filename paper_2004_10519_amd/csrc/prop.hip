// C ABI of the propagators: handle, shot windows, sparse plans, time loops, checkpointed gradient.
#include "prop.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "aux.h"
#include "jobs.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(PROP_EHIP, "%s: %s", #x, hipGetErrorString(e_));     \
    } while (0)

#define TRY(x)                    \
    do {                          \
        int r_ = (x);             \
        if (r_ != PROP_OK) return r_; \
    } while (0)

// Owned device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int ensure(size_t n)
    {
        if (n <= bytes && p) return PROP_OK;
        release();
        if (n == 0) n = 16;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return fail(PROP_ENOMEM, "hipMalloc of %zu bytes failed", n);
        }
        bytes = n;
        return PROP_OK;
    }
    // like ensure, but also gives memory back when the buffer is more than twice the need (large
    // workspaces of an earlier call would otherwise stay allocated beside the new ones)
    int fit(size_t n)
    {
        if (p && bytes > 2 * std::max<size_t>(n, 16)) release();
        return ensure(n);
    }
    template <class T> T *as() const { return (T *)p; }
};

template <class T>
int upload(DevBuf &b, const std::vector<T> &v, hipStream_t st)
{
    TRY(b.ensure(std::max<size_t>(v.size() * sizeof(T), 16)));
    if (!v.empty()) {
        HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return PROP_OK;
}

// ---------------------------------------------------------------------------------------------
// Finite-difference weights (closed forms), stability bound
// ---------------------------------------------------------------------------------------------
double fact(int n)
{
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
double dfact(int n)  // n!! for odd n
{
    double f = 1;
    for (int i = n; i > 1; i -= 2) f *= i;
    return f;
}
// centred, accuracy order 2r: a_j = (-1)^(j+1) (r!)^2 / (j (r-j)! (r+j)!)
void centred_weights(int r, double *a)
{
    for (int j = 1; j <= r; ++j) a[j - 1] = ((j & 1) ? 1.0 : -1.0) * fact(r) * fact(r) / (j * fact(r - j) * fact(r + j));
}
// staggered (nodes at +-(j - 1/2)), order 2r: c_j = (-1)^(j+1) ((2r-1)!!)^2 / ((2j-1)^2 (r+j-1)! (r-j)! 4^(r-1))
void staggered_weights(int r, double *c)
{
    for (int j = 1; j <= r; ++j)
        c[j - 1] = ((j & 1) ? 1.0 : -1.0) * dfact(2 * r - 1) * dfact(2 * r - 1) /
                   ((2.0 * j - 1) * (2.0 * j - 1) * fact(r + j - 1) * fact(r - j) * std::pow(4.0, r - 1));
}
// S_D = max_k (sum_j 2 a_j sin(j k))^2 over k in [0, pi]: coarse scan, then golden-section refinement.
double centred_symbol_max(int r)
{
    double a[8];
    centred_weights(r, a);
    auto f = [&](double k) {
        double s = 0;
        for (int j = 1; j <= r; ++j) s += 2 * a[j - 1] * std::sin(j * k);
        return s * s;
    };
    const int n = 4096;
    double best = 0, kb = 0;
    for (int i = 0; i <= n; ++i) {
        double k = M_PI * i / n, v = f(k);
        if (v > best) best = v, kb = k;
    }
    double lo = std::max(0.0, kb - M_PI / n), hi = std::min(M_PI, kb + M_PI / n);
    const double gr = 0.5 * (std::sqrt(5.0) - 1);
    for (int it = 0; it < 80; ++it) {
        double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
        if (f(c) > f(d)) hi = d; else lo = c;
    }
    return std::max(best, f(0.5 * (lo + hi)));
}

int check_grid(prop_kind kind, const prop_grid *g)
{
    if (!g) return fail(PROP_EINVAL, "grid is NULL");
    if (kind != PROP_TTI && kind != PROP_ELASTIC) return fail(PROP_EINVAL, "unknown propagator kind %d", (int)kind);
    if (g->ndim != 2 && g->ndim != 3) return fail(PROP_EINVAL, "ndim must be 2 or 3");
    if (g->ndim == 2 && g->shape[1] != 1) return fail(PROP_EINVAL, "2D grids need shape[1] == 1");
    if (g->space_order < 2 || g->space_order > 16 || (g->space_order & 1))
        return fail(PROP_EINVAL, "space_order must be even in [2, 16], got %d", g->space_order);
    if (kind == PROP_TTI && g->time_order != 2) return fail(PROP_EINVAL, "TTI needs time_order 2");
    if (kind == PROP_ELASTIC && g->time_order != 1) return fail(PROP_EINVAL, "elastic needs time_order 1");
    if (g->nbl < 0) return fail(PROP_EINVAL, "nbl must be >= 0");
    if (!(g->dt > 0) || g->nt < 1) return fail(PROP_EINVAL, "dt must be > 0 and nt >= 1");
    if (g->nbl > 0 && !(g->v_ref > 0)) return fail(PROP_EINVAL, "v_ref must be > 0 with an absorbing layer");
    if (g->free_surface < 0 || g->free_surface > 2) return fail(PROP_EINVAL, "free_surface must be 0, 1 or 2");
    if (g->free_surface && kind != PROP_ELASTIC) return fail(PROP_EINVAL, "a free surface is elastic only");
    if (g->free_surface && g->nbl < g->space_order / 2)
        return fail(PROP_EINVAL, "a free surface needs nbl >= space_order / 2 vacuum rows");
    if (g->free_surface == 2 && g->nbl < g->space_order - 2)
        return fail(PROP_EINVAL, "an image free surface needs nbl >= space_order - 2 image rows");
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) continue;
        if (!(g->spacing[a] > 0)) return fail(PROP_EINVAL, "spacing must be > 0");
        if (g->shape[a] < 2) return fail(PROP_EINVAL, "every active axis needs >= 2 points");
    }
    return PROP_OK;
}

double cfl_dt(prop_kind kind, const prop_grid *g, double vmax, double eps_max)
{
    const int r = g->space_order / 2;
    double inv2 = 0, hmin = 1e300;
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) continue;
        inv2 += 1.0 / (g->spacing[a] * g->spacing[a]);
        hmin = std::min(hmin, g->spacing[a]);
    }
    if (kind == PROP_TTI) {
        const double S = centred_symbol_max(r);
        return 2.0 / (vmax * std::sqrt((1 + 2 * std::max(eps_max, 0.0)) * S * inv2));
    }
    double c[8], sum = 0;
    staggered_weights(r, c);
    for (int j = 0; j < r; ++j) sum += std::fabs(c[j]);
    return hmin / (vmax * std::sqrt((double)g->ndim) * sum);
}

// ---------------------------------------------------------------------------------------------
// Shot window workspace
// ---------------------------------------------------------------------------------------------
struct Plans {
    DevBuf b[8];
    Csr csr{};
    Gather gat{};
};

struct Slot {
    Win w{};
    int64_t o[3] = {0, 0, 0};
    int64_t plane = 0;          // sy * nz: elements of one state field
    DevBuf fields;              // all wavefields of this window
    float *f[24] = {};          // TTI: 0-1 p, 2-3 q, 4-9 t/s, 10 grad, 11-12 yp, 13-14 yq, 15-18 w = C y
                                // (two levels of two components)
                                // elastic: 0-2 v, 3-8 tau, 9-14 sigma, 15-17 u (adjoint)
    DevBuf tabs;                // damping tables (nx + ny + nz floats)
    Plans src_inj, rec_inj, rec_inj_vz, rec_gat, rec_gat_vz, src_gat;
    DevBuf job_fwd, job_adj;    // TTIJob / ElJob on the device
    DevBuf tiles, tiles2;        // tile lists (TTI: pass 1 and pass 2 use different tile heights)
    int ntiles = 0, ntiles2 = 0, zc = 0, zc2 = 0;   // zc2: z-chunk of tiles2 (elastic stress pass)
    DevBuf tiles_ef, job_ef;     // elastic fused step: its tiles and its two jobs (one per buffer set)
    int ntiles_ef = 0, zc_ef = 0;
    int nsrc = 0, nrec = 0;
};

}  // namespace

struct prop_s {
    prop_kind kind;
    prop_grid g;
    hipStream_t st;
    prop_model model;
    int R;
    Weights W;
    DevBuf coef;                // TTI: A, B, nx, ny (axis with nz >= 0); elastic: lam, mu, b (whole grid)
    const float *c[5] = {};
    DevBuf stats, dotpart, dotout, flag;
    Slot slot;
    // gradient workspace
    DevBuf ckpt, ckscale, seg;
    // elastic gradient workspace: forward fields, accumulators, jobs
    DevBuf elfwd, elacc, eljob_f, eljob_g;
    // batched workspace
    std::vector<std::unique_ptr<Slot>> bslots;
    DevBuf bjobs_fwd, bjobs_adj, btiles;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> evpool;
    std::vector<std::pair<int, int>> pending[5];
    int evnext = 0;
    double ms[5] = {0, 0, 0, 0, 0};
    int64_t launches[5] = {0, 0, 0, 0, 0};
    int last_state = 0;         // 0 none, 1 forward, 2 adjoint
    int last_groups = 0;        // shot groups used by the last batched call
    // options (prop_set_option)
    int opt_graph = 0, opt_autotune = 0, opt_xcd = 0;
    int opt_el_fused = 0;       // elastic forward: the fused velocity-stress step where it applies
    int opt_shape[2] = {1, 1};  // tile variants: TTI pass 1 / pass 2 when not autotuning; elastic
                                // velocity / stress pass (and imaging condition)
    int opt_zc = 0;             // fixed z-chunk length (0: automatic)
    int opt_zc2 = 0;            // fixed z-chunk of TTI pass 2 or of the elastic stress pass (0: that
                                // of pass 1 / the velocity pass)
    int opt_scheme = TTI_SIX;   // TTI step scheme (TTI_SIX, TTI_FUSED, TTI_FOUR or TTI_SPLIT); set at create
    int64_t opt_batch_mb = 0;   // memory budget of the batched planner (0: 85 % of free memory)
    // autotuner: best tile variant and z-chunk per pass, per (direction, window set)
    struct Tune {
        int shape[2], zc[2];
    };
    std::map<std::string, Tune> tuned;
    Tune last_tune{{1, 1}, {0, 0}};
    // checkpoints left by a saving prop_forward (shot identity, count and type)
    struct Saved {
        bool valid = false;
        int n_ckpt = 0, dtype = 0, nsrc = 0;
        int64_t o[3] = {0, 0, 0}, n[3] = {0, 0, 0};
        const float *wav = nullptr;
        std::vector<float> src;
    } saved;
    // graph capture of time-step runs
    hipStream_t cap = nullptr;
    std::vector<hipGraphExec_t> execs;
    int64_t graphs_launched = 0;
};

namespace {

int64_t npts_grid(const prop_grid &g) { return g.shape[0] * g.shape[1] * g.shape[2]; }

// Damping profile (absorbing layer, nbl points inside the window on every face):
// kappa_a(i) = kmax_a (d/nbl)^2, d = depth in points into the layer, kmax_a = 3 vref ln(1000) / (2 nbl h_a).
double kappa(const prop_grid &g, int axis, int64_t i, int64_t n)
{
    if (g.nbl <= 0) return 0.0;
    if (g.ndim == 2 && axis == 1) return 0.0;
    const double top = (axis == 2 && g.free_surface) ? 0.0 : g.nbl - (double)i;   // free surface: no top layer
    double d = std::max<double>(std::max<double>(top, (double)i - (double)(n - 1 - g.nbl)), 0.0);
    double kmax = 3.0 * g.v_ref * std::log(1000.0) / (2.0 * g.nbl * g.spacing[axis]);
    return kmax * (d / g.nbl) * (d / g.nbl);
}

// The fused TTI pass addresses a point within its x-y plane by a 32-bit byte offset (state and
// model layouts); planes of 4 GiB or more take the two-pass scheme.
bool fused_fits(const prop_grid &g)
{
    const double plane = (double)((g.shape[0] + 63) / 64 * 64) * (double)g.shape[1] * 4.0;
    return plane < 4294967296.0 && (double)g.shape[0] * (double)g.shape[1] * 4.0 < 4294967296.0;
}

int tile_rows(const prop_s *h, int pass, int shape)
{
    if (h->kind == PROP_TTI) return tti_tile_rows(h->R, h->opt_scheme, pass, shape);
    // elastic: the launchers take el_tile_rows' height or, on 3D grids, 8 rows (tile variant 0)
    return h->g.ndim == 3 && shape == 0 ? 8 : el_tile_rows(h->R, h->g.ndim);
}

// Tiles of a set of windows in spatial order (x fastest, then y, then z chunk of zc planes).  With
// the XCD option the order is dealt round-robin over the 8 XCDs so that each XCD gets a contiguous
// range of neighbouring tiles (measured on the 512^3 workload: plain order is ~3% faster).
void make_tiles(const std::vector<Slot *> &slots, int TY, int zc, bool xcd, std::vector<Tile> &out, int TX = PROP_TX)
{
    std::vector<Tile> sp;
    for (size_t j = 0; j < slots.size(); ++j) {
        const Win &w = slots[j]->w;
        for (int z0 = 0; z0 < w.nz; z0 += zc)
            for (int y0 = 0; y0 < w.ny; y0 += TY)
                for (int x0 = 0; x0 < w.nx; x0 += TX) sp.push_back(Tile{(int)j, x0, y0, z0});
    }
    const size_t T = sp.size(), X = xcd ? 8 : 1;
    out.assign(T, Tile{});
    const size_t per = (T + X - 1) / X;
    size_t b = 0;
    // block b runs on XCD b % 8; give XCD c the spatial range [c*per, (c+1)*per)
    for (size_t i = 0; i < per; ++i)
        for (size_t c = 0; c < X; ++c) {
            size_t s = c * per + i;
            if (s < T) out[b++] = sp[s];
        }
}

// z-chunk length: enough chunks for ~2048 blocks (elastic: ~4096; its two passes have no
// autotuner, and 17-plane chunks measured 4 % faster than 34-plane ones at 400^3 so8), but chunks
// of at least 4R planes (the z halo of a chunk is re-read by its neighbour).  The fused and split
// TTI passes hold one block per CU (LDS, registers), so they aim at fewer blocks: longer chunks
// re-read less of the z halo.  The fused pass aims at ~512 (at 256^3 so8, 512 blocks ran 272 us a
// step against 343 us for 1024 and 442 us for 2048; 256 made the 64 plain shots of the batched
// workload 10 % slower), the split pair at ~256, one wave (at 512^3 so12 pass B ran 1.507 ms with
// 256 blocks against 1.529 with 512 and 1.579 with 1024).
// 2D elastic grids run one-row tiles with few of them per plane and fit in cache: chunks down to
// R planes (5-plane chunks measured 1.4x faster than 17-plane ones on the 1701 x 391 marine grid).
int choose_zc(const prop_s *h, int nz, int64_t tiles_xy)
{
    if (h->opt_zc > 0) return std::min(h->opt_zc, nz);
    const bool one_block_per_cu = h->opt_scheme == TTI_FUSED || h->opt_scheme == TTI_SPLIT;
    const int64_t target =
        h->kind == PROP_TTI ? (h->opt_scheme == TTI_SPLIT ? 256 : one_block_per_cu ? 512 : 2048) : 4096;
    const int minlen = h->kind == PROP_ELASTIC && h->g.ndim == 2 ? h->R : 4 * h->R;
    int64_t nch = (target + tiles_xy - 1) / tiles_xy;
    nch = std::max<int64_t>(1, std::min<int64_t>(nch, std::max(1, nz / minlen)));
    return (int)((nz + nch - 1) / nch);
}

// Window of a shot, validated against the grid.
int shot_window(const prop_s *h, const prop_shot *s, int64_t o[3], int64_t n[3])
{
    for (int a = 0; a < 3; ++a) {
        o[a] = s->win_origin[a];
        n[a] = s->win_shape[a];
    }
    if (n[0] == 0 && n[1] == 0 && n[2] == 0)
        for (int a = 0; a < 3; ++a) o[a] = 0, n[a] = h->g.shape[a];
    for (int a = 0; a < 3; ++a) {
        if (o[a] < 0 || n[a] < 1 || o[a] + n[a] > h->g.shape[a]) return fail(PROP_EINVAL, "window outside the grid");
        if (!(h->g.ndim == 2 && a == 1) && n[a] < 2) return fail(PROP_EINVAL, "window needs >= 2 points per axis");
        if (!(h->g.ndim == 2 && a == 1) && n[a] < 2 * (int64_t)h->g.nbl + 2)
            return fail(PROP_EINVAL, "window smaller than its absorbing layers");
    if (h->g.free_surface && o[2] != 0) return fail(PROP_EINVAL, "with a free surface a window starts at z index 0");
    }
    return PROP_OK;
}

// Corners and weights of off-grid points on a window (optionally staggered by half a cell in z).
struct PointCorners {
    std::vector<int64_t> sidx, midx;
    std::vector<int32_t> cell[3];
    std::vector<double> w;
    int nc = 0;
};

int corners(const prop_s *h, const Slot &sl, const float *xyz, int npt, double zstag, PointCorners &pc)
{
    const prop_grid &g = h->g;
    const int nd = g.ndim;
    const int axes[3] = {0, nd == 3 ? 1 : 2, 2};
    pc.nc = 1 << nd;
    pc.sidx.assign((size_t)npt * pc.nc, 0);
    pc.midx.assign((size_t)npt * pc.nc, 0);
    pc.w.assign((size_t)npt * pc.nc, 1.0);
    for (int a = 0; a < 3; ++a) pc.cell[a].assign((size_t)npt * pc.nc, 0);
    const int64_t nwin[3] = {sl.w.nx, sl.w.ny, sl.w.nz};
    for (int p = 0; p < npt; ++p) {
        int64_t i0[3] = {0, 0, 0};
        double al[3] = {0, 0, 0};
        for (int k = 0; k < nd; ++k) {
            const int ax = axes[k];
            const double x = xyz[(size_t)p * nd + k];
            const double stag = (ax == 2) ? zstag : 0.0;
            const double u = (x - g.origin[ax]) / g.spacing[ax] - stag - (double)sl.o[ax];
            if (!(u >= 0.0) || u > (double)(nwin[ax] - 1))
                return fail(PROP_EINVAL, "point %d (axis %d) lies outside the shot window", p, ax);
            int64_t i = (int64_t)std::floor(u);
            double a = u - (double)i;
            if (i >= nwin[ax] - 1) i = nwin[ax] - 2, a = 1.0;
            i0[ax] = i;
            al[ax] = a;
        }
        for (int c = 0; c < pc.nc; ++c) {
            int64_t ix[3] = {i0[0], i0[1], i0[2]};
            double wt = 1.0;
            for (int k = 0; k < nd; ++k) {
                const int ax = axes[k];
                const int bit = (c >> k) & 1;
                ix[ax] += bit;
                wt *= bit ? al[ax] : 1.0 - al[ax];
            }
            const size_t e = (size_t)p * pc.nc + c;
            pc.sidx[e] = ix[2] * sl.w.sy + ix[1] * sl.w.sx + ix[0];
            pc.midx[e] = sl.w.moff + ix[2] * sl.w.my + ix[1] * sl.w.mx + ix[0];
            for (int a = 0; a < 3; ++a) pc.cell[a][e] = (int32_t)ix[a];
            pc.w[e] = wt;
        }
    }
    return PROP_OK;
}

// Gather plan over the points listed in `sel` (indices into xyz), writing output column sel[o].
int build_gather(const prop_s *h, Slot &sl, const float *xyz, const std::vector<int> &sel, double zstag, Plans &pl)
{
    const int nd = h->g.ndim;
    std::vector<float> sub((size_t)sel.size() * nd);
    for (size_t i = 0; i < sel.size(); ++i)
        for (int k = 0; k < nd; ++k) sub[i * nd + k] = xyz[(size_t)sel[i] * nd + k];
    PointCorners pc;
    TRY(corners(h, sl, sub.data(), (int)sel.size(), zstag, pc));
    std::vector<float> wf(pc.w.begin(), pc.w.end());
    TRY(upload(pl.b[0], pc.sidx, h->st));
    TRY(upload(pl.b[1], wf, h->st));
    TRY(upload(pl.b[2], sel, h->st));
    pl.gat = Gather{(int)sel.size(), pc.nc, pl.b[0].as<int64_t>(), pl.b[1].as<float>(), pl.b[2].as<int>()};
    return PROP_OK;
}

// Node-wise injection plan (sorted by node, deterministic summation order within a row).
int build_csr(const prop_s *h, Slot &sl, const float *xyz, const std::vector<int> &sel, double zstag, Plans &pl)
{
    const int nd = h->g.ndim;
    std::vector<float> sub((size_t)sel.size() * nd);
    for (size_t i = 0; i < sel.size(); ++i)
        for (int k = 0; k < nd; ++k) sub[i * nd + k] = xyz[(size_t)sel[i] * nd + k];
    PointCorners pc;
    TRY(corners(h, sl, sub.data(), (int)sel.size(), zstag, pc));
    const size_t ne = pc.sidx.size();
    std::vector<size_t> ord(ne);
    for (size_t i = 0; i < ne; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return pc.sidx[a] < pc.sidx[b]; });
    std::vector<int64_t> node, mnode;
    std::vector<float> e, w;
    std::vector<int> ptr, col;
    for (size_t k = 0; k < ne; ++k) {
        const size_t i = ord[k];
        if (node.empty() || node.back() != pc.sidx[i]) {
            node.push_back(pc.sidx[i]);
            mnode.push_back(pc.midx[i]);
            ptr.push_back((int)col.size());
            // damping term eta/(2dt) of the node, summed in the kernel's order
            float ev = 0.f;
            if (h->kind == PROP_TTI) {
                const int64_t n3[3] = {sl.w.nx, sl.w.ny, sl.w.nz};
                float tx = (float)(kappa(h->g, 0, pc.cell[0][i], n3[0]) / (h->g.v_ref * h->g.v_ref) / (2 * h->g.dt));
                float ty = (float)(kappa(h->g, 1, pc.cell[1][i], n3[1]) / (h->g.v_ref * h->g.v_ref) / (2 * h->g.dt));
                float tz = (float)(kappa(h->g, 2, pc.cell[2][i], n3[2]) / (h->g.v_ref * h->g.v_ref) / (2 * h->g.dt));
                if (h->g.nbl <= 0) tx = ty = tz = 0.f;
                ev = tx + ty + tz;
            }
            e.push_back(ev);
        }
        col.push_back(sel[i / pc.nc]);
        w.push_back((float)pc.w[i]);
    }
    ptr.push_back((int)col.size());
    TRY(upload(pl.b[0], node, h->st));
    TRY(upload(pl.b[1], mnode, h->st));
    TRY(upload(pl.b[2], e, h->st));
    TRY(upload(pl.b[3], ptr, h->st));
    TRY(upload(pl.b[4], col, h->st));
    TRY(upload(pl.b[5], w, h->st));
    pl.csr = Csr{(int)node.size(), pl.b[0].as<int64_t>(), pl.b[1].as<int64_t>(), pl.b[2].as<float>(),
                 pl.b[3].as<int>(), pl.b[4].as<int>(), pl.b[5].as<float>()};
    return PROP_OK;
}

// Allocate the window's fields (reused when the shape is unchanged) and build its tables/jobs.
int setup_slot(prop_s *h, Slot &sl, const int64_t o[3], const int64_t n[3])
{
    const bool same = sl.fields.p && sl.w.nx == n[0] && sl.w.ny == n[1] && sl.w.nz == n[2] && sl.o[0] == o[0] &&
                      sl.o[1] == o[1] && sl.o[2] == o[2];
    Win w{};
    w.nx = (int)n[0];
    w.ny = (int)n[1];
    w.nz = (int)n[2];
    w.sx = (n[0] + 63) / 64 * 64;
    w.sy = w.sx * n[1];
    w.mx = h->g.shape[0];
    w.my = h->g.shape[0] * h->g.shape[1];
    w.moff = o[2] * w.my + o[1] * w.mx + o[0];
    sl.w = w;
    for (int a = 0; a < 3; ++a) sl.o[a] = o[a];
    sl.plane = w.sy * w.nz;
    const int nf = h->kind == PROP_TTI ? 19 : 18;
    if (!same) TRY(sl.fields.ensure((size_t)nf * sl.plane * sizeof(float)));
    for (int i = 0; i < nf; ++i) sl.f[i] = sl.fields.as<float>() + (size_t)i * sl.plane;
    // damping tables
    std::vector<float> tab((size_t)w.nx + w.ny + w.nz);
    const int64_t nn[3] = {w.nx, w.ny, w.nz};
    size_t off = 0;
    for (int a = 0; a < 3; ++a)
        for (int64_t i = 0; i < nn[a]; ++i) {
            const double k = kappa(h->g, a, i, nn[a]);
            tab[off++] = h->kind == PROP_TTI ? (float)(k / (h->g.v_ref * h->g.v_ref) / (2 * h->g.dt) * (h->g.nbl > 0))
                                             : (float)std::exp(-k * h->g.dt);
        }
    TRY(upload(sl.tabs, tab, h->st));
    // 3D elastic z-chunks are sized on 64 x 16 tile columns whatever the tile heights of the two passes
    // (400^3 so8: the 64 x 8 velocity pass ran 0.743 ms with the 17-plane chunks this gives, 0.775 ms
    // with the 34 that its own tile count would give; the 64 x 16 stress pass 0.990 ms with 17
    // planes, 0.999 with 16 or 13)
    const int TY = h->kind == PROP_ELASTIC && h->g.ndim == 3 ? 16 : tile_rows(h, 1, h->opt_shape[0]);
    const int64_t txy = (int64_t)((w.nx + PROP_TX - 1) / PROP_TX) * ((w.ny + TY - 1) / TY);
    sl.zc = choose_zc(h, w.nz, txy);
    sl.zc2 = sl.zc;   // the elastic stress pass runs its own tiles (TILE2) and may take its own z-chunk
    if (h->kind == PROP_ELASTIC && h->opt_zc2 > 0) sl.zc2 = std::min(h->opt_zc2, (int)w.nz);
    return PROP_OK;
}

TTIJob tti_job(const prop_s *h, const Slot &sl, bool adjoint)
{
    TTIJob J{};
    J.w = sl.w;
    const int b = adjoint ? 11 : 0;
    J.p[0] = sl.f[b + 0];
    J.p[1] = sl.f[b + 1];
    J.q[0] = sl.f[adjoint ? 13 : 2];
    J.q[1] = sl.f[adjoint ? 14 : 3];
    for (int l = 0; l < 2; ++l)
        for (int c = 0; c < 2; ++c) J.wmix[l][c] = adjoint ? sl.f[15 + 2 * l + c] : nullptr;
    for (int i = 0; i < 3; ++i) {
        J.t[i] = sl.f[4 + i];
        J.s[i] = sl.f[7 + i];
    }
    J.m = h->model.p[0];
    J.A = h->c[0];
    J.B = h->c[1];
    J.nx = h->c[2];
    J.ny = h->c[3];
    const float *tab = sl.tabs.as<float>();
    J.ex = tab;
    J.ey = tab + sl.w.nx;
    J.ez = tab + sl.w.nx + sl.w.ny;
    J.grad = sl.f[10];
    J.seg = nullptr;
    J.seg_field = sl.plane;
    return J;
}

ElJob el_job(const prop_s *h, const Slot &sl)
{
    ElJob J{};
    J.w = sl.w;
    for (int i = 0; i < 3; ++i) J.v[i] = J.vo[i] = sl.f[i];
    for (int i = 0; i < 6; ++i) J.t[i] = sl.f[3 + i];
    for (int i = 0; i < 6; ++i) J.aux[i] = sl.f[9 + i];
    for (int i = 0; i < 3; ++i) J.u[i] = sl.f[15 + i];
    J.lam = h->c[0];
    J.mu = h->c[1];
    J.b = h->c[2];
    const float *tab = sl.tabs.as<float>();
    J.gx = tab;
    J.gy = tab + sl.w.nx;
    J.gz = tab + sl.w.nx + sl.w.ny;
    return J;
}

template <class T>
int upload_one(DevBuf &b, const T &v, hipStream_t st)
{
    std::vector<T> tmp(1, v);
    return upload(b, tmp, st);
}

int set_tiles(prop_s *h, Slot &sl)
{
    std::vector<Slot *> one{&sl};
    std::vector<Tile> tiles;
    make_tiles(one, tile_rows(h, 1, h->opt_shape[0]), sl.zc, h->opt_xcd, tiles);
    sl.ntiles = (int)tiles.size();
    TRY(upload(sl.tiles, tiles, h->st));
    make_tiles(one, tile_rows(h, 2, h->opt_shape[1]), sl.zc2, h->opt_xcd, tiles);
    sl.ntiles2 = (int)tiles.size();
    return upload(sl.tiles2, tiles, h->st);
}

// Timing of the stencil launches.
hipEvent_t next_event(prop_s *h)
{
    if (h->evnext >= (int)h->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->evpool.push_back(e);
    }
    return h->evpool[h->evnext++];
}

int fold_timing(prop_s *h)
{
    bool any = false;
    for (int k = 0; k < 5; ++k) any |= !h->pending[k].empty();
    if (!any) return PROP_OK;
    HIPCHK(hipStreamSynchronize(h->st));
    for (int k = 0; k < 5; ++k) {
        for (auto &pr : h->pending[k]) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, h->evpool[pr.first], h->evpool[pr.second]));
            h->ms[k] += ms;
            h->launches[k]++;
        }
        h->pending[k].clear();
    }
    h->evnext = 0;
    return PROP_OK;
}

struct Timed {
    prop_s *h;
    int k;
    int a = -1;
    Timed(prop_s *h_, int k_) : h(h_), k(k_)
    {
        if (!h->timing) return;
        if (h->evnext + 2 > 8192) fold_timing(h);
        a = h->evnext;
        hipEvent_t e = next_event(h);
        if (e) (void)hipEventRecord(e, h->st); else a = -1;
    }
    ~Timed()
    {
        if (a < 0) return;
        int b = h->evnext;
        hipEvent_t e = next_event(h);
        if (!e) return;
        (void)hipEventRecord(e, h->st);
        h->pending[k].push_back({a, b});
    }
};

void release_graphs(prop_s *h)
{
    for (auto e : h->execs) (void)hipGraphExecDestroy(e);
    h->execs.clear();
}

int check_finite(prop_s *h, const float *f, const Win &w, const char *what = "wavefield", int step = -1, int shot = 0)
{
    aux_fill_u32(h->flag.as<unsigned>(), 1, 0u, h->st);
    aux_nonfinite_win(f, w, h->flag.as<unsigned>(), h->st);
    unsigned v = 0;
    HIPCHK(hipMemcpyAsync(&v, h->flag.p, sizeof v, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    release_graphs(h);
    if (v) return fail(PROP_EUNSTABLE, "non-finite values in %s (shot %d, step %d): instability", what, shot, step);
    return PROP_OK;
}

const int WATCH_EVERY = 500;

int prep_model(prop_s *h, const prop_model *m)
{
    if (!m) return fail(PROP_EINVAL, "model is NULL");
    const int need = h->kind == PROP_TTI ? (h->g.ndim == 3 ? 5 : 4) : 3;
    for (int i = 0; i < need; ++i)
        if (!m->p[i]) return fail(PROP_EINVAL, "model array %d is NULL", i);
    h->model = *m;
    const int64_t n = npts_grid(h->g);
    const int nc = h->kind == PROP_TTI ? 4 : 3;
    TRY(h->coef.ensure((size_t)nc * n * sizeof(float)));
    for (int i = 0; i < nc; ++i) h->c[i] = h->coef.as<float>() + (size_t)i * n;
    TRY(h->stats.ensure(4 * sizeof(unsigned)));
    aux_fill_u32(h->stats.as<unsigned>(), 4, 0u, h->st);
    float *cc = h->coef.as<float>();
    if (h->kind == PROP_TTI)
        aux_tti_prep(m->p[0], m->p[1], m->p[2], m->p[3], h->g.ndim == 3 ? m->p[4] : m->p[3], n, h->g.ndim, cc,
                     cc + n, cc + 2 * n, cc + 3 * n, h->stats.as<unsigned>(), h->st);
    else
        aux_el_prep(m->p[0], m->p[1], m->p[2], n, cc, cc + n, cc + 2 * n, h->stats.as<unsigned>(),
                    (int64_t)h->g.shape[0] * h->g.shape[1], h->g.nbl, h->g.free_surface == 2 ? h->g.nbl + h->R + 1 : 0,
                    h->st);
    if (h->kind == PROP_ELASTIC && h->g.free_surface) {   // vacuum rows above the free surface
        const int64_t plane = (int64_t)h->g.shape[1] * h->g.shape[0], nv = (int64_t)h->g.nbl * plane;
        aux_fill(cc, nv, 0.f, h->st);
        aux_fill(cc + n, nv, 0.f, h->st);
        if (h->g.free_surface == 2)   // image rows: the buoyancy of the rows below, mirrored
            for (int k = 1; k <= h->g.nbl; ++k)
                HIPCHK(hipMemcpyAsync(cc + 2 * n + (int64_t)(h->g.nbl - k) * plane,
                                      cc + 2 * n + (int64_t)(h->g.nbl + k) * plane, plane * sizeof(float),
                                      hipMemcpyDeviceToDevice, h->st));
    }
    HIPCHK(hipGetLastError());
    unsigned s[4];
    HIPCHK(hipMemcpyAsync(s, h->stats.p, sizeof s, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (s[2] & 1u) return fail(PROP_EINVAL, "model has non-positive or non-finite values");
    if (h->kind == PROP_TTI && (s[2] & 2u)) return fail(PROP_EUNSTABLE, "epsilon < delta somewhere (unstable)");
    if (h->kind == PROP_ELASTIC && (s[2] & 2u)) return fail(PROP_EINVAL, "vp^2 < 2 vs^2 somewhere (negative lambda)");
    if (h->kind == PROP_ELASTIC && (s[2] & 4u))
        return fail(PROP_EINVAL, "an image free surface needs a fluid (vs = 0) on rows nbl .. nbl + space_order / 2");
    float vmax, emax;
    std::memcpy(&vmax, &s[0], 4);
    std::memcpy(&emax, &s[1], 4);
    const double bound = cfl_dt(h->kind, &h->g, vmax, emax);
    if (h->g.dt > bound * (1 + 1e-9))
        return fail(PROP_EUNSTABLE, "dt = %g exceeds the stability bound %g (vmax %g)", h->g.dt, bound, (double)vmax);
    h->last_state = 0;
    h->saved.valid = false;
    return PROP_OK;
}

// -------------------------------------------------------------------------- single-shot setup (elastic)
int prepare_shot(prop_s *h, Slot &sl, const prop_shot *s, bool need_src_inj, bool need_rec_gat, bool need_rec_inj,
                 bool need_src_gat)
{
    if (!s) return fail(PROP_EINVAL, "shot is NULL");
    if (s->nsrc < 0 || s->nrec < 0) return fail(PROP_EINVAL, "negative point count");
    if (s->nsrc > 0 && !s->src_xyz) return fail(PROP_EINVAL, "src_xyz is NULL");
    if (s->nrec > 0 && !s->rec_xyz) return fail(PROP_EINVAL, "rec_xyz is NULL");
    int64_t o[3], n[3];
    TRY(shot_window(h, s, o, n));
    TRY(setup_slot(h, sl, o, n));
    TRY(set_tiles(h, sl));
    sl.nsrc = s->nsrc;
    sl.nrec = s->nrec;
    std::vector<int> all_src(s->nsrc), recP, recV;
    for (int i = 0; i < s->nsrc; ++i) all_src[i] = i;
    for (int i = 0; i < s->nrec; ++i) {
        const int k = s->rec_kind ? s->rec_kind[i] : 0;
        if (k != 0 && k != 1) return fail(PROP_EINVAL, "rec_kind must be 0 or 1");
        (k == 0 ? recP : recV).push_back(i);
    }
    sl.src_inj.csr = Csr{};
    sl.rec_inj.csr = Csr{};
    sl.rec_inj_vz.csr = Csr{};
    sl.rec_gat.gat = Gather{};
    sl.rec_gat_vz.gat = Gather{};
    sl.src_gat.gat = Gather{};
    if (need_src_inj && s->nsrc) TRY(build_csr(h, sl, s->src_xyz, all_src, 0.0, sl.src_inj));
    if (need_src_gat && s->nsrc) TRY(build_gather(h, sl, s->src_xyz, all_src, 0.0, sl.src_gat));
    if (need_rec_gat) {
        if (!recP.empty()) TRY(build_gather(h, sl, s->rec_xyz, recP, 0.0, sl.rec_gat));
        if (!recV.empty()) TRY(build_gather(h, sl, s->rec_xyz, recV, 0.5, sl.rec_gat_vz));
    }
    if (need_rec_inj) {
        if (!recP.empty()) TRY(build_csr(h, sl, s->rec_xyz, recP, 0.0, sl.rec_inj));
        if (!recV.empty()) TRY(build_csr(h, sl, s->rec_xyz, recV, 0.5, sl.rec_inj_vz));
    }
    TRY(upload_one(sl.job_fwd, el_job(h, sl), h->st));
    return PROP_OK;
}

// -------------------------------------------------------------------------- TTI shot groups
// A group is a set of shot windows stepped in lockstep: one job table, one tile list per pass
// covering the tiles of every shot, and concatenated source/receiver plans whose rows carry the
// shot's index.  A plain call is a group of one.
struct HostCsr {
    std::vector<int> shot, ptr, col;
    std::vector<int64_t> node, mnode;
    std::vector<float> e, w;
};
struct HostGather {
    std::vector<int> shot, pos;
    std::vector<int64_t> idx;
    std::vector<float> w;
    int nc = 0;
};

int append_csr(const prop_s *h, const Slot &sl, int shot, const float *xyz, int npt, HostCsr &hc)
{
    std::vector<int> sel(npt);
    for (int i = 0; i < npt; ++i) sel[i] = i;
    PointCorners pc;
    TRY(corners(h, sl, xyz, npt, 0.0, pc));
    const size_t ne = pc.sidx.size();
    std::vector<size_t> ord(ne);
    for (size_t i = 0; i < ne; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return pc.sidx[a] < pc.sidx[b]; });
    const int64_t n3[3] = {sl.w.nx, sl.w.ny, sl.w.nz};
    int64_t last = -1;
    for (size_t k = 0; k < ne; ++k) {
        const size_t i = ord[k];
        if (pc.sidx[i] != last) {
            last = pc.sidx[i];
            hc.shot.push_back(shot);
            hc.node.push_back(pc.sidx[i]);
            hc.mnode.push_back(pc.midx[i]);
            hc.ptr.push_back((int)hc.col.size());
            float ev = 0.f;
            if (h->g.nbl > 0) {
                const double s2 = h->g.v_ref * h->g.v_ref * 2 * h->g.dt;
                const float tx = (float)(kappa(h->g, 0, pc.cell[0][i], n3[0]) / s2);
                const float ty = (float)(kappa(h->g, 1, pc.cell[1][i], n3[1]) / s2);
                const float tz = (float)(kappa(h->g, 2, pc.cell[2][i], n3[2]) / s2);
                ev = tx + ty + tz;
            }
            hc.e.push_back(ev);
        }
        hc.col.push_back((int)(i / pc.nc));
        hc.w.push_back((float)pc.w[i]);
    }
    return PROP_OK;
}

int append_gather(const prop_s *h, const Slot &sl, int shot, const float *xyz, int npt, HostGather &hg)
{
    PointCorners pc;
    TRY(corners(h, sl, xyz, npt, 0.0, pc));
    hg.nc = pc.nc;
    for (int p = 0; p < npt; ++p) {
        hg.shot.push_back(shot);
        hg.pos.push_back(p);
        for (int c = 0; c < pc.nc; ++c) {
            hg.idx.push_back(pc.sidx[(size_t)p * pc.nc + c]);
            hg.w.push_back((float)pc.w[(size_t)p * pc.nc + c]);
        }
    }
    return PROP_OK;
}

struct Group {
    std::vector<Slot *> slots;
    std::vector<const prop_shot *> shots;
    DevBuf jobs_f, jobs_a, io;
    DevBuf pb[16];
    // tile lists per direction (0 forward, 1 adjoint) and pass, with their variant and z-chunk
    DevBuf tl[2][2];
    int ntl[2][2] = {}, shape[2][2] = {}, zc[2][2] = {};
    std::string key;                 // window set, for the autotuner
    BCsr src_inj{}, rec_inj{};
    BGather rec_gat{}, src_gat{};
    const float *const *src_data = nullptr;
    const int *nsrc = nullptr;
    const float *const *rec_data = nullptr;
    const int *nrec = nullptr;
    float *const *rec_out = nullptr;
    float *const *src_out = nullptr;
    // gradient storage offsets per shot
    std::vector<size_t> ck_off, sc_off, seg_off;
};

int upload_csr(prop_s *h, Group &G, int base, const HostCsr &hc, BCsr &c)
{
    std::vector<int> ptr = hc.ptr;
    ptr.push_back((int)hc.col.size());
    TRY(upload(G.pb[base + 0], hc.shot, h->st));
    TRY(upload(G.pb[base + 1], hc.node, h->st));
    TRY(upload(G.pb[base + 2], hc.mnode, h->st));
    TRY(upload(G.pb[base + 3], hc.e, h->st));
    TRY(upload(G.pb[base + 4], ptr, h->st));
    TRY(upload(G.pb[base + 5], hc.col, h->st));
    TRY(upload(G.pb[base + 6], hc.w, h->st));
    c = BCsr{(int)hc.node.size(), G.pb[base].as<int>(), G.pb[base + 1].as<int64_t>(), G.pb[base + 2].as<int64_t>(),
             G.pb[base + 3].as<float>(), G.pb[base + 4].as<int>(), G.pb[base + 5].as<int>(), G.pb[base + 6].as<float>()};
    return PROP_OK;
}

// z-chunk of a pass over a set of windows: one value for the group (each job clips it to its own
// depth), from the total tile count of one plane.
int group_zc(const prop_s *h, const std::vector<Slot *> &slots, int pass, int shape)
{
    const int TY = tile_rows(h, pass, shape);
    int64_t txy = 0;
    int nzmax = 1;
    for (auto *sl : slots) {
        txy += (int64_t)((sl->w.nx + PROP_TX - 1) / PROP_TX) * ((sl->w.ny + TY - 1) / TY);
        nzmax = std::max(nzmax, sl->w.nz);
    }
    return choose_zc(h, nzmax, txy);
}

// Untuned choice: the fixed tile variants, one z-chunk for both passes (from pass 1's tiles).
prop_s::Tune default_tune(const prop_s *h, const std::vector<Slot *> &slots)
{
    prop_s::Tune t;
    t.shape[0] = h->opt_shape[0];
    t.shape[1] = h->opt_shape[1];
    t.zc[0] = t.zc[1] = group_zc(h, slots, 1, t.shape[0]);
    if (h->opt_zc2 > 0) {
        int nzmax = 1;
        for (auto *sl : slots) nzmax = std::max(nzmax, sl->w.nz);
        t.zc[1] = std::min(h->opt_zc2, nzmax);
    }
    return t;
}

int apply_tune(prop_s *h, Group &G, int dir, const prop_s::Tune &t)
{
    std::vector<Tile> tl;
    for (int k = 0; k < 2; ++k) {
        make_tiles(G.slots, tile_rows(h, k + 1, t.shape[k]), t.zc[k], h->opt_xcd, tl);
        G.ntl[dir][k] = (int)tl.size();
        G.shape[dir][k] = t.shape[k];
        G.zc[dir][k] = t.zc[k];
        TRY(upload(G.tl[dir][k], tl, h->st));
    }
    h->last_tune = t;
    return PROP_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Autotuner: on the first call for a window set and direction, time every tile variant of each
// pass at three z-chunk lengths (half, one and two times the automatic one).  The untuned choice
// comes first and a candidate replaces the current pick only when it is at least 3 % faster, so
// that near-ties (within run-to-run noise) resolve the same way every time.  The trial launches
// run on the group's zero state, which they leave zero (no sources yet), so they change no result;
// the choice is cached on the handle.
int tune_group(prop_s *h, Group &G, bool adj)
{
    if (!h->opt_autotune) return PROP_OK;
    const int dir = adj ? 1 : 0;
    const std::string key = std::string(adj ? "A" : "F") + std::to_string(h->opt_scheme) + G.key;
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) return apply_tune(h, G, dir, it->second);
    const prop_s::Tune dflt = default_tune(h, G.slots);
    prop_s::Tune best = dflt;
    int nzmax = 1;
    for (auto *sl : G.slots) nzmax = std::max(nzmax, sl->w.nz);
    EventPair ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    const TTIJob *job = adj ? G.jobs_a.as<TTIJob>() : G.jobs_f.as<TTIJob>();
    const float idt2 = (float)(1.0 / (h->g.dt * h->g.dt));
    DevBuf tb;
    std::vector<Tile> tl;
    for (int pass = h->opt_scheme == TTI_FUSED ? 2 : 1; pass <= 2; ++pass) {
        std::vector<std::pair<int, int>> cand{{dflt.shape[pass - 1], dflt.zc[pass - 1]}};
        for (int shape = h->opt_scheme == TTI_SPLIT ? 1 : 0; shape < 2; ++shape) {
            const int z0 = group_zc(h, G.slots, pass, shape);
            for (int zc : {std::max(1, z0 / 2), z0, 2 * z0}) {
                const std::pair<int, int> c{shape, std::min(zc, nzmax)};
                if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
            }
        }
        // each candidate is timed in three rounds (after one warm-up launch each) and keeps its
        // fastest round, so that clock ramps and one-off stalls do not decide
        std::vector<double> cms(cand.size(), 1e300);
        for (int round = 0; round < 4; ++round)
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                const int shape = cand[ci].first, zc = cand[ci].second;
                make_tiles(G.slots, tile_rows(h, pass, shape), zc, h->opt_xcd, tl);
                TRY(upload(tb, tl, h->st));
                const int nt = (int)tl.size();
                auto run = [&]() {
                    if (pass == 1)
                        launch_tti_pass1(h->R, h->opt_scheme, shape, adj, job, tb.as<Tile>(), nt, zc, 0, h->W, h->st);
                    else
                        launch_tti_pass2(h->R, h->opt_scheme, shape, adj ? K2_ADJ : K2_FWD, job, tb.as<Tile>(), nt,
                                         zc, 0, h->W, idt2, 0, h->st);
                };
                if (round == 0) {
                    run();
                    continue;
                }
                HIPCHK(hipEventRecord(ev.a, h->st));
                for (int r = 0; r < 3; ++r) run();
                HIPCHK(hipEventRecord(ev.b, h->st));
                HIPCHK(hipEventSynchronize(ev.b));
                HIPCHK(hipGetLastError());
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
                cms[ci] = std::min(cms[ci], (double)ms);
            }
        double best_ms = 1e300;
        for (size_t ci = 0; ci < cand.size(); ++ci)
            if (cms[ci] < 0.97 * best_ms) {
                best_ms = cms[ci];
                best.shape[pass - 1] = cand[ci].first;
                best.zc[pass - 1] = cand[ci].second;
            }
    }
    h->tuned[key] = best;
    return apply_tune(h, G, dir, best);
}

// A run of time steps recorded into a HIP graph (graph option on, kernel timing off) and launched
// on the handle's stream when the run ends.  While recording, the handle's stream is an internal
// capture stream; nothing in a run synchronises with the host.  The executable graphs are freed
// at the next host synchronisation.
struct Capture {
    prop_s *h;
    hipStream_t orig = nullptr;
    bool on = false;
    explicit Capture(prop_s *h_) : h(h_) {}
    Capture(const Capture &) = delete;
    Capture &operator=(const Capture &) = delete;
    int begin()
    {
        if (!h->opt_graph || h->timing || on) return PROP_OK;
        if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        orig = h->st;
        h->st = h->cap;
        on = true;
        return PROP_OK;
    }
    int end()
    {
        if (!on) return PROP_OK;
        on = false;
        h->st = orig;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(h->cap, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(PROP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        h->execs.push_back(ex);
        HIPCHK(hipGraphLaunch(ex, h->st));
        h->graphs_launched++;
        return PROP_OK;
    }
    ~Capture()
    {
        if (!on) return;
        h->st = orig;
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(h->cap, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
    }
};

// Build a group over `shots` using workspaces `slots` (one per shot).  io pointer tables: wavelets,
// receiver-side inputs (rec_in / residual), receiver outputs, source outputs (each may be NULL).
int build_group(prop_s *h, Group &G, const std::vector<const prop_shot *> &shots, const std::vector<Slot *> &slots,
                bool src_inj, bool rec_gat, bool rec_inj, bool src_gat, const float *const *rec_in,
                float *const *rec_out, float *const *src_out)
{
    G.slots = slots;
    G.shots = shots;
    const int ns = (int)shots.size();
    HostCsr hs, hr;
    HostGather gr, gs;
    std::vector<TTIJob> jf, ja;
    G.key.clear();
    for (int j = 0; j < ns; ++j) {
        const prop_shot *s = shots[j];
        Slot &sl = *slots[j];
        if (!s) return fail(PROP_EINVAL, "shot %d is NULL", j);
        if (s->nsrc < 0 || s->nrec < 0) return fail(PROP_EINVAL, "negative point count");
        if (s->nsrc > 0 && (!s->src_xyz || (src_inj && !s->src_wavelet))) return fail(PROP_EINVAL, "source arrays NULL");
        if (s->nrec > 0 && !s->rec_xyz) return fail(PROP_EINVAL, "rec_xyz is NULL");
        if (s->nrec > 0 && rec_inj && (!rec_in || !rec_in[j])) return fail(PROP_EINVAL, "receiver input NULL");
        if (s->nrec > 0 && rec_gat && (!rec_out || !rec_out[j])) return fail(PROP_EINVAL, "rec_out is NULL");
        if (s->nsrc > 0 && src_gat && (!src_out || !src_out[j])) return fail(PROP_EINVAL, "src_out is NULL");
        int64_t o[3], n[3];
        TRY(shot_window(h, s, o, n));
        TRY(setup_slot(h, sl, o, n));
        sl.nsrc = s->nsrc;
        sl.nrec = s->nrec;
        if (src_inj && s->nsrc) TRY(append_csr(h, sl, j, s->src_xyz, s->nsrc, hs));
        if (rec_inj && s->nrec) TRY(append_csr(h, sl, j, s->rec_xyz, s->nrec, hr));
        if (rec_gat && s->nrec) TRY(append_gather(h, sl, j, s->rec_xyz, s->nrec, gr));
        if (src_gat && s->nsrc) TRY(append_gather(h, sl, j, s->src_xyz, s->nsrc, gs));
        jf.push_back(tti_job(h, sl, false));
        ja.push_back(tti_job(h, sl, true));
        G.key += std::to_string(sl.w.nx) + "x" + std::to_string(sl.w.ny) + "x" + std::to_string(sl.w.nz) + ";";
    }
    const prop_s::Tune t = default_tune(h, slots);
    TRY(apply_tune(h, G, 0, t));
    TRY(apply_tune(h, G, 1, t));
    TRY(upload(G.jobs_f, jf, h->st));
    TRY(upload(G.jobs_a, ja, h->st));
    G.src_inj = BCsr{};
    G.rec_inj = BCsr{};
    G.rec_gat = BGather{};
    G.src_gat = BGather{};
    if (!hs.node.empty()) TRY(upload_csr(h, G, 0, hs, G.src_inj));
    if (!hr.node.empty()) TRY(upload_csr(h, G, 7, hr, G.rec_inj));
    if (!gr.idx.empty()) {
        TRY(upload(G.pb[14], gr.idx, h->st));
        std::vector<char> packed;   // shot, pos, w packed in one buffer
        const size_t n = gr.shot.size();
        packed.resize(n * 8 + gr.w.size() * 4);
        std::memcpy(packed.data(), gr.shot.data(), n * 4);
        std::memcpy(packed.data() + n * 4, gr.pos.data(), n * 4);
        std::memcpy(packed.data() + n * 8, gr.w.data(), gr.w.size() * 4);
        TRY(upload(G.pb[15], packed, h->st));
        const char *b = G.pb[15].as<char>();
        G.rec_gat = BGather{(int)n, gr.nc, (const int *)b, G.pb[14].as<int64_t>(), (const float *)(b + n * 8),
                            (const int *)(b + n * 4)};
    }
    if (!gs.idx.empty()) {
        // few source points: keep them in the io buffer's tail
        G.src_gat.n = (int)gs.shot.size();
        G.src_gat.nc = gs.nc;
    }
    // io tables: pointers then counts
    std::vector<char> io(ns * 4 * sizeof(void *) + ns * 2 * sizeof(int) + gs.idx.size() * 8 + gs.shot.size() * 8 +
                         gs.w.size() * 4 + 64);
    char *p = io.data();
    std::vector<const void *> ptrs(4 * ns, nullptr);
    std::vector<int> cnt(2 * ns, 0);
    for (int j = 0; j < ns; ++j) {
        ptrs[j] = shots[j]->src_wavelet;
        ptrs[ns + j] = rec_in ? rec_in[j] : nullptr;
        ptrs[2 * ns + j] = rec_out ? rec_out[j] : nullptr;
        ptrs[3 * ns + j] = src_out ? src_out[j] : nullptr;
        cnt[j] = shots[j]->nsrc;
        cnt[ns + j] = shots[j]->nrec;
    }
    size_t off = 0;
    std::memcpy(p + off, ptrs.data(), ptrs.size() * sizeof(void *));
    off += ptrs.size() * sizeof(void *);
    const size_t cnt_off = off;
    std::memcpy(p + off, cnt.data(), cnt.size() * sizeof(int));
    off += cnt.size() * sizeof(int);
    off = (off + 7) / 8 * 8;
    const size_t gi_off = off;
    std::memcpy(p + off, gs.idx.data(), gs.idx.size() * 8);
    off += gs.idx.size() * 8;
    const size_t gsh_off = off;
    std::memcpy(p + off, gs.shot.data(), gs.shot.size() * 4);
    off += gs.shot.size() * 4;
    const size_t gp_off = off;
    std::memcpy(p + off, gs.pos.data(), gs.pos.size() * 4);
    off += gs.pos.size() * 4;
    const size_t gw_off = off;
    std::memcpy(p + off, gs.w.data(), gs.w.size() * 4);
    off += gs.w.size() * 4;
    io.resize(std::max<size_t>(off, 16));
    TRY(upload(G.io, io, h->st));
    const char *d = G.io.as<char>();
    G.src_data = (const float *const *)d;
    G.rec_data = (const float *const *)(d + ns * sizeof(void *));
    G.rec_out = (float *const *)(d + 2 * ns * sizeof(void *));
    G.src_out = (float *const *)(d + 3 * ns * sizeof(void *));
    G.nsrc = (const int *)(d + cnt_off);
    G.nrec = (const int *)(d + cnt_off + ns * sizeof(int));
    if (G.src_gat.n)
        G.src_gat = BGather{G.src_gat.n, gs.nc, (const int *)(d + gsh_off), (const int64_t *)(d + gi_off),
                            (const float *)(d + gw_off), (const int *)(d + gp_off)};
    return PROP_OK;
}

void tti_step(prop_s *h, Group &G, bool adj, int mode, int par, int seg_step)
{
    const TTIJob *job = adj ? G.jobs_a.as<TTIJob>() : G.jobs_f.as<TTIJob>();
    const int d = adj ? 1 : 0;
    if (h->opt_scheme != TTI_FUSED) {
        Timed t(h, 0);
        launch_tti_pass1(h->R, h->opt_scheme, G.shape[d][0], adj, job, G.tl[d][0].as<Tile>(), G.ntl[d][0], G.zc[d][0],
                         par, h->W,
                         h->st);
    }
    {
        Timed t(h, 1);
        launch_tti_pass2(h->R, h->opt_scheme, G.shape[d][1], mode, job, G.tl[d][1].as<Tile>(), G.ntl[d][1],
                         G.zc[d][1], par, h->W,
                         (float)(1.0 / (h->g.dt * h->g.dt)), seg_step, h->st);
    }
}

int check_group(prop_s *h, Group &G, int field, const char *what, int step)
{
    HIPCHK(hipGetLastError());
    for (size_t j = 0; j < G.slots.size(); ++j) TRY(check_finite(h, G.slots[j]->f[field], G.slots[j]->w, what, step, (int)j));
    return PROP_OK;
}

float idt2_of(const prop_s *h) { return (float)(1.0 / (h->g.dt * h->g.dt)); }

int tti_forward_group(prop_s *h, Group &G)
{
    for (auto *sl : G.slots) aux_fill(sl->f[0], 4 * sl->plane, 0.f, h->st);
    TRY(tune_group(h, G, false));
    const TTIJob *jf = G.jobs_f.as<TTIJob>();
    const int N = h->g.nt;
    Capture cap(h);
    TRY(cap.begin());
    for (int n = 0; n < N; ++n) {
        const int par = n & 1;
        tti_step(h, G, false, K2_FWD, par, 0);
        aux_tti_src(G.src_inj, jf, par, G.src_data, G.nsrc, n, idt2_of(h), -1, h->st);
        aux_tti_gather(G.rec_gat, jf, par, 0, G.rec_out, G.nrec, n, h->st);
        if ((n + 1) % WATCH_EVERY == 0 || n + 1 == N) {
            TRY(cap.end());
            TRY(check_group(h, G, par ^ 1, "p (forward)", n));
            if (n + 1 < N) TRY(cap.begin());
        }
    }
    return PROP_OK;
}

int tti_adjoint_group(prop_s *h, Group &G)
{
    for (auto *sl : G.slots) aux_fill(sl->f[11], 8 * sl->plane, 0.f, h->st);   // y and w (both levels)
    TRY(tune_group(h, G, true));
    const TTIJob *ja = G.jobs_a.as<TTIJob>();
    const int N = h->g.nt;
    Capture cap(h);
    TRY(cap.begin());
    for (int k = N; k >= 1; --k) {
        const int par = (N - k) & 1;
        tti_step(h, G, true, K2_ADJ, par, 0);
        aux_tti_rec_adj(G.rec_inj, ja, par, G.rec_data, G.nrec, k - 1, idt2_of(h), 0, 0, h->st);
        aux_tti_gather(G.src_gat, ja, par, 1, G.src_out, G.nsrc, k - 1, h->st);
        if ((N - k + 1) % WATCH_EVERY == 0 || k == 1) {
            TRY(cap.end());
            TRY(check_group(h, G, 11 + (par ^ 1), "y_p (adjoint)", k));
            if (k > 1) TRY(cap.begin());
        }
    }
    return PROP_OK;
}

// Checkpoint j of one shot holds (f^c, f^{c-1}) of p and q.  FP32: plain copies.  FP16/BF16: per
// field the current level and the level difference, each with per-x-row power-of-two scales.
void ckpt_save(prop_s *h, Slot &sl, char *ck, float *sc, int j, int par_new, int dtype)
{
    const size_t bpf = (size_t)sl.w.nx * sl.w.ny * sl.w.nz * (dtype == 0 ? 4 : 2);
    const int64_t nr = (int64_t)sl.w.ny * sl.w.nz;   // scales per field: one per x-row
    char *base = ck + (size_t)j * 4 * bpf;
    float *scl = sc + (size_t)j * 4 * nr;
    const float *cur[2] = {sl.f[par_new], sl.f[2 + par_new]};
    const float *prv[2] = {sl.f[par_new ^ 1], sl.f[2 + (par_new ^ 1)]};
    for (int i = 0; i < 2; ++i) {
        char *a = base + (size_t)(2 * i) * bpf, *b = a + bpf;
        if (dtype == 0) {
            aux_encode_win(cur[i], sl.w, nullptr, 0, a, scl + (2 * i) * nr, h->st);
            aux_encode_win(prv[i], sl.w, nullptr, 0, b, scl + (2 * i + 1) * nr, h->st);
        } else {
            aux_ckpt_pair_encode(cur[i], prv[i], sl.w, dtype, (uint16_t *)a, (uint16_t *)b, scl + (2 * i) * nr,
                                 scl + (2 * i + 1) * nr, h->st);
        }
    }
}

void ckpt_load(prop_s *h, Slot &sl, const char *ck, const float *sc, int j, int par_cur, int dtype)
{
    const size_t bpf = (size_t)sl.w.nx * sl.w.ny * sl.w.nz * (dtype == 0 ? 4 : 2);
    const int64_t nr = (int64_t)sl.w.ny * sl.w.nz;
    const char *base = ck + (size_t)j * 4 * bpf;
    const float *scl = sc + (size_t)j * 4 * nr;
    float *cur[2] = {sl.f[par_cur], sl.f[2 + par_cur]};
    float *prv[2] = {sl.f[par_cur ^ 1], sl.f[2 + (par_cur ^ 1)]};
    for (int i = 0; i < 2; ++i) {
        const char *a = base + (size_t)(2 * i) * bpf, *b = a + bpf;
        if (dtype == 0) {
            aux_decode_win(a, scl, sl.w, 0, cur[i], h->st);
            aux_decode_win(b, scl, sl.w, 0, prv[i], h->st);
        } else {
            aux_ckpt_pair_decode((const uint16_t *)a, (const uint16_t *)b, scl + (2 * i) * nr, scl + (2 * i + 1) * nr,
                                 sl.w, dtype, cur[i], prv[i], h->st);
        }
    }
}

// Device bytes of one shot's gradient workspace beyond its wavefields (checkpoints, scales, segment).
// Segment store of one shot: S steps of (p, q); FP32 in state layout, or 16-bit codes (dense) plus
// one FP32 scale per x-row, in the checkpoint type.
size_t seg_bytes(const Slot &sl, int S, int dtype)
{
    const size_t pts = (size_t)sl.w.nx * sl.w.ny * sl.w.nz, rows = (size_t)sl.w.ny * sl.w.nz;
    if (dtype == 0) return (size_t)S * 2 * sl.plane * 4;
    return ((size_t)S * 2 * pts * 2 + 255) / 256 * 256 + (size_t)S * 2 * rows * 4;
}

size_t grad_bytes(const Slot &sl, int C, int S, int dtype)
{
    const size_t pts = (size_t)sl.w.nx * sl.w.ny * sl.w.nz;
    const size_t ck = C > 1 ? (size_t)C * 4 * pts * (dtype == 0 ? 4 : 2) + (size_t)C * 4 * sl.w.ny * sl.w.nz * 4 : 0;
    return ck + seg_bytes(sl, S, C > 1 ? 0 : dtype) + 1024;
}

// Checkpointed gradient (or zero-lag image) of a group, in three parts: the plan (segment length,
// checkpoint count, workspaces, job tables), the forward sweep that stores the checkpoints (or, with
// a single segment, the whole run) and the reverse sweep.  A saving prop_forward runs the first two
// (gathering traces as it goes); a gradient reusing them runs the plan and the reverse sweep.
struct GradPlan {
    int N = 0, S = 0, C = 0, sdt = 0, dtype = 0;
    std::vector<TTIJob> jf;          // host copies of the forward job table (segment-store pointers)
};

int tti_grad_setup(prop_s *h, Group &G, int n_ckpt, int dtype, bool image, bool grow_only, GradPlan &P)
{
    const int N = h->g.nt;
    const int S = (N + n_ckpt - 1) / n_ckpt;      // segment length
    const int C = (N + S - 1) / S;                // checkpoints used (c_j = j S < N)
    const int ns = (int)G.slots.size();
    size_t ck_total = 0, sc_total = 0, seg_total = 0;
    const int Cs = C > 1 ? C : 0;                 // no checkpoint is stored when one segment covers all
    // segment store: FP32 between checkpoints (it costs the same bytes as a 16-bit store that is
    // encoded after each step, and keeps f^k exact); in the checkpoint type when one segment holds
    // the whole run (the memory then matters)
    const int sdt = C > 1 ? 0 : dtype;
    P.N = N;
    P.S = S;
    P.C = C;
    P.sdt = sdt;
    P.dtype = dtype;
    G.ck_off.assign(ns, 0);
    G.sc_off.assign(ns, 0);
    G.seg_off.assign(ns, 0);
    for (int j = 0; j < ns; ++j) {
        const Slot &sl = *G.slots[j];
        const size_t pts = (size_t)sl.w.nx * sl.w.ny * sl.w.nz;
        G.ck_off[j] = ck_total;
        ck_total += ((size_t)Cs * 4 * pts * (dtype == 0 ? 4 : 2) + 255) / 256 * 256;
        G.sc_off[j] = sc_total;
        sc_total += (size_t)Cs * 4 * sl.w.ny * sl.w.nz;
        G.seg_off[j] = seg_total;
        seg_total += (seg_bytes(sl, S, sdt) + 255) / 256 * 256;
    }
    // a batched call keeps its workspaces at the largest group's size (no re-allocation per group)
    auto want = [&](DevBuf &b, size_t n) { return grow_only ? b.ensure(n) : b.fit(n); };
    TRY(want(h->ckpt, std::max<size_t>(ck_total, 16)));
    TRY(want(h->ckscale, std::max<size_t>(sc_total * sizeof(float), 16)));
    TRY(want(h->seg, std::max<size_t>(seg_total, 16)));
    std::vector<TTIJob> ja;
    P.jf.clear();
    for (int j = 0; j < ns; ++j) {
        const Slot &sl = *G.slots[j];
        TTIJob a = tti_job(h, sl, false), b = tti_job(h, sl, true);
        char *base = h->seg.as<char>() + G.seg_off[j];
        for (TTIJob *J : {&a, &b}) {
            J->seg_dtype = sdt;
            if (sdt == 0) {
                J->seg = (float *)base;
            } else {
                const size_t pts = (size_t)sl.w.nx * sl.w.ny * sl.w.nz;
                J->seg16 = (uint16_t *)base;
                J->segsc = (float *)(base + ((size_t)S * 2 * pts * 2 + 255) / 256 * 256);
                J->seg16_field = (int64_t)pts;
                J->segsc_field = (int64_t)sl.w.ny * sl.w.nz;
            }
        }
        b.image = image ? 1 : 0;
        P.jf.push_back(a);
        ja.push_back(b);
    }
    TRY(upload(G.jobs_f, P.jf, h->st));
    TRY(upload(G.jobs_a, ja, h->st));
    return PROP_OK;
}

// Forward steps [start, end) of the segment that starts at `start`, storing each new level in the
// segment store (FP32: written by the update pass, the source added in place; 16-bit: encoded once
// the step, with its source, is complete); traces are gathered when the group has receiver plans.
void tti_seg_forward(prop_s *h, Group &G, const GradPlan &P, int start, int end)
{
    const TTIJob *djf = G.jobs_f.as<TTIJob>();
    const float idt2 = idt2_of(h);
    const int ns = (int)G.slots.size();
    for (int n = start; n < end; ++n) {
        const int par = n & 1;
        if (P.sdt == 0) {
            tti_step(h, G, false, K2_FWD_STORE, par, n - start);
            aux_tti_src(G.src_inj, djf, par, G.src_data, G.nsrc, n, idt2, n - start, h->st);
        } else {
            tti_step(h, G, false, K2_FWD, par, 0);
            aux_tti_src(G.src_inj, djf, par, G.src_data, G.nsrc, n, idt2, -1, h->st);
            for (int i = 0; i < ns; ++i) {
                const TTIJob &J = P.jf[i];
                const Slot &sl = *G.slots[i];
                const int64_t k = n - start;
                aux_encode_rows2(sl.f[par ^ 1], sl.f[2 + (par ^ 1)], sl.w, P.sdt, J.seg16 + k * 2 * J.seg16_field,
                                 J.seg16 + (k * 2 + 1) * J.seg16_field, J.segsc + k * 2 * J.segsc_field,
                                 J.segsc + (k * 2 + 1) * J.segsc_field, h->st);
            }
        }
        aux_tti_gather(G.rec_gat, djf, par, 0, G.rec_out, G.nrec, n, h->st);
    }
}

// The forward sweep: checkpoints at c_j = j S (j >= 1; c_0 = 0 is the zero state), or with a single
// segment the whole run in the segment store.
int tti_grad_forward(prop_s *h, Group &G, const GradPlan &P)
{
    const int N = P.N, S = P.S, C = P.C, ns = (int)G.slots.size();
    const TTIJob *djf = G.jobs_f.as<TTIJob>();
    const float idt2 = idt2_of(h);
    char *ck = h->ckpt.as<char>();
    float *sc = h->ckscale.as<float>();
    for (auto *sl : G.slots) aux_fill(sl->f[0], 4 * sl->plane, 0.f, h->st);
    TRY(tune_group(h, G, false));
    Capture cap(h);
    if (C == 1) {
        TRY(cap.begin());
        tti_seg_forward(h, G, P, 0, N);
        TRY(cap.end());
        return check_group(h, G, N & 1, "p (forward with storage)", N - 1);
    }
    TRY(cap.begin());
    for (int n = 0; n < N; ++n) {
        const int par = n & 1;
        tti_step(h, G, false, K2_FWD, par, 0);
        aux_tti_src(G.src_inj, djf, par, G.src_data, G.nsrc, n, idt2, -1, h->st);
        aux_tti_gather(G.rec_gat, djf, par, 0, G.rec_out, G.nrec, n, h->st);
        if ((n + 1) % S == 0 && (n + 1) / S < C)
            for (int j = 0; j < ns; ++j)
                ckpt_save(h, *G.slots[j], ck + G.ck_off[j], sc + G.sc_off[j], (n + 1) / S, par ^ 1, P.dtype);
        if ((n + 1) % WATCH_EVERY == 0 || n + 1 == N) {
            TRY(cap.end());
            TRY(check_group(h, G, par ^ 1, "p (forward with checkpoints)", n));
            if (n + 1 < N) TRY(cap.begin());
        }
    }
    return PROP_OK;
}

// The reverse sweep over segments: restore, recompute and store, then the adjoint steps with the
// imaging condition.  Each shot's window result is left in its slot (field 10).  With a single
// segment the forward sweep has already stored the whole run.
int tti_grad_reverse(prop_s *h, Group &G, const GradPlan &P)
{
    const int N = P.N, S = P.S, C = P.C, ns = (int)G.slots.size();
    const TTIJob *dja = G.jobs_a.as<TTIJob>();
    const float idt2 = idt2_of(h);
    char *ck = h->ckpt.as<char>();
    float *sc = h->ckscale.as<float>();
    for (auto *sl : G.slots) {
        aux_fill(sl->f[10], sl->plane, 0.f, h->st);          // gradient accumulator
        aux_fill(sl->f[11], 8 * sl->plane, 0.f, h->st);      // adjoint state and w (both levels)
    }
    if (C > 1) {   // the recomputation uses the forward tiles (the tuner's trials run on a zero state)
        for (auto *sl : G.slots) aux_fill(sl->f[0], 4 * sl->plane, 0.f, h->st);
        TRY(tune_group(h, G, false));
    }
    TRY(tune_group(h, G, true));
    Capture cap(h);
    for (int j = C - 1; j >= 0; --j) {
        const int start = j * S, end = std::min(N, (j + 1) * S);
        const int par0 = start & 1;
        TRY(cap.begin());
        if (C > 1) {
            for (int i = 0; i < ns; ++i) {
                Slot &sl = *G.slots[i];
                if (j == 0) aux_fill(sl.f[0], 4 * sl.plane, 0.f, h->st);
                else ckpt_load(h, sl, ck + G.ck_off[i], sc + G.sc_off[i], j, par0, P.dtype);
            }
            tti_seg_forward(h, G, P, start, end);
        }
        for (int k = end; k > start; --k) {
            const int par = (N - k) & 1;
            tti_step(h, G, true, K2_ADJ_IC, par, k - 1 - start);
            aux_tti_rec_adj(G.rec_inj, dja, par, G.rec_data, G.nrec, k - 1, idt2, 1, k - 1 - start, h->st);
        }
        TRY(cap.end());
        for (int i = 0; i < ns; ++i) {
            if (C > 1) TRY(check_finite(h, G.slots[i]->f[par0], G.slots[i]->w, "restored p", start, i));
            TRY(check_finite(h, G.slots[i]->f[11 + (((N - start - 1) & 1) ^ 1)], G.slots[i]->w, "y_p", start, i));
        }
        TRY(check_group(h, G, 10, "gradient", start));
    }
    return PROP_OK;
}

int tti_gradient_group(prop_s *h, Group &G, int n_ckpt, int dtype, bool image = false, bool grow_only = false)
{
    GradPlan P;
    TRY(tti_grad_setup(h, G, n_ckpt, dtype, image, grow_only, P));
    TRY(tti_grad_forward(h, G, P));
    return tti_grad_reverse(h, G, P);
}

// Checkpoints left by a saving prop_forward: valid for the shot and model they were made with.
bool saved_matches(const prop_s *h, const prop_shot *s, int n_ckpt, int dtype)
{
    const auto &sv = h->saved;
    if (!sv.valid || !s) return false;
    if (n_ckpt != 0 && (n_ckpt != sv.n_ckpt || dtype != sv.dtype)) return false;
    int64_t o[3], n[3];
    if (shot_window(h, s, o, n) != PROP_OK) {
        g_err.clear();
        return false;
    }
    for (int a = 0; a < 3; ++a)
        if (o[a] != sv.o[a] || n[a] != sv.n[a]) return false;
    if (s->nsrc != sv.nsrc || s->src_wavelet != sv.wav) return false;
    const size_t nv = (size_t)std::max(0, s->nsrc) * h->g.ndim;
    return nv == sv.src.size() && (nv == 0 || std::memcmp(s->src_xyz, sv.src.data(), nv * sizeof(float)) == 0);
}

void record_saved(prop_s *h, const prop_shot *s, int n_ckpt, int dtype)
{
    auto &sv = h->saved;
    int64_t o[3], n[3];
    if (shot_window(h, s, o, n) != PROP_OK) {
        sv.valid = false;
        return;
    }
    for (int a = 0; a < 3; ++a) sv.o[a] = o[a], sv.n[a] = n[a];
    sv.nsrc = s->nsrc;
    sv.wav = s->src_wavelet;
    const size_t nv = (size_t)std::max(0, s->nsrc) * h->g.ndim;
    sv.src.assign(s->src_xyz, s->src_xyz + nv);
    sv.n_ckpt = n_ckpt;
    sv.dtype = dtype;
    sv.valid = true;
}

int tti_forward(prop_s *h, const prop_shot *s, float *rec_out, int save, int dtype)
{
    Group G;
    float *outs[1] = {rec_out};
    if (save == 0) {
        TRY(build_group(h, G, {s}, {&h->slot}, true, true, false, false, nullptr, outs, nullptr));
        TRY(tti_forward_group(h, G));
        h->last_state = 1;
        return PROP_OK;
    }
    if (save < 0) return fail(PROP_EINVAL, "save_ckpt must be >= 0");
    if (dtype < 0 || dtype > 2) return fail(PROP_EINVAL, "unknown checkpoint dtype");
    h->saved.valid = false;
    TRY(build_group(h, G, {s}, {&h->slot}, true, true, false, false, nullptr, outs, nullptr));
    GradPlan P;
    TRY(tti_grad_setup(h, G, save, dtype, false, false, P));
    TRY(tti_grad_forward(h, G, P));
    record_saved(h, s, save, dtype);
    h->last_state = 1;
    return PROP_OK;
}

int tti_adjoint(prop_s *h, const prop_shot *s, const float *rec_in, float *src_out)
{
    Group G;
    const float *ins[1] = {rec_in};
    float *outs[1] = {src_out};
    TRY(build_group(h, G, {s}, {&h->slot}, false, false, true, true, ins, nullptr, outs));
    TRY(tti_adjoint_group(h, G));
    h->last_state = 2;
    return PROP_OK;
}

int tti_gradient(prop_s *h, const prop_shot *s, const float *residual, float *grad_m, int n_ckpt, int dtype,
                 bool image = false)
{
    if (n_ckpt < 0) return fail(PROP_EINVAL, "n_ckpt must be >= 0");
    if (dtype < 0 || dtype > 2) return fail(PROP_EINVAL, "unknown checkpoint dtype");
    if (!grad_m) return fail(PROP_EINVAL, image ? "image is NULL" : "grad_m is NULL");
    const bool reuse = saved_matches(h, s, n_ckpt, dtype);
    if (n_ckpt == 0 && !reuse)
        return fail(PROP_ESTATE, "no valid checkpoints of this shot on the handle (none saved by prop_forward, "
                                 "or invalidated since)");
    if (reuse) {
        n_ckpt = h->saved.n_ckpt;
        dtype = h->saved.dtype;
    } else {
        h->saved.valid = false;   // this call stores checkpoints of its own
    }
    Group G;
    const float *ins[1] = {residual};
    TRY(build_group(h, G, {s}, {&h->slot}, true, false, true, false, ins, nullptr, nullptr));
    GradPlan P;
    TRY(tti_grad_setup(h, G, n_ckpt, dtype, image, false, P));
    if (!reuse) TRY(tti_grad_forward(h, G, P));
    TRY(tti_grad_reverse(h, G, P));
    aux_copy_out(h->slot.f[10], h->slot.w, grad_m, h->st);
    HIPCHK(hipGetLastError());
    h->last_state = 0;
    return PROP_OK;
}

// Shots per group: greedy in shot order within a budget of the free device memory.
int plan_groups(prop_s *h, int nshot, const prop_shot *shots, bool grad, int n_ckpt, int dtype,
                std::vector<std::pair<int, int>> &groups)
{
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const int64_t budget_env = h->opt_batch_mb;
    // memory already held by the batch workspaces is reusable
    size_t held = h->ckpt.bytes + h->ckscale.bytes + h->seg.bytes;
    for (auto &sl : h->bslots) held += sl->fields.bytes;
    size_t budget = budget_env > 0 ? (size_t)budget_env << 20 : (size_t)((freeb + held) * 0.85);
    const int N = h->g.nt;
    const int S = (N + std::max(1, n_ckpt) - 1) / std::max(1, n_ckpt);
    const int C = (N + S - 1) / S;
    groups.clear();
    int start = 0;
    size_t used = 0;
    for (int i = 0; i < nshot; ++i) {
        int64_t o[3], n[3];
        TRY(shot_window(h, &shots[i], o, n));
        const size_t sx = (n[0] + 63) / 64 * 64, plane = sx * n[1] * n[2];
        size_t need = 19 * plane * 4 + 4096;
        if (grad) {
            Slot tmp;
            tmp.w.nx = (int)n[0];
            tmp.w.ny = (int)n[1];
            tmp.w.nz = (int)n[2];
            tmp.plane = plane;
            need += grad_bytes(tmp, C, S, dtype);
        }
        if (i > start && used + need > budget) {
            groups.push_back({start, i});
            start = i;
            used = 0;
        }
        used += need;
    }
    if (nshot > start) groups.push_back({start, nshot});
    return PROP_OK;
}

int tti_batched(prop_s *h, int nshot, const prop_shot *shots, float *const *rec_out, const float *const *residual,
                double *grad_global, int n_ckpt, int dtype, bool grad, bool image = false)
{
    if (nshot < 1 || !shots) return fail(PROP_EINVAL, "need at least one shot");
    if (grad) {
        if (n_ckpt < 1) return fail(PROP_EINVAL, "n_ckpt must be >= 1");
        if (dtype < 0 || dtype > 2) return fail(PROP_EINVAL, "unknown checkpoint dtype");
        if (!grad_global) return fail(PROP_EINVAL, "grad_global is NULL");
        if (!residual) return fail(PROP_EINVAL, "residual is NULL");
    } else if (!rec_out) {
        return fail(PROP_EINVAL, "rec_out is NULL");
    }
    std::vector<std::pair<int, int>> groups;
    TRY(plan_groups(h, nshot, shots, grad, n_ckpt, dtype, groups));
    h->last_groups = (int)groups.size();
    if (grad) {   // the planner counted these as reusable: give them back before the groups grow them
        h->saved.valid = false;
        h->ckpt.release();
        h->ckscale.release();
        h->seg.release();
    }
    for (auto &gr : groups) {
        const int ns = gr.second - gr.first;
        while ((int)h->bslots.size() < ns) h->bslots.emplace_back(new Slot());
        std::vector<const prop_shot *> sh;
        std::vector<Slot *> sl;
        for (int i = 0; i < ns; ++i) {
            sh.push_back(&shots[gr.first + i]);
            sl.push_back(h->bslots[i].get());
        }
        Group G;
        if (grad) {
            TRY(build_group(h, G, sh, sl, true, false, true, false, residual + gr.first, nullptr, nullptr));
            TRY(tti_gradient_group(h, G, n_ckpt, dtype, image, true));
            for (int i = 0; i < ns; ++i) aux_accum_f64(sl[i]->f[10], sl[i]->w, grad_global, h->st);  // shot order
        } else {
            TRY(build_group(h, G, sh, sl, true, true, false, false, nullptr, rec_out + gr.first, nullptr));
            TRY(tti_forward_group(h, G));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->st));   // group buffers are reused by the next group
    }
    h->last_state = 0;
    return PROP_OK;
}

// -------------------------------------------------------------------------- elastic time loops
// The normal stresses that the explosive source and the pressure receivers act on: txx, tyy, tzz in
// 3D; txx, tzz in 2D, where the stress tensor is 2 x 2 (tyy is then not part of it).
float *tyy_of(const prop_s *h, const Slot &sl) { return h->g.ndim == 3 ? sl.f[4] : nullptr; }

// Free surface by the method of images: the surface node row (0: none).
int image_row(const prop_s *h) { return h->kind == PROP_ELASTIC && h->g.free_surface == 2 ? h->g.nbl : 0; }

// The forward fill of the image rows on a set of nine fields (v, then tau).
void image_fill(prop_s *h, const Slot &sl, float *const *F)
{
    if (const int ks = image_row(h))
        aux_el_image_fill(sl.w, ks, F[3], F[4], F[5], F[7], h->g.ndim == 3 ? F[8] : nullptr, h->st);
}

// Its transpose on the slot's adjoint stresses, then sigma = C (g tau~) of the rows it touched.
void image_fold(prop_s *h, const Slot &sl)
{
    const int ks = image_row(h);
    if (!ks) return;
    ElImage J{};
    for (int i = 0; i < 6; ++i) {
        J.t[i] = sl.f[3 + i];
        J.s[i] = sl.f[9 + i];
    }
    J.lam = h->c[0];
    J.mu = h->c[1];
    const float *tab = sl.tabs.as<float>();
    J.gx = tab;
    J.gy = tab + sl.w.nx;
    J.gz = tab + sl.w.nx + sl.w.ny;
    aux_el_image_fold(sl.w, ks, h->g.ndim, J, h->st);
}

// The fused velocity-stress step (one launch a step, double-buffered state) applies to 3D windows
// up to space order 2 * el_fused_max_radius(); the two-pass step serves the rest.
bool el_fused_on(const prop_s *h)
{
    return h->kind == PROP_ELASTIC && h->g.ndim == 3 && h->R <= el_fused_max_radius() && h->opt_el_fused;
}

// z-chunks of the fused step: it recomputes v+ on 2R planes beyond each chunk and holds one block
// per CU, so the chunk count trades that recomputation against whole waves of blocks.
int choose_zc_ef(const prop_s *h, int nz, int64_t txy)
{
    if (h->opt_zc > 0) return std::min(h->opt_zc, nz);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    const int maxch = std::max(1, nz / (4 * h->R));
    double best = -1.0;
    int bz = nz;
    for (int nch = 1; nch <= maxch; ++nch) {
        const int zc = (nz + nch - 1) / nch;
        const int64_t nb = txy * ((nz + zc - 1) / zc);
        const double fill = (double)nb / (double)(((nb + ncu - 1) / ncu) * ncu);
        const double len = (double)nz / (double)((nz + zc - 1) / zc);
        const double eff = fill * len / (len + 2.0 * h->R);
        if (eff > best + 1e-9) {
            best = eff;
            bz = zc;
        }
    }
    return bz;
}

// Tiles and the two jobs of the fused step: job k reads buffer set k (fields 9k .. 9k+8 of the
// slot: v, then tau) and writes set k ^ 1.
int el_fused_setup(prop_s *h, Slot &sl)
{
    const Win &w = sl.w;
    const int64_t txy = (int64_t)((w.nx + EF_TX - 1) / EF_TX) * ((w.ny + EF_TY - 1) / EF_TY);
    sl.zc_ef = choose_zc_ef(h, w.nz, txy);
    std::vector<Slot *> one{&sl};
    std::vector<Tile> tiles;
    make_tiles(one, EF_TY, sl.zc_ef, h->opt_xcd, tiles, EF_TX);
    sl.ntiles_ef = (int)tiles.size();
    TRY(upload(sl.tiles_ef, tiles, h->st));
    std::vector<ElFusedJob> jobs(2);
    const float *tab = sl.tabs.as<float>();
    for (int k = 0; k < 2; ++k) {
        ElFusedJob &J = jobs[k];
        J.w = w;
        for (int i = 0; i < 3; ++i) {
            J.vi[i] = sl.f[9 * k + i];
            J.vo[i] = sl.f[9 * (k ^ 1) + i];
        }
        for (int i = 0; i < 6; ++i) {
            J.ti[i] = sl.f[9 * k + 3 + i];
            J.to[i] = sl.f[9 * (k ^ 1) + 3 + i];
        }
        J.lam = h->c[0];
        J.mu = h->c[1];
        J.b = h->c[2];
        J.gx = tab;
        J.gy = tab + w.nx;
        J.gz = tab + w.nx + w.ny;
    }
    return upload(sl.job_ef, jobs, h->st);
}

// One forward step: the velocity pass with `job`, the stress pass with `job_stress` (the same job
// for a step in place; another where the velocity pass writes v+ elsewhere).
void el_step_fwd(prop_s *h, Slot &sl, const ElJob *job, const ElJob *job_stress = nullptr)
{
    const float dt = (float)h->g.dt;
    {
        Timed t(h, 2);
        launch_el_vel(h->R, tile_rows(h, 1, h->opt_shape[0]), EL_FWD, job, sl.tiles.as<Tile>(), sl.ntiles, sl.zc, h->W, dt, h->st);
    }
    {
        Timed t(h, 3);
        launch_el_stress(h->R, tile_rows(h, 2, h->opt_shape[1]), EL_FWD, job_stress ? job_stress : job,
                         sl.tiles2.as<Tile>(), sl.ntiles2, sl.zc2, h->W, dt, h->st);
    }
}

// After the adjoint receiver injection into tau~ (the diagonal at the pressure nodes): sigma there,
// which the stress pass of the previous adjoint step formed from tau~ before the injection.
void el_remix(prop_s *h, Slot &sl)
{
    if (!sl.rec_inj.csr.nrows) return;
    const float *tab = sl.tabs.as<float>();
    aux_el_remix(sl.rec_inj.csr, sl.w, tab, tab + sl.w.nx, tab + sl.w.nx + sl.w.ny, h->c[0], h->c[1], sl.f[3], sl.f[4],
                 sl.f[5], sl.f[9], sl.f[10], sl.f[11], h->st);
}

int el_forward(prop_s *h, const prop_shot *s, float *rec_out, int save, int dtype)
{
    if (save < 0) return fail(PROP_EINVAL, "save_ckpt must be >= 0");
    if (save > 0 && dtype != PROP_CKPT_F32) return fail(PROP_EINVAL, "elastic checkpoints are FP32");
    Slot &sl = h->slot;
    TRY(prepare_shot(h, sl, s, true, true, false, false));
    if (s->nsrc > 0 && !s->src_wavelet) return fail(PROP_EINVAL, "src_wavelet is NULL");
    if (s->nrec > 0 && !rec_out) return fail(PROP_EINVAL, "rec_out is NULL");
    // a saving run keeps the state after steps j S (j = 1 .. C-1), the checkpoints of el_gradient
    const int N = h->g.nt;
    const int S = save > 0 ? (N + save - 1) / save : N + 1;
    const int C = save > 0 ? (N + S - 1) / S : 1;
    const size_t P = sl.plane;
    if (save > 0) {
        h->saved.valid = false;
        TRY(h->ckpt.fit(std::max<size_t>((size_t)(C - 1) * 9 * P * sizeof(float), 16)));
    }
    aux_fill(sl.f[0], 9 * sl.plane, 0.f, h->st);
    const ElJob *job = sl.job_fwd.as<ElJob>();
    const bool fused = el_fused_on(h);
    if (fused) TRY(el_fused_setup(h, sl));
    const float dt = (float)h->g.dt;
    for (int n = 0; n < N; ++n) {
        // the state after the step: buffer set 0 (fields 0-8), or with the fused step set (n + 1) & 1
        const int cur = fused ? (n + 1) & 1 : 0;
        float *const *F = sl.f + 9 * cur;
        if (fused) {
            Timed t(h, 4);
            launch_el_fused(h->R, sl.job_ef.as<ElFusedJob>() + (n & 1), sl.tiles_ef.as<Tile>(), sl.ntiles_ef,
                            sl.zc_ef, h->W, dt, h->st);
        } else {
            el_step_fwd(h, sl, job);
        }
        float *tyy = h->g.ndim == 3 ? F[4] : nullptr;
        if (s->nsrc) aux_el_inject(sl.src_inj.csr, s->src_wavelet + (size_t)n * s->nsrc, dt, F[3], tyy, F[5], h->st);
        image_fill(h, sl, F);
        float *row = s->nrec ? rec_out + (size_t)n * s->nrec : nullptr;
        if (sl.rec_gat.gat.n) aux_gather(sl.rec_gat.gat, F[3], tyy, F[5], 1.f, row, h->st);
        if (sl.rec_gat_vz.gat.n) aux_gather(sl.rec_gat_vz.gat, F[2], nullptr, nullptr, 1.f, row, h->st);
        if (save > 0 && (n + 1) % S == 0 && (n + 1) / S < C)
            HIPCHK(hipMemcpyAsync(h->ckpt.as<float>() + (size_t)((n + 1) / S - 1) * 9 * P, F[0],
                                  9 * P * sizeof(float), hipMemcpyDeviceToDevice, h->st));
        if ((n + 1) % WATCH_EVERY == 0 || n + 1 == N) {
            HIPCHK(hipGetLastError());
            TRY(check_finite(h, F[5], sl.w));
        }
    }
    // the final state where every later call looks for it: buffer set 0
    if (fused && (N & 1))
        HIPCHK(hipMemcpyAsync(sl.f[0], sl.f[9], 9 * P * sizeof(float), hipMemcpyDeviceToDevice, h->st));
    if (save > 0) record_saved(h, s, save, dtype);
    h->last_state = 1;
    return PROP_OK;
}

int el_adjoint(prop_s *h, const prop_shot *s, const float *rec_in, float *src_out)
{
    Slot &sl = h->slot;
    TRY(prepare_shot(h, sl, s, false, false, true, true));
    if (s->nrec > 0 && !rec_in) return fail(PROP_EINVAL, "rec_in is NULL");
    if (s->nsrc > 0 && !src_out) return fail(PROP_EINVAL, "src_out is NULL");
    aux_fill(sl.f[0], 18 * sl.plane, 0.f, h->st);
    const ElJob *job = sl.job_fwd.as<ElJob>();
    const float dt = (float)h->g.dt;
    for (int n = h->g.nt - 1; n >= 0; --n) {
        const float *row = s->nrec ? rec_in + (size_t)n * s->nrec : nullptr;
        if (sl.rec_inj.csr.nrows) aux_el_inject(sl.rec_inj.csr, row, 1.f, sl.f[3], tyy_of(h, sl), sl.f[5], h->st);
        if (sl.rec_inj_vz.csr.nrows) aux_el_inject(sl.rec_inj_vz.csr, row, 1.f, sl.f[2], nullptr, nullptr, h->st);
        el_remix(h, sl);
        image_fold(h, sl);
        if (s->nsrc) aux_gather(sl.src_gat.gat, sl.f[3], tyy_of(h, sl), sl.f[5], dt, src_out + (size_t)n * s->nsrc,
                                h->st);
        {
            Timed t(h, 2);
            launch_el_vel(h->R, tile_rows(h, 1, h->opt_shape[0]), EL_ADJ, job, sl.tiles.as<Tile>(), sl.ntiles, sl.zc, h->W, dt, h->st);
        }
        {
            Timed t(h, 3);
            launch_el_stress(h->R, tile_rows(h, 2, h->opt_shape[1]), EL_ADJ, job, sl.tiles2.as<Tile>(), sl.ntiles2, sl.zc2, h->W, dt, h->st);
        }
        if ((h->g.nt - n) % WATCH_EVERY == 0 || n == 0) {
            HIPCHK(hipGetLastError());
            TRY(check_finite(h, sl.f[5], sl.w));
        }
    }
    h->last_state = 2;
    return PROP_OK;
}

// Elastic gradient with respect to (vp, vs, rho): forward run with C = ceil(N/S) checkpoints of the
// nine fields (FP32), then segment by segment in reverse: restore, recompute the segment storing
// the velocities of every level, and run the adjoint steps with the imaging condition between the
// transposed velocity and stress updates.  out: three dense window fields (vp, vs, rho).
int el_gradient(prop_s *h, const prop_shot *s, const float *residual, float *out, int n_ckpt, int dtype)
{
    if (n_ckpt < 0) return fail(PROP_EINVAL, "n_ckpt must be >= 0");
    if (n_ckpt > 0 && dtype != PROP_CKPT_F32) return fail(PROP_EINVAL, "elastic gradients keep FP32 checkpoints");
    if (!out) return fail(PROP_EINVAL, "grad_m is NULL");
    const bool reuse = saved_matches(h, s, n_ckpt, dtype);
    if (n_ckpt == 0 && !reuse)
        return fail(PROP_ESTATE, "no valid checkpoints of this shot on the handle (none saved by prop_forward, "
                                 "or invalidated since)");
    if (reuse) n_ckpt = h->saved.n_ckpt;
    else h->saved.valid = false;   // this call stores checkpoints of its own
    Slot &sl = h->slot;
    TRY(prepare_shot(h, sl, s, true, false, true, false));
    if (s->nsrc > 0 && !s->src_wavelet) return fail(PROP_EINVAL, "src_wavelet is NULL");
    if (s->nrec > 0 && !residual) return fail(PROP_EINVAL, "residual is NULL");
    const int N = h->g.nt;
    const int S = (N + n_ckpt - 1) / n_ckpt;
    const int C = (N + S - 1) / S;
    const size_t P = sl.plane;
    // forward fields (9) + accumulators (8) + checkpoints (9 per stored checkpoint) + velocity store
    TRY(h->elfwd.ensure((size_t)9 * P * sizeof(float)));
    TRY(h->elacc.ensure((size_t)8 * P * sizeof(float)));
    TRY(h->ckpt.fit(std::max<size_t>((size_t)(C - 1) * 9 * P * sizeof(float), 16)));
    TRY(h->seg.fit((size_t)(S + 1) * 3 * P * sizeof(float)));
    float *fw = h->elfwd.as<float>(), *acc = h->elacc.as<float>(), *ck = h->ckpt.as<float>();
    float *vs_ = h->seg.as<float>();
    // 2D velocity passes never store v_y (it stays zero), so the store's v_y planes are cleared here
    if (h->g.ndim == 2) aux_fill(vs_, (size_t)(S + 1) * 3 * P, 0.f, h->st);
    ElJob jf = el_job(h, sl);
    for (int i = 0; i < 3; ++i) jf.v[i] = jf.vo[i] = fw + (size_t)i * P;
    for (int i = 0; i < 6; ++i) jf.t[i] = fw + (size_t)(3 + i) * P;
    // job 0: a step in place (checkpoint sweep); jobs 1 + 2k, 2 + 2k: step k of a segment's recompute,
    // whose velocity pass reads v from store slot k and writes v+ into slot k + 1, where the stress
    // pass reads it (the stresses stay in place)
    std::vector<ElJob> jfs(1 + 2 * (size_t)S, jf);
    for (int k = 0; k < S; ++k)
        for (int i = 0; i < 3; ++i) {
            float *const a = vs_ + ((size_t)k * 3 + i) * P, *const b = vs_ + ((size_t)(k + 1) * 3 + i) * P;
            jfs[1 + 2 * k].v[i] = a;
            jfs[1 + 2 * k].vo[i] = b;
            jfs[2 + 2 * k].v[i] = jfs[2 + 2 * k].vo[i] = b;
        }
    TRY(upload(h->eljob_f, jfs, h->st));
    const ElJob *djf = h->eljob_f.as<ElJob>();
    const ElJob *dja = sl.job_fwd.as<ElJob>();   // adjoint fields: the slot's own
    ElGradJob gj{};
    gj.w = sl.w;
    for (int i = 0; i < 6; ++i) gj.tt[i] = sl.f[3 + i];
    for (int i = 0; i < 3; ++i) gj.vt[i] = sl.f[i];
    gj.b = h->c[2];
    const float *tab = sl.tabs.as<float>();
    gj.gx = tab;
    gj.gy = tab + sl.w.nx;
    gj.gz = tab + sl.w.nx + sl.w.ny;
    for (int i = 0; i < 8; ++i) gj.acc[i] = acc + (size_t)i * P;
    std::vector<ElGradJob> gjs(S);   // one job per segment step (which stored levels it reads)
    for (int k = 0; k < S; ++k) {
        gjs[k] = gj;
        for (int i = 0; i < 3; ++i) {
            gjs[k].vn0[i] = vs_ + ((size_t)k * 3 + i) * P;
            gjs[k].vn1[i] = vs_ + ((size_t)(k + 1) * 3 + i) * P;
        }
    }
    TRY(upload(h->eljob_g, gjs, h->st));
    const ElGradJob *dgj = h->eljob_g.as<ElGradJob>();
    const float dt = (float)h->g.dt;
    float *const fwf[9] = {jf.v[0], jf.v[1], jf.v[2], jf.t[0], jf.t[1], jf.t[2], jf.t[3], jf.t[4], jf.t[5]};
    // forward step n; k >= 0: step k of a segment's recompute, v+ into store slot k + 1
    auto fwd_step = [&](int n, int k) {
        if (k < 0) el_step_fwd(h, sl, djf);
        else el_step_fwd(h, sl, djf + 1 + 2 * k, djf + 2 + 2 * k);
        if (s->nsrc) aux_el_inject(sl.src_inj.csr, s->src_wavelet + (size_t)n * s->nsrc, dt, jf.t[0],
                                   h->g.ndim == 3 ? jf.t[1] : nullptr, jf.t[2], h->st);
        image_fill(h, sl, fwf);
    };
    auto copy = [&](float *dst, const float *src, size_t nflt) -> int {
        HIPCHK(hipMemcpyAsync(dst, src, nflt * sizeof(float), hipMemcpyDeviceToDevice, h->st));
        return PROP_OK;
    };
    // 1) forward with checkpoints (state after step jS, j >= 1), unless a saving forward left them
    aux_fill(fw, 9 * P, 0.f, h->st);
    for (int n = 0; n < (C > 1 && !reuse ? N : 0); ++n) {
        fwd_step(n, -1);
        if ((n + 1) % S == 0 && (n + 1) / S < C) TRY(copy(ck + (size_t)((n + 1) / S - 1) * 9 * P, fw, 9 * P));
        if ((n + 1) % WATCH_EVERY == 0) {
            HIPCHK(hipGetLastError());
            TRY(check_finite(h, jf.t[2], sl.w, "tau_zz (gradient forward)", n));
        }
    }
    // 2) reverse sweep
    aux_fill(sl.f[0], 18 * P, 0.f, h->st);
    aux_fill(acc, 8 * P, 0.f, h->st);
    for (int j = C - 1; j >= 0; --j) {
        const int start = j * S, end = std::min(N, (j + 1) * S);
        if (j == 0) aux_fill(fw, 9 * P, 0.f, h->st);
        else TRY(copy(fw, ck + (size_t)(j - 1) * 9 * P, 9 * P));
        TRY(copy(vs_, fw, 3 * P));
        for (int n = start; n < end; ++n) fwd_step(n, n - start);
        for (int n = end - 1; n >= start; --n) {
            const float *row = s->nrec ? residual + (size_t)n * s->nrec : nullptr;
            if (sl.rec_inj.csr.nrows) aux_el_inject(sl.rec_inj.csr, row, 1.f, sl.f[3], tyy_of(h, sl), sl.f[5], h->st);
            if (sl.rec_inj_vz.csr.nrows) aux_el_inject(sl.rec_inj_vz.csr, row, 1.f, sl.f[2], nullptr, nullptr, h->st);
            el_remix(h, sl);
            image_fold(h, sl);
            {
                Timed t(h, 2);
                launch_el_vel(h->R, tile_rows(h, 1, h->opt_shape[0]), EL_ADJ, dja, sl.tiles.as<Tile>(), sl.ntiles, sl.zc, h->W, dt, h->st);
            }
            launch_el_grad_ic(h->R, tile_rows(h, 2, h->opt_shape[1]), dgj + (n - start), sl.tiles2.as<Tile>(), sl.ntiles2, sl.zc2, h->W,
                              dt, h->st);
            {
                Timed t(h, 3);
                launch_el_stress(h->R, tile_rows(h, 2, h->opt_shape[1]), EL_ADJ, dja, sl.tiles2.as<Tile>(), sl.ntiles2, sl.zc2, h->W, dt,
                                 h->st);
            }
        }
        HIPCHK(hipGetLastError());
        TRY(check_finite(h, sl.f[5], sl.w, "adjoint tau_zz (gradient)", start));
    }
    launch_el_grad_finish(dgj, sl.w, h->g.ndim, h->g.free_surface ? h->g.nbl : 0, image_row(h), h->model.p[0],
                          h->model.p[1], h->model.p[2], out, h->st);
    HIPCHK(hipGetLastError());
    TRY(check_finite(h, acc, sl.w, "gradient accumulator", 0));
    h->last_state = 0;
    return PROP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Allocation-free FP64 dot product.  Its scratch (the partial sums of the dot kernels' fixed grid
// and the result) is a file-scope device array; every device holds its own copy, whose device
// address is looked up once per device, with that device current, and kept.
// ---------------------------------------------------------------------------------------------
constexpr int NOALLOC_DOT_SCRATCH = 1024 + 1;    // doubles
static __device__ __align__(256) double scratch[NOALLOC_DOT_SCRATCH];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[MAX_DEVICES] = {};

// Device address of this device's scratch array (the host-side symbol is only a stand-in).
int scratch_ptr(double **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PROP_EINVAL, "device %d beyond the %d supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return PROP_OK;
}
}  // namespace

// ============================================================================ C ABI
extern "C" {

const char *prop_last_error(void) { return g_err.c_str(); }

double prop_cfl_dt(prop_kind kind, const prop_grid *grid, double vmax, double eps_max)
{
    prop_grid g;
    if (!grid) return -1.0;
    g = *grid;
    if (g.dt <= 0) g.dt = 1;   // not needed for the bound
    if (g.nt < 1) g.nt = 1;
    if (check_grid(kind, &g) != PROP_OK || !(vmax > 0)) return -1.0;
    return cfl_dt(kind, &g, vmax, eps_max);
}

int prop_create(prop_t *out, prop_kind kind, const prop_grid *grid, const prop_model *model, void *stream)
{
    g_err.clear();
    if (!out) return fail(PROP_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(check_grid(kind, grid));
    prop_s *h = new (std::nothrow) prop_s();
    if (!h) return fail(PROP_ENOMEM, "host allocation failed");
    h->kind = kind;
    h->g = *grid;
    h->st = (hipStream_t)stream;
    h->R = grid->space_order / 2;
    // elastic 3D grids: 64 x 8 tiles for the velocity pass (three blocks of 512 threads a CU; 400^3
    // so8: 0.74 against 0.87 ms), 64 x 16 for the stress pass and the imaging condition (stress:
    // 0.99 against 0.98-1.04 ms, and the velocity pass after a 64 x 8 stress pass ran slower)
    if (kind == PROP_ELASTIC) h->opt_shape[0] = 0;
    // default TTI scheme (512^3 workload, ms per step): space order 8 and below, the fused pass
    // (so8: 1.70 against 1.50 + 0.80 for the split pair and 2.94 for two passes); space orders 10-12,
    // the split pair of fused single-field passes (so12: 1.05 + 1.59 = 2.64 against 2.95 for the
    // four-field two-pass pair; the fused pass is register-bound there, 4.65); above, the six-field
    // two-pass pair (the others' queues outgrow the registers and LDS of a CU).
    if (kind == PROP_TTI)
        h->opt_scheme = h->R <= 4 && fused_fits(*grid) ? TTI_FUSED
                        : h->R <= 6 && fused_fits(*grid) ? TTI_SPLIT
                        : h->R <= 6 ? TTI_FOUR : TTI_SIX;
    double w[8] = {0};
    if (kind == PROP_TTI) centred_weights(h->R, w);
    else staggered_weights(h->R, w);
    for (int j = 0; j < 8; ++j) {
        h->W.wx[j] = (float)(w[j] / grid->spacing[0]);
        h->W.wy[j] = grid->ndim == 3 ? (float)(w[j] / grid->spacing[1]) : 0.f;
        h->W.wz[j] = (float)(w[j] / grid->spacing[2]);
    }
    int rc = h->flag.ensure(16 * sizeof(unsigned));
    if (rc == PROP_OK) rc = h->dotpart.ensure(aux_dot_blocks() * sizeof(double));
    if (rc == PROP_OK) rc = h->dotout.ensure(sizeof(double));
    if (rc == PROP_OK) rc = prep_model(h, model);
    if (rc != PROP_OK) {
        std::string msg = g_err;
        delete h;
        g_err = msg;
        return rc;
    }
    *out = h;
    return PROP_OK;
}

int prop_set_model(prop_t h, const prop_model *model)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    return prep_model(h, model);
}

int prop_forward(prop_t h, const prop_shot *shot, float *rec_out, int32_t save_ckpt, prop_ckpt_dtype ckpt_dtype)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    return h->kind == PROP_TTI ? tti_forward(h, shot, rec_out, save_ckpt, (int)ckpt_dtype)
                               : el_forward(h, shot, rec_out, save_ckpt, (int)ckpt_dtype);
}

int prop_adjoint(prop_t h, const prop_shot *shot, const float *rec_in, float *src_out)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    return h->kind == PROP_TTI ? tti_adjoint(h, shot, rec_in, src_out) : el_adjoint(h, shot, rec_in, src_out);
}

int prop_gradient(prop_t h, const prop_shot *shot, const float *residual, float *grad_m, int32_t n_ckpt,
                  prop_ckpt_dtype ckpt_dtype)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    if (h->kind == PROP_ELASTIC) return el_gradient(h, shot, residual, grad_m, n_ckpt, (int)ckpt_dtype);
    return tti_gradient(h, shot, residual, grad_m, n_ckpt, (int)ckpt_dtype);
}

int prop_image(prop_t h, const prop_shot *shot, const float *rec_in, float *image, int32_t n_ckpt,
               prop_ckpt_dtype ckpt_dtype)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    if (h->kind != PROP_TTI) return fail(PROP_EINVAL, "images are provided for PROP_TTI only");
    return tti_gradient(h, shot, rec_in, image, n_ckpt, (int)ckpt_dtype, true);
}

int prop_image_batched(prop_t h, int32_t nshot, const prop_shot *shots, const float *const *rec_in,
                       double *image_global, int32_t n_ckpt, prop_ckpt_dtype ckpt_dtype)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    if (h->kind != PROP_TTI) return fail(PROP_EINVAL, "batched calls are provided for PROP_TTI");
    return tti_batched(h, nshot, shots, nullptr, rec_in, image_global, n_ckpt, (int)ckpt_dtype, true, true);
}

int prop_forward_batched(prop_t h, int32_t nshot, const prop_shot *shots, float *const *rec_out)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    if (h->kind != PROP_TTI) return fail(PROP_EINVAL, "batched calls are provided for PROP_TTI");
    return tti_batched(h, nshot, shots, rec_out, nullptr, nullptr, 0, 0, false);
}

int prop_gradient_batched(prop_t h, int32_t nshot, const prop_shot *shots, const float *const *residual,
                          double *grad_global, int32_t n_ckpt, prop_ckpt_dtype ckpt_dtype)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    if (h->kind != PROP_TTI) return fail(PROP_EINVAL, "batched calls are provided for PROP_TTI");
    return tti_batched(h, nshot, shots, nullptr, residual, grad_global, n_ckpt, (int)ckpt_dtype, true);
}

int prop_read_state(prop_t h, int32_t field, float *out)
{
    g_err.clear();
    if (!h || !out) return fail(PROP_EINVAL, "NULL argument");
    if (h->last_state == 0) return fail(PROP_ESTATE, "no forward or adjoint result to read");
    const Slot &sl = h->slot;
    const float *src = nullptr;
    if (h->kind == PROP_TTI) {
        if (field < 0 || field > 3) return fail(PROP_EINVAL, "TTI state field must be 0..3");
        const int N = h->g.nt;
        if (h->last_state == 1) {
            const int cur = N & 1;   // f^N lives in buffer (N-1)&1 ^ 1 == N & 1
            const int idx[4] = {cur, 2 + cur, cur ^ 1, 2 + (cur ^ 1)};
            src = sl.f[idx[field]];
        } else {
            const int cur = N & 1;   // y^1 written at iteration N-1 into buffer ((N-1)&1)^1
            const int idx[4] = {11 + cur, 13 + cur, 11 + (cur ^ 1), 13 + (cur ^ 1)};
            src = sl.f[idx[field]];
        }
    } else {
        if (field < 0 || field > 8) return fail(PROP_EINVAL, "elastic state field must be 0..8");
        src = sl.f[field];
    }
    aux_copy_out(src, sl.w, out, h->st);
    HIPCHK(hipGetLastError());
    return PROP_OK;
}

int prop_set_timing(prop_t h, int32_t enable)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    TRY(fold_timing(h));
    h->timing = enable != 0;
    for (int k = 0; k < 5; ++k) h->ms[k] = 0, h->launches[k] = 0;
    return PROP_OK;
}

int prop_set_option(prop_t h, int32_t option, int64_t value)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    switch (option) {
    case PROP_OPT_GRAPH: h->opt_graph = value != 0; return PROP_OK;
    case PROP_OPT_AUTOTUNE: h->opt_autotune = value != 0; return PROP_OK;
    case PROP_OPT_TILE1:
    case PROP_OPT_TILE2:
        if (value != 0 && value != 1) return fail(PROP_EINVAL, "tile variant must be 0 or 1");
        h->opt_shape[option == PROP_OPT_TILE1 ? 0 : 1] = (int)value;
        return PROP_OK;
    case PROP_OPT_ZC:
        if (value < 0 || value > (1 << 20)) return fail(PROP_EINVAL, "z-chunk must be in [0, 2^20]");
        h->opt_zc = (int)value;
        return PROP_OK;
    case PROP_OPT_ZC2:
        if (value < 0 || value > (1 << 20)) return fail(PROP_EINVAL, "z-chunk must be in [0, 2^20]");
        h->opt_zc2 = (int)value;
        return PROP_OK;
    case PROP_OPT_XCD: h->opt_xcd = value != 0; return PROP_OK;
    case PROP_OPT_EL_FUSED: h->opt_el_fused = value != 0; return PROP_OK;
    case PROP_OPT_BATCH_MB:
        if (value < 0) return fail(PROP_EINVAL, "batch budget must be >= 0");
        h->opt_batch_mb = value;
        return PROP_OK;
    case PROP_OPT_SCHEME:
        if (value != TTI_SIX && value != TTI_FUSED && value != TTI_FOUR && value != TTI_SPLIT)
            return fail(PROP_EINVAL, "scheme must be 0, 2, 3 or 4");
        if (value == TTI_SPLIT && h->R > tti_split_max_radius())
            return fail(PROP_EINVAL, "the split scheme supports space orders up to %d", 2 * tti_split_max_radius());
        if (value == TTI_SPLIT && !fused_fits(h->g))
            return fail(PROP_EINVAL, "the split scheme needs x-y planes below 4 GiB");
        if (value == TTI_FUSED && h->R > tti_fused_max_radius())
            return fail(PROP_EINVAL, "the fused scheme supports space orders up to %d", 2 * tti_fused_max_radius());
        if (value == TTI_FUSED && !fused_fits(h->g))
            return fail(PROP_EINVAL, "the fused scheme needs x-y planes below 4 GiB");
        h->opt_scheme = (int)value;
        return PROP_OK;
    default: return fail(PROP_EINVAL, "option %d cannot be set", (int)option);
    }
}

int prop_get_option(prop_t h, int32_t option, int64_t *value)
{
    g_err.clear();
    if (!h || !value) return fail(PROP_EINVAL, "NULL argument");
    switch (option) {
    case PROP_OPT_GRAPH: *value = h->opt_graph; break;
    case PROP_OPT_AUTOTUNE: *value = h->opt_autotune; break;
    case PROP_OPT_TILE1: *value = h->opt_shape[0]; break;
    case PROP_OPT_TILE2: *value = h->opt_shape[1]; break;
    case PROP_OPT_ZC: *value = h->opt_zc; break;
    case PROP_OPT_ZC2: *value = h->opt_zc2; break;
    case PROP_OPT_XCD: *value = h->opt_xcd; break;
    case PROP_OPT_BATCH_MB: *value = h->opt_batch_mb; break;
    case PROP_OPT_EL_FUSED: *value = h->opt_el_fused; break;
    case PROP_OPT_SCHEME: *value = h->opt_scheme; break;
    case PROP_INFO_TILE1: *value = h->last_tune.shape[0]; break;
    case PROP_INFO_TILE2: *value = h->last_tune.shape[1]; break;
    case PROP_INFO_ZC1: *value = h->last_tune.zc[0]; break;
    case PROP_INFO_ZC2: *value = h->last_tune.zc[1]; break;
    case PROP_INFO_GRAPHS: *value = h->graphs_launched; break;
    case PROP_INFO_GROUPS: *value = h->last_groups; break;
    default: return fail(PROP_EINVAL, "unknown option %d", (int)option);
    }
    return PROP_OK;
}

int prop_kernel_time(prop_t h, int32_t kclass, double *ms, int64_t *launches, const char **name)
{
    g_err.clear();
    static const char *names[5] = {"tti_pass1 (gradient + axis projection)", "tti_pass2 (divergence + update)",
                                   "el_vel (velocity pass)", "el_stress (stress pass)",
                                   "el_fused (velocity + stress)"};
    if (!h || kclass < 0 || kclass > 4) return fail(PROP_EINVAL, "bad handle or kernel class");
    TRY(fold_timing(h));
    if (ms) *ms = h->ms[kclass];
    if (launches) *launches = h->launches[kclass];
    if (name) {
        *name = names[kclass];
        if (h->kind == PROP_TTI && h->opt_scheme == TTI_FUSED && kclass == 1) *name = "tti_fused (single pass)";
        if (h->kind == PROP_TTI && h->opt_scheme == TTI_SPLIT)
            *name = kclass == 0 ? "tti_split A (H0 u)" : kclass == 1 ? "tti_split B (Hz v + update)" : names[kclass];
    }
    return PROP_OK;
}

int prop_ckpt_encode(const float *f, int64_t n, prop_ckpt_dtype dtype, void *codes, float *scale_dev, void *stream)
{
    g_err.clear();
    if (!f || !codes || !scale_dev || n < 0) return fail(PROP_EINVAL, "bad codec argument");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PROP_CKPT_F32) {
        HIPCHK(hipMemcpyAsync(codes, f, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
        const float one = 1.0f;
        HIPCHK(hipMemcpyAsync(scale_dev, &one, 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return PROP_OK;
    }
    if (dtype != PROP_CKPT_F16 && dtype != PROP_CKPT_BF16) return fail(PROP_EINVAL, "unknown dtype");
    DevBuf mx;
    TRY(mx.ensure(sizeof(unsigned)));
    aux_fill_u32(mx.as<unsigned>(), 1, 0u, st);
    aux_absmax(f, n, mx.as<unsigned>(), st);
    aux_encode(f, n, mx.as<unsigned>(), (int)dtype, (uint16_t *)codes, scale_dev, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PROP_OK;
}

int prop_ckpt_decode(const void *codes, const float *scale_dev, int64_t n, prop_ckpt_dtype dtype, float *f,
                     void *stream)
{
    g_err.clear();
    if (!f || !codes || !scale_dev || n < 0) return fail(PROP_EINVAL, "bad codec argument");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PROP_CKPT_F32) {
        HIPCHK(hipMemcpyAsync(f, codes, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
        return PROP_OK;
    }
    if (dtype != PROP_CKPT_F16 && dtype != PROP_CKPT_BF16) return fail(PROP_EINVAL, "unknown dtype");
    aux_decode((const uint16_t *)codes, scale_dev, n, (int)dtype, f, st);
    HIPCHK(hipGetLastError());
    return PROP_OK;
}

// A dense (nz, ny, nx) array seen as a window (row pitch nx) for the row-codec kernels.
static int dense_win(int64_t nx, int64_t ny, int64_t nz, Win &w)
{
    if (nx < 1 || nx > 2147483647 || ny < 1 || ny > 65535 || nz < 1 || nz > 65535)
        return fail(PROP_EINVAL, "row codec needs 1 <= nx < 2^31 and 1 <= ny, nz <= 65535");
    w = Win{};
    w.nx = (int)nx;
    w.ny = (int)ny;
    w.nz = (int)nz;
    w.sx = nx;
    w.sy = nx * ny;
    w.mx = nx;
    w.my = nx * ny;
    w.moff = 0;
    return PROP_OK;
}

int prop_ckpt_encode_rows(const float *cur, const float *prev, int64_t nx, int64_t ny, int64_t nz, int32_t pair,
                          prop_ckpt_dtype dtype, uint16_t *codes_a, uint16_t *codes_b, float *scale_a, float *scale_b,
                          void *stream)
{
    g_err.clear();
    if (!cur || !prev || !codes_a || !codes_b || !scale_a || !scale_b) return fail(PROP_EINVAL, "NULL row-codec argument");
    if (dtype != PROP_CKPT_F16 && dtype != PROP_CKPT_BF16) return fail(PROP_EINVAL, "row codecs are FP16 or BF16");
    if (pair != 0 && pair != 1) return fail(PROP_EINVAL, "pair must be 0 or 1");
    Win w;
    TRY(dense_win(nx, ny, nz, w));
    hipStream_t st = (hipStream_t)stream;
    if (pair) aux_ckpt_pair_encode(cur, prev, w, (int)dtype, codes_a, codes_b, scale_a, scale_b, st);
    else aux_encode_rows2(cur, prev, w, (int)dtype, codes_a, codes_b, scale_a, scale_b, st);
    HIPCHK(hipGetLastError());
    return PROP_OK;
}

int prop_ckpt_decode_rows(const uint16_t *codes_a, const uint16_t *codes_b, const float *scale_a, const float *scale_b,
                          int64_t nx, int64_t ny, int64_t nz, prop_ckpt_dtype dtype, float *cur, float *prev,
                          void *stream)
{
    g_err.clear();
    if (!cur || !prev || !codes_a || !codes_b || !scale_a || !scale_b) return fail(PROP_EINVAL, "NULL row-codec argument");
    if (dtype != PROP_CKPT_F16 && dtype != PROP_CKPT_BF16) return fail(PROP_EINVAL, "row codecs are FP16 or BF16");
    Win w;
    TRY(dense_win(nx, ny, nz, w));
    aux_ckpt_pair_decode(codes_a, codes_b, scale_a, scale_b, w, (int)dtype, cur, prev, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return PROP_OK;
}

int prop_dot_f64(const float *a, const float *b, int64_t n, double *result, void *stream)
{
    g_err.clear();
    if (!a || !b || !result || n < 0) return fail(PROP_EINVAL, "bad dot argument");
    hipStream_t st = (hipStream_t)stream;
    DevBuf part, out;
    TRY(part.ensure(aux_dot_blocks() * sizeof(double)));
    TRY(out.ensure(sizeof(double)));
    aux_dot_f64(a, b, n, part.as<double>(), out.as<double>(), st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(result, out.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PROP_OK;
}

int prop_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *result, void *stream)
{
    g_err.clear();
    if (!a || !b || !result || n < 0) return fail(PROP_EINVAL, "bad dot argument");
    const int parts = aux_dot_blocks();
    if (parts + 1 > NOALLOC_DOT_SCRATCH)
        return fail(PROP_EINVAL, "the dot kernels need %d doubles of scratch, the static array holds %d", parts + 1,
                    NOALLOC_DOT_SCRATCH);
    double *s = nullptr;
    TRY(scratch_ptr(&s));
    hipStream_t st = (hipStream_t)stream;
    aux_dot_f64(a, b, n, s, s + parts, st);   // every partial sum and the result are written: nothing to clear
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(result, s + parts, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PROP_OK;
}

int prop_destroy(prop_t h)
{
    g_err.clear();
    if (!h) return fail(PROP_EINVAL, "handle is NULL");
    (void)hipStreamSynchronize(h->st);
    release_graphs(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (auto e : h->evpool) (void)hipEventDestroy(e);
    delete h;
    return PROP_OK;
}

}  // extern "C"
