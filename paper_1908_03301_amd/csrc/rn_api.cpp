// rn_api.cpp -- C ABI of librn: argument checks, device memory, launch
// sequencing and result assembly for the random-network flow solve.
//
// The iteration loop is device-driven: every pass kernel reads the next mode
// (CG step, FP64 refresh, done) written by the previous pass, so the host only
// enqueues launches in chunks and reads the control block between chunks.
#include "../../include/rn.h"
#include "rn_device.hpp"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

using namespace rn;

struct rn_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t own = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    Scalars *host_scal = nullptr;  // pinned [3]
    unsigned long long *host_cnt = nullptr;  // pinned [2]
    hipEvent_t ev_chunk[2] = {nullptr, nullptr};
    hipEvent_t ev_t[4] = {nullptr, nullptr, nullptr, nullptr};
    int tile_y = 16, tile_z = 16;
};

namespace {

const char *kStatusNames[] = {"ok", "invalid argument", "out of memory", "not converged",
                              "numerical breakdown", "device error", "not finished", "unknown ticket"};

#define RN_TRY(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
            return RN_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Shape checks shared by every entry point (no data access).
int check_shape(const rn_problem *p)
{
    if (!p) return RN_EINVAL;
    if (p->dim != 2 && p->dim != 3) return RN_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return RN_EINVAL;
    if (p->dim == 2 && p->nz != 1) return RN_EINVAL;
    if (p->axis < 0 || p->axis >= p->dim) return RN_EINVAL;
    const int64_t na = p->axis == 0 ? p->nx : (p->axis == 1 ? p->ny : p->nz);
    if (na < 2) return RN_EINVAL;
    if (p->nx > INT32_MAX || p->ny > INT32_MAX || p->nz > INT32_MAX) return RN_EINVAL;
    const double n = (double)p->nx * (double)p->ny * (double)p->nz;
    if (n >= 2147483647.0) return RN_EINVAL;
    if (p->mem != RN_MEM_HOST && p->mem != RN_MEM_DEVICE) return RN_EINVAL;
    if (p->reserved != 0) return RN_EINVAL;
    for (int k = 0; k < p->dim; ++k)
        if (!p->g[k]) return RN_EINVAL;
    if (p->dim == 2 && p->g[2]) return RN_EINVAL;
    return RN_OK;
}

int check_opts(const rn_opts *o)
{
    if (!o) return RN_EINVAL;
    if (o->precision != RN_FP64 && o->precision != RN_MIXED) return RN_EINVAL;
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return RN_EINVAL;
    if (o->max_iter < 0) return RN_EINVAL;
    if (!(o->delta >= 0.0) || o->delta >= 1.0) return RN_EINVAL;
    if (o->reserved != 0) return RN_EINVAL;
    return RN_OK;
}

// Host-memory conductances: finite and >= 0 on every in-lattice bond.
bool host_values_ok(const rn_problem *p)
{
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
    for (int k = 0; k < p->dim; ++k) {
        const double *g = p->g[k];
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y) {
                const double *row = g + nx * (y + ny * z);
                int64_t xe = nx;
                if (k == 0) xe = nx - 1;
                else if (k == 1 && y == ny - 1) xe = 0;
                else if (k == 2 && z == nz - 1) xe = 0;
                for (int64_t x = 0; x < xe; ++x) {
                    const double v = row[x];
                    if (!(v >= 0.0) || std::isinf(v)) return false;
                }
            }
    }
    return true;
}

struct Layout {
    int64_t n = 0;
    int dim = 2, s = 8;
    bool copy_g = false;
    int grid = 8, ntx = 1, nty = 1, ntz = 1, ntiles = 1, tile_y = 16, tile_z = 16;
    size_t off_g64 = 0, off_P = 0, off_dl = 0, off_mask = 0, off_gT = 0, off_invd = 0, off_vec = 0,
           off_part = 0, off_scal = 0, off_cnt = 0, total = 0;
};

Layout make_layout(const rn_problem *p, const rn_opts *o, int tile_y, int tile_z)
{
    Layout L;
    L.n = p->nx * p->ny * p->nz;
    L.dim = p->dim;
    L.s = (o && o->precision == RN_MIXED) ? 4 : 8;
    L.copy_g = p->mem == RN_MEM_HOST;
    L.tile_y = tile_y;
    L.tile_z = tile_z;
    if (p->dim == 2) {
        L.ntx = div_up((int)p->nx, kWave);
        L.nty = div_up((int)p->ny, L.s == 4 ? kTY2f : kTY2d);
        L.ntz = 1;
        L.ntiles = L.ntx * L.nty;
        L.grid = div_up(L.ntiles, kBlock / kWave);
    } else {
        L.ntx = div_up((int)p->nx, kTX);
        L.nty = div_up((int)p->ny, kTY);
        L.ntz = div_up((int)p->nz, tile_z);
        L.ntiles = L.ntx * L.nty * L.ntz;
        L.grid = L.ntiles;
    }
    L.grid = (L.grid + 7) / 8 * 8;
    const size_t n = (size_t)L.n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o_ = off;
        off += align256(bytes);
        return o_;
    };
    L.off_g64 = take(L.copy_g ? (size_t)8 * L.dim * n : 0);
    L.off_P = take(16 * n);
    L.off_dl = take(8 * n);
    L.off_mask = take(n);
    L.off_gT = take((size_t)L.s * L.dim * n);
    L.off_invd = take((size_t)L.s * n);
    L.off_vec = take((size_t)6 * L.s * n);   // two sets of r, p, q; labels (8 bytes/node) alias here
    L.off_part = take((size_t)L.grid * kRed * 8);
    L.off_scal = take(sizeof(Scalars));
    L.off_cnt = take(4 * sizeof(unsigned long long));
    L.total = off;
    return L;
}

int ensure_arena(rn_ctx *ctx, size_t bytes)
{
    if (bytes > ctx->budget) return RN_ENOMEM;
    if (ctx->arena_bytes >= bytes) return RN_OK;
    if (ctx->arena) {
        RN_TRY(hipStreamSynchronize(ctx->stream));
        RN_TRY(hipFree(ctx->arena));
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->arena, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        ctx->arena = nullptr;
        return RN_ENOMEM;
    }
    RN_TRY(e);
    ctx->arena_bytes = bytes;
    return RN_OK;
}

double ev_seconds(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

// Upload (or borrow) conductances, validate device-resident ones, build the
// mask, Jacobi scale and initial field. Fills *n_live.
int prepare(rn_ctx *ctx, const rn_problem *p, const Layout &L, const double *gd[3], int64_t *n_live,
            bool want_mask_buffer)
{
    char *base = (char *)ctx->arena;
    const size_t n = (size_t)L.n;
    Lat lat{p->dim, p->axis, (int)p->nx, (int)p->ny, (int)p->nz, L.n};
    unsigned long long *cnt = (unsigned long long *)(base + L.off_cnt);
    gd[0] = gd[1] = gd[2] = nullptr;
    if (L.copy_g) {
        for (int k = 0; k < p->dim; ++k) {
            double *dst = (double *)(base + L.off_g64) + (size_t)k * n;
            RN_TRY(hipMemcpyAsync(dst, p->g[k], 8 * n, hipMemcpyHostToDevice, ctx->stream));
            gd[k] = dst;
        }
    } else {
        for (int k = 0; k < p->dim; ++k) gd[k] = p->g[k];
    }
    RN_TRY(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), ctx->stream));
    if (!L.copy_g) {
        RN_TRY(launch_validate(lat, gd, cnt + 1, ctx->stream));
    }
    int *parent = (int *)(base + L.off_vec);
    unsigned *flags = (unsigned *)(base + L.off_vec + 4 * n);
    uint8_t *mask = want_mask_buffer ? (uint8_t *)(base + L.off_mask) : nullptr;
    double *dl = (double *)(base + L.off_dl);
    double *P0 = (double *)(base + L.off_P);
    RN_TRY(launch_mask(lat, gd, parent, flags, mask, dl, P0, cnt, ctx->stream));
    RN_TRY(hipMemcpyAsync(ctx->host_cnt, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
    RN_TRY(hipStreamSynchronize(ctx->stream));
    if (ctx->host_cnt[1] != 0) return RN_EINVAL;
    *n_live = (int64_t)ctx->host_cnt[0];
    return RN_OK;
}

int copy_out(rn_ctx *ctx, void *dst, const void *src, size_t bytes, int mem)
{
    RN_TRY(hipMemcpyAsync(dst, src, bytes, mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          ctx->stream));
    return RN_OK;
}

template <typename T>
int run_loop(rn_ctx *ctx, const rn_problem *p, const rn_opts *o, const Layout &L, const double *const gd[3],
             Scalars *hs)
{
    char *base = (char *)ctx->arena;
    const size_t n = (size_t)L.n;
    Lat lat{p->dim, p->axis, (int)p->nx, (int)p->ny, (int)p->nz, L.n};
    T *gT[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < p->dim; ++k) gT[k] = (T *)(base + L.off_gT) + (size_t)k * n;
    T *invd = (T *)(base + L.off_invd);
    T *vec = (T *)(base + L.off_vec);
    RN_TRY(launch_scale<T>(lat, gd, (const double *)(base + L.off_dl), gT, invd, vec, (int64_t)(6 * n),
                           ctx->stream));

    Scalars *ds = (Scalars *)(base + L.off_scal);
    Scalars init;
    std::memset(&init, 0, sizeof(init));
    init.mode = MODE_REFRESH;
    init.first = 1;
    init.fp32 = L.s == 4;
    init.max_iter = o->max_iter;
    init.sigma = 1.0;
    init.sigma_next = 1.0;
    init.tol = o->tol;
    init.delta = (L.s == 4) ? (o->delta > 0.0 ? o->delta : 0.1) : 0.0;
    init.kappa = 1.0;
    init.bhat = 1.0;
    init.last_check = INFINITY;
    ctx->host_scal[2] = init;
    RN_TRY(hipMemcpyAsync(ds, &ctx->host_scal[2], sizeof(Scalars), hipMemcpyHostToDevice, ctx->stream));

    PassArgs<T> a[2];
    for (int par = 0; par < 2; ++par) {
        PassArgs<T> &A = a[par];
        std::memset(&A, 0, sizeof(A));
        A.nx = (int)p->nx;
        A.ny = (int)p->ny;
        A.nz = (int)p->nz;
        A.axis = p->axis;
        A.ntx = L.ntx;
        A.nty = L.nty;
        A.ntz = L.ntz;
        A.tile_y = L.tile_y;
        A.tile_z = L.tile_z;
        A.ntiles = L.ntiles;
        A.grid = L.grid;
        for (int k = 0; k < 3; ++k) {
            A.g64[k] = gd[k];
            A.gT[k] = gT[k];
        }
        A.P[0] = (double *)(base + L.off_P);
        A.P[1] = A.P[0] + n;
        A.invd = invd;
        VecSet<T> s0{vec, vec + n, vec + 2 * n};
        VecSet<T> s1{vec + 3 * n, vec + 4 * n, vec + 5 * n};
        A.src = par == 0 ? s0 : s1;
        A.dst = par == 0 ? s1 : s0;
        A.partials = (double *)(base + L.off_part);
        A.s = ds;
    }

    RN_TRY(hipEventRecord(ctx->ev_t[2], ctx->stream));
    const int64_t hard_cap = 2 * o->max_iter + 256;
    int64_t launched = 0;
    int chunk = 16;
    int pending = -1, slot = 0;
    double prev_est = -1.0;
    int64_t prev_iters = 0;
    int last_chunk = 0;
    while (launched < hard_cap) {
        const int c = (int)std::min<int64_t>(chunk, hard_cap - launched);
        for (int i = 0; i < c; ++i) {
            RN_TRY(launch_pass<T>(p->dim, a[launched & 1], ctx->stream));
            ++launched;
        }
        RN_TRY(hipMemcpyAsync(&ctx->host_scal[slot], ds, sizeof(Scalars), hipMemcpyDeviceToHost, ctx->stream));
        RN_TRY(hipEventRecord(ctx->ev_chunk[slot], ctx->stream));
        if (pending >= 0) {
            RN_TRY(hipEventSynchronize(ctx->ev_chunk[pending]));
            const Scalars &h = ctx->host_scal[pending];
            if (h.mode == MODE_DONE) break;
            // size the next chunk from the observed convergence rate; the
            // chunk enqueued last is still in flight, and launches left over
            // after convergence are idle, so aim slightly short
            int next = std::min(chunk * 2, 256);
            if (prev_est > 0.0 && h.est_rel > 0.0 && h.est_rel < prev_est && h.iters > prev_iters) {
                const double rate = std::log(prev_est / h.est_rel) / (double)(h.iters - prev_iters);
                const double remain = std::log(std::max(h.est_rel / o->tol, 1.0)) / rate;
                const double want = 0.9 * remain - (double)last_chunk;
                next = (int)std::min(256.0, std::max(8.0, want));
            }
            prev_est = h.est_rel;
            prev_iters = h.iters;
            chunk = next;
        }
        last_chunk = c;
        pending = slot;
        slot ^= 1;
    }
    RN_TRY(hipEventRecord(ctx->ev_t[3], ctx->stream));
    RN_TRY(hipMemcpyAsync(hs, ds, sizeof(Scalars), hipMemcpyDeviceToHost, ctx->stream));
    RN_TRY(hipStreamSynchronize(ctx->stream));
    hs->passes = launched;   // report launches (the device counts only working passes)
    return RN_OK;
}

double cross_section(const rn_problem *p)
{
    double s = 1.0;
    const int64_t n[3] = {p->nx, p->ny, p->nz};
    for (int k = 0; k < p->dim; ++k)
        if (k != p->axis) s *= (double)n[k];
    return s;
}

}  // namespace

extern "C" {

int rn_version(void) { return 100; }

const char *rn_strerror(int status)
{
    if (status > 0 || status < -7) return "unknown status";
    return kStatusNames[-status];
}

int rn_opts_default(rn_opts *o)
{
    if (!o) return RN_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->precision = RN_FP64;
    o->tol = 1e-8;
    o->max_iter = 10000000;
    o->delta = 0.0;
    return RN_OK;
}

int rn_create(int device, size_t budget, rn_ctx **out)
{
    if (!out) return RN_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return RN_EDEVICE;
    if (device < 0 || device >= count) return RN_EINVAL;
    rn_ctx *ctx = new rn_ctx();
    ctx->device = device;
    auto fail = [&](hipError_t e) {
        (void)e;
        rn_destroy(ctx);
        return RN_EDEVICE;
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return fail(e);
    size_t free_b = 0, total_b = 0;
    if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return fail(e);
    ctx->budget = budget ? budget : (size_t)(0.9 * (double)free_b);
    if ((e = hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking)) != hipSuccess) return fail(e);
    ctx->stream = ctx->own;
    if ((e = hipHostMalloc((void **)&ctx->host_scal, 3 * sizeof(Scalars), hipHostMallocDefault)) != hipSuccess)
        return fail(e);
    if ((e = hipHostMalloc((void **)&ctx->host_cnt, 4 * sizeof(unsigned long long), hipHostMallocDefault)) !=
        hipSuccess)
        return fail(e);
    for (auto &ev : ctx->ev_chunk)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return fail(e);
    for (auto &ev : ctx->ev_t)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return fail(e);
    *out = ctx;
    return RN_OK;
}

int rn_destroy(rn_ctx *ctx)
{
    if (!ctx) return RN_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
    if (ctx->host_cnt) (void)hipHostFree(ctx->host_cnt);
    for (auto ev : ctx->ev_chunk)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->ev_t)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    delete ctx;
    return RN_OK;
}

int rn_set_stream(rn_ctx *ctx, void *stream)
{
    if (!ctx) return RN_EINVAL;
    ctx->stream = stream ? (hipStream_t)stream : ctx->own;
    return RN_OK;
}

const char *rn_last_error(rn_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int rn_validate(const rn_problem *p, const rn_opts *opts)
{
    int st = check_shape(p);
    if (st) return st;
    rn_opts o;
    if (opts) o = *opts;
    else rn_opts_default(&o);
    if ((st = check_opts(&o))) return st;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    return RN_OK;
}

size_t rn_footprint(const rn_problem *p, const rn_opts *o)
{
    if (check_shape(p) != RN_OK) return 0;
    rn_opts d;
    rn_opts_default(&d);
    return make_layout(p, o ? o : &d, 16, 16).total;
}

int rn_build_mask(rn_ctx *ctx, const rn_problem *p, int64_t *n_live_out)
{
    if (!ctx) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    if (!p->mask_out) return RN_EINVAL;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    RN_TRY(hipSetDevice(ctx->device));
    rn_opts o;
    rn_opts_default(&o);
    o.precision = RN_MIXED;   // smallest layout: the mask needs no FP64 CG state
    Layout L = make_layout(p, &o, ctx->tile_y, ctx->tile_z);
    if ((st = ensure_arena(ctx, L.total))) return st;
    const double *gd[3];
    int64_t n_live = 0;
    if ((st = prepare(ctx, p, L, gd, &n_live, true))) return st;
    if ((st = copy_out(ctx, p->mask_out, (char *)ctx->arena + L.off_mask, (size_t)L.n, p->mem))) return st;
    RN_TRY(hipStreamSynchronize(ctx->stream));
    if (n_live_out) *n_live_out = n_live;
    return RN_OK;
}

int rn_solve(rn_ctx *ctx, const rn_problem *p, const rn_opts *opts, rn_result *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !out) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    rn_opts o;
    if (opts) o = *opts;
    else rn_opts_default(&o);
    if ((st = check_opts(&o))) return st;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    RN_TRY(hipSetDevice(ctx->device));
    Layout L = make_layout(p, &o, ctx->tile_y, ctx->tile_z);
    if ((st = ensure_arena(ctx, L.total))) return st;

    RN_TRY(hipEventRecord(ctx->ev_t[0], ctx->stream));
    const double *gd[3];
    int64_t n_live = 0;
    if ((st = prepare(ctx, p, L, gd, &n_live, true))) return st;
    RN_TRY(hipEventRecord(ctx->ev_t[1], ctx->stream));

    rn_result r;
    std::memset(&r, 0, sizeof(r));
    r.n_live = n_live;
    char *base = (char *)ctx->arena;
    const double *P_final = (const double *)(base + L.off_P);
    const int64_t na = p->axis == 0 ? p->nx : (p->axis == 1 ? p->ny : p->nz);
    if (n_live == 0) {
        double G = 0.0;
        if (na == 2) {
            Lat lat{p->dim, p->axis, (int)p->nx, (int)p->ny, (int)p->nz, L.n};
            double *dG = (double *)(base + L.off_cnt) + 2;
            RN_TRY(launch_direct_flux(lat, gd[p->axis], dG, ctx->stream));
            RN_TRY(hipMemcpyAsync(&ctx->host_scal[2].Q_in, dG, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            RN_TRY(hipStreamSynchronize(ctx->stream));
            G = ctx->host_scal[2].Q_in;
        }
        r.status = RN_OK;
        r.converged = 1;
        r.Q_in = r.Q_out = r.G = G;
        r.K = G * (double)(na - 1) / cross_section(p);
        RN_TRY(hipEventRecord(ctx->ev_t[2], ctx->stream));
        RN_TRY(hipEventRecord(ctx->ev_t[3], ctx->stream));
    } else {
        Scalars hs;
        st = (L.s == 4) ? run_loop<float>(ctx, p, &o, L, gd, &hs) : run_loop<double>(ctx, p, &o, L, gd, &hs);
        if (st) return st;
        P_final = (const double *)(base + L.off_P) + (size_t)(hs.refreshes & 1) * (size_t)L.n;
        r.status = hs.status;
        r.converged = hs.converged;
        r.Q_in = hs.Q_in;
        r.Q_out = hs.Q_out;
        r.G = hs.Q_in - hs.xr;
        r.K = r.G * (double)(na - 1) / cross_section(p);
        r.rel_resid = hs.rel_resid;
        r.iters = hs.iters;
        r.refreshes = hs.refreshes;
        r.passes = hs.passes;
        if (r.status == 0 && !r.converged) r.status = RN_ENOCONV;
    }
    if (p->p_out && (st = copy_out(ctx, p->p_out, P_final, 8 * (size_t)L.n, p->mem))) return st;
    if (p->mask_out && (st = copy_out(ctx, p->mask_out, base + L.off_mask, (size_t)L.n, p->mem))) return st;
    RN_TRY(hipStreamSynchronize(ctx->stream));
    r.t_mask_s = ev_seconds(ctx->ev_t[0], ctx->ev_t[1]);
    r.t_loop_s = ev_seconds(ctx->ev_t[2], ctx->ev_t[3]);
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = r;
    return r.status;
}

}  // extern "C"
