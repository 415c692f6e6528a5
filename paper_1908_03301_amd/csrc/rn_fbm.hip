// rn_fbm.hip -- correlated conductance fields on the GPU (Sec. II, Eqs. 1-2):
// fractional Brownian motion by Fourier filtering of caller-drawn white noise,
// and the bond conductances built from the node field, with optional bond
// dilution by caller-drawn uniforms. This replaces, on one GPU, the paper's
// distributed generator; the flow solve does not depend on it.
//
// Transforms are hipFFT's double-precision real-to-complex and back; the
// spectral filter, the standardisation and the bonds are kernels here.
#include "rn_runtime.hpp"

#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>

namespace rn {
namespace {

// Spectral filter on the half spectrum of a real nz x ny x nx grid (x
// fastest, nxh = nx/2 + 1 modes along x): multiply by the amplitude
// (sum_k beta_k f_k^2)^-(H + d/2)/2, with f the mode's frequency in cycles per
// node (f = j/n for j <= (n-1)/2, else (j - n)/n), zero the k = 0 mode, and
// fold in the 1/N of the inverse transform.
__global__ void fbm_filter_kernel(hipfftDoubleComplex *spec, int nx, int ny, int nz, int dim, double bx, double by,
                                  double bz, double expo, double inv_n)
{
    const int nxh = nx / 2 + 1;
    const int64_t total = (int64_t)nz * ny * nxh;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int jx = (int)(i % nxh);
        const int64_t t = i / nxh;
        const int jy = (int)(t % ny);
        const int jz = (int)(t / ny);
        const double fx = (double)jx / nx;   // jx <= nx/2: non-negative frequencies only
        const double fy = (double)(jy <= (ny - 1) / 2 ? jy : jy - ny) / ny;
        const double fz = dim == 3 ? (double)(jz <= (nz - 1) / 2 ? jz : jz - nz) / nz : 0.0;
        const double k2 = bx * fx * fx + by * fy * fy + bz * fz * fz;
        const double a = k2 > 0.0 ? pow(k2, expo) * inv_n : 0.0;
        hipfftDoubleComplex v = spec[i];
        v.x *= a;
        v.y *= a;
        spec[i] = v;
    }
}

// Block sums in a fixed order: block b adds elements b, b + grid, ... (per
// thread, in index order), then a tree over the block; a second launch of one
// block adds the block sums in order. mode 0: sum x; mode 1: sum (x - c)^2.
constexpr int kRedThreads = 256, kRedBlocks = 1024;

__global__ void fbm_sum_kernel(const double *x, int64_t n, double c, int mode, double *partial)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = mode ? (x[i] - c) * (x[i] - c) : x[i];
        acc += v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void fbm_total_kernel(const double *partial, int m, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < m; ++b) t += partial[b];
        *out = t;
    }
}

// (x - mean) / sd with the two sums produced above (sd = 0: all zeros)
__global__ void fbm_standardise_kernel(double *x, int64_t n, const double *sums)
{
    const double mean = sums[0] / (double)n;
    const double var = sums[1] / (double)n;
    const double inv = var > 0.0 ? 1.0 / sqrt(var) : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = var > 0.0 ? (x[i] - mean) * inv : 0.0;
}

__global__ void fbm_mean_kernel(const double *sums, int64_t n, double *mean)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *mean = sums[0] / (double)n;
}

// g_k[i] = exp(sigma (phi_i + phi_{i+e_k}) / 2) on the periodic grid; 0 on the
// last plane along k unless periodic; 0 where u_k[i] >= occupancy (u_k given)
__global__ void fbm_bonds_kernel(const double *phi, int nx, int ny, int nz, int dim, double sigma, int periodic,
                                 const double *u0, const double *u1, const double *u2, double occ, double *g0,
                                 double *g1, double *g2)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t st[3] = {1, nx, (int64_t)nx * ny};
    const int ext[3] = {nx, ny, nz};
    const double *u[3] = {u0, u1, u2};
    double *g[3] = {g0, g1, g2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((int64_t)nx * ny))};
        for (int k = 0; k < dim; ++k) {
            const bool last = c[k] == ext[k] - 1;
            const int64_t j = last ? i - (int64_t)(ext[k] - 1) * st[k] : i + st[k];
            double v = exp(sigma * 0.5 * (phi[i] + phi[j]));
            if (last && !periodic) v = 0.0;
            if (u[k] && !(u[k][i] < occ)) v = 0.0;
            g[k][i] = v;
        }
    }
}

int grid_of(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

bool shape_ok(int dim, int64_t nx, int64_t ny, int64_t nz)
{
    if (dim != 2 && dim != 3) return false;
    if (nx < 1 || ny < 1 || nz < 1 || (dim == 2 && nz != 1)) return false;
    if (nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX) return false;
    return (double)nx * (double)ny * (double)nz < 2147483647.0;
}

// The forward and inverse plans of the last grid, kept on the context: plan
// creation costs milliseconds, more than the transforms of a 2048^2 grid.
struct FbmPlans {
    int dim = 0, nx = 0, ny = 0, nz = 0;
    hipfftHandle fwd = 0, inv = 0;
    ~FbmPlans()
    {
        if (fwd) (void)hipfftDestroy(fwd);
        if (inv) (void)hipfftDestroy(inv);
    }
};

struct Scratch {
    rn_ctx *ctx;
    char *base = nullptr;
    explicit Scratch(rn_ctx *c) : ctx(c) {}
    ~Scratch()
    {
        if (base) {
            (void)hipStreamSynchronize(ctx->stream);
            ctx->pool.free(base);
        }
    }
};

}  // namespace

void fbm_release(rn_ctx *ctx)
{
    delete static_cast<FbmPlans *>(ctx->fbm_plans);
    ctx->fbm_plans = nullptr;
}

}  // namespace rn

using namespace rn;

#define FBM_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
            return RN_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

#define FFT_TRY(expr)                                                                 \
    do {                                                                              \
        hipfftResult r_ = (expr);                                                     \
        if (r_ != HIPFFT_SUCCESS) {                                                   \
            ctx->err = std::string(#expr) + ": hipfft status " + std::to_string((int)r_); \
            return RN_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

extern "C" int rn_fbm_field(rn_ctx *ctx, int32_t dim, int64_t nx, int64_t ny, int64_t nz, double H,
                            const double *beta, const double *noise, double *field_out, int32_t mem)
{
    if (!ctx || !noise || !field_out || !shape_ok(dim, nx, ny, nz) || !std::isfinite(H)) return RN_EINVAL;
    if (mem != RN_MEM_HOST && mem != RN_MEM_DEVICE) return RN_EINVAL;
    double b[3] = {1.0, 1.0, 1.0};
    for (int k = 0; beta && k < dim; ++k) {
        if (!(beta[k] > 0.0) || !std::isfinite(beta[k])) return RN_EINVAL;
        b[k] = beta[k];
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (ctx->server) return RN_EINVAL;        // the server owns the stream once started
    FBM_TRY(hipSetDevice(ctx->device));
    const int64_t n = nx * ny * nz;
    const int64_t nspec = nz * ny * (nx / 2 + 1);
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t off_x = 0, off_s = a256(8 * n), off_p = off_s + a256(16 * nspec), off_sum = off_p + a256(8 * kRedBlocks),
                 total = off_sum + 256;
    Scratch sc(ctx);
    hipError_t he;
    sc.base = (char *)ctx->pool.alloc(total, &he);
    if (!sc.base) return RN_ENOMEM;
    double *x = (double *)(sc.base + off_x);
    hipfftDoubleComplex *spec = (hipfftDoubleComplex *)(sc.base + off_s);
    double *partial = (double *)(sc.base + off_p), *sums = (double *)(sc.base + off_sum);
    const hipStream_t st = ctx->stream;
    FBM_TRY(hipMemcpyAsync(x, noise, 8 * n, mem == RN_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    FbmPlans *pl = static_cast<FbmPlans *>(ctx->fbm_plans);
    if (!pl || pl->dim != dim || pl->nx != nx || pl->ny != ny || pl->nz != nz) {
        fbm_release(ctx);
        pl = new FbmPlans();
        ctx->fbm_plans = pl;
        // hipFFT's first extent is the slowest: (ny, nx) and (nz, ny, nx)
        if (dim == 2) {
            FFT_TRY(hipfftPlan2d(&pl->fwd, (int)ny, (int)nx, HIPFFT_D2Z));
            FFT_TRY(hipfftPlan2d(&pl->inv, (int)ny, (int)nx, HIPFFT_Z2D));
        } else {
            FFT_TRY(hipfftPlan3d(&pl->fwd, (int)nz, (int)ny, (int)nx, HIPFFT_D2Z));
            FFT_TRY(hipfftPlan3d(&pl->inv, (int)nz, (int)ny, (int)nx, HIPFFT_Z2D));
        }
        pl->dim = dim;
        pl->nx = (int)nx;
        pl->ny = (int)ny;
        pl->nz = (int)nz;
    }
    const hipfftHandle fwd = pl->fwd, inv = pl->inv;
    FFT_TRY(hipfftSetStream(fwd, st));
    FFT_TRY(hipfftSetStream(inv, st));
    FFT_TRY(hipfftExecD2Z(fwd, x, spec));
    fbm_filter_kernel<<<grid_of(nspec), 256, 0, st>>>(spec, (int)nx, (int)ny, (int)nz, dim, b[0], b[1],
                                                       dim == 3 ? b[2] : 0.0, -(H + 0.5 * dim) / 2.0,
                                                       1.0 / (double)n);
    FBM_TRY(hipGetLastError());
    FFT_TRY(hipfftExecZ2D(inv, spec, x));
    // standardise: mean, then the mean square deviation (population), both in a fixed order
    fbm_sum_kernel<<<kRedBlocks, kRedThreads, 0, st>>>(x, n, 0.0, 0, partial);
    fbm_total_kernel<<<1, 64, 0, st>>>(partial, kRedBlocks, sums);
    fbm_mean_kernel<<<1, 64, 0, st>>>(sums, n, sums + 2);
    FBM_TRY(hipGetLastError());
    double mean = 0.0;
    FBM_TRY(hipMemcpyAsync(&mean, sums + 2, 8, hipMemcpyDeviceToHost, st));
    FBM_TRY(hipStreamSynchronize(st));
    fbm_sum_kernel<<<kRedBlocks, kRedThreads, 0, st>>>(x, n, mean, 1, partial);
    fbm_total_kernel<<<1, 64, 0, st>>>(partial, kRedBlocks, sums + 1);
    fbm_standardise_kernel<<<grid_of(n), 256, 0, st>>>(x, n, sums);
    FBM_TRY(hipGetLastError());
    FBM_TRY(hipMemcpyAsync(field_out, x, 8 * n, mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           st));
    FBM_TRY(hipStreamSynchronize(st));
    return RN_OK;
}

extern "C" int rn_fbm_bonds(rn_ctx *ctx, int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *field,
                            double sigma, int32_t periodic, const double *const u[3], double occupancy,
                            double *const g_out[3], int32_t mem)
{
    if (!ctx || !field || !g_out || !shape_ok(dim, nx, ny, nz) || !std::isfinite(sigma)) return RN_EINVAL;
    if (mem != RN_MEM_HOST && mem != RN_MEM_DEVICE) return RN_EINVAL;
    if (periodic != 0 && periodic != 1) return RN_EINVAL;
    for (int k = 0; k < dim; ++k)
        if (!g_out[k]) return RN_EINVAL;
    const bool dilute = u && u[0];
    if (dilute) {
        for (int k = 0; k < dim; ++k)
            if (!u[k]) return RN_EINVAL;
        if (!std::isfinite(occupancy)) return RN_EINVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (ctx->server) return RN_EINVAL;
    FBM_TRY(hipSetDevice(ctx->device));
    const int64_t n = nx * ny * nz;
    const hipStream_t st = ctx->stream;
    const double *phi = field;
    const double *ud[3] = {nullptr, nullptr, nullptr};
    double *gd[3] = {nullptr, nullptr, nullptr};
    Scratch sc(ctx);
    if (mem == RN_MEM_HOST) {
        // stage: field, the uniforms and the bond arrays
        const size_t a = (8 * (size_t)n + 255) & ~(size_t)255;
        const size_t total = a * (1 + (dilute ? dim : 0) + dim);
        hipError_t he;
        sc.base = (char *)ctx->pool.alloc(total, &he);
        if (!sc.base) return RN_ENOMEM;
        char *p = sc.base;
        FBM_TRY(hipMemcpyAsync(p, field, 8 * n, hipMemcpyHostToDevice, st));
        phi = (const double *)p;
        p += a;
        for (int k = 0; dilute && k < dim; ++k, p += a) {
            FBM_TRY(hipMemcpyAsync(p, u[k], 8 * n, hipMemcpyHostToDevice, st));
            ud[k] = (const double *)p;
        }
        for (int k = 0; k < dim; ++k, p += a) gd[k] = (double *)p;
    } else {
        for (int k = 0; k < dim; ++k) {
            gd[k] = g_out[k];
            if (dilute) ud[k] = u[k];
        }
    }
    fbm_bonds_kernel<<<grid_of(n), 256, 0, st>>>(phi, (int)nx, (int)ny, (int)nz, dim, sigma, periodic, ud[0], ud[1],
                                                 ud[2], occupancy, gd[0], gd[1], gd[2]);
    FBM_TRY(hipGetLastError());
    if (mem == RN_MEM_HOST)
        for (int k = 0; k < dim; ++k) FBM_TRY(hipMemcpyAsync(g_out[k], gd[k], 8 * n, hipMemcpyDeviceToHost, st));
    FBM_TRY(hipStreamSynchronize(st));
    return RN_OK;
}
