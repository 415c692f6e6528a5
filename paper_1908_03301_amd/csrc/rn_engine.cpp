// rn_engine.cpp -- device memory pool, per-network lifecycle and the
// multi-network iteration engine.
//
// Every network in the engine owns a control-block slot. Each pass round
// launches one pass kernel per kind (2D full or small tiles / 3D x FP32/FP64) over a block table
// listing (slot, local block) for every active network, so networks of any
// size and dimension advance together while each keeps its own reduction,
// scalars and convergence. A network's arithmetic depends only on its own
// data and tile shape, never on the rest of the launch: a network gives the
// same bits alone and in a batch.
#include "rn_runtime.hpp"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

namespace rn {

#define ENG_TRY(expr)                                                  \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) {                                        \
            if (err) *err = std::string(#expr) + ": " + hipGetErrorString(e_); \
            return RN_EDEVICE;                                         \
        }                                                              \
    } while (0)

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ checks

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
    if (p->flags & ~RN_PERIODIC) return RN_EINVAL;
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
    if (o->precond != RN_JACOBI && o->precond != RN_NONE) return RN_EINVAL;
    if (o->x0 != RN_X0_LINEAR && o->x0 != RN_X0_ZERO) return RN_EINVAL;
    if (o->flags & ~(RN_OPT_BACKBONE | RN_OPT_COMPACT)) return RN_EINVAL;
    return RN_OK;
}

int wrap_bits(const rn_problem *p)
{
    if (!(p->flags & RN_PERIODIC)) return 0;
    const int64_t n[3] = {p->nx, p->ny, p->nz};
    int bits = 0;
    for (int k = 0; k < p->dim; ++k)
        if (k != p->axis && n[k] >= 2) bits |= 1 << k;
    return bits;
}

Lat make_lat(const rn_problem *p)
{
    return Lat{p->dim, p->axis, (int)p->nx, (int)p->ny, (int)p->nz, p->nx * p->ny * p->nz, wrap_bits(p)};
}

bool host_values_ok(const rn_problem *p)
{
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
    const int wrap = wrap_bits(p);
    for (int k = 0; k < p->dim; ++k) {
        const double *g = p->g[k];
        const bool wk = (wrap >> k) & 1;   // the last plane's entries are wrap bonds
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y) {
                const double *row = g + nx * (y + ny * z);
                int64_t xe = nx;
                if (k == 0 && !wk) xe = nx - 1;
                else if (k == 1 && y == ny - 1 && !wk) xe = 0;
                else if (k == 2 && z == nz - 1 && !wk) xe = 0;
                for (int64_t x = 0; x < xe; ++x) {
                    const double v = row[x];
                    if (!(v >= 0.0) || std::isinf(v)) return false;
                }
            }
    }
    return true;
}

double cross_section(const rn_problem *p)
{
    double s = 1.0;
    const int64_t n[3] = {p->nx, p->ny, p->nz};
    for (int k = 0; k < p->dim; ++k)
        if (k != p->axis) s *= (double)n[k];
    return s;
}

// A 2D workgroup runs two tiles per pass when the network has more tiles than
// one round of workgroups holds (256 CUs x 4 workgroups = 1024): every
// workgroup is then resident from the start instead of a few running in a
// second round, and the per-workgroup tail (partials, ticket) is paid once
// per two tiles. Measured per mixed pass: 1448^2 (1,092 tiles) 27.3 -> 26.6
// us, 1600^2 29.6 -> 27.3 us, 1800^2 34.7 -> 31.9 us against one tile per
// workgroup. On the 2048^2 FP64 pass, three or four tiles per workgroup were
// 2% slower than two.
constexpr int kWGTarget2D = 1024, kTpwMax2D = 2, kSmall2D = 128;
constexpr int kResident3D = 512;   // 3D workgroups resident at once (256 CUs x 2)


// ------------------------------------------------------------------ launch-shape table

namespace {
std::mutex g_shape_mu;
ShapeTable g_shapes;   // every entry follows the built-in rules until a table is installed
}  // namespace

int shape_class(int64_t n)
{
    int c = 0;
    while (c + 1 < kShapeClasses && ((int64_t)1 << (c + 1)) <= n) ++c;
    return c;
}

ShapeChoice shape_choice(int dim, int s, int64_t n)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    return g_shapes.c[dim == 3 ? 1 : 0][s == 4 ? 1 : 0][shape_class(n)];
}

ShapeTable shape_table_get()
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    return g_shapes;
}

void shape_table_install(const ShapeTable &t)
{
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shapes = t;
}

bool shape_choice_valid(int dim, const ShapeChoice &c)
{
    if (dim == 2) return c.shape < 0 || ((c.shape == 0 || c.shape == 1) && c.tpw >= 1 && c.tpw <= 4);
    return c.tile_z == 0 || (c.tile_z >= 1 && c.tile_z <= 64);
}

// Text form, one line per tuned entry:
//   <dim> <fp32|fp64> <class> <shape> <tiles per workgroup> <tile_z> <ns per node and pass>
// ('#' starts a comment line).
std::string shape_table_format(const ShapeTable &t)
{
    std::string out = "# librn launch shapes: dim precision class shape tiles_per_wg tile_z ns_per_node_pass\n";
    char line[160];
    for (int d = 0; d < 2; ++d)
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < kShapeClasses; ++c) {
                const ShapeChoice &e = t.c[d][f][c];
                if (d == 0 ? e.shape < 0 : e.tile_z == 0) continue;
                std::snprintf(line, sizeof(line), "%d %s %d %d %d %d %.6f\n", d + 2, f ? "fp32" : "fp64", c, e.shape,
                              e.tpw, e.tile_z, e.ns_per_node);
                out += line;
            }
    return out;
}

int shape_table_parse(const std::string &text, ShapeTable *out)
{
    ShapeTable t;
    size_t pos = 0;
    while (pos < text.size()) {
        size_t end = text.find('\n', pos);
        if (end == std::string::npos) end = text.size();
        std::string line = text.substr(pos, end - pos);
        pos = end + 1;
        const size_t first = line.find_first_not_of(" \t\r");
        if (first == std::string::npos || line[first] == '#') continue;
        int dim = 0, cls = -1, shape = 0, tpw = 0, tz = 0, used = 0;
        char prec[8] = {0};
        double ns = 0.0;
        if (std::sscanf(line.c_str(), "%d %7s %d %d %d %d %lf %n", &dim, prec, &cls, &shape, &tpw, &tz, &ns, &used) < 7)
            return RN_EINVAL;
        if (line.find_first_not_of(" \t\r", (size_t)used) != std::string::npos) return RN_EINVAL;
        const std::string ps(prec);
        if ((dim != 2 && dim != 3) || (ps != "fp32" && ps != "fp64") || cls < 0 || cls >= kShapeClasses)
            return RN_EINVAL;
        ShapeChoice e;
        e.ns_per_node = ns;
        if (dim == 2) {
            e.shape = shape;
            e.tpw = tpw;
            if (shape < 0) return RN_EINVAL;
        } else {
            e.tile_z = tz;
            if (tz <= 0) return RN_EINVAL;
        }
        if (!shape_choice_valid(dim, e) || !std::isfinite(ns) || ns < 0.0) return RN_EINVAL;
        t.c[dim - 2][ps == "fp32" ? 1 : 0][cls] = e;
    }
    *out = t;
    return RN_OK;
}

Layout make_layout(const rn_problem *p, const rn_opts *o)
{
    Layout L;
    L.n = p->nx * p->ny * p->nz;
    L.dim = p->dim;
    L.s = (o && o->precision == RN_MIXED) ? 4 : 8;
    L.copy_g = p->mem == RN_MEM_HOST;
    if (p->dim == 2) {
        // full tiles unless the network has fewer than kSmall2D of them: its
        // pass is then bound by the latency of one tile, which the
        // quarter-size tile (64 columns, half the rows) shortens. Measured
        // per pass: 128^2 10.2 -> 8.5 us, 256^2 9.3 -> 8.4 us; at 512^2 and
        // 1024^2 the small tile was no faster alone and slower in batches.
        L.ntx = div_up((int)p->nx, kWave * (L.s == 4 ? kSEG2f : kSEG2d));
        L.nty = div_up((int)p->ny, (L.s == 4 ? kTY2f : kTY2d) * (kBlock / kWave));
        const ShapeChoice ch = shape_choice(2, L.s, L.n);
        L.shape = ch.shape >= 0 ? ch.shape : (L.ntx * L.nty < kSmall2D ? 1 : 0);
        if (L.shape) {
            L.ntx = div_up((int)p->nx, kWave);
            L.nty = div_up((int)p->ny, (L.s == 4 ? kTY2fS : kTY2dS) * (kBlock / kWave));
        }
        L.ntz = 1;
        L.ntiles = L.ntx * L.nty;
        L.tpw = ch.shape >= 0 ? ch.tpw : std::max(1, std::min(kTpwMax2D, div_up(L.ntiles, kWGTarget2D)));
        L.tpw = std::min(L.tpw, L.ntiles);
        L.grid = div_up(L.ntiles, L.tpw);
    } else {
        // planes per tile: a tile streams its planes one after another, so
        // a small network's pass takes as long as one tile's stream, while a
        // large one is bound by bytes. The 3D kernel runs 2 waves per SIMD,
        // i.e. kResident3D = 512 workgroups at once; tile_z is the one that
        // needs the fewest rounds of workgroups and, among those, gives the
        // most tiles. Measured per mixed pass, against the tile depth this
        // rule does not pick: 32^3 16.6 -> 12.7 us (4 -> 2 planes), 64^3
        // 16.8 -> 13.6 us (4 -> 2), 192^3 80.5 -> 76.3 us (8 -> 16), 256^3
        // 169.1 -> 164.9 us (16 -> 32), 256^2 x 64 48.5 -> 40.2 us (16 -> 8).
        // A batch of 512 networks of 32^3 to 128^3 and 64^2 to 1024^2 was 5%
        // slower with 2-plane tiles on every network below 3 M nodes.
        L.ntx = div_up((int)p->nx, kTX);
        L.nty = div_up((int)p->ny, kTY);
        {
            int best_tz = kTZ / 8, best_rounds = 0, best_tiles = 0;
            for (int tz = 2 * kTZ; tz >= kTZ / 8; tz /= 2) {
                const int tiles = L.ntx * L.nty * div_up((int)p->nz, tz);
                const int rounds = div_up(tiles, kResident3D);
                if (best_tiles == 0 || rounds < best_rounds || (rounds == best_rounds && tiles > best_tiles)) {
                    best_tz = tz;
                    best_rounds = rounds;
                    best_tiles = tiles;
                }
            }
            L.tile_z = best_tz;
            const ShapeChoice ch = shape_choice(3, L.s, L.n);
            if (ch.tile_z > 0) L.tile_z = ch.tile_z;
        }
        L.ntz = div_up((int)p->nz, L.tile_z);
        L.ntiles = L.ntx * L.nty * L.ntz;
        L.grid = L.ntiles;
    }
    // completion-ticket groups: about one per 64 workgroups, a power of two
    // up to kGroupsMax; the grid is a multiple of 8 (XCD remap) and of groups
    L.groups = 1;
    while (L.groups * 2 <= kGroupsMax && L.groups * 2 * 64 <= L.grid) L.groups *= 2;
    const int gq = L.groups > 8 ? L.groups : 8;
    L.grid = (L.grid + gq - 1) / gq * gq;
    const size_t n = (size_t)L.n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o_ = off;
        off += align256(bytes);
        return o_;
    };
    L.off_g64 = take(L.copy_g ? (size_t)8 * L.dim * n : 0);
    L.off_P = take(16 * n);
    L.off_mask = take(n);
    L.off_gT = take((size_t)L.s * L.dim * n);
    L.kpend = L.s == 4 ? 4 : 2;
    // two sets of z and u and kpend + 1 directions; the labels of the
    // connectivity kernels (8 bytes per node) alias here
    L.off_vec = take((size_t)(5 + L.kpend) * L.s * n);
    L.off_part = take((size_t)L.grid * kRed * 8);
    L.off_tk = take(ticket_bytes(L.groups));
    L.off_cnt = take(4 * sizeof(unsigned long long));
    L.total = off;
    return L;
}

// ------------------------------------------------------------------ pool

Pool::~Pool() { release_all(); }

void Pool::release_all()
{
    for (auto &s : slabs_) (void)hipFree(s.base);
    slabs_.clear();
    reserved_ = in_use_ = 0;
}

void *Pool::alloc(size_t bytes, hipError_t *err)
{
    *err = hipSuccess;
    bytes = align256(bytes ? bytes : 256);
    for (auto &s : slabs_) {
        for (auto it = s.free_.begin(); it != s.free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            s.free_.erase(it);
            if (len > bytes) s.free_[off + bytes] = len - bytes;
            s.used_[off] = bytes;
            in_use_ += bytes;
            return s.base + off;
        }
    }
    const size_t gib = (size_t)1 << 30;
    // a new slab: 1 GiB or the request, whichever is larger, within the budget.
    // When the budget is taken by slabs, the ones nothing is carved from are
    // released first: otherwise a request larger than every free range would
    // wait for memory that no running network will ever return.
    if (reserved_ + bytes > budget_) trim();
    size_t size = std::max(bytes, gib);
    if (reserved_ + size > budget_) size = bytes;
    if (reserved_ + size > budget_) return nullptr;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *err = e;
        return nullptr;
    }
    Slab s{(char *)p, size, {}, {}};
    if (size > bytes) s.free_[bytes] = size - bytes;
    s.used_[0] = bytes;
    slabs_.push_back(std::move(s));
    reserved_ += size;
    in_use_ += bytes;
    return p;
}

void Pool::trim()
{
    // every pool user frees its range only after the work that uses it has
    // completed on the stream, so an empty slab has no work in flight
    std::vector<Slab> keep;
    for (auto &s : slabs_) {
        if (s.used_.empty()) {
            (void)hipFree(s.base);
            reserved_ -= s.size;
        } else {
            keep.push_back(std::move(s));
        }
    }
    slabs_.swap(keep);
}

void Pool::free(void *ptr)
{
    if (!ptr) return;
    char *p = (char *)ptr;
    for (auto &s : slabs_) {
        if (p < s.base || p >= s.base + s.size) continue;
        const size_t off = (size_t)(p - s.base);
        auto u = s.used_.find(off);
        if (u == s.used_.end()) return;
        size_t len = u->second;
        s.used_.erase(u);
        in_use_ -= len;
        size_t start = off;
        auto nx = s.free_.lower_bound(off);
        if (nx != s.free_.end() && nx->first == off + len) {
            len += nx->second;
            s.free_.erase(nx);
        }
        auto pv = s.free_.lower_bound(off);
        if (pv != s.free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                len += pv->second;
                s.free_.erase(pv);
            }
        }
        s.free_[start] = len;
        return;
    }
}

// ------------------------------------------------------------------ engine

int Engine::init(hipStream_t st, std::string *err)
{
    (void)st;
    // Graph replay of pass rounds is opt-in (RN_GRAPHS=1): on a launch-bound
    // 128^2 solve it measured 5% slower than direct launches, since the time
    // of a small pass is spent on the device, not in the launch call.
    const char *g = std::getenv("RN_GRAPHS");
    use_graph_ = g && g[0] == '1';
    // persistent launches are opt-in, bit-identical to one launch per round:
    // RN_PERSIST=1 (items on all XCDs) measured slower on every workload here,
    // RN_PERSIST=2 (each small network on one XCD) 2% faster on a 128^2
    // solve and even on batches, whose time is in the large networks
    const char *pe = std::getenv("RN_PERSIST");
    persist_mode_ = (pe && pe[0] == '1') ? 1 : ((pe && pe[0] == '2') ? 2 : 0);
    persist_ = persist_mode_ != 0;
    if (persist_) use_graph_ = false;
    ENG_TRY(hipMalloc(&d_queue_, kQueueWords * sizeof(unsigned long long) * kKinds));
    ENG_TRY(hipMalloc(&d_xoff_, sizeof(int) * 16 * kKinds));
    ENG_TRY(hipHostMalloc((void **)&h_xoff_, sizeof(int) * 16 * kKinds * 2, hipHostMallocDefault));
    ENG_TRY(hipMalloc(&d_err_, 256));
    ENG_TRY(hipMemset(d_err_, 0, 256));
    ENG_TRY(hipHostMalloc((void **)&h_err_, 256, hipHostMallocDefault));
    std::memset(h_err_, 0, 256);
    ENG_TRY(hipMalloc(&d_scal_, sizeof(Scalars) * kSlots));
    ENG_TRY(hipMalloc(&d_tabf_, sizeof(PassArgs<float>) * 2 * kSlots));
    ENG_TRY(hipMalloc(&d_tabd_, sizeof(PassArgs<double>) * 2 * kSlots));
    for (int b = 0; b < 2; ++b) ENG_TRY(hipHostMalloc((void **)&h_scal_[b], sizeof(Scalars) * kSlots, hipHostMallocDefault));
    ENG_TRY(hipHostMalloc((void **)&h_init_, sizeof(Scalars) * kSlots, hipHostMallocDefault));
    ENG_TRY(hipHostMalloc((void **)&h_tabf_, sizeof(PassArgs<float>) * 2 * kSlots, hipHostMallocDefault));
    ENG_TRY(hipHostMalloc((void **)&h_tabd_, sizeof(PassArgs<double>) * 2 * kSlots, hipHostMallocDefault));
    ENG_TRY(hipHostMalloc((void **)&h_cnt_, sizeof(unsigned long long) * 4 * kSlots, hipHostMallocDefault));
    for (auto &e : ev_chunk_) ENG_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    free_slots_.clear();
    for (int s = kSlots - 1; s >= 0; --s) free_slots_.push_back(s);
    return RN_OK;
}

void Engine::destroy()
{
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    (void)hipFree(d_scal_);
    (void)hipFree(d_tabf_);
    (void)hipFree(d_tabd_);
    for (auto p : h_scal_) (void)hipHostFree(p);
    (void)hipHostFree(h_init_);
    (void)hipHostFree(h_tabf_);
    (void)hipHostFree(h_tabd_);
    (void)hipHostFree(h_cnt_);
    (void)hipFree(d_err_);
    (void)hipFree(d_queue_);
    d_queue_ = nullptr;
    (void)hipFree(d_xoff_);
    (void)hipHostFree(h_xoff_);
    d_xoff_ = nullptr;
    h_xoff_ = nullptr;
    (void)hipHostFree(h_err_);
    d_err_ = h_err_ = nullptr;
    for (int k = 0; k < kKinds; ++k) {
        (void)hipFree(d_blk_[k]);
        (void)hipHostFree(h_blk_[k]);
    }
    for (auto e : ev_chunk_)
        if (e) (void)hipEventDestroy(e);
    for (auto &v : tev_) {
        for (auto e : v) (void)hipEventDestroy(e);
        v.clear();
    }
    d_scal_ = nullptr;
}

// Setup runs on the side stream when the context has one (its own compute
// stream is in use): the upload, validation and connectivity kernels of a new
// network then overlap the pass launches of the running ones.
int Engine::prepare(Net *net, hipStream_t st_compute, std::string *err)
{
    const hipStream_t st = side_ ? side_ : st_compute;
    const rn_problem *p = &net->prob;
    const Layout &L = net->L;
    char *base = net->base;
    const size_t n = (size_t)L.n;
    net->slot = free_slots_.back();
    free_slots_.pop_back();
    by_slot_[net->slot] = net;
    net->na = p->axis == 0 ? p->nx : (p->axis == 1 ? p->ny : p->nz);
    const Lat lat = make_lat(p);
    unsigned long long *cnt = (unsigned long long *)(base + L.off_cnt);
    if (!net->ev) ENG_TRY(hipEventCreateWithFlags(&net->ev, hipEventDisableTiming));
    for (hipEvent_t *e : {&net->ev_a, &net->ev_b, &net->ev_c, &net->ev_d})
        if (!*e) ENG_TRY(hipEventCreate(e));
    ENG_TRY(hipEventRecord(net->ev_a, st));
    if (L.copy_g) {
        for (int k = 0; k < p->dim; ++k) {
            double *dst = (double *)(base + L.off_g64) + (size_t)k * n;
            ENG_TRY(hipMemcpyAsync(dst, p->g[k], 8 * n, hipMemcpyHostToDevice, st));
            net->gd[k] = dst;
        }
    } else {
        for (int k = 0; k < p->dim; ++k) net->gd[k] = p->g[k];
    }
    ENG_TRY(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), st));
    ENG_TRY(hipMemsetAsync(base + L.off_tk, 0, ticket_bytes(L.groups), st));
    if (!L.copy_g) ENG_TRY(launch_validate(lat, net->gd, cnt + 1, st));
    int *parent = (int *)(base + L.off_vec);
    unsigned *flags = (unsigned *)(base + L.off_vec + 4 * n);
    ENG_TRY(launch_mask(lat, net->gd, parent, flags, (uint8_t *)(base + L.off_mask), (double *)(base + L.off_P),
                        cnt, net->opts.x0 == RN_X0_LINEAR, st));
    if (net->na == 2) ENG_TRY(launch_direct_flux(lat, net->gd[p->axis], (double *)(cnt + 2), st));
    ENG_TRY(hipEventRecord(net->ev_b, st));
    ENG_TRY(hipMemcpyAsync(h_cnt_ + 4 * net->slot, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    ENG_TRY(hipEventRecord(net->ev, st));
    net->phase = NET_PREPARING;
    return RN_OK;
}

template <typename T>
static void fill_args(PassArgs<T> *a2, const Net *net, int first_parity, Scalars *ds)
{
    const rn_problem *p = &net->prob;
    const Layout &L = net->L;
    char *base = net->base;
    const size_t n = (size_t)L.n;
    T *vec = (T *)(base + L.off_vec);
    VecSet<T> s0{vec, vec + n};
    VecSet<T> s1{vec + 2 * n, vec + 3 * n};
    for (int k = 0; k < 2; ++k) {
        PassArgs<T> A;
        std::memset(&A, 0, sizeof(A));
        A.nx = (int)p->nx;
        A.ny = (int)p->ny;
        A.nz = (int)p->nz;
        A.axis = p->axis;
        A.ntx = L.ntx;
        A.nty = L.nty;
        A.ntz = L.ntz;
        A.wrap = wrap_bits(p);
        A.tile_z = L.tile_z;
        A.jacobi = net->opts.precond == RN_JACOBI ? 1 : 0;
        A.ntiles = L.ntiles;
        A.tpw = L.tpw;
        A.grid = L.grid;
        A.groups = L.groups;
        A.round0 = net->round0;
        for (int d = 0; d < 3; ++d) {
            A.g64[d] = net->gd[d];
            A.gT[d] = d < p->dim ? (const T *)(base + L.off_gT) + (size_t)d * n : nullptr;
        }
        A.P[0] = (double *)(base + L.off_P);
        A.P[1] = A.P[0] + n;
        A.mask = (const uint8_t *)(base + L.off_mask);
        A.src = k == 0 ? s0 : s1;
        for (int b = 0; b < 5; ++b) A.pbuf[b] = b <= L.kpend ? vec + (4 + b) * n : nullptr;
        A.npbuf = L.kpend + 1;
        A.dst = k == 0 ? s1 : s0;
        A.partials = (double *)(base + L.off_part);
        A.tickets = (unsigned *)(base + L.off_tk);
        A.s = ds;
        a2[(first_parity + k) & 1] = A;
    }
}

int Engine::after_prepare(Net *net, hipStream_t st, std::string *err)
{
    const rn_problem *p = &net->prob;
    const Layout &L = net->L;
    char *base = net->base;
    const size_t n = (size_t)L.n;
    const unsigned long long *c = h_cnt_ + 4 * net->slot;
    std::memset(&net->res, 0, sizeof(net->res));
    if (c[1] != 0) {                                   // invalid device-resident values
        net->status = RN_EINVAL;
        net->res.status = RN_EINVAL;
        by_slot_[net->slot] = nullptr;
        free_slots_.push_back(net->slot);
        net->slot = -1;
        net->phase = NET_DONE;
        return RN_EINVAL;
    }
    net->n_live = (int64_t)c[0];
    net->res.n_live = net->n_live;
    if (net->n_live == 0) {
        double G = 0.0;
        if (net->na == 2) std::memcpy(&G, &c[2], sizeof(double));
        net->res.status = RN_OK;
        net->res.converged = 1;
        net->res.Q_in = net->res.Q_out = net->res.G = G;
        net->res.K = G * (double)(net->na - 1) / cross_section(p);
        net->status = RN_OK;
        // outputs of the setup alone (complete: the host has seen its event)
        const hipStream_t so = side_ ? side_ : st;
        ENG_TRY(hipEventRecord(net->ev_c, so));
        ENG_TRY(hipEventRecord(net->ev_d, so));
        if (p->p_out)
            ENG_TRY(hipMemcpyAsync(p->p_out, base + L.off_P, 8 * n,
                                   p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, so));
        if (p->mask_out)
            ENG_TRY(hipMemcpyAsync(p->mask_out, base + L.off_mask, n,
                                   p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, so));
        ENG_TRY(hipEventRecord(net->ev, so));
        by_slot_[net->slot] = nullptr;
        free_slots_.push_back(net->slot);
        net->slot = -1;
        net->phase = NET_FINISHING;
        return RN_OK;
    }
    const Lat lat = make_lat(p);
    const int slot = net->slot;
    Scalars *ds = d_scal_ + slot;
    Scalars &init = h_init_[slot];
    std::memset(&init, 0, sizeof(init));
    init.mode = MODE_REFRESH;
    init.first = 1;
    init.fp32 = L.s == 4;
    init.max_iter = net->opts.max_iter;
    init.sigma = 1.0;
    init.sigma_next = 1.0;
    init.tol = net->opts.tol;
    init.delta = (L.s == 4) ? (net->opts.delta > 0.0 ? net->opts.delta : 0.1) : 0.0;
    init.kappa = 1.0;
    init.bhat = 1.0;
    init.last_check = INFINITY;
    init.kpend = L.kpend;
    const int par0 = (int)(rounds_ & 1);
    net->round0 = rounds_;   // the network's first pass runs in the next round
    if (L.s == 4) {
        float *gT[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < p->dim; ++k) gT[k] = (float *)(base + L.off_gT) + (size_t)k * n;
        ENG_TRY(launch_scale<float>(lat, net->gd, (const uint8_t *)(base + L.off_mask), gT,
                                    (float *)(base + L.off_vec), (int64_t)((5 + L.kpend) * n), st));
        fill_args<float>(h_tabf_ + 2 * slot, net, par0, ds);
        ENG_TRY(hipMemcpyAsync(d_tabf_ + 2 * slot, h_tabf_ + 2 * slot, 2 * sizeof(PassArgs<float>),
                               hipMemcpyHostToDevice, st));
    } else {
        double *gT[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < p->dim; ++k) gT[k] = (double *)(base + L.off_gT) + (size_t)k * n;
        ENG_TRY(launch_scale<double>(lat, net->gd, (const uint8_t *)(base + L.off_mask), gT,
                                     (double *)(base + L.off_vec), (int64_t)((5 + L.kpend) * n), st));
        fill_args<double>(h_tabd_ + 2 * slot, net, par0, ds);
        ENG_TRY(hipMemcpyAsync(d_tabd_ + 2 * slot, h_tabd_ + 2 * slot, 2 * sizeof(PassArgs<double>),
                               hipMemcpyHostToDevice, st));
    }
    ENG_TRY(hipMemcpyAsync(ds, &init, sizeof(Scalars), hipMemcpyHostToDevice, st));
    ENG_TRY(hipEventRecord(net->ev_c, st));
    net->kind = kind_of(net);
    net->first_chunk = chunk_seq_ + 1;
    net->prev_est = -1.0;
    net->prev_iters = 0;
    net->phase = NET_ACTIVE;
    active_.push_back(net);
    dirty_ = true;
    return RN_OK;
}

int Engine::rebuild(hipStream_t st, std::string *err)
{
    int count[kKinds] = {};
    for (Net *n : active_) count[n->kind] += n->L.grid;
    for (int k = 0; k < kKinds; ++k) {
        if (count[k] > blk_cap_[k]) {
            const int cap = std::max(count[k], blk_cap_[k] * 3 / 2 + 1024);
            ENG_TRY(hipStreamSynchronize(st));
            (void)hipFree(d_blk_[k]);
            (void)hipHostFree(h_blk_[k]);
            d_blk_[k] = nullptr;
            h_blk_[k] = nullptr;
            ENG_TRY(hipMalloc(&d_blk_[k], sizeof(uint2) * cap));
            ENG_TRY(hipHostMalloc((void **)&h_blk_[k], sizeof(uint2) * 2 * cap, hipHostMallocDefault));
            blk_cap_[k] = cap;
        }
    }
    // host staging is double-buffered: the copy queued by the previous rebuild
    // may not have run yet (one chunk stays in flight)
    half_ ^= 1;
    for (int k = 0; k < kKinds; ++k) {
        nblk_[k] = count[k];
        single_[k] = -1;
        if (!count[k]) continue;
        int nets = 0;
        for (Net *n : active_)
            if (n->kind == k) {
                ++nets;
                single_[k] = n->slot;
            }
        if (nets != 1) single_[k] = -1;
        // how this kind's chunk runs: one launch per round (coherence 0), a
        // persistent launch over all XCDs (1), or a persistent launch with
        // each network on one XCD (2, when every network of the kind is small
        // enough that one XCD's workgroups hold a pass of it)
        int grid_max = 0;
        for (Net *n : active_)
            if (n->kind == k) grid_max = std::max(grid_max, n->L.grid);
        kind_coh_[k] = persist_mode_ == 1 ? 1 : ((persist_mode_ == 2 && grid_max <= kXcdMaxGrid) ? 2 : 0);
        uint2 *h = h_blk_[k] + (size_t)half_ * blk_cap_[k];
        int *xo = h_xoff_ + (size_t)(half_ * kKinds + k) * 16;
        int m = 0;
        if (kind_coh_[k] == 2) {
            // place the networks on the 8 XCDs, largest first, each on the XCD
            // with the fewest workgroups so far; the table lists XCD 0's
            // networks, then XCD 1's, and so on
            std::vector<Net *> nk;
            for (Net *n : active_)
                if (n->kind == k) nk.push_back(n);
            std::stable_sort(nk.begin(), nk.end(), [](const Net *a, const Net *b) { return a->L.grid > b->L.grid; });
            int64_t load[8] = {};
            std::vector<int> place(nk.size());
            for (size_t i = 0; i < nk.size(); ++i) {
                int best = 0;
                for (int x = 1; x < 8; ++x)
                    if (load[x] < load[best]) best = x;
                place[i] = best;
                load[best] += nk[i]->L.grid;
            }
            for (int x = 0; x < 8; ++x) {
                xo[x] = m;
                for (size_t i = 0; i < nk.size(); ++i)
                    if (place[i] == x)
                        for (int b = 0; b < nk[i]->L.grid; ++b) h[m++] = make_uint2((unsigned)nk[i]->slot, (unsigned)b);
            }
            xo[8] = m;
            single_[k] = -1;
        } else {
            for (Net *n : active_)
                if (n->kind == k)
                    for (int b = 0; b < n->L.grid; ++b) h[m++] = make_uint2((unsigned)n->slot, (unsigned)b);
            xo[0] = 0;
            for (int x = 1; x <= 8; ++x) xo[x] = m;
        }
        ENG_TRY(hipMemcpyAsync(d_blk_[k], h, sizeof(uint2) * m, hipMemcpyHostToDevice, st));
        ENG_TRY(hipMemcpyAsync(d_xoff_ + 16 * k, xo, sizeof(int) * 9, hipMemcpyHostToDevice, st));
    }
    dirty_ = false;
    return RN_OK;
}

void Engine::set_timing(bool on)
{
    timing_ = on;
    if (on)
        for (int k = 0; k < kKinds; ++k) {
            kind_s_[k] = 0.0;
            kind_n_[k] = 0;
        }
}

// Record the next timing event of the chunk being launched; kind < 0 marks
// the chunk's first event (before any launch).
int Engine::record_timing(int kind, hipStream_t st, std::string *err)
{
    std::vector<hipEvent_t> &ev = tev_[tmirror_];
    if (kind < 0) {
        trec_ = 0;
        tkind_[tmirror_].clear();
    } else {
        tkind_[tmirror_].push_back(kind);
    }
    if ((int)ev.size() <= trec_) {
        hipEvent_t e = nullptr;
        ENG_TRY(hipEventCreate(&e));
        ev.push_back(e);
    }
    ENG_TRY(hipEventRecord(ev[trec_], st));
    ++trec_;
    return RN_OK;
}

// Plain launches of `rounds` pass rounds (no rounds_ bookkeeping).
int Engine::launch_rounds(int rounds, hipStream_t st, std::string *err)
{
    for (int i = 0; i < rounds; ++i) {
        const int par = (int)((rounds_ + i) & 1);
        for (int k = 0; k < kKinds; ++k) {
            if (!nblk_[k] || kind_coh_[k] != 0) continue;
            const int dim = kind_dim(k);
            const uint2 *blk = single_[k] >= 0 ? nullptr : d_blk_[k];
            if (!kind_fp64(k))
                ENG_TRY(launch_pass<float>(dim, d_tabf_, blk, d_scal_, nblk_[k], par, single_[k], st));
            else
                ENG_TRY(launch_pass<double>(dim, d_tabd_, blk, d_scal_, nblk_[k], par, single_[k], st));
            if (recording_) {
                int r = record_timing(k, st, err);
                if (r) return r;
            }
        }
    }
    return RN_OK;
}

// One persistent launch per kind whose coherence mode is 1 or 2 runs all
// `rounds` rounds of its networks; the other kinds get one launch per round.
int Engine::launch_persistent(int rounds, hipStream_t st, std::string *err)
{
    for (int k = 0; k < kKinds; ++k) {
        if (!nblk_[k] || kind_coh_[k] == 0) continue;
        const int dim = kind_dim(k);
        const uint2 *blk = single_[k] >= 0 ? nullptr : d_blk_[k];
        unsigned long long *q = d_queue_ + (size_t)kQueueWords * k;
        const int *xo = d_xoff_ + 16 * k;
        if (!kind_fp64(k))
            ENG_TRY(launch_pass_persist<float>(dim, kind_coh_[k], d_tabf_, blk, xo, d_scal_, nblk_[k], rounds_, rounds,
                                               single_[k], d_err_, q, st));
        else
            ENG_TRY(launch_pass_persist<double>(dim, kind_coh_[k], d_tabd_, blk, xo, d_scal_, nblk_[k], rounds_,
                                                rounds, single_[k], d_err_, q, st));
        if (recording_) {
            int r = record_timing(k, st, err);
            if (r) return r;
        }
    }
    return launch_rounds(rounds, st, err);
}

int Engine::capture(hipStream_t st, std::string *err)
{
    if (gexec_) {
        (void)hipGraphExecDestroy(gexec_);
        gexec_ = nullptr;
    }
    hipGraph_t g = nullptr;
    ENG_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int r = launch_rounds(kGraphRounds, st, err);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    ENG_TRY(e);
    e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    ENG_TRY(e);
    graph_parity_ = (int)(rounds_ & 1);
    return RN_OK;
}

int Engine::launch_chunk(int rounds, hipStream_t st, std::string *err)
{
    if (active_.empty()) return RN_OK;
    if (dirty_) {
        int r = rebuild(st, err);
        if (r) return r;
        if (gexec_) {
            (void)hipGraphExecDestroy(gexec_);
            gexec_ = nullptr;
        }
    }
    peak_active_ = std::max(peak_active_, (int)active_.size());
    int kinds = 0;
    for (int k = 0; k < kKinds; ++k) kinds += nblk_[k] ? 1 : 0;
    tkind_[next_mirror_].clear();
    if (use_graph_ && rounds >= kGraphRounds) {
        // whole graphs only: the chunk is rounded up to a multiple of the
        // graph's (even) round count, so every replay starts on its parity
        const int reps = (rounds + kGraphRounds - 1) / kGraphRounds;
        if (!gexec_ || graph_parity_ != (int)(rounds_ & 1)) {
            int r = capture(st, err);
            if (r) return r;
        }
        for (int i = 0; i < reps; ++i) ENG_TRY(hipGraphLaunch(gexec_, st));
        rounds = reps * kGraphRounds;
    } else {
        // with timing on, events bracket every launch of this chunk
        recording_ = timing_;
        tmirror_ = next_mirror_;
        tkind_[tmirror_].clear();
        if (recording_) {
            int r = record_timing(-1, st, err);
            if (r) {
                recording_ = false;
                return r;
            }
        }
        int r = persist_ ? launch_persistent(rounds, st, err) : launch_rounds(rounds, st, err);
        recording_ = false;
        if (r) return r;
    }
    rounds_ += rounds;
    for (int k = 0; k < kKinds; ++k)
        if (nblk_[k]) launches_ += (persist_ && kind_coh_[k] != 0) ? 1 : rounds;
    int hi = 0;
    for (Net *n : active_) hi = std::max(hi, n->slot + 1);
    const int b = next_mirror_;
    ENG_TRY(hipMemcpyAsync(h_scal_[b], d_scal_, sizeof(Scalars) * hi, hipMemcpyDeviceToHost, st));
    if (persist_) ENG_TRY(hipMemcpyAsync(h_err_ + 16 * b, d_err_, 8 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
    ENG_TRY(hipEventRecord(ev_chunk_[b], st));
    mirror_hi_[b] = hi;
    mirror_seq_[b] = ++chunk_seq_;
    mirror_rounds_[b] = rounds;
    outstanding_.push_back(b);
    next_mirror_ ^= 1;
    return RN_OK;
}

int Engine::collect(std::vector<Net *> *finished, bool all, hipStream_t st, std::string *err)
{
    while (!outstanding_.empty() && (all || outstanding_.size() >= 2)) {
        const int b = outstanding_.front();
        outstanding_.pop_front();
        ENG_TRY(hipEventSynchronize(ev_chunk_[b]));
        if (persist_ && h_err_[16 * b] != 0) {
            const unsigned *e = h_err_ + 16 * b;
            if (err)
                *err = "persistent pass kernel: a wait for a network's previous pass exceeded its bound (slot " +
                       std::to_string(e[1]) + ", passes needed " + std::to_string(e[2]) + ", seen " +
                       std::to_string(e[3]) + ", mode " + std::to_string(e[4]) + ", round " + std::to_string(e[5]) +
                       " of the launch, table entry " + std::to_string(e[6]) + ")";
            return RN_EDEVICE;
        }
        for (size_t i = 0; i < tkind_[b].size(); ++i) {
            float ms = 0.f;
            ENG_TRY(hipEventElapsedTime(&ms, tev_[b][i], tev_[b][i + 1]));
            kind_s_[tkind_[b][i]] += 1e-3 * (double)ms;
            kind_n_[tkind_[b][i]] += 1;
        }
        tkind_[b].clear();
        const int in_flight = outstanding_.empty() ? 0 : mirror_rounds_[outstanding_.front()];
        double min_remain = 1e30;
        int64_t min_iters = INT64_MAX;
        std::vector<Net *> keep;
        keep.reserve(active_.size());
        for (Net *n : active_) {
            if (n->first_chunk > mirror_seq_[b] || n->slot >= mirror_hi_[b]) {
                keep.push_back(n);
                continue;
            }
            const Scalars &h = h_scal_[b][n->slot];
            if (h.mode == MODE_DONE) {
                int r = finalize(n, h, st, err);
                if (r) return r;
                if (finished) finished->push_back(n);
                dirty_ = true;
                continue;
            }
            keep.push_back(n);
            // remaining iterations from the observed convergence rate
            if (n->prev_est > 0.0 && h.est_rel > 0.0 && h.est_rel < n->prev_est && h.iters > n->prev_iters) {
                const double rate = std::log(n->prev_est / h.est_rel) / (double)(h.iters - n->prev_iters);
                const double remain = std::log(std::max(h.est_rel / h.tol, 1.0)) / rate;
                min_remain = std::min(min_remain, remain);
            }
            n->prev_est = h.est_rel;
            n->prev_iters = h.iters;
            min_iters = std::min(min_iters, h.iters);
        }
        active_.swap(keep);
        // next chunk: the predicted remaining iterations of the closest network,
        // less what is already in flight; rounds issued after a network
        // converges are idle, so the chunk also stays below a quarter of the
        // iterations done so far (a bound on the overshoot of fast solves)
        int next = std::min(chunk_ * 2, 256);
        if (min_remain < 1e29) next = (int)std::min(256.0, std::max(8.0, 0.9 * min_remain - in_flight));
        if (min_iters != INT64_MAX) next = (int)std::min<int64_t>(next, std::max<int64_t>(16, min_iters / 4));
        chunk_ = active_.empty() ? 16 : next;
    }
    return RN_OK;
}

void Engine::abort_all()
{
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    active_.clear();
    outstanding_.clear();
    for (auto &v : tkind_) v.clear();
    free_slots_.clear();
    for (int s = kSlots - 1; s >= 0; --s) free_slots_.push_back(s);
    for (auto &b : by_slot_) b = nullptr;
    dirty_ = true;
    chunk_ = 16;
}

int Engine::finalize(Net *net, const Scalars &h, hipStream_t st, std::string *err)
{
    const rn_problem *p = &net->prob;
    const Layout &L = net->L;
    char *base = net->base;
    const size_t n = (size_t)L.n;
    rn_result &r = net->res;
    r.status = h.status;
    r.converged = h.converged;
    r.Q_in = h.Q_in;
    r.Q_out = h.Q_out;
    r.G = h.Q_in - h.xr;
    r.K = r.G * (double)(net->na - 1) / cross_section(p);
    r.rel_resid = h.rel_resid;
    r.iters = h.iters;
    r.refreshes = h.refreshes;
    r.n_live = net->n_live;
    r.passes = rounds_ - net->round0;
    if (r.status == 0 && !r.converged) r.status = RN_ENOCONV;
    net->status = r.status;
    const double *P_final = (const double *)(base + L.off_P) + (size_t)(h.refreshes & 1) * n;
    const hipMemcpyKind kd = p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    ENG_TRY(hipEventRecord(net->ev_d, st));
    // the output copies wait for every launch issued so far (the network's
    // last pass may be in a chunk still in flight) and then run on the side
    // stream, so that copies to host memory do not hold up the next chunk
    const hipStream_t so = (side_ && (p->p_out || p->mask_out)) ? side_ : st;
    if (so != st) ENG_TRY(hipStreamWaitEvent(so, net->ev_d, 0));
    if (p->p_out) ENG_TRY(hipMemcpyAsync(p->p_out, P_final, 8 * n, kd, so));
    if (p->mask_out) ENG_TRY(hipMemcpyAsync(p->mask_out, base + L.off_mask, n, kd, so));
    ENG_TRY(hipEventRecord(net->ev, so));
    by_slot_[net->slot] = nullptr;
    free_slots_.push_back(net->slot);
    net->slot = -1;
    net->phase = NET_FINISHING;
    return RN_OK;
}

}  // namespace rn
