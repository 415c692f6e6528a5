// rn_api.cpp -- C ABI of librn (include/rn.h).
//
// Every solve goes through one scheduler per context: a submitted network
// waits for device memory (the HBM budget) and a control slot, is prepared
// (upload, validation, connectivity), joins the engine's pass rounds at the
// next chunk boundary, and leaves it as soon as it converges, releasing its
// memory for the next one (continuous batching). rn_solve and rn_solve_batch
// drive the scheduler on the calling thread; rn_submit starts a server thread
// that drives it in the background.
#include "rn_runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

using namespace rn;

struct rn_server {
    std::thread th;
    std::condition_variable cv;
    bool stop = false;
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

// ------------------------------------------------------------------ scheduler state
struct Sched {
    std::deque<Net *> waiting;       // submitted; waiting for memory or a control slot
    std::vector<Net *> preparing;    // setup enqueued; counters not yet on the host
    std::vector<Net *> finishing;    // outputs enqueued; waiting for their copies
    std::map<uint64_t, Net *> all;   // submitted through rn_submit and not yet collected
    uint64_t next_ticket = 1;
};

std::mutex g_sched_mu;
std::map<const rn_ctx *, Sched *> g_sched;

Sched *sched_of(const rn_ctx *ctx)
{
    std::lock_guard<std::mutex> lk(g_sched_mu);
    auto it = g_sched.find(ctx);
    return it == g_sched.end() ? nullptr : it->second;
}

void fail_net(Net *net, int status)
{
    net->status = status;
    std::memset(&net->res, 0, sizeof(net->res));
    net->res.status = status;
    net->phase = NET_DONE;
}

double elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (!a || !b || hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

// One scheduling step; the caller holds ctx->call_mu. Returns RN_OK or RN_EDEVICE.
int tick(rn_ctx *ctx, Sched *S, bool *progressed)
{
    *progressed = false;
    hipStream_t st = ctx->stream;
    // on a caller's stream everything stays on it (the caller's work that
    // produces device inputs is ordered before the setup)
    ctx->engine.set_side(ctx->stream == ctx->own ? ctx->side : nullptr);
    // 1. admit waiting networks while memory and control slots allow. The
    // head of the queue goes first; when it does not fit the memory free now,
    // later requests that fit may go ahead of it (first fit), each such pass
    // counted on the head, until it has been passed kMaxBypass times: then
    // nothing overtakes it until it is admitted, so a large request waits for
    // memory at most that many admissions longer than in first-in first-out.
    constexpr int kMaxBypass = 8;
    size_t i = 0;
    while (i < S->waiting.size() && !ctx->engine.full()) {
        Net *net = S->waiting[i];
        const bool head = i == 0;
        void *p = nullptr;
        hipError_t he = hipSuccess;
        // optional cap on the memory of the networks in flight (RN_ACTIVE_BYTES)
        const bool capped = ctx->active_cap && ctx->pool.in_use() > 0 &&
                            ctx->pool.in_use() + net->L.total > ctx->active_cap;
        if (!capped) p = ctx->pool.alloc(net->L.total, &he);
        if (!p) {
            if (he != hipSuccess) {              // the device itself is out of memory
                S->waiting.erase(S->waiting.begin() + (long)i);
                fail_net(net, RN_ENOMEM);
                *progressed = true;
                continue;
            }
            if (head && S->preparing.empty() && S->finishing.empty() && ctx->engine.active_count() == 0 &&
                ctx->engine.outstanding() == 0) {
                // nothing runs that could return memory: waiting would never end
                S->waiting.pop_front();
                fail_net(net, RN_ENOMEM);
                *progressed = true;
                continue;
            }
            if (S->waiting.front()->bypassed >= kMaxBypass) break;   // the head's turn
            ++i;                                 // a later, smaller request may fit
            continue;
        }
        if (!head) S->waiting.front()->bypassed += 1;
        S->waiting.erase(S->waiting.begin() + (long)i);
        net->base = (char *)p;
        int r = ctx->engine.prepare(net, st, &ctx->err);
        if (r) return r;
        S->preparing.push_back(net);
        *progressed = true;
    }
    // 2. prepared networks: activate them (or finish them at once)
    for (size_t i = 0; i < S->preparing.size();) {
        Net *net = S->preparing[i];
        const hipError_t q = hipEventQuery(net->ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        RN_TRY(q);
        S->preparing.erase(S->preparing.begin() + i);
        int r = ctx->engine.after_prepare(net, st, &ctx->err);
        if (r == RN_EDEVICE) return r;
        if (net->phase == NET_FINISHING) S->finishing.push_back(net);
        if (net->phase == NET_DONE) {           // invalid values: nothing was written
            ctx->pool.free(net->base);
            net->base = nullptr;
        }
        *progressed = true;
    }
    // 3. one chunk of pass rounds for every active network
    std::vector<Net *> fin;
    if (ctx->engine.active_count() > 0) {
        int r = ctx->engine.launch_chunk(ctx->engine.next_chunk(), st, &ctx->err);
        if (r) return r;
        r = ctx->engine.collect(&fin, false, st, &ctx->err);
        if (r) return r;
        *progressed = true;
    } else if (ctx->engine.outstanding() > 0) {
        int r = ctx->engine.collect(&fin, true, st, &ctx->err);
        if (r) return r;
        *progressed = true;
    }
    for (Net *n : fin) S->finishing.push_back(n);
    // 4. finished networks whose outputs have landed: release their memory
    for (size_t i = 0; i < S->finishing.size();) {
        Net *net = S->finishing[i];
        const hipError_t q = hipEventQuery(net->ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        RN_TRY(q);
        S->finishing.erase(S->finishing.begin() + i);
        ctx->pool.free(net->base);
        net->base = nullptr;
        net->res.t_mask_s = elapsed(net->ev_a, net->ev_b);
        net->res.t_loop_s = elapsed(net->ev_c, net->ev_d);
        net->res.t_total_s = now_s() - net->t_start;
        net->phase = NET_DONE;
        *progressed = true;
    }
    return RN_OK;
}

bool busy(const rn_ctx *ctx, const Sched *S)
{
    return !S->waiting.empty() || !S->preparing.empty() || !S->finishing.empty() ||
           ctx->engine.active_count() > 0 || ctx->engine.outstanding() > 0;
}

// Block while nothing can progress (only setup or output copies in flight).
void idle_wait(Sched *S)
{
    if (!S->preparing.empty()) (void)hipEventSynchronize(S->preparing.front()->ev);
    else if (!S->finishing.empty()) (void)hipEventSynchronize(S->finishing.front()->ev);
    else std::this_thread::sleep_for(std::chrono::microseconds(50));
}

// A network record (validated, laid out) for the scheduler.
int make_net(rn_ctx *ctx, const rn_problem *p, const rn_opts *opts, Net **out)
{
    int st = check_shape(p);
    if (st) return st;
    rn_opts o;
    if (opts) o = *opts;
    else rn_opts_default(&o);
    if ((st = check_opts(&o))) return st;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    Net *net = new Net();
    net->prob = *p;
    net->opts = o;
    net->L = make_layout(p, &o);
    if (net->L.total > ctx->pool.budget()) {
        delete net;
        return RN_ENOMEM;
    }
    net->t_start = now_s();
    *out = net;
    return RN_OK;
}

void release_net(Net *net)
{
    for (hipEvent_t e : {net->ev, net->ev_a, net->ev_b, net->ev_c, net->ev_d})
        if (e) (void)hipEventDestroy(e);
    delete net;
}

// Drive the scheduler on this thread until every listed network is done.
int drive_until(rn_ctx *ctx, Sched *S, const std::vector<Net *> &nets)
{
    auto all_done = [&]() {
        for (Net *n : nets)
            if (n->phase != NET_DONE) return false;
        return true;
    };
    while (!all_done()) {
        bool prog = false;
        int r = tick(ctx, S, &prog);
        if (r) return r;
        if (!prog) idle_wait(S);
    }
    return RN_OK;
}

void fail_all(rn_ctx *ctx, Sched *S, int status)
{
    ctx->engine.abort_all();
    for (Net *n : S->waiting) fail_net(n, status);
    for (Net *n : S->preparing) fail_net(n, status);
    for (Net *n : S->finishing) fail_net(n, status);
    for (auto &kv : S->all)
        if (kv.second->phase != NET_DONE) fail_net(kv.second, status);
    S->waiting.clear();
    S->preparing.clear();
    S->finishing.clear();
}

// Lock held by an API call; the server thread yields the context to it.
struct CallLock {
    rn_ctx *ctx;
    std::unique_lock<std::mutex> lk;
    explicit CallLock(rn_ctx *c) : ctx(c)
    {
        ctx->callers.fetch_add(1);
        lk = std::unique_lock<std::mutex>(ctx->call_mu);
        ctx->callers.fetch_sub(1);
    }
};

void server_main(rn_ctx *ctx)
{
    Sched *S = sched_of(ctx);
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->call_mu);
    bool broken = false;
    while (!ctx->server->stop) {
        if (broken || !busy(ctx, S)) {
            ctx->server->cv.wait_for(lk, std::chrono::milliseconds(20));
            if (broken) fail_all(ctx, S, RN_EDEVICE);
            continue;
        }
        bool prog = false;
        if (tick(ctx, S, &prog)) {
            // a device error fails every network in flight; the context is unusable
            broken = true;
            fail_all(ctx, S, RN_EDEVICE);
            continue;
        }
        if (!prog) {
            lk.unlock();
            idle_wait(S);
            lk.lock();
        } else if (ctx->callers.load() > 0) {
            // let submitters and pollers in between chunks
            lk.unlock();
            for (int spin = 0; spin < 1000 && ctx->callers.load() > 0; ++spin)
                std::this_thread::sleep_for(std::chrono::microseconds(5));
            lk.lock();
        }
    }
}

// ------------------------------------------------------------------ solves on the backbone
// RN_OPT_BACKBONE: before the engine sees the network, its bonds are copied
// to the device, the mask and the backbone are built, the pieces of dangling
// nodes and the backbone node each hangs from are found, and every bond with
// a dangling end is zeroed in the copy. The engine then solves that copy
// (device bonds, device pressures); afterwards the dangling nodes take the
// pressure of their backbone node and the outputs go to the caller.
struct BackbonePrep {
    rn_problem q{};               // the problem the engine solves
    char *aux = nullptr;          // pruned bonds | mask | uf | att | pressures (host callers) | counters
    uint8_t *mask = nullptr;
    int *uf = nullptr, *att = nullptr;
    int64_t n_live = 0, n_backbone = 0;
};

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t backbone_aux_bytes(const rn_problem *p)
{
    const size_t n = (size_t)(p->nx * p->ny * p->nz);
    return a256(8 * (size_t)p->dim * n) + a256(n) + 2 * a256(4 * n) + a256(8 * n) + 256;
}

static size_t backbone_transient_bytes(const rn_problem *p)
{
    const int64_t n = p->nx * p->ny * p->nz;
    return a256(8 * (size_t)n) + backbone_scratch_bytes(n);
}

// Caller holds call_mu and the device is current; the server is not running.
static int backbone_prepare(rn_ctx *ctx, const rn_problem *p, BackbonePrep *b)
{
    const int64_t n = p->nx * p->ny * p->nz;
    if (n + 2 > (int64_t)INT32_MAX) return RN_EINVAL;
    const size_t nn = (size_t)n;
    hipError_t he;
    b->aux = (char *)ctx->pool.alloc(backbone_aux_bytes(p), &he);
    if (!b->aux) return RN_ENOMEM;
    char *tr = (char *)ctx->pool.alloc(backbone_transient_bytes(p), &he);
    if (!tr) return RN_ENOMEM;
    hipStream_t st = ctx->stream;
    char *q = b->aux;
    double *g[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < p->dim; ++k) g[k] = (double *)q + (size_t)k * nn;
    q += a256(8 * (size_t)p->dim * nn);
    b->mask = (uint8_t *)q;
    q += a256(nn);
    b->uf = (int *)q;
    q += a256(4 * nn);
    b->att = (int *)q;
    q += a256(4 * nn);
    double *P = (double *)q;
    q += a256(8 * nn);
    unsigned long long *cnt = (unsigned long long *)q;
    unsigned long long *hc = ctx->h_small;
    const Lat lat = make_lat(p);
    const double *gc[3] = {g[0], g[1], g[2]};
    auto fail = [&](int r) {
        (void)hipStreamSynchronize(st);
        ctx->pool.free(tr);
        return r;
    };
    for (int k = 0; k < p->dim; ++k)
        if (hipMemcpyAsync(g[k], p->g[k], 8 * nn, p->mem == RN_MEM_HOST ? hipMemcpyHostToDevice
                                                                           : hipMemcpyDeviceToDevice, st) != hipSuccess)
            return fail(RN_EDEVICE);
    if (launch_clear_u64(cnt, 4, st) != hipSuccess) return fail(RN_EDEVICE);
    if (p->mem == RN_MEM_DEVICE) {
        if (launch_validate(lat, gc, cnt + 1, st) != hipSuccess) return fail(RN_EDEVICE);
        if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(RN_EDEVICE);
        if (hc[1] != 0) return fail(RN_EINVAL);
    }
    if (launch_mask(lat, gc, (int *)tr, (unsigned *)(tr + 4 * nn), b->mask, nullptr, cnt, true, st) != hipSuccess)
        return fail(RN_EDEVICE);
    const int n_axis = p->axis == 0 ? (int)p->nx : (p->axis == 1 ? (int)p->ny : (int)p->nz);
    if (n_axis >= 3 && launch_backbone(lat, gc, b->mask, tr + a256(8 * nn), cnt + 2, (int *)ctx->h_small, nullptr,
                                       st) != hipSuccess)
        return fail(RN_EDEVICE);
    if (launch_backbone_prune(lat, gc, g, b->mask, b->uf, b->att, st) != hipSuccess) return fail(RN_EDEVICE);
    if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(RN_EDEVICE);
    b->n_live = (int64_t)hc[0];
    b->n_backbone = (int64_t)hc[2];
    ctx->pool.free(tr);
    b->q = *p;
    for (int k = 0; k < 3; ++k) b->q.g[k] = k < p->dim ? g[k] : nullptr;
    b->q.mem = RN_MEM_DEVICE;
    b->q.mask_out = nullptr;
    b->q.p_out = p->p_out ? (p->mem == RN_MEM_DEVICE ? p->p_out : P) : nullptr;
    return RN_OK;
}

// Caller holds call_mu and the device is current.
static int backbone_finish(rn_ctx *ctx, const rn_problem *p, BackbonePrep *b, rn_result *r)
{
    const size_t nn = (size_t)(p->nx * p->ny * p->nz);
    hipStream_t st = ctx->stream;
    const Lat lat = make_lat(p);
    const hipMemcpyKind kind = p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (p->p_out) {
        RN_TRY(launch_backbone_fill(lat, b->mask, b->uf, b->att, b->q.p_out, st));
        if (p->mem == RN_MEM_HOST) RN_TRY(hipMemcpyAsync(p->p_out, b->q.p_out, 8 * nn, kind, st));
    }
    if (p->mask_out) RN_TRY(hipMemcpyAsync(p->mask_out, b->mask, nn, kind, st));
    RN_TRY(hipStreamSynchronize(st));
    r->n_live = b->n_live;
    r->n_backbone = b->n_backbone;
    return RN_OK;
}

// ------------------------------------------------------------------ compact solves
// RN_OPT_COMPACT: the CG runs on the list of the nodes that take part (the
// live set, or the backbone with RN_OPT_BACKBONE) through neighbour slots, on
// the caller's thread, outside the engine. Returns RN_OK with *done = false
// when nothing takes part (the engine then handles the network: direct
// inlet-outlet bonds, dead pressures). Caller holds call_mu, device current.
static int compact_solve(rn_ctx *ctx, const rn_problem *p, const rn_opts *o, rn_result *out, bool *done)
{
    *done = false;
    const double t0 = now_s();
    const int64_t n = p->nx * p->ny * p->nz;
    if (n + 2 > (int64_t)INT32_MAX) return RN_EINVAL;
    const size_t nn = (size_t)n;
    const bool backbone = (o->flags & RN_OPT_BACKBONE) != 0;
    const bool f32 = o->precision == RN_MIXED;
    const size_t s = f32 ? 4 : 8;
    const int slots = 2 * p->dim;
    const int nb = compact_blocks(n);
    hipStream_t st = ctx->stream;
    const hipMemcpyKind kind = p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    // lattice-side buffers: bonds (host input), mask, field, the pieces of
    // dangling nodes, counters and index scans; then the transient arrays of
    // the mask and the backbone
    const bool copy_g = p->mem == RN_MEM_HOST;
    const size_t off_g = 0, off_mask = off_g + a256(copy_g ? 8 * (size_t)p->dim * nn : 0),
                 off_P = off_mask + a256(nn), off_uf = off_P + a256(8 * nn),
                 off_att = off_uf + a256(backbone ? 4 * nn : 0), off_cmap = off_att + a256(backbone ? 4 * nn : 0),
                 off_cnt = off_cmap + a256(4 * nn), off_scan = off_cnt + 256,
                 lat_bytes = off_scan + a256(4 * (2 * (size_t)nb + 1));
    hipError_t he;
    char *lb = (char *)ctx->pool.alloc(lat_bytes, &he);
    if (!lb) return RN_ENOMEM;
    char *tr = (char *)ctx->pool.alloc(a256(8 * nn) + (backbone ? backbone_scratch_bytes(n) : 0), &he);
    char *cb = nullptr;
    auto finish = [&](int r) {
        (void)hipStreamSynchronize(st);
        if (tr) ctx->pool.free(tr);
        if (cb) ctx->pool.free(cb);
        ctx->pool.free(lb);
        return r;
    };
    if (!tr) return finish(RN_ENOMEM);
    const double *g[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < p->dim; ++k) {
        if (copy_g) {
            double *dst = (double *)(lb + off_g) + (size_t)k * nn;
            if (hipMemcpyAsync(dst, p->g[k], 8 * nn, hipMemcpyHostToDevice, st) != hipSuccess) return finish(RN_EDEVICE);
            g[k] = dst;
        } else {
            g[k] = p->g[k];
        }
    }
    uint8_t *mask = (uint8_t *)(lb + off_mask);
    double *Pl = (double *)(lb + off_P);
    int *uf = (int *)(lb + off_uf), *att = (int *)(lb + off_att), *cmap = (int *)(lb + off_cmap);
    unsigned long long *cnt = (unsigned long long *)(lb + off_cnt);
    int *counts = (int *)(lb + off_scan), *offsets = counts + nb;
    unsigned long long *hc = ctx->h_small;
    const Lat lat = make_lat(p);
    if (launch_clear_u64(cnt, 4, st) != hipSuccess) return finish(RN_EDEVICE);
    if (!copy_g) {
        if (launch_validate(lat, g, cnt + 1, st) != hipSuccess) return finish(RN_EDEVICE);
        if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return finish(RN_EDEVICE);
        if (hc[1] != 0) return finish(RN_EINVAL);
    }
    if (launch_mask(lat, g, (int *)tr, (unsigned *)(tr + 4 * nn), mask, Pl, cnt, o->x0 == RN_X0_LINEAR, st) !=
        hipSuccess)
        return finish(RN_EDEVICE);
    const int n_axis = p->axis == 0 ? (int)p->nx : (p->axis == 1 ? (int)p->ny : (int)p->nz);
    if (backbone && n_axis >= 3) {
        if (launch_backbone(lat, g, mask, tr + a256(8 * nn), cnt + 2, (int *)ctx->h_small, nullptr, st) != hipSuccess)
            return finish(RN_EDEVICE);
        if (launch_backbone_prune(lat, g, nullptr, mask, uf, att, st) != hipSuccess) return finish(RN_EDEVICE);
    }
    if (launch_compact_index(mask, n, backbone ? 11 : 3, counts, offsets, (int *)tr, cmap, st) != hipSuccess)
        return finish(RN_EDEVICE);
    int mh = 0;
    if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&mh, offsets + nb, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return finish(RN_EDEVICE);
    const int64_t n_live = (int64_t)hc[0], n_bb = backbone ? (int64_t)hc[2] : 0;
    const int m = mh;
    if (m == 0) return finish(RN_OK);           // nothing takes part: the engine's path
    // member-side buffers (the member list is moved out of the transient area first)
    int grid = (int)std::min<int64_t>(((int64_t)m + kBlock - 1) / kBlock, 4096);
    grid = (grid + 7) & ~7;
    int groups = 1;
    while (groups < kGroupsMax && groups * 2 * 64 <= grid) groups *= 2;
    const size_t off_idx = 0, off_nbr = a256(4 * (size_t)m), off_gT = off_nbr + a256(4 * (size_t)slots * m),
                 off_g64 = off_gT + a256(s * slots * m), off_d = off_g64 + a256(8 * (size_t)slots * m),
                 off_P0 = off_d + a256(s * m), off_P1 = off_P0 + a256(8 * (size_t)m),
                 off_z = off_P1 + a256(8 * (size_t)m), off_u = off_z + a256(s * m), off_p = off_u + a256(s * m),
                 off_part = off_p + a256(s * m), off_tk = off_part + a256(8 * kRed * (size_t)grid),
                 off_sc = off_tk + a256(ticket_bytes(groups)), cbytes = off_sc + a256(sizeof(Scalars));
    cb = (char *)ctx->pool.alloc(cbytes, &he);
    if (!cb) return finish(RN_ENOMEM);
    int *idx = (int *)(cb + off_idx);
    if (hipMemcpyAsync(idx, tr, 4 * (size_t)m, hipMemcpyDeviceToDevice, st) != hipSuccess) return finish(RN_EDEVICE);
    Scalars *ds = (Scalars *)(cb + off_sc);
    static_assert(sizeof(Scalars) <= 32 * sizeof(unsigned long long), "control block staged in h_small");
    Scalars &init = *(Scalars *)ctx->h_small;   // pinned; read back into the same words later, in stream order
    std::memset(&init, 0, sizeof(init));
    init.mode = MODE_REFRESH;
    init.first = 1;
    init.fp32 = f32;
    init.max_iter = o->max_iter;
    init.sigma = init.sigma_next = 1.0;
    init.tol = o->tol;
    init.delta = f32 ? (o->delta > 0.0 ? o->delta : 0.1) : 0.0;
    init.kappa = init.bhat = 1.0;
    init.last_check = INFINITY;
    init.kpend = 2;                             // unused here: pass A applies each step in the next round
    if (hipMemcpyAsync(ds, &init, sizeof(init), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(cb + off_tk, 0, ticket_bytes(groups), st) != hipSuccess)
        return finish(RN_EDEVICE);
    auto run = [&](auto zero) -> int {
        using T = decltype(zero);
        CompactArgs<T> a;
        a.m = m;
        a.slots = slots;
        a.grid = grid;
        a.groups = groups;
        a.jacobi = o->precond == RN_JACOBI ? 1 : 0;
        a.nbr = (const int *)(cb + off_nbr);
        a.gT = (const T *)(cb + off_gT);
        a.g64 = (const double *)(cb + off_g64);
        a.d = (const T *)(cb + off_d);
        a.P[0] = (double *)(cb + off_P0);
        a.P[1] = (double *)(cb + off_P1);
        a.z = (T *)(cb + off_z);
        a.u = (T *)(cb + off_u);
        a.p = (T *)(cb + off_p);
        a.partials = (double *)(cb + off_part);
        a.tickets = (unsigned *)(cb + off_tk);
        if (launch_compact_tables<T>(lat, g, idx, cmap, m, (int *)a.nbr, (T *)a.gT, (double *)a.g64, (T *)a.d, Pl,
                                     a.P[0], a.z, a.u, a.p, st) != hipSuccess)
            return RN_EDEVICE;
        const double tl = now_s();
        int64_t rounds = 0;
        int chunk = 16;
        Scalars *hs = (Scalars *)ctx->h_small;
        while (true) {
            for (int r = 0; r < chunk; ++r)
                if (launch_compact_round<T>(a, ds, st) != hipSuccess) return RN_EDEVICE;
            rounds += chunk;
            if (hipMemcpyAsync(hs, ds, sizeof(Scalars), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return RN_EDEVICE;
            if (hs->mode == MODE_DONE) break;
            chunk = std::min(chunk * 2, 256);
        }
        const Scalars h = *hs;
        std::memset(out, 0, sizeof(*out));
        out->status = h.status;
        out->converged = h.converged;
        out->Q_in = h.Q_in;
        out->Q_out = h.Q_out;
        out->G = h.Q_in - h.xr;
        out->K = out->G * (double)(n_axis - 1) / cross_section(p);
        out->rel_resid = h.rel_resid;
        out->iters = h.iters;
        out->refreshes = h.refreshes;
        out->n_live = n_live;
        out->n_backbone = n_bb;
        out->passes = rounds;
        if (out->status == 0 && !out->converged) out->status = RN_ENOCONV;
        // outputs: the members' field into the lattice field, the dangling
        // ends' pressures from their backbone nodes, then the caller's buffers
        if (p->p_out) {
            if (launch_compact_scatter(idx, m, a.P[h.refreshes & 1], Pl, st) != hipSuccess) return RN_EDEVICE;
            if (backbone && n_axis >= 3 && launch_backbone_fill(lat, mask, uf, att, Pl, st) != hipSuccess)
                return RN_EDEVICE;
            if (hipMemcpyAsync(p->p_out, Pl, 8 * nn, kind, st) != hipSuccess) return RN_EDEVICE;
        }
        if (p->mask_out && hipMemcpyAsync(p->mask_out, mask, nn, kind, st) != hipSuccess) return RN_EDEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return RN_EDEVICE;
        out->t_loop_s = now_s() - tl;
        out->t_total_s = now_s() - t0;
        return RN_OK;
    };
    const int r = f32 ? run(0.0f) : run(0.0);
    if (r == RN_OK) *done = true;
    return finish(r);
}

int solve_many(rn_ctx *ctx, int32_t count, const rn_problem *probs, const rn_opts *opts, int32_t n_opts,
               rn_result *out)
{
    if (!ctx || !out || !probs || count < 1) return RN_EINVAL;
    if (!(n_opts == 0 || n_opts == 1 || n_opts == count)) return RN_EINVAL;
    if (n_opts > 0 && !opts) return RN_EINVAL;
    auto opts_of = [&](int i) { return n_opts == 0 ? nullptr : (n_opts == 1 ? opts : opts + i); };
    // solves with options the engine does not take: check them all first
    std::vector<char> flagged((size_t)count, 0);
    bool any = false;
    for (int i = 0; i < count; ++i) {
        const rn_opts *o = opts_of(i);
        if (!o || !(o->flags & (RN_OPT_BACKBONE | RN_OPT_COMPACT))) continue;
        int st = check_shape(probs + i);
        if (!st) st = check_opts(o);
        if (!st && probs[i].mem == RN_MEM_HOST && !host_values_ok(probs + i)) st = RN_EINVAL;
        if (!st && ctx->server) st = RN_EINVAL;      // the server owns the stream
        if (st) return st;
        flagged[(size_t)i] = 1;
        any = true;
    }
    // compact solves run here, one by one; solves on the backbone have their
    // bonds pruned before the engine sees them
    std::vector<BackbonePrep> bb((size_t)count);
    std::vector<char> on_bb((size_t)count, 0), done((size_t)count, 0);
    std::vector<rn_problem> eff(probs, probs + count);
    auto free_bb = [&]() {
        for (BackbonePrep &b : bb)
            if (b.aux) {
                ctx->pool.free(b.aux);
                b.aux = nullptr;
            }
    };
    if (any) {
        std::lock_guard<std::mutex> lk(ctx->call_mu);
        if (ctx->server) return RN_EINVAL;
        if (hipSetDevice(ctx->device) != hipSuccess) return RN_EDEVICE;
        for (int i = 0; i < count; ++i) {
            if (!flagged[(size_t)i]) continue;
            const rn_opts *o = opts_of(i);
            if (o->flags & RN_OPT_COMPACT) {
                bool fin = false;
                const int st = compact_solve(ctx, probs + i, o, out + i, &fin);
                if (st) {
                    free_bb();
                    return st;
                }
                if (fin) {
                    done[(size_t)i] = 1;
                    continue;
                }
            }
            if (o->flags & RN_OPT_BACKBONE) {
                const int st = backbone_prepare(ctx, probs + i, &bb[(size_t)i]);
                if (st) {
                    free_bb();
                    return st;
                }
                eff[(size_t)i] = bb[(size_t)i].q;
                on_bb[(size_t)i] = 1;
            }
        }
    }
    std::vector<Net *> nets((size_t)count, nullptr);
    std::vector<Net *> live;
    for (int i = 0; i < count; ++i) {
        if (done[(size_t)i]) continue;
        int st = make_net(ctx, &eff[(size_t)i], opts_of(i), &nets[i]);
        if (st) {
            for (Net *n : nets)
                if (n) release_net(n);
            free_bb();
            return st;
        }
        live.push_back(nets[i]);
    }
    Sched *S = sched_of(ctx);
    int r = RN_OK;
    if (!live.empty()) {
        if (ctx->server) {
            // the server thread drives: hand the networks over and wait for them
            {
                CallLock cl(ctx);
                for (Net *n : live) S->waiting.push_back(n);
            }
            ctx->server->cv.notify_all();
            while (true) {
                std::this_thread::sleep_for(std::chrono::microseconds(200));
                CallLock cl(ctx);
                bool all_done = true;
                for (Net *n : live) all_done = all_done && n->phase == NET_DONE;
                if (all_done) break;
            }
        } else {
            std::lock_guard<std::mutex> lk(ctx->call_mu);
            if (hipSetDevice(ctx->device) != hipSuccess) {
                for (Net *n : live) release_net(n);
                free_bb();
                return RN_EDEVICE;
            }
            for (Net *n : live) S->waiting.push_back(n);
            r = drive_until(ctx, S, live);
            if (r) {
                fail_all(ctx, S, r);
                (void)hipStreamSynchronize(ctx->stream);
                (void)hipStreamSynchronize(ctx->side);
            }
        }
    }
    int first = RN_OK;
    for (int i = 0; i < count; ++i) {
        if (done[(size_t)i]) {
            if (out[i].status != RN_OK && first == RN_OK) first = out[i].status;
            continue;
        }
        if (!r) out[i] = nets[i]->res;
        if (nets[i]->status != RN_OK && first == RN_OK) first = nets[i]->status;
        if (nets[i]->base) ctx->pool.free(nets[i]->base);
        release_net(nets[i]);
    }
    if (any && !r) {
        // outputs of the solves on the backbone (those that ran: RN_OK or RN_ENOCONV)
        std::lock_guard<std::mutex> lk(ctx->call_mu);
        for (int i = 0; i < count && !r; ++i)
            if (on_bb[(size_t)i] && (out[i].status == RN_OK || out[i].status == RN_ENOCONV))
                r = backbone_finish(ctx, probs + i, &bb[(size_t)i], out + i);
    }
    free_bb();
    return r ? r : first;
}

// ------------------------------------------------------------------ launch-shape search
// A trial runs `copies` identical networks of one size class together for
// kTrialPasses CG passes from x = 0 (the tolerance is out of reach), with one
// candidate shape installed for that class, and measures the device time of
// the pass launches per node and pass with the library's event timing. The
// copies make a round move about 2^25 nodes (tens of thousands of
// workgroups, as in the 512-network batch): a shape that is fastest for one
// small network alone, where a pass is bound by the latency of one tile, is
// not the fastest in a launch that fills the chip many times over.
constexpr int kTrialPasses = 64;
constexpr int kTrialRepeats = 2;     // each candidate is measured this often; the fastest run counts
constexpr double kTrialMargin = 0.97; // a candidate replaces the built-in shape only when this much faster
constexpr int64_t kTrialNodes = (int64_t)1 << 25;
constexpr int kTrialCopiesMax = 256;

int shape_trial(rn_ctx *ctx, int dim, int s, int side, int copies, const ShapeChoice &cand, double *ns_per_node)
{
    const int64_t n = dim == 2 ? (int64_t)side * side : (int64_t)side * side * side;
    ShapeTable t = shape_table_get();
    t.c[dim - 2][s == 4 ? 1 : 0][shape_class(n)] = cand;
    shape_table_install(t);
    std::vector<rn_problem> probs((size_t)copies);
    hipError_t he;
    char *gmem = (char *)ctx->pool.alloc((size_t)8 * dim * n * copies, &he);
    if (!gmem) return he != hipSuccess ? RN_EDEVICE : RN_ENOMEM;
    int r = RN_OK;
    for (int c = 0; c < copies && !r; ++c) {
        rn_problem &p = probs[(size_t)c];
        std::memset(&p, 0, sizeof(p));
        p.dim = dim;
        p.axis = 0;
        p.nx = p.ny = side;
        p.nz = dim == 3 ? side : 1;
        p.mem = RN_MEM_DEVICE;
        for (int k = 0; k < dim; ++k) {
            double *g = (double *)gmem + ((size_t)c * dim + k) * (size_t)n;
            p.g[k] = g;
            if (launch_fill_trial(g, n, (uint32_t)(977 * c + 131 * k + 7), ctx->stream) != hipSuccess) r = RN_EDEVICE;
        }
    }
    if (!r && hipStreamSynchronize(ctx->stream) != hipSuccess) r = RN_EDEVICE;
    if (!r) {
        rn_opts o;
        rn_opts_default(&o);
        o.precision = s == 4 ? RN_MIXED : RN_FP64;
        o.tol = 1e-30;
        o.max_iter = kTrialPasses;
        o.x0 = RN_X0_ZERO;
        std::vector<rn_result> res((size_t)copies);
        {
            std::lock_guard<std::mutex> lk(ctx->call_mu);
            ctx->engine.set_timing(true);
        }
        const int st = solve_many(ctx, copies, probs.data(), &o, 1, res.data());
        double secs = 0.0;
        {
            std::lock_guard<std::mutex> lk(ctx->call_mu);
            for (int k = 0; k < Engine::kKinds; ++k)
                if ((Engine::kind_path(k) == RN_PATH_3D) == (dim == 3) && Engine::kind_precision(k) == o.precision)
                    secs += ctx->engine.kind_seconds(k);
            ctx->engine.set_timing(false);
        }
        // per node and working pass: the launches of rounds after the copies
        // finished (until the host notices) count in the time but do no work
        int64_t passes = 0;
        for (const rn_result &x : res) passes = std::max(passes, x.iters + x.refreshes);
        if (st != RN_OK && st != RN_ENOCONV) r = st;
        else if (passes <= 0 || secs <= 0.0) r = RN_EDEVICE;
        else *ns_per_node = 1e9 * secs / ((double)passes * (double)copies * (double)n);
    }
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pool.free(gmem);
    return r;
}

}  // namespace

extern "C" {

int rn_version(void) { return 102; }

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
    o->precond = RN_JACOBI;
    o->tol = 1e-8;
    o->max_iter = 10000000;
    o->delta = 0.0;
    o->x0 = RN_X0_LINEAR;
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
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_sched[ctx] = new Sched();
    }
    auto fail = [&]() {
        rn_destroy(ctx);
        return RN_EDEVICE;
    };
    if (hipSetDevice(device) != hipSuccess) return fail();
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail();
    ctx->budget = budget ? budget : (size_t)(0.9 * (double)free_b);
    if (const char *cap = std::getenv("RN_ACTIVE_BYTES")) ctx->active_cap = (size_t)std::strtoull(cap, nullptr, 10);
    ctx->pool.set_budget(ctx->budget);
    if (hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess) return fail();
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess) return fail();
    ctx->stream = ctx->own;
    if (ctx->engine.init(ctx->stream, &ctx->err)) return fail();
    ctx->engine_ok = true;
    if (hipHostMalloc((void **)&ctx->h_small, 32 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
        return fail();
    // this device's copy of the static scratch of rn_build_mask_noalloc
    if (noalloc_setup(device) != hipSuccess) return fail();
    *out = ctx;
    return RN_OK;
}

int rn_destroy(rn_ctx *ctx)
{
    if (!ctx) return RN_OK;
    if (ctx->server) {
        {
            std::lock_guard<std::mutex> lk(ctx->call_mu);
            ctx->server->stop = true;
        }
        ctx->server->cv.notify_all();
        if (ctx->server->th.joinable()) ctx->server->th.join();
        delete ctx->server;
        ctx->server = nullptr;
    }
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    fbm_release(ctx);
    Sched *S = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        auto it = g_sched.find(ctx);
        if (it != g_sched.end()) {
            S = it->second;
            g_sched.erase(it);
        }
    }
    if (S) {
        for (auto &kv : S->all) release_net(kv.second);
        delete S;
    }
    if (ctx->engine_ok) ctx->engine.destroy();
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    ctx->pool.release_all();
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
    return RN_OK;
}

int rn_set_stream(rn_ctx *ctx, void *stream)
{
    if (!ctx) return RN_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (ctx->server) return RN_EINVAL;        // the server owns the stream once started
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
    size_t bytes = make_layout(p, o ? o : &d).total;
    if (o && (o->flags & RN_OPT_COMPACT)) {
        // the lattice side (bonds, mask, field, maps, transient arrays of the
        // mask and the backbone) and the member side with every node a member
        const size_t n = (size_t)(p->nx * p->ny * p->nz), s = o->precision == RN_MIXED ? 4 : 8;
        const size_t slots = 2 * (size_t)p->dim;
        return 8 * (size_t)p->dim * n + 25 * n + 8 * n + backbone_transient_bytes(p) +
               n * (4 + slots * (12 + s) + 4 * s + 16) + (1 << 20);
    }
    if (o && (o->flags & RN_OPT_BACKBONE))   // the pruned copy and its maps, plus the larger of the
        bytes += backbone_aux_bytes(p) +      // backbone's transient arrays and the solve itself
                 (backbone_transient_bytes(p) > bytes ? backbone_transient_bytes(p) - bytes : 0);
    return bytes;
}

int rn_plan(const rn_problem *p, const rn_opts *opts, rn_plan_t *out)
{
    if (!out) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    rn_opts o;
    if (opts) o = *opts;
    else rn_opts_default(&o);
    if ((st = check_opts(&o))) return st;
    const Layout L = make_layout(p, &o);
    std::memset(out, 0, sizeof(*out));
    if (p->dim == 3) {
        out->path = RN_PATH_3D;
        out->tile_x = kTX;
        out->tile_y = kTY;
        out->tile_z = L.tile_z;
    } else {
        const bool f32 = L.s == 4;
        out->path = L.shape ? RN_PATH_2D_SMALL : RN_PATH_2D_FULL;
        out->tile_x = L.shape ? kWave : kWave * (f32 ? kSEG2f : kSEG2d);
        out->tile_y = (kBlock / kWave) * (L.shape ? (f32 ? kTY2fS : kTY2dS) : (f32 ? kTY2f : kTY2d));
        out->tile_z = 1;
    }
    out->tiles_per_wg = L.tpw;
    out->tiles = L.ntiles;
    out->workgroups = L.grid;
    out->groups = L.groups;
    out->footprint = (int64_t)L.total;
    return RN_OK;
}

int rn_build_mask(rn_ctx *ctx, const rn_problem *p, int64_t *n_live_out)
{
    if (!ctx) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    if (!p->mask_out) return RN_EINVAL;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (ctx->server) return RN_EINVAL;        // the server owns the stream once started
    RN_TRY(hipSetDevice(ctx->device));
    // the mask needs the FP64 bonds (host input), the field scratch, the
    // mask, 8 bytes of labels per node and the counters
    const size_t n = (size_t)(p->nx * p->ny * p->nz);
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const bool copy_g = p->mem == RN_MEM_HOST;
    const size_t off_g = 0, off_P = off_g + a256(copy_g ? 8 * p->dim * n : 0), off_mask = off_P + a256(8 * n),
                 off_lab = off_mask + a256(n), off_cnt = off_lab + a256(8 * n), total = off_cnt + 256;
    hipError_t he;
    char *base = (char *)ctx->pool.alloc(total, &he);
    if (!base) return RN_ENOMEM;
    const Lat lat = make_lat(p);
    const double *gd[3] = {nullptr, nullptr, nullptr};
    auto done = [&](int r) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->pool.free(base);
        return r;
    };
    if (copy_g) {
        for (int k = 0; k < p->dim; ++k) {
            double *dst = (double *)(base + off_g) + (size_t)k * n;
            if (hipMemcpyAsync(dst, p->g[k], 8 * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
                return done(RN_EDEVICE);
            gd[k] = dst;
        }
    } else {
        for (int k = 0; k < p->dim; ++k) gd[k] = p->g[k];
    }
    unsigned long long *cnt = (unsigned long long *)(base + off_cnt);
    unsigned long long hc[4] = {0, 0, 0, 0};
    if (hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (!copy_g && launch_validate(lat, gd, cnt + 1, ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (launch_mask(lat, gd, (int *)(base + off_lab), (unsigned *)(base + off_lab + 4 * n),
                    (uint8_t *)(base + off_mask), (double *)(base + off_P), cnt, true, ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    if (hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (hc[1] != 0) return done(RN_EINVAL);
    if (hipMemcpyAsync(p->mask_out, base + off_mask, n,
                       p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    if (n_live_out) *n_live_out = (int64_t)hc[0];
    return done(RN_OK);
}

int rn_build_backbone(rn_ctx *ctx, const rn_problem *p, int64_t *n_live_out, int64_t *n_backbone_out)
{
    if (!ctx) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    if (!p->mask_out) return RN_EINVAL;
    if (p->mem == RN_MEM_HOST && !host_values_ok(p)) return RN_EINVAL;
    static_assert(kBackboneStage <= 64, "level offsets staged in the 32-word pinned buffer");
    const int64_t n = p->nx * p->ny * p->nz;
    if (n + 2 > (int64_t)INT32_MAX) return RN_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (ctx->server) return RN_EINVAL;        // the server owns the stream once started
    RN_TRY(hipSetDevice(ctx->device));
    // FP64 bonds (host input), the mask, the mask's labels (8 bytes per node),
    // the counters, then the backbone's own arrays
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t nn = (size_t)n;
    const bool copy_g = p->mem == RN_MEM_HOST;
    const size_t off_g = 0, off_mask = off_g + a256(copy_g ? 8 * p->dim * nn : 0), off_lab = off_mask + a256(nn),
                 off_cnt = off_lab + a256(8 * nn), off_bb = off_cnt + 256,
                 total = off_bb + backbone_scratch_bytes(n);
    hipError_t he;
    char *base = (char *)ctx->pool.alloc(total, &he);
    if (!base) return RN_ENOMEM;
    const Lat lat = make_lat(p);
    const double *gd[3] = {nullptr, nullptr, nullptr};
    auto done = [&](int r) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->pool.free(base);
        return r;
    };
    if (copy_g) {
        for (int k = 0; k < p->dim; ++k) {
            double *dst = (double *)(base + off_g) + (size_t)k * nn;
            if (hipMemcpyAsync(dst, p->g[k], 8 * nn, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
                return done(RN_EDEVICE);
            gd[k] = dst;
        }
    } else {
        for (int k = 0; k < p->dim; ++k) gd[k] = p->g[k];
    }
    unsigned long long *cnt = (unsigned long long *)(base + off_cnt);
    unsigned long long *hc = ctx->h_small;
    uint8_t *mask = (uint8_t *)(base + off_mask);
    if (launch_clear_u64(cnt, 4, ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (!copy_g && launch_validate(lat, gd, cnt + 1, ctx->stream) != hipSuccess) return done(RN_EDEVICE);
    if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    if (hc[1] != 0) return done(RN_EINVAL);
    if (launch_mask(lat, gd, (int *)(base + off_lab), (unsigned *)(base + off_lab + 4 * nn), mask, nullptr, cnt, true,
                    ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    // with fewer than 3 planes on the flow axis there is no interior node
    const int n_axis = p->axis == 0 ? (int)p->nx : (p->axis == 1 ? (int)p->ny : (int)p->nz);
    if (n_axis >= 3 && launch_backbone(lat, gd, mask, base + off_bb, cnt + 2, (int *)ctx->h_small, nullptr,
                                       ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    if (hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    const int64_t n_live = (int64_t)hc[0], n_bb = (int64_t)hc[2];
    if (hipMemcpyAsync(p->mask_out, mask, nn, p->mem == RN_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess)
        return done(RN_EDEVICE);
    if (n_live_out) *n_live_out = n_live;
    if (n_backbone_out) *n_backbone_out = n_bb;
    return done(RN_OK);
}

int rn_build_mask_noalloc(rn_ctx *ctx, const rn_problem *p, int64_t *n_live_out)
{
    if (!ctx) return RN_EINVAL;
    int st = check_shape(p);
    if (st) return st;
    if (!p->mask_out || p->mem != RN_MEM_DEVICE) return RN_EINVAL;
    const int64_t n = p->nx * p->ny * p->nz;
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    if (n > kNoAllocMaxNodes) {
        ctx->err = "rn_build_mask_noalloc: " + std::to_string(n) + " nodes exceed the static scratch of " +
                   std::to_string(kNoAllocMaxNodes) + " nodes";
        return RN_ENOMEM;
    }
    if (ctx->server) return RN_EINVAL;        // the server owns the stream once started
    RN_TRY(hipSetDevice(ctx->device));
    char *base = (char *)noalloc_scratch(ctx->device);
    if (!base) {
        ctx->err = "rn_build_mask_noalloc: no static scratch on this device";
        return RN_EDEVICE;
    }
    int *parent = (int *)base;
    unsigned *flags = (unsigned *)(base + 4 * (size_t)n);
    unsigned long long *cnt = (unsigned long long *)(base + kNoAllocCounterOffset);
    unsigned long long *hc = ctx->h_small;
    const Lat lat = make_lat(p);
    const double *gd[3] = {p->g[0], p->g[1], p->dim == 3 ? p->g[2] : nullptr};
    hipStream_t s = ctx->stream;
    // the counters keep the previous call's values: clear them, then check the
    // conductances before anything is written to mask_out
    RN_TRY(launch_clear_u64(cnt, 4, s));
    RN_TRY(launch_validate(lat, gd, cnt + 1, s));
    RN_TRY(hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    RN_TRY(hipStreamSynchronize(s));
    if (hc[1] != 0) return RN_EINVAL;
    RN_TRY(launch_mask(lat, gd, parent, flags, p->mask_out, nullptr, cnt, true, s));
    RN_TRY(hipMemcpyAsync(hc, cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    RN_TRY(hipStreamSynchronize(s));
    if (n_live_out) *n_live_out = (int64_t)hc[0];
    return RN_OK;
}

int rn_solve(rn_ctx *ctx, const rn_problem *p, const rn_opts *opts, rn_result *out)
{
    if (!ctx || !out) return RN_EINVAL;
    return solve_many(ctx, 1, p, opts, opts ? 1 : 0, out);
}

int rn_solve_batch(rn_ctx *ctx, int32_t count, const rn_problem *probs, const rn_opts *opts, int32_t n_opts,
                   rn_result *out)
{
    return solve_many(ctx, count, probs, opts, n_opts, out);
}

int rn_submit(rn_ctx *ctx, const rn_problem *p, const rn_opts *opts, uint64_t *ticket_out)
{
    if (!ctx || !ticket_out) return RN_EINVAL;
    if (opts && (opts->flags & (RN_OPT_BACKBONE | RN_OPT_COMPACT))) return RN_EINVAL;   // rn_solve(_batch) only
    Net *net = nullptr;
    int st = make_net(ctx, p, opts, &net);
    if (st) return st;
    Sched *S = sched_of(ctx);
    CallLock cl(ctx);
    if (!ctx->server) {
        ctx->server = new rn_server();
        ctx->server->th = std::thread(server_main, ctx);
    }
    net->ticket = S->next_ticket++;
    S->all[net->ticket] = net;
    S->waiting.push_back(net);
    *ticket_out = net->ticket;
    ctx->server->cv.notify_all();
    return RN_OK;
}

int rn_poll(rn_ctx *ctx, uint64_t ticket, rn_result *out)
{
    if (!ctx || !out) return RN_EINVAL;
    Sched *S = sched_of(ctx);
    CallLock cl(ctx);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return RN_ENOTFOUND;
    Net *net = it->second;
    if (net->phase != NET_DONE) return RN_EAGAIN;
    *out = net->res;
    const int st = net->status;
    S->all.erase(it);
    release_net(net);
    return st;
}

int rn_stats(rn_ctx *ctx, rn_stats_t *out)
{
    if (!ctx || !out) return RN_EINVAL;
    Sched *S = sched_of(ctx);
    CallLock cl(ctx);
    std::memset(out, 0, sizeof(*out));
    out->waiting = (int64_t)S->waiting.size();
    out->preparing = (int64_t)S->preparing.size();
    out->active = ctx->engine.active_count();
    out->finishing = (int64_t)S->finishing.size();
    out->bytes_in_use = (int64_t)ctx->pool.in_use();
    out->budget = (int64_t)ctx->pool.budget();
    out->launches = ctx->engine.launches();
    out->peak_active = ctx->engine.peak_active();
    for (int k = 0; k < Engine::kKinds; ++k) {
        const int pa = Engine::kind_path(k), pr = Engine::kind_precision(k);
        out->pass_device_s[pa][pr] += ctx->engine.kind_seconds(k);
        out->pass_timed_launches[pa][pr] += ctx->engine.kind_launches(k);
    }
    return RN_OK;
}

int rn_autotune(rn_ctx *ctx, const char *cache_path, int32_t flags)
{
    if (!ctx || (flags & ~RN_TUNE_QUICK)) return RN_EINVAL;
    {
        std::lock_guard<std::mutex> lk(ctx->call_mu);
        if (ctx->server) return RN_EINVAL;
        if (hipSetDevice(ctx->device) != hipSuccess) return RN_EDEVICE;
    }
    const bool quick = (flags & RN_TUNE_QUICK) != 0;
    ShapeTable result;   // built-in rules wherever nothing is measured
    shape_table_install(result);
    int r = RN_OK;
    for (int dim = 2; dim <= 3 && !r; ++dim)
        for (int s : {4, 8}) {
            if (r) break;
            const int c_lo = dim == 2 ? 12 : 15, c_hi = quick ? (dim == 2 ? 18 : 17) : 24;
            for (int cls = c_lo; cls <= c_hi && !r; ++cls) {
                // a side whose node count falls in the class
                int side = (int)std::llround(std::pow(2.0, (cls + 0.5) / dim));
                auto nodes = [&](int sd) { return dim == 2 ? (int64_t)sd * sd : (int64_t)sd * sd * sd; };
                while (shape_class(nodes(side)) > cls) --side;
                while (shape_class(nodes(side)) < cls) ++side;
                const int64_t n = nodes(side);
                const int64_t want = quick ? ((int64_t)1 << 22) : kTrialNodes;
                const int cmax = quick ? 16 : kTrialCopiesMax;
                const int copies = (int)std::max<int64_t>(1, std::min<int64_t>(cmax, want / n));
                std::vector<ShapeChoice> cands;
                if (dim == 2) {
                    for (int shape : {0, 1})
                        for (int tpw : {1, 2, 3, 4}) {
                            if (shape == 1 && tpw > 2) continue;   // the small tile is for latency, not depth
                            ShapeChoice c;
                            c.shape = shape;
                            c.tpw = tpw;
                            cands.push_back(c);
                        }
                } else {
                    for (int tz : {2, 4, 8, 16, 32})
                        if (tz <= side) {
                            ShapeChoice c;
                            c.tile_z = tz;
                            cands.push_back(c);
                        }
                }
                // the shape the built-in rules give this class's trial network
                ShapeChoice builtin;
                {
                    shape_table_install(ShapeTable());
                    rn_problem bp;
                    std::memset(&bp, 0, sizeof(bp));
                    bp.dim = dim;
                    bp.nx = bp.ny = side;
                    bp.nz = dim == 3 ? side : 1;
                    bp.mem = RN_MEM_DEVICE;
                    rn_opts bo;
                    rn_opts_default(&bo);
                    bo.precision = s == 4 ? RN_MIXED : RN_FP64;
                    const Layout BL = make_layout(&bp, &bo);
                    if (dim == 2) {
                        builtin.shape = BL.shape;
                        builtin.tpw = BL.tpw;
                    } else {
                        builtin.tile_z = BL.tile_z;
                    }
                    shape_table_install(result);
                }
                ShapeChoice best;
                double best_ns = 0.0, builtin_ns = 0.0;
                for (const ShapeChoice &c : cands) {
                    double ns = 0.0;
                    for (int rep = 0; rep < kTrialRepeats && !r; ++rep) {
                        double t = 0.0;
                        r = shape_trial(ctx, dim, s, side, copies, c, &t);
                        if (!r && (ns == 0.0 || t < ns)) ns = t;
                    }
                    if (r) break;
                    const bool is_builtin = dim == 2 ? (c.shape == builtin.shape && c.tpw == builtin.tpw)
                                                     : c.tile_z == builtin.tile_z;
                    if (is_builtin) builtin_ns = ns;
                    if (best_ns == 0.0 || ns < best_ns) {
                        best = c;
                        best_ns = ns;
                    }
                }
                if (r) break;
                // keep the built-in shape unless a candidate is clearly faster
                // (the trials' run-to-run spread is a few percent)
                if (builtin_ns > 0.0 && best_ns > kTrialMargin * builtin_ns) {
                    best = builtin;
                    best_ns = builtin_ns;
                }
                best.ns_per_node = best_ns;
                result.c[dim - 2][s == 4 ? 1 : 0][cls] = best;
            }
        }
    shape_table_install(result);
    if (r) return r;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (!f) return RN_EINVAL;
        const std::string text = shape_table_format(result);
        const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
        if (std::fclose(f) != 0 || !ok) return RN_EINVAL;
    }
    return RN_OK;
}

int rn_tune_load(const char *path)
{
    if (!path) return RN_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return RN_EINVAL;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    ShapeTable t;
    if (shape_table_parse(text, &t) != RN_OK) return RN_EINVAL;
    shape_table_install(t);
    return RN_OK;
}

int rn_tune_reset(void)
{
    shape_table_install(ShapeTable());
    return RN_OK;
}

int rn_set_timing(rn_ctx *ctx, int enable)
{
    if (!ctx || (enable != 0 && enable != 1)) return RN_EINVAL;
    CallLock cl(ctx);
    ctx->engine.set_timing(enable != 0);
    return RN_OK;
}

}  // extern "C"
