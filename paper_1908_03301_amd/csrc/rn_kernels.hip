// rn_kernels.hip -- gfx950 kernels of the random-network flow solve.
//
// Operator (Sec. II, Eq. 3): on the live set, (A x)_i = sum_j g_ij (x_i - x_j)
// with x = 0 on the faces for the correction (the face pressures 1 / 0 of the
// full field enter through b). The CG is Jacobi-preconditioned (M = diag d,
// d_i = sum_j g_ij) and always applies A in this difference form: rounding the
// conductances to FP32 then perturbs each bond by a relative 2^-24, which
// keeps the FP32 operator spectrally within (1 +- 2^-24) of the FP64 one
// (Rayleigh quotient sum g (x_i - x_j)^2), whatever the condition number.
//
// One pass per CG iteration k (single global reduction). The state is kept
// preconditioned: z = D^-1 r and u = D^-1 q, so that the halo needs no
// diagonal:
//     z_k = z_{k-1} - a u_{k-1};  p_k = z_k + b p_{k-1}
//     q_k = A p_k (5/7-point stencil, p_k recomputed at the halo);  u_k = q_k / d
//     every other pass: P += sigma a' p_{k-2} + sigma a p_{k-1} (FP64)
//     sums p.q, z.q, q.u (= q.D^-1 q), d z.z (= r.z) in FP64
// and a = (r.z)/(p.q), r_{k+1}.z_{k+1} = r.z - 2a z.q + a^2 q.D^-1 q give the
// next step without a second reduction. d_i is recomputed in every pass as the
// sum of the node's bonds in the inner precision (in a fixed order, the same
// in the refresh): setup zeroes every bond that touches an interior node off
// the live set, so d > 0 exactly on live and face nodes, and face nodes are
// told apart by their coordinate. The solution is accumulated straight into
// the FP64 pressure field, two steps at a time from the stored directions
// (p is triple-buffered for this), so the field is read and written every
// other pass: an FP32 accumulator would round the correction by 2^-24 of its
// size, i.e. a residual error of order 2^-24 times the condition number at
// every refresh. Nodes outside the live set hold z = p = u = 0, so the same
// arithmetic keeps them at zero; they are read and stored like the others so
// that cache lines move whole. z and u are double-buffered because
// neighbours read them from the previous pass.
//
// The same kernel, in refresh mode, evaluates the FP64 true residual b - A x
// of the pressure field with the original conductances, the face fluxes and
// x.(b - A x) for the energy conductance, and restarts the inner recurrence
// from that residual (reliable update).
#include "rn_device.hpp"

#include <math.h>

#include <algorithm>
#include <mutex>
#include <stddef.h>

namespace rn {

// ---------------------------------------------------------------- helpers

// Lane moves inside a wave without the LDS crossbar. __shfl and its kin
// compile to ds_bpermute, which takes an LDS instruction and a wait on the
// lgkm counter per move; a DPP move is one VALU instruction and v_readlane
// one more. lane_below(v): lane l receives lane l-1's v (whole-wave shift by
// one, DPP wave_shr); lane_above(v): lane l receives lane l+1's v (wave_shl).
// The lane at the wave's edge, which has no source, keeps its own v; every
// caller overrides it. lane_bcast(v, l): lane l's v in every lane (l a
// compile-time constant).
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, dpp_move<CTRL>(__builtin_bit_cast(int, v)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_move<CTRL>((int)(b & 0xffffffffll)), hi = dpp_move<CTRL>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
__device__ __forceinline__ T lane_below(T v) { return dpp_move<kDppWaveShr1>(v); }

template <typename T>
__device__ __forceinline__ T lane_above(T v) { return dpp_move<kDppWaveShl1>(v); }

__device__ __forceinline__ float lane_bcast(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ __forceinline__ double lane_bcast(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes, the same value in every lane (every lane active):
// pairs, then quads (DPP quad permutations), then eights and sixteens (DPP
// half-row and row mirrors: lane i meets lane 7 - i, then 15 - i, so both
// partners form the same sum), then the four row sums in a fixed order.
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E, kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141;

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<kDppQuadSwap1>(v);
    v += dpp_move<kDppQuadSwap2>(v);
    v += dpp_move<kDppRowHalfMirror>(v);
    v += dpp_move<kDppRowMirror>(v);
    return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

// The CG state, the bonds and the field live in device memory: accesses
// through these casts compile to global_load / global_store, which count on
// the vector-memory counter only. Through a generic pointer (every pointer
// read from an argument table is one) they are flat accesses, which count on
// the lgkm counter as well, so each wait for an LDS read or a lane move would
// also wait for every load and store still in flight.
#define RN_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ T ldg(const T *p) { return *(const RN_GLOBAL T *)p; }

template <typename T>
__device__ __forceinline__ void stg(T *p, T v) { *(RN_GLOBAL T *)p = v; }

// Partial sums travel between workgroups through write-through (system-scope)
// stores and loads that bypass the per-XCD L2s, so no workgroup has to write
// back or invalidate its L2 (a device-scope fence would do both).
__device__ __forceinline__ double ld_through(const double *p)
{
    return __hip_atomic_load((const RN_GLOBAL double *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void st_through(double *p, double v)
{
    __hip_atomic_store((RN_GLOBAL double *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Loads and stores of the CG state, by coherence mode:
//   COH 0 (one launch per round): plain accesses; a kernel boundary makes
//     every store visible to the next launch, on any XCD.
//   COH 1 (persistent launch, a network's items on any XCD): a pass reads
//     what workgroups on other XCDs, with their own L2s, wrote in the previous
//     pass, and its own XCD's L2 may still hold the buffer from two passes
//     back, so the state moves by device-scope accesses (global_load /
//     global_store with sc1), which write through the L2 and do not return a
//     line another XCD has since written.
//   COH 2 (persistent launch, all items of a network on one XCD): the state
//     is coherent in that XCD's L2, so stores are plain (the per-CU L1 writes
//     through to it). Loads are still device-scope (sc1): a workgroup-scope
//     load (sc0) or a plain one is served by the CU's own L1, which keeps a
//     line another CU has since written (outside threadgroup-split mode the
//     memory model lets workgroup scope hit L1); sc1 loads skip L1 and hit L2.
// The bonds, the mask and the FP64 conductances are read-only during the
// iterations and keep plain loads in every mode.
// The same through a generic pointer (flat_load / flat_store): the 3D plane
// stream below uses these; it measured faster with them (168.6 against 176.8
// us per pass on a 256^3 network), the 2D tile slower.
template <int COH, typename T>
__device__ __forceinline__ T ldc_flat(const T *p)
{
    if constexpr (COH != 0) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}

template <int COH, typename T>
__device__ __forceinline__ void stc_flat(T *p, T v)
{
    if constexpr (COH == 1) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <int COH, typename T>
__device__ __forceinline__ T ldc(const T *p)
{
    if constexpr (COH != 0) return __hip_atomic_load((const RN_GLOBAL T *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return ldg(p);
}

template <int COH, typename T>
__device__ __forceinline__ void stc(T *p, T v)
{
    if constexpr (COH == 1) __hip_atomic_store((RN_GLOBAL T *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else stg(p, v);
}

// The memory scope of the reduction's own stores (partials, ticket resets,
// control block) in each mode: across XCDs unless the network is on one.
// Its loads are device-scope in every persistent mode (see ldc).
template <int COH>
constexpr int store_scope() { return COH == 2 ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT; }

// Workgroup index -> tile index so that each XCD (workgroups are dealt to the
// 8 XCDs round-robin) owns one contiguous range of tiles and shares halos in
// its own L2. `grid` is a multiple of 8.
__device__ __forceinline__ int xcd_remap(int b, int grid)
{
    const int per = grid >> 3;
    return (b & 7) * per + (b >> 3);
}

// Jacobi diagonal of a node from its bonds to -x, +x, -y, +y (and -z, +z),
// summed in this fixed order so that the pass and the refresh round it the
// same way.
template <typename T>
__device__ __forceinline__ T diag_sum(T gxm, T gxp, T gym, T gyp)
{
    return (gxm + gxp) + (gym + gyp);
}

template <typename T>
__device__ __forceinline__ T diag_sum(T gxm, T gxp, T gym, T gyp, T gzm, T gzp)
{
    return ((gxm + gxp) + (gym + gyp)) + (gzm + gzp);
}

// Jacobi scaling v / d. FP32: the hardware reciprocal (about 1 ulp, and a
// fixed function of d, so the preconditioner stays one fixed diagonal) in
// place of the much longer correctly rounded division; FP64: the division.
__device__ __forceinline__ float jscale(float v, float d) { return v * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double jscale(double v, double d) { return v / d; }

// M^-1 v at a node of diagonal d: v / d with the Jacobi preconditioner, v
// without one (then every use of d as the weight of M also becomes 1).
template <typename T>
__device__ __forceinline__ T apply_minv(T v, T d, bool jacobi) { return jacobi ? jscale(v, d) : v; }

// Scalar update after a CG pass. t = (p.q, z.q, q.D^-1 q, r.z, 0).
__device__ void step_after_cg(Scalars *s, const double *t)
{
    const double pq = t[0], zq = t[1], qq = t[2], rz = t[3];
    // a pass that left the FP64 field alone leaves the steps before it
    // pending; once kpend are pending the next CG pass adds them all
    const bool flushed = s->flush != 0;
    if (flushed) {
        s->alpha2 = s->alpha3 = s->alpha4 = 0.0;
        s->npend = 1;
    } else {
        s->alpha4 = s->alpha3;
        s->alpha3 = s->alpha2;
        s->alpha2 = s->alpha;
        s->npend += 1;
    }
    s->flush = s->npend >= s->kpend ? 1 : 0;
    s->passes += 1;
    s->iters += 1;
    s->rho = rz;
    s->rmax = fmax(s->rmax, sqrt(fmax(rz, 0.0)));
    if (!(rz > 0.0) && isfinite(rz)) {        // residual exactly zero: verify and stop
        s->alpha = 0.0;
        s->sigma_next = s->sigma;
        s->check = 1;
        s->mode = MODE_REFRESH;
        return;
    }
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(zq) || !isfinite(qq) || !isfinite(rz)) {
        s->status = -4;                       // breakdown: finish on the last good iterate
        s->stop = 1;
        s->alpha = 0.0;
        s->sigma_next = s->sigma;
        s->mode = MODE_REFRESH;
        return;
    }
    const double alpha = rz / pq;
    double rho_next = rz - 2.0 * alpha * zq + alpha * alpha * qq;
    if (!(rho_next > 0.0)) rho_next = 0.0;
    const double est = s->kappa * s->sigma * sqrt(rho_next) / s->bhat;
    s->est_rel = est;
    s->alpha = alpha;
    const bool check = est <= s->tol || rho_next <= 0.0;
    const bool refresh = check || s->iters >= s->max_iter ||
                         (s->delta > 0.0 && sqrt(rho_next) <= s->delta * s->rmax);
    if (refresh) {
        s->check = check;
        s->est_check = est;
        s->sigma_next = s->sigma * sqrt(fmax(rho_next, rz * 1e-24));
        s->mode = MODE_REFRESH;
    } else {
        s->beta = rho_next / rz;
        s->mode = MODE_CG;
    }
}

// Scalar update after a refresh pass. t = (||r64||^2, r.D^-1 r of the stored residual, x.r64, Q_in, Q_out).
// s->first: 1 before the refresh that evaluates b, 2 before the one that
// evaluates the residual of the initial guess, 0 afterwards.
__device__ void step_after_refresh(Scalars *s, const double *t)
{
    const double rr64 = t[0], rrs = t[1];
    s->passes += 1;
    s->refreshes += 1;
    s->alpha2 = s->alpha3 = s->alpha4 = 0.0;     // the refresh applied every pending step
    s->flush = 0;
    s->npend = 1;                                // its own step is 0: counted as pending
    const double sigma_old = s->sigma;
    const double sigma = s->sigma_next;
    s->sigma = sigma;
    const int first = s->first;
    if (first == 1) {
        // this refresh evaluated b alone (the inflow at x = 0): fix the norms the
        // stopping rule and the estimates refer to, then evaluate the residual
        // of the initial guess (the linear profile along the flow axis)
        s->bnorm = sqrt(rr64);
        s->bhat = sigma * sqrt(rrs);
        s->kappa = 1.0;
        s->xr = t[2];
        s->Q_in = t[3];
        s->Q_out = t[4];
        if (!(s->bnorm > 0.0) || !isfinite(rr64) || !isfinite(rrs)) {
            if (s->bnorm == 0.0) s->converged = 1;      // nothing flows in
            else s->status = -4;
            s->rel_resid = s->est_rel = 0.0;
            s->mode = MODE_DONE;
        } else {
            s->first = 2;
            s->rel_resid = s->est_rel = 1.0;
            s->alpha = 0.0;
            s->sigma_next = sigma;
            s->mode = MODE_REFRESH;
        }
        s->check = 0;
        return;
    }
    const bool restart = first == 2;             // the first residual: start the recurrence
    s->first = 0;
    const double rel = s->bnorm > 0.0 ? sqrt(rr64) / s->bnorm : 0.0;
    const double srel = s->bhat > 0.0 ? sigma * sqrt(rrs) / s->bhat : 0.0;
    if (srel > 0.0 && rel > 0.0) s->kappa = rel / srel;
    s->rel_resid = rel;
    s->est_rel = rel;
    s->xr = t[2];
    s->Q_in = t[3];
    s->Q_out = t[4];
    if (s->stop) {
        s->mode = MODE_DONE;
    } else if (rel <= s->tol || s->bnorm == 0.0) {
        s->converged = 1;
        s->mode = MODE_DONE;
    } else if (s->iters >= s->max_iter) {
        s->status = -3;
        s->mode = MODE_DONE;
    } else if (!isfinite(rr64) || !isfinite(rrs)) {
        s->status = -4;
        s->mode = MODE_DONE;
    } else if (s->check && !(rel < 0.5 * s->last_check) && rel > 10.0 * s->est_check) {
        // the recurrence says converged, the true residual is far above it and
        // no longer halves between checks: its rounding floor is reached
        s->status = -3;
        s->mode = MODE_DONE;
    } else {
        if (s->check) s->last_check = rel;
        s->mode = MODE_CG;
        s->alpha = 0.0;
        s->beta = restart ? 0.0 : sigma * rrs / (sigma_old * s->rho);
        s->rmax = sqrt(rrs);
    }
    s->check = 0;
}

// The control block is read at the start of every pass by the threads that
// will need it at the end: thread t < kScalWords loads its 8-byte word into a
// register, so the last workgroup's scalar step runs on an LDS copy instead of
// waiting for a chain of memory round trips after the reduction.
constexpr int kScalWords = (int)(sizeof(Scalars) / 8);
static_assert(sizeof(Scalars) == 256 && kScalWords <= kBlock, "control block words: one 256-byte block per network");
constexpr int kModeWord = (int)(offsetof(Scalars, mode) / 8);
static_assert(offsetof(Scalars, mode) == 0, "mode is the low half of the first control block word");
constexpr int kPassesWord = (int)(offsetof(Scalars, passes) / 8);
static_assert(offsetof(Scalars, passes) % 8 == 0 && kModeWord != kPassesWord, "control block words");

__device__ __forceinline__ unsigned long long prefetch_scalars(const Scalars *s)
{
    const int t = threadIdx.x < kScalWords ? (int)threadIdx.x : 0;
    const unsigned long long v = reinterpret_cast<const unsigned long long *>(s)[t];
    return threadIdx.x < kScalWords ? v : 0ull;
}

// Per-workgroup partials, then the last workgroup to arrive sums them in
// block order (a fixed order, so the result does not depend on scheduling)
// and runs the scalar update. Arrival is counted in two levels: on the counter
// of the workgroup's group (lb mod groups), then, by the last of each group,
// on the top counter. Device-scope atomics on one address are serviced one
// after another, so a single counter for a 2048-workgroup pass queued 2048
// atomics at the end of every pass.
// COH 1, 2 (persistent launches): every wave first waits for its own state
// stores to complete, so that a workgroup counts only once its tile is
// visible, and the last workgroup publishes the control block, the pass count
// last (the word later passes of the same network wait on). With COH 2 the
// partials, tickets and control block stay in the network's XCD's L2.
template <int COH>
__device__ void finish_pass(double (&acc)[kRed], double *partials, unsigned *tickets, Scalars *s, int lb, int grid,
                            int groups, int mode, unsigned long long spre)
{
    __shared__ double red[kBlock / kWave][kRed];
    __shared__ int is_last;
    __shared__ unsigned long long sl[kScalWords];
    constexpr int kStride = kTicketStride / (int)sizeof(unsigned);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if constexpr (COH != 0) __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int k = 0; k < kRed; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) red[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < kRed; ++k) {
            double v = 0.0;
            for (int ww = 0; ww < kBlock / kWave; ++ww) v += red[ww][k];
            if constexpr (COH == 2) partials[(size_t)lb * kRed + k] = v;
            else st_through(&partials[(size_t)lb * kRed + k], v);
        }
        // wait until this thread's write-through stores have completed
        // (s_waitcnt with every counter at 0), then count (device-scope
        // atomics, coherent across XCDs); groups is a power of two dividing grid
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned prev = __hip_atomic_fetch_add((RN_GLOBAL unsigned *)(tickets + (lb & (groups - 1)) * kStride),
                                                     1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int last = prev == (unsigned)(grid / groups) - 1u;
        if (last && groups > 1) {
            const unsigned top = __hip_atomic_fetch_add((RN_GLOBAL unsigned *)(tickets + groups * kStride), 1u,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = top == (unsigned)groups - 1u;
        }
        is_last = last;
    }
    __syncthreads();
    if (!is_last) return;
    double tot[kRed];
#pragma unroll
    for (int k = 0; k < kRed; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < grid; b += kBlock)
#pragma unroll
        for (int k = 0; k < kRed; ++k)
            tot[k] += COH == 2 ? __hip_atomic_load(&partials[(size_t)b * kRed + k], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : ld_through(&partials[(size_t)b * kRed + k]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRed; ++k) {
        double v = wave_sum(tot[k]);
        if (lane == 0) red[w][k] = v;
    }
    // every workgroup has counted: clear the counters for the next pass
    if (threadIdx.x <= groups)
        __hip_atomic_store(tickets + threadIdx.x * kStride, 0u, __ATOMIC_RELAXED, store_scope<COH>());
    if (threadIdx.x < kScalWords) sl[threadIdx.x] = spre;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[kRed];
        for (int k = 0; k < kRed; ++k) {
            t[k] = 0.0;
            for (int ww = 0; ww < kBlock / kWave; ++ww) t[k] += red[ww][k];
        }
        Scalars *ls = reinterpret_cast<Scalars *>(sl);
        if (mode == MODE_CG) step_after_cg(ls, t);
        else step_after_refresh(ls, t);
    }
    __syncthreads();
    unsigned long long *sw = reinterpret_cast<unsigned long long *>(s);
    if constexpr (COH != 0) {
        const int t = (int)threadIdx.x;
        if (t < kScalWords && t != kPassesWord) __hip_atomic_store(sw + t, sl[t], __ATOMIC_RELAXED, store_scope<COH>());
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t == kPassesWord) __hip_atomic_store(sw + t, sl[t], __ATOMIC_RELAXED, store_scope<COH>());
    } else {
        if (threadIdx.x < kScalWords) sw[threadIdx.x] = sl[threadIdx.x];
    }
}

// What one pass does with the direction and the FP64 field, from the control
// block: p1 holds p_{k-1}, whose step sa = sigma alpha is pending; p2, p3, p4
// hold p_{k-2}, p_{k-3}, p_{k-4}, whose steps sa2, sa3, sa4 are also pending
// while the CG passes after them left the field alone (a step not pending is
// 0; a CG pass with `flush` adds them all); p0 receives p_k. A network keeps
// up to kpend steps pending (4 for the FP32 passes, 2 for the FP64 ones,
// whose registers are scarcer) in kpend + 1 buffers.
template <typename T>
struct Step {
    const T *p1, *p2, *p3, *p4;
    T *p0;
    double sa, sa2, sa3, sa4;
    bool flush;
};

template <typename T>
__device__ __forceinline__ Step<T> make_step(const PassArgs<T> &a, const Scalars *s)
{
    // the buffer of pass c - d: constant divisors and conditional wraps, not
    // a 64-bit division by a runtime count at the start of every workgroup
    const int nb = a.npbuf;
    const int c = nb == 5 ? (int)(s->passes % 5) : (int)(s->passes % 3);
    auto back = [&](int d) {
        int v = c - d;
        if (v < 0) v += nb;
        if (v < 0) v += nb;
        return v;
    };
    Step<T> k;
    k.p0 = a.pbuf[c];
    k.p1 = a.pbuf[back(1)];
    k.p2 = a.pbuf[back(2)];
    k.p3 = a.pbuf[back(3)];
    k.p4 = a.pbuf[back(4)];
    k.sa = s->sigma * s->alpha;
    k.sa2 = s->sigma * s->alpha2;
    k.sa3 = s->sigma * s->alpha3;
    k.sa4 = s->sigma * s->alpha4;
    k.flush = s->flush != 0;
    return k;
}

// FP64 field with the pending steps added, oldest first (the order in which
// one step per pass would have added them).
__device__ __forceinline__ double with_steps(double P, double sa2, double p2, double sa, double p1)
{
    double v = P;
    if (sa2 != 0.0) v = fma(sa2, p2, v);
    if (sa != 0.0) v = fma(sa, p1, v);
    return v;
}



// ---------------------------------------------------------------- refresh (FP64)
// Node-local FP64 work of a refresh pass. The pending steps (sa p1, and
// sa2 p2 when the last CG pass left the field alone) are added on the fly to
// every pressure the stencil reads; p is zero off the live set, so this is
// the updated field everywhere. The node's loads go out in two batches (the
// mask and bonds, then, on live nodes, the pressures and directions), each
// issued before any branch on its data: two memory round trips per node, and
// few enough registers that the rare refresh does not lower the occupancy of
// the CG pass that shares its kernel.
template <typename T, int DIM, int COH>
__device__ __forceinline__ void refresh_node(const PassArgs<T> &a, const double *__restrict__ Ps,
                                             double *__restrict__ Pd, int x, int y, int z, const Step<T> &k_,
                                             double sigma_next, bool bonly, double (&acc)[kRed])
{
    const int64_t sx = 1, sy = a.nx, sz = (int64_t)a.nx * a.ny;
    const int64_t i = x + sy * y + sz * z;
    const int c[3] = {x, y, z};
    const int n[3] = {a.nx, a.ny, a.nz};
    const int64_t st[3] = {sx, sy, sz};
    const double sa = k_.sa, sa2 = k_.sa2, sa3 = k_.sa3, sa4 = k_.sa4;
    // neighbour j of the -k / +k bond (the node itself where there is none)
    int64_t jn[2 * DIM];
    bool has[2 * DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool wk = (a.wrap >> k) & 1;       // never the flow axis
        const int64_t span = (int64_t)(n[k] - 1) * st[k];
        has[2 * k] = c[k] > 0 || wk;
        has[2 * k + 1] = c[k] + 1 < n[k] || wk;
        jn[2 * k] = c[k] > 0 ? i - st[k] : (wk ? i + span : i);
        jn[2 * k + 1] = c[k] + 1 < n[k] ? i + st[k] : (wk ? i - span : i);
    }
    // batch 1: mask and bonds
    const bool live = ldg(a.mask + i) == 3;
    T gb[2 * DIM];
    double gd[2 * DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T gbm = ldg(a.gT[k] + jn[2 * k]), gbp = ldg(a.gT[k] + i);
        const double gdm = ldg(a.g64[k] + jn[2 * k]), gdp = ldg(a.g64[k] + i);
        gb[2 * k] = has[2 * k] ? gbm : T(0);
        gb[2 * k + 1] = gbp;                     // 0 past the lattice edge
        gd[2 * k] = has[2 * k] ? gdm : 0.0;
        gd[2 * k + 1] = has[2 * k + 1] ? gdp : 0.0;
    }
    if (!live) {
        stc<COH>(Pd + i, ldc<COH>(Ps + i));
        return;
    }
    // batch 2: the node's and its neighbours' pressures and directions
    double Pi = ldc<COH>(Ps + i);
    double Pn[2 * DIM];
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) Pn[e] = ldc<COH>(Ps + jn[e]);
    // the steps before the last two, pending only with kpend 4 (the FP32
    // passes; a uniform branch, never on the first refresh): added first,
    // oldest first, so that their directions are not held beside the others
    if (sizeof(T) == 4 && (sa3 != 0.0 || sa4 != 0.0)) {
        Pi = with_steps(Pi, sa4, (double)ldc<COH>(k_.p4 + i), sa3, (double)ldc<COH>(k_.p3 + i));
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e)
            Pn[e] = with_steps(Pn[e], sa4, (double)ldc<COH>(k_.p4 + jn[e]), sa3, (double)ldc<COH>(k_.p3 + jn[e]));
    }
    const T pi_ = ldc<COH>(k_.p1 + i), pi2_ = ldc<COH>(k_.p2 + i);
    T pn_[2 * DIM], pn2_[2 * DIM];
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) {
        pn_[e] = ldc<COH>(k_.p1 + jn[e]);
        pn2_[e] = ldc<COH>(k_.p2 + jn[e]);
    }
    // bonly: evaluate b = b - A 0, the interior pressures taken as 0 and the
    // inlet face at 1 (the first refresh of a solve)
    const double pi = bonly ? 0.0 : with_steps(Pi, sa2, (double)pi2_, sa, (double)pi_);
    double r64 = 0.0, qin = 0.0, qout = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double gm = gd[2 * k], gp = gd[2 * k + 1];
        const double pm = with_steps(Pn[2 * k], sa2, (double)pn2_[2 * k], sa, (double)pn_[2 * k]);
        const double pp = with_steps(Pn[2 * k + 1], sa2, (double)pn2_[2 * k + 1], sa, (double)pn_[2 * k + 1]);
        if (gm != 0.0) {
            const bool inlet = k == a.axis && c[k] == 1;
            r64 += gm * ((bonly ? (inlet ? 1.0 : 0.0) : pm) - pi);
            if (inlet) qin += gm * (1.0 - pi);
        }
        if (gp != 0.0) {
            r64 += gp * ((bonly ? 0.0 : pp) - pi);
            if (k == a.axis && c[k] == n[k] - 2) qout += gp * pi;
        }
    }
    // the inner diagonal, exactly as the CG pass forms it (> 0 on a live
    // node unless its bonds underflow the inner precision)
    T dT;
    if constexpr (DIM == 2) dT = diag_sum(gb[0], gb[1], gb[2], gb[3]);
    else dT = diag_sum(gb[0], gb[1], gb[2], gb[3], gb[4], gb[5]);
    const T rs = (T)(r64 / sigma_next);
    const T zs = dT > T(0) ? apply_minv(rs, dT, a.jacobi != 0) : T(0);
    stc<COH>(Pd + i, bonly ? Pi : pi);
    stc<COH>(a.dst.z + i, zs);
    stc<COH>(k_.p0 + i, pi_);
    stc<COH>(a.dst.u + i, T(0));
    acc[0] += r64 * r64;
    acc[1] += (double)rs * (double)zs;
    acc[2] += pi * r64;
    acc[3] += qin;
    acc[4] += qout;
}

// ---------------------------------------------------------------- 2D pass
// A workgroup owns a tile of 64 SEG consecutive x and 4 TY rows; wave w holds
// rows w TY .. w TY + TY - 1, each as SEG segments of 64 columns (lane l holds
// columns x0 + 64 s + l). Every load of the tile (the rows, one halo row above
// and below the workgroup, the halo columns and the bonds) is issued up front
// at a clamped, in-bounds address with no branch on loaded data, so the
// tile's whole memory traffic is in flight at once; out-of-lattice values are
// then zeroed with selects. Rows next to another wave's rows get that wave's
// p' through LDS (one barrier), so only 2 rows in 4 TY are re-read. Off the
// live set z = u = p = 0 in memory, so p' needs no mask; q is zeroed off the
// live set, where the bond sum d is 0 (dead node) or the node is on a face;
// only stores are restricted to the lattice.
// x-neighbours come from lane shuffles (across a segment junction from lane 63
// of one segment and lane 0 of the next); lanes 0..TY-1 and 64-TY..63 load the
// halo columns x0-1 and x0+64 SEG (one row each), which shuffles hand to lane
// 0 of the first segment and lane 63 of the last.
// SHAPE 0: the tile for networks with enough tiles to fill the chip; SHAPE 1:
// a quarter-size tile (one segment, half the rows) for smaller networks,
// which would otherwise leave most CUs with one or two workgroups.
template <typename T, int SHAPE>
struct Tile2D {
    static constexpr int TY = SHAPE == 0 ? (sizeof(T) == 4 ? kTY2f : kTY2d)           // rows per wave
                                         : (sizeof(T) == 4 ? kTY2fS : kTY2dS);
    static constexpr int SEG = SHAPE == 0 ? (sizeof(T) == 4 ? kSEG2f : kSEG2d) : 1;   // 64-column segments per row
    static constexpr int ROWS = TY * (kBlock / kWave);                                // rows per workgroup
    static constexpr int COLS = kWave * SEG;                                          // columns per workgroup
};

template <typename T, int SHAPE, int COH>
__device__ __forceinline__ void cg2d_tile(const PassArgs<T> &a, double *__restrict__ P, int x0, int yb, int lane,
                                          int w, T alpha, T beta, const Step<T> &k, double (&acc)[kRed])
{
    constexpr int TY = Tile2D<T, SHAPE>::TY;
    constexpr int SEG = Tile2D<T, SHAPE>::SEG;
    constexpr int NW = kBlock / kWave;
    __shared__ T edge[2][NW][SEG][kWave];   // [0]: first row of each wave, [1]: last row
    const int nx = a.nx, ny = a.ny;
    const int y0 = yb + w * TY;        // first row of this wave
    // Plane a lane or row slot holds: its own inside the lattice; across a
    // periodic direction the plane just past either edge holds the image of
    // the opposite edge (x = nx is column 0, y = -1 is row ny - 1), so the
    // stencil reads the wrapped neighbours like any other; -1 = none.
    const bool wx = a.wrap & 1, wy = (a.wrap >> 1) & 1;
    auto colm = [&](int xx) { return xx >= 0 && xx < nx ? xx : (wx && xx == nx ? 0 : (wx && xx == -1 ? nx - 1 : -1)); };
    auto rowm = [&](int yy) { return yy >= 0 && yy < ny ? yy : (wy && yy == ny ? 0 : (wy && yy == -1 ? ny - 1 : -1)); };
    auto rowc = [&](int yy) {          // row to load for slot yy (clamped where it holds none)
        const int m = rowm(yy);
        return m >= 0 ? m : (yy < 0 ? 0 : ny - 1);
    };
    bool valid[SEG], lv[SEG];          // a lattice node (stored, reduced) / holds a column or an image
    int xc[SEG];
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) {
        const int x = x0 + kWave * sg + lane;
        const int xm = colm(x);
        valid[sg] = x < nx;
        lv[sg] = xm >= 0;
        xc[sg] = lv[sg] ? xm : nx - 1;
    }
    const T *__restrict__ zs = a.src.z;
    const T *__restrict__ us = a.src.u;
    const T *__restrict__ ps = k.p1;
    const T *__restrict__ p2s = k.p2;
    T *__restrict__ zd = a.dst.z;
    T *__restrict__ ud = a.dst.u;
    T *__restrict__ pd = k.p0;
    const T *__restrict__ gx = a.gT[0];
    const T *__restrict__ gy = a.gT[1];
    const bool flush = k.flush;        // uniform: this pass adds the pending steps to P
    const bool jacobi = a.jacobi != 0;

    // ---- the FP64 field (every other pass). It does not depend on the
    // stencil: with FP32 vectors it is updated first, which frees its
    // registers for the rest of the tile (measured faster on the FP32 pass);
    // with FP64 vectors its loads join the tile's and it is stored at the end
    // (measured faster there).
    constexpr bool kFieldFirst = sizeof(T) == 4;
    if (kFieldFirst && flush) {
        // up to four pending steps (kpend 4): the older two only when pending
        const bool older = k.sa3 != 0.0 || k.sa4 != 0.0;
        const T *__restrict__ p3s = k.p3;
        const T *__restrict__ p4s = k.p4;
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int yy = y0 + j;
#pragma unroll
            for (int sg = 0; sg < SEG; ++sg) {
                const int64_t i = (int64_t)rowc(yy) * nx + xc[sg];
                double v = ldc<COH>(P + i);
                if (older) v = with_steps(v, k.sa4, (double)ldc<COH>(p4s + i), k.sa3, (double)ldc<COH>(p3s + i));
                v = with_steps(v, k.sa2, (double)ldc<COH>(p2s + i), k.sa, (double)ldc<COH>(ps + i));
                if (valid[sg] && yy < ny) stc<COH>(P + i, v);
            }
        }
    }

    // ---- issue every load
    T z_[SEG][TY], u_[SEG][TY], p_[SEG][TY];
    T gxv[SEG][TY], gyv[SEG][TY + 1];
#pragma unroll
    for (int j = 0; j < TY; ++j) {
        const int64_t ro = (int64_t)rowc(y0 + j) * nx;
#pragma unroll
        for (int sg = 0; sg < SEG; ++sg) {
            const int64_t i = ro + xc[sg];
            z_[sg][j] = ldc<COH>(zs + i);
            u_[sg][j] = ldc<COH>(us + i);
            p_[sg][j] = ldc<COH>(ps + i);
            gxv[sg][j] = ldg(gx + i);
            gyv[sg][j + 1] = ldg(gy + i);
        }
    }
    double Pv[SEG][TY];
    T p2_[SEG][TY];
    if (!kFieldFirst && flush) {
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int64_t ro = (int64_t)rowc(y0 + j) * nx;
#pragma unroll
            for (int sg = 0; sg < SEG; ++sg) {
                const int64_t i = ro + xc[sg];
                Pv[sg][j] = ldc<COH>(P + i);
                p2_[sg][j] = k.sa2 != 0.0 ? ldc<COH>(p2s + i) : T(0);   // none pending right after a refresh
            }
        }
    }
    {   // bond below the wave: none at y = 0 unless y wraps (then the bond ny-1 -> 0)
        const bool below = rowm(y0 - 1) >= 0;
        const int64_t ro = (int64_t)rowc(y0 - 1) * nx;
#pragma unroll
        for (int sg = 0; sg < SEG; ++sg) {
            const T g0 = ldg(gy + ro + xc[sg]);
            gyv[sg][0] = below ? g0 : T(0);
        }
    }
    // the workgroup's outer halo rows: wave 0 the row above, the last wave the row below
    T ez[SEG], eu[SEG], ep[SEG];
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) ez[sg] = eu[sg] = ep[sg] = T(0);
    if (w == 0 || w == NW - 1) {   // wave-uniform
        const int yh = w == 0 ? yb - 1 : yb + NW * TY;
        const bool hrow = rowm(yh) >= 0;
        const int64_t ro = (int64_t)rowc(yh) * nx;
#pragma unroll
        for (int sg = 0; sg < SEG; ++sg) {
            const int64_t i = ro + xc[sg];
            const T z0 = ldc<COH>(zs + i), u0 = ldc<COH>(us + i), p0 = ldc<COH>(ps + i);
            if (hrow && lv[sg]) {
                ez[sg] = z0;
                eu[sg] = u0;
                ep[sg] = p0;
            }
        }
    }
    // halo columns: lane l < TY holds (x0-1, y0+l), lane 64-TY+l holds (x0+64 SEG, y0+l)
    const bool hleft = lane < TY, hright = lane >= kWave - TY;
    const int hr_ = hleft ? lane : lane - (kWave - TY);
    const int hx = colm(hleft ? x0 - 1 : x0 + Tile2D<T, SHAPE>::COLS);
    const bool hok = (hleft || hright) && hx >= 0 && y0 + hr_ < ny;
    T hz = T(0), hu = T(0), hp = T(0), hg = T(0);
    {
        const int64_t i = hok ? (int64_t)(y0 + hr_) * nx + hx : 0;
        const T z0 = ldc<COH>(zs + i), u0 = ldc<COH>(us + i), p0 = ldc<COH>(ps + i), g0 = ldg(gx + i);
        if (hok) {
            hz = z0;
            hu = u0;
            hp = p0;
            hg = hleft ? g0 : T(0);        // bond (x0-1) -> x0 for lane 0 (nx-1 -> 0 when x wraps)
        }
    }

    // ---- p' on the wave's rows, exchanged with the neighbouring waves
    T pv[SEG][TY + 2];   // rows y0-1 .. y0+TY
#pragma unroll
    for (int j = 0; j < TY; ++j) {
        const bool rheld = rowm(y0 + j) >= 0;
#pragma unroll
        for (int sg = 0; sg < SEG; ++sg) {
            const T v = (z_[sg][j] - alpha * u_[sg][j]) + beta * p_[sg][j];
            pv[sg][j + 1] = (rheld && lv[sg]) ? v : T(0);
        }
    }
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) {
        edge[0][w][sg][lane] = pv[sg][1];
        edge[1][w][sg][lane] = pv[sg][TY];
    }
    T hv[SEG];
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) hv[sg] = (ez[sg] - alpha * eu[sg]) + beta * ep[sg];   // zero unless held
    __syncthreads();
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) {
        pv[sg][0] = w == 0 ? hv[sg] : edge[1][w - 1][sg][lane];
        pv[sg][TY + 1] = w == NW - 1 ? hv[sg] : edge[0][w + 1][sg][lane];
    }
    const T hpv = (hz - alpha * hu) + beta * hp;    // zero when !hok

    const bool xaxis = a.axis == 0;
#pragma unroll
    for (int j = 0; j < TY; ++j) {
        const int yy = y0 + j;
        const T hl = lane_bcast(hpv, j);
        const T hrr = lane_bcast(hpv, kWave - TY + j);
        const T hgl = lane_bcast(hg, j);
#pragma unroll
        for (int sg = 0; sg < SEG; ++sg) {
            const int x = x0 + kWave * sg + lane;
            const bool ok = valid[sg] && yy < ny;
            const T zc = z_[sg][j] - alpha * u_[sg][j];
            const T pc = pv[sg][j + 1];
            // neighbours across x: shuffles inside a segment, the neighbouring
            // segment's edge lane across a junction, the halo at the tile edges
            T pl = lane_below(pc);
            T pr = lane_above(pc);
            T gxl = lane_below(gxv[sg][j]);
            const T lj = sg == 0 ? hl : lane_bcast(pv[sg > 0 ? sg - 1 : 0][j + 1], kWave - 1);
            const T gj = sg == 0 ? hgl : lane_bcast(gxv[sg > 0 ? sg - 1 : 0][j], kWave - 1);
            const T rj = sg == SEG - 1 ? hrr : lane_bcast(pv[sg < SEG - 1 ? sg + 1 : 0][j + 1], 0);
            if (lane == 0) {
                pl = lj;
                gxl = gj;
            }
            if (lane == kWave - 1) pr = rj;
            T qv = gxl * (pc - pl) + gxv[sg][j] * (pc - pr) + gyv[sg][j] * (pc - pv[sg][j]) +
                   gyv[sg][j + 1] * (pc - pv[sg][j + 2]);
            const T d = diag_sum(gxl, gxv[sg][j], gyv[sg][j], gyv[sg][j + 1]);
            const bool face = xaxis ? (x == 0 || x == nx - 1) : (yy == 0 || yy == ny - 1);
            const bool live = ok && d > T(0) && !face;
            if (!live) qv = T(0);
            const T uv = live ? apply_minv(qv, d, jacobi) : T(0);
            // every in-lattice node is stored (zeros and unchanged pressures off the
            // live set) so that cache lines are written whole
            if (ok) {
                const int64_t i = (int64_t)yy * nx + x;
                if (!kFieldFirst && flush)
                    stc<COH>(P + i, with_steps(Pv[sg][j], k.sa2, (double)p2_[sg][j], k.sa, (double)p_[sg][j]));
                stc<COH>(zd + i, zc);
                stc<COH>(pd + i, pc);
                stc<COH>(ud + i, uv);
            }
            const double dq = (double)qv, du = (double)uv;
            const double dp = (double)pc, dz = live ? (double)zc : 0.0;
            acc[0] += dp * dq;
            acc[1] += dz * dq;
            acc[2] += dq * du;
            acc[3] += (double)(jacobi ? d : T(1)) * dz * dz;
        }
    }
}

// One launch runs one pass of every network listed in the block table: entry
// blk[b] = (network, block index within that network's grid). Each network
// has its own arguments (two parities of the double-buffered state), partial
// sums, ticket and control block, so networks advance independently and a
// network's arithmetic does not depend on what else is in the launch.
template <typename T, int SHAPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void pass2d_kernel(const PassArgs<T> *__restrict__ tab,
                                                        const uint2 *__restrict__ blk, Scalars *scal, int parity,
                                                        int slot)
{
    // a launch of one network passes its slot instead of a block table, which
    // saves a dependent load at the start of every workgroup
    const uint2 e = blk ? blk[blockIdx.x] : make_uint2((unsigned)slot, blockIdx.x);
    const PassArgs<T> &a = tab[2 * e.x + parity];
    const int lb = (int)e.y;
    Scalars *s = scal + e.x;          // == a.s; indexed directly to shorten the load chain
    const int mode = s->mode;
    if (mode == MODE_DONE) return;
    double acc[kRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int first = xcd_remap(lb, a.grid);     // uniform per workgroup
    const int m = (int)(s->refreshes & 1);
    const Step<T> st = make_step(a, s);
    if (mode != MODE_CG) {
        // refresh: node by node over the workgroup's tiles (no LDS)
        const double sigma_next = s->sigma_next;
        const bool bonly = s->first == 1;
        for (int k = 0; k < a.tpw; ++k) {
            const int tile = first + k * a.grid;
            if (tile >= a.ntiles) break;
            const int tx = tile % a.ntx, ty = tile / a.ntx;
            const int x0 = tx * Tile2D<T, SHAPE>::COLS;
            const int y0 = ty * Tile2D<T, SHAPE>::ROWS + w * Tile2D<T, SHAPE>::TY;
            const int y1 = min(y0 + Tile2D<T, SHAPE>::TY, a.ny);
            for (int sg = 0; sg < Tile2D<T, SHAPE>::SEG; ++sg) {
                const int x = x0 + kWave * sg + lane;
                if (x < a.nx)
                    for (int yy = y0; yy < y1; ++yy)
                        refresh_node<T, 2, 0>(a, a.P[m], a.P[m ^ 1], x, yy, 0, st, sigma_next, bonly, acc);
            }
        }
        // (a rare pass: the control block is read here, not held through the refresh)
        finish_pass<0>(acc, a.partials, a.tickets, s, lb, a.grid, a.groups, mode, prefetch_scalars(s));
        return;
    }
    const unsigned long long spre = prefetch_scalars(s);
    // a workgroup takes a.tpw tiles, grid apart (each XCD keeps contiguous ranges)
    for (int k = 0; k < a.tpw; ++k) {
        const int tile = first + k * a.grid;
        if (tile >= a.ntiles) break;
        if (k > 0) __syncthreads();              // the previous tile's LDS rows are reused
        const int tx = tile % a.ntx, ty = tile / a.ntx;
        const int x0 = tx * Tile2D<T, SHAPE>::COLS;
        const int yb = ty * Tile2D<T, SHAPE>::ROWS;
        cg2d_tile<T, SHAPE, 0>(a, a.P[m], x0, yb, lane, w, (T)s->alpha, (T)s->beta, st, acc);
    }
    finish_pass<0>(acc, a.partials, a.tickets, s, lb, a.grid, a.groups, mode, spre);
}

// ---------------------------------------------------------------- 3D pass
// A workgroup owns a 64 (x) x 16 (y) x tile_z (z) block; wave w covers rows
// 4w..4w+3 of the 16, one node per lane per row. It streams up z with a
// software pipeline: in the iteration that applies the stencil on plane z it
// turns the already loaded plane z+1 into p' (registers, and the LDS tile with
// its halo ring when z+1 is inside the block) and issues the loads of plane
// z+2 and of the bonds of plane z+1, so each plane's memory traffic is in
// flight while the previous plane is computed. The p' plane tile is
// triple-buffered in LDS (one barrier per plane). Loads use clamped in-bounds
// addresses and no branch on loaded data; off-lattice values are zeroed by
// selects. Bonds to the -x, -y, -z neighbours come from a shuffle, the row
// above in the same thread, and the previous plane.
constexpr int kRows = kTY / (kBlock / kWave);

template <typename T>
struct Raw3 {                  // one plane's loads for this thread
    T z[kRows], u[kRows], p[kRows], p2[kRows], p3[kRows], p4[kRows];
    double P[kRows];
    T hz, hu, hp;              // halo-ring node of this thread (if any)
};

template <typename T>
struct Bond3 {                 // bonds of one plane for this thread's rows
    T x[kRows], y[kRows], z[kRows];
    T xh;                      // lanes 0..kRows-1: bond (x0-1) -> x0 of row `lane`
    T yh;                      // bond from the row above this wave's first row
};

template <typename T, int COH>
__device__ __forceinline__ void cg3d_tile(const PassArgs<T> &a, double *__restrict__ P, int x0, int y0, int z0,
                                          int z1, T alpha, T beta, const Step<T> &k, double (&acc)[kRed])
{
    __shared__ T lp[3][kTY + 2][kTX + 2];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int x = x0 + lane;
    // Plane a lane, row slot or z step holds: its own inside the lattice;
    // across a periodic direction the plane just past either edge holds the
    // image of the opposite edge, so wrapped neighbours are read like any
    // other; -1 = none.
    const bool wx = a.wrap & 1, wy = (a.wrap >> 1) & 1, wz = (a.wrap >> 2) & 1;
    auto colm = [&](int v) { return v >= 0 && v < nx ? v : (wx && v == nx ? 0 : (wx && v == -1 ? nx - 1 : -1)); };
    auto rowm = [&](int v) { return v >= 0 && v < ny ? v : (wy && v == ny ? 0 : (wy && v == -1 ? ny - 1 : -1)); };
    auto plm = [&](int v) { return v >= 0 && v < nz ? v : (wz && v == nz ? 0 : (wz && v == -1 ? nz - 1 : -1)); };
    const bool xok = x < nx;           // a lattice node: stored and reduced
    const int xm = colm(x);
    const bool xl = xm >= 0;           // holds a column (its own or an image)
    const int xc = xl ? xm : nx - 1;
    const T *__restrict__ zs = a.src.z;
    const T *__restrict__ us = a.src.u;
    const T *__restrict__ ps = k.p1;
    const T *__restrict__ p2s = k.p2;
    const T *__restrict__ p3s = k.p3;
    const T *__restrict__ p4s = k.p4;
    T *__restrict__ zd = a.dst.z;
    T *__restrict__ ud = a.dst.u;
    T *__restrict__ pd = k.p0;
    const T *__restrict__ gx = a.gT[0];
    const T *__restrict__ gy = a.gT[1];
    const T *__restrict__ gz = a.gT[2];
    const bool flush = k.flush;        // uniform: this pass adds the pending steps to P
    const bool jacobi = a.jacobi != 0;
    const double sa = k.sa, sa2 = k.sa2, sa3 = k.sa3, sa4 = k.sa4;
    // up to four pending steps (kpend 4, FP32 only): the older two only when pending (uniform)
    const bool older = sizeof(T) == 4 && flush && (sa3 != 0.0 || sa4 != 0.0);
    // the FP64 field of a plane with every pending step added, oldest first
    auto field = [&](const Raw3<T> &R, int j) {
        double v = R.P[j];
        if (older) v = with_steps(v, sa4, (double)R.p4[j], sa3, (double)R.p3[j]);
        return with_steps(v, sa2, (double)R.p2[j], sa, (double)R.p[j]);
    };
    const int yw = y0 + w * kRows;                 // first row of this wave
    bool rok[kRows], lok[kRows];                   // lattice node / slot holding a node or an image
    int64_t rowoff[kRows];                         // clamped x + sy * y of each row
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        const int yy = yw + j;
        const int ym = rowm(yy);
        rok[j] = xok && yy < ny;
        lok[j] = xl && ym >= 0;
        rowoff[j] = xc + sy * (ym >= 0 ? ym : ny - 1);
    }
    // halo ring: wave 0 row y0-1, wave 1 row y0+16, wave 2 lanes 0..15 column
    // x0-1 and lanes 16..31 column x0+64 (rows y0..y0+15)
    int hx, hy, hrow, hcol;
    if (w == 0) { hx = x; hy = y0 - 1; hrow = 0; hcol = 1 + lane; }
    else if (w == 1) { hx = x; hy = y0 + kTY; hrow = kTY + 1; hcol = 1 + lane; }
    else if (w == 2 && lane < kTY) { hx = x0 - 1; hy = y0 + lane; hrow = 1 + lane; hcol = 0; }
    else if (w == 2 && lane < 2 * kTY) { hx = x0 + kTX; hy = y0 + lane - kTY; hrow = 1 + lane - kTY; hcol = kTX + 1; }
    else { hx = -1; hy = -1; hrow = -1; hcol = 0; }
    const int hxm = hrow >= 0 ? colm(hx) : -1, hym = hrow >= 0 ? rowm(hy) : -1;
    const bool hok = hxm >= 0 && hym >= 0;
    const int64_t hoff = hok ? hxm + sy * hym : 0;
    // bond halos: lane j < kRows holds gx at (x0-1, yw+j); every lane holds gy
    // at (x, yw-1) (on a periodic direction the wrap bond at the first plane)
    const int xbm = colm(x0 - 1), ybm = rowm(yw - 1);
    const bool xhok = lane < kRows && xbm >= 0 && yw + lane < ny;
    const int64_t xhoff = xhok ? xbm + sy * (yw + lane) : 0;
    const bool yhok = xl && ybm >= 0;
    const int64_t yhoff = yhok ? xc + sy * ybm : 0;

    auto zc_ = [&](int zz) {
        const int m = plm(zz);
        return (int64_t)(m >= 0 ? m : (zz < 0 ? 0 : nz - 1)) * sz;
    };
    auto load_raw = [&](Raw3<T> &R, int zz, bool ring) {
        const int64_t zo = zc_(zz);
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const int64_t i = rowoff[j] + zo;
            R.z[j] = ldc_flat<COH>(zs + i);
            R.u[j] = ldc_flat<COH>(us + i);
            R.p[j] = ldc_flat<COH>(ps + i);
        }
        if (flush && ring) {           // a plane this tile stores: its FP64 field
#pragma unroll
            for (int j = 0; j < kRows; ++j) {
                const int64_t i = rowoff[j] + zo;
                R.P[j] = ldc_flat<COH>(P + i);
                R.p2[j] = ldc_flat<COH>(p2s + i);
            }
            if (older) {
#pragma unroll
                for (int j = 0; j < kRows; ++j) {
                    const int64_t i = rowoff[j] + zo;
                    R.p3[j] = ldc_flat<COH>(p3s + i);
                    R.p4[j] = ldc_flat<COH>(p4s + i);
                }
            }
        }
        if (ring) {
            const int64_t i = hoff + zo;
            R.hz = ldc_flat<COH>(zs + i);
            R.hu = ldc_flat<COH>(us + i);
            R.hp = ldc_flat<COH>(ps + i);
        }
    };
    auto load_bonds = [&](Bond3<T> &G, int zz) {
        const int64_t zo = zc_(zz);
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const int64_t i = rowoff[j] + zo;
            G.x[j] = ldc_flat<0>(gx + i);
            G.y[j] = ldc_flat<0>(gy + i);
            G.z[j] = ldc_flat<0>(gz + i);
        }
        const T xh = ldc_flat<0>(gx + xhoff + zo), yh = ldc_flat<0>(gy + yhoff + zo);
        G.xh = xhok ? xh : T(0);           // no bond left of x = 0
        G.yh = yhok ? yh : T(0);           // no bond below y = 0
    };
    auto pprime = [&](T z, T u, T p) { return (z - alpha * u) + beta * p; };
    // face planes of the flow axis (z = 0 and z = nz - 1 when the flow is along z)
    const int ax = a.axis;

    T pm[kRows], pc[kRows], pn[kRows];   // p' of planes zc-1, zc, zc+1 (own rows)
    T zvc[kRows], zvn[kRows];            // z' of planes zc and zc+1
    T gzm[kRows];                        // gz of the bond (zc-1) -> zc
    Raw3<T> R;
    Bond3<T> Gc, Gn;

    // ---- prologue: plane z0-1 (own rows), plane z0 (rows, ring, LDS), bonds of z0
    {
        const bool in = plm(z0 - 1) >= 0;
        load_raw(R, z0 - 1, false);
#pragma unroll
        for (int j = 0; j < kRows; ++j) pm[j] = (in && lok[j]) ? pprime(R.z[j], R.u[j], R.p[j]) : T(0);
        load_raw(R, z0, true);
        load_bonds(Gc, z0);
#pragma unroll
        for (int j = 0; j < kRows; ++j) gzm[j] = (in && rok[j]) ? ldc_flat<0>(gz + rowoff[j] + zc_(z0 - 1)) : T(0);
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const bool ok = rok[j];
            const T z_ = R.z[j] - alpha * R.u[j];
            pc[j] = lok[j] ? z_ + beta * R.p[j] : T(0);
            zvc[j] = ok ? z_ : T(0);
            if (ok) {
                const int64_t i = rowoff[j] + (int64_t)z0 * sz;
                if (flush) stc_flat<COH>(P + i, field(R, j));
                stc_flat<COH>(zd + i, z_);
            }
            lp[z0 % 3][1 + w * kRows + j][1 + lane] = pc[j];
        }
        if (hrow >= 0) lp[z0 % 3][hrow][hcol] = hok ? pprime(R.hz, R.hu, R.hp) : T(0);
        load_raw(R, z0 + 1, z0 + 1 < z1);
    }

    for (int zc = z0; zc < z1; ++zc) {
        const int zn = zc + 1;
        const bool nin = zn < z1;                // plane zc+1 belongs to this block
        const bool nlat = zn < nz;               // plane zc+1 is inside the lattice
        const bool nheld = plm(zn) >= 0;         // ... or is the image of plane 0
        // (a) plane zc+1 from the loads issued one iteration ago
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const bool ok = rok[j] && nlat;
            const T z_ = R.z[j] - alpha * R.u[j];
            pn[j] = (lok[j] && nheld) ? z_ + beta * R.p[j] : T(0);
            zvn[j] = ok ? z_ : T(0);
            if (ok && nin) {
                const int64_t i = rowoff[j] + (int64_t)zn * sz;
                if (flush) stc_flat<COH>(P + i, field(R, j));
                stc_flat<COH>(zd + i, z_);
            }
            if (nin) lp[zn % 3][1 + w * kRows + j][1 + lane] = pn[j];
        }
        if (nin && hrow >= 0) lp[zn % 3][hrow][hcol] = hok ? pprime(R.hz, R.hu, R.hp) : T(0);
        // (b) loads for the next iteration
        if (zn + 1 <= z1) load_raw(R, zn + 1, zn + 1 < z1);
        if (nin) load_bonds(Gn, zn);
        __syncthreads();
        // (c) stencil on plane zc
        const int b = zc % 3;
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            const int ly = 1 + w * kRows + j;
            T gxl = lane_below(Gc.x[j]);
            const T gxh = lane_bcast(Gc.xh, j);
            if (lane == 0) gxl = gxh;
            const T gyl = j == 0 ? Gc.yh : Gc.y[j - 1];
            const T p0 = pc[j];
            T qv = gxl * (p0 - lp[b][ly][lane]) + Gc.x[j] * (p0 - lp[b][ly][lane + 2]) +
                   gyl * (p0 - lp[b][ly - 1][1 + lane]) + Gc.y[j] * (p0 - lp[b][ly + 1][1 + lane]) +
                   gzm[j] * (p0 - pm[j]) + Gc.z[j] * (p0 - pn[j]);
            const T d = diag_sum(gxl, Gc.x[j], gyl, Gc.y[j], gzm[j], Gc.z[j]);
            const int yy = yw + j;
            const bool face = ax == 0 ? (x == 0 || x == nx - 1)
                                      : (ax == 1 ? (yy == 0 || yy == ny - 1) : (zc == 0 || zc == nz - 1));
            const bool live = rok[j] && d > T(0) && !face;
            if (!live) qv = T(0);
            const T uv = live ? apply_minv(qv, d, jacobi) : T(0);
            if (rok[j]) {
                const int64_t i = rowoff[j] + (int64_t)zc * sz;
                stc_flat<COH>(pd + i, p0);
                stc_flat<COH>(ud + i, uv);
            }
            const double dp = (double)p0, dq = (double)qv, du = (double)uv;
            const double dz = live ? (double)zvc[j] : 0.0;
            acc[0] += dp * dq;
            acc[1] += dz * dq;
            acc[2] += dq * du;
            acc[3] += (double)(jacobi ? d : T(1)) * dz * dz;
        }
        // rotate
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
            gzm[j] = rok[j] ? Gc.z[j] : T(0);
            pm[j] = pc[j];
            pc[j] = pn[j];
            zvc[j] = zvn[j];
        }
        if (nin) Gc = Gn;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void pass3d_kernel(const PassArgs<T> *__restrict__ tab,
                                                        const uint2 *__restrict__ blk, Scalars *scal, int parity,
                                                        int slot)
{
    // a launch of one network passes its slot instead of a block table, which
    // saves a dependent load at the start of every workgroup
    const uint2 e = blk ? blk[blockIdx.x] : make_uint2((unsigned)slot, blockIdx.x);
    const PassArgs<T> &a = tab[2 * e.x + parity];
    const int lb = (int)e.y;
    Scalars *s = scal + e.x;          // == a.s; indexed directly to shorten the load chain
    const unsigned long long spre = prefetch_scalars(s);
    const int mode = s->mode;
    if (mode == MODE_DONE) return;
    double acc[kRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int tile = xcd_remap(lb, a.grid);
    const int m = (int)(s->refreshes & 1);
    const Step<T> st = make_step(a, s);
    // tile index is uniform per workgroup: idle workgroups still reach the reduction
    if (tile < a.ntiles) {
        const int tx = tile % a.ntx;
        const int ty = (tile / a.ntx) % a.nty;
        const int tz = tile / (a.ntx * a.nty);
        const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * a.tile_z;
        const int z1 = min(z0 + a.tile_z, a.nz);
        if (mode == MODE_CG) {
            cg3d_tile<T, 0>(a, a.P[m], x0, y0, z0, z1, (T)s->alpha, (T)s->beta, st, acc);
        } else {
            const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
            const double sigma_next = s->sigma_next;
            const bool bonly = s->first == 1;
            const int x = x0 + lane;
            if (x < a.nx)
                for (int j = 0; j < kRows; ++j) {
                    const int yy = y0 + w * kRows + j;
                    if (yy >= a.ny) break;
                    for (int zz = z0; zz < z1; ++zz)
                        refresh_node<T, 3, 0>(a, a.P[m], a.P[m ^ 1], x, yy, zz, st, sigma_next, bonly, acc);
                }
        }
    }
    finish_pass<0>(acc, a.partials, a.tickets, s, lb, a.grid, a.groups, mode, spre);
}

// ---------------------------------------------------------------- persistent pass kernels
// One launch runs `rounds` pass rounds of every network in the block table:
// item it = r * nblk + j is round r of table entry j (network, local block).
// Workgroups claim items in increasing order from a queue counter (one
// atomic per item, the next one claimed while the current one runs). Before
// an item of round r a workgroup waits until its network has completed the
// passes of the rounds before (its control block's pass count, which the
// network's last workgroup publishes after everything else of the pass,
// reaches round - round0) or has finished. An item waits only on items of
// lower index, and every item of lower index has been claimed by a
// workgroup that is running: the lowest unfinished item's workgroup is
// running it (anything it claimed before is finished), and nothing it waits
// on is unfinished. So the launch drains whatever other kernels occupy the
// GPU and however many of its workgroups are resident. Every wait is still
// bounded: past kSpinTicks, or once another wait has given up, the workgroup
// sets *err and skips the item, so every wave ends normally and the host
// reports the error. A network's passes run the same tile code and the same
// reduction as in the single-round kernels, so its results are bit-identical
// to theirs.
constexpr uint64_t kSpinTicks = 200000000ull;   // 2 s of the 100 MHz s_memrealtime clock

// err[0] = 1 once a wait gave up; the first to give up records what it saw
// in err[1..6]: network slot, passes needed, passes seen, mode seen, round
// and table entry of its item.
template <int COH>
__device__ __forceinline__ int await_pass(const Scalars *s, int64_t need, unsigned *err, unsigned slot,
                                          int round, int entry)
{
    const unsigned long long *w = reinterpret_cast<const unsigned long long *>(s);
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (true) {
        const unsigned long long done = __hip_atomic_load(w + kPassesWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long mw = __hip_atomic_load(w + kModeWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int)(uint32_t)mw == MODE_DONE) return 1;   // finished: the item is skipped
        if ((int64_t)done >= need) return 1;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
            unsigned expected = 0u;
            if (__hip_atomic_compare_exchange_strong(err, &expected, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                const unsigned info[6] = {slot, (unsigned)need, (unsigned)done, (unsigned)(uint32_t)mw,
                                          (unsigned)round, (unsigned)entry};
                for (int k = 0; k < 6; ++k)
                    __hip_atomic_store(err + 1 + k, info[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return 0;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Wait for the item's network, then load its control block into LDS (one
// 8-byte word per thread, device-scope loads). Returns the word this thread
// holds (for finish_pass) and whether the item runs.
template <int COH>
__device__ __forceinline__ bool begin_item(Scalars *s, int64_t need, unsigned *err, int it_parity,
                                           unsigned long long (&snap)[kScalWords], int (&go)[2],
                                           unsigned long long &spre, unsigned slot, int round, int entry)
{
    if (threadIdx.x == 0) go[it_parity] = await_pass<COH>(s, need, err, slot, round, entry);
    __syncthreads();
    if (!go[it_parity]) return false;
    const unsigned long long *w = reinterpret_cast<const unsigned long long *>(s);
    const int t = threadIdx.x < kScalWords ? (int)threadIdx.x : 0;
    const unsigned long long v = __hip_atomic_load(w + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    spre = threadIdx.x < kScalWords ? v : 0ull;
    if (threadIdx.x < kScalWords) snap[threadIdx.x] = spre;
    __syncthreads();
    return reinterpret_cast<const Scalars *>(snap)->mode != MODE_DONE;
}

// The item's control-block fields as wave-uniform values (read from the LDS
// snapshot and made scalar with readfirstlane), so that they live in SGPRs and
// branches on them stay uniform, as with the scalar loads of the one-round
// kernels.
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl(int64_t v)
{
    const uint32_t lo = (uint32_t)rfl((int)(uint32_t)v), hi = (uint32_t)rfl((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double rfl(double v) { return __longlong_as_double(rfl((int64_t)__double_as_longlong(v))); }

__device__ __forceinline__ Scalars uniform_scalars(const Scalars *sv)
{
    Scalars u;
    u.mode = rfl(sv->mode);
    u.first = rfl(sv->first);
    u.flush = rfl(sv->flush);
    u.refreshes = rfl(sv->refreshes);
    u.passes = rfl(sv->passes);
    u.sigma = rfl(sv->sigma);
    u.sigma_next = rfl(sv->sigma_next);
    u.alpha = rfl(sv->alpha);
    u.alpha2 = rfl(sv->alpha2);
    u.alpha3 = rfl(sv->alpha3);
    u.alpha4 = rfl(sv->alpha4);
    u.beta = rfl(sv->beta);
    return u;
}

// The queue: thread 0 claims an item index (an atomic on the launch's
// counter) into claim[], which the barriers of the item publish to the
// workgroup. The first claim is made before the loop; inside the loop the
// claim of the next item (claim[p ^ 1]) is issued at the start of the current
// one, so its latency overlaps the item's work, and read after the item.
__device__ __forceinline__ int64_t first_claim(unsigned long long *queue, unsigned long long (&claim)[2])
{
    if (threadIdx.x == 0) claim[0] = __hip_atomic_fetch_add(queue, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return (int64_t)claim[0];
}

__device__ __forceinline__ int64_t next_claim(unsigned long long (&claim)[2], int itp)
{
    __syncthreads();                      // thread 0's claim of the next item is in LDS
    const int64_t v = (int64_t)claim[itp ^ 1];
    __syncthreads();                      // read by all before claim[itp ^ 1] is reused
    return v;
}

// The XCD a workgroup runs on (the XCC_ID hardware register), for COH 2,
// where a network's items are claimed only by workgroups of the XCD the host
// placed it on.
__device__ __forceinline__ int my_xcd()
{
    return __builtin_amdgcn_readfirstlane(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20)) & 7;
}

// Items of the launch: table entries xoff[x] .. xoff[x + 1] - 1 belong to
// queue x (x = the workgroup's XCD with COH 2, else 0), and item it of queue x
// is round it / n_x of entry xoff[x] + it % n_x.
template <typename T, int SHAPE, int COH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void pass2d_persist(const PassArgs<T> *__restrict__ tab,
                                                         const uint2 *__restrict__ blk, const int *__restrict__ xoff,
                                                         Scalars *scal, int64_t round_base, int rounds, int slot,
                                                         unsigned *err, unsigned long long *queues)
{
    __shared__ unsigned long long snap[kScalWords];
    __shared__ int go[2];
    __shared__ unsigned long long claim[2];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int x = COH == 2 ? my_xcd() : 0;
    const int base = xoff[x], nblk = xoff[x + 1] - base;
    unsigned long long *queue = queues + 32 * x;
    const int64_t total = (int64_t)rounds * nblk;
    int itp = 0;
    for (int64_t it = first_claim(queue, claim); it < total; it = next_claim(claim, itp), itp ^= 1) {
        if (threadIdx.x == 0) claim[itp ^ 1] = __hip_atomic_fetch_add(queue, 1ull, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
        const int r = (int)(it / nblk);
        const int j = base + (int)(it - (int64_t)r * nblk);
        const uint2 e = blk ? blk[j] : make_uint2((unsigned)slot, (unsigned)j);
        const int parity = (int)((round_base + r) & 1);
        const PassArgs<T> &a = tab[2 * e.x + parity];
        Scalars *s = scal + e.x;
        unsigned long long spre = 0;
        if (!begin_item<COH>(s, round_base + r - a.round0, err, itp, snap, go, spre, e.x, r, j)) continue;
        const Scalars u = uniform_scalars(reinterpret_cast<const Scalars *>(snap));
        const Scalars *sv = &u;
        const int mode = sv->mode;
        const int lb = (int)e.y;
        double acc[kRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const int first = xcd_remap(lb, a.grid);
        const int m = (int)(sv->refreshes & 1);
        const Step<T> st = make_step(a, sv);
        if (mode != MODE_CG) {
            const double sigma_next = sv->sigma_next;
            const bool bonly = sv->first == 1;
            for (int k = 0; k < a.tpw; ++k) {
                const int tile = first + k * a.grid;
                if (tile >= a.ntiles) break;
                const int tx = tile % a.ntx, ty = tile / a.ntx;
                const int x0 = tx * Tile2D<T, SHAPE>::COLS;
                const int y0 = ty * Tile2D<T, SHAPE>::ROWS + w * Tile2D<T, SHAPE>::TY;
                const int y1 = min(y0 + Tile2D<T, SHAPE>::TY, a.ny);
                for (int sg = 0; sg < Tile2D<T, SHAPE>::SEG; ++sg) {
                    const int xx = x0 + kWave * sg + lane;
                    if (xx < a.nx)
                        for (int yy = y0; yy < y1; ++yy)
                            refresh_node<T, 2, COH>(a, a.P[m], a.P[m ^ 1], xx, yy, 0, st, sigma_next, bonly, acc);
                }
            }
        } else {
            const T alpha = (T)sv->alpha, beta = (T)sv->beta;
            for (int k = 0; k < a.tpw; ++k) {
                const int tile = first + k * a.grid;
                if (tile >= a.ntiles) break;
                if (k > 0) __syncthreads();          // the previous tile's LDS rows are reused
                const int tx = tile % a.ntx, ty = tile / a.ntx;
                cg2d_tile<T, SHAPE, COH>(a, a.P[m], tx * Tile2D<T, SHAPE>::COLS, ty * Tile2D<T, SHAPE>::ROWS, lane,
                                         w, alpha, beta, st, acc);
            }
        }
        finish_pass<COH>(acc, a.partials, a.tickets, s, lb, a.grid, a.groups, mode, spre);
    }
}

template <typename T, int COH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void pass3d_persist(
    const PassArgs<T> *__restrict__ tab, const uint2 *__restrict__ blk, const int *__restrict__ xoff, Scalars *scal,
    int64_t round_base, int rounds, int slot, unsigned *err, unsigned long long *queues)
{
    __shared__ unsigned long long snap[kScalWords];
    __shared__ int go[2];
    __shared__ unsigned long long claim[2];
    const int x = COH == 2 ? my_xcd() : 0;
    const int base = xoff[x], nblk = xoff[x + 1] - base;
    unsigned long long *queue = queues + 32 * x;
    const int64_t total = (int64_t)rounds * nblk;
    int itp = 0;
    for (int64_t it = first_claim(queue, claim); it < total; it = next_claim(claim, itp), itp ^= 1) {
        if (threadIdx.x == 0) claim[itp ^ 1] = __hip_atomic_fetch_add(queue, 1ull, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
        const int r = (int)(it / nblk);
        const int j = base + (int)(it - (int64_t)r * nblk);
        const uint2 e = blk ? blk[j] : make_uint2((unsigned)slot, (unsigned)j);
        const int parity = (int)((round_base + r) & 1);
        const PassArgs<T> &a = tab[2 * e.x + parity];
        Scalars *s = scal + e.x;
        unsigned long long spre = 0;
        if (!begin_item<COH>(s, round_base + r - a.round0, err, itp, snap, go, spre, e.x, r, j)) continue;
        const Scalars u = uniform_scalars(reinterpret_cast<const Scalars *>(snap));
        const Scalars *sv = &u;
        const int mode = sv->mode;
        const int lb = (int)e.y;
        double acc[kRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const int tile = xcd_remap(lb, a.grid);
        const int m = (int)(sv->refreshes & 1);
        const Step<T> st = make_step(a, sv);
        if (tile < a.ntiles) {
            const int tx = tile % a.ntx;
            const int ty = (tile / a.ntx) % a.nty;
            const int tz = tile / (a.ntx * a.nty);
            const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * a.tile_z;
            const int z1 = min(z0 + a.tile_z, a.nz);
            if (mode == MODE_CG) {
                cg3d_tile<T, COH>(a, a.P[m], x0, y0, z0, z1, (T)sv->alpha, (T)sv->beta, st, acc);
            } else {
                const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
                const double sigma_next = sv->sigma_next;
                const bool bonly = sv->first == 1;
                const int xx = x0 + lane;
                if (xx < a.nx)
                    for (int jj = 0; jj < kRows; ++jj) {
                        const int yy = y0 + w * kRows + jj;
                        if (yy >= a.ny) break;
                        for (int zz = z0; zz < z1; ++zz)
                            refresh_node<T, 3, COH>(a, a.P[m], a.P[m ^ 1], xx, yy, zz, st, sigma_next, bonly, acc);
                    }
            }
        }
        // an idle workgroup of the padded grid still reaches the reduction
        finish_pass<COH>(acc, a.partials, a.tickets, s, lb, a.grid, a.groups, mode, spre);
    }
}

// ---------------------------------------------------------------- setup kernels

__device__ __forceinline__ void coords(const Lat &L, int64_t i, int &x, int &y, int &z)
{
    x = (int)(i % L.nx);
    const int64_t t = i / L.nx;
    y = (int)(t % L.ny);
    z = (int)(t / L.ny);
}

__device__ __forceinline__ int face_code(const Lat &L, int x, int y, int z)
{
    const int c = L.axis == 0 ? x : (L.axis == 1 ? y : z);
    const int na = L.axis == 0 ? L.nx : (L.axis == 1 ? L.ny : L.nz);
    return c == 0 ? 1 : (c == na - 1 ? 2 : 0);
}

// Count lattice conductances (wrap bonds included) that are negative, NaN or infinite.
__global__ void validate_kernel(Lat L, const double *g0, const double *g1, const double *g2,
                                unsigned long long *bad)
{
    unsigned long long cnt = 0;
    const double *g[3] = {g0, g1, g2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        const int c[3] = {x, y, z};
        const int n[3] = {L.nx, L.ny, L.nz};
        for (int k = 0; k < L.dim; ++k) {
            if (c[k] + 1 >= n[k] && !((L.wrap >> k) & 1)) continue;   // ignored edge entry
            const double v = g[k][i];
            if (!(v >= 0.0) || isinf(v)) ++cnt;
        }
    }
    if (cnt) atomicAdd(bad, cnt);
}

// Lock-free union-find on int32 labels: a root is linked under the smaller
// root by CAS, so every component ends with its minimum node index as root,
// whatever the order of the unions.
__device__ __forceinline__ int uf_load(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int *parent, int x)
{
    while (true) {
        const int p = uf_load(parent + x);
        if (p == x) return x;
        const int gp = uf_load(parent + p);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

__device__ __forceinline__ void uf_union(int *parent, int a, int b)
{
    while (true) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expected = a;
        if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

__global__ void uf_init_kernel(int64_t n, int *parent, unsigned *flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        parent[i] = (int)i;
        flags[i] = 0u;
    }
}

// Union across every occupied bond joining two interior nodes (a wrap bond
// joins two nodes of the same plane along the flow axis).
__global__ void uf_union_kernel(Lat L, const double *g0, const double *g1, const double *g2, int *parent)
{
    const double *g[3] = {g0, g1, g2};
    const int64_t st[3] = {1, L.nx, (int64_t)L.nx * L.ny};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        if (face_code(L, x, y, z)) continue;
        const int c[3] = {x, y, z};
        const int n[3] = {L.nx, L.ny, L.nz};
        for (int k = 0; k < L.dim; ++k) {
            int64_t j;
            if (c[k] + 1 < n[k]) j = i + st[k];
            else if ((L.wrap >> k) & 1) j = i - (int64_t)(n[k] - 1) * st[k];   // wrap bond (never the flow axis)
            else continue;
            if (!(g[k][i] > 0.0)) continue;
            if (k == L.axis && c[k] + 1 == n[k] - 1) continue;     // neighbour on the outlet face
            uf_union(parent, (int)i, (int)j);
        }
    }
}

// Tag each component with the faces it touches through occupied bonds (only
// neighbours along the flow axis can be face nodes).
__global__ void uf_flags_kernel(Lat L, const double *ga, int *parent, unsigned *flags)
{
    const int64_t sa = L.axis == 0 ? 1 : (L.axis == 1 ? (int64_t)L.nx : (int64_t)L.nx * L.ny);
    const int na = L.axis == 0 ? L.nx : (L.axis == 1 ? L.ny : L.nz);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        const int c = L.axis == 0 ? x : (L.axis == 1 ? y : z);
        if (c == 0 || c == na - 1) continue;
        unsigned bits = 0u;
        if (c == 1 && ga[i - sa] > 0.0) bits |= 1u;
        if (c == na - 2 && ga[i] > 0.0) bits |= 2u;
        if (bits) atomicOr(flags + uf_find(parent, (int)i), bits);
    }
}

// Mask byte, initial pressure field (faces 1 / 0, dead nodes 1 when tied to
// the inlet only, live nodes the CG's initial guess: the linear profile
// 1 - c_axis / (n_axis - 1) when `linear`, else 0; not written when P is
// null) and the live count.
__global__ void mask_final_kernel(Lat L, int *parent, const unsigned *flags, uint8_t *mask, double *P,
                                  unsigned long long *n_live, int linear)
{
    unsigned long long cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        const int f = face_code(L, x, y, z);
        uint8_t m;
        double p0;
        if (f == 1) {
            m = 5;
            p0 = 1.0;
        } else if (f == 2) {
            m = 6;
            p0 = 0.0;
        } else {
            m = (uint8_t)flags[uf_find(parent, (int)i)];
            p0 = (m == 1) ? 1.0 : 0.0;
            if (m == 3) {   // initial guess on the live set: the linear profile along the flow axis, or 0
                const int ca = L.axis == 0 ? x : (L.axis == 1 ? y : z);
                const int na = L.axis == 0 ? L.nx : (L.axis == 1 ? L.ny : L.nz);
                p0 = linear ? 1.0 - (double)ca / (double)(na - 1) : 0.0;
                ++cnt;
            }
        }
        mask[i] = m;
        if (P) P[i] = p0;
    }
    cnt = (unsigned long long)wave_sum((double)cnt);
    if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(n_live, cnt);
}

// Conductances in the inner precision and zeroed CG state. A bond is kept
// when it lies in the lattice (or is a wrap bond) and both of its ends are
// live or face nodes (mask 3, 5 or 6): every occupied bond of a live node
// leads to a live or face node, so a live node keeps all of its bonds and
// their sum is its Jacobi diagonal, while a dead interior node keeps none.
template <typename T>
__global__ void scale_kernel(Lat L, const double *g0, const double *g1, const double *g2, const uint8_t *mask,
                             T *h0, T *h1, T *h2, T *vec, int64_t nvec)
{
    const double *g[3] = {g0, g1, g2};
    T *h[3] = {h0, h1, h2};
    const int64_t st[3] = {1, L.nx, (int64_t)L.nx * L.ny};
    auto keep = [](uint8_t m) { return m == 3 || m >= 5; };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        const int c[3] = {x, y, z};
        const int n[3] = {L.nx, L.ny, L.nz};
        const bool ki = keep(mask[i]);
        for (int k = 0; k < L.dim; ++k) {
            int64_t j = -1;
            if (c[k] + 1 < n[k]) j = i + st[k];
            else if ((L.wrap >> k) & 1) j = i - (int64_t)(n[k] - 1) * st[k];
            h[k][i] = (j >= 0 && ki && keep(mask[j])) ? (T)g[k][i] : T(0);
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
         i += (int64_t)gridDim.x * blockDim.x)
        vec[i] = T(0);
}

// Sum of direct inlet-outlet bonds (only when the flow axis has 2 planes).
__global__ void direct_flux_kernel(Lat L, const double *ga, double *out)
{
    __shared__ double red[kBlock / kWave];
    const int64_t sa = L.axis == 0 ? 1 : (L.axis == 1 ? (int64_t)L.nx : (int64_t)L.nx * L.ny);
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < L.n; i += blockDim.x) {
        int x, y, z;
        coords(L, i, x, y, z);
        if (face_code(L, x, y, z) != 1) continue;
        const double v = ga[i];
        if (v > 0.0) acc += v;
        (void)sa;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / kWave; ++k) t += red[k];
        *out = t;
    }
}

__global__ void clear_u64_kernel(unsigned long long *p, int n)
{
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) p[i] = 0ull;
}

// Conductances of the launch-shape trials: values in [1, 2) from a
// multiplicative hash of the entry index (no zero, so every node is live).
__global__ void fill_trial_kernel(double *g, int64_t n, uint32_t salt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = ((uint32_t)i ^ salt) * 2654435761u;
        g[i] = 1.0 + (double)(h >> 8) * (1.0 / 16777216.0);
    }
}

// ---------------------------------------------------------------- static scratch
// Device memory of the allocation-free mask entry point: the union-find
// parents and the component flags (4 bytes each per node) and four 8-byte
// counters, for lattices of up to kNoAllocMaxNodes nodes. Every GPU the
// library runs on holds its own copy until the process ends. Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address): noalloc_setup() looks up the device
// address once per device, with that device current, and every launch uses
// that address.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;      // the caller makes `device` current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

hipError_t launch_fill_trial(double *g, int64_t n, uint32_t salt, hipStream_t st)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    fill_trial_kernel<<<(int)(b < 1 ? 1 : b), kBlock, 0, st>>>(g, n, salt);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t st)
{
    clear_u64_kernel<<<1, kWave, 0, st>>>(p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- compact (gather) path
// For networks where few nodes take part (the live set, or the backbone, near
// the percolation threshold) the lattice sweep moves the bytes of every node.
// The compact path lists the m nodes that take part, in lattice order, with
// their 2 dim neighbour slots (the neighbour's list index; -2 / -3 for a bond
// to the inlet / outlet face; -1 for none), and runs the same CG in two
// launches per iteration:
//   A: the FP64 field takes the pending step (P += sigma alpha p), then
//      z' = z - alpha u and p' = z' + beta p, in place;
//   B: q = A p' by gathering the neighbours' p', u = M^-1 q, and the four dot
//      products of the dense pass, reduced by finish_pass (same tickets,
//      same scalar step). A refresh round runs in B alone (A sees its mode
//      and does nothing): r = b - A P in FP64 with the pending step added to
//      every pressure read, as refresh_node does, into the other P buffer.
// Each pending step is applied in the next A, so at most one is pending.
template <typename T>
__global__ __launch_bounds__(kBlock) void compact_pass_a(CompactArgs<T> a, const Scalars *s)
{
    if (s->mode != MODE_CG) return;
    const T alpha = (T)s->alpha, beta = (T)s->beta;
    const double sa = s->sigma * s->alpha;
    double *P = a.P[s->refreshes & 1];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.m; c += gridDim.x * blockDim.x) {
        const T p0 = a.p[c];
        if (sa != 0.0) P[c] = fma(sa, (double)p0, P[c]);
        const T zc = a.z[c] - alpha * a.u[c];
        a.z[c] = zc;
        a.p[c] = zc + beta * p0;
    }
}

// SLOTS = 2 dim, a compile-time count so that a node's neighbour indices,
// bonds and gathered directions are all in flight at once.
template <typename T, int SLOTS>
__global__ __launch_bounds__(kBlock) void compact_pass_b(CompactArgs<T> a, Scalars *s)
{
    const int mode = s->mode;
    if (mode == MODE_DONE) return;
    const unsigned long long spre = prefetch_scalars(s);
    double acc[kRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const bool jacobi = a.jacobi != 0;
    if (mode == MODE_CG) {
        for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.m; c += gridDim.x * blockDim.x) {
            const T pc = a.p[c];
            int j[SLOTS];
            T g[SLOTS], pn[SLOTS];
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) {
                j[e] = a.nbr[(size_t)e * a.m + c];
                g[e] = a.gT[(size_t)e * a.m + c];
            }
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) pn[e] = a.p[j[e] >= 0 ? j[e] : c];   // in-bounds address, then select
            T q = T(0);
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) q += g[e] * (pc - (j[e] >= 0 ? pn[e] : T(0)));
            const T d = a.d[c];
            const T uv = d > T(0) ? apply_minv(q, d, jacobi) : T(0);
            a.u[c] = uv;
            const double dq = (double)q, dz = (double)a.z[c];
            acc[0] += (double)pc * dq;
            acc[1] += dz * dq;
            acc[2] += dq * (double)uv;
            acc[3] += (double)(jacobi ? d : T(1)) * dz * dz;
        }
    } else {
        const int m = (int)(s->refreshes & 1);
        const double *Ps = a.P[m];
        double *Pd = a.P[m ^ 1];
        const double sa = s->sigma * s->alpha, sigma_next = s->sigma_next;
        const bool bonly = s->first == 1;
        for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.m; c += gridDim.x * blockDim.x) {
            const double Pi = Ps[c];
            const double pi = bonly ? 0.0 : (sa != 0.0 ? fma(sa, (double)a.p[c], Pi) : Pi);
            int j[SLOTS];
            double g[SLOTS], Pj[SLOTS];
            T pj[SLOTS];
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) {
                j[e] = a.nbr[(size_t)e * a.m + c];
                g[e] = a.g64[(size_t)e * a.m + c];
            }
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) {
                const int jj = j[e] >= 0 ? j[e] : c;
                Pj[e] = Ps[jj];
                pj[e] = a.p[jj];
            }
            double r64 = 0.0, qin = 0.0, qout = 0.0;
#pragma unroll
            for (int e = 0; e < SLOTS; ++e) {
                if (g[e] == 0.0) continue;
                if (j[e] >= 0) {
                    const double pn = bonly ? 0.0 : (sa != 0.0 ? fma(sa, (double)pj[e], Pj[e]) : Pj[e]);
                    r64 += g[e] * (pn - pi);
                } else if (j[e] == -2) {
                    r64 += g[e] * (1.0 - pi);
                    qin += g[e] * (1.0 - pi);
                } else {
                    r64 += g[e] * (0.0 - pi);
                    qout += g[e] * pi;
                }
            }
            const T dT = a.d[c];
            const T rs = (T)(r64 / sigma_next);
            const T zs = dT > T(0) ? apply_minv(rs, dT, jacobi) : T(0);
            Pd[c] = bonly ? Pi : pi;
            a.z[c] = zs;
            a.u[c] = T(0);
            acc[0] += r64 * r64;
            acc[1] += (double)rs * (double)zs;
            acc[2] += pi * r64;
            acc[3] += qin;
            acc[4] += qout;
        }
    }
    finish_pass<0>(acc, a.partials, a.tickets, s, (int)blockIdx.x, a.grid, a.groups, mode, spre);
}

// Members (mask == want) counted per block of kCmpChunk nodes.
constexpr int kCmpChunk = 4 * kBlock;

__global__ __launch_bounds__(kBlock) void compact_count(const uint8_t *mask, int64_t n, uint8_t want, int *counts)
{
    const int64_t b0 = (int64_t)blockIdx.x * kCmpChunk;
    int c = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + (int64_t)k * kBlock + threadIdx.x;
        if (i < n && mask[i] == want) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, kWave);
    __shared__ int ws[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += ws[w];
        counts[blockIdx.x] = t;
    }
}

// Exclusive scan of the block counts in one workgroup; offsets[nb] = total.
__global__ __launch_bounds__(kBlock) void compact_scan(const int *counts, int nb, int *offsets)
{
    __shared__ int ws[kBlock / kWave];
    __shared__ int carry;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kBlock) {
        const int v = b0 + (int)threadIdx.x < nb ? counts[b0 + threadIdx.x] : 0;
        int inc = v;
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) ws[w] = inc;
        __syncthreads();
        int before = carry;
        for (int ww = 0; ww < w; ++ww) before += ws[ww];
        if (b0 + (int)threadIdx.x < nb) offsets[b0 + threadIdx.x] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[nb] = carry;
}

// List index of every member (in lattice order) and the lattice -> list map.
__global__ __launch_bounds__(kBlock) void compact_place(const uint8_t *mask, int64_t n, uint8_t want,
                                                        const int *offsets, int *idx, int *cmap)
{
    __shared__ int ws[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t b0 = (int64_t)blockIdx.x * kCmpChunk;
    int base = offsets[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + (int64_t)k * kBlock + threadIdx.x;
        const int f = (i < n && mask[i] == want) ? 1 : 0;
        int inc = f;
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) ws[w] = inc;
        __syncthreads();
        int before = base;
        for (int ww = 0; ww < w; ++ww) before += ws[ww];
        int total = base;
        for (int ww = 0; ww < kBlock / kWave; ++ww) total += ws[ww];
        if (i < n) {
            const int c = before + inc - f;
            cmap[i] = f ? c : -1;
            if (f) idx[c] = (int)i;
        }
        __syncthreads();
        base = total;
    }
}

// Neighbour slots, bonds, inner diagonal and the state of every member; the
// initial field from the lattice field P0.
template <typename T>
__global__ __launch_bounds__(kBlock) void compact_tables(Lat L, const double *g0, const double *g1, const double *g2,
                                                         const int *idx, const int *cmap, int m, int *nbr, T *gT,
                                                         double *g64, T *d, const double *P0, double *P, T *z, T *u,
                                                         T *p)
{
    const double *g[3] = {g0, g1, g2};
    const int n3[3] = {L.nx, L.ny, L.nz};
    const int64_t st[3] = {1, (int64_t)L.nx, (int64_t)L.nx * L.ny};
    const int na = n3[L.axis];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m; c += gridDim.x * blockDim.x) {
        const int64_t i = idx[c];
        const int cc[3] = {(int)(i % L.nx), (int)((i / L.nx) % L.ny), (int)(i / ((int64_t)L.nx * L.ny))};
        T gs[6];
        for (int e = 0; e < 2 * L.dim; ++e) {
            const int k = e >> 1;
            const bool up = e & 1, wk = (L.wrap >> k) & 1;
            int64_t j = -1;
            double gv = 0.0;
            if (up) {
                if (cc[k] + 1 < n3[k]) j = i + st[k];
                else if (wk) j = i - (int64_t)(n3[k] - 1) * st[k];
                if (j >= 0) gv = g[k][i];
            } else {
                if (cc[k] > 0) j = i - st[k];
                else if (wk) j = i + (int64_t)(n3[k] - 1) * st[k];
                if (j >= 0) gv = g[k][j];
            }
            int code = -1;
            if (j >= 0 && gv > 0.0) {
                const int ca = k == L.axis ? cc[k] + (up ? 1 : -1) : cc[L.axis];
                if (ca == 0) code = -2;
                else if (ca == na - 1) code = -3;
                else code = cmap[j];              // -1: not a member (a bond that carries no current)
            }
            if (code == -1) gv = 0.0;
            nbr[(size_t)e * m + c] = code;
            g64[(size_t)e * m + c] = gv;
            gs[e] = (T)gv;
            gT[(size_t)e * m + c] = gs[e];
        }
        d[c] = L.dim == 2 ? diag_sum(gs[0], gs[1], gs[2], gs[3]) : diag_sum(gs[0], gs[1], gs[2], gs[3], gs[4], gs[5]);
        P[c] = P0[i];
        z[c] = u[c] = p[c] = T(0);
    }
}

__global__ __launch_bounds__(kBlock) void compact_scatter(const int *idx, int m, const double *P, double *Pl)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m; c += gridDim.x * blockDim.x) Pl[idx[c]] = P[c];
}

// ---------------------------------------------------------------- host launchers

static inline int grid_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_validate(const Lat &L, const double *const g[3], unsigned long long *bad, hipStream_t st)
{
    validate_kernel<<<grid_for(L.n), kBlock, 0, st>>>(L, g[0], g[1], L.dim == 3 ? g[2] : nullptr, bad);
    return hipGetLastError();
}

hipError_t launch_mask(const Lat &L, const double *const g[3], int *parent, unsigned *flags, uint8_t *mask,
                       double *P, unsigned long long *n_live, bool linear, hipStream_t st)
{
    const int gr = grid_for(L.n);
    const double *g2 = L.dim == 3 ? g[2] : nullptr;
    uf_init_kernel<<<gr, kBlock, 0, st>>>(L.n, parent, flags);
    uf_union_kernel<<<gr, kBlock, 0, st>>>(L, g[0], g[1], g2, parent);
    uf_flags_kernel<<<gr, kBlock, 0, st>>>(L, g[L.axis], parent, flags);
    mask_final_kernel<<<gr, kBlock, 0, st>>>(L, parent, flags, mask, P, n_live, linear ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(const Lat &L, const double *const g[3], const uint8_t *mask, T *const gT[3], T *vec,
                        int64_t nvec, hipStream_t st)
{
    scale_kernel<T><<<grid_for(L.n), kBlock, 0, st>>>(L, g[0], g[1], L.dim == 3 ? g[2] : nullptr, mask, gT[0],
                                                      gT[1], L.dim == 3 ? gT[2] : nullptr, vec, nvec);
    return hipGetLastError();
}

hipError_t launch_direct_flux(const Lat &L, const double *ga, double *out, hipStream_t st)
{
    direct_flux_kernel<<<1, kBlock, 0, st>>>(L, ga, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass(int dim, const PassArgs<T> *tab, const uint2 *blk, Scalars *scal, int nblocks, int parity,
                       int slot, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (dim == 2) pass2d_kernel<T, 0><<<nblocks, kBlock, 0, st>>>(tab, blk, scal, parity, slot);
    else if (dim == -2) pass2d_kernel<T, 1><<<nblocks, kBlock, 0, st>>>(tab, blk, scal, parity, slot);
    else pass3d_kernel<T><<<nblocks, kBlock, 0, st>>>(tab, blk, scal, parity, slot);
    return hipGetLastError();
}

// Workgroups of one persistent launch: as many as the kernel's occupancy
// keeps resident on all CUs at once (more would only queue behind them).
template <typename T, int COH>
static hipError_t persist_capacity(int dim, int *cap)
{
    static int cached[2][3] = {{0, 0, 0}, {0, 0, 0}};
    const int fi = sizeof(T) == 8 ? 1 : 0, di = dim == 2 ? 0 : (dim == -2 ? 1 : 2);
    if (cached[fi][di]) {
        *cap = cached[fi][di];
        return hipSuccess;
    }
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (dim == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pass2d_persist<T, 0, COH>, kBlock, 0);
    else if (dim == -2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pass2d_persist<T, 1, COH>, kBlock, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pass3d_persist<T, COH>, kBlock, 0);
    if (e != hipSuccess) return e;
    if (per < 1 || cus < 1) return hipErrorInvalidConfiguration;
    cached[fi][di] = per * cus;
    *cap = cached[fi][di];
    return hipSuccess;
}

template <typename T, int COH>
static hipError_t persist_launch(int dim, const PassArgs<T> *tab, const uint2 *blk, const int *xoff, Scalars *scal,
                                 int nblocks, int64_t round_base, int rounds, int slot, unsigned *err,
                                 unsigned long long *queues, hipStream_t st)
{
    int cap = 0;
    hipError_t e = persist_capacity<T, COH>(dim, &cap);
    if (e != hipSuccess) return e;
    // every XCD needs workgroups of its own for COH 2 (workgroups are dealt to
    // the 8 XCDs in turn, so any grid of at least 8 covers them)
    const int64_t items = (int64_t)nblocks * rounds;
    const int grid = (int)std::max<int64_t>(COH == 2 ? 64 : 1, std::min<int64_t>(items, (int64_t)cap));
    // the queue counters start at 0 (a kernel, not a memset node)
    e = launch_clear_u64(queues, 32 * 8, st);
    if (e != hipSuccess) return e;
    if (dim == 2)
        pass2d_persist<T, 0, COH><<<grid, kBlock, 0, st>>>(tab, blk, xoff, scal, round_base, rounds, slot, err, queues);
    else if (dim == -2)
        pass2d_persist<T, 1, COH><<<grid, kBlock, 0, st>>>(tab, blk, xoff, scal, round_base, rounds, slot, err, queues);
    else
        pass3d_persist<T, COH><<<grid, kBlock, 0, st>>>(tab, blk, xoff, scal, round_base, rounds, slot, err, queues);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_persist(int dim, int coh, const PassArgs<T> *tab, const uint2 *blk, const int *xoff,
                               Scalars *scal, int nblocks, int64_t round_base, int rounds, int slot, unsigned *err,
                               unsigned long long *queues, hipStream_t st)
{
    if (nblocks <= 0 || rounds <= 0) return hipSuccess;
    if (coh == 2) return persist_launch<T, 2>(dim, tab, blk, xoff, scal, nblocks, round_base, rounds, slot, err, queues, st);
    return persist_launch<T, 1>(dim, tab, blk, xoff, scal, nblocks, round_base, rounds, slot, err, queues, st);
}

template hipError_t launch_pass_persist<float>(int, int, const PassArgs<float> *, const uint2 *, const int *,
                                               Scalars *, int, int64_t, int, int, unsigned *, unsigned long long *,
                                               hipStream_t);
template hipError_t launch_pass_persist<double>(int, int, const PassArgs<double> *, const uint2 *, const int *,
                                                Scalars *, int, int64_t, int, int, unsigned *, unsigned long long *,
                                                hipStream_t);
template hipError_t launch_scale<float>(const Lat &, const double *const[3], const uint8_t *, float *const[3],
                                        float *, int64_t, hipStream_t);
template hipError_t launch_scale<double>(const Lat &, const double *const[3], const uint8_t *, double *const[3],
                                         double *, int64_t, hipStream_t);
template hipError_t launch_pass<float>(int, const PassArgs<float> *, const uint2 *, Scalars *, int, int, int,
                                       hipStream_t);
template hipError_t launch_pass<double>(int, const PassArgs<double> *, const uint2 *, Scalars *, int, int, int,
                                        hipStream_t);


// ---------------------------------------------------------------- compact launchers
int compact_blocks(int64_t n) { return (int)((n + kCmpChunk - 1) / kCmpChunk); }

hipError_t launch_compact_index(const uint8_t *mask, int64_t n, uint8_t want, int *counts, int *offsets, int *idx,
                                int *cmap, hipStream_t st)
{
    const int nb = compact_blocks(n);
    compact_count<<<nb, kBlock, 0, st>>>(mask, n, want, counts);
    compact_scan<<<1, kBlock, 0, st>>>(counts, nb, offsets);
    compact_place<<<nb, kBlock, 0, st>>>(mask, n, want, offsets, idx, cmap);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_compact_tables(const Lat &L, const double *const g[3], const int *idx, const int *cmap, int m,
                                 int *nbr, T *gT, double *g64, T *d, const double *P0, double *P, T *z, T *u, T *p,
                                 hipStream_t st)
{
    compact_tables<T><<<grid_for(m), kBlock, 0, st>>>(L, g[0], g[1], L.dim == 3 ? g[2] : nullptr, idx, cmap, m, nbr,
                                                      gT, g64, d, P0, P, z, u, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_compact_round(const CompactArgs<T> &a, Scalars *s, hipStream_t st)
{
    compact_pass_a<T><<<a.grid, kBlock, 0, st>>>(a, s);
    if (a.slots == 6) compact_pass_b<T, 6><<<a.grid, kBlock, 0, st>>>(a, s);
    else compact_pass_b<T, 4><<<a.grid, kBlock, 0, st>>>(a, s);
    return hipGetLastError();
}

hipError_t launch_compact_scatter(const int *idx, int m, const double *P, double *Pl, hipStream_t st)
{
    compact_scatter<<<grid_for(m), kBlock, 0, st>>>(idx, m, P, Pl);
    return hipGetLastError();
}

template hipError_t launch_compact_tables<float>(const Lat &, const double *const[3], const int *, const int *, int,
                                                 int *, float *, double *, float *, const double *, double *, float *,
                                                 float *, float *, hipStream_t);
template hipError_t launch_compact_tables<double>(const Lat &, const double *const[3], const int *, const int *, int,
                                                  int *, double *, double *, double *, const double *, double *,
                                                  double *, double *, double *, hipStream_t);
template hipError_t launch_compact_round<float>(const CompactArgs<float> &, Scalars *, hipStream_t);
template hipError_t launch_compact_round<double>(const CompactArgs<double> &, Scalars *, hipStream_t);

}  // namespace rn
