// rn_backbone.hip -- the backbone of the sample-spanning cluster on the GPU.
//
// Near the percolation threshold (Sec. VI) most live nodes sit on dangling
// ends: branches and loops that meet the rest of the cluster at one node and
// carry no flow. The backbone is the set of interior nodes on an inlet-outlet
// path that visits no node twice. With the inlet face contracted to a vertex
// S, the outlet face to T and an edge S-T added, it is the vertex set of the
// biconnected component (block) that holds S-T.
//
// Blocks by Tarjan and Vishkin's parallel method, on a breadth-first spanning
// tree rooted at S:
//   1. BFS, one launch per level; new vertices are appended to one queue with
//      one atomic per wave, so each level is a contiguous segment of it. T is
//      S's first child; S's other children are the live nodes with a bond to
//      the inlet face, T's children those with a bond to the outlet face that
//      no lattice node reached first. A vertex stores the direction of its
//      tree bond (so the second bond between two nodes of a periodic
//      direction of extent 2 stays a separate, non-tree edge).
//   2. Subtree sizes nd, level by level from the deepest.
//   3. Preorder numbers pre, level by level from the root: a child of a
//      lattice node comes after its siblings of lower direction index;
//      S's and T's children follow their place in the queue (a scan).
//   4. low / high: the extreme preorder numbers reachable from a subtree by
//      one non-tree edge, level by level from the deepest.
//   5. Tree edges (named by their child vertex) are joined in a lock-free
//      union-find: a non-tree edge whose ends are not ancestor and
//      descendant joins the two ends' tree edges; a tree edge (p, v) with p
//      not the root joins p's when low(v) < pre(p) or high(v) >=
//      pre(p) + nd(p). The classes are the blocks.
//   6. The backbone is the set of lattice ends of the tree edges in T's class
//      (T's tree edge is S-T): bit 3 (8) of the mask.
// Any spanning tree works for the method, so the BFS races (which parent a
// vertex gets) change the tree but not the blocks: the mask is deterministic.
#include "rn_runtime.hpp"

#include <algorithm>
#include <vector>

namespace rn {
namespace {

constexpr int kBbBlock = 256;
constexpr int kBbGrid = 512;              // grid-stride launches over one level
constexpr uint8_t kParS = 6, kParT = 7, kParNone = 255;

struct BbGraph {
    const double *g[3];
    const uint8_t *mask;
    int dim, axis, nx, ny, nz, wrap;
    int n, S, T;                          // lattice vertices 0..n-1, then S = n, T = n + 1
};

__device__ __forceinline__ void coords(const BbGraph &G, int v, int c[3])
{
    c[0] = v % G.nx;
    c[1] = (v / G.nx) % G.ny;
    c[2] = v / (G.nx * G.ny);
}

// Lattice index across direction e (k = e / 2, towards +k when e is odd) of
// node v, or -1 off the lattice; *gij the bond's conductance.
__device__ __forceinline__ int lat_step(const BbGraph &G, int v, const int c[3], int e, double *gij)
{
    const int k = e >> 1;
    const int n[3] = {G.nx, G.ny, G.nz};
    const int st[3] = {1, G.nx, G.nx * G.ny};
    const bool wk = (G.wrap >> k) & 1;
    if (e & 1) {
        int j;
        if (c[k] + 1 < n[k]) j = v + st[k];
        else if (wk) j = v - (n[k] - 1) * st[k];
        else return -1;
        *gij = G.g[k][v];
        return j;
    }
    int j;
    if (c[k] > 0) j = v - st[k];
    else if (wk) j = v + (n[k] - 1) * st[k];
    else return -1;
    *gij = G.g[k][j];
    return j;
}

// Vertex joined to interior node v by its bond in direction e: a live
// interior node, S or T for a face node, -1 for no occupied bond or a node
// off the live set.
__device__ __forceinline__ int bb_nbr(const BbGraph &G, int v, const int c[3], int e)
{
    if ((e >> 1) >= G.dim) return -1;
    double gij = 0.0;
    const int j = lat_step(G, v, c, e, &gij);
    if (j < 0 || !(gij > 0.0)) return -1;
    if ((e >> 1) == G.axis) {
        const int na = G.axis == 0 ? G.nx : (G.axis == 1 ? G.ny : G.nz);
        const int ca = c[G.axis] + ((e & 1) ? 1 : -1);
        if (ca == 0) return G.S;
        if (ca == na - 1) return G.T;
    }
    return G.mask[j] == 3 ? j : -1;
}

// Parent vertex of v from its tree-bond direction.
__device__ __forceinline__ int bb_parent(const BbGraph &G, int v, uint8_t pd)
{
    if (v == G.T || pd == kParS) return G.S;
    if (pd == kParT) return G.T;
    int c[3];
    coords(G, v, c);
    double gij;
    return lat_step(G, v, c, pd, &gij);
}

// Append the lanes with `take` set to the queue, one atomic per wave.
__device__ __forceinline__ void wave_append(bool take, int v, int *order, int *tail)
{
    const unsigned long long m = __ballot(take);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(tail, __popcll(m));
    base = __shfl(base, leader, 64);
    if (take) order[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

__global__ void bb_init(int *lev, uint8_t *pdir, int *nd, int *pre, int *uf, uint8_t *on, int V, int S, int T,
                        int *order, int *lev_off, int *tail)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
        lev[v] = v == S ? 0 : (v == T ? 1 : -1);
        pdir[v] = v == T ? kParS : kParNone;
        nd[v] = 1;
        pre[v] = 0;                     // S keeps 0, the root's number
        uf[v] = v;
        on[v] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        order[0] = S;
        order[1] = T;
        lev_off[0] = 0;
        lev_off[1] = 1;
        *tail = 2;
    }
}

// The live nodes next to face `which` (1 inlet, 2 outlet) with a bond to it
// join level l as children of S (which = 1) or T (2), unless already seen.
__global__ void bb_face_children(BbGraph G, int which, int l, int *lev, uint8_t *pdir, int *order, int *tail)
{
    const int na = G.axis == 0 ? G.nx : (G.axis == 1 ? G.ny : G.nz);
    const int ca = which == 1 ? 1 : na - 2;
    const int m = G.axis == 0 ? G.ny * G.nz : (G.axis == 1 ? G.nx * G.nz : G.nx * G.ny);   // nodes of the plane
    const int rounds = (m + (int)(gridDim.x * blockDim.x) - 1) / (int)(gridDim.x * blockDim.x);
    for (int r = 0; r < rounds; ++r) {
        const int q = r * (int)(gridDim.x * blockDim.x) + blockIdx.x * blockDim.x + threadIdx.x;
        bool take = false;
        int v = 0;
        if (q < m) {
            int c[3];
            if (G.axis == 0) { c[0] = ca; c[1] = q % G.ny; c[2] = q / G.ny; }
            else if (G.axis == 1) { c[0] = q % G.nx; c[1] = ca; c[2] = q / G.nx; }
            else { c[0] = q % G.nx; c[1] = q / G.nx; c[2] = ca; }
            v = c[0] + G.nx * (c[1] + G.ny * c[2]);
            if (G.mask[v] == 3) {
                const int e = 2 * G.axis + (which == 1 ? 0 : 1);
                if (bb_nbr(G, v, c, e) == (which == 1 ? G.S : G.T) && atomicCAS(&lev[v], -1, l) == -1) {
                    pdir[v] = which == 1 ? kParS : kParT;
                    take = true;
                }
            }
        }
        wave_append(take, v, order, tail);
    }
}

// Expand level l: every lattice vertex of it claims its unseen neighbours for l + 1.
__global__ void bb_expand(BbGraph G, int l, const int *lev_off, int *lev, uint8_t *pdir, int *order, int *tail)
{
    const int b = lev_off[l], e = lev_off[l + 1];
    const int stride = (int)(gridDim.x * blockDim.x);
    const int rounds = (e - b + stride - 1) / stride;
    for (int r = 0; r < rounds; ++r) {
        const int q = b + r * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const int v = q < e ? order[q] : G.S;
        int c[3] = {0, 0, 0};
        const bool lat = v < G.n;
        if (lat) coords(G, v, c);
        for (int d = 0; d < 6; ++d) {
            bool take = false;
            int w = -1;
            if (lat) {
                w = bb_nbr(G, v, c, d);
                if (w >= 0 && w < G.n && atomicCAS(&lev[w], -1, l + 1) == -1) {
                    pdir[w] = (uint8_t)(d ^ 1);
                    take = true;
                }
            }
            wave_append(take, w, order, tail);
        }
    }
}

__global__ void bb_snap(int *lev_off, const int *tail, int l)
{
    if (threadIdx.x == 0) lev_off[l + 2] = *tail;
}

// Subtree sizes: the vertices of level l add theirs to their parents.
__global__ void bb_sizes(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, int *nd)
{
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        const int p = bb_parent(G, v, pdir[v]);
        if (p != G.S) atomicAdd(&nd[p], nd[v]);
    }
}

// Preorder numbers of the children of S (the level-1 segment, all of them) or
// of T (the entries of the level-2 segment whose parent is T): base + the
// sizes of the earlier children, by one workgroup scanning the segment.
__global__ void bb_scan_children(int b, int e, const int *order, const uint8_t *pdir, uint8_t want, int base,
                                 const int *nd, int *pre)
{
    constexpr int kPer = 8;
    __shared__ int wsum[kBbBlock / 64];
    __shared__ int carry_s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = b; c0 < e; c0 += kBbBlock * kPer) {
        int val[kPer], tot = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int q = c0 + threadIdx.x * kPer + k;
            int v = 0;
            if (q < e) {
                const int u = order[q];
                v = pdir[u] == want ? nd[u] : 0;
            }
            val[k] = v;
            tot += v;
        }
        // inclusive scan of the per-thread totals within the wave, then across waves
        int inc = tot;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int before = carry_s;
        for (int ww = 0; ww < w; ++ww) before += wsum[ww];
        int run = before + inc - tot;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int q = c0 + threadIdx.x * kPer + k;
            if (q < e) {
                const int u = order[q];
                if (pdir[u] == want) pre[u] = base + run;
            }
            run += val[k];
        }
        __syncthreads();
        if (threadIdx.x == kBbBlock - 1) carry_s = run;
        __syncthreads();
    }
}

// Preorder numbers of level l's vertices whose parent is a lattice node:
// pre(parent) + 1 + the sizes of the parent's children of lower direction.
__global__ void bb_preorder(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, const int *nd,
                            int *pre)
{
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        const uint8_t pd = pdir[v];
        if (pd >= kParS) continue;
        int c[3];
        coords(G, v, c);
        double gij;
        const int p = lat_step(G, v, c, pd, &gij);
        int cp[3];
        coords(G, p, cp);
        const int ev = pd ^ 1;                   // direction from p to v
        int s = 0;
        for (int d = 0; d < ev; ++d) {
            const int u = bb_nbr(G, p, cp, d);
            if (u >= 0 && u < G.n && pdir[u] == (uint8_t)(d ^ 1)) s += nd[u];
        }
        pre[v] = pre[p] + 1 + s;
    }
}

// Whether the edge from v in direction d to w is a tree edge.
__device__ __forceinline__ bool is_tree(const BbGraph &G, int w, uint8_t pv, const uint8_t *pdir, int d)
{
    if (w == G.S) return pv == kParS;
    if (w == G.T) return pv == kParT;
    return pv == (uint8_t)d || pdir[w] == (uint8_t)(d ^ 1);
}

// low / high of every visited vertex from its own non-tree edges. T's are
// left out: T's tree edge goes to the root, where no join looks at them.
__global__ void bb_lohi_init(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, const int *pre,
                             int *lo, int *hi)
{
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        int l = pre[v], h = pre[v];
        if (v < G.n) {
            int c[3];
            coords(G, v, c);
            const uint8_t pv = pdir[v];
            for (int d = 0; d < 2 * G.dim; ++d) {
                const int w = bb_nbr(G, v, c, d);
                if (w < 0 || is_tree(G, w, pv, pdir, d)) continue;
                l = min(l, pre[w]);
                h = max(h, pre[w]);
            }
        }
        lo[v] = l;
        hi[v] = h;
    }
}

__global__ void bb_lohi_up(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, int *lo, int *hi)
{
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        const int p = bb_parent(G, v, pdir[v]);
        if (p == G.S) continue;
        atomicMin(&lo[p], lo[v]);
        atomicMax(&hi[p], hi[v]);
    }
}

// The union-find reads and writes through the L2 (device scope): a plain load
// may be served from the CU's L1, which keeps a line another CU has since
// hooked, and a root that looks unhooked there would be retried forever.
__device__ __forceinline__ int uf_get(const int *uf, int x)
{
    return __hip_atomic_load(uf + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int *uf, int x)
{
    int p = uf_get(uf, x);
    while (p != x) {
        const int gp = uf_get(uf, p);
        // halve the path: gp is an ancestor of x (parents have smaller
        // indices), and only non-roots are written, never a root a hook targets
        if (gp != p) __hip_atomic_store(uf + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = uf_get(uf, x);
    }
    return x;
}

__device__ __forceinline__ void uf_union(int *uf, int a, int b)
{
    while (true) {
        a = uf_find(uf, a);
        b = uf_find(uf, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&uf[a], a, b) == a) return;   // hook the larger root under the smaller
    }
}

__device__ __forceinline__ bool ancestor(const int *pre, const int *nd, int a, int v)
{
    return pre[a] <= pre[v] && pre[v] < pre[a] + nd[a];
}

// The Tarjan-Vishkin joins for every visited vertex other than S.
__global__ void bb_join(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, const int *pre,
                        const int *nd, const int *lo, const int *hi, int *uf)
{
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        const uint8_t pv = pdir[v];
        const int p = bb_parent(G, v, pv);
        if (p != G.S && (lo[v] < pre[p] || hi[v] >= pre[p] + nd[p])) uf_union(uf, v, p);
        if (v >= G.n) continue;
        int c[3];
        coords(G, v, c);
        for (int d = 0; d < 2 * G.dim; ++d) {
            const int w = bb_nbr(G, v, c, d);
            if (w < 0 || w == G.S || is_tree(G, w, pv, pdir, d)) continue;
            if (!ancestor(pre, nd, w, v) && !ancestor(pre, nd, v, w)) uf_union(uf, v, w);
        }
    }
}

// Lattice ends of the tree edges in T's class.
__global__ void bb_mark(BbGraph G, int b, int e, const int *order, const uint8_t *pdir, int *uf, uint8_t *on)
{
    const int rt = uf_find(uf, G.T);
    for (int q = b + blockIdx.x * blockDim.x + threadIdx.x; q < e; q += gridDim.x * blockDim.x) {
        const int v = order[q];
        if (uf_find(uf, v) != rt) continue;
        if (v < G.n) on[v] = 1;
        const int p = bb_parent(G, v, pdir[v]);
        if (p < G.n) on[p] = 1;
    }
}

__global__ void bb_apply(uint8_t *mask, const uint8_t *on, int n, unsigned long long *count)
{
    int c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (on[i]) {
            mask[i] |= 8u;
            ++c;
        }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

// ---------------------------------------------------------------- solves on the backbone
// With the backbone marked (11) and the other live nodes dangling (3), a solve
// may cut the dangling ends out: they carry no current, so the backbone's
// pressures and every flux are unchanged. Each connected piece of dangling
// nodes meets the backbone at exactly one node a (a piece joined to two
// backbone nodes, or to a face and the backbone, would lie on a path that
// visits no node twice) and, carrying no current, sits at a's pressure.

// Pieces of dangling nodes: union over occupied bonds between two of them.
__global__ void bb_piece_union(BbGraph G, int *uf, int *att)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        if (G.mask[i] != 3) continue;
        att[i] = -1;
        int c[3];
        coords(G, i, c);
        for (int d = 1; d < 2 * G.dim; d += 2) {           // each bond once, from its -k end
            const int w = bb_nbr(G, i, c, d);               // a dangling neighbour (mask 3), or S, T, -1
            if (w >= 0 && w < G.n) uf_union(uf, i, w);
        }
    }
}

// The backbone node each piece hangs from, stored at the piece's root (every
// dangling node next to it writes the same index).
__global__ void bb_piece_attach(BbGraph G, int *uf, int *att)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        if (G.mask[i] != 3) continue;
        int c[3];
        coords(G, i, c);
        for (int d = 0; d < 2 * G.dim; ++d) {
            double gij = 0.0;
            const int j = lat_step(G, i, c, d, &gij);
            if (j >= 0 && gij > 0.0 && G.mask[j] == 11) att[uf_find(uf, i)] = j;
        }
    }
}

// Zero every bond with a dangling end (in place: entry g[k][i] is the bond
// from i to its +k neighbour).
__global__ void bb_prune(BbGraph G, double *g0, double *g1, double *g2)
{
    double *gk[3] = {g0, g1, g2};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += gridDim.x * blockDim.x) {
        int c[3];
        coords(G, i, c);
        const bool di = G.mask[i] == 3;
        for (int k = 0; k < G.dim; ++k) {
            double gij = 0.0;
            const int j = lat_step(G, i, c, 2 * k + 1, &gij);
            if (j >= 0 && (di || G.mask[j] == 3)) gk[k][i] = 0.0;
        }
    }
}

// Pressures of the dangling nodes: that of the backbone node their piece hangs from.
__global__ void bb_fill(const uint8_t *mask, int *uf, const int *att, double *P, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mask[i] != 3) continue;
        const int a = att[uf_find(uf, i)];
        if (a >= 0) P[i] = P[a];
    }
}

__global__ void bb_iota(int *uf, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) uf[i] = i;
}

BbGraph graph_of(const Lat &L, const double *const g[3], const uint8_t *mask)
{
    BbGraph G;
    for (int k = 0; k < 3; ++k) G.g[k] = k < L.dim ? g[k] : nullptr;
    G.mask = mask;
    G.dim = L.dim;
    G.axis = L.axis;
    G.nx = L.nx;
    G.ny = L.ny;
    G.nz = L.nz;
    G.wrap = L.wrap;
    G.n = (int)L.n;
    G.S = (int)L.n;
    G.T = (int)L.n + 1;
    return G;
}

int grid_of(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBbBlock - 1) / kBbBlock, 8192));
}

}  // namespace

size_t backbone_scratch_bytes(int64_t n)
{
    const size_t V = (size_t)n + 2;
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    return 7 * a256(4 * V) + 2 * a256(V) + a256(4 * (V + 40)) + 256;
}

hipError_t launch_backbone(const Lat &L, const double *const g[3], uint8_t *mask, void *scratch,
                           unsigned long long *n_backbone, int *h_stage, int *depth_out, hipStream_t st)
{
    const int64_t n = L.n;
    const int V = (int)(n + 2);
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char *p = (char *)scratch;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += a256(bytes);
        return r;
    };
    int *lev = (int *)take(4 * (size_t)V), *nd = (int *)take(4 * (size_t)V), *pre = (int *)take(4 * (size_t)V);
    int *lo = (int *)take(4 * (size_t)V), *hi = (int *)take(4 * (size_t)V), *uf = (int *)take(4 * (size_t)V);
    int *order = (int *)take(4 * (size_t)V);
    uint8_t *pdir = (uint8_t *)take((size_t)V), *on = (uint8_t *)take((size_t)V);
    int *lev_off = (int *)take(4 * ((size_t)V + 40));
    int *tail = (int *)take(256);

    const BbGraph G = graph_of(L, g, mask);

    hipError_t e;
    bb_init<<<grid_of(V), kBbBlock, 0, st>>>(lev, pdir, nd, pre, uf, on, V, G.S, G.T, order, lev_off, tail);
    // 1. BFS: level 0 = S, level 1 = T and S's lattice children
    bb_face_children<<<kBbGrid, kBbBlock, 0, st>>>(G, 1, 1, lev, pdir, order, tail);
    bb_snap<<<1, 64, 0, st>>>(lev_off, tail, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // levels l >= 1 in batches of kBatch launches, then one read-back of the
    // level offsets; a level past the last is empty and does nothing
    // (h_stage: kBackboneStage pinned ints)
    constexpr int kBatch = kBackboneStage - 2;
    std::vector<int> off = {0, 1};       // level offsets read back so far
    int depth = -1;                      // number of levels, once an empty one is seen
    for (int l0 = 1; depth < 0; l0 += kBatch) {
        if (l0 + kBatch + 2 > V + 40) return hipErrorInvalidValue;   // cannot happen: levels <= V
        for (int l = l0; l < l0 + kBatch; ++l) {
            bb_expand<<<kBbGrid, kBbBlock, 0, st>>>(G, l, lev_off, lev, pdir, order, tail);
            if (l == 1) bb_face_children<<<kBbGrid, kBbBlock, 0, st>>>(G, 2, 2, lev, pdir, order, tail);
            bb_snap<<<1, 64, 0, st>>>(lev_off, tail, l);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // offsets l0 + 1 .. l0 + kBatch + 1 (the ones this batch wrote)
        if ((e = hipMemcpyAsync(h_stage, lev_off + l0 + 1, sizeof(int) * (size_t)(kBatch + 1), hipMemcpyDeviceToHost,
                                st)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        off.resize((size_t)l0 + 1);
        for (int k = 0; k <= kBatch; ++k) off.push_back(h_stage[k]);
        for (int l = l0; l < l0 + kBatch; ++l)
            if (off[(size_t)l + 1] == off[(size_t)l]) {
                depth = l;
                break;
            }
    }
    // levels 0 .. depth-1 hold vertices: level l is order[off[l] .. off[l+1])
    const int nvis = off[depth];
    // 2. subtree sizes, deepest level first
    for (int l = depth - 1; l >= 1; --l)
        bb_sizes<<<grid_of(off[l + 1] - off[l]), kBbBlock, 0, st>>>(G, off[l], off[l + 1], order, pdir, nd);
    // 3. preorder: S = 0 (never read), S's children, T's children, then the rest by level
    bb_scan_children<<<1, kBbBlock, 0, st>>>(off[1], off[2], order, pdir, kParS, 1, nd, pre);
    if (depth > 2) {
        bb_scan_children<<<1, kBbBlock, 0, st>>>(off[2], off[3], order, pdir, kParT, 2, nd, pre);
        for (int l = 2; l < depth; ++l)
            bb_preorder<<<grid_of(off[l + 1] - off[l]), kBbBlock, 0, st>>>(G, off[l], off[l + 1], order, pdir, nd,
                                                                             pre);
    }
    // 4. low / high
    bb_lohi_init<<<grid_of(nvis - 1), kBbBlock, 0, st>>>(G, 1, nvis, order, pdir, pre, lo, hi);
    for (int l = depth - 1; l >= 2; --l)
        bb_lohi_up<<<grid_of(off[l + 1] - off[l]), kBbBlock, 0, st>>>(G, off[l], off[l + 1], order, pdir, lo, hi);
    // 5. joins, 6. marks
    bb_join<<<grid_of(nvis - 1), kBbBlock, 0, st>>>(G, 1, nvis, order, pdir, pre, nd, lo, hi, uf);
    bb_mark<<<grid_of(nvis - 1), kBbBlock, 0, st>>>(G, 1, nvis, order, pdir, uf, on);
    bb_apply<<<grid_of(n), kBbBlock, 0, st>>>(mask, on, (int)n, n_backbone);
    if (depth_out) *depth_out = depth;
    return hipGetLastError();
}

hipError_t launch_backbone_prune(const Lat &L, const double *const g[3], double *const gw[3], const uint8_t *mask,
                                 int *uf, int *att, hipStream_t st)
{
    const BbGraph G = graph_of(L, g, mask);
    const int gr = grid_of(L.n);
    bb_iota<<<gr, kBbBlock, 0, st>>>(uf, (int)L.n);
    bb_piece_union<<<gr, kBbBlock, 0, st>>>(G, uf, att);
    bb_piece_attach<<<gr, kBbBlock, 0, st>>>(G, uf, att);
    if (gw) bb_prune<<<gr, kBbBlock, 0, st>>>(G, gw[0], gw[1], L.dim == 3 ? gw[2] : nullptr);
    return hipGetLastError();
}

hipError_t launch_backbone_fill(const Lat &L, const uint8_t *mask, int *uf, const int *att, double *P,
                                hipStream_t st)
{
    bb_fill<<<grid_of(L.n), kBbBlock, 0, st>>>(mask, uf, att, P, (int)L.n);
    return hipGetLastError();
}

}  // namespace rn
