// rn_device.hpp -- structures shared by the host runtime and the gfx950 kernels.
//
// The CG state of one network lives in HBM for the whole solve; the host only
// enqueues launches and reads a small status block now and then.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rn {

// Per-network control block (device memory). One pass kernel launch reads
// mode / alpha / beta / sigma at entry; the last workgroup to finish reduces
// the partial sums in a fixed order and writes the next mode and scalars. The
// host copies the blocks to pinned memory after each chunk of launches.
enum PassMode : int32_t { MODE_CG = 0, MODE_REFRESH = 1, MODE_DONE = 2 };

struct Scalars {
    int32_t mode;       // PassMode of the next launch
    int32_t status;     // 0 ok, -3 not converged, -4 breakdown
    int32_t converged;
    int32_t first;      // the next refresh evaluates b (x = 0)
    int32_t stop;       // finish after the pending refresh (breakdown path)
    int32_t fp32;       // inner vectors are FP32
    int32_t check;      // the pending refresh is a convergence check
    int32_t flush;      // the next CG pass adds every pending step to the FP64 field
    int32_t kpend;      // steps a CG pass may leave pending before one adds them all (2 or 4)
    int32_t npend;      // steps pending after the last pass (a refresh counts one, of size 0)
    int64_t iters;      // CG passes executed
    int64_t refreshes;  // refresh passes executed
    int64_t passes;     // passes that did work
    int64_t max_iter;
    double alpha;       // step of the pending update x += alpha p, z -= alpha u
    double alpha2;      // steps of the updates before it, newest first, still pending while
    double alpha3;      // the CG passes after them left the FP64 field alone (else 0)
    double alpha4;
    double beta;        // p = z + beta p in the next CG pass
    double rho;         // exact r_k.z_k of the stored residual at the last CG pass
    double sigma;       // the stored state (z = D^-1 r, p, u = D^-1 A p) is scaled by 1 / sigma
    double sigma_next;  // sigma the pending refresh will use
    double rmax;        // largest stored sqrt(r.z) since the last refresh
    double tol, delta;
    double bnorm;       // ||b||_2 (unscaled)
    double bhat;        // sqrt(b.D^{-1}b)
    double kappa;       // (||r|| / ||b||) / sqrt(r.D^-1 r / b.D^-1 b), measured at the last refresh
    double est_rel;     // predicted unscaled relative residual after the last CG pass
    double rel_resid;   // true relative residual measured by the last refresh
    double last_check;  // true relative residual at the previous failed convergence check
    double est_check;   // predicted relative residual that triggered the pending check
    double Q_in, Q_out, xr;  // fluxes and x.(b - A x) from the last refresh
    // to 256 bytes: control blocks of different networks share no 128-byte
    // line, so networks placed on different XCDs never write one line
    uint32_t pad_[4];
};

constexpr int kRed = 5;          // partial sums per workgroup
// Completion tickets of a pass: workgroup lb counts on the counter of its
// group lb % groups (groups = a power of two up to kGroupsMax, about one per
// 64 workgroups); the last of each group counts on the top counter. Counters
// sit kTicketStride bytes apart (17 x 256 B: another 256-byte channel slot and
// 4 KB page each) so that the groups' atomics proceed in parallel instead of
// queueing on one address.
#ifndef RN_GROUPS_MAX
#define RN_GROUPS_MAX 8
#endif
constexpr int kGroupsMax = RN_GROUPS_MAX;
constexpr int kTicketStride = 17 * 256;
inline size_t ticket_bytes(int groups) { return (size_t)(groups + 1) * kTicketStride; }
constexpr int kBlock = 256;      // threads per workgroup of every kernel here
constexpr int kWave = 64;

// CG state of one parity: z = D^-1 r and u = D^-1 A p. The direction p has
// kpend + 1 buffers (PassArgs::pbuf) because a pass may still need the ones
// of the kpend - 1 passes before.
template <typename T>
struct VecSet {
    T *z, *u;
};

// Arguments of the pass kernel (2D and 3D share the layout). Every working
// pass reads `src` and writes `dst`; the host alternates the two sets.
template <typename T>
struct PassArgs {
    // lattice
    int nx, ny, nz, axis;
    int ntx, nty, ntz;           // tile counts
    int wrap;                    // bit k: direction k wraps around (periodic sides)
    int tile_z;                  // planes per 3D tile
    int jacobi;                  // 1: M = diag(d) (z = D^-1 r, u = D^-1 q); 0: M = I (z = r, u = q)
    int ntiles;                  // total workgroup tiles
    int tpw;                     // tiles per workgroup, `grid` tiles apart (2D; 3D: 1)
    int grid;                    // workgroups of this network per pass (multiple of 8 and of groups)
    int groups;                  // completion-ticket groups (power of two, divides grid)
    int64_t round0;              // engine pass round of the network's first pass (persistent launches
                                 // wait for round - round0 completed passes before a round's item)
    // FP64 data
    const double *g64[3];        // original conductances
    double *P[2];                // full FP64 pressure field: CG passes after refresh m add their
                                 // step to P[m%2] in place; refresh m reads P[m%2], writes P[(m+1)%2]
    // inner-precision CG state
    const T *gT[3];              // conductances in the inner precision: 0 past the lattice edge
                                 // (the wrap bond on the last plane of a periodic direction) and
                                 // 0 where either end is an interior node off the live set, so
                                 // the sum of a node's bonds is its Jacobi diagonal d_i, > 0
                                 // exactly on live and face nodes
    const uint8_t *mask;         // mask byte per node (3 = live)
    VecSet<T> src, dst;
    T *pbuf[5];                  // direction p in npbuf = kpend + 1 buffers: the c-th pass of a
                                 // solve (Scalars::passes = c) writes pbuf[c % npbuf] and reads
                                 // pbuf[(c - 1) % npbuf]; a CG pass that flushes the FP64 field
                                 // also reads the buffers of the older pending steps
    int npbuf;
    // reduction
    double *partials;            // [grid][kRed]
    unsigned *tickets;           // groups + 1 counters, kTicketStride bytes apart, zero between passes
    Scalars *s;
};

struct Lat {
    int dim, axis, nx, ny, nz;
    int64_t n;
    int wrap;    // bit k: direction k wraps around (periodic sides, extent >= 2)
};

// launchers (rn_kernels.hip)
hipError_t launch_validate(const Lat &L, const double *const g[3], unsigned long long *bad, hipStream_t st);
// linear: the live nodes' initial pressure is the linear profile along the
// flow axis (else 0); P may be null (mask and live count only)
hipError_t launch_mask(const Lat &L, const double *const g[3], int *parent, unsigned *flags, uint8_t *mask,
                       double *P, unsigned long long *n_live, bool linear, hipStream_t st);
template <typename T>
hipError_t launch_scale(const Lat &L, const double *const g[3], const uint8_t *mask, T *const gT[3], T *vec,
                        int64_t nvec, hipStream_t st);
hipError_t launch_direct_flux(const Lat &L, const double *ga, double *out, hipStream_t st);
// zero n counters with a kernel (no memset node, so a captured graph may hold it)
hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t st);
// g[i] in [1, 2) from a hash of i and salt (the networks of the launch-shape trials)
hipError_t launch_fill_trial(double *g, int64_t n, uint32_t salt, hipStream_t st);

// Compact (gather) path: the m nodes that take part, in lattice order, with
// 2 dim neighbour slots each (see rn_kernels.hip).
template <typename T>
struct CompactArgs {
    int m, slots, grid, groups, jacobi;
    const int *nbr;              // [slots][m]: list index, -2 inlet face, -3 outlet face, -1 none
    const T *gT;                 // [slots][m] inner-precision bonds (0 where none)
    const double *g64;           // [slots][m]
    const T *d;                  // [m] inner diagonal: the sum of the node's gT
    double *P[2];                // FP64 field; a refresh reads P[refreshes & 1] and writes the other
    T *z, *u, *p;                // [m]
    double *partials;            // [grid][kRed]
    unsigned *tickets;           // groups + 1 counters, kTicketStride bytes apart
};
int compact_blocks(int64_t n);   // blocks of the member count / placement launches
// idx[c]: lattice index of member c (mask == want), in lattice order; cmap[i]:
// member index of lattice node i or -1; counts: compact_blocks(n) ints;
// offsets: compact_blocks(n) + 1 ints, offsets[last] = m.
hipError_t launch_compact_index(const uint8_t *mask, int64_t n, uint8_t want, int *counts, int *offsets, int *idx,
                                int *cmap, hipStream_t st);
template <typename T>
hipError_t launch_compact_tables(const Lat &L, const double *const g[3], const int *idx, const int *cmap, int m,
                                 int *nbr, T *gT, double *g64, T *d, const double *P0, double *P, T *z, T *u, T *p,
                                 hipStream_t st);
// one CG or refresh round (the control block's mode decides): two launches
template <typename T>
hipError_t launch_compact_round(const CompactArgs<T> &a, Scalars *s, hipStream_t st);
hipError_t launch_compact_scatter(const int *idx, int m, const double *P, double *Pl, hipStream_t st);

// Backbone (rn_backbone.hip): with `mask` the connectivity mask of the
// lattice, set bit 3 on every interior node of the backbone and add their
// number to *n_backbone (a device counter). `scratch` holds
// backbone_scratch_bytes(n) device bytes; h_stage is pinned host memory of
// kBackboneStage ints for the level offsets the breadth-first search reads
// back (one synchronisation of `st` per kBackboneStage - 2 levels). Needs
// n + 2 < 2^31 and at least 3 planes on the flow axis. *depth_out (nullable)
// receives the number of levels of the search.
constexpr int kBackboneStage = 34;
size_t backbone_scratch_bytes(int64_t n);
hipError_t launch_backbone(const Lat &L, const double *const g[3], uint8_t *mask, void *scratch,
                           unsigned long long *n_backbone, int *h_stage, int *depth_out, hipStream_t st);
// With `mask` from launch_backbone (backbone 11, dangling 3): find the pieces
// of dangling nodes (uf, n ints) and the backbone node each hangs from (att,
// n ints, at the piece's root) from the bonds g, then, when gw (a writable
// device copy of g) is given, zero in place every bond of gw with a dangling end.
hipError_t launch_backbone_prune(const Lat &L, const double *const g[3], double *const gw[3], const uint8_t *mask,
                                 int *uf, int *att, hipStream_t st);
// After the solve of the pruned network: every dangling node takes the
// pressure of the backbone node its piece hangs from.
hipError_t launch_backbone_fill(const Lat &L, const uint8_t *mask, int *uf, const int *att, double *P,
                                hipStream_t st);

// Static scratch of the allocation-free mask entry point: 8 bytes per node
// (union-find parents and component flags) for up to kNoAllocMaxNodes nodes,
// then four 8-byte counters. noalloc_setup(device), called with `device`
// current, looks up that device's copy once; noalloc_scratch(device) returns
// it afterwards (nullptr before the setup).
constexpr int64_t kNoAllocMaxNodes = (int64_t)1 << 22;
constexpr size_t kNoAllocCounterOffset = (size_t)kNoAllocMaxNodes * 8;
constexpr size_t kNoAllocScratchBytes = kNoAllocCounterOffset + 256;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_setup(int device);
void *noalloc_scratch(int device);
// One pass of every network in the block table blk[0..nblocks): entry
// (network, local block); tab[2 * network + parity] are that network's
// arguments and scal[network] its control block. dim: 2 (2D, full tiles),
// -2 (2D, small tiles) or 3. With blk == nullptr the launch covers the one
// network in `slot`, local block = blockIdx.x.
template <typename T>
hipError_t launch_pass(int dim, const PassArgs<T> *tab, const uint2 *blk, Scalars *scal, int nblocks, int parity,
                       int slot, hipStream_t st);
// `rounds` pass rounds of every network in the block table in one launch
// (rounds round_base .. round_base + rounds - 1 of the engine); dim, tab,
// blk, scal and slot as for launch_pass, nblocks the table's length. coh 1:
// items in one queue (xoff = {0, nblocks, ..., nblocks}), any workgroup takes
// any item, the state moves by device-scope accesses; coh 2: entries
// xoff[x] .. xoff[x + 1] - 1 (9 ints, device memory) are the networks the
// host placed on XCD x, claimed only by workgroups running there. *err
// (device memory, zero on entry) becomes nonzero when a wait exceeded its
// bound; queues (device memory, 8 x 32 words, cleared by the launcher) are
// the per-XCD item counters.
template <typename T>
hipError_t launch_pass_persist(int dim, int coh, const PassArgs<T> *tab, const uint2 *blk, const int *xoff,
                               Scalars *scal, int nblocks, int64_t round_base, int rounds, int slot, unsigned *err,
                               unsigned long long *queues, hipStream_t st);

// tile geometry of the pass kernels: a 2D workgroup tile is 64 kSEG2f x
// 4 kTY2f (FP32) or 64 kSEG2d x 4 kTY2d (FP64): each wave holds kTY2f / kTY2d
// rows of kSEG2f / kSEG2d 64-column segments; a 3D workgroup tile is
// 64 x kTY x tile_z
#ifndef RN_TY2F
#define RN_TY2F 4
#endif
#ifndef RN_TY2D
#define RN_TY2D 2
#endif
#ifndef RN_SEG2F
#define RN_SEG2F 2
#endif
#ifndef RN_SEG2D
#define RN_SEG2D 2
#endif
#ifndef RN_TY3
#define RN_TY3 16
#endif
#ifndef RN_TZ3
#define RN_TZ3 16
#endif
constexpr int kTX = 64, kTY = RN_TY3, kTZ = RN_TZ3;
constexpr int kTY2f = RN_TY2F, kTY2d = RN_TY2D, kSEG2f = RN_SEG2F, kSEG2d = RN_SEG2D;
constexpr int kTY2fS = 2, kTY2dS = 1;   // rows per wave of the small 2D tile (one 64-column segment)


__host__ __device__ inline int div_up(int a, int b) { return (a + b - 1) / b; }

}  // namespace rn
