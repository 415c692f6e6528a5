/*
 * rn.h -- C ABI of librn, a gfx950 (MI355X) solver for steady flow through
 * random resistor / pore networks (Dashtian & Sahimi, Sec. II).
 *
 * Problem (Sec. II, Eq. 3): a square (2D) or simple-cubic (3D) lattice of
 * nodes joined by bonds of conductance g_ij >= 0 (g = 0: removed bond, the
 * percolation dilution of Sec. V-VI). Mass balance sum_j g_ij (P_j - P_i) = 0
 * holds at every interior node; the first node plane along the flow axis
 * (inlet face) is held at P = 1, the last plane (outlet face) at P = 0, and
 * either no flow crosses the side faces or, with RN_PERIODIC, the directions
 * other than the flow axis wrap around (the periodic side condition of
 * Sec. II). The library returns the total flux Q and
 * Darcy's K (Eq. 4) = Q (n_axis - 1) / S, with S the product of the extents
 * other than the flow axis (unit viscosity, bond length and pressure drop).
 *
 * Only interior nodes connected through occupied interior bonds to both
 * faces carry flow (the "live" set). The solve is preconditioned conjugate
 * gradients (Sec. II/IV; Jacobi by default) on the live set, either all in FP64 or
 * with FP32 inner iterations and FP64 residual refreshes, FP64 solution
 * accumulation and FP64 flux (the mixed-precision scheme of Sec. IV).
 *
 * Conventions
 *   - Every call returns an int status: RN_OK (0) or a negative RN_E* code.
 *     No C++ exception crosses the ABI.
 *   - Lattice layout: node i = x + nx*(y + ny*z) (x fastest). g[k] is an
 *     array of nx*ny*nz doubles; g[k][i] is the bond from node i to its
 *     neighbour i + e_k (k = 0,1,2 for x,y,z). Entries whose neighbour lies
 *     past the lattice edge are ignored (any value, even NaN), except on a
 *     periodic direction, where the last plane's entry is the bond to the
 *     first plane. g[2] must be NULL in 2D. Every other entry must be finite
 *     and >= 0 (RN_EINVAL otherwise).
 *   - Pointers in rn_problem live in the memory space named by its `mem`
 *     field: RN_MEM_HOST (pageable or pinned host memory) or RN_MEM_DEVICE
 *     (device memory on the context's GPU, e.g. a torch tensor's data_ptr).
 *   - All caller buffers are borrowed for the duration of the call and never
 *     freed by the library. Device memory the library needs belongs to the
 *     rn_ctx and is bounded by its HBM budget.
 *   - Calls on one rn_ctx are serialised internally; rn_submit, rn_poll and
 *     rn_stats may be called from any thread. Different contexts are
 *     independent.
 */
#ifndef RN_H
#define RN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RN_OK 0
#define RN_EINVAL (-1)    /* bad argument: dims, axis, NULL pointer, g < 0 / NaN / Inf, tol <= 0 */
#define RN_ENOMEM (-2)    /* the request does not fit the context's HBM budget or device memory */
#define RN_ENOCONV (-3)   /* max_iter reached; result holds the last iterate, converged = 0 */
#define RN_ENUMERIC (-4)  /* CG breakdown (p.Ap <= 0 or a non-finite reduction) */
#define RN_EDEVICE (-5)   /* a HIP runtime call failed; rn_last_error() has the message */
#define RN_EAGAIN (-6)    /* rn_poll: the ticket is still running */
#define RN_ENOTFOUND (-7) /* rn_poll: unknown or already collected ticket */

/* rn_opts.precision */
#define RN_FP64 0   /* FP64 CG throughout */
#define RN_MIXED 1  /* FP32 inner CG, FP64 residual refresh, solution and flux. The
                       inner CG uses the conductances rounded to FP32: a live node whose
                       bonds all round to 0 (below about 1e-38) is never corrected by it,
                       and the solve then ends with RN_ENOCONV; scale such inputs, since
                       K is linear in g. */

/* rn_opts.precond */
#define RN_JACOBI 0  /* M = diag(d), d_i = sum of the node's bond conductances (default) */
#define RN_NONE 1    /* no preconditioner (M = I) */

/* rn_opts.x0: initial guess of the pressures on the live set */
#define RN_X0_LINEAR 0  /* 1 - c_axis / (n_axis - 1), the exact solution of a uniform network
                           with no-flow sides (default) */
#define RN_X0_ZERO 1    /* 0 */

/* rn_opts.flags */
#define RN_OPT_BACKBONE 1  /* solve on the backbone (rn_build_backbone): the dangling ends, which
                              carry no current, are cut out before the CG and each takes the
                              pressure of the backbone node it hangs from afterwards. K, G, the
                              fluxes and every pressure are those of the whole network; the CG
                              runs on fewer nodes and, near the percolation threshold, in fewer
                              iterations. rn_solve and rn_solve_batch only (rn_submit: RN_EINVAL).
                              mask_out receives rn_build_backbone's mask; rn_result.n_live counts
                              the whole live set and n_backbone the backbone. */
#define RN_OPT_COMPACT 2   /* run the CG on a list of the nodes that take part (the live set, or the
                              backbone with RN_OPT_BACKBONE), each with its neighbours' list
                              indices, instead of sweeping the whole lattice: fewer bytes per
                              iteration when few nodes take part (near the percolation threshold).
                              The same method and stopping rule, so results agree with the lattice
                              path within the tolerance, not bit for bit. rn_solve and
                              rn_solve_batch only (rn_submit: RN_EINVAL); each such solve runs on
                              its own, before the rest of a batch. rn_result.passes counts the
                              rounds launched (two launches each). */

/* rn_problem.mem */
#define RN_MEM_HOST 0
#define RN_MEM_DEVICE 1

/* rn_problem.flags */
#define RN_PERIODIC 1  /* periodic sides (Sec. II): every direction k other than the flow axis
                          with extent >= 2 wraps around; g[k][i] on the last plane along k is
                          the bond to the node on the first plane. Without it the sides are
                          no-flow and those entries are ignored. */

typedef struct rn_ctx rn_ctx;

/* One network: lattice, flow axis, conductances, optional outputs. */
typedef struct {
    int32_t dim;        /* 2 or 3 */
    int32_t axis;       /* flow axis: 0 = x, 1 = y, 2 = z (< dim); its extent must be >= 2 */
    int64_t nx, ny, nz; /* extents >= 1; nz == 1 in 2D; nx*ny*nz < 2^31 */
    const double *g[3]; /* bond conductances, layout above; g[2] == NULL in 2D */
    double *p_out;      /* nullable, nx*ny*nz doubles: nodal pressures. Faces 1 / 0; live
                           nodes the solution; dead interior nodes 1 if connected to the
                           inlet only, else 0 */
    uint8_t *mask_out;  /* nullable, nx*ny*nz bytes: connectivity mask (rn_build_mask) */
    int32_t mem;        /* RN_MEM_HOST or RN_MEM_DEVICE for g, p_out and mask_out */
    int32_t flags;      /* 0 (no-flow sides) or RN_PERIODIC; other bits: RN_EINVAL */
} rn_problem;

/* Solver options; rn_opts_default() fills the defaults (all-zero fields other
 * than tol and max_iter are the defaults too). */
typedef struct {
    int32_t precision;  /* RN_FP64 (default) or RN_MIXED */
    int32_t precond;    /* RN_JACOBI (default) or RN_NONE */
    double tol;         /* stop when ||b - A x||_2 <= tol ||b||_2, the FP64 true residual on
                           the live set (default 1e-8) */
    int64_t max_iter;   /* cap on CG iterations, i.e. operator applications (default 10^7) */
    double delta;       /* RN_MIXED: the inner tolerance of the FP32 iterations. The FP64
                           residual is recomputed once the FP32 residual has fallen by this
                           factor since the last recomputation (0 = default 0.1); the inner
                           recurrence then continues from the FP64 residual (reliable update).
                           Ignored by RN_FP64. Must lie in [0, 1). */
    int32_t x0;         /* RN_X0_LINEAR (default) or RN_X0_ZERO */
    int32_t flags;      /* 0 (default), RN_OPT_BACKBONE, RN_OPT_COMPACT or both; other bits: RN_EINVAL */
} rn_opts;

/* Outcome of one solve. */
typedef struct {
    int32_t status;     /* RN_OK, RN_ENOCONV or RN_ENUMERIC */
    int32_t converged;  /* 1 when the true relative residual is <= tol */
    double Q_in;        /* flux leaving the inlet face (plus direct inlet-outlet bonds) */
    double Q_out;       /* flux entering the outlet face (plus direct bonds) */
    double G;           /* conductance in energy form: Q_in - x.(b - A x) = sum g dP^2 */
    double K;           /* Darcy K of Eq. 4: G (n_axis - 1) / S */
    double rel_resid;   /* final ||b - A x|| / ||b|| in FP64 (0 when nothing is live) */
    int64_t iters;      /* CG iterations */
    int64_t refreshes;  /* FP64 true-residual refreshes (the first computes b, the second the
                           residual of the initial guess, rn_opts.x0) */
    int64_t n_live;     /* interior nodes connected to both faces */
    int64_t passes;     /* pass rounds launched while this network iterated (a round launches
                           one pass kernel per kind of network present; idle rounds after
                           convergence, until the host notices, are included) */
    double t_mask_s;    /* device time: upload, validation and connectivity */
    double t_loop_s;    /* device time from the start of this network's iterations to the
                           end of its last round */
    double t_total_s;   /* host wall time from the call (or rn_submit) to completion */
    int64_t n_backbone; /* backbone nodes with RN_OPT_BACKBONE, else 0 */
} rn_result;

/* Library version, 100 * major + minor. */
int rn_version(void);

/* Human-readable name of a status code; never NULL. */
const char *rn_strerror(int status);

/* Fill *opts with the defaults above. RN_EINVAL if opts is NULL. */
int rn_opts_default(rn_opts *opts);

/*
 * Create a context on HIP device `device` with an HBM budget of
 * `hbm_budget_bytes` for the library's own buffers (0 = 90% of the device's
 * free memory at creation). The context owns a non-blocking stream at default
 * priority until rn_set_stream() replaces it. *out receives the handle.
 * How pass rounds are launched is read from the environment at creation;
 * results are bit-identical in every mode:
 *   RN_PERSIST=1  one persistent work-queue launch per chunk of rounds and
 *                 network kind, items claimed on all XCDs;
 *   RN_PERSIST=2  the same with each network of a kind of small networks
 *                 placed on one XCD (other kinds: one launch per round);
 *   RN_GRAPHS=1   rounds replayed from a captured hipGraph;
 *   otherwise one launch per round and kind.
 * Errors: RN_EINVAL (NULL out, bad device), RN_EDEVICE.
 */
int rn_create(int device, size_t hbm_budget_bytes, rn_ctx **out);

/* Release every device and host resource of the context. NULL is accepted. */
int rn_destroy(rn_ctx *ctx);

/*
 * Launch all further work of this context on `stream` (a hipStream_t, e.g.
 * torch.cuda.current_stream().cuda_stream); NULL restores the context's own
 * stream. The caller keeps ownership of the stream and must keep it alive.
 */
int rn_set_stream(rn_ctx *ctx, void *stream);

/* Message of the last RN_EDEVICE on this context, or of the last RN_ENOMEM of
 * rn_build_mask_noalloc ("" if none). */
const char *rn_last_error(rn_ctx *ctx);

/*
 * Check a problem and options without touching a device: shapes, axis,
 * pointers, flags, options and, for RN_MEM_HOST, every
 * conductance the lattice uses (finite, >= 0). opts may be NULL (defaults). Returns RN_OK or
 * RN_EINVAL; the same checks open rn_solve and rn_build_mask.
 */
int rn_validate(const rn_problem *prob, const rn_opts *opts);

/*
 * Device bytes one solve of `prob` with `opts` needs (opts NULL: defaults);
 * 0 when the problem is invalid. Used for admission against the budget.
 */
size_t rn_footprint(const rn_problem *prob, const rn_opts *opts);

/*
 * Connectivity mask of a network (the "live set" definition above; Sec. V-VI
 * dilution makes it non-trivial). Writes prob->mask_out (required), one byte
 * per node: bit0 = the node's interior component has an occupied bond to an
 * inlet-face node, bit1 = the same for the outlet face, bit2 = face node.
 * Inlet-face nodes are 5, outlet-face nodes 6, live interior nodes 3, other
 * interior nodes 0, 1 or 2. Paths run only through occupied interior-interior
 * bonds. *n_live_out (nullable) receives the number of live nodes.
 * Errors: RN_EINVAL, RN_ENOMEM, RN_EDEVICE; outputs untouched on error.
 */
int rn_build_mask(rn_ctx *ctx, const rn_problem *prob, int64_t *n_live_out);

/*
 * rn_build_mask for callers that cannot allocate device memory (code under
 * HIP graph construction, tight serving loops, harnesses that forbid
 * hipMalloc): the same mask and live count, computed in a static scratch
 * array that every GPU the library runs on holds until the process ends
 * (RN_NOALLOC_MAX_NODES x 8 bytes + 256 bytes, 32 MiB; the device address
 * is looked up once per device by rn_create). The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *   - prob->mem must be RN_MEM_DEVICE: g and mask_out are device buffers of
 *     the caller (mask_out required, nx*ny*nz bytes, written directly).
 *   - nx*ny*nz above RN_NOALLOC_MAX_NODES: RN_ENOMEM, and rn_last_error()
 *     names the limit; nothing runs.
 *   - Invalid conductances (negative, NaN, Inf): RN_EINVAL with mask_out
 *     untouched. RN_EINVAL also for a bad shape, host memory, a NULL
 *     mask_out or while the request server runs; RN_EDEVICE on a HIP error.
 *   - Runs on the context's stream and waits for it. Every call on one GPU
 *     shares that GPU's scratch: calls that overlap on one GPU (from two
 *     contexts, or two threads with different contexts) race and must be
 *     serialised by the caller. Each call clears the counters it uses.
 */
#define RN_NOALLOC_MAX_NODES (1 << 22)
int rn_build_mask_noalloc(rn_ctx *ctx, const rn_problem *prob, int64_t *n_live_out);

/*
 * Backbone of the sample-spanning cluster. Near the percolation threshold
 * (Sec. VI: the RRN with q -> q_c) most live nodes sit on dangling ends,
 * branches and loops that meet the rest of the cluster at one node and carry
 * no flow. The paper does not define the backbone; here it is the textbook
 * one: the interior nodes that lie on some path from an inlet-face node to an
 * outlet-face node visiting no node twice. Equivalently, with each face
 * contracted to one vertex and an edge added between the two, the nodes of
 * the biconnected component holding that edge. Computed on the device
 * (a breadth-first spanning tree and Tarjan and Vishkin's joins); the result
 * does not depend on the order in which the device visits nodes.
 * Writes prob->mask_out (required): the mask of rn_build_mask with bit3 (8)
 * set on backbone nodes, so backbone nodes are 11 and other live nodes stay
 * 3. *n_live_out and *n_backbone_out (nullable) receive the counts. Removing
 * the live nodes off the backbone changes no flux, and leaves a network whose
 * live set is the backbone. Memory: prob->mem for g and mask_out; the call
 * takes about 37 device bytes per node from the context's pool and
 * synchronises its stream once per 32 levels of the search.
 * Errors: RN_EINVAL (bad problem, NULL mask_out, nx*ny*nz + 2 >= 2^31, while
 * the request server runs), RN_ENOMEM, RN_EDEVICE; outputs untouched on error.
 */
int rn_build_backbone(rn_ctx *ctx, const rn_problem *prob, int64_t *n_live_out, int64_t *n_backbone_out);

/*
 * Solve one network (Sec. II, Eqs. 3-4): mask, preconditioned CG (opts->precond,
 * Jacobi by default) on the live set from the initial guess opts->x0 (the
 * linear profile along the flow axis by default, or 0) to opts->tol, then
 * fluxes, energy conductance and K, all reduced in FP64 on the device. Writes *out, and prob->p_out / prob->mask_out when
 * non-NULL. A network with no live node returns RN_OK, converged = 1,
 * iters = 0 and G = K = 0 except for direct inlet-outlet bonds (n_axis = 2).
 * Returns out->status (RN_OK, RN_ENOCONV, RN_ENUMERIC) once the solve ran;
 * RN_EINVAL / RN_ENOMEM / RN_EDEVICE before it (outputs untouched).
 */
int rn_solve(rn_ctx *ctx, const rn_problem *prob, const rn_opts *opts, rn_result *out);

/*
 * Solve `count` independent networks together (the batched form of rn_solve).
 * opts holds n_opts entries: 0 (opts may be NULL: defaults for all), 1 (the
 * same options for all) or count (one per network). out receives count
 * results. Networks of any size, dimension and precision share each pass
 * launch while keeping their own reductions and convergence; a network's
 * result is bit-identical to rn_solve of it alone. Networks wait for device
 * memory when the HBM budget is exhausted and start as others finish.
 * Returns RN_OK when every network converged, else the first non-OK
 * network status (per-network status in out[i].status); RN_EINVAL /
 * RN_ENOMEM (a network larger than the whole budget) / RN_EDEVICE before
 * any solve, with outputs untouched.
 */
int rn_solve_batch(rn_ctx *ctx, int32_t count, const rn_problem *probs, const rn_opts *opts, int32_t n_opts,
                   rn_result *out);

/*
 * Serving: queue one network for solving and return at once with a ticket.
 * The first call starts the context's server thread, which admits queued
 * networks as device memory (the HBM budget, per rn_footprint) and control
 * slots allow (in arrival order; when the oldest waiting network does not fit
 * the memory free now, later ones that fit go ahead of it, at most 8 times
 * before it is admitted), runs every admitted network in the same pass launches
 * (continuous batching: a network joins at the next chunk boundary and leaves
 * as soon as it converges) and frees its memory at once. The buffers named
 * by prob (g, p_out, mask_out) must stay valid and unmodified until rn_poll
 * returns for that ticket. Errors: RN_EINVAL, RN_ENOMEM (larger than the whole
 * budget); nothing is queued then. Thread-safe with rn_poll and rn_stats.
 * After the first rn_submit, rn_set_stream and rn_build_mask return
 * RN_EINVAL; rn_solve and rn_solve_batch go through the server.
 */
int rn_submit(rn_ctx *ctx, const rn_problem *prob, const rn_opts *opts, uint64_t *ticket_out);

/*
 * Result of a submitted network: RN_EAGAIN while it is queued or running;
 * once it is done, fills *out, forgets the ticket and returns out->status
 * (RN_OK, RN_ENOCONV, RN_ENUMERIC, RN_EINVAL for device-resident invalid
 * values, RN_ENOMEM, RN_EDEVICE); RN_ENOTFOUND for an unknown or already
 * collected ticket. out->t_total_s is the time from rn_submit to completion.
 */
int rn_poll(rn_ctx *ctx, uint64_t ticket, rn_result *out);

/* rn_plan_t.path: which pass kernel runs a network */
#define RN_PATH_2D_FULL 0   /* 2D, full tiles (64 x segments columns, 4 waves of rows) */
#define RN_PATH_2D_SMALL 1  /* 2D, quarter-size tiles (one 64-column segment, half the rows) */
#define RN_PATH_3D 2        /* 3D, 64 x 16 x tile_z blocks streamed along z */

/* Launch plan of one network: the tile its pass kernel uses and how many
 * workgroups one pass of it takes. The plan depends only on the network's
 * shape, dimension and precision, so a network runs the same arithmetic alone,
 * in a batch or in the served stream. */
typedef struct {
    int32_t path;          /* RN_PATH_* */
    int32_t tiles_per_wg;  /* tiles one workgroup runs per pass (2D: 1 to 4; 3D: 1) */
    int32_t tile_x, tile_y, tile_z;   /* nodes per tile along x, y, z (tile_z = 1 in 2D) */
    int32_t tiles;         /* tiles covering the lattice */
    int32_t workgroups;    /* workgroups per pass (a multiple of 8) */
    int32_t groups;        /* completion-counter groups of the cross-workgroup reduction */
    int64_t footprint;     /* device bytes of the solve (rn_footprint) */
} rn_plan_t;

/* Fill *out with the launch plan of `prob` under `opts` (NULL: defaults)
 * without touching a device. RN_EINVAL for an invalid shape or options (the
 * conductances themselves are not read). */
int rn_plan(const rn_problem *prob, const rn_opts *opts, rn_plan_t *out);

/* ------------------------------------------------------------------ launch shapes
 * The launch shape of each network's pass kernel (RN_PATH_* tile, tiles per
 * workgroup, 3D tile depth) comes from a process-wide table indexed by size
 * class (floor(log2 of the node count)), dimension and inner precision; an
 * entry the table does not set follows built-in rules (the defaults). The
 * paper's kernels ran on a fixed 256 x 64 launch grid (Sec. IV); here the
 * shapes are measured on the device. The table changes only through the
 * three calls below, so a network's shape, and with it its arithmetic, is the
 * same alone, in a batch and in the served stream; a network queued or
 * running keeps the shape it was given when it was submitted.
 */
#define RN_TUNE_QUICK 1   /* rn_autotune: only classes up to 2^18 (2D) / 2^17 (3D) nodes, small trials */

/*
 * Measure every candidate shape of every size class (2D: 2^12 .. 2^24 nodes,
 * the full tile with 1 to 4 tiles per workgroup or the small tile with 1 or 2; 3D: 2^15 .. 2^24 nodes,
 * tile depth 2 .. 32 planes) in both precisions on ctx's device: for each,
 * identical synthetic networks of the class, enough that a round moves about
 * 2^25 nodes (at most 256 copies; the objective is the throughput of large
 * batches), are solved together for 64 CG passes and the pass kernels'
 * device time per node and working pass is taken from the event timing of
 * rn_set_timing (the faster of two runs). With RN_TUNE_QUICK a round moves
 * about 2^22 nodes (at most 16 copies). The fastest shape of each class, or
 * the built-in one unless the fastest beats it by 3% or more, is
 * installed process-wide and, if cache_path is not NULL, written to that file
 * (text, one line per class; rn_tune_load reads it back). Takes seconds and
 * device memory from the context's budget. Do not solve on other contexts
 * while it runs (the trials install their candidates process-wide). flags: 0
 * or RN_TUNE_QUICK. RN_EINVAL (bad flags, the server is running, the cache
 * file cannot be written), RN_ENOMEM, RN_EDEVICE.
 */
int rn_autotune(rn_ctx *ctx, const char *cache_path, int32_t flags);

/* Install the table written by rn_autotune to `path` (host only). RN_EINVAL
 * when the file cannot be read or a line is malformed (nothing installed). */
int rn_tune_load(const char *path);

/* Back to the built-in rules for every class. */
int rn_tune_reset(void);

/* Scheduler occupancy of a context (for monitoring and admission tests). */
typedef struct {
    int64_t waiting;      /* queued, waiting for memory or a control slot */
    int64_t preparing;    /* setup (upload, mask) in flight */
    int64_t active;       /* in the pass launches */
    int64_t finishing;    /* outputs being copied back */
    int64_t bytes_in_use; /* device bytes held by networks */
    int64_t budget;       /* the context's HBM budget */
    int64_t launches;     /* pass kernel launches issued so far */
    int64_t peak_active;  /* most networks that have shared one pass launch */
    /* With rn_set_timing on: device time of the pass kernel launches, by the
     * path that ran them (RN_PATH_*) and their inner precision (RN_FP64,
     * RN_MIXED), measured with HIP events recorded on the launch stream
     * between consecutive launches, and the number of launches timed. */
    double pass_device_s[3][2];
    int64_t pass_timed_launches[3][2];
} rn_stats_t;

int rn_stats(rn_ctx *ctx, rn_stats_t *out);

/*
 * Turn the per-launch timing of rn_stats on (enable = 1) or off (0). While it
 * is on, one HIP event is recorded on the launch stream after every pass
 * launch (and one before each chunk of launches); the elapsed time between
 * consecutive events is added to pass_device_s of the launch's path and
 * precision when the chunk's control blocks are read back. Turning it on
 * clears the accumulated times. Off by default; ignored while pass rounds
 * are replayed from a hipGraph (RN_GRAPHS=1). Thread-safe like rn_stats.
 */
int rn_set_timing(rn_ctx *ctx, int enable);

/* ------------------------------------------------------------------ inputs on the GPU
 * Correlated conductance fields (Sec. II, Eqs. 1-2), the input generation the
 * paper distributes over MPI processes (Sec. II, Table I), on one GPU. The
 * random numbers are the caller's: white normals for the field, uniforms for
 * the dilution. These calls are independent of the solve. Arrays use the
 * lattice layout above and live in the memory space named by `mem`
 * (RN_MEM_HOST or RN_MEM_DEVICE). Both calls return RN_EINVAL while the
 * request server runs. The FFT plans are hipFFT's; their work areas are
 * outside the context's budget.
 */

/*
 * Node field by Fourier filtering on the periodic node grid (dim 2: nz = 1):
 * the white normals `noise` (one per node) are transformed, each mode is
 * multiplied by (sum_k beta[k] f_k^2)^(-(H + dim/2) / 2), with f_k the mode's
 * frequency along direction k in cycles per node (f = j/n for j <= (n-1)/2,
 * else (j - n)/n), the k = 0 mode is removed, and the inverse transform is
 * standardised to mean 0 and population standard deviation 1 (all zeros if it
 * is constant). For dim = 2 the exponent is Eq. 1's H + 1; beta (NULL: all 1,
 * else beta[k] > 0 for k < dim) gives Eq. 2's anisotropic spectrum.
 * field_out may equal noise. RN_EINVAL on a bad shape (as rn_problem), a
 * non-finite H or a bad beta; RN_ENOMEM / RN_EDEVICE otherwise.
 */
int rn_fbm_field(rn_ctx *ctx, int32_t dim, int64_t nx, int64_t ny, int64_t nz, double H, const double *beta,
                 const double *noise, double *field_out, int32_t mem);

/*
 * Bond conductances from a node field: g_out[k][i] = exp(sigma (phi_i +
 * phi_j) / 2) for the bond from node i to j = i + e_k, j taken on the
 * periodic grid. The last-plane entries along k are kept when `periodic` is 1
 * (the wrap bonds of RN_PERIODIC) and set to 0 when it is 0. With u non-NULL,
 * u[k] (k < dim, one uniform per entry) dilutes the bonds: an entry is kept
 * where u[k][i] < occupancy and set to 0 elsewhere. RN_EINVAL on a bad shape,
 * a non-finite sigma or occupancy, periodic not 0/1, or a NULL array.
 */
int rn_fbm_bonds(rn_ctx *ctx, int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *field, double sigma,
                 int32_t periodic, const double *const u[3], double occupancy, double *const g_out[3], int32_t mem);

#ifdef __cplusplus
}
#endif

#endif /* RN_H */
