// rn_runtime.hpp -- host runtime of librn: device memory pool, per-network
// solve state and the multi-network iteration engine shared by rn_solve,
// rn_solve_batch and the request server.
#pragma once

#include "../../include/rn.h"
#include "rn_device.hpp"

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace rn {

// ------------------------------------------------------------------ memory pool
// Device memory in slabs (hipMalloc'd on demand, released with the context or
// when a request needs their budget), carved first-fit. The sum of slab sizes
// never exceeds the context budget.
class Pool {
public:
    explicit Pool(size_t budget = 0) : budget_(budget) {}
    ~Pool();
    void set_budget(size_t b) { budget_ = b; }
    size_t budget() const { return budget_; }
    size_t in_use() const { return in_use_; }
    // nullptr with *err = hipSuccess when the request does not fit the budget now
    void *alloc(size_t bytes, hipError_t *err);
    void free(void *p);
    void release_all();
    // hipFree every slab that nothing is carved from
    void trim();
    size_t reserved() const { return reserved_; }

private:
    struct Slab {
        char *base;
        size_t size;
        std::map<size_t, size_t> free_;   // offset -> length
        std::map<size_t, size_t> used_;   // offset -> length
    };
    std::vector<Slab> slabs_;
    size_t budget_ = 0, reserved_ = 0, in_use_ = 0;
};

// ------------------------------------------------------------------ layout
struct Layout {
    int64_t n = 0;
    int dim = 2, s = 8;
    bool copy_g = false;
    int grid = 8, groups = 1, tpw = 1, ntx = 1, nty = 1, ntz = 1, ntiles = 1, tile_z = 16;
    int shape = 0;   // 2D tile: 0 full, 1 small
    int kpend = 2;   // CG steps the FP64 field may fall behind (4 with FP32 vectors, 2 with FP64)
    size_t off_g64 = 0, off_P = 0, off_mask = 0, off_gT = 0, off_vec = 0,
           off_part = 0, off_tk = 0, off_cnt = 0, total = 0;
};
Layout make_layout(const rn_problem *p, const rn_opts *o);

// ------------------------------------------------------------------ launch-shape table
// The launch shape of a network's pass kernel by size class (floor(log2 of
// its node count)), dimension and inner precision: the 2D tile (0 full, 1
// small) and tiles per workgroup, the 3D tile depth. It is process-wide and
// changes only when a table is installed (rn_autotune, rn_tune_load,
// rn_tune_reset), so a network's shape, hence its arithmetic, never depends on
// the other networks it runs with. An entry with shape < 0 (2D) or tile_z == 0
// (3D) follows the built-in rules of make_layout.
struct ShapeChoice {
    int shape = -1, tpw = 0, tile_z = 0;
    double ns_per_node = 0.0;   // measured device time per node and pass (0: not measured)
};
constexpr int kShapeClasses = 32;
struct ShapeTable {
    ShapeChoice c[2][2][kShapeClasses];   // [dim - 2][inner FP32 ? 1 : 0][class]
};
int shape_class(int64_t n);
ShapeChoice shape_choice(int dim, int s, int64_t n);
ShapeTable shape_table_get();
void shape_table_install(const ShapeTable &t);
bool shape_choice_valid(int dim, const ShapeChoice &c);
int shape_table_parse(const std::string &text, ShapeTable *out);   // RN_OK or RN_EINVAL
std::string shape_table_format(const ShapeTable &t);

// ------------------------------------------------------------------ one network
enum NetPhase { NET_NEW, NET_PREPARING, NET_ACTIVE, NET_FINISHING, NET_DONE };

struct Net {
    rn_problem prob{};
    rn_opts opts{};
    Layout L;
    char *base = nullptr;           // device arena (pool)
    const double *gd[3] = {nullptr, nullptr, nullptr};
    int slot = -1;                  // control block / descriptor slot in the engine
    int kind = 0;                   // tile family x FP32/FP64, see Engine::kind_of
    NetPhase phase = NET_NEW;
    int64_t n_live = 0;
    int64_t na = 0;                 // extent along the flow axis
    hipEvent_t ev = nullptr;        // end of the last enqueued phase (setup or outputs)
    hipEvent_t ev_a = nullptr, ev_b = nullptr;   // setup start / end (timing)
    hipEvent_t ev_c = nullptr, ev_d = nullptr;   // iteration loop start / end (timing)
    int64_t round0 = 0;             // engine pass round at activation
    rn_result res{};
    int status = RN_OK;
    double t_start = 0.0;           // host clock at submission
    uint64_t ticket = 0;
    int bypassed = 0;               // admissions of later requests while this one waited at the head
    double prev_est = -1.0;
    int64_t prev_iters = 0;
    int64_t first_chunk = 0;        // first chunk whose status mirror covers this network
    // host copies (server path: the caller's buffers stay valid until completion)
};

// ------------------------------------------------------------------ engine
class Engine {
public:
    static constexpr int kSlots = 4096;
    // kinds: 0 2D full tiles, 1 3D, 2 and 3 the same in FP64, 4 2D small tiles, 5 the same in FP64
    static constexpr int kKinds = 6;

    int init(hipStream_t st, std::string *err);
    void destroy();
    bool full() const { return free_slots_.empty(); }
    // enqueue upload, validation, connectivity and counters of a network
    int prepare(Net *net, hipStream_t st, std::string *err);
    // the prepared network's counters are on the host: activate it, or finish it
    // at once (no live node, invalid values). Returns RN_OK or an error status.
    int after_prepare(Net *net, hipStream_t st, std::string *err);
    // launch `rounds` pass rounds of every active network, then queue a read
    // of every control block into a host mirror
    int launch_chunk(int rounds, hipStream_t st, std::string *err);
    // wait for the oldest outstanding mirror (all of them when `all`) while two
    // are outstanding; finalize the networks it shows finished (outputs
    // enqueued, ev recorded) and append them to *finished
    int collect(std::vector<Net *> *finished, bool all, hipStream_t st, std::string *err);
    int active_count() const { return (int)active_.size(); }
    int outstanding() const { return (int)outstanding_.size(); }
    int next_chunk() const { return chunk_; }
    int64_t launches() const { return launches_; }
    int64_t chunk_seq() const { return chunk_seq_; }
    int peak_active() const { return peak_active_; }
    // forget every network (after a device error): slots, tables, mirrors
    void abort_all();
    // stream for setup and output copies (nullptr: everything on the compute stream)
    void set_side(hipStream_t s) { side_ = s; }
    // per-launch device timing of the pass kernels (events between launches)
    void set_timing(bool on);
    double kind_seconds(int k) const { return kind_s_[k]; }
    int64_t kind_launches(int k) const { return kind_n_[k]; }
    // kind -> (RN_PATH_*, precision RN_FP64 / RN_MIXED)
    static int kind_path(int k) { return (k == 1 || k == 3) ? RN_PATH_3D : (k >= 4 ? RN_PATH_2D_SMALL : RN_PATH_2D_FULL); }
    static int kind_precision(int k) { return kind_fp64(k) ? RN_FP64 : RN_MIXED; }

private:
    int kind_of(const Net *n) const
    {
        const int fp64 = n->L.s == 8 ? 1 : 0;
        if (n->prob.dim == 3) return 1 + 2 * fp64;
        return n->L.shape ? 4 + fp64 : 2 * fp64;
    }
    static bool kind_fp64(int k) { return k == 2 || k == 3 || k == 5; }
    static int kind_dim(int k) { return (k == 1 || k == 3) ? 3 : (k >= 4 ? -2 : 2); }   // launch_pass's dim
    int rebuild(hipStream_t st, std::string *err);
    int finalize(Net *net, const Scalars &h, hipStream_t st, std::string *err);

    Scalars *d_scal_ = nullptr, *h_scal_[2] = {nullptr, nullptr}, *h_init_ = nullptr;
    PassArgs<float> *d_tabf_ = nullptr, *h_tabf_ = nullptr;
    PassArgs<double> *d_tabd_ = nullptr, *h_tabd_ = nullptr;
    unsigned long long *h_cnt_ = nullptr;   // [kSlots][4] pinned
    uint2 *d_blk_[kKinds] = {};
    uint2 *h_blk_[kKinds] = {};
    int blk_cap_[kKinds] = {};
    int nblk_[kKinds] = {};
    int single_[kKinds] = {};              // slot of the only network of a kind, or -1
    hipEvent_t ev_chunk_[2] = {nullptr, nullptr};
    std::deque<int> outstanding_;           // mirrors with a queued status read, oldest first
    int next_mirror_ = 0, half_ = 0;
    int mirror_hi_[2] = {0, 0};             // slots copied into each mirror
    int64_t mirror_seq_[2] = {0, 0};        // chunk number each mirror follows
    int mirror_rounds_[2] = {0, 0};
    int64_t chunk_seq_ = 0;
    std::vector<int> free_slots_;
    std::vector<Net *> active_;
    Net *by_slot_[kSlots] = {};
    bool dirty_ = true;
    int64_t rounds_ = 0;                    // pass rounds issued (parity of the next round)
    int64_t launches_ = 0;
    int chunk_ = 16;
    int peak_active_ = 0;                   // most networks that shared one launch
    // hipGraph of kGraphRounds pass rounds for the current block tables,
    // replayed for the bulk of each chunk (the round count is even, so the
    // parities baked into the graph stay valid from replay to replay)
    static constexpr int kGraphRounds = 8;
    bool use_graph_ = false;
    hipGraphExec_t gexec_ = nullptr;
    int graph_parity_ = -1;
    int launch_rounds(int rounds, hipStream_t st, std::string *err);
    int launch_persistent(int rounds, hipStream_t st, std::string *err);
    int capture(hipStream_t st, std::string *err);
    // persistent launches (RN_PERSIST=1 or 2): `rounds` pass rounds of a kind in one launch
    bool persist_ = false;
    int persist_mode_ = 0;                   // RN_PERSIST: 0 off, 1 persistent over all XCDs, 2 one XCD per network
    int kind_coh_[kKinds] = {};              // per kind, this chunk: 0 one launch per round, 1 or 2 persistent
    static constexpr int kXcdMaxGrid = 256;  // largest network (workgroups per pass) placed on one XCD
    static constexpr int kQueueWords = 8 * 32;   // per kind: 8 item counters, 256 bytes apart
    int *d_xoff_ = nullptr, *h_xoff_ = nullptr;  // per kind, 9 table offsets (16 ints), host staging x2
    hipStream_t side_ = nullptr;
    unsigned *d_err_ = nullptr, *h_err_ = nullptr;   // a bounded wait gave up (device word, pinned mirror)
    unsigned long long *d_queue_ = nullptr;          // item counters of the persistent launches, kQueueWords per kind
    // timing: events of the chunk behind mirror b, tev_[b][0] before its first
    // launch and tev_[b][i + 1] after launch i, whose kind is tkind_[b][i]
    bool timing_ = false, recording_ = false;
    std::vector<hipEvent_t> tev_[2];
    std::vector<int> tkind_[2];
    int trec_ = 0, tmirror_ = 0;
    double kind_s_[kKinds] = {};
    int64_t kind_n_[kKinds] = {};
    int record_timing(int kind, hipStream_t st, std::string *err);
};

}  // namespace rn

// ------------------------------------------------------------------ context
struct rn_server;

struct rn_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t own = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;     // the context's second stream: setup and output copies of networks
                                    // (used while the context runs on its own stream)
    std::string err;
    rn::Pool pool;
    rn::Engine engine;
    bool engine_ok = false;
    hipEvent_t ev_t[4] = {nullptr, nullptr, nullptr, nullptr};
    std::mutex call_mu;             // serialises the synchronous entry points with the server
    std::atomic<int> callers{0};    // threads waiting for call_mu (the server steps aside for them)
    rn_server *server = nullptr;
    void *fbm_plans = nullptr;      // FFT plans of the last generated grid (rn_fbm.hip)
    size_t active_cap = 0;          // RN_ACTIVE_BYTES: cap on the device bytes of networks in flight (0: none)
    unsigned long long *h_small = nullptr;   // pinned, 32 words: counters read back by rn_build_mask_noalloc,
                                             // level offsets of rn_build_backbone
};

namespace rn {
void fbm_release(rn_ctx *ctx);   // frees ctx->fbm_plans (rn_fbm.hip)
int check_shape(const rn_problem *p);
int check_opts(const rn_opts *o);
bool host_values_ok(const rn_problem *p);
int wrap_bits(const rn_problem *p);   // bit k: direction k is periodic
Lat make_lat(const rn_problem *p);
double cross_section(const rn_problem *p);
double now_s();
}  // namespace rn
