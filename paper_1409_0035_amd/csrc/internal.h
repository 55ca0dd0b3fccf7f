// Internal declarations shared by the HIP kernel files and the runtime.
// Not part of the C ABI (see include/ccgpu.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace ccg {

// ---------------------------------------------------------------- errors
struct HipError {
    hipError_t err;
    std::string where;
};

#define CCG_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) throw ::ccg::HipError{e_, std::string(#call) + " @ " + \
                                                              __FILE__ + ":" + std::to_string(__LINE__)}; \
    } while (0)

// Device-side status words, one block per job.  Kernels only ever set flags
// (plain stores of 1) or add to counters, so the order of updates is
// irrelevant.
struct DevFlags {
    int32_t disconnected;   // a node never reached by some sample
    int32_t overflow;       // a distance or numerator out of range
    int32_t bad_sample;     // duplicate / out-of-range sample
    int32_t timeout;        // a bounded wait or a time limit expired
    int64_t maxd;           // largest distance seen (weighted traversal)
    int64_t reserved[3];
};

// Per-level counters written by one traversal launch and read by the host.
// Kernels add into kCounterSlots copies (one cache line each, slot chosen by
// block) so that thousands of blocks do not serialise on one address; the
// host sums the copies.
struct alignas(128) LevelCounters {
    int32_t n_out;          // groups (or nodes) still in play after this level
    int32_t n_new;          // nodes that received new bits / distances this level
    int32_t n_out_q;        // nodes appended to the next frontier list
    int32_t hub_open;       // batched BFS: hub nodes not yet full after this level
    int64_t arcs;           // adjacency entries scanned (pull) or pushed along (push)
    int64_t frontier_arcs;  // sum of the out-degrees of the next frontier
    int64_t matched;        // scanned arcs whose tail was on the previous level
    uint32_t ticket;        // batched BFS: blocks of this slot that have finished the merge launch
};
constexpr int kCounterSlots = 64;

inline void sum_counters(const LevelCounters* slots, int count, LevelCounters& out) {
    out = LevelCounters{};
    for (int i = 0; i < count; i++) {
        out.n_out += slots[i].n_out;
        out.n_new += slots[i].n_new;
        out.n_out_q += slots[i].n_out_q;
        out.arcs += slots[i].arcs;
        out.frontier_arcs += slots[i].frontier_arcs;
        out.matched += slots[i].matched;
    }
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int readlane32(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x |= __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ int32_t wave_sum32(int32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t y = __shfl_xor(x, off);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Append-to-list index for the lanes with pred set; works in divergent code
// (only active lanes take part).  One atomic per call per wave.
__device__ __forceinline__ int wave_append(int32_t* counter, bool pred) {
    uint64_t act = __ballot(1);
    uint64_t m = __ballot(pred);
    int leader = __ffsll((unsigned long long)act) - 1;
    int base = 0;
    if (lane_id() == leader && m) base = atomicAdd(counter, (int32_t)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + (int)__popcll(m & lanemask_lt()) : -1;
}

// ---------------------------------------------------------------- distances
template <typename DT> struct DistT;
template <> struct DistT<uint8_t> {
    static constexpr uint32_t never = 0xFFu;
    static constexpr int64_t max_level = 254;
};
template <> struct DistT<uint16_t> {
    static constexpr uint32_t never = 0xFFFFu;
    static constexpr int64_t max_level = 65534;
};
template <> struct DistT<uint32_t> {
    static constexpr uint32_t never = 0xFFFFFFFFu;
    static constexpr int64_t max_level = 0x7FFFFFFE;
};

// ---------------------------------------------------------------- graph
// Device copy of a graph in the library's internal node order: ids sorted by
// degree, largest first (the "graph builder" step of the upload).
struct DevGraph {
    int64_t n = 0;
    int64_t arcs = 0;
    bool directed = false;
    bool weighted = false;
    // out-arcs
    const uint32_t* rp = nullptr;
    const int32_t* col = nullptr;
    const int32_t* w = nullptr;
    // in-arcs (transpose); equal to the out-arcs for undirected graphs
    const uint32_t* rrp = nullptr;
    const int32_t* rcol = nullptr;
    const int32_t* rw = nullptr;
    // weighted graphs: each arc's (end, length) side by side, out-arcs and in-arcs
    const int2* cw = nullptr;
    const int2* rcw = nullptr;
    const int32_t* orig = nullptr;  // internal id -> caller's id
    const int32_t* inv = nullptr;   // caller's id -> internal id
    uint32_t delta = 1;             // delta-stepping bucket width (weighted graphs)
    // high-degree prefix [0, nh) scanned in chunks; chunk lists per pull direction
    int64_t nh = 0;
    const int32_t* hub_chunks_in = nullptr;   // over in-arcs (forward distances)
    int32_t n_hub_chunks_in = 0;
    const int32_t* hub_chunks_out = nullptr;  // over out-arcs (reverse distances)
    int32_t n_hub_chunks_out = 0;
    // graphs kept in the caller's order (borrowed device CSRs): the 64-node
    // groups that hold a high-degree node, flagged, instead of the prefix [0, nh)
    const uint8_t* ghub = nullptr;
};

// The adjacency one batched traversal uses: pull over rp/col (in-arcs), push
// over out_rp/out_col (out-arcs).
struct BfsView {
    int64_t n = 0;
    int64_t arcs = 0;
    const uint32_t* rp = nullptr;
    const int32_t* col = nullptr;
    const uint32_t* out_rp = nullptr;
    const int32_t* out_col = nullptr;
    int64_t nh = 0;
    const int32_t* hub_chunks = nullptr;  // (node, first arc, end arc) triples over rp/col
    int32_t n_hub_chunks = 0;
    const int32_t* push_chunks = nullptr;  // the same over out_rp/out_col
    int32_t n_push_chunks = 0;
    // Several graphs in one traversal (a batch): node ranges aligned to 64, so
    // hub nodes are whole groups flagged here instead of a prefix of the ids,
    // and every node starts with the bits of the other graphs' samples set
    // (preset[g*W..], for the first gvalid[g] nodes of group g; the rest of a
    // group are padding and start full).  All three null for one graph.
    const uint8_t* ghub = nullptr;
    const uint64_t* preset = nullptr;
    const int32_t* gvalid = nullptr;
    int32_t alpha = 4;  // a level pushes iff its frontier's out-arcs * alpha < what the last pull scanned
    int32_t level_blocks = 1024;    // merge launch grid cap
    int32_t scatter_blocks = 8192;  // scatter launch grid cap
};

// Traversal state the batched BFS level kernels read at entry and the last
// block of each merge launch updates, so that a batch of levels runs without
// the host.
struct BfsCtl {
    int32_t done;         // 1 once the traversal has ended (status says how)
    int32_t status;       // 0 every node full, 1 level capacity exhausted, 2 a node no sample reaches
    int32_t lmax;         // last level at which some node gained a bit
    int32_t pull;         // direction of the next level: 1 pull, 0 push
    int32_t levels;       // levels run
    int32_t pull_levels;  // of which pulls
    uint32_t ticket;      // blocks of the current merge launch that have finished
    int32_t hubs_full;    // every hub node was full after the last level: a pull has no hub work
    int32_t sparse;       // few nodes changed at the last level: pulls read only their masks
    int32_t pad;
    int64_t frontier_arcs;  // out-arcs of the nodes that changed at the last level
    int64_t pull_arcs;      // arcs the last pull scanned (what a pull would cost now)
    int64_t arcs;           // arcs scanned or pushed along, all levels
    int64_t hub_arcs;       // of which by the hub-chunk pull
    int64_t push_arcs;
    int64_t push_atomics;
    int64_t nodes;          // node slots of live groups visited
};

// Where the batched BFS records its per-level seen masks.
struct BfsLevels {
    uint64_t* snap = nullptr;     // [cap][n][W]: snap[L][v] = {i : d(c_i, v) <= L}
    int32_t cap = 0;              // levels the buffer holds
    int32_t* fill_level = nullptr;  // [ceil(n/64)]: last level each 64-node group wrote
    int32_t* hist = nullptr;      // optional [kHistSlotsBatched][k][hlen] per-sample level histogram
    int64_t hlen = 0;
    int32_t* lmax = nullptr;      // host: largest level with new bits (max over calls)
    int32_t hint = 0;             // levels the host enqueues before its first check (0 = a few)
    // optional, for a traversal of all of the job's samples (src_base 0, kg = k): the job's setup
    // folded into the traversal's first two launches instead of launches of its own
    DevFlags* zero_flags = nullptr;  // zeroed
    int32_t* sidx_fill = nullptr;    // [n]: -1, then each sample's index
    bool zero_hist = false;          // hist ([kHistSlotsBatched][k][hlen]) zeroed
    // optional, same condition: the samples are read by the first launch from pinned host memory
    // (device-visible addresses) and stored to samples_dev there, so nothing is copied before it
    const int32_t* stage_ids = nullptr;     // [k] internal ids, read with system-scope loads
    const int32_t* stage_caller = nullptr;  // [k] the same samples as the caller numbers them
    int32_t* samples_out = nullptr;         // device [k]: receives stage_caller (optional)
    int32_t enqueue_only = 0;     // > 0: enqueue exactly this many levels and return at once (stream capture)
};

// ---------------------------------------------------------------- traversal API
// Traversal statistics accumulated by the drivers.
struct TravStats {
    int64_t levels = 0;
    int64_t arcs_scanned = 0;
    int64_t nodes_visited = 0;
    int64_t launches = 0;
    int64_t maxd = 0;        // largest distance written
    int64_t arcs_matched = 0;
    double kernel_ms = 0;    // summed duration of the per-level traversal kernels
    int64_t kernel_launches = 0;
    int64_t pull_levels = 0;
    int64_t push_arcs = 0;
    double scatter_ms = 0;        // summed duration of the scatter (push / hub pull) launches
    int64_t scatter_launches = 0;
    int64_t scatter_arcs = 0;     // arcs they scanned (hub pulls) or pushed along (pushes)
    double pull_scatter_ms = 0;   // of scatter_ms, the levels that pulled
    int64_t hub_arcs = 0;         // arcs the hub pulls scanned
    int64_t push_atomics = 0;  // atomic ORs issued by push levels
    int32_t bfs_levels = 0;    // most levels one batched traversal ran
};

// Event pair for timing one kernel launch on a stream.
struct KernelTimer {
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer() {
        CCG_HIP(hipEventCreate(&a));
        CCG_HIP(hipEventCreate(&b));
    }
    ~KernelTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) { CCG_HIP(hipEventRecord(a, s)); }
    void stop(hipStream_t s) { CCG_HIP(hipEventRecord(b, s)); }
    // call after the stream has been synchronised
    double ms() const {
        float t = 0.f;
        CCG_HIP(hipEventElapsedTime(&t, a, b));
        return t;
    }
};

// Events created on first use and reused, for timing single launches.
struct EventPool {
    std::vector<hipEvent_t> ev;
    hipEvent_t at(size_t i) {
        while (ev.size() <= i) {
            hipEvent_t e = nullptr;
            CCG_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        return ev[i];
    }
    EventPool() = default;
    EventPool(const EventPool&) = delete;
    EventPool& operator=(const EventPool&) = delete;
    ~EventPool() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

enum class DistKind { U8 = 1, U16 = 2, U32 = 4 };

constexpr int kHistSlotsBatched = 32;  // spread copies of the per-level histogram counters


// Batched bit-parallel BFS over one group of kg <= 256 samples (internal
// ids samples_dev[src_base .. src_base+kg), written by the traversal itself
// when out.stage_ids is set), recording per-level seen masks in `out`; with out.hist it also counts hist[slot][src_base+i][L] over
// non-sampled nodes (sidx[v] < 0).
// Returns 0 = done, 1 = snapshot capacity too small (retry with more levels),
// 2 = some node is unreachable from some sample.
int bfs_batched(hipStream_t st, const BfsView& gv, int32_t* samples_dev, int32_t kg, int32_t src_base,
                int32_t k, const BfsLevels& out, const int32_t* sidx, void* scratch, size_t scratch_size,
                LevelCounters* cnt_dev, TravStats* stats, EventPool* evp);
size_t bfs_batched_scratch(int64_t n, int32_t kg, int64_t nh);
// The control block inside a batched traversal's scratch.
BfsCtl* bfs_batched_ctl(void* scratch, int64_t n, int32_t kg);

// Distances of one sample group from its level masks into the node-major
// matrix D (columns src_base .. src_base+kg), in the given width.
void materialize_distances(hipStream_t st, const uint64_t* snap, size_t plane, int32_t lmax, const int32_t* fill_level,
                           int64_t n, int32_t kg, int32_t src_base, int32_t k, void* D, DistKind dk, DevFlags* flags,
                           bool add = false);

// Plain single-source BFS for every sample, source-major output Dt[k][n].
bool bfs_plain(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
               const int32_t* in_col, int64_t n, int64_t arcs, const int32_t* samples_host, int32_t k,
               void* Dt, DistKind dk, void* scratch, size_t scratch_size, DevFlags* flags,
               LevelCounters* cnt_dev, LevelCounters* cnt_host, TravStats* stats);
size_t bfs_plain_scratch(int64_t n, int64_t arcs, int32_t k);

// Transpose source-major Dt[k][n] into node-major D[n][k].
void transpose_dist(hipStream_t st, const void* Dt, void* D, int64_t n, int32_t k, DistKind dk);

// Weighted distances (positive integer lengths) from samples_dev[0..kg)
// (internal ids) into source-major Dt[j][v] by near/far delta-stepping.
// Returns 0 = done, 2 = some node unreached, 4 = overflow.
// Launch shape of the delta-stepping rounds.
struct WeightedShape {
    uint32_t delta = 1;         // bucket width
    int32_t round_blocks = 1024;
    int32_t local_passes = 64;  // block-local relaxation passes per round
};
int sssp_weighted(hipStream_t st, const uint32_t* rp, const int32_t* col, const int32_t* w, int64_t n,
                  const int32_t* samples_dev, int32_t kg, uint32_t* Dt, const WeightedShape& shape, void* scratch,
                  size_t scratch_size, int64_t* maxd, TravStats* stats);
size_t sssp_weighted_scratch(int64_t n, int32_t kg);
// The batched path: every sample's search in its own workgroup of one launch.
int sssp_weighted_batched(hipStream_t st, const uint32_t* rp, const int2* cw, int64_t n, const int32_t* samples_dev,
                          int32_t kg, uint32_t* Dt, uint32_t delta, void* scratch, size_t scratch_size, int64_t* maxd,
                          TravStats* stats);
size_t sssp_wsearch_scratch(int64_t n, int32_t kg);
// The same launches without host reads (stream capture): status and largest
// distance folded into flags and *maxd_out on the device
void sssp_weighted_batched_enqueue(hipStream_t st, const uint32_t* rp, const int2* cw, int64_t n,
                                   const int32_t* samples_dev, int32_t kg, uint32_t* Dt, uint32_t delta,
                                   void* scratch, size_t scratch_size, DevFlags* flags, uint32_t* maxd_out);
// (end, length) pairs of a weighted adjacency, for the batched searches
void zip_arcs(hipStream_t st, const int32_t* col, const int32_t* w, int64_t arcs, int2* out);

// ---------------------------------------------------------------- epilogue API
struct EpilogueArgs {
    int64_t n = 0;
    int32_t k = 0;
    DistKind dk = DistKind::U8;
    const void* D = nullptr;     // node-major distances, internal node order
    const void* Dr = nullptr;    // reverse-direction distances (round trip) or nullptr
    const int32_t* samples = nullptr;  // device, internal ids
    const int32_t* sidx = nullptr;     // device, internal id -> sample index or -1
    const int32_t* orig = nullptr;     // device, internal id -> caller's id
    // device, caller's id -> internal id: when set, the row estimate walks the
    // nodes in the caller's order (v = inv[o]) and stores the Sec. 2 outputs at
    // o, consecutive for a wave (instead of seven scattered stores per node)
    const int32_t* inv = nullptr;
    int64_t maxd = 0;            // upper bound on every (combined) distance
    int64_t eps_num = 1, eps_den = 1;
    // histogram already counted by the traversal: hist[slot][i][d], rows of hist_len
    bool hist_done = false;
    int32_t* hist = nullptr;
    int32_t hist_slots = 0;
    int64_t hist_len = 0;
    // outputs (device, at the caller's node ids; may be null)
    double* S_hyb = nullptr;
    double* S_samp = nullptr;
    int64_t* S_piv = nullptr;
    int64_t* S_pub = nullptr;
    int32_t* pivot = nullptr;
    int32_t* delta = nullptr;
    int64_t* sampsum = nullptr;
    int64_t* src_sum = nullptr;  // required (workspace if caller does not want it)
    int32_t* dmat = nullptr;     // required (workspace if caller does not want it)
    int32_t* Dout = nullptr;     // optional int32 copy of D (combined), caller's node order
    double* S_err = nullptr;     // Sec. 4 outputs (optional)
    double* S_ad = nullptr;
    double* S_ad_err = nullptr;
    double* S_sweep = nullptr;   // Algorithm 2 / Sec. 4.2 outputs (optional)
    double* S_sweep_err = nullptr;
};
// bytes of the error-estimate pass's tables (Sec. 4, Algorithm 2): each
// sample's sorted row of the sample distance matrix and the nodes grouped by
// pivot; added to an epilogue's scratch when any of its outputs is wanted
size_t sweep_scratch_bytes(int64_t n, int32_t k);
size_t epilogue_scratch(int64_t n, int32_t k, int64_t maxd, bool hist_done, bool err = false);
void run_epilogue(hipStream_t st, const EpilogueArgs& a, void* scratch, size_t scratch_size, DevFlags* flags);
// Round-trip distances of one group of k (a multiple of 64, at most 256)
// samples as one-byte rows D[v][i] = d(c_i, v) + d(v, c_i), from the forward
// and the reverse search's level masks and fill levels in one pass (each
// direction's largest distance given; their sum must be at most 254)
void materialize_round_trip(hipStream_t st, const uint64_t* snap_f, const int32_t* fill_f, int32_t lmax_f,
                            const uint64_t* snap_r, const int32_t* fill_r, int32_t lmax_r, int64_t n, int32_t k,
                            void* D, DevFlags* flags);
// The staged 64-byte node records written out in the caller's order
void put_outputs(hipStream_t st, int64_t n, const int32_t* inv, const void* stage, double* S_hyb, double* S_samp,
                 int64_t* S_piv, int64_t* S_pub, int32_t* pivot, int32_t* delta, int64_t* sampsum);
void compute_sidx(hipStream_t st, const int32_t* samples, int32_t k, int32_t* sidx, int64_t n);

// Tail tables and exact sample sums from a histogram with `nslots` copies.
void run_suffix(hipStream_t st, const int32_t* hist, int32_t nslots, int32_t k, int32_t hist_rows, int64_t hlen,
                int64_t maxd,
                const int32_t* dmat, int32_t* Tcnt, int64_t* Tsum, int64_t* src_sum, int64_t* chunk_scratch);
size_t suffix_chunk_scratch(int32_t k, int64_t maxd);

// Epilogue over the level masks of one sample group (k <= 256, undirected).
struct BitsEpilogueArgs {
    int64_t n = 0;
    int32_t k = 0;
    const uint64_t* snap = nullptr;
    size_t plane = 0;            // n * W words per level
    int32_t lmax = 0;
    const int32_t* fill_level = nullptr;
    const int32_t* samples = nullptr;  // device, internal ids
    const int32_t* sidx = nullptr;
    const int32_t* orig = nullptr;
    // caller's id -> internal id: the per-node outputs then go through a
    // staging area in internal order and are written out in the caller's
    // order, coalesced (null: each written in place through orig)
    const int32_t* inv = nullptr;
    const int32_t* hist = nullptr;
    int32_t hist_slots = 0;
    int64_t hist_len = 0;
    int64_t eps_num = 1, eps_den = 1;
    double* S_hyb = nullptr;
    double* S_samp = nullptr;
    int64_t* S_piv = nullptr;
    int64_t* S_pub = nullptr;
    int32_t* pivot = nullptr;
    int32_t* delta = nullptr;
    int64_t* sampsum = nullptr;
    int64_t* src_sum = nullptr;  // required
    int32_t* dmat = nullptr;     // required
    int32_t* Dout = nullptr;     // optional int32 distances, caller's node order
    double* S_err = nullptr;     // Sec. 4 outputs (optional)
    double* S_ad = nullptr;
    double* S_ad_err = nullptr;
    double* S_sweep = nullptr;   // Algorithm 2 / Sec. 4.2 outputs (optional)
    double* S_sweep_err = nullptr;
    // this graph's part of a batch's shared rows (defaults: the whole rows)
    int64_t node_off = 0;   // first row of this graph's nodes
    int32_t word_off = 0;   // first word of its samples in a row
    int32_t row_words = 0;  // words per row (0: the graph's own W)
    int32_t bit_base = 0;   // its first sample's index in sidx and in the histogram rows
    int32_t hist_rows = 0;  // histogram rows per slot (0: k)
};
// stage_rows: n when the per-node outputs are staged (inv set and some requested)
size_t bits_epilogue_scratch(int32_t k, int32_t lmax, int64_t err_rows = 0, bool err = false, int64_t stage_rows = 0);

// The eps values the experiments (Sec. 8) choose from per node for the
// adaptive hybrid estimate: 0.001, 0.025, 0.05, 0.1, 0.2, 0.5, 0.99.
constexpr int32_t kAdaptiveEps = 7;
constexpr int64_t kAdaptiveEpsNum[kAdaptiveEps] = {1, 1, 1, 1, 1, 1, 99};
constexpr int64_t kAdaptiveEpsDen[kAdaptiveEps] = {1000, 40, 20, 10, 5, 2, 100};

// Inputs of the error-estimate pass (Sec. 4) and the threshold sweep
// (Algorithm 2) over distance rows.
struct ErrArgs {
    const void* D = nullptr;    // node-major rows, dk bytes per entry
    const void* Dr = nullptr;   // reverse rows (round trip) or null
    DistKind dk = DistKind::U8;
    int64_t n = 0;
    int32_t k = 0;
    const int32_t* sidx = nullptr;  // per row: sample index + bit_base, or -1
    int32_t bit_base = 0;
    const int32_t* orig = nullptr;
    const void* dmat_c = nullptr;   // k x k sample distances, mt_bytes each
    int mt_bytes = 1;
    const int32_t* Tcnt = nullptr;
    const int64_t* Tsum = nullptr;
    int64_t tlen = 0;
    const int64_t* src_sum = nullptr;
    int64_t eps_num = 1, eps_den = 1;
    double* S_err = nullptr;
    double* S_ad = nullptr;
    double* S_ad_err = nullptr;
    double* S_sweep = nullptr;       // threshold sweep (Algorithm 2)
    double* S_sweep_err = nullptr;
    void* sweep_scratch = nullptr;   // sweep_scratch_bytes(n, k): the pass's tables
};
void run_errest(hipStream_t st, const ErrArgs& a, DevFlags* flags);
void run_bits_epilogue(hipStream_t st, const BitsEpilogueArgs& a, void* scratch, size_t scratch_size, DevFlags* flags);

void fill_u32(hipStream_t st, void* p, uint32_t value, size_t count);

// Node-weighted hybrid estimate (Sec. 5, Algorithm 3) from int32 distance
// rows at the caller's ids.
struct BetaArgs {
    int64_t n = 0;
    int32_t k = 0;
    const int32_t* D = nullptr;        // [n][k] d(c_i, v)
    const int32_t* dmat = nullptr;     // [k][k] d(c_i, c_j)
    const int32_t* sidx = nullptr;     // [n] sample index or -1
    const int32_t* samples = nullptr;  // [k] caller ids
    const uint32_t* beta = nullptr;    // [n] node weights
    const uint8_t* light = nullptr;    // [k] 1: adjusted weight tau
    int64_t R = 0;                     // tau = R / m
    int32_t m = 1;
    int64_t eps_num = 1, eps_den = 1;
    double* S = nullptr;
    double* var = nullptr;
    double* err = nullptr;             // Sec. 4.1's error estimate with beta masses (optional)
    int64_t maxd = -1;                 // an upper bound on the distances in D, or -1: found by a pass over D
    void* small_scratch = nullptr;     // 256 bytes
    std::function<void*(size_t)> get_scratch;  // device buffer of at least the given size
};
void run_beta_epilogue(hipStream_t st, const BetaArgs& a, DevFlags* flags);

// Outbound / inbound reachability sampling (Sec. 6.2, Algorithm 4).
constexpr int kReachWords = 16;  // up to 1024 sources of consecutive ranks per batch
struct ReachArgs {
    int64_t n = 0;
    int64_t arcs = 0;  // propagation arcs (rp[n])
    int32_t k = 0;
    const uint32_t* rp = nullptr;  // propagation arcs: outbound the in-arcs, inbound the out-arcs
    const int32_t* col = nullptr;
    const int32_t* order = nullptr;  // host: internal ids in rank order (a permutation)
    const int32_t* order_dev = nullptr;  // or device: the nsrc sources in rank order
    const int32_t* orig = nullptr;   // device: internal id -> caller's id
    // device outputs at the caller's ids (each may be null)
    int32_t* count = nullptr;
    int64_t* distsum = nullptr;
    int64_t* T = nullptr;
    double* B = nullptr;
    double* R = nullptr;
    int32_t push_blocks = 512;
    int32_t merge_blocks = 128;
    int32_t account_blocks = 64;
    // node-weighted sampling (Algorithm 5): order lists only the nsrc nodes of
    // positive weight; beta and U (priority-rank numerators) per internal id, on
    // the device; outputs count, kth (the k-th member), S_w and R
    int64_t nsrc = 0;
    const uint32_t* beta = nullptr;
    const uint64_t* U = nullptr;
    int32_t* kth = nullptr;
    double* S_w = nullptr;
    // graphs with arc lengths: the propagation arcs as (end, length) pairs,
    // the delta-stepping bucket width, and the sources searched per batch
    // (one workgroup each); cw set selects run_reach_lengths
    const int2* cw = nullptr;
    uint32_t delta = 1;
    int32_t len_sources = 0;
};
struct ReachStats {
    int64_t cycles = 0;   // push/merge/account/init cycles enqueued
    int64_t batches = 0;
    int64_t levels = 0;   // BFS levels (arc lengths: delta-stepping phases) run over all batches
    bool overflow = false;  // some level above 65535 (arc lengths: a distance or sum out of range)
    bool timeout = false;   // arc lengths: a search ran past its time limit
    int64_t relaxed = 0;    // arc lengths: arcs relaxed by all searches
};
size_t reach_scratch_bytes(int64_t n, int64_t arcs, int32_t k_weighted = 0);
// Sources per batch and scratch of the arc-length searches (24 bytes per node
// and source, plus per-node state)
size_t reach_len_scratch_bytes(int64_t n, int32_t sources, int32_t k_weighted);
// Algorithm 5's priority ranks: beta and U at internal ids, and the m nodes of
// positive weight (internal ids) by increasing rank U / (2^53 beta)
size_t priority_scratch_bytes(int64_t n);
void priority_order(hipStream_t st, int64_t n, int64_t m, uint64_t seed, const uint32_t* beta_caller,
                    const int32_t* orig, uint32_t* beta_i, uint64_t* U_i, int32_t* by_rank, void* scratch,
                    size_t scratch_size);
void run_reach(hipStream_t st, const ReachArgs& a, void* scratch, size_t scratch_size, ReachStats* stats);

}  // namespace ccg
