// Host runtime and C ABI of the closeness-centrality library (see
// include/ccgpu.h).  Orchestrates: sample draw -> k-source traversal (batched
// bit-parallel BFS, plain BFS, or delta-stepping for integer lengths) ->
// estimator epilogue, on one HIP stream, plus a continuous-batching job
// service over resident graphs.
#include "ccgpu.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace ccg;

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

static cc_status fail(cc_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

extern "C" const char* cc_status_str(cc_status s) {
    switch (s) {
        case CC_OK: return "ok";
        case CC_EINVAL: return "invalid argument";
        case CC_EDISCONNECTED: return "graph not (strongly) connected";
        case CC_ENOMEM: return "out of memory";
        case CC_EOVERFLOW: return "overflow";
        case CC_EDEVICE: return "device error";
        case CC_EBUSY: return "busy";
        case CC_ECANCELLED: return "cancelled";
        case CC_ENOTREADY: return "not ready";
    }
    return "unknown status";
}

extern "C" const char* cc_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------- sampler

namespace {

struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // Lemire: uniform in [0, range)
    uint64_t below(uint64_t range) {
        unsigned __int128 m = (unsigned __int128)next() * range;
        uint64_t lo = (uint64_t)m;
        if (lo < range) {
            const uint64_t t = (0 - range) % range;
            while (lo < t) {
                m = (unsigned __int128)next() * range;
                lo = (uint64_t)m;
            }
        }
        return (uint64_t)(m >> 64);
    }
};

// Fisher-Yates over a[0..n): the same draws and swaps, in the same order, as
// swapping a[i] with a[i + below(n - i)] for i = 0, 1, ..., n - 1. The draws do
// not depend on the array, so each swap target is drawn kAhead steps early and
// its line prefetched; the generator ends in the same state.
void shuffle(SplitMix64& rng, int32_t* a, int64_t n) {
    constexpr int64_t kAhead = 16;
    int64_t ring[kAhead];
    for (int64_t i = 0; i < std::min(kAhead, n); i++) {
        ring[i] = i + (int64_t)rng.below((uint64_t)(n - i));
        __builtin_prefetch(a + ring[i], 1);
    }
    for (int64_t i = 0; i < n; i++) {
        const int64_t j = ring[i % kAhead];
        const int64_t ia = i + kAhead;
        if (ia < n) {
            const int64_t ja = ia + (int64_t)rng.below((uint64_t)(n - ia));
            ring[ia % kAhead] = ja;
            __builtin_prefetch(a + ja, 1);
        }
        std::swap(a[i], a[j]);
    }
}

}  // namespace

extern "C" cc_status cc_draw_samples(int64_t n, int32_t k, uint64_t seed, int32_t* out) {
    if (!out || k < 1 || n < k || n > INT32_MAX) return fail(CC_EINVAL, "cc_draw_samples: need 1 <= k <= n < 2^31");
    SplitMix64 r{seed};
    std::unordered_map<int64_t, int64_t> moved;
    moved.reserve((size_t)k * 2);
    for (int32_t i = 0; i < k; i++) {
        const int64_t j = i + (int64_t)r.below((uint64_t)(n - i));
        auto it_i = moved.find(i);
        auto it_j = moved.find(j);
        const int64_t ai = it_i == moved.end() ? i : it_i->second;
        const int64_t aj = it_j == moved.end() ? j : it_j->second;
        moved[i] = aj;
        moved[j] = ai;
        out[i] = (int32_t)aj;
    }
    return CC_OK;
}

// Node-weighted sample (Sec. 5): VarOpt's threshold in exact integers, heavy
// nodes taken, light ones by ordered pivotal sampling over a random order.
extern "C" cc_status cc_draw_weighted(int64_t n, const uint32_t* beta, int32_t k, uint64_t seed, int32_t* ids,
                                      uint8_t* light, int64_t* R_out, int32_t* m_out, int32_t* count) {
    if (!beta || !ids || !light || !R_out || !m_out || !count || k < 1 || n < 1 || n > INT32_MAX)
        return fail(CC_EINVAL, "cc_draw_weighted: bad argument");
    std::vector<int32_t> pos;
    int64_t total = 0;
    for (int64_t v = 0; v < n; v++) {
        if (beta[v] == 0) continue;
        pos.push_back((int32_t)v);
        total += beta[v];
        if (total >= ((int64_t)1 << 62)) return fail(CC_EINVAL, "cc_draw_weighted: total weight reaches 2^62");
    }
    if (pos.empty()) return fail(CC_EINVAL, "cc_draw_weighted: no node of positive weight");
    if ((int64_t)pos.size() <= k) {  // every positive node, at its own weight
        for (size_t i = 0; i < pos.size(); i++) {
            ids[i] = pos[i];
            light[i] = 0;
        }
        *R_out = 0;
        *m_out = 1;
        *count = (int32_t)pos.size();
        return CC_OK;
    }
    // VarOpt's threshold: the heavy nodes are the first L in weight order
    // only the k heaviest can be heavy: order those (weight down, id up)
    std::vector<int32_t> heavy_first = pos;
    // a heap of the k heaviest: with heavy-tailed weights few nodes ever enter it
    std::partial_sort(heavy_first.begin(), heavy_first.begin() + k, heavy_first.end(), [&](int32_t a, int32_t b) {
        return beta[a] != beta[b] ? beta[a] > beta[b] : a < b;
    });
    int64_t R = total;
    int32_t L = 0;
    while (!((int64_t)beta[heavy_first[(size_t)L]] * (int64_t)(k - L) < R)) {
        R -= beta[heavy_first[(size_t)L]];
        L++;
    }
    const int64_t m = k - L;
    std::vector<char> is_heavy((size_t)n, 0), taken((size_t)n, 0);
    for (int32_t i = 0; i < L; i++) is_heavy[(size_t)heavy_first[(size_t)i]] = taken[(size_t)heavy_first[(size_t)i]] = 1;
    // the random order: cc_draw_samples(n, n, seed)'s permutation; its generator continues for the decisions
    SplitMix64 rng{seed};
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; i++) perm[(size_t)i] = (int32_t)i;
    shuffle(rng, perm.data(), n);
    const uint64_t Q = (uint64_t)R;
    auto yes = [&](uint64_t num, uint64_t den) {
        return (unsigned __int128)rng.next() * den < ((unsigned __int128)num << 64);
    };
    int64_t cur = -1;
    uint64_t ca = 0;
    constexpr int64_t kAhead = 16;  // nodes ahead whose weight and flag are prefetched
    for (int64_t r = 0; r < n; r++) {
        if (r + kAhead < n) {
            const int32_t u = perm[(size_t)(r + kAhead)];
            __builtin_prefetch(beta + u);
            __builtin_prefetch(is_heavy.data() + u);
        }
        const int32_t v = perm[(size_t)r];
        if (beta[v] == 0 || is_heavy[(size_t)v]) continue;
        const uint64_t b = (uint64_t)beta[v] * (uint64_t)m;
        if (cur < 0) {
            cur = v;
            ca = b;
            continue;
        }
        const uint64_t sum = ca + b;
        if (sum <= Q) {  // one of the two gets the sum, the other is dropped
            if (!yes(ca, sum)) cur = v;
            ca = sum;
            if (ca == Q) {
                taken[(size_t)cur] = 1;
                cur = -1;
                ca = 0;
            }
        } else {  // one of the two is taken, the other keeps sum - Q
            if (yes(Q - b, 2 * Q - sum)) {
                taken[(size_t)cur] = 1;
                cur = v;
            } else {
                taken[(size_t)v] = 1;
            }
            ca = sum - Q;
        }
    }
    if (cur >= 0) return fail(CC_EINVAL, "cc_draw_weighted: pivotal sampling left a fractional mass");
    int32_t c = 0;
    for (int64_t v = 0; v < n; v++) {
        if (!taken[(size_t)v]) continue;
        if (c >= k) return fail(CC_EINVAL, "cc_draw_weighted: sample larger than k");
        ids[c] = (int32_t)v;
        light[c] = is_heavy[(size_t)v] ? 0 : 1;
        c++;
    }
    if (c != k) return fail(CC_EINVAL, "cc_draw_weighted: sample smaller than k");
    *R_out = R;
    *m_out = (int32_t)m;
    *count = c;
    return CC_OK;
}

// ---------------------------------------------------------------- device arena

namespace {

// Thrown when an estimate needs more than a fixed (allocation-free) buffer holds.
struct FixedScratchFull {
    size_t need, have;
};

// A growable device buffer; one per stream that runs jobs.  A fixed arena
// is a slice of the static scratch array and never allocates.
struct Arena {
    void* ptr = nullptr;
    size_t size = 0;
    bool fixed = false;
    uint64_t* gen = nullptr;  // bumped whenever the buffer moves (captured graphs refer to it)
    ~Arena() {
        if (ptr && !fixed) (void)hipFree(ptr);
    }
    void* get(size_t need) {
        if (need <= size) return ptr;
        if (fixed) throw FixedScratchFull{need, size};
        if (gen) ++*gen;
        if (ptr) {
            CCG_HIP(hipFree(ptr));
            ptr = nullptr;
            size = 0;
        }
        need = (need + (1u << 20)) & ~size_t((1u << 20) - 1);
        hipError_t e = hipMalloc(&ptr, need);
        if (e != hipSuccess) {
            ptr = nullptr;
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
        size = need;
        return ptr;
    }
};

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(size_t count) {
        T* p = (T*)(base + off);
        off += (sizeof(T) * count + 255) & ~size_t(255);
        return p;
    }
    static size_t sz(size_t bytes) { return (bytes + 255) & ~size_t(255); }
};

// Everything one job needs on one stream.
// Copies a finished estimate's control block and flags into pinned host memory
// through its device-visible address (system-scope stores), so that a replayed
// estimate needs no copy commands after its last kernel.
__global__ void k_status_out(const uint32_t* __restrict__ ctl, const uint32_t* __restrict__ flags,
                             uint32_t* ctl_host, uint32_t* flags_host) {
    constexpr int nc = (int)(sizeof(BfsCtl) / 4), nf = (int)(sizeof(DevFlags) / 4);
    static_assert(sizeof(BfsCtl) % 4 == 0 && sizeof(DevFlags) % 4 == 0 && nc + nf <= 64, "one wave copies both");
    const int t = threadIdx.x;
    if (t < nc) __hip_atomic_store(ctl_host + t, ctl[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    else if (t < nc + nf)
        __hip_atomic_store(flags_host + (t - nc), flags[t - nc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The samples from the lane's pinned staging buffer (system-scope loads see
// what the host wrote before the launch): internal ids to samples, the
// caller's ids to the samples output when one is requested.
__global__ void k_stage_samples(const int32_t* stage_ids, const int32_t* stage_caller, int32_t k, int32_t* samples,
                                int32_t* samples_out) {
    for (int32_t i = threadIdx.x; i < k; i += blockDim.x) {
        samples[i] = __hip_atomic_load(stage_ids + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (samples_out) samples_out[i] = __hip_atomic_load(stage_caller + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// A captured weighted estimate's last launch: its flags and the largest
// distance of each direction's searches, into pinned memory.
__global__ void k_wstatus_out(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ maxd,
                              uint32_t* flags_host, uint32_t* maxd_host) {
    constexpr int nf = (int)(sizeof(DevFlags) / 4);
    const int t = threadIdx.x;
    if (t < nf) __hip_atomic_store(flags_host + t, flags[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    else if (t < nf + 2) __hip_atomic_store(maxd_host + (t - nf), maxd[t - nf], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

constexpr int32_t kStagedSamples = 256;  // samples of an estimate that can be replayed from a captured graph

struct Lane {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Arena arena;      // per-job small buffers and traversal state
    Arena arenaD;     // distance matrices / level masks
    Arena arena2;     // epilogue tables (sized once the largest distance is known)
    Arena arenaW;     // node-weighted estimate: its distance rows and per-node arrays
    Arena arenaO;     // device staging of host outputs
    char* pin = nullptr;  // pinned host staging of host outputs (grown when a larger job comes)
    size_t pin_size = 0;
    char* pinned_host(size_t need) {
        if (need <= pin_size) return pin;
        if (pin) CCG_HIP(hipHostFree(pin));
        pin = nullptr;
        pin_size = 0;
        need = (need + (1u << 20)) & ~size_t((1u << 20) - 1);
        if (hipHostMalloc((void**)&pin, need, hipHostMallocDefault) != hipSuccess) {
            pin = nullptr;
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
        pin_size = need;
        return pin;
    }
    size_t retained() const { return arena.size + arenaD.size + arena2.size + arenaW.size + arenaO.size; }
    void trim() {  // give the buffers back (the next job allocates afresh)
        Arena* as[5] = {&arena, &arenaD, &arena2, &arenaW, &arenaO};
        for (Arena* a : as)
            if (a->ptr && !a->fixed) {
                if (a->gen) ++*a->gen;
                (void)hipFree(a->ptr);
                a->ptr = nullptr;
                a->size = 0;
            }
    }
    LevelCounters* cnt_host = nullptr;  // pinned
    struct Readback {
        BfsCtl ctl;
        DevFlags flags;
        BfsCtl ctl_fwd;  // a round-trip replay: the forward search's control block
        DevFlags flags_fwd;
        uint32_t wmaxd[2];  // a weighted replay: the largest distance of each direction's searches
        int32_t ids[kStagedSamples];     // the samples, internal ids (read by the traversal's first launch)
        int32_t caller[kStagedSamples];  // the same, as the caller numbers them
    };
    Readback* rb_host = nullptr;  // pinned: a replay's control block and flags, and the staged samples
    Readback* rb_dev = nullptr;   // its device-visible address
    hipEvent_t ev[4] = {};
    // a captured round trip runs its reverse search on a second stream, a
    // parallel branch of the graph (created when first needed)
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    void ensure_side() {
        if (side) return;
        CCG_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        CCG_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
        CCG_HIP(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
    }
    EventPool events;  // per-launch timing inside the traversals
    uint64_t gen = 0;  // arena generation
    int64_t last_maxd = -1;  // an upper bound on the last job's largest distance (-1: unknown)
    bool no_alloc = false;   // the allocation-free lane: fixed arenas, no event pool, no capture
    // Captured estimates (stream capture of a whole estimate), replayed when
    // the same graph, parameters, buffers and outputs come again.
    struct Captured {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
        int32_t lmax = 0, levels = 0;
        int32_t lmax_fwd = -1, levels_fwd = 0;  // round trip: the forward search (the reverse one above)
        bool weighted = false;  // weighted searches: lmax_fwd, lmax bound each direction's largest distance
    };
    std::vector<Captured> captured;  // most recently used last
    static constexpr size_t kMaxCaptured = 8;
    Captured* find_captured(const std::vector<uint64_t>& key) {
        for (size_t i = 0; i < captured.size(); i++) {
            if (captured[i].key == key) {
                std::rotate(captured.begin() + i, captured.begin() + i + 1, captured.end());
                return &captured.back();
            }
        }
        return nullptr;
    }
    void add_captured(Captured c) {
        if (captured.size() >= kMaxCaptured) {
            (void)hipGraphExecDestroy(captured.front().exec);
            captured.erase(captured.begin());
        }
        captured.push_back(std::move(c));
    }
    void init(hipStream_t s) {
        arena.gen = arenaD.gen = arena2.gen = arenaO.gen = &gen;
        if (s) {
            stream = s;
        } else {
            CCG_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            own_stream = true;
        }
        CCG_HIP(hipHostMalloc((void**)&cnt_host, sizeof(LevelCounters) * kCounterSlots, hipHostMallocDefault));
        CCG_HIP(hipHostMalloc((void**)&rb_host, sizeof(Readback), hipHostMallocDefault));
        CCG_HIP(hipHostGetDevicePointer((void**)&rb_dev, rb_host, 0));
        for (auto& e : ev) CCG_HIP(hipEventCreate(&e));
    }
    void destroy() {
        for (auto& c : captured) (void)hipGraphExecDestroy(c.exec);
        captured.clear();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (side) (void)hipStreamDestroy(side);
        fork_ev = join_ev = nullptr;
        side = nullptr;
        if (cnt_host) (void)hipHostFree(cnt_host);
        if (rb_host) (void)hipHostFree(rb_host);
        if (pin) (void)hipHostFree(pin);
        pin = nullptr;
        pin_size = 0;
        rb_host = nullptr;
        rb_dev = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        cnt_host = nullptr;
        stream = nullptr;
    }
};

}  // namespace

// ---------------------------------------------------------------- objects

struct cc_graph {
    cc_context* ctx = nullptr;
    DevGraph dg;
    uint32_t flags = 0;
    std::atomic<int> refs{1};
    void* mem[12] = {};
    size_t bytes = 0;
    std::vector<int32_t> inv;  // caller's id -> internal id
    uint64_t id = 0;  // never reused: keys captured estimates
    std::vector<int32_t> chunks_host;  // hub chunk triples (undirected graphs), for batching
    bool borrowed = false;  // the arcs (and lengths) are the caller's device arrays, never freed here
    mutable std::atomic<int32_t> bfs_hint{0};  // levels the last batched traversal of this graph ran
    cc_tuning tune{4, 1024, 8192, 1, 1024, 64};  // launch shapes (cc_graph_set_tuning / cc_autotune)
};

struct cc_job {
    cc_context* ctx = nullptr;
    cc_graph* g = nullptr;
    cc_params p{};
    std::vector<int32_t> samples;
    cc_result out{};
    std::atomic<int> state{0};  // 0 queued, 1 running, 2 done, 3 cancelled
    cc_status status = CC_ENOTREADY;
    std::string err;
    size_t need = 0;
    int32_t overtaken = 0;  // younger jobs admitted while this one waited at the front
    std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
    std::mutex m;
    std::condition_variable cv;
    std::atomic<int> refs{2};  // caller + service
};

struct cc_context {
    int device = 0;
    cc_config cfg{};
    std::mutex mu;  // serialises synchronous calls on the default lane
    Lane lane;
    cc_timing last{};
    // the allocation-free entry point: a lane whose buffers are slices of the
    // device's static scratch array (set up when the context is created)
    Lane fixed_lane;
    bool fixed_ready = false;
    // serving
    std::mutex qmu;
    std::condition_variable qcv;
    std::deque<cc_job*> queue;
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Lane>> worker_lanes;
    int64_t budget = 0;
    int64_t in_use = 0;
    int inflight = 0;
    bool stopping = false;
    bool service_started = false;
};

static void graph_unref(cc_graph* g) {
    if (!g) return;
    if (g->refs.fetch_sub(1) == 1) {
        (void)hipSetDevice(g->ctx->device);
        for (void* p : g->mem)
            if (p) (void)hipFree(p);
        delete g;
    }
}

// ---------------------------------------------------------------- context

// ---------------------------------------------------------------- static scratch
// Device memory for cc_estimate_device_noalloc: a file-scope array that every
// GPU the library runs on holds until the process ends.  Host code never uses
// its name as an address: the address is taken once per device with that
// device current (scratch_address) and kept.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr size_t kNoAllocSmall = (size_t)16 << 20;   // per-job buffers, traversal state, level histograms
constexpr size_t kNoAllocMasks = (size_t)40 << 20;   // level snapshots (and D)
constexpr size_t kNoAllocTables = kNoAllocBytes - kNoAllocSmall - kNoAllocMasks;  // epilogue tables
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static std::unordered_map<int, void*> g_scratch_ptr;      // device -> address of its copy of scratch
static std::unordered_map<int, std::mutex*> g_scratch_use;  // device -> serialises its users

// The current device's copy of `scratch` (looked up once per device).
static void* scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void* p = nullptr;
    CCG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
    g_scratch_use[device] = new std::mutex();
    return p;
}

static std::mutex& scratch_user_lock(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return *g_scratch_use.at(device);
}

extern "C" cc_status cc_context_create(int device, const cc_config* cfg, cc_context** out) {
    if (!out) return fail(CC_EINVAL, "cc_context_create: out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return fail(CC_EDEVICE, "cc_context_create: no such HIP device");
    }
    cc_context* ctx = new (std::nothrow) cc_context();
    if (!ctx) return fail(CC_ENOMEM, "cc_context_create: host allocation");
    ctx->device = device;
    if (cfg) ctx->cfg = *cfg;
    try {
        CCG_HIP(hipSetDevice(device));
        ctx->lane.init(nullptr);
        // the allocation-free lane: its buffers are fixed slices of `scratch`
        char* sp = (char*)scratch_address(device);
        ctx->fixed_lane.init(nullptr);
        Arena* parts[3] = {&ctx->fixed_lane.arena, &ctx->fixed_lane.arenaD, &ctx->fixed_lane.arena2};
        const size_t sizes[3] = {kNoAllocSmall, kNoAllocMasks, kNoAllocTables};
        for (int q = 0; q < 3; q++) {
            parts[q]->fixed = true;
            parts[q]->ptr = sp;
            parts[q]->size = sizes[q];
            sp += sizes[q];
        }
        ctx->fixed_lane.no_alloc = true;
        ctx->fixed_ready = true;
        size_t fr = 0, tot = 0;
        CCG_HIP(hipMemGetInfo(&fr, &tot));
        ctx->budget = ctx->cfg.mem_budget_bytes > 0 ? ctx->cfg.mem_budget_bytes : (int64_t)(0.8 * (double)fr);
    } catch (const HipError& e) {
        delete ctx;
        return fail(CC_EDEVICE, "cc_context_create: " + e.where + ": " + hipGetErrorString(e.err));
    }
    *out = ctx;
    return CC_OK;
}

extern "C" void cc_context_destroy(cc_context* ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        ctx->stopping = true;
        for (cc_job* j : ctx->queue) {
            j->state = 3;
            j->status = CC_ECANCELLED;
            graph_unref(j->g);
            j->g = nullptr;
            {
                std::lock_guard<std::mutex> jl(j->m);
            }
            j->cv.notify_all();
            if (j->refs.fetch_sub(1) == 1) delete j;
        }
        ctx->queue.clear();
    }
    ctx->qcv.notify_all();
    for (auto& t : ctx->workers) t.join();
    (void)hipSetDevice(ctx->device);
    for (auto& l : ctx->worker_lanes) {
        (void)hipStreamSynchronize(l->stream);
        l->destroy();
    }
    ctx->worker_lanes.clear();
    (void)hipStreamSynchronize(ctx->lane.stream);
    ctx->lane.destroy();
    if (ctx->fixed_ready) {
        (void)hipStreamSynchronize(ctx->fixed_lane.stream);
        ctx->fixed_lane.destroy();
    }
    delete ctx;
}

// ---------------------------------------------------------------- graphs

static bool check_csr(int64_t n, int64_t arcs, const int64_t* rp, const int32_t* col, const int32_t* w,
                      bool directed, std::string& why) {
    if (rp[0] != 0 || rp[n] != arcs) {
        why = "row_ptr[0] must be 0 and row_ptr[n] must equal arcs";
        return false;
    }
    for (int64_t v = 0; v < n; v++)
        if (rp[v + 1] < rp[v]) {
            why = "row_ptr must be non-decreasing";
            return false;
        }
    for (int64_t e = 0; e < arcs; e++) {
        if (col[e] < 0 || col[e] >= n) {
            why = "col_idx out of range";
            return false;
        }
        if (w && w[e] < 1) {
            why = "arc lengths must be >= 1";
            return false;
        }
    }
    if (!directed) {
        // symmetric: count (u,v) pairs both ways with a transpose and compare
        std::vector<int64_t> trp(n + 1, 0);
        for (int64_t e = 0; e < arcs; e++) trp[col[e] + 1]++;
        for (int64_t v = 0; v < n; v++) trp[v + 1] += trp[v];
        for (int64_t v = 0; v < n; v++)
            if (trp[v + 1] - trp[v] != rp[v + 1] - rp[v]) {
                why = "undirected CSR is not symmetric (in-degree != out-degree)";
                return false;
            }
        std::vector<int64_t> pos(trp.begin(), trp.end() - 1);
        std::vector<std::pair<int32_t, int32_t>> t((size_t)arcs);
        for (int64_t u = 0; u < n; u++)
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) t[(size_t)pos[col[e]]++] = {(int32_t)u, w ? w[e] : 1};
        for (int64_t v = 0; v < n; v++) {
            std::vector<std::pair<int32_t, int32_t>> a, b;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) a.push_back({col[e], w ? w[e] : 1});
            for (int64_t e = trp[v]; e < trp[v + 1]; e++) b.push_back(t[(size_t)e]);
            std::sort(a.begin(), a.end());
            std::sort(b.begin(), b.end());
            if (a != b) {
                why = "undirected CSR is not symmetric";
                return false;
            }
        }
    }
    return true;
}

// Graph builder: internal ids sort nodes by degree (out + in), largest first,
// ties by the caller's id, so that consecutive ids have similar degree (one
// traversal wave handles 64 consecutive ids) and the high-degree nodes form a
// prefix whose adjacency is cut into fixed chunks of arcs.
namespace {
// Degree above which a node's arcs are scanned in chunks (a whole wave per
// chunk, with an early exit) rather than by a few lanes of its group.  On
// digraphs the prefix is much wider at the same threshold (17% of the nodes
// of a directed R-MAT graph pass 32), and hubs just above it leave most of a
// wave idle: 128 measured fastest there (rmat22dir round trip 3.11 -> 3.00 ms;
// 64: 3.11, 192: 3.18), while 32 stays best on undirected graphs (rmat20:
// 0.81 ms, 0.89 ms at 128).
constexpr uint32_t kHubDegree = 32;
constexpr uint32_t kHubDegreeDirected = 128;
inline uint32_t hub_degree(bool directed) { return directed ? kHubDegreeDirected : kHubDegree; }
// Arcs per chunk.  Undirected graphs take 2048 (rmat20: 0.82 -> 0.79 ms, fewer
// chunk records to claim per level); on digraphs 2048 is slower (rmat22dir
// round trip 2.98 -> 3.10 ms) and 512 no faster than 1024.
constexpr uint32_t kHubChunk = 2048;
constexpr uint32_t kHubChunkDirected = 1024;
inline uint32_t hub_chunk(bool directed) { return directed ? kHubChunkDirected : kHubChunk; }

// Runs f over [lo, hi) split into contiguous ranges on the host's threads
// (one range for small inputs).
void parallel_ranges(int64_t lo, int64_t hi, const std::function<void(int64_t, int64_t)>& f) {
    const int64_t count = hi - lo;
    const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(std::thread::hardware_concurrency(), 16));
    const int64_t parts = count < 65536 ? 1 : hw;
    if (parts <= 1) {
        if (count > 0) f(lo, hi);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t p = 0; p < parts; p++) {
        const int64_t a = lo + count * p / parts, b = lo + count * (p + 1) / parts;
        th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto& t : th) t.join();
}

std::vector<int32_t> hub_chunk_list(const std::vector<uint32_t>& rp, int64_t nh, uint32_t chunk) {
    std::vector<int32_t> c;
    for (int64_t h = 0; h < nh; h++)
        for (uint32_t b = rp[(size_t)h]; b < rp[(size_t)h + 1]; b += chunk) {
            c.push_back((int32_t)h);
            c.push_back((int32_t)b);
            c.push_back((int32_t)std::min<uint32_t>(b + chunk, rp[(size_t)h + 1]));
        }
    return c;
}

void transpose_host(int64_t n, const std::vector<uint32_t>& rp, const std::vector<int32_t>& col,
                    const std::vector<int32_t>& w, std::vector<uint32_t>& trp, std::vector<int32_t>& tcol,
                    std::vector<int32_t>& tw) {
    const size_t arcs = col.size();
    trp.assign((size_t)n + 1, 0);
    for (size_t e = 0; e < arcs; e++) trp[(size_t)col[e] + 1]++;
    for (int64_t v = 0; v < n; v++) trp[(size_t)v + 1] += trp[(size_t)v];
    std::vector<uint32_t> pos(trp.begin(), trp.end() - 1);
    tcol.resize(arcs);
    tw.resize(w.empty() ? 0 : arcs);
    for (int64_t u = 0; u < n; u++)
        for (uint32_t e = rp[(size_t)u]; e < rp[(size_t)u + 1]; e++) {
            const uint32_t q = pos[(size_t)col[e]]++;
            tcol[q] = (int32_t)u;
            if (!w.empty()) tw[q] = w[e];
        }
}
}  // namespace

// The (end, length) pairs the batched weighted searches read, for both
// directions, into library-owned slots a and b.
static void zip_weighted(cc_graph* g, int a, int b, hipStream_t st) {
    const int64_t arcs = g->dg.arcs;
    for (int dir = 0; dir < (g->dg.directed ? 2 : 1); dir++) {
        void* d = nullptr;
        if (hipMalloc(&d, sizeof(int2) * (size_t)std::max<int64_t>(arcs, 1)) != hipSuccess) {
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
        g->mem[dir == 0 ? a : b] = d;
        g->bytes += sizeof(int2) * (size_t)arcs;
        zip_arcs(st, dir == 0 ? g->dg.col : g->dg.rcol, dir == 0 ? g->dg.w : g->dg.rw, arcs, (int2*)d);
        (dir == 0 ? g->dg.cw : g->dg.rcw) = (const int2*)d;
    }
    if (!g->dg.directed) g->dg.rcw = g->dg.cw;
    CCG_HIP(hipStreamSynchronize(st));
}

extern "C" cc_status cc_graph_upload(cc_context* ctx, int64_t n, int64_t arcs, const int64_t* row_ptr,
                                     const int32_t* col_idx, const int32_t* w, uint32_t flags, cc_graph** out) {
    if (!ctx || !out || !row_ptr || (arcs > 0 && !col_idx)) return fail(CC_EINVAL, "cc_graph_upload: null argument");
    if (n < 1 || n >= INT32_MAX || arcs < 0 || arcs >= (int64_t)UINT32_MAX)
        return fail(CC_EINVAL, "cc_graph_upload: need 1 <= n < 2^31 and arcs < 2^32");
    const bool directed = (flags & CC_DIRECTED) != 0;
    if (row_ptr[0] != 0 || row_ptr[n] != arcs) return fail(CC_EINVAL, "cc_graph_upload: row_ptr[0]/row_ptr[n] mismatch");
    {
        // shape, id range and lengths are always checked (kernels index with
        // them); symmetry of undirected graphs only with CC_VALIDATE
        std::string why;
        if (!check_csr(n, arcs, row_ptr, col_idx, w, directed || !(flags & CC_VALIDATE), why))
            return fail(CC_EINVAL, "cc_graph_upload: " + why);
    }
    cc_graph* g = new (std::nothrow) cc_graph();
    if (!g) return fail(CC_ENOMEM, "cc_graph_upload: host allocation");
    g->ctx = ctx;
    static std::atomic<uint64_t> next_graph_id{1};
    g->id = next_graph_id.fetch_add(1);
    g->flags = flags;
    g->dg.n = n;
    g->dg.arcs = arcs;
    g->dg.directed = directed;
    g->dg.weighted = w != nullptr;
    try {
        CCG_HIP(hipSetDevice(ctx->device));
        // ---- degree order
        std::vector<int64_t> deg((size_t)n, 0);
        for (int64_t v = 0; v < n; v++) deg[(size_t)v] = row_ptr[v + 1] - row_ptr[v];
        if (directed)
            for (int64_t e = 0; e < arcs; e++) deg[(size_t)col_idx[e]]++;
        std::vector<int32_t> orig((size_t)n);
        for (int64_t v = 0; v < n; v++) orig[(size_t)v] = (int32_t)v;
        // weighted graphs keep the caller's order (delta-stepping works on
        // (sample, node) pairs and profits from the input's own locality)
        if (!w)
            std::stable_sort(orig.begin(), orig.end(),
                             [&](int32_t a, int32_t b) { return deg[(size_t)a] > deg[(size_t)b]; });
        if (!w) {
            // Locality for the hub pulls: after the hubs (a prefix by degree;
            // for digraphs by in+out degree, which keeps every node whose in-
            // or out-degree passes the hub threshold inside the prefix), nodes
            // go by coarse degree class (so 64-node groups stay even) and then
            // by their first hub (out-)neighbour, so that the neighbours a
            // hub's chunk gathers sit close together in id order.
            int64_t H = 0;
            while (H < n && deg[(size_t)orig[(size_t)H]] > (int64_t)hub_degree(directed)) H++;
            std::vector<int64_t> rank((size_t)n);
            for (int64_t i = 0; i < n; i++) rank[(size_t)orig[(size_t)i]] = i;
            std::vector<int64_t> first_hub((size_t)n, H);
            parallel_ranges(H, n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; i++) {
                    const int64_t v = orig[(size_t)i];
                    int64_t f = H;
                    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) f = std::min(f, rank[(size_t)col_idx[e]]);
                    first_hub[(size_t)v] = f;
                }
            });
            auto cls = [&](int64_t v) { return 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(deg[(size_t)v], 1)); };
            std::stable_sort(orig.begin() + H, orig.end(), [&](int32_t a, int32_t b) {
                const int ca = cls(a), cb = cls(b);
                if (ca != cb) return ca > cb;
                return first_hub[(size_t)a] < first_hub[(size_t)b];
            });
        }
        g->inv.assign((size_t)n, 0);
        for (int64_t i = 0; i < n; i++) g->inv[(size_t)orig[(size_t)i]] = (int32_t)i;
        // ---- relabelled out-arcs
        std::vector<uint32_t> rp((size_t)n + 1, 0);
        std::vector<int32_t> col((size_t)arcs), ww(w ? (size_t)arcs : 0);
        for (int64_t i = 0; i < n; i++) {
            const int64_t v = orig[(size_t)i];
            rp[(size_t)i + 1] = rp[(size_t)i] + (uint32_t)(row_ptr[v + 1] - row_ptr[v]);
        }
        parallel_ranges(0, n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; i++) {
                const int64_t v = orig[(size_t)i];
                uint32_t q = rp[(size_t)i];
                for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++, q++) {
                    col[q] = g->inv[(size_t)col_idx[e]];
                    if (w) ww[q] = w[e];
                }
                // rows in id order: a chunk's lanes then read neighbouring masks
                if (!w) std::sort(col.begin() + rp[(size_t)i], col.begin() + rp[(size_t)i + 1]);
            }
        });
        std::vector<uint32_t> trp;
        std::vector<int32_t> tcol, tw;
        if (directed) transpose_host(n, rp, col, ww, trp, tcol, tw);
        // ---- hub prefix (by in-degree of the pull direction; for digraphs by
        //      the larger of the two, ids being sorted by total degree)
        const std::vector<uint32_t>& prp = directed ? trp : rp;
        int64_t hubs = 0;
        for (int64_t i = 0; i < n; i++) {
            const uint32_t din = prp[(size_t)i + 1] - prp[(size_t)i];
            const uint32_t dout = rp[(size_t)i + 1] - rp[(size_t)i];
            if (std::max(din, dout) > hub_degree(directed)) hubs = i + 1;
        }
        int64_t nh = (hubs + 63) / 64 * 64;
        if (nh > n) nh = n;
        if (w) nh = 0;
        g->dg.nh = nh;
        if (w) {
            double sw = 0;
            for (int64_t e = 0; e < arcs; e++) sw += w[e];
            const double mean = arcs > 0 ? sw / (double)arcs : 1.0;
            g->dg.delta = (uint32_t)std::max<double>(1.0, std::llround(1.5 * mean));
        }
        g->tune.delta = (int32_t)std::min<uint32_t>(std::max<uint32_t>(g->dg.delta, 1u), INT32_MAX);
        std::vector<int32_t> ch_in = hub_chunk_list(prp, nh, hub_chunk(directed));
        std::vector<int32_t> ch_out = directed ? hub_chunk_list(rp, nh, hub_chunk(directed)) : std::vector<int32_t>();
        if (!directed) g->chunks_host = ch_in;

        auto up = [&](int slot, const void* src, size_t bytes) -> void* {
            void* d = nullptr;
            hipError_t e = hipMalloc(&d, bytes ? bytes : 4);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw std::bad_alloc();
            }
            g->mem[slot] = d;
            g->bytes += bytes;
            if (bytes) CCG_HIP(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
            return d;
        };
        g->dg.rp = (const uint32_t*)up(0, rp.data(), sizeof(uint32_t) * (n + 1));
        g->dg.col = (const int32_t*)up(1, col.data(), sizeof(int32_t) * arcs);
        if (w) g->dg.w = (const int32_t*)up(2, ww.data(), sizeof(int32_t) * arcs);
        if (directed) {
            g->dg.rrp = (const uint32_t*)up(3, trp.data(), sizeof(uint32_t) * (n + 1));
            g->dg.rcol = (const int32_t*)up(4, tcol.data(), sizeof(int32_t) * arcs);
            if (w) g->dg.rw = (const int32_t*)up(5, tw.data(), sizeof(int32_t) * arcs);
        } else {
            g->dg.rrp = g->dg.rp;
            g->dg.rcol = g->dg.col;
            g->dg.rw = g->dg.w;
        }
        g->dg.orig = (const int32_t*)up(6, orig.data(), sizeof(int32_t) * n);
        g->dg.inv = (const int32_t*)up(9, g->inv.data(), sizeof(int32_t) * n);
        g->dg.hub_chunks_in = (const int32_t*)up(7, ch_in.data(), sizeof(int32_t) * ch_in.size());
        g->dg.n_hub_chunks_in = (int32_t)(ch_in.size() / 3);
        if (directed) {
            g->dg.hub_chunks_out = (const int32_t*)up(8, ch_out.data(), sizeof(int32_t) * ch_out.size());
            g->dg.n_hub_chunks_out = (int32_t)(ch_out.size() / 3);
        } else {
            g->dg.hub_chunks_out = g->dg.hub_chunks_in;
            g->dg.n_hub_chunks_out = g->dg.n_hub_chunks_in;
        }
        if (w) zip_weighted(g, 10, 11, nullptr);
    } catch (const std::bad_alloc&) {
        graph_unref(g);
        return fail(CC_ENOMEM, "cc_graph_upload: device allocation failed");
    } catch (const HipError& e) {
        graph_unref(g);
        return fail(CC_EDEVICE, "cc_graph_upload: " + e.where + ": " + hipGetErrorString(e.err));
    }
    *out = g;
    return CC_OK;
}

// ---------------------------------------------------------------- borrowed device CSR

namespace {
constexpr int kPrepBlock = 256;

// Range checks of a borrowed CSR's arcs: end ids in [0, n), lengths >= 1.
__global__ void k_borrow_check(const int32_t* __restrict__ col, const int32_t* __restrict__ w, int64_t arcs,
                               int64_t n, int32_t* bad) {
    bool b = false;
    for (int64_t e = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x; e < arcs; e += (int64_t)gridDim.x * kPrepBlock)
        b = b || col[e] < 0 || col[e] >= n || (w && w[e] < 1);
    if (b) *bad = 1;
}

// Sum of the arc lengths (for the default bucket width) and the in-degrees.
__global__ void k_borrow_sums(const int32_t* __restrict__ col, const int32_t* __restrict__ w, int64_t arcs,
                              unsigned long long* wsum, uint32_t* indeg) {
    unsigned long long s = 0;
    for (int64_t e = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x; e < arcs; e += (int64_t)gridDim.x * kPrepBlock) {
        if (w) s += (unsigned long long)w[e];
        if (indeg) atomicAdd(&indeg[col[e]], 1u);
    }
    if (w) atomicAdd(wsum, s);
}

// The transposed arcs of a digraph: each node's out-arcs land in their
// targets' rows (row order is immaterial to every search).
__global__ void k_borrow_transpose(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                   const int32_t* __restrict__ w, int64_t n, uint32_t* pos, int32_t* tcol,
                                   int32_t* tw) {
    for (int64_t u = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kPrepBlock)
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            const uint32_t q = atomicAdd(&pos[col[e]], 1u);
            tcol[q] = (int32_t)u;
            if (w) tw[q] = w[e];
        }
}

__global__ void k_iota(int32_t* a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPrepBlock)
        a[i] = (int32_t)i;
}

unsigned prep_grid(int64_t items) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + kPrepBlock - 1) / kPrepBlock, 8192)); }
}  // namespace

extern "C" cc_status cc_graph_borrow_device(cc_context* ctx, int64_t n, int64_t arcs, const int64_t* row_ptr,
                                            const int32_t* col_idx, const int32_t* w, uint32_t flags,
                                            cc_graph** out) {
    if (!ctx || !out || !row_ptr || (arcs > 0 && !col_idx))
        return fail(CC_EINVAL, "cc_graph_borrow_device: null argument");
    if (n < 1 || n >= INT32_MAX || arcs < 0 || arcs >= (int64_t)UINT32_MAX)
        return fail(CC_EINVAL, "cc_graph_borrow_device: need 1 <= n < 2^31 and arcs < 2^32");
    const bool directed = (flags & CC_DIRECTED) != 0;
    cc_graph* g = new (std::nothrow) cc_graph();
    if (!g) return fail(CC_ENOMEM, "cc_graph_borrow_device: host allocation");
    g->ctx = ctx;
    static std::atomic<uint64_t> next_borrow_id{1ull << 62};
    g->id = next_borrow_id.fetch_add(1);
    g->flags = flags;
    g->borrowed = true;
    g->dg.n = n;
    g->dg.arcs = arcs;
    g->dg.directed = directed;
    g->dg.weighted = w != nullptr;
    std::lock_guard<std::mutex> lk(ctx->mu);  // the context's own stream does the preparation
    try {
        CCG_HIP(hipSetDevice(ctx->device));
        // the three arrays must be device memory of this context's device
        for (const void* p : {(const void*)row_ptr, (const void*)col_idx, (const void*)w}) {
            if (!p) continue;
            hipPointerAttribute_t at{};
            if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice ||
                at.device != ctx->device) {
                (void)hipGetLastError();
                graph_unref(g);
                return fail(CC_EINVAL, "cc_graph_borrow_device: an array is not device memory of the context's device");
            }
        }
        auto own = [&](int slot, size_t bytes) -> void* {
            void* d = nullptr;
            if (hipMalloc(&d, bytes ? bytes : 4) != hipSuccess) {
                (void)hipGetLastError();
                throw std::bad_alloc();
            }
            g->mem[slot] = d;
            g->bytes += bytes;
            return d;
        };
        hipStream_t st = ctx->lane.stream;
        // row bounds: read once to the host for the shape checks, the 32-bit
        // copy the kernels index with and the hub chunk lists
        std::vector<int64_t> rp64((size_t)n + 1);
        CCG_HIP(hipMemcpy(rp64.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
        if (rp64[0] != 0 || rp64[(size_t)n] != arcs) {
            graph_unref(g);
            return fail(CC_EINVAL, "cc_graph_borrow_device: row_ptr[0] must be 0 and row_ptr[n] must equal arcs");
        }
        std::vector<uint32_t> rp((size_t)n + 1);
        for (int64_t v = 0; v <= n; v++) {
            if (v < n && rp64[(size_t)v + 1] < rp64[(size_t)v]) {
                graph_unref(g);
                return fail(CC_EINVAL, "cc_graph_borrow_device: row_ptr must be non-decreasing");
            }
            rp[(size_t)v] = (uint32_t)rp64[(size_t)v];
        }
        // ids and lengths, on the device; in-degrees and the length sum with them
        // [0]: a bad id or length seen; [2..3]: the sum of the lengths
        int32_t* bad = (int32_t*)own(0, 2 * sizeof(int32_t) + sizeof(unsigned long long));
        unsigned long long* wsum = (unsigned long long*)(bad + 2);
        CCG_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(int32_t) + sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_borrow_check, dim3(prep_grid(arcs)), dim3(kPrepBlock), 0, st, col_idx, w, arcs, n, bad);
        int32_t bad_h = 0;
        CCG_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        if (bad_h) {
            graph_unref(g);
            return fail(CC_EINVAL, "cc_graph_borrow_device: col_idx out of range or an arc length below 1");
        }
        if ((flags & CC_VALIDATE) && !directed) {
            // symmetry needs the arcs on the host
            std::vector<int32_t> col_h((size_t)arcs), w_h(w ? (size_t)arcs : 0);
            CCG_HIP(hipMemcpy(col_h.data(), col_idx, sizeof(int32_t) * arcs, hipMemcpyDeviceToHost));
            if (w) CCG_HIP(hipMemcpy(w_h.data(), w, sizeof(int32_t) * arcs, hipMemcpyDeviceToHost));
            std::string why;
            if (!check_csr(n, arcs, rp64.data(), col_h.data(), w ? w_h.data() : nullptr, false, why)) {
                graph_unref(g);
                return fail(CC_EINVAL, "cc_graph_borrow_device: " + why);
            }
        }
        uint32_t* indeg = directed ? (uint32_t*)own(9, sizeof(uint32_t) * (n + 1)) : nullptr;
        if (indeg) CCG_HIP(hipMemsetAsync(indeg, 0, sizeof(uint32_t) * (n + 1), st));
        if (w || indeg)
            hipLaunchKernelGGL(k_borrow_sums, dim3(prep_grid(arcs)), dim3(kPrepBlock), 0, st, col_idx, w, arcs, wsum,
                               indeg);
        std::vector<uint32_t> trp;
        if (directed) {
            std::vector<uint32_t> cnt((size_t)n);
            CCG_HIP(hipMemcpyAsync(cnt.data(), indeg, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, st));
            CCG_HIP(hipStreamSynchronize(st));
            trp.assign((size_t)n + 1, 0);
            for (int64_t v = 0; v < n; v++) trp[(size_t)v + 1] = trp[(size_t)v] + cnt[(size_t)v];
        }
        if (w) {
            unsigned long long ws = 0;
            CCG_HIP(hipMemcpyAsync(&ws, wsum, sizeof(ws), hipMemcpyDeviceToHost, st));
            CCG_HIP(hipStreamSynchronize(st));
            const double mean = arcs > 0 ? (double)ws / (double)arcs : 1.0;
            g->dg.delta = (uint32_t)std::max<double>(1.0, std::llround(1.5 * mean));
        }
        g->tune.delta = (int32_t)std::min<uint32_t>(std::max<uint32_t>(g->dg.delta, 1u), INT32_MAX);
        // the caller's order stays: 64-node groups that hold a node of high
        // in- or out-degree are flagged and all their nodes' arcs are chunked
        const int64_t ngroups = (n + 63) / 64;
        std::vector<uint8_t> ghub((size_t)ngroups, 0);
        const std::vector<uint32_t>& prp = directed ? trp : rp;
        if (!w)
            for (int64_t v = 0; v < n; v++) {
                const uint32_t din = prp[(size_t)v + 1] - prp[(size_t)v], dout = rp[(size_t)v + 1] - rp[(size_t)v];
                if (std::max(din, dout) > hub_degree(directed)) ghub[(size_t)(v / 64)] = 1;
            }
        auto chunk_list = [&](const std::vector<uint32_t>& r) {
            std::vector<int32_t> c;
            for (int64_t v = 0; v < n; v++) {
                if (!ghub[(size_t)(v / 64)]) continue;
                for (uint32_t b = r[(size_t)v]; b < r[(size_t)v + 1]; b += hub_chunk(directed)) {
                    c.push_back((int32_t)v);
                    c.push_back((int32_t)b);
                    c.push_back((int32_t)std::min<uint32_t>(b + hub_chunk(directed), r[(size_t)v + 1]));
                }
            }
            return c;
        };
        std::vector<int32_t> ch_in = chunk_list(prp);
        std::vector<int32_t> ch_out = directed ? chunk_list(rp) : std::vector<int32_t>();
        auto up = [&](int slot, const void* src, size_t bytes) -> void* {
            void* d = own(slot, bytes);
            if (bytes) CCG_HIP(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
            return d;
        };
        g->dg.rp = (const uint32_t*)up(1, rp.data(), sizeof(uint32_t) * (n + 1));
        g->dg.col = col_idx;
        g->dg.w = w;
        if (directed) {
            g->dg.rrp = (const uint32_t*)up(2, trp.data(), sizeof(uint32_t) * (n + 1));
            int32_t* tcol = (int32_t*)own(3, sizeof(int32_t) * arcs);
            int32_t* tw = w ? (int32_t*)own(4, sizeof(int32_t) * arcs) : nullptr;
            uint32_t* pos = indeg;  // reused: the in-degree counts become write positions
            CCG_HIP(hipMemcpyAsync(pos, trp.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_borrow_transpose, dim3(prep_grid(n)), dim3(kPrepBlock), 0, st, row_ptr, col_idx, w, n,
                               pos, tcol, tw);
            g->dg.rcol = tcol;
            g->dg.rw = tw;
        } else {
            g->dg.rrp = g->dg.rp;
            g->dg.rcol = g->dg.col;
            g->dg.rw = g->dg.w;
        }
        int32_t* ident = (int32_t*)own(5, sizeof(int32_t) * n);
        hipLaunchKernelGGL(k_iota, dim3(prep_grid(n)), dim3(kPrepBlock), 0, st, ident, n);
        g->dg.orig = g->dg.inv = ident;
        g->inv.resize((size_t)n);
        for (int64_t v = 0; v < n; v++) g->inv[(size_t)v] = (int32_t)v;
        g->dg.nh = 0;
        if (!w) g->dg.ghub = (const uint8_t*)up(6, ghub.data(), ghub.size());
        g->dg.hub_chunks_in = (const int32_t*)up(7, ch_in.data(), sizeof(int32_t) * ch_in.size());
        g->dg.n_hub_chunks_in = (int32_t)(ch_in.size() / 3);
        if (directed) {
            g->dg.hub_chunks_out = (const int32_t*)up(8, ch_out.data(), sizeof(int32_t) * ch_out.size());
            g->dg.n_hub_chunks_out = (int32_t)(ch_out.size() / 3);
        } else {
            g->dg.hub_chunks_out = g->dg.hub_chunks_in;
            g->dg.n_hub_chunks_out = g->dg.n_hub_chunks_in;
        }
        if (w) zip_weighted(g, 10, 11, st);
        CCG_HIP(hipStreamSynchronize(st));
    } catch (const std::bad_alloc&) {
        graph_unref(g);
        return fail(CC_ENOMEM, "cc_graph_borrow_device: device allocation failed");
    } catch (const HipError& e) {
        graph_unref(g);
        return fail(CC_EDEVICE, "cc_graph_borrow_device: " + e.where + ": " + hipGetErrorString(e.err));
    }
    *out = g;
    return CC_OK;
}

extern "C" void cc_graph_release(cc_graph* g) { graph_unref(g); }

extern "C" cc_status cc_graph_info(const cc_graph* g, int64_t* n, int64_t* arcs, uint32_t* flags) {
    if (!g) return fail(CC_EINVAL, "cc_graph_info: null graph");
    if (n) *n = g->dg.n;
    if (arcs) *arcs = g->dg.arcs;
    if (flags) *flags = g->flags;
    return CC_OK;
}

// ---------------------------------------------------------------- estimate

namespace {

struct Resolved {
    int32_t k = 0;
    int32_t mode = CC_BATCHED;  // CC_BATCHED or CC_PLAIN
    bool graph = false;         // CC_GRAPH requested
    int64_t en = 1, ed = 1;
    std::vector<int32_t> samples;
};

cc_status resolve_params(const cc_graph* g, const cc_params* p, Resolved& r) {
    if (!g || !p) return fail(CC_EINVAL, "null graph or params");
    const int64_t n = g->dg.n;
    if (p->k < 1 || p->k > n || p->k > 4096) return fail(CC_EINVAL, "need 1 <= k <= min(n, 4096)");
    const int32_t base = p->mode & ~CC_GRAPH;
    if (base != CC_BATCHED && base != CC_PLAIN) return fail(CC_EINVAL, "mode must be CC_BATCHED or CC_PLAIN");
    if ((p->mode & CC_GRAPH) && base != CC_BATCHED) return fail(CC_EINVAL, "CC_GRAPH applies to CC_BATCHED");
    r.k = p->k;
    r.mode = base;
    r.graph = (p->mode & CC_GRAPH) != 0;
    if (p->eps_num == 0 && p->eps_den == 0) {
        r.en = 1;
        r.ed = std::max<int64_t>(1, (int64_t)std::llround(std::sqrt((double)p->k)));
    } else {
        if (p->eps_num < 1 || p->eps_den < p->eps_num) return fail(CC_EINVAL, "eps = num/den must lie in (0, 1]");
        r.en = p->eps_num;
        r.ed = p->eps_den;
    }
    r.samples.resize((size_t)r.k);
    if (p->samples) {
        std::vector<char> seen((size_t)n, 0);
        for (int32_t i = 0; i < r.k; i++) {
            const int32_t v = p->samples[i];
            if (v < 0 || v >= n) return fail(CC_EINVAL, "sample id out of range");
            if (seen[(size_t)v]) return fail(CC_EINVAL, "duplicate sample");
            seen[(size_t)v] = 1;
            r.samples[(size_t)i] = v;
        }
    } else {
        cc_status s = cc_draw_samples(n, r.k, p->seed, r.samples.data());
        if (s != CC_OK) return s;
    }
    return CC_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

// Device bytes one job needs (excluding the caller's outputs), for admission.
size_t job_bytes(const DevGraph& g, int32_t k, int32_t mode, int db) {
    const int64_t n = g.n;
    const size_t dbytes = Carver::sz((size_t)n * k * db);
    size_t b = Carver::sz(sizeof(int32_t) * k) * 2 + Carver::sz(sizeof(DevFlags)) + Carver::sz(sizeof(LevelCounters) * kCounterSlots) +
               Carver::sz(sizeof(int32_t) * n);
    if (g.weighted) {
        b += dbytes * (g.directed ? 3 : 2) + (mode == CC_PLAIN ? sssp_weighted_scratch(n, 1) : sssp_wsearch_scratch(n, k));
    } else if (mode == CC_PLAIN) {
        b += dbytes * (g.directed ? 3 : 2) + bfs_plain_scratch(n, g.arcs, k);
    } else {
        const int32_t kg = std::min(k, 256);
        b += bfs_batched_scratch(n, kg, g.nh) + (size_t)32 * n * ((kg + 63) / 64) * 8;
        if (g.directed || k > 256) b += dbytes * (g.directed ? 2 : 1);
    }
    b += Carver::sz(sizeof(int64_t) * k) + Carver::sz(sizeof(int32_t) * (size_t)k * k);
    return b;
}

void record_timing(cc_timing* timing, Lane& L, const TravStats& stats, int db) {
    if (!timing) return;
    timing->traverse_ms = elapsed(L.ev[0], L.ev[1]);
    timing->epilogue_ms = elapsed(L.ev[1], L.ev[2]);
    timing->total_ms = elapsed(L.ev[0], L.ev[2]);
    timing->levels = stats.levels;
    timing->arcs_scanned = stats.arcs_scanned;
    timing->nodes_visited = stats.nodes_visited;
    timing->launches = stats.launches;
    timing->dist_bytes = db;
    timing->kernel_ms = stats.kernel_ms;
    timing->kernel_launches = stats.kernel_launches;
    timing->arcs_matched = stats.push_arcs;
    timing->scatter_ms = stats.scatter_ms;
    timing->scatter_launches = stats.scatter_launches;
    timing->scatter_arcs = stats.scatter_arcs;
    timing->hub_arcs = stats.hub_arcs;
    timing->pull_scatter_ms = stats.pull_scatter_ms;
    timing->pull_levels = stats.pull_levels;
}

void add_stats(TravStats& a, const TravStats& b) {
    a.levels += b.levels;
    a.arcs_scanned += b.arcs_scanned;
    a.nodes_visited += b.nodes_visited;
    a.launches += b.launches;
    a.arcs_matched += b.arcs_matched;
    a.kernel_ms += b.kernel_ms;
    a.kernel_launches += b.kernel_launches;
    a.pull_levels += b.pull_levels;
    a.push_arcs += b.push_arcs;
    a.push_atomics += b.push_atomics;
    a.bfs_levels = std::max(a.bfs_levels, b.bfs_levels);
    a.scatter_ms += b.scatter_ms;
    a.scatter_launches += b.scatter_launches;
    a.scatter_arcs += b.scatter_arcs;
    a.pull_scatter_ms += b.pull_scatter_ms;
    a.hub_arcs += b.hub_arcs;
    a.maxd = std::max(a.maxd, b.maxd);
}

cc_status finish_flags(const DevFlags& hf) {
    if (hf.disconnected) return fail(CC_EDISCONNECTED, "some node is unreachable from some sample");
    if (hf.overflow) return fail(CC_EOVERFLOW, "an estimate numerator reached 2^53");
    if (hf.bad_sample) return fail(CC_EINVAL, "bad sample");
    if (hf.timeout) return fail(CC_EDEVICE, "a bounded device wait expired");
    return CC_OK;
}

void fill_epilogue_outputs(EpilogueArgs& ea, const cc_result* out, int64_t* src_sum, int32_t* dmat) {
    ea.S_err = out->S_err;
    ea.S_ad = out->S_ad;
    ea.S_ad_err = out->S_ad_err;
    ea.S_sweep = out->S_sweep;
    ea.S_sweep_err = out->S_sweep_err;
    ea.S_hyb = out->S_hyb;
    ea.S_samp = out->S_samp;
    ea.S_piv = out->S_piv;
    ea.S_pub = out->S_pub;
    ea.pivot = out->pivot;
    ea.delta = out->delta;
    ea.sampsum = out->sampsum;
    ea.src_sum = src_sum;
    ea.dmat = dmat;
    ea.Dout = out->D;
}

// Runs the whole pipeline on lane `L`; `out` holds DEVICE pointers (caller's node ids).
cc_status run_job(cc_context* ctx, const cc_graph* gr, const Resolved& r, const cc_result* out, Lane& L,
                  cc_timing* timing) {
    const DevGraph& g = gr->dg;
    const int64_t n = g.n;
    const int32_t k = r.k;
    const int32_t ngroups = (int32_t)((n + 63) / 64);
    hipStream_t st = L.stream;
    std::vector<int32_t> samples_int((size_t)k);
    for (int32_t i = 0; i < k; i++) samples_int[(size_t)i] = gr->inv[(size_t)r.samples[(size_t)i]];

    // small per-job buffers
    const size_t small = Carver::sz(sizeof(int32_t) * k) + Carver::sz(sizeof(DevFlags)) +
                         Carver::sz(sizeof(LevelCounters) * kCounterSlots) + Carver::sz(sizeof(int32_t) * n) +
                         Carver::sz(sizeof(int64_t) * k) + Carver::sz(sizeof(int32_t) * (size_t)k * k) +
                         Carver::sz(sizeof(int32_t) * ngroups) * 2 + Carver::sz(sizeof(uint32_t) * 2);
    const int32_t kg0 = std::min(k, 256);
    const int Wg = (kg0 + 63) / 64;
    // free device memory, queried (once) only where a size depends on it: the
    // weighted piles, and the level-mask budget of a search deeper than cap
    size_t free_b = 0;
    auto free_mem = [&]() {
        if (free_b == 0) {
            size_t total_b = 0;
            CCG_HIP(hipMemGetInfo(&free_b, &total_b));
        }
        return free_b;
    };
    // level masks take cap * n * W words; deep graphs whose masks would not fit
    // this budget are traversed one sample at a time instead
    auto mask_budget = [&]() { return std::min<size_t>(free_mem() / 3, (size_t)32 << 30); };
    int32_t mode = r.mode;

    int32_t cap = 32;              // level-mask capacity of the batched BFS
    DistKind dk = g.weighted ? DistKind::U32 : DistKind::U8;
    for (int attempt = 0; attempt < 16; attempt++) {
        const bool batched = mode == CC_BATCHED && !g.weighted;
        const bool bits_path = batched && !g.directed && k <= 256;
        // a round trip of one sample group: both searches and the D-based epilogue can be captured
        const bool rt_single = batched && g.directed && k <= kStagedSamples;
        TravStats stats;
        const size_t dbytes = (size_t)n * k * (int)dk;
        // weighted: samples per call (one workgroup and 16n + n/8 bytes of
        // piles per sample in the batched path; one sample per call in plain)
        int32_t kw = 1;
        if (g.weighted && mode != CC_PLAIN) {
            const size_t per = sssp_wsearch_scratch(n, 2) - sssp_wsearch_scratch(n, 1);
            kw = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)k, (free_mem() / 4) / std::max<size_t>(per, 1)));
        }
        // weighted batched searches of up to 256 samples in one launch per direction can be captured
        const bool w_single = g.weighted && mode != CC_PLAIN && kw >= k && k <= kStagedSamples;
        size_t trav_scratch;
        if (g.weighted)
            trav_scratch = mode == CC_PLAIN ? sssp_weighted_scratch(n, 1) : sssp_wsearch_scratch(n, kw);
        else
            trav_scratch = mode == CC_PLAIN ? bfs_plain_scratch(n, g.arcs, k) : bfs_batched_scratch(n, kg0, g.nh);
        const size_t hist_elems = bits_path ? (size_t)kHistSlotsBatched * k * cap : 0;
        // a round trip of one group: the reverse search's own traversal state, so that a captured
        // estimate can run both searches side by side
        const size_t rt_extra =
            rt_single ? Carver::sz(trav_scratch) + Carver::sz(sizeof(LevelCounters) * kCounterSlots) : 0;
        Carver c(L.arena.get(small + Carver::sz(trav_scratch) + Carver::sz(sizeof(int32_t) * hist_elems) + rt_extra));
        int32_t* samples_dev = c.take<int32_t>(k);
        DevFlags* flags = c.take<DevFlags>(1);
        LevelCounters* cnt = c.take<LevelCounters>(kCounterSlots);
        int32_t* sidx = c.take<int32_t>(n);
        int64_t* src_sum = out->src_sum ? out->src_sum : c.take<int64_t>(k);
        int32_t* dmat = out->dmat ? out->dmat : c.take<int32_t>((size_t)k * k);
        int32_t* fill_level = c.take<int32_t>(ngroups);
        int32_t* fill_level_r = c.take<int32_t>(ngroups);  // the reverse search's, on a round trip
        uint32_t* wmaxd_dev = c.take<uint32_t>(2);  // captured weighted searches: each direction's largest distance
        void* ts = c.take<char>(trav_scratch);
        void* ts_r = rt_single ? c.take<char>(trav_scratch) : nullptr;
        LevelCounters* cnt_r = rt_single ? c.take<LevelCounters>(kCounterSlots) : nullptr;
        int32_t* hist = bits_path ? c.take<int32_t>(hist_elems) : nullptr;
        // distance matrices and/or level masks (a round trip of one group keeps
        // both directions' masks, whose distances are then summed in one pass)
        const size_t snap_bytes = batched ? Carver::sz((size_t)cap * n * Wg * 8) * (rt_single ? 2 : 1) : 0;
        const bool need_Dt = mode == CC_PLAIN || g.weighted;
        const size_t need_D = (bits_path ? 0 : Carver::sz(dbytes) * (g.directed ? 2 : 1)) +
                              (need_Dt ? Carver::sz(dbytes) : 0);
        Carver cd(L.arenaD.get(snap_bytes + need_D + 256));
        uint64_t* snap = batched ? cd.take<uint64_t>((size_t)cap * n * Wg) : nullptr;
        uint64_t* snap_r = rt_single ? cd.take<uint64_t>((size_t)cap * n * Wg) : nullptr;
        void* D = bits_path ? nullptr : cd.take<char>(dbytes);
        void* Dr = (!bits_path && g.directed) ? cd.take<char>(dbytes) : nullptr;
        void* Dt = need_Dt ? cd.take<char>(dbytes) : nullptr;

        // a single-group traversal takes its samples from the lane's pinned staging
        // buffer in its first launch (replays included), others from a copy
        const bool stage_samples = (bits_path || rt_single || w_single) && k <= kStagedSamples;
        if (stage_samples) {
            CCG_HIP(hipStreamSynchronize(st));  // the lane's earlier launches are done with the buffer
            std::memcpy(L.rb_host->ids, samples_int.data(), sizeof(int32_t) * k);
            std::memcpy(L.rb_host->caller, r.samples.data(), sizeof(int32_t) * k);
        } else {
            CCG_HIP(hipMemcpyAsync(samples_dev, samples_int.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
        }
        auto stage_into = [&](BfsLevels& lv) {
            if (!stage_samples) return;
            lv.stage_ids = L.rb_dev->ids;
            lv.stage_caller = L.rb_dev->caller;
            lv.samples_out = out->samples;
        };

        // the adjacency a batched traversal uses in direction dir (0: forward
        // distances, pull over in-arcs / push over out-arcs; 1: reverse)
        auto make_view = [&](int dir) {
            BfsView gv;
            gv.n = n;
            gv.arcs = g.arcs;
            gv.rp = dir == 0 ? g.rrp : g.rp;
            gv.col = dir == 0 ? g.rcol : g.col;
            gv.out_rp = dir == 0 ? g.rp : g.rrp;
            gv.out_col = dir == 0 ? g.col : g.rcol;
            gv.nh = g.nh;
            gv.hub_chunks = dir == 0 ? g.hub_chunks_in : g.hub_chunks_out;
            gv.n_hub_chunks = dir == 0 ? g.n_hub_chunks_in : g.n_hub_chunks_out;
            gv.push_chunks = dir == 0 ? g.hub_chunks_out : g.hub_chunks_in;
            gv.n_push_chunks = dir == 0 ? g.n_hub_chunks_out : g.n_hub_chunks_in;
            gv.alpha = gr->tune.alpha;
            gv.level_blocks = gr->tune.level_blocks;
            gv.scatter_blocks = gr->tune.scatter_blocks;
            gv.ghub = g.ghub;
            return gv;
        };
        // a captured estimate is keyed by everything its launches refer to
        const bool want_graph = r.graph && (bits_path || rt_single || w_single);
        auto graph_key = [&]() {
            return std::vector<uint64_t>{gr->id, (uint64_t)k, (uint64_t)r.en, (uint64_t)r.ed, (uint64_t)cap,
                                         (uint64_t)(uintptr_t)st, L.gen, (uint64_t)(uintptr_t)out->S_hyb,
                                         (uint64_t)(uintptr_t)out->S_samp, (uint64_t)(uintptr_t)out->S_piv,
                                         (uint64_t)(uintptr_t)out->S_pub, (uint64_t)(uintptr_t)out->pivot,
                                         (uint64_t)(uintptr_t)out->delta, (uint64_t)(uintptr_t)out->sampsum,
                                         (uint64_t)(uintptr_t)out->src_sum, (uint64_t)(uintptr_t)out->dmat,
                                         (uint64_t)(uintptr_t)out->D, (uint64_t)(uintptr_t)out->S_err,
                                         (uint64_t)(uintptr_t)out->S_ad, (uint64_t)(uintptr_t)out->S_ad_err,
                                         (uint64_t)(uintptr_t)out->S_sweep, (uint64_t)(uintptr_t)out->S_sweep_err,
                                         (uint64_t)(uintptr_t)out->samples, (uint64_t)gr->tune.alpha,
                                         (uint64_t)gr->tune.level_blocks, (uint64_t)gr->tune.scatter_blocks};
        };
        if (want_graph) {
            if (Lane::Captured* cap_e = L.find_captured(graph_key())) {
                // the graph takes the staged samples and writes the control block and
                // flags back itself; a readback that did not land fails the check below
                L.rb_host->ctl.done = -1;
                L.rb_host->ctl_fwd.done = -1;
                L.rb_host->wmaxd[0] = 0xFFFFFFFFu;
                CCG_HIP(hipEventRecord(L.ev[0], st));
                CCG_HIP(hipGraphLaunch(cap_e->exec, st));
                CCG_HIP(hipEventRecord(L.ev[2], st));
                CCG_HIP(hipStreamSynchronize(st));
                const BfsCtl hc = L.rb_host->ctl;
                const DevFlags hf = L.rb_host->flags;
                // a round trip: the forward search must also have ended where the captured one did
                bool fwd_ok = true;
                if (cap_e->weighted) {
                    // the searches' largest distances within the captured ones (the epilogue's tables
                    // were sized for those); no traversal control block
                    const DevFlags wf = L.rb_host->flags;
                    const uint32_t m0 = L.rb_host->wmaxd[0], m1 = L.rb_host->wmaxd[1];
                    const bool ok = m0 != 0xFFFFFFFFu && !wf.disconnected && !wf.overflow && !wf.bad_sample &&
                                    !wf.timeout && (int64_t)m0 <= (int64_t)(g.directed ? cap_e->lmax_fwd : cap_e->lmax) &&
                                    (!g.directed || (int64_t)m1 <= (int64_t)cap_e->lmax);
                    if (ok) {
                        if (timing) {
                            *timing = cc_timing{};
                            timing->total_ms = timing->traverse_ms = elapsed(L.ev[0], L.ev[2]);
                            timing->launches = 1;
                        }
                        return CC_OK;
                    }
                    fwd_ok = false;  // recompute as usual
                } else if (cap_e->lmax_fwd >= 0) {
                    const BfsCtl hc0 = L.rb_host->ctl_fwd;
                    fwd_ok = hc0.done == 1 && hc0.status == 0 && hc0.lmax == cap_e->lmax_fwd &&
                             hc0.levels <= cap_e->levels_fwd;
                }
                if (fwd_ok && hc.done == 1 && hc.status == 0 && hc.lmax == cap_e->lmax &&
                    hc.levels <= cap_e->levels && !hf.disconnected && !hf.overflow && !hf.bad_sample &&
                    !hf.timeout) {
                    if (timing) {
                        *timing = cc_timing{};
                        timing->total_ms = timing->traverse_ms = elapsed(L.ev[0], L.ev[2]);
                        timing->levels = hc.levels;
                        timing->arcs_scanned = hc.arcs;
                        timing->nodes_visited = hc.nodes;
                        timing->launches = 1;
                        timing->pull_levels = hc.pull_levels;
                    }
                    return CC_OK;
                }
                // the search went deeper (or elsewhere) than the captured one:
                // recompute as usual, which rewrites every output
            }
        }
        // the batched traversal of a single sample group zeroes the flags and
        // the histogram and fills sidx in its own first launches
        if (!bits_path && !rt_single) fill_u32(st, flags, 0u, sizeof(DevFlags) / 4);
        CCG_HIP(hipEventRecord(L.ev[0], st));
        if (w_single && stage_samples)
            hipLaunchKernelGGL(k_stage_samples, dim3(1), dim3(256), 0, st, (const int32_t*)L.rb_dev->ids,
                               (const int32_t*)L.rb_dev->caller, k, samples_dev, out->samples);
        if (!bits_path && !rt_single) compute_sidx(st, samples_dev, k, sidx, n);

        // ---- traversal
        int rc = 0;
        int32_t lmax_dir[2] = {0, 0};
        int32_t levels_dir[2] = {0, 0};  // levels each direction's batched traversal ran
        bool rt_summed = false;          // D holds the round-trip distances (no separate reverse array)
        // a round trip of one sample group, after both searches: with one-byte
        // rows whose sums fit (and whole words), one pass writes the summed
        // distances to D, so the epilogue reads one array (returns true);
        // otherwise each direction's distances go to D and Dr
        auto materialize_rt = [&](int32_t lm_f, int32_t lm_r) -> bool {
            const size_t plane = (size_t)n * ((k + 63) / 64);
            if (dk == DistKind::U8 && k % 64 == 0 && (int64_t)lm_f + lm_r <= DistT<uint8_t>::max_level) {
                materialize_round_trip(st, snap, fill_level, lm_f, snap_r, fill_level_r, lm_r, n, k, D, flags);
                return true;
            }
            materialize_distances(st, snap, plane, lm_f, fill_level, n, k, 0, k, D, dk, flags, false);
            materialize_distances(st, snap_r, plane, lm_r, fill_level_r, n, k, 0, k, Dr, dk, flags, false);
            return false;
        };
        for (int dir = 0; dir < (g.directed ? 2 : 1) && rc == 0; dir++) {
            // forward distances d(c_i -> v): push over out-arcs, pull over in-arcs;
            // reverse distances d(v -> c_i): the same on the transposed graph
            const uint32_t* out_rp = dir == 0 ? g.rp : g.rrp;
            const int32_t* out_col = dir == 0 ? g.col : g.rcol;
            const uint32_t* in_rp = dir == 0 ? g.rrp : g.rp;
            const int32_t* in_col = dir == 0 ? g.rcol : g.col;
            void* Dd = dir == 0 ? D : Dr;
            TravStats ds;
            if (g.weighted) {
                const int32_t* wv = dir == 0 ? g.w : g.rw;
                int64_t md = 0;
                for (int32_t s0 = 0; s0 < k && rc == 0; s0 += kw) {
                    const int32_t kg = std::min(kw, k - s0);
                    WeightedShape shape;
                    shape.delta = (uint32_t)std::max(1, gr->tune.delta);
                    shape.round_blocks = gr->tune.round_blocks;
                    shape.local_passes = gr->tune.local_passes;
                    const int wr =
                        mode == CC_PLAIN
                            ? sssp_weighted(st, out_rp, out_col, wv, n, samples_dev + s0, kg,
                                            (uint32_t*)Dt + (size_t)s0 * n, shape, ts, trav_scratch, &md, &ds)
                            : sssp_weighted_batched(st, out_rp, dir == 0 ? g.cw : g.rcw, n, samples_dev + s0, kg,
                                                    (uint32_t*)Dt + (size_t)s0 * n, shape.delta, ts, trav_scratch,
                                                    &md, &ds);
                    if (wr == 2) rc = 2;
                    else if (wr == 4) return fail(CC_EOVERFLOW, "a weighted distance or work pile overflowed");
                    else if (wr == 5) return fail(CC_EDEVICE, "a weighted search did not finish within its time limit");
                }
                if (rc == 0) transpose_dist(st, Dt, Dd, n, k, dk);
                lmax_dir[dir] = (int32_t)std::min<int64_t>(md, INT32_MAX);
            } else if (mode == CC_PLAIN) {
                const bool ok = bfs_plain(st, out_rp, out_col, in_rp, in_col, n, g.arcs, samples_int.data(), k, Dt,
                                          dk, ts, trav_scratch, flags, cnt, L.cnt_host, &ds);
                rc = ok ? 0 : 3;
                if (ok) transpose_dist(st, Dt, Dd, n, k, dk);
                lmax_dir[dir] = (int32_t)ds.maxd;
            } else {
                const BfsView gv = make_view(dir);
                for (int32_t s0 = 0; s0 < k && rc == 0; s0 += 256) {
                    const int32_t kg = std::min(256, k - s0);
                    int32_t lm = 0;
                    BfsLevels lv;
                    lv.snap = (rt_single && dir == 1) ? snap_r : snap;
                    lv.cap = cap;
                    lv.fill_level = (rt_single && dir == 1) ? fill_level_r : fill_level;
                    lv.hist = hist;
                    lv.hlen = cap;
                    lv.lmax = &lm;
                    lv.hint = gr->bfs_hint.load(std::memory_order_relaxed);
                    if (bits_path || (rt_single && dir == 0)) {
                        // the job's setup in the first traversal's launches
                        lv.zero_flags = flags;
                        lv.sidx_fill = sidx;
                        lv.zero_hist = bits_path;
                        stage_into(lv);
                    }
                    rc = bfs_batched(st, gv, samples_dev, kg, s0, k, lv, sidx, ts, trav_scratch, cnt, &ds,
                                     L.no_alloc ? nullptr : &L.events);
                    if (rc == 0) gr->bfs_hint.store(ds.bfs_levels, std::memory_order_relaxed);
                    if (rc != 0) break;
                    lmax_dir[dir] = std::max(lmax_dir[dir], lm);
                    levels_dir[dir] = std::max(levels_dir[dir], ds.bfs_levels);
                    if (!bits_path) {
                        if ((int64_t)lm > DistT<uint8_t>::max_level && dk == DistKind::U8) { rc = 3; break; }
                        if ((int64_t)lm > DistT<uint16_t>::max_level && dk == DistKind::U16) { rc = 3; break; }
                        if (rt_single) {
                            // both searches first, then the distances from both directions' masks
                            if (dir == 1) rt_summed = materialize_rt(lmax_dir[0], lm);
                        } else {
                            materialize_distances(st, snap, (size_t)n * ((kg + 63) / 64), lm, fill_level, n, kg, s0,
                                                  k, Dd, dk, flags, false);
                        }
                    }
                }
            }
            add_stats(stats, ds);
        }
        if (rc == 1) {  // more levels than the mask buffer holds
            cap = (int32_t)std::min<int64_t>((int64_t)cap * 4, n + 2);
            const size_t masks = (size_t)cap * n * Wg * 8 * (rt_single ? 2 : 1);
            if (L.no_alloc && masks > L.arenaD.size)  // the fixed buffers cannot hold the masks
                throw FixedScratchFull{masks, L.arenaD.size};
            if (masks > mask_budget()) mode = CC_PLAIN;
            continue;
        }
        if (rc == 3) {  // distance type too narrow
            if (dk == DistKind::U8) dk = DistKind::U16;
            else if (dk == DistKind::U16) dk = DistKind::U32;
            else return fail(CC_EOVERFLOW, "a distance does not fit in 32 bits");
            continue;
        }
        CCG_HIP(hipEventRecord(L.ev[1], st));
        DevFlags hf;
        CCG_HIP(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        if (rc == 2 || hf.disconnected) return fail(CC_EDISCONNECTED, "some node is unreachable from some sample");
        if (hf.timeout) return fail(CC_EDEVICE, "traversal wait expired");

        // ---- epilogue
        BitsEpilogueArgs ba;
        void* ba_scratch = nullptr;
        size_t ba_es = 0;
        EpilogueArgs ea;
        void* ea_scratch = nullptr;
        size_t ea_es = 0;
        if (bits_path) {
            ba.n = n;
            ba.k = k;
            ba.snap = snap;
            ba.plane = (size_t)n * Wg;
            ba.lmax = lmax_dir[0];
            ba.fill_level = fill_level;
            ba.samples = samples_dev;
            ba.sidx = sidx;
            ba.orig = g.orig;
            ba.inv = g.inv;
            ba.hist = hist;
            ba.hist_slots = kHistSlotsBatched;
            ba.hist_len = cap;
            ba.eps_num = r.en;
            ba.eps_den = r.ed;
            ba.S_hyb = out->S_hyb;
            ba.S_samp = out->S_samp;
            ba.S_piv = out->S_piv;
            ba.S_pub = out->S_pub;
            ba.pivot = out->pivot;
            ba.delta = out->delta;
            ba.sampsum = out->sampsum;
            ba.src_sum = src_sum;
            ba.dmat = dmat;
            ba.Dout = out->D;
            ba.S_err = out->S_err;
            ba.S_ad = out->S_ad;
            ba.S_ad_err = out->S_ad_err;
            ba.S_sweep = out->S_sweep;
            ba.S_sweep_err = out->S_sweep_err;
            const bool want_err = out->S_err || out->S_ad || out->S_ad_err || out->S_sweep || out->S_sweep_err;
            const bool staged = out->S_hyb || out->S_samp || out->S_piv || out->S_pub || out->pivot || out->delta ||
                                out->sampsum;
            ba_es = bits_epilogue_scratch(k, ba.lmax, want_err ? n : 0, want_err, staged ? n : 0);
            // the traversal's scratch is free now, up to its control block,
            // which a replay of this estimate reads back afterwards
            const size_t ts_free = (size_t)((char*)bfs_batched_ctl(ts, n, kg0) - (char*)ts);
            ba_scratch = ba_es <= ts_free ? ts : L.arena2.get(ba_es);
            run_bits_epilogue(st, ba, ba_scratch, ba_es, flags);
            L.last_maxd = ba.lmax;
        } else {
            ea.n = n;
            ea.k = k;
            ea.dk = dk;
            ea.D = D;
            ea.Dr = rt_summed ? nullptr : Dr;
            ea.samples = samples_dev;
            ea.sidx = sidx;
            ea.orig = g.orig;
            // relabelled graphs: the row estimate walks the nodes in the caller's order
            ea.inv = (g.weighted || gr->borrowed) ? nullptr : g.inv;
            ea.maxd = (int64_t)lmax_dir[0] + lmax_dir[1];
            ea.eps_num = r.en;
            ea.eps_den = r.ed;
            fill_epilogue_outputs(ea, out, src_sum, dmat);
            ea_es = epilogue_scratch(n, k, ea.maxd, false,
                                     out->S_err || out->S_ad || out->S_ad_err || out->S_sweep || out->S_sweep_err);
            // a round trip that may be replayed keeps the traversal's control block
            // intact: a replay reads it back after the epilogue
            const size_t ts_free =
                rt_single ? (size_t)((char*)bfs_batched_ctl(ts, n, kg0) - (char*)ts) : trav_scratch;
            ea_scratch = ea_es <= ts_free ? ts : L.arena2.get(ea_es);
            run_epilogue(st, ea, ea_scratch, ea_es, flags);
            L.last_maxd = ea.maxd;
        }
        if (out->samples && !stage_samples)
            CCG_HIP(hipMemcpyAsync(out->samples, r.samples.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
        CCG_HIP(hipEventRecord(L.ev[2], st));
        CCG_HIP(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        record_timing(timing, L, stats, bits_path ? 0 : (int)dk);
        if (timing) timing->levels = stats.levels;
        const cc_status fs = finish_flags(hf);
        if (want_graph && fs == CC_OK && (stats.bfs_levels > 0 || w_single)) {
            // capture the same estimate (exactly the levels this search ran,
            // the epilogue for its deepest level) for replay; nothing runs now
            Lane::Captured cap_e;
            cap_e.key = graph_key();
            cap_e.lmax = bits_path ? ba.lmax : lmax_dir[1];
            cap_e.levels = bits_path ? stats.bfs_levels : levels_dir[1];
            if (rt_single) {
                cap_e.lmax_fwd = lmax_dir[0];
                cap_e.levels_fwd = levels_dir[0];
            }
            if (w_single) {
                cap_e.weighted = true;
                cap_e.lmax = g.directed ? lmax_dir[1] : lmax_dir[0];
                cap_e.lmax_fwd = g.directed ? lmax_dir[0] : -1;
                cap_e.levels = 0;
            }
            hipGraph_t graph = nullptr;
            // the round trip's second stream, created outside the capture; without it, no replay
            bool side_ok = true;
            if (rt_single) try {
                L.ensure_side();
            } catch (const HipError&) {
                side_ok = false;
                (void)hipGetLastError();
            }
            const bool began = side_ok && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
            bool captured_ok = began;
            if (began && w_single) try {
                // the weighted searches (one launch per direction), their distances and the D-based epilogue
                fill_u32(st, flags, 0u, sizeof(DevFlags) / 4);
                hipLaunchKernelGGL(k_stage_samples, dim3(1), dim3(256), 0, st, (const int32_t*)L.rb_dev->ids,
                                   (const int32_t*)L.rb_dev->caller, k, samples_dev, out->samples);
                compute_sidx(st, samples_dev, k, sidx, n);
                for (int dir = 0; dir < (g.directed ? 2 : 1); dir++) {
                    sssp_weighted_batched_enqueue(st, dir == 0 ? g.rp : g.rrp, dir == 0 ? g.cw : g.rcw, n, samples_dev,
                                                  k, (uint32_t*)Dt, (uint32_t)std::max(1, gr->tune.delta), ts,
                                                  trav_scratch, flags, wmaxd_dev + dir);
                    transpose_dist(st, Dt, dir == 0 ? D : Dr, n, k, dk);
                }
                run_epilogue(st, ea, ea_scratch, ea_es, flags);
                hipLaunchKernelGGL(k_wstatus_out, dim3(1), dim3(64), 0, st, (const uint32_t*)flags,
                                   (const uint32_t*)wmaxd_dev, (uint32_t*)&L.rb_dev->flags, L.rb_dev->wmaxd);
                CCG_HIP(hipGetLastError());
            } catch (const HipError&) {
                captured_ok = false;
            }
            else if (began && rt_single) try {
                // the round trip: the job's setup, then the forward search on the lane's
                // stream and the reverse one on the side stream (parallel branches of the
                // graph, each with its own traversal state), joined for the distances
                fill_u32(st, flags, 0u, sizeof(DevFlags) / 4);
                hipLaunchKernelGGL(k_stage_samples, dim3(1), dim3(256), 0, st, (const int32_t*)L.rb_dev->ids,
                                   (const int32_t*)L.rb_dev->caller, k, samples_dev, out->samples);
                compute_sidx(st, samples_dev, k, sidx, n);
                CCG_HIP(hipEventRecord(L.fork_ev, st));
                CCG_HIP(hipStreamWaitEvent(L.side, L.fork_ev, 0));
                for (int dir = 0; dir < 2; dir++) {
                    int32_t lm = 0;
                    BfsLevels lv;
                    lv.snap = dir == 0 ? snap : snap_r;
                    lv.cap = cap;
                    lv.fill_level = dir == 0 ? fill_level : fill_level_r;
                    lv.hlen = cap;
                    lv.lmax = &lm;
                    lv.enqueue_only = levels_dir[dir];
                    TravStats ignored;
                    (void)bfs_batched(dir == 0 ? st : L.side, make_view(dir), samples_dev, k, 0, k, lv, sidx,
                                      dir == 0 ? ts : ts_r, trav_scratch, dir == 0 ? cnt : cnt_r, &ignored, nullptr);
                }
                // the forward search's control block
                hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st,
                                   (const uint32_t*)bfs_batched_ctl(ts, n, kg0), (const uint32_t*)flags,
                                   (uint32_t*)&L.rb_dev->ctl_fwd, (uint32_t*)&L.rb_dev->flags_fwd);
                CCG_HIP(hipEventRecord(L.join_ev, L.side));
                CCG_HIP(hipStreamWaitEvent(st, L.join_ev, 0));
                (void)materialize_rt(lmax_dir[0], lmax_dir[1]);  // the same choice as the eager run
                run_epilogue(st, ea, ea_scratch, ea_es, flags);
                hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st,
                                   (const uint32_t*)bfs_batched_ctl(ts_r, n, kg0), (const uint32_t*)flags,
                                   (uint32_t*)&L.rb_dev->ctl, (uint32_t*)&L.rb_dev->flags);
                CCG_HIP(hipGetLastError());
            } catch (const HipError&) {
                captured_ok = false;
                // rejoin the side stream so that the capture can be ended (a join already made adds nothing)
                if (hipEventRecord(L.join_ev, L.side) == hipSuccess) (void)hipStreamWaitEvent(st, L.join_ev, 0);
            }
            else if (began) try {
                const uint32_t* ctl_dev = (const uint32_t*)bfs_batched_ctl(ts, n, kg0);
                for (int dir = 0; dir < (rt_single ? 2 : 1); dir++) {
                    int32_t lm = 0;
                    BfsLevels lv;
                    lv.snap = (rt_single && dir == 1) ? snap_r : snap;
                    lv.cap = cap;
                    lv.fill_level = (rt_single && dir == 1) ? fill_level_r : fill_level;
                    lv.hist = hist;
                    lv.hlen = cap;
                    lv.lmax = &lm;
                    lv.enqueue_only = bits_path ? stats.bfs_levels : levels_dir[dir];
                    if (dir == 0) {
                        lv.zero_flags = flags;
                        lv.sidx_fill = sidx;
                        lv.zero_hist = bits_path;
                        stage_into(lv);
                    }
                    TravStats ignored;
                    (void)bfs_batched(st, make_view(dir), samples_dev, k, 0, k, lv, sidx, ts, trav_scratch, cnt,
                                      &ignored, nullptr);
                    if (rt_single) {
                        if (dir == 0)  // the forward search's control block, before the reverse one reuses it
                            hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st, ctl_dev,
                                               (const uint32_t*)flags, (uint32_t*)&L.rb_dev->ctl_fwd,
                                               (uint32_t*)&L.rb_dev->flags_fwd);
                        else  // the same choice as the eager run (replays check that the depths agree)
                            (void)materialize_rt(lmax_dir[0], lmax_dir[1]);
                    }
                }
                if (bits_path) run_bits_epilogue(st, ba, ba_scratch, ba_es, flags);
                else run_epilogue(st, ea, ea_scratch, ea_es, flags);
                hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st, ctl_dev, (const uint32_t*)flags,
                                   (uint32_t*)&L.rb_dev->ctl, (uint32_t*)&L.rb_dev->flags);
                CCG_HIP(hipGetLastError());
            } catch (const HipError&) {
                captured_ok = false;
            }
            // a stream that cannot be captured only means no replay later
            if (began) {
                const hipError_t ee = hipStreamEndCapture(st, &graph);  // always close a begun capture
                captured_ok = captured_ok && ee == hipSuccess && graph != nullptr;
            }
            hipGraphExec_t exec = nullptr;
            hipError_t ie = hipErrorUnknown;
            if (captured_ok) ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (ie == hipSuccess) {
                if (Lane::Captured* old_e = L.find_captured(cap_e.key)) {  // a deeper search replaced it
                    (void)hipGraphExecDestroy(old_e->exec);
                    L.captured.pop_back();
                }
                cap_e.exec = exec;
                L.add_captured(std::move(cap_e));
            }
        }
        return fs;
    }
    return fail(CC_EDEVICE, "traversal did not settle after repeated resizing");
}

cc_status guarded(cc_context* ctx, const std::function<cc_status()>& fn) {
    try {
        CCG_HIP(hipSetDevice(ctx->device));
        return fn();
    } catch (const std::bad_alloc&) {
        return fail(CC_ENOMEM, "device allocation failed");
    } catch (const HipError& e) {
        if (e.err == hipErrorOutOfMemory) return fail(CC_ENOMEM, e.where);
        if (e.err == hipErrorNotSupported) return fail(CC_EINVAL, e.where);
        return fail(CC_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
    }
}

}  // namespace

extern "C" cc_status cc_estimate_device(cc_context* ctx, const cc_graph* g, const cc_params* p, cc_result* out,
                                        void* hip_stream) {
    if (!ctx || !g || !p || !out) return fail(CC_EINVAL, "cc_estimate_device: null argument");
    Resolved r;
    cc_status s = resolve_params(g, p, r);
    if (s != CC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        Lane* L = &ctx->lane;
        hipStream_t saved = L->stream;
        if (hip_stream) L->stream = (hipStream_t)hip_stream;
        cc_timing t{};
        cc_status st;
        try {
            st = run_job(ctx, g, r, out, *L, &t);
        } catch (...) {
            L->stream = saved;
            throw;
        }
        L->stream = saved;
        if (st == CC_OK) ctx->last = t;
        return st;
    });
}

extern "C" cc_status cc_estimate_device_noalloc(cc_context* ctx, const cc_graph* g, const cc_params* p,
                                                cc_result* out, void* hip_stream) {
    if (!ctx || !g || !p || !out) return fail(CC_EINVAL, "cc_estimate_device_noalloc: null argument");
    if (!ctx->fixed_ready) return fail(CC_EDEVICE, "cc_estimate_device_noalloc: no static scratch on this device");
    if (g->dg.directed || g->dg.weighted || p->mode != CC_BATCHED || p->k > 256)
        return fail(CC_EINVAL, "cc_estimate_device_noalloc: undirected graphs without arc lengths, CC_BATCHED, "
                               "k <= 256 only");
    Resolved r;
    cc_status s = resolve_params(g, p, r);
    if (s != CC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> use(scratch_user_lock(ctx->device));  // one user of the device's array at a time
    return guarded(ctx, [&]() -> cc_status {
        Lane* L = &ctx->fixed_lane;
        hipStream_t saved = L->stream;
        if (hip_stream) L->stream = (hipStream_t)hip_stream;
        cc_timing t{};
        cc_status st;
        try {
            st = run_job(ctx, g, r, out, *L, &t);
        } catch (const FixedScratchFull& e) {
            L->stream = saved;
            (void)hipStreamSynchronize(L->stream);
            return fail(CC_ENOMEM, "cc_estimate_device_noalloc: the estimate needs " + std::to_string(e.need) +
                                       " bytes of one scratch part of " + std::to_string(e.have) + " (static scratch " +
                                       std::to_string(kNoAllocBytes >> 20) + " MiB)");
        } catch (...) {
            L->stream = saved;
            throw;
        }
        L->stream = saved;
        if (st == CC_OK) ctx->last = t;
        return st;
    });
}

namespace {

// Staging for host outputs: the requested fields laid out in the lane's
// persistent device buffer (arenaO, grown only when a larger job comes), the
// results copied into the lane's pinned host buffer, then into the caller's
// arrays, so a served job allocates and frees nothing once its lane has held
// a job as large.
struct Staging {
    struct F {
        void* h;
        size_t bytes;
        size_t off;
        void* d;
    };
    std::vector<F> fields;
    cc_result dev{};
    size_t total = 0;
    void plan(const cc_result* host, int64_t n, int32_t k) {
        auto add = [&](void* h, size_t bytes) {
            if (h) {
                fields.push_back({h, bytes, total, nullptr});
                total += Carver::sz(bytes);
            }
        };
        add(host->S_hyb, sizeof(double) * n);
        add(host->S_samp, sizeof(double) * n);
        add(host->S_piv, sizeof(int64_t) * n);
        add(host->S_pub, sizeof(int64_t) * n);
        add(host->pivot, sizeof(int32_t) * n);
        add(host->delta, sizeof(int32_t) * n);
        add(host->sampsum, sizeof(int64_t) * n);
        add(host->src_sum, sizeof(int64_t) * k);
        add(host->samples, sizeof(int32_t) * k);
        add(host->dmat, sizeof(int32_t) * (size_t)k * k);
        add(host->D, sizeof(int32_t) * (size_t)n * k);
        add(host->S_err, sizeof(double) * n);
        add(host->S_ad, sizeof(double) * n);
        add(host->S_ad_err, sizeof(double) * n);
        add(host->S_sweep, sizeof(double) * n);
        add(host->S_sweep_err, sizeof(double) * n);
    }
    // the fields at dbase + their offsets (device)
    void place(const cc_result* host, char* dbase) {
        for (auto& f : fields) f.d = dbase + f.off;
        auto dptr = [&](void* h) -> void* {
            for (auto& f : fields)
                if (f.h == h) return f.d;
            return nullptr;
        };
        dev.S_hyb = (double*)dptr(host->S_hyb);
        dev.S_samp = (double*)dptr(host->S_samp);
        dev.S_piv = (int64_t*)dptr(host->S_piv);
        dev.S_pub = (int64_t*)dptr(host->S_pub);
        dev.pivot = (int32_t*)dptr(host->pivot);
        dev.delta = (int32_t*)dptr(host->delta);
        dev.sampsum = (int64_t*)dptr(host->sampsum);
        dev.src_sum = (int64_t*)dptr(host->src_sum);
        dev.samples = (int32_t*)dptr(host->samples);
        dev.dmat = (int32_t*)dptr(host->dmat);
        dev.D = (int32_t*)dptr(host->D);
        dev.S_err = (double*)dptr(host->S_err);
        dev.S_ad = (double*)dptr(host->S_ad);
        dev.S_ad_err = (double*)dptr(host->S_ad_err);
        dev.S_sweep = (double*)dptr(host->S_sweep);
        dev.S_sweep_err = (double*)dptr(host->S_sweep_err);
    }
    void to_pinned(hipStream_t st, char* pbase) const {
        for (const auto& f : fields)
            CCG_HIP(hipMemcpyAsync(pbase + f.off, f.d, f.bytes, hipMemcpyDeviceToHost, st));
    }
    void deliver(const char* pbase) const {
        for (const auto& f : fields) std::memcpy(f.h, pbase + f.off, f.bytes);
    }
};

cc_status estimate_to_host(cc_context* ctx, const cc_graph* g, const Resolved& r, const cc_result* host, Lane& L,
                           cc_timing* t) {
    Staging sg;
    sg.plan(host, g->dg.n, r.k);
    sg.place(host, sg.total ? (char*)L.arenaO.get(sg.total) : nullptr);
    cc_status s = run_job(ctx, g, r, &sg.dev, L, t);
    if (s == CC_OK && sg.total) {
        char* hp = L.pinned_host(sg.total);
        sg.to_pinned(L.stream, hp);
        CCG_HIP(hipStreamSynchronize(L.stream));
        sg.deliver(hp);
    }
    return s;
}

// ---------------------------------------------------------------- batches
// Several small graphs traversed as one: their CSRs are laid side by side
// (node ranges aligned to 64), each graph's samples take whole 64-bit words
// of one 256-sample traversal, and every node starts with the other graphs'
// bits set, so "full" keeps its meaning and the level kernels are unchanged.
// Each graph's estimator epilogue then reads its rows and words of the shared
// snapshots.  One launch per level serves every graph of the batch.

constexpr int64_t kBatchNodeLimit = 1 << 17;  // graphs at most this large are batched
constexpr int32_t kMaxOvertakes = 16;          // younger jobs that may pass a waiting oldest job
constexpr int32_t kBatchWords = 4;

bool batchable(const cc_graph* g, const Resolved& r) {
    return !g->borrowed && !g->dg.directed && !g->dg.weighted && r.mode == CC_BATCHED && r.k <= 192 && g->dg.n <= kBatchNodeLimit &&
           g->dg.arcs < ((int64_t)1 << 30);
}

__global__ void k_union_copy(const uint32_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n, int64_t npad,
                             int64_t arcs, int64_t node_off, int64_t arc_off, uint32_t* __restrict__ urp,
                             int32_t* __restrict__ ucol) {
    const int64_t m = npad > arcs ? npad : arcs;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < npad) urp[node_off + t] = (uint32_t)(arc_off + (t < n ? (int64_t)rp[t] : arcs));
        if (t < arcs) ucol[arc_off + t] = col[t] + (int32_t)node_off;
    }
}

struct BatchItem {
    const cc_graph* g = nullptr;
    const Resolved* r = nullptr;
    const cc_result* out = nullptr;  // device pointers
    int32_t words = 0, word_off = 0;
    int64_t node_off = 0, arc_off = 0, npad = 0;
};

// Assigns word offsets (jobs of two or more words on even words, so 16-byte
// row loads stay aligned); false if the jobs do not fit in one traversal.
bool pack_words(std::vector<BatchItem>& items) {
    std::vector<size_t> order(items.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return items[a].words > items[b].words; });
    int32_t next = 0;
    for (size_t i : order) {
        int32_t w = items[i].words;
        if (w >= 2 && (next & 1)) next++;
        if (next + w > kBatchWords) return false;
        items[i].word_off = next;
        next += w;
    }
    return true;
}

// Runs a batch into DEVICE outputs.  Any failure of the shared traversal
// (capacity, disconnection, overflow) is reported as a non-OK status and the
// caller reruns the jobs one by one, so every job gets its own status.
cc_status run_batch(cc_context* ctx, std::vector<BatchItem>& items, Lane& L, cc_timing* timing) {
    hipStream_t st = L.stream;
    int64_t n_u = 0, arcs_u = 0;
    for (auto& it : items) {
        it.words = (it.r->k + 63) / 64;
        it.node_off = n_u;
        it.npad = (it.g->dg.n + 63) / 64 * 64;
        n_u += it.npad;
        it.arc_off = arcs_u;
        arcs_u += it.g->dg.arcs;
    }
    if (!pack_words(items) || arcs_u >= ((int64_t)1 << 31)) return fail(CC_EINVAL, "batch does not fit");
    const int32_t ngroups = (int32_t)(n_u / 64);
    constexpr int W = kBatchWords;
    // group tables and chunk list, built on the host
    std::vector<uint8_t> ghub((size_t)ngroups, 0);
    std::vector<uint64_t> preset((size_t)ngroups * W, 0);
    std::vector<int32_t> gvalid((size_t)ngroups, 0);
    std::vector<int32_t> chunks;
    std::vector<int32_t> samples_u(64 * W, -1);
    std::vector<int32_t> local;  // each job's samples as its graph's internal ids
    for (auto& it : items) {
        const DevGraph& g = it.g->dg;
        uint64_t jm[W] = {0, 0, 0, 0};
        for (int32_t i = 0; i < it.r->k; i++) jm[it.word_off + i / 64] |= 1ull << (i % 64);
        const int32_t g0 = (int32_t)(it.node_off / 64);
        for (int32_t q = 0; q < (int32_t)(it.npad / 64); q++) {
            ghub[(size_t)(g0 + q)] = (int64_t)q * 64 < g.nh ? 1 : 0;
            gvalid[(size_t)(g0 + q)] = (int32_t)std::min<int64_t>(64, std::max<int64_t>(0, g.n - (int64_t)q * 64));
            for (int w = 0; w < W; w++) preset[(size_t)(g0 + q) * W + w] = ~jm[w];
        }
        const std::vector<int32_t>& ch = it.g->chunks_host;
        for (size_t c = 0; c + 2 < ch.size(); c += 3) {
            chunks.push_back(ch[c] + (int32_t)it.node_off);
            chunks.push_back(ch[c + 1] + (int32_t)it.arc_off);
            chunks.push_back(ch[c + 2] + (int32_t)it.arc_off);
        }
        for (int32_t i = 0; i < it.r->k; i++) {
            const int32_t u = it.g->inv[(size_t)it.r->samples[(size_t)i]];
            samples_u[(size_t)(64 * it.word_off + i)] = (int32_t)it.node_off + u;
            local.push_back(u);
        }
    }
    const int32_t n_chunks = (int32_t)(chunks.size() / 3);
    size_t free_b = 0, total_b = 0;
    CCG_HIP(hipMemGetInfo(&free_b, &total_b));
    int32_t cap = 32;
    for (int attempt = 0; attempt < 4; attempt++) {
        const size_t trav_scratch = bfs_batched_scratch(n_u, 64 * W, 0);
        const size_t hist_elems = (size_t)kHistSlotsBatched * 64 * W * cap;
        size_t small = Carver::sz(sizeof(uint32_t) * (n_u + 1)) + Carver::sz(sizeof(int32_t) * arcs_u) +
                       Carver::sz(ngroups) + Carver::sz(sizeof(uint64_t) * preset.size()) +
                       Carver::sz(sizeof(int32_t) * ngroups) * 2 + Carver::sz(sizeof(int32_t) * (chunks.size() + 3)) +
                       Carver::sz(sizeof(int32_t) * samples_u.size()) + Carver::sz(sizeof(int32_t) * local.size()) +
                       Carver::sz(sizeof(int32_t) * n_u) + Carver::sz(sizeof(DevFlags)) +
                       Carver::sz(sizeof(LevelCounters) * kCounterSlots) + Carver::sz(trav_scratch) +
                       Carver::sz(sizeof(int32_t) * hist_elems);
        for (auto& it : items)
            small += Carver::sz(sizeof(int64_t) * it.r->k) + Carver::sz(sizeof(int32_t) * (size_t)it.r->k * it.r->k);
        const size_t snap_bytes = Carver::sz((size_t)cap * n_u * W * 8);
        if (snap_bytes > free_b / 3) return fail(CC_ENOMEM, "batch level masks do not fit");
        Carver c(L.arena.get(small));
        uint32_t* urp = c.take<uint32_t>(n_u + 1);
        int32_t* ucol = c.take<int32_t>(arcs_u);
        uint8_t* d_ghub = c.take<uint8_t>(ngroups);
        uint64_t* d_preset = c.take<uint64_t>(preset.size());
        int32_t* d_gvalid = c.take<int32_t>(ngroups);
        int32_t* fill_level = c.take<int32_t>(ngroups);
        int32_t* d_chunks = c.take<int32_t>(chunks.size() + 3);
        int32_t* d_samples = c.take<int32_t>(samples_u.size());
        int32_t* d_local = c.take<int32_t>(local.size());
        int32_t* sidx = c.take<int32_t>(n_u);
        DevFlags* flags = c.take<DevFlags>(1);
        LevelCounters* cnt = c.take<LevelCounters>(kCounterSlots);
        void* ts = c.take<char>(trav_scratch);
        int32_t* hist = c.take<int32_t>(hist_elems);
        std::vector<int64_t*> src_sums;
        std::vector<int32_t*> dmats;
        for (auto& it : items) {
            src_sums.push_back(it.out->src_sum ? it.out->src_sum : c.take<int64_t>(it.r->k));
            dmats.push_back(it.out->dmat ? it.out->dmat : c.take<int32_t>((size_t)it.r->k * it.r->k));
        }
        Carver cd(L.arenaD.get(snap_bytes + 256));
        uint64_t* snap = cd.take<uint64_t>((size_t)cap * n_u * W);

        CCG_HIP(hipMemcpyAsync(d_ghub, ghub.data(), ghub.size(), hipMemcpyHostToDevice, st));
        CCG_HIP(hipMemcpyAsync(d_preset, preset.data(), sizeof(uint64_t) * preset.size(), hipMemcpyHostToDevice, st));
        CCG_HIP(hipMemcpyAsync(d_gvalid, gvalid.data(), sizeof(int32_t) * gvalid.size(), hipMemcpyHostToDevice, st));
        if (!chunks.empty())
            CCG_HIP(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(int32_t) * chunks.size(), hipMemcpyHostToDevice, st));
        CCG_HIP(hipMemcpyAsync(d_samples, samples_u.data(), sizeof(int32_t) * samples_u.size(), hipMemcpyHostToDevice,
                               st));
        CCG_HIP(hipMemcpyAsync(d_local, local.data(), sizeof(int32_t) * local.size(), hipMemcpyHostToDevice, st));
        CCG_HIP(hipEventRecord(L.ev[0], st));
        for (auto& it : items) {
            const DevGraph& g = it.g->dg;
            const int64_t m = std::max<int64_t>(it.npad, g.arcs);
            hipLaunchKernelGGL(k_union_copy, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 65536)), dim3(256), 0, st,
                               g.rp, g.col, g.n, it.npad, g.arcs, it.node_off, it.arc_off, urp, ucol);
        }
        fill_u32(st, urp + n_u, (uint32_t)arcs_u, 1);
        fill_u32(st, flags, 0u, sizeof(DevFlags) / 4);
        compute_sidx(st, d_samples, 64 * W, sidx, n_u);
        fill_u32(st, hist, 0u, hist_elems);

        BfsView gv;
        gv.n = n_u;
        gv.arcs = arcs_u;
        gv.rp = gv.out_rp = urp;
        gv.col = gv.out_col = ucol;
        gv.nh = 0;
        gv.hub_chunks = gv.push_chunks = n_chunks > 0 ? d_chunks : nullptr;
        gv.n_hub_chunks = gv.n_push_chunks = n_chunks;
        gv.ghub = d_ghub;
        gv.preset = d_preset;
        gv.gvalid = d_gvalid;
        int32_t lm = 0;
        BfsLevels lv;
        lv.snap = snap;
        lv.cap = cap;
        lv.fill_level = fill_level;
        lv.hist = hist;
        lv.hlen = cap;
        lv.lmax = &lm;
        lv.hint = 0;
        TravStats stats;
        const int rc = bfs_batched(st, gv, d_samples, 64 * W, 0, 64 * W, lv, sidx, ts, trav_scratch, cnt, &stats,
                                   &L.events);
        if (rc == 1) {
            cap = (int32_t)std::min<int64_t>((int64_t)cap * 4, n_u + 2);
            continue;
        }
        CCG_HIP(hipEventRecord(L.ev[1], st));
        if (rc != 0) return fail(CC_EDISCONNECTED, "a graph of the batch is not connected");
        size_t es = 0;
        for (auto& it : items) {
            const bool want_err =
                it.out->S_err || it.out->S_ad || it.out->S_ad_err || it.out->S_sweep || it.out->S_sweep_err;
            es = std::max(es, bits_epilogue_scratch(it.r->k, lm, want_err ? it.g->dg.n : 0, want_err));
        }
        void* escr = L.arena2.get(es);
        size_t loff = 0;
        for (size_t j = 0; j < items.size(); j++) {
            const BatchItem& it = items[j];
            const cc_result* out = it.out;
            BitsEpilogueArgs ba;
            ba.n = it.g->dg.n;
            ba.k = it.r->k;
            ba.snap = snap;
            ba.plane = (size_t)n_u * W;
            ba.lmax = lm;
            ba.fill_level = fill_level;
            ba.samples = d_local + loff;
            ba.sidx = sidx;
            ba.orig = it.g->dg.orig;
            ba.hist = hist;
            ba.hist_slots = kHistSlotsBatched;
            ba.hist_len = cap;
            ba.eps_num = it.r->en;
            ba.eps_den = it.r->ed;
            ba.S_hyb = out->S_hyb;
            ba.S_samp = out->S_samp;
            ba.S_piv = out->S_piv;
            ba.S_pub = out->S_pub;
            ba.pivot = out->pivot;
            ba.delta = out->delta;
            ba.sampsum = out->sampsum;
            ba.src_sum = src_sums[j];
            ba.dmat = dmats[j];
            ba.Dout = out->D;
            ba.S_err = out->S_err;
            ba.S_ad = out->S_ad;
            ba.S_ad_err = out->S_ad_err;
            ba.S_sweep = out->S_sweep;
            ba.S_sweep_err = out->S_sweep_err;
            ba.node_off = it.node_off;
            ba.word_off = it.word_off;
            ba.row_words = W;
            ba.bit_base = 64 * it.word_off;
            ba.hist_rows = 64 * W;
            run_bits_epilogue(st, ba, escr, es, flags);
            if (out->samples)
                CCG_HIP(hipMemcpyAsync(out->samples, it.r->samples.data(), sizeof(int32_t) * it.r->k,
                                       hipMemcpyHostToDevice, st));
            loff += (size_t)it.r->k;
        }
        CCG_HIP(hipEventRecord(L.ev[2], st));
        DevFlags hf;
        CCG_HIP(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        record_timing(timing, L, stats, 0);
        return finish_flags(hf);
    }
    return fail(CC_EDEVICE, "batch traversal did not settle");
}

// A batch with host outputs; on any failure of the shared run every job is
// rerun alone.  statuses[j] receives each job's result.
void batch_to_host(cc_context* ctx, const std::vector<const cc_graph*>& graphs, const std::vector<const Resolved*>& rs,
                   const std::vector<const cc_result*>& hosts, Lane& L, std::vector<cc_status>& statuses) {
    const size_t nj = graphs.size();
    statuses.assign(nj, CC_OK);
    bool ok = nj > 1;
    std::vector<Staging> stg(nj);
    std::vector<BatchItem> items(nj);
    size_t total = 0;
    for (size_t j = 0; j < nj; j++) {
        stg[j].plan(hosts[j], graphs[j]->dg.n, rs[j]->k);
        total += stg[j].total;
    }
    if (ok) {
        char* dbase = total ? (char*)L.arenaO.get(total) : nullptr;
        size_t off = 0;
        for (size_t j = 0; j < nj; j++) {
            stg[j].place(hosts[j], dbase ? dbase + off : nullptr);
            off += stg[j].total;
            items[j].g = graphs[j];
            items[j].r = rs[j];
            items[j].out = &stg[j].dev;
        }
        cc_timing t{};
        ok = run_batch(ctx, items, L, &t) == CC_OK;
        if (ok) {
            char* hp = total ? L.pinned_host(total) : nullptr;
            off = 0;
            for (size_t j = 0; j < nj; j++) {
                if (stg[j].total) stg[j].to_pinned(L.stream, hp + off);
                off += stg[j].total;
            }
            CCG_HIP(hipStreamSynchronize(L.stream));
            off = 0;
            for (size_t j = 0; j < nj; j++) {
                if (stg[j].total) stg[j].deliver(hp + off);
                off += stg[j].total;
            }
            return;
        }
    }
    for (size_t j = 0; j < nj; j++) {
        cc_timing t{};
        statuses[j] = estimate_to_host(ctx, graphs[j], *rs[j], hosts[j], L, &t);
    }
}

}  // namespace

extern "C" cc_status cc_estimate(cc_context* ctx, const cc_graph* g, const cc_params* p, cc_result* out) {
    if (!ctx || !g || !p || !out) return fail(CC_EINVAL, "cc_estimate: null argument");
    Resolved r;
    cc_status s = resolve_params(g, p, r);
    if (s != CC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        cc_timing t{};
        cc_status st = estimate_to_host(ctx, g, r, out, ctx->lane, &t);
        if (st == CC_OK) ctx->last = t;
        return st;
    });
}

extern "C" cc_status cc_estimate_weighted(cc_context* ctx, const cc_graph* g, const cc_weighted_params* p,
                                          cc_weighted_result* out) {
    if (!ctx || !g || !p || !out || !p->beta) return fail(CC_EINVAL, "cc_estimate_weighted: null argument");
    const int64_t n = g->dg.n;
    if (p->k < 1) return fail(CC_EINVAL, "cc_estimate_weighted: need k >= 1");
    std::vector<int32_t> ids((size_t)p->k);
    std::vector<uint8_t> light((size_t)p->k);
    int64_t R = 0;
    int32_t m = 1, kk = 0;
    cc_status s = cc_draw_weighted(n, p->beta, p->k, p->seed, ids.data(), light.data(), &R, &m, &kk);
    if (s != CC_OK) return s;
    ids.resize((size_t)kk);
    light.resize((size_t)kk);
    cc_params pp{};
    pp.k = kk;
    pp.mode = p->mode;
    pp.seed = 0;
    pp.samples = ids.data();
    pp.eps_num = p->eps_num;
    pp.eps_den = p->eps_den;
    Resolved r;
    s = resolve_params(g, &pp, r);
    if (s != CC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        Lane& L = ctx->lane;
        hipStream_t st = L.stream;
        auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
        // device block: D, dmat, beta, sidx, samples, light, S, var, flags, small scratch
        const size_t bytes = al(sizeof(int32_t) * (size_t)n * kk) + al(sizeof(int32_t) * (size_t)kk * kk) +
                             al(sizeof(uint32_t) * n) + al(sizeof(int32_t) * n) + al(sizeof(int32_t) * kk) + al(kk) +
                             3 * al(sizeof(double) * n) + al(sizeof(DevFlags)) + 256;
        char* q = (char*)L.arenaW.get(bytes);
        auto take = [&](size_t b) {
            char* x = q;
            q += al(b);
            return (void*)x;
        };
        int32_t* D = (int32_t*)take(sizeof(int32_t) * (size_t)n * kk);
        int32_t* dmat = (int32_t*)take(sizeof(int32_t) * (size_t)kk * kk);
        uint32_t* beta_d = (uint32_t*)take(sizeof(uint32_t) * n);
        int32_t* sidx = (int32_t*)take(sizeof(int32_t) * n);
        int32_t* samples_d = (int32_t*)take(sizeof(int32_t) * kk);
        uint8_t* light_d = (uint8_t*)take(kk);
        double* S = (double*)take(sizeof(double) * n);
        double* var = (double*)take(sizeof(double) * n);
        double* err = (double*)take(sizeof(double) * n);
        DevFlags* flags = (DevFlags*)take(sizeof(DevFlags));
        void* small = take(256);
        // the traversal and distance rows of cc_estimate, from this sample
        cc_result res{};
        res.D = D;
        res.dmat = dmat;
        cc_timing t{};
        L.last_maxd = -1;
        const cc_status js = run_job(ctx, g, r, &res, L, &t);
        if (js != CC_OK) return js;
        CCG_HIP(hipMemcpyAsync(beta_d, p->beta, sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
        CCG_HIP(hipMemcpyAsync(samples_d, ids.data(), sizeof(int32_t) * kk, hipMemcpyHostToDevice, st));
        CCG_HIP(hipMemcpyAsync(light_d, light.data(), (size_t)kk, hipMemcpyHostToDevice, st));
        compute_sidx(st, samples_d, kk, sidx, n);
        fill_u32(st, flags, 0u, sizeof(DevFlags) / 4);
        BetaArgs ba;
        ba.n = n;
        ba.k = kk;
        ba.D = D;
        ba.dmat = dmat;
        ba.sidx = sidx;
        ba.samples = samples_d;
        ba.beta = beta_d;
        ba.light = light_d;
        ba.R = R;
        ba.m = m;
        ba.eps_num = r.en;
        ba.eps_den = r.ed;
        ba.S = S;
        ba.var = var;
        ba.err = err;
        ba.small_scratch = small;
        ba.maxd = L.last_maxd;  // the traversal's bound on the distances, when it knows one
        ba.get_scratch = [&](size_t need) { return L.arena2.get(need); };
        run_beta_epilogue(st, ba, flags);
        DevFlags hf;
        CCG_HIP(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        if (out->S_beta) CCG_HIP(hipMemcpyAsync(out->S_beta, S, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        if (out->S_beta_var)
            CCG_HIP(hipMemcpyAsync(out->S_beta_var, var, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        if (out->S_beta_err)
            CCG_HIP(hipMemcpyAsync(out->S_beta_err, err, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        if (hf.overflow) return fail(CC_EOVERFLOW, "cc_estimate_weighted: a weighted sum leaves the exact range");
        const double tau = (double)R / (double)m;
        for (int32_t i = 0; i < p->k; i++) {
            if (out->samples) out->samples[i] = i < kk ? ids[(size_t)i] : -1;
            if (out->adjusted) out->adjusted[i] = i < kk ? (light[(size_t)i] ? tau : (double)p->beta[ids[(size_t)i]]) : 0.0;
        }
        if (out->tau) *out->tau = tau;
        if (out->sample_size) *out->sample_size = kk;
        t.epilogue_ms = 0;
        ctx->last = t;
        return CC_OK;
    });
}

// Scratch of a reachability run.  With arc lengths the searches take the
// propagation arcs as (end, length) pairs and run up to 256 sources per batch,
// fewer when a quarter of the free memory cannot hold their rows and piles.
static size_t reach_scratch_for(const cc_graph* g, ReachArgs& a, int32_t inbound, int32_t k_weighted) {
    if (!g->dg.weighted) return reach_scratch_bytes(a.n, a.arcs, k_weighted);
    a.cw = inbound ? g->dg.cw : g->dg.rcw;
    a.delta = (uint32_t)std::max(1, g->tune.delta);
    const size_t base = reach_len_scratch_bytes(a.n, 1, k_weighted);
    const size_t per = reach_len_scratch_bytes(a.n, 2, k_weighted) - base;
    size_t free_b = 0, total_b = 0;
    CCG_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t budget = free_b / 4;
    int32_t S = 256;
    while (S > 1 && base + per * (size_t)(S - 1) > budget) S /= 2;
    a.len_sources = S;
    return reach_len_scratch_bytes(a.n, S, k_weighted);
}

extern "C" cc_status cc_reach_weighted(cc_context* ctx, const cc_graph* g, const cc_reach_weighted_params* p,
                                       cc_reach_weighted_result* out) {
    if (!ctx || !g || !p || !out || !p->beta) return fail(CC_EINVAL, "cc_reach_weighted: null argument");
    const int64_t n = g->dg.n;
    if (p->k < 1 || p->k > 4096) return fail(CC_EINVAL, "cc_reach_weighted: need 1 <= k <= 4096");
    if (p->inbound != 0 && p->inbound != 1) return fail(CC_EINVAL, "cc_reach_weighted: inbound must be 0 or 1");
    // the nodes of positive weight are the sources; their priority ranks are
    // drawn and sorted on the device
    int64_t m = 0;
    for (int64_t u = 0; u < n; u++) m += p->beta[u] > 0 ? 1 : 0;
    if (m == 0) return fail(CC_EINVAL, "cc_reach_weighted: no node of positive weight");
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        Lane& L = ctx->lane;
        hipStream_t st = L.stream;
        CCG_HIP(hipEventRecord(L.ev[0], st));
        auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
        const size_t outb = 2 * al(sizeof(int32_t) * (size_t)n) + 2 * al(sizeof(double) * (size_t)n) +
                            2 * al(sizeof(uint32_t) * (size_t)n) + al(sizeof(uint64_t) * (size_t)n) +
                            al(sizeof(int32_t) * (size_t)n) + al(priority_scratch_bytes(n)) + 1024;
        char* ob = (char*)L.arena2.get(outb);
        auto take = [&](size_t b) {
            char* x = ob;
            ob += al(b);
            return (void*)x;
        };
        ReachArgs a;
        a.n = n;
        a.arcs = g->dg.arcs;
        a.k = p->k;
        a.rp = p->inbound ? g->dg.rp : g->dg.rrp;
        a.col = p->inbound ? g->dg.col : g->dg.rcol;
        a.nsrc = m;
        a.orig = g->dg.orig;
        a.count = (int32_t*)take(sizeof(int32_t) * n);
        a.kth = (int32_t*)take(sizeof(int32_t) * n);
        a.S_w = (double*)take(sizeof(double) * n);
        a.R = (double*)take(sizeof(double) * n);
        uint32_t* bc = (uint32_t*)take(sizeof(uint32_t) * n);  // caller's ids
        uint32_t* bd = (uint32_t*)take(sizeof(uint32_t) * n);  // internal ids
        uint64_t* Ud = (uint64_t*)take(sizeof(uint64_t) * n);
        int32_t* by_rank = (int32_t*)take(sizeof(int32_t) * n);
        void* ps = take(priority_scratch_bytes(n));
        CCG_HIP(hipMemcpyAsync(bc, p->beta, sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
        priority_order(st, n, m, p->seed, bc, g->dg.orig, bd, Ud, by_rank, ps, priority_scratch_bytes(n));
        a.order_dev = by_rank;
        a.beta = bd;
        a.U = Ud;
        const size_t need = reach_scratch_for(g, a, p->inbound, p->k);
        ReachStats rs;
        run_reach(st, a, L.arena.get(need), need, &rs);
        if (out->count) CCG_HIP(hipMemcpyAsync(out->count, a.count, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        if (out->kth) CCG_HIP(hipMemcpyAsync(out->kth, a.kth, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        if (out->S) CCG_HIP(hipMemcpyAsync(out->S, a.S_w, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        if (out->R) CCG_HIP(hipMemcpyAsync(out->R, a.R, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        CCG_HIP(hipEventRecord(L.ev[1], st));
        CCG_HIP(hipStreamSynchronize(st));
        if (rs.timeout) return fail(CC_EDEVICE, "cc_reach_weighted: a search did not finish within its time limit");
        if (rs.overflow)
            return fail(CC_EOVERFLOW, g->dg.weighted ? "cc_reach_weighted: a distance or weighted sum out of range"
                                                     : "cc_reach_weighted: a search deeper than 65535 levels");
        cc_timing t{};
        float ms = 0.f;
        CCG_HIP(hipEventElapsedTime(&ms, L.ev[0], L.ev[1]));
        t.total_ms = t.traverse_ms = ms;
        t.levels = rs.levels;
        t.launches = rs.cycles * (g->dg.weighted ? 2 : 3);
        t.arcs_scanned = rs.relaxed;
        ctx->last = t;
        return CC_OK;
    });
}

extern "C" cc_status cc_reach_estimate(cc_context* ctx, const cc_graph* g, const cc_reach_params* p,
                                       cc_reach_result* out) {
    if (!ctx || !g || !p || !out) return fail(CC_EINVAL, "cc_reach_estimate: null argument");
    const int64_t n = g->dg.n;
    if (p->k < 1) return fail(CC_EINVAL, "cc_reach_estimate: need k >= 1");
    if (p->inbound != 0 && p->inbound != 1) return fail(CC_EINVAL, "cc_reach_estimate: inbound must be 0 or 1");
    // rank order in internal ids
    std::vector<int32_t> order((size_t)n);
    if (p->order) {
        std::vector<char> hit((size_t)n, 0);
        for (int64_t r = 0; r < n; r++) {
            const int32_t u = p->order[r];
            if (u < 0 || u >= n || hit[(size_t)u]) return fail(CC_EINVAL, "cc_reach_estimate: order is not a permutation");
            hit[(size_t)u] = 1;
            order[(size_t)r] = u;
        }
    } else {
        // the same draws as cc_draw_samples(n, n, seed), on a dense array
        SplitMix64 rng{p->seed};
        for (int64_t i = 0; i < n; i++) order[(size_t)i] = (int32_t)i;
        shuffle(rng, order.data(), n);
    }
    for (int64_t r = 0; r < n; r++) {
        if (r + 16 < n) __builtin_prefetch(g->inv.data() + order[(size_t)(r + 16)]);
        order[(size_t)r] = g->inv[(size_t)order[(size_t)r]];
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        Lane& L = ctx->lane;
        hipStream_t st = L.stream;
        CCG_HIP(hipEventRecord(L.ev[0], st));
        // device outputs, then the traversal state
        const size_t outb = (sizeof(int32_t) + 4 * sizeof(int64_t)) * (size_t)n + 1024;
        char* ob = (char*)L.arena2.get(outb);
        ReachArgs a;
        a.n = n;
        a.arcs = g->dg.arcs;
        a.k = p->k;
        a.rp = p->inbound ? g->dg.rp : g->dg.rrp;
        a.col = p->inbound ? g->dg.col : g->dg.rcol;
        a.order = order.data();
        a.orig = g->dg.orig;
        a.count = (int32_t*)ob;
        a.distsum = (int64_t*)(ob + ((sizeof(int32_t) * (size_t)n + 255) & ~size_t(255)));
        a.T = a.distsum + n;
        a.B = (double*)(a.T + n);
        a.R = a.B + n;
        const size_t need = reach_scratch_for(g, a, p->inbound, 0);
        ReachStats rs;
        run_reach(st, a, L.arena.get(need), need, &rs);
        if (out->count) CCG_HIP(hipMemcpyAsync(out->count, a.count, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        if (out->distsum)
            CCG_HIP(hipMemcpyAsync(out->distsum, a.distsum, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
        if (out->T) CCG_HIP(hipMemcpyAsync(out->T, a.T, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
        if (out->B) CCG_HIP(hipMemcpyAsync(out->B, a.B, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        if (out->R) CCG_HIP(hipMemcpyAsync(out->R, a.R, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        CCG_HIP(hipEventRecord(L.ev[1], st));
        CCG_HIP(hipStreamSynchronize(st));
        if (rs.timeout) return fail(CC_EDEVICE, "cc_reach_estimate: a search did not finish within its time limit");
        if (rs.overflow)
            return fail(CC_EOVERFLOW, g->dg.weighted ? "cc_reach_estimate: a distance out of range"
                                                     : "cc_reach_estimate: a search deeper than 65535 levels");
        cc_timing t{};
        float ms = 0.f;
        CCG_HIP(hipEventElapsedTime(&ms, L.ev[0], L.ev[1]));
        t.total_ms = t.traverse_ms = ms;
        t.levels = rs.levels;
        t.launches = rs.cycles * (g->dg.weighted ? 2 : 3);
        t.arcs_scanned = rs.relaxed;
        ctx->last = t;
        return CC_OK;
    });
}

extern "C" cc_status cc_estimate_batch(cc_context* ctx, int32_t count, const cc_graph* const* graphs,
                                       const cc_params* params, cc_result* outs, cc_status* statuses) {
    if (!ctx || count < 1 || !graphs || !params || !outs) return fail(CC_EINVAL, "cc_estimate_batch: null argument");
    std::vector<Resolved> rs((size_t)count);
    std::vector<cc_status> st((size_t)count, CC_OK);
    for (int32_t j = 0; j < count; j++) {
        if (!graphs[j]) return fail(CC_EINVAL, "cc_estimate_batch: null graph");
        const cc_status s = resolve_params(graphs[j], &params[j], rs[(size_t)j]);
        if (s != CC_OK) return s;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    const cc_status overall = guarded(ctx, [&]() -> cc_status {
        // greedy packing in the given order: batchable jobs fill batches of at
        // most kBatchWords words; the others run alone
        std::vector<size_t> open;
        int32_t open_words = 0;
        auto flush = [&]() {
            if (open.empty()) return;
            std::vector<const cc_graph*> gs;
            std::vector<const Resolved*> rp;
            std::vector<const cc_result*> hs;
            for (size_t j : open) {
                gs.push_back(graphs[j]);
                rp.push_back(&rs[j]);
                hs.push_back(&outs[j]);
            }
            std::vector<cc_status> sts;
            batch_to_host(ctx, gs, rp, hs, ctx->lane, sts);
            for (size_t q = 0; q < open.size(); q++) st[open[q]] = sts[q];
            open.clear();
            open_words = 0;
        };
        for (int32_t j = 0; j < count; j++) {
            const Resolved& r = rs[(size_t)j];
            if (!batchable(graphs[j], r)) {
                cc_timing t{};
                st[(size_t)j] = estimate_to_host(ctx, graphs[j], r, &outs[j], ctx->lane, &t);
                continue;
            }
            const int32_t w = (r.k + 63) / 64;
            std::vector<BatchItem> trial;
            for (size_t q : open) {
                BatchItem it;
                it.words = (rs[q].k + 63) / 64;
                trial.push_back(it);
            }
            BatchItem me;
            me.words = w;
            trial.push_back(me);
            if (open_words + w > kBatchWords || !pack_words(trial)) flush();
            open.push_back((size_t)j);
            open_words += w;
        }
        flush();
        for (int32_t j = 0; j < count; j++)
            if (st[(size_t)j] != CC_OK) return st[(size_t)j];
        return CC_OK;
    });
    if (statuses)
        for (int32_t j = 0; j < count; j++) statuses[j] = st[(size_t)j];
    return overall;
}

extern "C" cc_status cc_last_timing(const cc_context* ctx, cc_timing* t) {
    if (!ctx || !t) return fail(CC_EINVAL, "cc_last_timing: null argument");
    *t = ctx->last;
    return CC_OK;
}

// ---------------------------------------------------------------- tuning

namespace {

cc_status check_tuning(const cc_tuning* t) {
    if (t->alpha < 1 || t->alpha > 1024) return fail(CC_EINVAL, "alpha must be in 1..1024");
    if (t->level_blocks < 1 || t->level_blocks > 65535) return fail(CC_EINVAL, "level_blocks must be in 1..65535");
    if (t->scatter_blocks < 1 || t->scatter_blocks > 65535) return fail(CC_EINVAL, "scatter_blocks must be in 1..65535");
    if (t->delta < 1) return fail(CC_EINVAL, "delta must be >= 1");
    if (t->round_blocks < 1 || t->round_blocks > 65535) return fail(CC_EINVAL, "round_blocks must be in 1..65535");
    if (t->local_passes < 0 || t->local_passes > 1024) return fail(CC_EINVAL, "local_passes must be in 0..1024");
    return CC_OK;
}

}  // namespace

extern "C" cc_status cc_graph_get_tuning(const cc_graph* g, cc_tuning* t) {
    if (!g || !t) return fail(CC_EINVAL, "cc_graph_get_tuning: null argument");
    *t = g->tune;
    return CC_OK;
}

extern "C" cc_status cc_graph_set_tuning(cc_graph* g, const cc_tuning* t) {
    if (!g || !t) return fail(CC_EINVAL, "cc_graph_set_tuning: null argument");
    const cc_status s = check_tuning(t);
    if (s != CC_OK) return s;
    g->tune = *t;
    return CC_OK;
}

extern "C" cc_status cc_autotune(cc_context* ctx, cc_graph* g, int32_t k, uint64_t seed, int32_t reps,
                                 cc_tuning* best, double* best_ms) {
    if (!ctx || !g) return fail(CC_EINVAL, "cc_autotune: null argument");
    if (reps < 1 || reps > 100) return fail(CC_EINVAL, "cc_autotune: reps must be in 1..100");
    cc_params p{};
    p.k = k;
    p.mode = CC_BATCHED;
    p.seed = seed;
    Resolved r;
    cc_status s = resolve_params(g, &p, r);
    if (s != CC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return guarded(ctx, [&]() -> cc_status {
        const int64_t n = g->dg.n;
        double* S = nullptr;
        if (hipMalloc((void**)&S, sizeof(double) * (size_t)n) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CC_ENOMEM, "cc_autotune: output allocation failed");
        }
        cc_result out{};
        out.S_hyb = S;
        const cc_tuning start = g->tune;
        // median device time of `reps` estimates with setting t (+inf on error)
        auto measure = [&](const cc_tuning& t) -> double {
            g->tune = t;
            std::vector<double> ms;
            for (int i = 0; i < reps; i++) {
                cc_timing tm{};
                if (run_job(ctx, g, r, &out, ctx->lane, &tm) != CC_OK) return HUGE_VAL;
                ms.push_back(tm.total_ms);
            }
            std::sort(ms.begin(), ms.end());
            return ms[ms.size() / 2];
        };
        cc_tuning cur = start;
        double cur_ms = HUGE_VAL;
        try {
            (void)measure(cur);  // warm the lane's buffers and the level hint
            cur_ms = measure(cur);
            auto try_knob = [&](int32_t cc_tuning::*field, const std::vector<int32_t>& cands) {
                for (int32_t v : cands) {
                    if (v == cur.*field) continue;
                    cc_tuning t = cur;
                    t.*field = v;
                    if (check_tuning(&t) != CC_OK) continue;
                    const double m = measure(t);
                    if (m < 0.95 * cur_ms) {  // keep the current setting unless clearly faster (timing noise)
                        cur_ms = m;
                        cur = t;
                    }
                }
            };
            if (g->dg.weighted) {
                const int32_t d0 = std::max(1, start.delta);
                std::vector<int32_t> ds;
                // the batched searches take the bucket width only (the round
                // shape knobs belong to the plain path's device-wide rounds)
                for (double f : {0.5, 1.5, 2.0, 3.0, 4.0, 8.0})
                    ds.push_back((int32_t)std::max<double>(1.0, std::llround(d0 * f)));
                try_knob(&cc_tuning::delta, ds);
            } else {
                try_knob(&cc_tuning::alpha, {1, 2, 8, 16, 32, 64});
                try_knob(&cc_tuning::scatter_blocks, {2048, 4096, 8192, 16384});
                try_knob(&cc_tuning::level_blocks, {512, 1024, 2048, 4096});
            }
        } catch (...) {
            g->tune = start;
            (void)hipFree(S);
            throw;
        }
        (void)hipFree(S);
        if (cur_ms == HUGE_VAL) {
            g->tune = start;
            return fail(CC_EDEVICE, "cc_autotune: no candidate ran");
        }
        g->tune = cur;
        if (best) *best = cur;
        if (best_ms) *best_ms = cur_ms;
        return CC_OK;
    });
}

// ---------------------------------------------------------------- serving

namespace {

double ms_between(std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

void finish_job(cc_context* ctx, cc_job* j, cc_status s, const std::string& err) {
    j->status = s;
    j->err = err;
    j->t_done = std::chrono::steady_clock::now();
    graph_unref(j->g);
    j->g = nullptr;
    {
        std::lock_guard<std::mutex> lk(j->m);
        j->state = 2;
    }
    j->cv.notify_all();
    if (j->refs.fetch_sub(1) == 1) delete j;
}

void worker_main(cc_context* ctx, Lane* L) {
    (void)hipSetDevice(ctx->device);
    auto resolved_of = [](const cc_job* j) {
        Resolved r;
        r.k = j->p.k;
        r.mode = j->p.mode & ~CC_GRAPH;
        r.graph = (j->p.mode & CC_GRAPH) != 0;
        r.en = j->p.eps_num;
        r.ed = j->p.eps_den;
        r.samples = j->samples;
        return r;
    };
    for (;;) {
        std::vector<cc_job*> js;
        {
            std::unique_lock<std::mutex> lk(ctx->qmu);
            for (;;) {
                if (ctx->stopping) return;
                // admit the oldest job that fits the memory budget (continuous
                // batching: a job that fits may overtake an older one that waits
                // for memory, but at most kMaxOvertakes times; after that the
                // oldest job goes next, as soon as memory frees up)
                auto it = ctx->queue.begin();
                const bool front_first = it != ctx->queue.end() && (*it)->overtaken >= kMaxOvertakes;
                for (; it != ctx->queue.end(); ++it) {
                    if (ctx->in_use + (int64_t)(*it)->need <= ctx->budget || ctx->inflight == 0) break;
                    if (front_first) {
                        it = ctx->queue.end();
                        break;
                    }
                }
                if (it != ctx->queue.end()) {
                    cc_job* j = *it;
                    if (it != ctx->queue.begin()) ctx->queue.front()->overtaken++;
                    ctx->queue.erase(it);
                    ctx->in_use += (int64_t)j->need;
                    ctx->inflight += 1;
                    js.push_back(j);
                    // small jobs waiting behind it join the same traversal
                    const Resolved r0 = resolved_of(j);
                    if (batchable(j->g, r0)) {
                        int32_t words = (r0.k + 63) / 64;
                        for (auto q = ctx->queue.begin(); q != ctx->queue.end() && words < kBatchWords && !front_first;) {
                            cc_job* o = *q;
                            const Resolved ro = resolved_of(o);
                            const int32_t w = (ro.k + 63) / 64;
                            bool fits = batchable(o->g, ro) && words + w <= kBatchWords &&
                                        ctx->in_use + (int64_t)o->need <= ctx->budget;
                            if (fits) {
                                std::vector<BatchItem> trial(js.size() + 1);
                                for (size_t t = 0; t < js.size(); t++) trial[t].words = (js[t]->p.k + 63) / 64;
                                trial.back().words = w;
                                fits = pack_words(trial);
                            }
                            if (fits) {
                                q = ctx->queue.erase(q);
                                ctx->in_use += (int64_t)o->need;
                                js.push_back(o);
                                words += w;
                            } else {
                                ++q;
                            }
                        }
                    }
                    break;
                }
                ctx->qcv.wait(lk);
            }
        }
        const auto now = std::chrono::steady_clock::now();
        for (cc_job* j : js) {
            j->state = 1;
            j->t_admit = now;
        }
        std::vector<Resolved> rs;
        for (cc_job* j : js) rs.push_back(resolved_of(j));
        std::vector<cc_status> sts(js.size(), CC_OK);
        std::vector<std::string> errs(js.size());
        try {
            if (js.size() == 1) {
                cc_timing t{};
                sts[0] = estimate_to_host(ctx, js[0]->g, rs[0], &js[0]->out, *L, &t);
                if (sts[0] != CC_OK) errs[0] = g_last_error;
            } else {
                std::vector<const cc_graph*> gs;
                std::vector<const Resolved*> rp;
                std::vector<const cc_result*> hs;
                for (size_t q = 0; q < js.size(); q++) {
                    gs.push_back(js[q]->g);
                    rp.push_back(&rs[q]);
                    hs.push_back(&js[q]->out);
                }
                batch_to_host(ctx, gs, rp, hs, *L, sts);
                for (size_t q = 0; q < js.size(); q++)
                    if (sts[q] != CC_OK) errs[q] = g_last_error;
            }
        } catch (const std::bad_alloc&) {
            for (size_t q = 0; q < js.size(); q++) {
                sts[q] = CC_ENOMEM;
                errs[q] = "device allocation failed";
            }
        } catch (const HipError& e) {
            for (size_t q = 0; q < js.size(); q++) {
                sts[q] = CC_EDEVICE;
                errs[q] = e.where + ": " + hipGetErrorString(e.err);
            }
        }
        // a lane keeps its buffers for the next job; beyond its share of the
        // budget it gives them back, so that retained memory cannot crowd out
        // jobs the budget admits
        const int slots = (int)ctx->worker_lanes.size();
        if (slots > 0 && (int64_t)L->retained() > ctx->budget / slots) {
            (void)hipStreamSynchronize(L->stream);
            L->trim();
        }
        {
            std::lock_guard<std::mutex> lk(ctx->qmu);
            for (cc_job* j : js) ctx->in_use -= (int64_t)j->need;
            ctx->inflight -= 1;
        }
        ctx->qcv.notify_all();
        for (size_t q = 0; q < js.size(); q++) finish_job(ctx, js[q], sts[q], errs[q]);
    }
}

void start_service(cc_context* ctx) {
    if (ctx->service_started) return;
    // one stream per slot; the default matches the device's hardware queues
    // per process (4), beyond which streams share queues and only add waiting
    const int slots = ctx->cfg.max_inflight > 0 ? ctx->cfg.max_inflight : 4;
    for (int i = 0; i < slots; i++) {
        auto L = std::make_unique<Lane>();
        L->init(nullptr);
        ctx->worker_lanes.push_back(std::move(L));
    }
    for (int i = 0; i < slots; i++) ctx->workers.emplace_back(worker_main, ctx, ctx->worker_lanes[(size_t)i].get());
    ctx->service_started = true;
}

}  // namespace

extern "C" cc_status cc_submit(cc_context* ctx, const cc_graph* g, const cc_params* p, const cc_result* out,
                               cc_job** job) {
    if (!ctx || !g || !p || !out || !job) return fail(CC_EINVAL, "cc_submit: null argument");
    Resolved r;
    cc_status s = resolve_params(g, p, r);
    if (s != CC_OK) return s;
    cc_job* j = new (std::nothrow) cc_job();
    if (!j) return fail(CC_ENOMEM, "cc_submit: host allocation");
    j->ctx = ctx;
    j->g = const_cast<cc_graph*>(g);
    j->g->refs.fetch_add(1);
    j->p = *p;
    j->p.eps_num = (int32_t)r.en;
    j->p.eps_den = (int32_t)r.ed;
    j->samples = r.samples;
    j->p.samples = nullptr;
    j->out = *out;
    j->need = job_bytes(g->dg, r.k, r.mode, g->dg.weighted ? 4 : 1);
    j->t_submit = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(ctx->qmu);
        try {
            CCG_HIP(hipSetDevice(ctx->device));
            start_service(ctx);
        } catch (const HipError& e) {
            graph_unref(j->g);
            delete j;
            return fail(CC_EDEVICE, "cc_submit: " + e.where);
        }
        ctx->queue.push_back(j);
    }
    ctx->qcv.notify_all();
    *job = j;
    return CC_OK;
}

extern "C" cc_status cc_poll(cc_job* j) {
    if (!j) return fail(CC_EINVAL, "cc_poll: null job");
    const int s = j->state.load();
    if (s == 2 || s == 3) return j->status;
    return CC_ENOTREADY;
}

extern "C" cc_status cc_wait(cc_job* j) {
    if (!j) return fail(CC_EINVAL, "cc_wait: null job");
    std::unique_lock<std::mutex> lk(j->m);
    j->cv.wait(lk, [&] { return j->state.load() >= 2; });
    if (j->status != CC_OK && !j->err.empty()) g_last_error = j->err;
    return j->status;
}

extern "C" cc_status cc_cancel(cc_job* j) {
    if (!j) return fail(CC_EINVAL, "cc_cancel: null job");
    cc_context* ctx = j->ctx;
    std::lock_guard<std::mutex> lk(ctx->qmu);
    auto it = std::find(ctx->queue.begin(), ctx->queue.end(), j);
    if (it == ctx->queue.end()) return fail(CC_EBUSY, "job already running or finished");
    ctx->queue.erase(it);
    j->status = CC_ECANCELLED;
    j->t_done = std::chrono::steady_clock::now();
    graph_unref(j->g);
    j->g = nullptr;
    {
        std::lock_guard<std::mutex> jl(j->m);
        j->state = 3;
    }
    j->cv.notify_all();
    if (j->refs.fetch_sub(1) == 1) delete j;
    return CC_OK;
}

extern "C" cc_status cc_job_times(const cc_job* j, double* queue_ms, double* total_ms) {
    if (!j) return fail(CC_EINVAL, "cc_job_times: null job");
    if (j->state.load() < 2) return CC_ENOTREADY;
    if (queue_ms) *queue_ms = j->state.load() == 3 ? ms_between(j->t_submit, j->t_done)
                                                  : ms_between(j->t_submit, j->t_admit);
    if (total_ms) *total_ms = ms_between(j->t_submit, j->t_done);
    return CC_OK;
}

extern "C" void cc_job_release(cc_job* j) {
    if (!j) return;
    if (j->refs.fetch_sub(1) == 1) delete j;
}
