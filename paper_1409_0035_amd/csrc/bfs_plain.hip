// Plain single-source breadth-first search, one sample after another: the
// one-source-at-a-time baseline.  Direction-optimising (Beamer, Asanovic &
// Patterson, SC 2012): top-down levels expand a frontier queue over out-arcs
// and claim unvisited targets with an atomic OR on a visited bitmap;
// bottom-up levels let every unvisited node look for a parent on the previous
// level over its in-arcs and stop at the first one.  Switching rule: go
// bottom-up when the frontier's arcs exceed the unexplored arcs / 14, go back
// top-down when the frontier holds fewer than n / 24 nodes.
//
// Output is source-major: Dt[i][v] = d(c_i, v); a tiled transpose produces the
// node-major matrix the estimator reads.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kSmallDeg = 32;
constexpr uint32_t kChunkArcs = 256;  // out-arcs per chunk of a high-degree frontier node

template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_init(int64_t n, DT* dist, uint32_t* vis) {
    int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < n) dist[v] = (DT)DistT<DT>::never;
    if (v < (n + 31) / 32) vis[v] = 0;
}

// The search's state between launches, so that the host enqueues levels
// without reading anything back: the frontier of the level that runs next
// (queue buffer, size, out-arcs), the arcs and nodes reached so far, the
// direction, and whether the search is over.
struct PlainCtl {
    int32_t done;
    int32_t pull;
    uint32_t level;     // the level the next push or pull finds
    int32_t qsel;       // frontier buffer of the next level
    int32_t nf;         // frontier size
    int32_t overflow;   // a level beyond what the distance type holds
    int64_t mf;         // the frontier's out-arcs
    int64_t explored;   // out-arcs of every node found so far
    int64_t visited;    // nodes found so far
    int64_t arcs;       // arcs scanned, this source
    int64_t nodes;      // frontier / unvisited nodes processed, this source
    int32_t nchunks;    // chunks of high-degree frontier nodes listed by this push level
    uint32_t ticket;    // blocks of the level's second launch that have finished
};
// What one source's search left: levels run, nodes found, whether it ended
// inside the levels enqueued for it, overflow.
struct PlainRec {
    int32_t done;
    int32_t overflow;
    uint32_t levels;
    int32_t pad;
    int64_t visited;
    int64_t arcs;
    int64_t nodes;
};

// push while the frontier's out-arcs are at most the unexplored arcs / 14, then
// pull until the frontier holds fewer than n / 24 nodes
__device__ __forceinline__ int32_t plain_direction(const PlainCtl& c, int64_t n, int64_t arcs) {
    const int64_t mu = arcs - c.explored;
    if (!c.pull && c.mf > mu / 14) return 1;
    if (c.pull && (int64_t)c.nf < n / 24) return 0;
    return c.pull;
}

template <typename DT>
__global__ void k_plain_source(int32_t s, DT* dist, uint32_t* vis, int32_t* q, const uint32_t* rp,
                               LevelCounters* cnt, PlainCtl* ctl, int64_t n, int64_t arcs) {
    if (threadIdx.x == 0) {
        dist[s] = 0;
        vis[s >> 5] |= 1u << (s & 31);
        q[0] = s;
        cnt->n_out = 0;
        cnt->n_new = 0;
        cnt->arcs = 0;
        cnt->frontier_arcs = 0;
        cnt->matched = 0;
        PlainCtl c{};
        c.level = 1;
        c.nf = 1;
        c.mf = rp[s + 1] - rp[s];
        c.explored = c.mf;
        c.visited = 1;
        c.pull = 0;
        c.pull = plain_direction(c, n, arcs);
        *ctl = c;
    }
}

template <typename DT>
__device__ __forceinline__ void claim(int32_t w, uint32_t* vis, DT* dist, uint32_t level, const uint32_t* rp,
                                      int32_t* q_out, LevelCounters* cnt, int64_t& farcs, int32_t& nnew) {
    const uint32_t bit = 1u << (w & 31);
    bool mine = false;
    if (!(__hip_atomic_load(&vis[w >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) {
        const uint32_t old = atomicOr(&vis[w >> 5], bit);
        mine = !(old & bit);
    }
    if (mine) {
        dist[w] = (DT)level;
        farcs += rp[w + 1] - rp[w];
        nnew += 1;
    }
    const int pos = wave_append(&cnt->n_out, mine);
    if (mine) q_out[pos] = w;
}

// One level, pushing or pulling as the control block says.
//   push  one lane per frontier node of low degree; a node of higher degree
//         is cut into chunks of kChunkArcs out-arcs, listed for the second
//         launch, where a wave takes each chunk (a hub no longer holds one
//         wave for its whole arc list)
//   pull  every unvisited node scans its in-arcs for a node of the last level
//         and stops at the first
template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_level(const uint32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const uint32_t* __restrict__ in_rp,
                                                        const int32_t* __restrict__ in_col, int64_t n, uint32_t* vis,
                                                        DT* dist, int32_t* q0, int32_t* q1, uint64_t* chunks,
                                                        PlainCtl* ctl, LevelCounters* cnt) {
    if (ctl->done) return;
    const uint32_t level = ctl->level;
    const int32_t* q_in = ctl->qsel ? q1 : q0;
    int32_t* q_out = ctl->qsel ? q0 : q1;
    const int lane = lane_id();
    int64_t farcs = 0, scanned = 0;
    int32_t nnew = 0;
    if (!ctl->pull) {
        const int32_t n_in = ctl->nf;
        for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n_in; base += (int64_t)gridDim.x * kBlock) {
            const int64_t idx = base + threadIdx.x;
            const bool valid = idx < n_in;
            const int32_t u = valid ? q_in[idx] : 0;
            uint32_t beg = 0, end = 0;
            if (valid) {
                beg = rp[u];
                end = rp[u + 1];
            }
            const bool big = valid && (end - beg > kSmallDeg);
            if (valid && !big) {
                for (uint32_t e = beg; e < end; ++e) {
                    ++scanned;
                    claim<DT>(col[e], vis, dist, level, rp, q_out, cnt, farcs, nnew);
                }
            }
            if (big) {  // its chunks, for the second launch
                const uint32_t c = (end - beg + kChunkArcs - 1) / kChunkArcs;
                const int32_t at = atomicAdd(&ctl->nchunks, (int32_t)c);
                for (uint32_t q = 0; q < c; q++) chunks[at + q] = ((uint64_t)(uint32_t)u << 32) | (q * kChunkArcs);
            }
        }
    } else {
        for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
            const int64_t v = base + threadIdx.x;
            bool found = false;
            int64_t fa = 0;
            if (v < n && !(vis[v >> 5] & (1u << (v & 31)))) {
                const DT want = (DT)(level - 1);
                const uint32_t b = in_rp[v], en = in_rp[v + 1];
                for (uint32_t e = b; e < en; ++e) {
                    ++scanned;
                    if (dist[in_col[e]] == want) {
                        found = true;
                        break;
                    }
                }
                if (found) {
                    dist[v] = (DT)level;
                    atomicOr(&vis[v >> 5], 1u << (v & 31));
                    fa = rp[v + 1] - rp[v];
                }
            }
            farcs += fa;
            nnew += found ? 1 : 0;
            const int pos = wave_append(&cnt->n_out, found);
            if (found) q_out[pos] = (int32_t)v;
        }
    }
    const int64_t fa = wave_sum64(farcs);
    const int64_t sc = wave_sum64(scanned);
    const int32_t nn = wave_sum32(nnew);
    if (lane == 0) {
        if (fa) atomicAdd((unsigned long long*)&cnt->frontier_arcs, (unsigned long long)fa);
        if (sc) atomicAdd((unsigned long long*)&cnt->arcs, (unsigned long long)sc);
        if (nn) atomicAdd(&cnt->n_new, nn);
    }
}

// The second launch of a level: the chunks of the high-degree frontier nodes
// (push levels), one wave per chunk; then the last block ends the level: the
// next frontier becomes current, the search ends when it is empty, and the
// next level's direction is decided.
template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_chunks_post(const uint32_t* __restrict__ rp,
                                                              const int32_t* __restrict__ col, int64_t n,
                                                              int64_t arcs, uint32_t* vis, DT* dist, int32_t* q0,
                                                              int32_t* q1, const uint64_t* __restrict__ chunks,
                                                              PlainCtl* ctl, LevelCounters* cnt, uint32_t max_level) {
    if (ctl->done) return;
    const int lane = lane_id();
    if (!ctl->pull) {
        const uint32_t level = ctl->level;
        int32_t* q_out = ctl->qsel ? q0 : q1;
        const int32_t nc = ctl->nchunks;
        int64_t farcs = 0, scanned = 0;
        int32_t nnew = 0;
        const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
        for (int64_t c = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); c < nc; c += waves) {
            const uint64_t ent = chunks[c];
            const int32_t u = (int32_t)(ent >> 32);
            const uint32_t b = rp[u] + (uint32_t)ent, en = min(rp[u + 1], b + kChunkArcs);
            for (uint32_t e0 = b; e0 < en; e0 += 64) {  // the same trip count in every lane
                const uint32_t e = e0 + lane;
                if (e < en) {
                    ++scanned;
                    claim<DT>(col[e], vis, dist, level, rp, q_out, cnt, farcs, nnew);
                }
            }
        }
        const int64_t fa = wave_sum64(farcs);
        const int64_t sc = wave_sum64(scanned);
        const int32_t nn = wave_sum32(nnew);
        if (lane == 0) {
            if (fa) atomicAdd((unsigned long long*)&cnt->frontier_arcs, (unsigned long long)fa);
            if (sc) atomicAdd((unsigned long long*)&cnt->arcs, (unsigned long long)sc);
            if (nn) atomicAdd(&cnt->n_new, nn);
        }
    }
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    PlainCtl c = *ctl;
    c.ticket = 0;
    c.nchunks = 0;
    c.nodes += c.pull ? n - c.visited : c.nf;
    c.arcs += cnt->arcs;
    c.nf = cnt->n_out;
    c.mf = cnt->frontier_arcs;
    c.explored += c.mf;
    c.visited += c.nf;
    cnt->n_out = 0;
    cnt->n_new = 0;
    cnt->arcs = 0;
    cnt->frontier_arcs = 0;
    if (c.nf == 0) {
        c.done = 1;
    } else {
        c.qsel ^= 1;
        c.level += 1;
        if (c.level > max_level) {
            c.overflow = 1;
            c.done = 1;
        } else {
            c.pull = plain_direction(c, n, arcs);
        }
    }
    *ctl = c;
    __threadfence();
}

__global__ void k_plain_record(const PlainCtl* ctl, PlainRec* rec) {
    if (threadIdx.x != 0) return;
    const PlainCtl c = *ctl;
    PlainRec r{};
    r.done = c.done;
    r.overflow = c.overflow;
    r.levels = c.level;
    r.visited = c.visited;
    r.arcs = c.arcs;
    r.nodes = c.nodes;
    *rec = r;
}

template <typename DT>
__global__ __launch_bounds__(256) void k_transpose(const DT* __restrict__ Dt, DT* __restrict__ D, int64_t n,
                                                   int32_t k) {
    __shared__ DT tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int32_t i0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int32_t i = i0 + r;
        const int64_t v = v0 + tx;
        if (i < k && v < n) tile[r][tx] = Dt[(int64_t)i * n + v];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t v = v0 + r;
        const int32_t i = i0 + tx;
        if (i < k && v < n) D[v * k + i] = tile[tx][r];
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// One source: its initialisation and `levels` levels (push, pull, post), the
// levels past its end returning at once, then its record.
template <typename DT>
void enqueue_source(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
                    const int32_t* in_col, int64_t n, int64_t arcs, int32_t s, DT* dist, uint32_t* vis, int32_t* q0,
                    int32_t* q1, uint64_t* chunks, PlainCtl* ctl, LevelCounters* cnt, PlainRec* rec,
                    uint32_t levels) {
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    const unsigned lb = std::min<unsigned>(nb, 4096), cb = std::min<unsigned>(nb, 2048);
    hipLaunchKernelGGL((k_plain_init<DT>), dim3(nb), dim3(kBlock), 0, st, n, dist, vis);
    hipLaunchKernelGGL((k_plain_source<DT>), dim3(1), dim3(64), 0, st, s, dist, vis, q0, out_rp, cnt, ctl, n, arcs);
    for (uint32_t l = 0; l < levels; l++) {
        hipLaunchKernelGGL((k_plain_level<DT>), dim3(lb), dim3(kBlock), 0, st, out_rp, out_col, in_rp, in_col, n, vis,
                           dist, q0, q1, chunks, ctl, cnt);
        hipLaunchKernelGGL((k_plain_chunks_post<DT>), dim3(cb), dim3(kBlock), 0, st, out_rp, out_col, n, arcs, vis,
                           dist, q0, q1, (const uint64_t*)chunks, ctl, cnt, (uint32_t)DistT<DT>::max_level);
    }
    hipLaunchKernelGGL(k_plain_record, dim3(1), dim3(64), 0, st, (const PlainCtl*)ctl, rec);
}

// The k searches one after another.  The host enqueues every source with as
// many levels as the deepest search so far needed (plus two), reads the
// sources' records once at the end, and runs again, with more levels, any
// source whose search had not ended.
template <typename DT>
int plain_t(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
            const int32_t* in_col, int64_t n, int64_t arcs, const int32_t* samples_host, int32_t k, DT* Dt,
            void* scratch, LevelCounters* cnt_dev, TravStats* stats) {
    char* p = (char*)scratch;
    uint32_t* vis = (uint32_t*)p;
    p += align256(sizeof(uint32_t) * ((n + 31) / 32));
    int32_t* q0 = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    int32_t* q1 = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    PlainCtl* ctl = (PlainCtl*)p;
    p += align256(sizeof(PlainCtl));
    uint64_t* chunks = (uint64_t*)p;
    p += align256(sizeof(uint64_t) * (size_t)(n + arcs / kChunkArcs + 1));
    PlainRec* rec = (PlainRec*)p;
    std::vector<PlainRec> hr((size_t)k);
    // the first source alone, to learn the depth; then all the others at once
    std::vector<int32_t> todo{0}, rest;
    for (int32_t i = 1; i < k; i++) rest.push_back(i);
    uint32_t levels = 16;
    KernelTimer kt;
    int rc = 0;
    while (!todo.empty() || !rest.empty()) {
        if (todo.empty()) todo.swap(rest);
        kt.start(st);
        for (int32_t i : todo)
            enqueue_source<DT>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host[i], Dt + (int64_t)i * n, vis,
                               q0, q1, chunks, ctl, cnt_dev, rec + i, levels);
        CCG_HIP(hipGetLastError());
        kt.stop(st);
        CCG_HIP(hipMemcpyAsync(hr.data(), rec, sizeof(PlainRec) * k, hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        stats->kernel_ms += kt.ms();
        stats->kernel_launches += (int64_t)todo.size() * (2 * levels + 3);
        stats->launches += (int64_t)todo.size() * (2 * levels + 3);
        std::vector<int32_t> again;
        uint32_t deepest = 0;
        for (int32_t i : todo) {
            const PlainRec& r = hr[(size_t)i];
            if (r.overflow) return 1;
            if (!r.done) {
                again.push_back(i);
                continue;
            }
            stats->levels += r.levels;
            stats->arcs_scanned += r.arcs;
            stats->nodes_visited += r.nodes;
            if ((int64_t)r.levels - 1 > stats->maxd) stats->maxd = r.levels - 1;
            deepest = std::max(deepest, r.levels);
            if (r.visited < n) rc = 2;
        }
        // the searches that had not ended run deeper; the others as deep as the deepest one so far, plus two
        levels = again.empty() ? std::max<uint32_t>(deepest + 2, 4) : std::max(levels * 4, deepest + 2);
        todo.swap(again);
        if ((int64_t)levels > (int64_t)DistT<DT>::max_level + 2) levels = (uint32_t)DistT<DT>::max_level + 2;
    }
    return rc;
}

}  // namespace

size_t bfs_plain_scratch(int64_t n, int64_t arcs, int32_t k) {
    return align256(sizeof(uint32_t) * ((n + 31) / 32)) + 2 * align256(sizeof(int32_t) * n) +
           align256(sizeof(PlainCtl)) + align256(sizeof(uint64_t) * (size_t)(n + arcs / kChunkArcs + 1)) +
           align256(sizeof(PlainRec) * (size_t)std::max(k, 1)) + 1024;
}

bool bfs_plain(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
               const int32_t* in_col, int64_t n, int64_t arcs, const int32_t* samples_host, int32_t k, void* Dt,
               DistKind dk, void* scratch, size_t scratch_size, DevFlags* flags, LevelCounters* cnt_dev,
               LevelCounters* cnt_host, TravStats* stats) {
    if (scratch_size < bfs_plain_scratch(n, arcs, k)) throw HipError{hipErrorOutOfMemory, "bfs_plain scratch"};
    int r;
    switch (dk) {
        case DistKind::U8:
            r = plain_t<uint8_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint8_t*)Dt, scratch,
                                 cnt_dev, stats);
            break;
        case DistKind::U16:
            r = plain_t<uint16_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint16_t*)Dt,
                                  scratch, cnt_dev, stats);
            break;
        default:
            r = plain_t<uint32_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint32_t*)Dt,
                                  scratch, cnt_dev, stats);
            break;
    }
    if (r == 1) return false;
    if (r == 2) {
        int32_t one = 1;
        CCG_HIP(hipMemcpyAsync(&flags->disconnected, &one, sizeof(one), hipMemcpyHostToDevice, st));
        CCG_HIP(hipStreamSynchronize(st));
    }
    return true;
}

void transpose_dist(hipStream_t st, const void* Dt, void* D, int64_t n, int32_t k, DistKind dk) {
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64));
    switch (dk) {
        case DistKind::U8:
            hipLaunchKernelGGL((k_transpose<uint8_t>), grid, dim3(256), 0, st, (const uint8_t*)Dt, (uint8_t*)D, n, k);
            break;
        case DistKind::U16:
            hipLaunchKernelGGL((k_transpose<uint16_t>), grid, dim3(256), 0, st, (const uint16_t*)Dt, (uint16_t*)D, n,
                               k);
            break;
        default:
            hipLaunchKernelGGL((k_transpose<uint32_t>), grid, dim3(256), 0, st, (const uint32_t*)Dt, (uint32_t*)D, n,
                               k);
            break;
    }
    CCG_HIP(hipGetLastError());
}

}  // namespace ccg
