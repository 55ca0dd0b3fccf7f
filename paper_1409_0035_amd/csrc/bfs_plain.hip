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

template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_init(int64_t n, DT* dist, uint32_t* vis) {
    int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v < n) dist[v] = (DT)DistT<DT>::never;
    if (v < (n + 31) / 32) vis[v] = 0;
}

template <typename DT>
__global__ void k_plain_source(int32_t s, DT* dist, uint32_t* vis, int32_t* q, const uint32_t* rp,
                               LevelCounters* cnt) {
    if (threadIdx.x == 0) {
        dist[s] = 0;
        vis[s >> 5] |= 1u << (s & 31);
        q[0] = s;
        cnt->n_out = 1;
        cnt->n_new = 1;
        cnt->frontier_arcs = rp[s + 1] - rp[s];
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

// top-down: one lane per low-degree frontier node, the whole wave per
// high-degree one
template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_push(const uint32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ q_in, int32_t n_in,
                                                       int32_t* __restrict__ q_out, uint32_t* vis, DT* dist,
                                                       uint32_t level, LevelCounters* cnt) {
    const int lane = lane_id();
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = idx < n_in;
    const int32_t u = valid ? q_in[idx] : 0;
    uint32_t beg = 0, end = 0;
    if (valid) {
        beg = rp[u];
        end = rp[u + 1];
    }
    const bool big = valid && (end - beg > kSmallDeg);
    int64_t farcs = 0, scanned = 0;
    int32_t nnew = 0;
    if (valid && !big) {
        for (uint32_t e = beg; e < end; ++e) {
            ++scanned;
            claim<DT>(col[e], vis, dist, level, rp, q_out, cnt, farcs, nnew);
        }
    }
    uint64_t bm = __ballot(big);
    while (bm) {
        const int s = __ffsll((unsigned long long)bm) - 1;
        bm &= bm - 1;
        const uint32_t b = (uint32_t)readlane32((int)beg, s);
        const uint32_t en = (uint32_t)readlane32((int)end, s);
        for (uint32_t e0 = b; e0 < en; e0 += 64) {
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

// bottom-up: every unvisited node scans its in-arcs for a node at level-1
template <typename DT>
__global__ __launch_bounds__(kBlock) void k_plain_pull(const uint32_t* __restrict__ in_rp,
                                                       const int32_t* __restrict__ in_col,
                                                       const uint32_t* __restrict__ out_rp, int64_t n,
                                                       uint32_t* vis, DT* dist, uint32_t level,
                                                       int32_t* __restrict__ q_out, LevelCounters* cnt) {
    const int lane = lane_id();
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool found = false;
    int64_t scanned = 0, farcs = 0;
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
            farcs = out_rp[v + 1] - out_rp[v];
        }
    }
    const int pos = wave_append(&cnt->n_out, found);
    if (found) q_out[pos] = (int32_t)v;
    const int64_t fa = wave_sum64(farcs);
    const int64_t sc = wave_sum64(scanned);
    const int32_t nn = (int32_t)__popcll(__ballot(found));
    if (lane == 0) {
        if (fa) atomicAdd((unsigned long long*)&cnt->frontier_arcs, (unsigned long long)fa);
        if (sc) atomicAdd((unsigned long long*)&cnt->arcs, (unsigned long long)sc);
        if (nn) atomicAdd(&cnt->n_new, nn);
    }
}

__global__ void k_zero_counters_plain(LevelCounters* c) {
    if (threadIdx.x == 0) {
        c->n_out = 0;
        c->n_new = 0;
        c->arcs = 0;
        c->frontier_arcs = 0;
        c->matched = 0;
    }
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

template <typename DT>
int plain_t(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
            const int32_t* in_col, int64_t n, int64_t arcs, const int32_t* samples_host, int32_t k, DT* Dt,
            void* scratch, LevelCounters* cnt_dev, LevelCounters* cnt_host, TravStats* stats) {
    char* p = (char*)scratch;
    uint32_t* vis = (uint32_t*)p;
    p += align256(sizeof(uint32_t) * ((n + 31) / 32));
    int32_t* q0 = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    int32_t* q1 = (int32_t*)p;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    int rc = 0;
    KernelTimer kt;
    for (int32_t i = 0; i < k; i++) {
        DT* dist = Dt + (int64_t)i * n;
        hipLaunchKernelGGL((k_plain_init<DT>), dim3(nb), dim3(kBlock), 0, st, n, dist, vis);
        hipLaunchKernelGGL((k_plain_source<DT>), dim3(1), dim3(64), 0, st, samples_host[i], dist, vis, q0, out_rp,
                           cnt_dev);
        CCG_HIP(hipMemcpyAsync(cnt_host, cnt_dev, sizeof(LevelCounters), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        stats->launches += 2;
        int32_t nf = 1;
        int64_t mf = cnt_host->frontier_arcs;
        int64_t explored = mf;
        int64_t visited = 1;
        bool pull = false;
        int32_t* qin = q0;
        int32_t* qout = q1;
        for (uint32_t level = 1;; ++level) {
            if ((int64_t)level > DistT<DT>::max_level) return 1;
            const int64_t mu = arcs - explored;
            if (!pull && mf > mu / 14) pull = true;
            else if (pull && (int64_t)nf < n / 24) pull = false;
            hipLaunchKernelGGL(k_zero_counters_plain, dim3(1), dim3(64), 0, st, cnt_dev);
            kt.start(st);
            if (pull) {
                hipLaunchKernelGGL((k_plain_pull<DT>), dim3(nb), dim3(kBlock), 0, st, in_rp, in_col, out_rp, n, vis,
                                   dist, level, qout, cnt_dev);
                stats->nodes_visited += n - visited;
            } else {
                const unsigned g = (unsigned)((nf + kBlock - 1) / kBlock);
                hipLaunchKernelGGL((k_plain_push<DT>), dim3(g), dim3(kBlock), 0, st, out_rp, out_col, qin, nf, qout,
                                   vis, dist, level, cnt_dev);
                stats->nodes_visited += nf;
            }
            CCG_HIP(hipGetLastError());
            kt.stop(st);
            CCG_HIP(hipMemcpyAsync(cnt_host, cnt_dev, sizeof(LevelCounters), hipMemcpyDeviceToHost, st));
            CCG_HIP(hipStreamSynchronize(st));
            stats->kernel_ms += kt.ms();
            stats->kernel_launches += 1;
            stats->launches += 1;
            stats->levels += 1;
            stats->arcs_scanned += cnt_host->arcs;
            nf = cnt_host->n_out;
            mf = cnt_host->frontier_arcs;
            explored += mf;
            visited += nf;
            if (nf == 0) break;
            if ((int64_t)level > stats->maxd) stats->maxd = level;
            std::swap(qin, qout);
        }
        if (visited < n) rc = 2;
    }
    return rc;
}

}  // namespace

size_t bfs_plain_scratch(int64_t n) {
    return align256(sizeof(uint32_t) * ((n + 31) / 32)) + 2 * align256(sizeof(int32_t) * n) + 1024;
}

bool bfs_plain(hipStream_t st, const uint32_t* out_rp, const int32_t* out_col, const uint32_t* in_rp,
               const int32_t* in_col, int64_t n, int64_t arcs, const int32_t* samples_host, int32_t k, void* Dt,
               DistKind dk, void* scratch, size_t scratch_size, DevFlags* flags, LevelCounters* cnt_dev,
               LevelCounters* cnt_host, TravStats* stats) {
    if (scratch_size < bfs_plain_scratch(n)) throw HipError{hipErrorOutOfMemory, "bfs_plain scratch"};
    int r;
    switch (dk) {
        case DistKind::U8:
            r = plain_t<uint8_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint8_t*)Dt, scratch,
                                 cnt_dev, cnt_host, stats);
            break;
        case DistKind::U16:
            r = plain_t<uint16_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint16_t*)Dt,
                                  scratch, cnt_dev, cnt_host, stats);
            break;
        default:
            r = plain_t<uint32_t>(st, out_rp, out_col, in_rp, in_col, n, arcs, samples_host, k, (uint32_t*)Dt,
                                  scratch, cnt_dev, cnt_host, stats);
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
