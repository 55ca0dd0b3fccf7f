// Batched bit-parallel breadth-first search: up to 256 samples at once, one
// bit per sample in W = ceil(kg/64) 64-bit words per node.
//
// Computes D[v][i] = d(c_i, v) (hop distances) for one group of samples: the
// k single-source computations of Sec. 3 of the paper, run together.  The
// paper runs them one after another with Dijkstra; on the GPU the samples
// share every adjacency read.
//
// Level-synchronous pull ("bottom-up") formulation with double-buffered seen
// masks S_prev / S_cur:
//   new_L(v) = (OR_{u in N_in(v)} S_{L-1}(u)) & ~S_{L-1}(v)
// This is exact without a separate frontier set: if v has not been reached
// from c_i by level L-1, then any in-neighbour u that has been reached from
// c_i satisfies d(c_i,u) >= d(c_i,v) - 1 >= L-1, hence d(c_i,u) = L-1.
// A per-node level stamp (parity double-buffered, same width as a distance)
// marks nodes that gained bits at the previous level, so only those
// neighbours' masks are read.  Nodes whose mask is full (all samples have
// reached them) leave the work list one level after they fill up (so both
// buffers hold the full mask).
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kSmallDeg = 32;   // degree up to which one lane scans a node alone
constexpr int kCheckEvery = 8;       // wave path: test for a full mask every 8*64 arcs

template <int W>
__device__ __forceinline__ uint64_t full_word(int w, uint64_t lastmask) {
    return w == W - 1 ? lastmask : ~0ull;
}

template <int W, typename DT>
__global__ __launch_bounds__(kBlock) void k_init_nodes(int64_t n, uint64_t* S0, DT* st0, DT* st1,
                                                       int32_t* act) {
    int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
#pragma unroll
    for (int w = 0; w < W; w++) S0[v * W + w] = 0;
    st0[v] = (DT)DistT<DT>::never;
    st1[v] = (DT)DistT<DT>::never;
    act[v] = (int32_t)v;
}

// Sets the level-0 state of the samples: bit i in c_i's mask, stamp 0 and
// D[c_i][src_base+i] = 0.  Samples are distinct, so every thread writes its
// own word.
template <int W, typename DT>
__global__ void k_init_samples(const int32_t* samples, int32_t kg, uint64_t* S0, DT* st0, DT* D, int64_t k,
                               int32_t src_base) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kg) return;
    int64_t v = samples[src_base + i];
    atomicOr((unsigned long long*)&S0[v * W + (i >> 6)], 1ull << (i & 63));
    st0[v] = (DT)0;
    D[v * k + src_base + i] = (DT)0;
}

template <int W, typename DT>
__global__ __launch_bounds__(kBlock) void k_pull_level(
    const uint32_t* __restrict__ rp, const int32_t* __restrict__ col, const uint64_t* __restrict__ Sprev,
    uint64_t* __restrict__ Scur, const DT* __restrict__ st_prev, DT* __restrict__ st_cur,
    const int32_t* __restrict__ act_in, int32_t n_act, int32_t* __restrict__ act_out, DT* __restrict__ D,
    int64_t k, int32_t src_base, uint64_t lastmask, uint32_t level, LevelCounters* __restrict__ cnt) {
    const int lane = lane_id();
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = idx < n_act;
    const int32_t v = valid ? act_in[idx] : 0;
    const DT want = (DT)(level - 1);

    uint64_t sv[W], acc[W];
    bool full = true;
#pragma unroll
    for (int w = 0; w < W; w++) {
        sv[w] = valid ? Sprev[(int64_t)v * W + w] : ~0ull;
        acc[w] = 0;
        full = full && (sv[w] == full_word<W>(w, lastmask));
    }
    const bool active = valid && !full;
    uint32_t beg = 0, end = 0;
    if (active) {
        beg = rp[v];
        end = rp[v + 1];
    }
    const bool big = active && (end - beg > kSmallDeg);
    int64_t scanned = 0, matched = 0;

    // one lane per low-degree node
    if (active && !big) {
        for (uint32_t e = beg; e < end; ++e) {
            const int32_t u = col[e];
            ++scanned;
            if (st_prev[u] == want) {
                ++matched;
                bool done = true;
#pragma unroll
                for (int w = 0; w < W; w++) {
                    acc[w] |= Sprev[(int64_t)u * W + w];
                    done = done && ((acc[w] | sv[w]) == full_word<W>(w, lastmask));
                }
                if (done) break;
            }
        }
    }

    // the whole wave per high-degree node
    uint64_t bm = __ballot(big);
    while (bm) {
        const int s = __ffsll((unsigned long long)bm) - 1;
        bm &= bm - 1;
        const uint32_t b = (uint32_t)readlane32((int)beg, s);
        const uint32_t en = (uint32_t)readlane32((int)end, s);
        uint64_t svs[W], a[W];
#pragma unroll
        for (int w = 0; w < W; w++) {
            svs[w] = readlane64(sv[w], s);
            a[w] = 0;
        }
        int round = 0;
        for (uint32_t e0 = b; e0 < en; e0 += 64) {
            const uint32_t e = e0 + lane;
            if (e < en) {
                const int32_t u = col[e];
                ++scanned;
                if (st_prev[u] == want) {
                    ++matched;
#pragma unroll
                    for (int w = 0; w < W; w++) a[w] |= Sprev[(int64_t)u * W + w];
                }
            }
            if (++round == kCheckEvery) {
                round = 0;
                bool done = true;
#pragma unroll
                for (int w = 0; w < W; w++) {
                    a[w] = wave_or64(a[w]);
                    done = done && ((a[w] | svs[w]) == full_word<W>(w, lastmask));
                }
                if (done) break;
            }
        }
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint64_t r = wave_or64(a[w]);
            if (lane == s) acc[w] = r;
        }
    }

    uint64_t nw[W];
    bool anynew = false;
#pragma unroll
    for (int w = 0; w < W; w++) {
        nw[w] = active ? (acc[w] & ~sv[w]) : 0ull;
        anynew = anynew || (nw[w] != 0);
    }
    if (valid) {
#pragma unroll
        for (int w = 0; w < W; w++) Scur[(int64_t)v * W + w] = sv[w] | nw[w];
        if (anynew) st_cur[v] = (DT)level;
    }

    // distances: for every node with new bits, lane j writes D[v][w*64+j]
    uint64_t m = __ballot(anynew);
    const int32_t n_new = (int32_t)__popcll(m);
    while (m) {
        const int s = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t vs = readlane32(v, s);
        DT* row = D + vs * k + src_base;
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint64_t x = readlane64(nw[w], s);
            if ((x >> lane) & 1ull) row[w * 64 + lane] = (DT)level;
        }
    }

    // nodes not full at the start of this level stay on the list
    const int pos = wave_append(&cnt->n_out, active);
    if (active) act_out[pos] = v;
    const int64_t tot = wave_sum64(scanned);
    const int64_t mat = wave_sum64(matched);
    if (lane == 0) {
        if (n_new) atomicAdd(&cnt->n_new, n_new);
        if (tot) atomicAdd((unsigned long long*)&cnt->arcs, (unsigned long long)tot);
        if (mat) atomicAdd((unsigned long long*)&cnt->matched, (unsigned long long)mat);
    }
}

__global__ void k_zero_counters(LevelCounters* c) {
    if (threadIdx.x == 0) {
        c->n_out = 0;
        c->n_new = 0;
        c->arcs = 0;
        c->frontier_arcs = 0;
        c->matched = 0;
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int W, typename DT>
int bfs_batched_t(hipStream_t st, const uint32_t* in_rp, const int32_t* in_col, int64_t n,
                  const int32_t* samples_dev, int32_t kg, int32_t src_base, int32_t k, DT* D, void* scratch,
                  LevelCounters* cnt_dev, LevelCounters* cnt_host, TravStats* stats) {
    char* p = (char*)scratch;
    uint64_t* S0 = (uint64_t*)p;
    p += align256(sizeof(uint64_t) * n * W);
    uint64_t* S1 = (uint64_t*)p;
    p += align256(sizeof(uint64_t) * n * W);
    DT* st0 = (DT*)p;
    p += align256(sizeof(DT) * n);
    DT* st1 = (DT*)p;
    p += align256(sizeof(DT) * n);
    int32_t* act0 = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    int32_t* act1 = (int32_t*)p;

    const int rem = kg - (W - 1) * 64;
    const uint64_t lastmask = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_init_nodes<W, DT>), dim3(nb), dim3(kBlock), 0, st, n, S0, st0, st1, act0);
    hipLaunchKernelGGL((k_init_samples<W, DT>), dim3((kg + 63) / 64), dim3(64), 0, st, samples_dev, kg, S0, st0,
                       D, (int64_t)k, src_base);
    stats->launches += 2;

    int32_t n_act = (int32_t)n;
    uint64_t* Sp = S0;
    uint64_t* Sc = S1;
    DT* sp = st0;
    DT* sc = st1;
    int32_t* ain = act0;
    int32_t* aout = act1;
    KernelTimer kt;
    for (uint32_t level = 1;; ++level) {
        if ((int64_t)level > DistT<DT>::max_level) return 1;  // distance type too narrow
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, cnt_dev);
        const unsigned g = (unsigned)((n_act + kBlock - 1) / kBlock);
        kt.start(st);
        hipLaunchKernelGGL((k_pull_level<W, DT>), dim3(g), dim3(kBlock), 0, st, in_rp, in_col, Sp, Sc, sp, sc,
                           ain, n_act, aout, D, (int64_t)k, src_base, lastmask, level, cnt_dev);
        CCG_HIP(hipGetLastError());
        kt.stop(st);
        CCG_HIP(hipMemcpyAsync(cnt_host, cnt_dev, sizeof(LevelCounters), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        stats->kernel_ms += kt.ms();
        stats->kernel_launches += 1;
        stats->arcs_matched += cnt_host->matched;
        stats->launches += 1;
        stats->levels += 1;
        stats->arcs_scanned += cnt_host->arcs;
        stats->nodes_visited += n_act;
        if (cnt_host->n_new > 0 && (int64_t)level > stats->maxd) stats->maxd = level;
        n_act = cnt_host->n_out;
        if (n_act == 0) break;
        if (cnt_host->n_new == 0) return 2;  // nodes left that no sample can reach
        std::swap(Sp, Sc);
        std::swap(sp, sc);
        std::swap(ain, aout);
    }
    return 0;
}

template <int W>
int dispatch_dt(hipStream_t st, const uint32_t* in_rp, const int32_t* in_col, int64_t n, const int32_t* samples_dev,
                int32_t kg, int32_t src_base, int32_t k, void* D, DistKind dk, void* scratch,
                LevelCounters* cnt_dev, LevelCounters* cnt_host, TravStats* stats) {
    switch (dk) {
        case DistKind::U8:
            return bfs_batched_t<W, uint8_t>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, (uint8_t*)D, scratch,
                                             cnt_dev, cnt_host, stats);
        case DistKind::U16:
            return bfs_batched_t<W, uint16_t>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, (uint16_t*)D,
                                              scratch, cnt_dev, cnt_host, stats);
        default:
            return bfs_batched_t<W, uint32_t>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, (uint32_t*)D,
                                              scratch, cnt_dev, cnt_host, stats);
    }
}

}  // namespace

size_t bfs_batched_scratch(int64_t n, int32_t kg) {
    const int W = (kg + 63) / 64;
    return align256(sizeof(uint64_t) * n * W) * 2 + align256(sizeof(uint32_t) * n) * 2 +
           align256(sizeof(int32_t) * n) * 2 + 1024;
}

// Returns through the bool: false = the distance type overflowed.  A
// disconnected graph sets flags->disconnected (host-visible copy is made by
// the caller) -- here signalled by writing to the device flag word.
bool bfs_batched(hipStream_t st, const uint32_t* in_rp, const int32_t* in_col, int64_t n,
                 const int32_t* samples_dev, int32_t kg, int32_t src_base, int32_t k, void* D, DistKind dk,
                 void* scratch, size_t scratch_size, DevFlags* flags, LevelCounters* cnt_dev,
                 LevelCounters* cnt_host, TravStats* stats) {
    if (scratch_size < bfs_batched_scratch(n, kg)) throw HipError{hipErrorOutOfMemory, "bfs_batched scratch"};
    const int W = (kg + 63) / 64;
    int r;
    switch (W) {
        case 1: r = dispatch_dt<1>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, D, dk, scratch, cnt_dev, cnt_host, stats); break;
        case 2: r = dispatch_dt<2>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, D, dk, scratch, cnt_dev, cnt_host, stats); break;
        case 3: r = dispatch_dt<3>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, D, dk, scratch, cnt_dev, cnt_host, stats); break;
        default: r = dispatch_dt<4>(st, in_rp, in_col, n, samples_dev, kg, src_base, k, D, dk, scratch, cnt_dev, cnt_host, stats); break;
    }
    if (r == 1) return false;
    if (r == 2) {
        int32_t one = 1;
        CCG_HIP(hipMemcpyAsync(&flags->disconnected, &one, sizeof(one), hipMemcpyHostToDevice, st));
        CCG_HIP(hipStreamSynchronize(st));
    }
    return true;
}

}  // namespace ccg
