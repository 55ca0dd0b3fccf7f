// Batched bit-parallel breadth-first search: up to 256 samples at once, one
// bit per sample in W = ceil(kg/64) 64-bit words per node.
//
// This is the k single-source computations of Sec. 3 of the paper run
// together: every adjacency read serves all samples of the group.  The
// traversal never materialises the distance matrix; it records, for every
// level L, the seen mask S_L(v) = {i : d(c_i, v) <= L} (a "snapshot").  The
// estimator epilogue derives distances, pivots, sums and the L/HC split from
// these masks with bit operations (d(c_i, v) = number of levels at which bit
// i is still clear).
//
// Level-synchronous, direction-optimising:
//   pull  new_L(v) = (OR_{u in N_in(v)} S_{L-1}(u)) & ~S_{L-1}(v).  Exact with
//         no frontier test: if bit i is clear in S_{L-1}(v), every in-neighbour
//         u with bit i set has d(c_i,u) >= d(c_i,v) - 1 >= L-1, i.e. = L-1.
//   push  for every node u that gained bits at level L-1 and every out-arc
//         u->v: NX(v) |= S_{L-1}(u) (atomic OR); then new_L(v) = NX(v) & ~S_{L-1}(v).
//         The same triangle argument makes the extra (older) bits harmless.
// Push is chosen while the frontier's out-arcs are few compared with the
// arcs a pull would scan.  That choice, and the end of the search, are made on
// the device by the last block of each level's merge launch, so the host
// enqueues a batch of levels (as many as the graph's last search needed) and
// reads the control block once per batch; levels past the end exit at once.
// Two launches per level: k_scatter_level (push, or the hub pull) and
// k_group_level (the other nodes' pull, the merge and the decision).
//
// Sparse hub pulls: only in-neighbours that gained bits at the previous level
// can pass new bits on (same triangle argument), so when few nodes changed, a
// hub chunk reads a neighbour's mask only if the neighbour's bit is set in the bitmap of
// nodes that changed at the previous level (one bit per node, written by the
// merge).  There are two bitmaps, by level parity, so a merge writing level
// L's bits never races with reads of level L-1's.  (The merge's own pulls of
// low-degree nodes gain nothing from the test: it costs what it saves.)  Groups that left the
// work list keep older bits; reading a full neighbour adds nothing, so a
// superset of the changed nodes is exact.
//
// Pull work decomposition (node ids are degree-sorted by the graph builder):
//   * hub nodes (the leading nh ids) are scanned by k_scatter_level in fixed chunks
//     of arcs, one wave per chunk, reduced with DPP and OR-ed atomically into
//     NX(hub);
//   * every other node belongs to a group of 64 consecutive ids handled by one
//     wave in k_group_level: G lanes per node (G from the group's largest
//     degree) read the node's arcs in coalesced runs and OR-reduce with DPP.
// k_group_level then finalises every node of the group (in both modes): the
// new bits, the next seen mask, the level snapshot, the frontier list for a
// following push level, and the per-sample histogram
// hist[i][L] = #{v not sampled : d(c_i, v) = L} by ballot transposition.
// A group leaves the work list once all of its nodes were full (reached by
// every sample) at the start of a level; fill_level[g] records the last level
// it was processed at.  Its later snapshots are written all-ones, so every
// level's snapshot plane is complete and is the next level's working mask:
// there is no separate working copy of the masks.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

template <int W>
__device__ __forceinline__ uint64_t full_word(int w, uint64_t lastmask) {
    return w == W - 1 ? lastmask : ~0ull;
}

// OR over aligned groups of 2^lg lanes (lg <= 4) inside a 16-lane row, by DPP
// lane permutations; afterwards every lane holds its group's OR.
__device__ __forceinline__ uint32_t dpp_or_group32(uint32_t x, int lg) {
    if (lg >= 1) x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if (lg >= 2) x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if (lg >= 3) x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (lg >= 4) x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false);  // row_mirror
    return x;
}

__device__ __forceinline__ uint64_t dpp_or_group64(uint64_t x, int lg) {
    const uint32_t lo = dpp_or_group32((uint32_t)x, lg);
    const uint32_t hi = dpp_or_group32((uint32_t)(x >> 32), lg);
    return ((uint64_t)hi << 32) | lo;
}

// OR of a value over the whole wave, valid in every lane: rows by DPP, then
// the four row results by lane reads.
__device__ __forceinline__ uint32_t wave_or32_dpp(uint32_t x) {
    x = dpp_or_group32(x, 4);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 0) | (uint32_t)__builtin_amdgcn_readlane((int)x, 16) |
           (uint32_t)__builtin_amdgcn_readlane((int)x, 32) | (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
}

__device__ __forceinline__ uint64_t wave_or64_dpp(uint64_t x) {
    const uint32_t lo = wave_or32_dpp((uint32_t)x);
    const uint32_t hi = wave_or32_dpp((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Loads the words of node u's mask that `need` selects (bit p = word pair p,
// words 2p and 2p+1), as 16-byte loads where two words are present.
template <int W>
__device__ __forceinline__ void load_mask(const uint64_t* __restrict__ S, int64_t u, uint32_t need, uint64_t out[W]) {
    const uint64_t* row = S + u * W;
#pragma unroll
    for (int p = 0; p < (W + 1) / 2; p++) {
        if (2 * p + 1 < W) {
            uint4 q = make_uint4(0, 0, 0, 0);
            if (need & (1u << p)) q = *(const uint4*)(row + 2 * p);
            out[2 * p] = ((uint64_t)q.y << 32) | q.x;
            out[2 * p + 1] = ((uint64_t)q.w << 32) | q.z;
        } else {
            out[2 * p] = (need & (1u << p)) ? row[2 * p] : 0ull;
        }
    }
}

template <int W>
__device__ __forceinline__ void store_mask(uint64_t* __restrict__ S, int64_t v, const uint64_t x[W]) {
    uint64_t* row = S + v * W;
#pragma unroll
    for (int p = 0; p < (W + 1) / 2; p++) {
        if (2 * p + 1 < W) {
            *(uint4*)(row + 2 * p) = make_uint4((uint32_t)x[2 * p], (uint32_t)(x[2 * p] >> 32), (uint32_t)x[2 * p + 1],
                                                (uint32_t)(x[2 * p + 1] >> 32));
        } else {
            row[2 * p] = x[2 * p];
        }
    }
}

// word pairs of a mask that are not yet all-ones
template <int W>
__device__ __forceinline__ uint32_t pairs_needed(const uint64_t s[W], uint64_t lastmask) {
    uint32_t need = 0;
#pragma unroll
    for (int p = 0; p < (W + 1) / 2; p++) {
        bool f = s[2 * p] == full_word<W>(2 * p, lastmask);
        if (2 * p + 1 < W) f = f && (s[2 * p + 1] == full_word<W>(2 * p + 1, lastmask));
        if (!f) need |= 1u << p;
    }
    return need;
}

// Adds per-wave partial counts into the block's counter slot: one atomic
// per field per block.
struct WaveCounts {
    int64_t arcs = 0, farcs = 0, hub = 0;
    int32_t n_new = 0, n_out = 0, hub_open = 0;
};

// Returns, in thread 0, a value that depends on every counter atomic's result
// (always 0): using it makes the thread wait until those atomics have been
// performed, so a later atomic can announce them to other blocks.
__device__ __forceinline__ uint32_t flush_counts(WaveCounts c, LevelCounters* slots) {
    __shared__ int64_t red[kWaves][6];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int64_t a = wave_sum64(c.arcs), f = wave_sum64(c.farcs), h = wave_sum64(c.hub);
    const int32_t nn = wave_sum32(c.n_new), no = wave_sum32(c.n_out), ho = wave_sum32(c.hub_open);
    if (lane == 0) {
        red[wave][0] = a;
        red[wave][1] = f;
        red[wave][2] = nn;
        red[wave][3] = no;
        red[wave][4] = h;
        red[wave][5] = ho;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t[6] = {0, 0, 0, 0, 0, 0};
        for (int w = 0; w < kWaves; w++)
            for (int q = 0; q < 6; q++) t[q] += red[w][q];
        LevelCounters* c0 = slots + (blockIdx.x % kCounterSlots);
        uint64_t r = 0;
        if (t[0]) r |= atomicAdd((unsigned long long*)&c0->arcs, (unsigned long long)t[0]);
        if (t[1]) r |= atomicAdd((unsigned long long*)&c0->frontier_arcs, (unsigned long long)t[1]);
        if (t[2]) r |= (uint32_t)atomicAdd(&c0->n_new, (int32_t)t[2]);
        if (t[3]) r |= (uint32_t)atomicAdd(&c0->n_out, (int32_t)t[3]);
        if (t[4]) r |= atomicAdd((unsigned long long*)&c0->matched, (unsigned long long)t[4]);
        if (t[5]) r |= (uint32_t)atomicAdd(&c0->hub_open, (int32_t)t[5]);
        return (uint32_t)(r >> 63);  // counts stay far below 2^63
    }
    return 0;
}

__device__ void decide_wave(LevelCounters* cnt, BfsCtl* ctl, int32_t* mode_log, int32_t level, int32_t cap,
                            int64_t arcs_total, int32_t alpha, int64_t n);

template <int W>
__global__ __launch_bounds__(kBlock) void k_init(int64_t n, int32_t ngroups, uint64_t* snap0,
                                                 uint64_t* NX, int32_t* chg, uint8_t* gfull, int32_t* fill_level,
                                                 uint64_t* chgbits, const uint64_t* __restrict__ preset,
                                                 const int32_t* __restrict__ gvalid, LevelCounters* cnt,
                                                 DevFlags* zero_flags, int32_t* sidx_fill, int32_t* hist_zero,
                                                 int64_t hist_elems) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) {
        const int64_t g = t >> 6;
        const bool pad = preset && (int32_t)(t & 63) >= gvalid[g];
        uint64_t s0[W], z[W];
#pragma unroll
        for (int w = 0; w < W; w++) {
            s0[w] = preset ? (pad ? ~0ull : preset[g * W + w]) : 0ull;
            z[w] = 0;
        }
        store_mask<W>(snap0, t, s0);  // 16-byte stores
        store_mask<W>(NX, t, z);
        chg[t] = -1;
        if (sidx_fill) sidx_fill[t] = -1;
    }
    if (t < ngroups) {
        gfull[t] = 0;
        fill_level[t] = 0;
        chgbits[t] = 0;
        chgbits[ngroups + t] = 0;
    }
    if (t < hist_elems) hist_zero[t] = 0;
    if (t < kCounterSlots) cnt[t] = LevelCounters{};
    if (zero_flags && t == 0) *zero_flags = DevFlags{};
}

// Level-0 state, one block: bit i in c_i's mask (the working mask is the
// level-0 snapshot); the samples form the level-0 frontier.  Samples are
// distinct nodes.  Then the block's first wave makes the level-0 decision.
// With stage_ids the samples are taken from pinned host memory and stored to
// `samples` for the later launches (the caller's numbering to samples_out).
template <int W>
__global__ __launch_bounds__(kBlock) void k_init_samples(int32_t* samples, const int32_t* stage_ids,
                                                         const int32_t* stage_caller, int32_t* samples_out,
                                                         int32_t kg, int32_t src_base,
                                                         uint64_t* snap0, int32_t* chg, uint64_t* chgbits,
                                                         const uint32_t* out_rp, LevelCounters* cnt,
                                                         int32_t* sidx_fill, BfsCtl* ctl, int32_t* mode_log,
                                                         int32_t cap, int64_t arcs_total, int32_t alpha, int64_t n) {
    for (int i = threadIdx.x; i < kg; i += kBlock) {
        const int32_t j = src_base + i;
        int64_t v;
        if (stage_ids) {  // pinned host memory: system-scope loads see what the host wrote before the launch
            const int32_t s = __hip_atomic_load(stage_ids + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            samples[j] = s;
            if (samples_out)
                samples_out[j] = __hip_atomic_load(stage_caller + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            v = s;
        } else {
            v = samples[j];
        }
        if (v < 0) continue;  // a bit position no sample uses (batches)
        const unsigned long long bit = 1ull << (i & 63);
        atomicOr((unsigned long long*)&snap0[v * W + (i >> 6)], bit);
        chg[v] = 0;
        if (sidx_fill) sidx_fill[v] = src_base + i;
        atomicOr((unsigned long long*)&chgbits[v >> 6], 1ull << (v & 63));
        atomicAdd((unsigned long long*)&cnt[i % kCounterSlots].frontier_arcs,
                  (unsigned long long)(out_rp[v + 1] - out_rp[v]));
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x < 64) decide_wave(cnt, ctl, mode_log, 0, cap, arcs_total, alpha, n);
}

constexpr int32_t kModeLog = 4096;  // levels whose direction is logged for the host
constexpr int64_t kSparseDiv = 8;   // a level is sparse when fewer than n / kSparseDiv nodes changed

// One wave (lanes = counter slots): sums and clears the counter slots of the
// level just run, records it, and decides whether and how the next level
// runs (push iff the frontier's out-arcs times alpha are below what the last
// pull scanned).  Level 0 only initialises the state from the samples'
// frontier.  Counters are read with device-scope atomic loads: they were
// written by atomics of other blocks.
__device__ void decide_wave(LevelCounters* cnt, BfsCtl* ctl, int32_t* mode_log, int32_t level, int32_t cap,
                            int64_t arcs_total, int32_t alpha, int64_t n) {
    const int t = lane_id();
    LevelCounters* c = cnt + t;
    const int64_t arcs = wave_sum64(__hip_atomic_load(&c->arcs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int64_t farcs = wave_sum64(__hip_atomic_load(&c->frontier_arcs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int64_t matched = wave_sum64(__hip_atomic_load(&c->matched, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int64_t n_new = wave_sum64(__hip_atomic_load(&c->n_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int64_t n_out = wave_sum64(__hip_atomic_load(&c->n_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int64_t hub_open = wave_sum64(__hip_atomic_load(&c->hub_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    *c = LevelCounters{};
    if (t != 0) return;
    BfsCtl s = *ctl;
    s.ticket = 0;
    if (level == 0) {
        s = BfsCtl{};
        s.pull_arcs = arcs_total > 0 ? arcs_total : 1;
        s.frontier_arcs = farcs;
        s.pull = farcs * alpha >= s.pull_arcs ? 1 : 0;
        *ctl = s;
        return;
    }
    if (s.done) {
        *ctl = s;
        return;
    }
    s.levels += 1;
    if (level < kModeLog) mode_log[level] = s.pull;
    if (s.pull) {
        s.pull_levels += 1;
        s.arcs += arcs + matched;
        s.hub_arcs += matched;
        s.pull_arcs = arcs + matched > 0 ? arcs + matched : 1;
    } else {
        s.arcs += arcs;
        s.push_arcs += arcs;
        s.push_atomics += matched;
    }
    s.nodes += n_out * 64;
    s.hubs_full = hub_open == 0 ? 1 : 0;
    s.sparse = n_new * kSparseDiv < n ? 1 : 0;
    if (n_new > 0) s.lmax = level;
    s.frontier_arcs = farcs;
    if (n_out == 0) {
        s.done = 1;
    } else if (n_new == 0) {
        s.done = 1;
        s.status = 2;
    } else if (level + 1 >= cap) {
        s.done = 1;
        s.status = 1;
    } else {
        s.pull = farcs * alpha >= s.pull_arcs ? 1 : 0;
    }
    *ctl = s;
}


// push along arc u->x of the mask su (u's seen mask): only bits not already
// pending in NX(x) need the atomic, so popular targets stop taking atomics
// once they hold the frontier's bits (a stale NX read only lets a redundant
// atomic through).  Bits x has already seen are not filtered here: the merge
// drops them (new = NX & ~S), and skipping the load of x's mask makes the push
// one random read and at most one atomic per word (rmat22dir: push levels
// 0.745 -> 0.641 ms; without the pending test too, 0.703 ms, as hubs then
// take every atomic).  Targets past the most popular part of the hub prefix
// (ids >= check_below) are rarely pushed to twice in one level, so they take
// the atomic without the read.
template <int W>
__device__ __forceinline__ void push_arc(uint64_t* NX, int64_t x, const uint64_t (&su)[W], int64_t check_below,
                                         int64_t& atomics) {
#pragma unroll
    for (int w = 0; w < W; w++) {
        if (!su[w]) continue;
        const uint64_t pending =
            x < check_below ? __hip_atomic_load(&NX[x * W + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
        const uint64_t r = su[w] & ~pending;
        if (r) {
            atomicOr((unsigned long long*)&NX[x * W + w], (unsigned long long)r);
            ++atomics;
        }
    }
}

// Push from the nodes of group g that gained bits at the previous level
// (nodes past the hub prefix, out-degree at most the hub threshold): lanes
// over each changed node's out-arcs.
template <int W>
__device__ __forceinline__ void push_group(const uint32_t* __restrict__ out_rp, const int32_t* __restrict__ out_col,
                                           const int32_t* __restrict__ chg, const uint8_t* __restrict__ ghub,
                                           int64_t n, int32_t g, int32_t prev_level,
                                           const uint64_t* __restrict__ Sprev, uint64_t* NX, int64_t check_below,
                                           WaveCounts& wc, int64_t& atomics) {
    const int lane = lane_id();
    if (ghub && ghub[g]) return;  // hubs push by chunks
    const int64_t v = (int64_t)g * 64 + lane;
    uint64_t m = __ballot(v < n && chg[v] == prev_level);
    while (m) {
        const int s = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t u = (int64_t)g * 64 + s;
        uint64_t su[W];
#pragma unroll
        for (int w = 0; w < W; w++) su[w] = Sprev[u * W + w];
        const uint32_t b = out_rp[u], e = out_rp[u + 1];
        for (uint32_t t = b + lane; t < e; t += 64) {
            ++wc.arcs;
            push_arc<W>(NX, out_col[t], su, check_below, atomics);
        }
    }
}

// Push along one chunk (node, first arc, end arc) of a hub's out-arcs, so a
// frontier node with a huge out-degree is spread over many waves.
template <int W>
__device__ __forceinline__ void push_chunk(const int32_t* __restrict__ out_col, const int32_t* __restrict__ chunk,
                                           const int32_t* __restrict__ chg, int32_t prev_level,
                                           const uint64_t* __restrict__ Sprev, uint64_t* NX, int64_t check_below,
                                           WaveCounts& wc, int64_t& atomics) {
    const int64_t h = chunk[0];
    if (chg[h] != prev_level) return;
    const uint32_t b = (uint32_t)chunk[1], e = (uint32_t)chunk[2];
    uint64_t su[W];
#pragma unroll
    for (int w = 0; w < W; w++) su[w] = Sprev[h * W + w];
    for (uint32_t t = b + lane_id(); t < e; t += 64) {
        ++wc.arcs;
        push_arc<W>(NX, out_col[t], su, check_below, atomics);
    }
}

// Pull over one chunk (hub, first arc, end arc) of a hub's in-arcs: OR of the
// neighbours' masks, new bits into NX with one atomic per word.
template <int W>
__device__ __forceinline__ void hub_chunk(const int32_t* __restrict__ col, const uint64_t* __restrict__ Sprev,
                                          const int32_t* __restrict__ chunk, uint64_t* NX, uint64_t lastmask,
                                          const uint64_t* __restrict__ chgbits, bool sparse, int64_t& scanned) {
    const int lane = lane_id();
    const int64_t h = chunk[0];
    const uint32_t b = (uint32_t)chunk[1], e = (uint32_t)chunk[2];
    uint64_t sh[W];
#pragma unroll
    for (int w = 0; w < W; w++) sh[w] = Sprev[h * W + w];
    const uint32_t need = pairs_needed<W>(sh, lastmask);
    if (!need) return;  // full hub: nothing to find
    uint64_t acc[W];
#pragma unroll
    for (int w = 0; w < W; w++) acc[w] = 0;
    // the bits the hub can still gain this level
    uint64_t miss[W];
#pragma unroll
    for (int w = 0; w < W; w++) miss[w] = full_word<W>(w, lastmask) & ~sh[w];
    // The trip count is the same for every lane (loads predicated), so the
    // wave-wide check below always sees every lane.
    for (uint32_t base = b; base < e; base += 128) {
        const uint32_t t0 = base + lane, t1 = t0 + 64;
        uint64_t a0[W], a1[W];
        // a sparse level reads only the masks of neighbours that changed at the last level
        const int64_t u0 = t0 < e ? col[t0] : -1, u1 = t1 < e ? col[t1] : -1;
        const bool r0 = u0 >= 0 && (!sparse || ((chgbits[u0 >> 6] >> (u0 & 63)) & 1ull));
        const bool r1 = u1 >= 0 && (!sparse || ((chgbits[u1 >> 6] >> (u1 & 63)) & 1ull));
        scanned += r0 + r1;  // arcs whose mask was read (36 bytes each)
        if (r0) {
            load_mask<W>(Sprev, u0, need, a0);
        } else {
#pragma unroll
            for (int w = 0; w < W; w++) a0[w] = 0;
        }
        if (r1) {
            load_mask<W>(Sprev, u1, need, a1);
        } else {
#pragma unroll
            for (int w = 0; w < W; w++) a1[w] = 0;
        }
#pragma unroll
        for (int w = 0; w < W; w++) acc[w] |= a0[w] | a1[w];
        // stop once the chunk has found every bit the hub misses: the rest of
        // its arcs cannot add any (exact early exit)
        bool done = true;
#pragma unroll
        for (int w = 0; w < W; w++) done = done && (miss[w] & ~wave_or64_dpp(acc[w])) == 0;
        if (done) break;
    }
#pragma unroll
    for (int w = 0; w < W; w++) {
        const uint64_t r = wave_or64_dpp(acc[w]) & ~sh[w];
        if (lane == 0 && r) atomicOr((unsigned long long*)&NX[h * W + w], (unsigned long long)r);
    }
}

// The scatter half of a level, its direction taken from the control block:
//   pull: one wave per chunk of a hub's in-arcs (the other nodes pull in the
//         merge kernel);
//   push: one wave per chunk of a hub's out-arcs, then one wave per group of
//         the other nodes, each sending the masks of nodes that changed at
//         the previous level along their out-arcs.
template <int W>
__global__ __launch_bounds__(kBlock) void k_scatter_level(
    const int32_t* __restrict__ col, const int32_t* __restrict__ hub_chunks, int32_t n_hub_chunks,
    const uint32_t* __restrict__ out_rp, const int32_t* __restrict__ out_col, const int32_t* __restrict__ push_chunks,
    int32_t n_push_chunks, int32_t g0, int32_t ngroups, const int32_t* __restrict__ chg,
    const uint8_t* __restrict__ ghub, int64_t n,
    int32_t prev_level, const uint64_t* __restrict__ Sprev, uint64_t* NX, uint64_t lastmask, LevelCounters* cnt,
    const BfsCtl* __restrict__ ctl, const uint64_t* __restrict__ chgbits) {
    if (ctl->done) return;
    const int pull = ctl->pull;
    const bool sparse = ctl->sparse != 0;
    if (pull && ctl->hubs_full) return;  // every hub holds every bit: its chunks would find nothing
    const int32_t waves = gridDim.x * kWaves;
    const int32_t wid = blockIdx.x * kWaves + (threadIdx.x >> 6);
    WaveCounts wc;
    int64_t extra = 0;  // pull: arcs scanned; push: atomics issued
    if (pull) {
        for (int32_t c = wid; c < n_hub_chunks; c += waves)
            hub_chunk<W>(col, Sprev, hub_chunks + 3 * (int64_t)c, NX, lastmask, chgbits, sparse, extra);
    } else {
        const int64_t items = (int64_t)n_push_chunks + (ngroups - g0);
        // only the most popular targets, the first quarter of the hub prefix
        // (highest in-degree), are likely to hold pushed bits already; the
        // others take the atomic without the read (rmat22dir: reading at every
        // target 2.356 ms, at the whole hub prefix 2.285 ms, at its first
        // quarter 2.260 ms, at its first sixteenth 2.285 ms)
        const int64_t check_below = (ghub || g0 == 0) ? n : (int64_t)g0 * 16;
        for (int64_t t = wid; t < items; t += waves) {
            if (t < n_push_chunks)
                push_chunk<W>(out_col, push_chunks + 3 * t, chg, prev_level, Sprev, NX, check_below, wc, extra);
            else
                push_group<W>(out_rp, out_col, chg, ghub, n, g0 + (int32_t)(t - n_push_chunks), prev_level, Sprev,
                              NX, check_below, wc, extra);
        }
    }
    wc.hub = extra;
    (void)flush_counts(wc, cnt);
}

// Column sums of a 64 x 64 bit matrix held one row per lane (bit j of lane
// i's word is entry (i, j)): six butterfly stages transpose it, each swapping
// the off-diagonal s x s blocks of every 2s x 2s diagonal block (s = 32 .. 1),
// after which lane j holds column j; returns that column's popcount.
__device__ inline int32_t column_count64(uint64_t x, int lane) {
    constexpr uint64_t kLow[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                  0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int t = 0; t < 6; t++) {
        const int s = 32 >> t;
        const uint64_t lo = kLow[t];
        const uint64_t p = __shfl_xor(x, s);
        x = (lane & s) ? ((x & ~lo) | ((p & ~lo) >> s)) : ((x & lo) | ((p & lo) << s));
    }
    return (int32_t)__popcll(x);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_group_level(
    const uint32_t* __restrict__ rp, const int32_t* __restrict__ col, const uint32_t* __restrict__ out_rp,
    const uint64_t* __restrict__ Sprev, uint64_t* __restrict__ snap,
    int32_t* __restrict__ fill_level, uint8_t* __restrict__ gfull, int32_t* __restrict__ chg, int32_t ngroups,
    int64_t n, int64_t nh, uint64_t* __restrict__ NX, uint64_t lastmask, int32_t level,
    const int32_t* __restrict__ sidx, int32_t* __restrict__ hist, int64_t hlen, int64_t k, int32_t src_base,
    LevelCounters* __restrict__ cnt, BfsCtl* ctl, int32_t* mode_log, int32_t cap, int64_t arcs_total, int32_t alpha,
    const uint8_t* __restrict__ ghub, uint64_t* __restrict__ chg_out) {
    if (ctl->done) return;
    const int pull = ctl->pull;
    __shared__ uint64_t lds_acc[kWaves][64][W];
    __shared__ int32_t lds_hist[W * 64];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const bool do_hist = hist != nullptr;
    if (do_hist) {
        for (int t = threadIdx.x; t < W * 64; t += kBlock) lds_hist[t] = 0;
        __syncthreads();
    }
    int32_t hcnt[W];
#pragma unroll
    for (int w = 0; w < W; w++) hcnt[w] = 0;
    WaveCounts wc;

    const int32_t stride = gridDim.x * kWaves;
    for (int32_t g = blockIdx.x * kWaves + wave; g < ngroups; g += stride) {
        if (gfull[g]) {  // every node of the group is full in every later mask: write it so
            const int64_t v = (int64_t)g * 64 + lane;
            if (v < n) {
                uint64_t f[W];
#pragma unroll
                for (int w = 0; w < W; w++) f[w] = full_word<W>(w, lastmask);
                store_mask<W>(snap, v, f);
            }
            continue;
        }
        const int64_t v = (int64_t)g * 64 + lane;
        const bool valid = v < n;
        uint64_t sv[W];
        if (valid) {
            load_mask<W>(Sprev, v, 0xFu, sv);
        } else {
#pragma unroll
            for (int w = 0; w < W; w++) sv[w] = full_word<W>(w, lastmask);
        }
        const uint32_t need = pairs_needed<W>(sv, lastmask);
        const bool fullv = need == 0;
        const bool ishub = ghub ? ghub[g] != 0 : v < nh;
        uint64_t acc[W];
#pragma unroll
        for (int w = 0; w < W; w++) acc[w] = 0;

        if (pull) {
            uint32_t rb = 0, deg = 0;
            if (valid && !ishub && !fullv) {
                rb = rp[v];
                deg = rp[v + 1] - rb;
            }
            uint32_t maxdeg = deg;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const uint32_t o = (uint32_t)__shfl_xor((int)maxdeg, off);
                maxdeg = o > maxdeg ? o : maxdeg;
            }
            if (maxdeg > 0) {
                // G = 2^lg lanes per node, about maxdeg/G >= 2 arcs per lane
                int lg = 0;
                while (lg < 3 && (2u << lg) <= maxdeg / 2) lg++;
                const int G = 1 << lg;
                const int npp = 64 >> lg;
                const int sub = lane & (G - 1);
                const int slot = lane >> lg;
                int64_t scanned = 0;
                for (int pass = 0; pass < G; pass++) {
                    const int r = pass * npp + slot;
                    const uint32_t b = (uint32_t)__shfl((int)rb, r);
                    const uint32_t dg = (uint32_t)__shfl((int)deg, r);
                    const uint32_t nd = (uint32_t)__shfl((int)need, r);
                    uint64_t x[W];
#pragma unroll
                    for (int w = 0; w < W; w++) x[w] = 0;
                    uint32_t t = sub;
                    for (; t + G < dg; t += 2 * G) {
                        const int64_t u0 = col[b + t], u1 = col[b + t + G];
                        uint64_t a0[W], a1[W];
                        load_mask<W>(Sprev, u0, nd, a0);
                        load_mask<W>(Sprev, u1, nd, a1);
#pragma unroll
                        for (int w = 0; w < W; w++) x[w] |= a0[w] | a1[w];
                        scanned += 2;
                    }
                    if (t < dg) {
                        uint64_t a0[W];
                        load_mask<W>(Sprev, col[b + t], nd, a0);
#pragma unroll
                        for (int w = 0; w < W; w++) x[w] |= a0[w];
                        scanned += 1;
                    }
#pragma unroll
                    for (int w = 0; w < W; w++) x[w] = dpp_or_group64(x[w], lg);
                    if (sub == 0) {
#pragma unroll
                        for (int w = 0; w < W; w++) lds_acc[wave][r][w] = x[w];
                    }
                }
                wc.arcs += scanned;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
                for (int w = 0; w < W; w++) acc[w] = lds_acc[wave][lane][w];
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (valid && !fullv && (!pull || ishub)) {
            uint64_t nx[W];
            load_mask<W>(NX, v, 0xFu, nx);
            bool nz = false;
#pragma unroll
            for (int w = 0; w < W; w++) {
                acc[w] |= nx[w];
                nz = nz || nx[w] != 0;
            }
            if (nz) {
                const uint64_t zero[W] = {};
                store_mask<W>(NX, v, zero);  // ready for the next level
            }
        }

        uint64_t nw[W], sn[W];
        bool anynew = false;
#pragma unroll
        for (int w = 0; w < W; w++) {
            nw[w] = (valid && !fullv) ? (acc[w] & ~sv[w]) : 0ull;
            sn[w] = sv[w] | nw[w];
            anynew = anynew || (nw[w] != 0);
        }
        if (valid) store_mask<W>(snap, v, sn);
        if (anynew) {
            chg[v] = level;
            wc.farcs += out_rp[v + 1] - out_rp[v];
        }
        const uint64_t changed = __ballot(anynew);
        if (lane == 0) {
            wc.n_new += (int32_t)__popcll(changed);
            chg_out[g] = changed;
        }
        // hub nodes that still miss a bit after this level (the next pull's hub work)
        const uint64_t open = __ballot(valid && ishub && pairs_needed<W>(sn, lastmask) != 0);
        if (lane == 0) wc.hub_open += (int32_t)__popcll(open);
        const bool active = __ballot(valid && !fullv) != 0;
        if (lane == 0) {
            fill_level[g] = level;
            if (!active) gfull[g] = 1;  // all full at the start of this level; masks written full
        }
        if (active && lane == 0) wc.n_out += 1;

        // histogram: lane j accumulates, for word w, how many non-sampled
        // nodes of the group gained bit w*64+j at this level (the column sums
        // of the group's 64 x 64 bit matrix of new bits)
        if (do_hist) {
            const bool counted = anynew && sidx[v] < 0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                const uint64_t x = counted ? nw[w] : 0ull;
                if (!__ballot(x != 0)) continue;
                hcnt[w] += column_count64(x, lane);
            }
        }
    }

    const uint32_t token = flush_counts(wc, cnt);
    if (do_hist) {
#pragma unroll
        for (int w = 0; w < W; w++)
            if (hcnt[w]) atomicAdd(&lds_hist[w * 64 + lane], hcnt[w]);
        __syncthreads();
        const int32_t slot = blockIdx.x % kHistSlotsBatched;
        for (int t = threadIdx.x; t < W * 64; t += kBlock) {
            const int32_t c = lds_hist[t];
            if (c) atomicAdd(&hist[((int64_t)slot * k + src_base + t) * hlen + level], c);
        }
    }
    // the last block to finish decides the next level. Tickets in two steps,
    // so that no address takes an atomic from every block: a block counts in
    // its counter slot, the slot's last block in the control block. The
    // counters are complete then: a block takes its slot ticket only after its
    // counter atomics have returned, and a slot's last block takes the
    // control block's ticket only after the slot's count is complete.
    __shared__ uint32_t last;
    if (threadIdx.x == 0) {
        const uint32_t slot = blockIdx.x % kCounterSlots;
        const uint32_t in_slot = (gridDim.x - slot + kCounterSlots - 1) / kCounterSlots;
        const uint32_t used = gridDim.x < (uint32_t)kCounterSlots ? gridDim.x : (uint32_t)kCounterSlots;
        last = 0;
        if (atomicAdd(&cnt[slot].ticket, 1u + token) == in_slot - 1)
            last = atomicAdd(&ctl->ticket, 1u) == used - 1;
    }
    __syncthreads();
    if (last && threadIdx.x < 64) decide_wave(cnt, ctl, mode_log, level, cap, arcs_total, alpha, n);
}


inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }


template <int W>
int bfs_batched_t(hipStream_t st, const BfsView& gv, int32_t* samples_dev, int32_t kg, int32_t src_base,
                  int32_t k, const BfsLevels& out, const int32_t* sidx, void* scratch, LevelCounters* cnt_dev,
                  TravStats* stats, EventPool* evp) {
    const int64_t n = gv.n;
    const int32_t ngroups = (int32_t)((n + 63) / 64);
    char* p = (char*)scratch;
    uint64_t* NX = (uint64_t*)p;
    p += align256(sizeof(uint64_t) * n * W);
    int32_t* chg = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    uint8_t* gfull = (uint8_t*)p;
    p += align256((size_t)ngroups);
    BfsCtl* ctl = (BfsCtl*)p;
    p += align256(sizeof(BfsCtl));
    int32_t* mode_log = (int32_t*)p;
    p += align256(sizeof(int32_t) * kModeLog);
    uint64_t* chgbits = (uint64_t*)p;  // [2][ngroups]: nodes that changed, by level parity

    const size_t plane = (size_t)n * W;
    const int rem = kg - (W - 1) * 64;
    const uint64_t lastmask = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
    const int64_t hist_elems = out.zero_hist ? (int64_t)kHistSlotsBatched * k * out.hlen : 0;
    const int64_t nmax = std::max<int64_t>(std::max<int64_t>(n, ngroups), std::max<int64_t>(hist_elems, kCounterSlots));
    hipLaunchKernelGGL((k_init<W>), dim3((unsigned)((nmax + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, ngroups,
                       out.snap, NX, chg, gfull, out.fill_level, chgbits, gv.preset, gv.gvalid, cnt_dev,
                       out.zero_flags, out.sidx_fill, out.hist, hist_elems);
    hipLaunchKernelGGL((k_init_samples<W>), dim3(1), dim3(kBlock), 0, st, samples_dev, out.stage_ids,
                       out.stage_caller, out.samples_out, kg, src_base, out.snap, chg,
                       chgbits, gv.out_rp, cnt_dev, out.sidx_fill, ctl, mode_log, out.cap, gv.arcs, gv.alpha, n);
    stats->launches += 2;

    const unsigned gb = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((ngroups + kWaves - 1) / kWaves, std::max(1, gv.level_blocks)));
    const bool enqueue_only = out.enqueue_only > 0;  // for stream capture: no events, reads or waits
    // hubs push by chunks: a prefix of the groups, or the flagged groups of a batch
    const int32_t g0 = (gv.n_push_chunks > 0 && !gv.ghub) ? (int32_t)((gv.nh + 63) / 64) : 0;
    const int64_t scatter_items = std::max<int64_t>(gv.n_hub_chunks, (int64_t)gv.n_push_chunks + (ngroups - g0));
    const unsigned sb = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((scatter_items + kWaves - 1) / kWaves, std::max(1, gv.scatter_blocks)));
    constexpr int32_t kTimedLevels = 256;  // levels whose scatter launch gets its own events
    std::vector<int32_t> modes;
    BfsCtl hc{};
    int32_t level = 1;
    int32_t batch = enqueue_only ? out.enqueue_only : std::max<int32_t>(out.hint, 4);
    if (enqueue_only) evp = nullptr;
    for (;;) {
        const int32_t end = (int32_t)std::min<int64_t>((int64_t)level + batch, out.cap);
        if (evp) CCG_HIP(hipEventRecord(evp->at(0), st));
        for (int32_t L = level; L < end; L++) {
            const uint64_t* Sp = out.snap + (size_t)(L - 1) * plane;  // the previous level's plane
            const bool timed = evp && L < kTimedLevels;
            if (timed) CCG_HIP(hipEventRecord(evp->at(2 + 2 * (size_t)L), st));
            hipLaunchKernelGGL((k_scatter_level<W>), dim3(sb), dim3(kBlock), 0, st, gv.col, gv.hub_chunks,
                               gv.n_hub_chunks, gv.out_rp, gv.out_col, gv.push_chunks, gv.n_push_chunks, g0, ngroups,
                               chg, gv.ghub, n, L - 1, Sp, NX, lastmask, cnt_dev, ctl,
                               (const uint64_t*)(chgbits + (size_t)((L - 1) & 1) * ngroups));
            if (timed) CCG_HIP(hipEventRecord(evp->at(3 + 2 * (size_t)L), st));
            hipLaunchKernelGGL((k_group_level<W>), dim3(gb), dim3(kBlock), 0, st, gv.rp, gv.col, gv.out_rp, Sp,
                               out.snap + (size_t)L * plane, out.fill_level, gfull, chg, ngroups, n, gv.nh, NX,
                               lastmask, L, sidx, out.hist, out.hlen, (int64_t)k, src_base, cnt_dev, ctl, mode_log,
                               out.cap, gv.arcs, gv.alpha, gv.ghub, chgbits + (size_t)(L & 1) * ngroups);
        }
        CCG_HIP(hipGetLastError());
        if (enqueue_only) return 0;
        if (evp) CCG_HIP(hipEventRecord(evp->at(1), st));
        stats->launches += (int64_t)(end - level) * 2;
        stats->kernel_launches += end - level;
        const int32_t lo = std::min(level, kModeLog), hi = std::min(end, kModeLog);
        modes.resize((size_t)std::max(hi, 1));
        CCG_HIP(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
        if (hi > lo)
            CCG_HIP(hipMemcpyAsync(modes.data() + lo, mode_log + lo, sizeof(int32_t) * (hi - lo), hipMemcpyDeviceToHost,
                                   st));
        CCG_HIP(hipStreamSynchronize(st));
        if (evp) {
            float t = 0.f;
            CCG_HIP(hipEventElapsedTime(&t, evp->at(0), evp->at(1)));
            stats->kernel_ms += t;
            for (int32_t L = level; L < std::min(end, kTimedLevels); L++) {
                CCG_HIP(hipEventElapsedTime(&t, evp->at(2 + 2 * (size_t)L), evp->at(3 + 2 * (size_t)L)));
                stats->scatter_ms += t;  // every launch, idle ones past the end included
                stats->scatter_launches += 1;
                if (L <= hc.levels && L < (int32_t)modes.size() && modes[(size_t)L]) stats->pull_scatter_ms += t;
            }
        }
        if (hc.done || end >= out.cap) break;
        level = end;
        batch = std::max<int32_t>(batch * 2, 8);
    }
    stats->levels += hc.levels;
    stats->arcs_scanned += hc.arcs;
    stats->nodes_visited += hc.nodes;
    stats->push_arcs += hc.push_arcs;
    stats->push_atomics += hc.push_atomics;
    stats->hub_arcs += hc.hub_arcs;
    stats->scatter_arcs += hc.hub_arcs + hc.push_arcs;
    stats->pull_levels += hc.pull_levels;
    stats->bfs_levels = std::max<int32_t>(stats->bfs_levels, hc.levels);
    if (!hc.done || hc.status == 1) return 1;  // level-mask capacity exhausted: retry with more levels
    if (hc.status == 2) return 2;              // nodes left that no sample can reach
    if (hc.lmax > stats->maxd) stats->maxd = hc.lmax;
    *out.lmax = std::max(*out.lmax, hc.lmax);
    return 0;
}

}  // namespace

BfsCtl* bfs_batched_ctl(void* scratch, int64_t n, int32_t kg) {
    const int W = (kg + 63) / 64;
    const int64_t ngroups = (n + 63) / 64;
    char* p = (char*)scratch;
    p += align256(sizeof(uint64_t) * n * W) + align256(sizeof(int32_t) * n) + align256((size_t)ngroups);
    return (BfsCtl*)p;
}

size_t bfs_batched_scratch(int64_t n, int32_t kg, int64_t nh) {
    (void)nh;
    const int W = (kg + 63) / 64;
    const int64_t ngroups = (n + 63) / 64;
    return align256(sizeof(uint64_t) * n * W) + align256(sizeof(int32_t) * n) + align256((size_t)ngroups) +
           align256(sizeof(BfsCtl)) + align256(sizeof(int32_t) * kModeLog) + align256(sizeof(uint64_t) * 2 * ngroups) +
           1024;
}

int bfs_batched(hipStream_t st, const BfsView& gv, int32_t* samples_dev, int32_t kg, int32_t src_base,
                int32_t k, const BfsLevels& out, const int32_t* sidx, void* scratch, size_t scratch_size,
                LevelCounters* cnt_dev, TravStats* stats, EventPool* evp) {
    if (scratch_size < bfs_batched_scratch(gv.n, kg, gv.nh)) throw HipError{hipErrorOutOfMemory, "bfs_batched scratch"};
    const int W = (kg + 63) / 64;
    switch (W) {
        case 1: return bfs_batched_t<1>(st, gv, samples_dev, kg, src_base, k, out, sidx, scratch, cnt_dev, stats, evp);
        case 2: return bfs_batched_t<2>(st, gv, samples_dev, kg, src_base, k, out, sidx, scratch, cnt_dev, stats, evp);
        case 3: return bfs_batched_t<3>(st, gv, samples_dev, kg, src_base, k, out, sidx, scratch, cnt_dev, stats, evp);
        default: return bfs_batched_t<4>(st, gv, samples_dev, kg, src_base, k, out, sidx, scratch, cnt_dev, stats, evp);
    }
}

}  // namespace ccg
