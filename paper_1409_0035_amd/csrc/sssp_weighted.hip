// Shortest paths with positive integer arc lengths (the paper's Dijkstra
// runs, Sec. 3, with 32-bit lengths as in Sec. 8) by delta-stepping
// (Meyer & Sanders, J. Algorithms 2003) in its near/far-pile GPU form
// (Davidson, Baxter, Garland & Owens, IPDPS 2014), for many samples at once.
//
// Work items are (sample j, node v) pairs; distances are source-major,
// Dt[j][v] (UINT32_MAX = not reached).  A round relaxes every pair of the
// near pile (tentative distance below the window bound hi): for each arc
// v->u of length w, cand = Dt[j][v] + w is applied with atomicMin; an
// improved pair goes to the next near pile if cand < hi, else to the far pile.
// When a round leaves the near pile empty, the next round splits the far
// pile at a raised bound hi (to the first bucket that holds a far pair): the
// pairs below it are relaxed in that same round, the rest move to the next
// far pile.
// Label-correcting: a pair may be relaxed again after its distance drops,
// and the result is the exact shortest distance when the piles run dry.
//
// Samples of one call share every round, so k samples cost about as many
// rounds as one.  The plain mode calls the same kernel with one sample at a
// time.
//
// Control without host round trips: round r reads the state round r-1 left
// (bound, far-pile buffer, counters; three-slot rings by round) at its start,
// so every block takes the same decision; the host enqueues rounds in batches
// and only checks the done flag between batches.
//
// Duplicates are kept out of the near pile by a flag in the distance word
// itself: during the search Dt holds e = 2d + f, with f = 0 while the pair
// sits in a near pile and f = 1 otherwise.  Taking a pair out of the pile is
// one atomic OR of 1, which returns the distance to relax with; an improver's
// atomic min with 2*cand clears the flag in the same operation and tells the
// improver whether it was the one to clear it (and so must enqueue).  Both
// act on one word, so no relaxation can miss an improvement.  The far pile
// keeps a bit per pair; it is only drained by split rounds.  The last pass
// rewrites Dt to plain distances.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kInf = 0xFFFFFFFFu;        // unreached (encoded and decoded)
constexpr uint32_t kMaxDist = 0x7FFFFFFEu;    // largest distance the encoding (and int32 output) holds

struct WState {
    uint32_t hi;      // window bound for the round that reads this slot
    int32_t epoch;    // far-pile epoch (number of splits so far)
    int32_t done;
    int32_t pad;
};

// Far pile of epoch e: buffer e % 2, size fcnt[e % 3], least distance
// minfar[e % 3]; the split ending epoch e clears the slot of epoch e+2.
struct WDev {
    WState ctl[3];
    int32_t ncnt[3];        // near pile sizes by round (mod 3)
    int32_t fcnt[3];
    uint32_t minfar[3];
    int32_t overflow;
};

__device__ __forceinline__ uint64_t pair_of(int32_t j, int32_t v) { return ((uint64_t)(uint32_t)j << 32) | (uint32_t)v; }

__global__ void k_winit(uint32_t* Dt, int64_t count) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        Dt[t] = kInf;
}

__global__ void k_wzero(uint32_t* p, int64_t count) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0;
}

__global__ void k_wseed(const int32_t* samples, int32_t kg, int64_t n, uint32_t* Dt, uint64_t* N0, WDev* dev,
                        uint32_t delta) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kg) {
        const int64_t v = samples[j];
        Dt[(int64_t)j * n + v] = 0;  // distance 0, in the first near pile
        N0[j] = pair_of(j, (int32_t)v);
    }
    if (j == 0) {
        dev->ctl[0] = WState{delta, 0, 0, 0};
        for (int q = 0; q < 3; q++) {
            dev->ncnt[q] = 0;
            dev->fcnt[q] = 0;
            dev->minfar[q] = kInf;
        }
        dev->ncnt[0] = kg;
        dev->overflow = 0;
    }
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)x, off);
        x = o < x ? o : x;
    }
    return x;
}

// Pile appends are staged in LDS per block and reserved in the global pile
// with one atomic per block and flush (thousands of waves appending to one
// counter would serialise on it).
constexpr int kStage = 1024;

struct Stage {
    uint64_t item[2][kStage];
    int32_t count[2];
    int32_t base[2];
};

__device__ __forceinline__ void stage_put(Stage& S, int q, bool pred, uint64_t item) {
    const uint64_t m = __ballot(pred);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&S.count[q], (int32_t)__popcll(m));
    base = __shfl(base, leader);
    if (pred) S.item[q][base + (int)__popcll(m & lanemask_lt())] = item;
}

// block-uniform: copies the staged items to the global piles and empties the stage
__device__ __forceinline__ void stage_flush(Stage& S, uint64_t* pile0, int32_t* cnt0, uint64_t* pile1, int32_t* cnt1,
                                            int64_t cap, int32_t* overflow) {
    __syncthreads();
    if (threadIdx.x == 0) {
        S.base[0] = S.count[0] ? atomicAdd(cnt0, S.count[0]) : 0;
        S.base[1] = S.count[1] ? atomicAdd(cnt1, S.count[1]) : 0;
    }
    __syncthreads();
    for (int q = 0; q < 2; q++) {
        uint64_t* pile = q == 0 ? pile0 : pile1;
        for (int t = threadIdx.x; t < S.count[q]; t += kBlock) {
            const int64_t pos = (int64_t)S.base[q] + t;
            if (pos < cap) pile[pos] = S.item[q][t];
            else *overflow = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        S.count[0] = 0;
        S.count[1] = 0;
    }
    __syncthreads();
}

// block-uniform: flush when another step could overfill the stage
__device__ __forceinline__ void stage_maybe_flush(Stage& S, uint64_t* pile0, int32_t* cnt0, uint64_t* pile1,
                                                  int32_t* cnt1, int64_t cap, int32_t* overflow) {
    __syncthreads();
    const bool full = S.count[0] > kStage - kBlock || S.count[1] > kStage - kBlock;
    __syncthreads();
    if (full) stage_flush(S, pile0, cnt0, pile1, cnt1, cap, overflow);
}

struct WArgs {
    const uint32_t* rp;
    const int32_t* col;
    const int32_t* wt;
    int64_t n;
    uint32_t* Dt;
    uint32_t* fbit;
    uint64_t* N0;
    uint64_t* N1;
    uint64_t* F0;
    uint64_t* F1;
    int64_t cap;
    WDev* dev;
    uint32_t delta;
    int32_t local_passes;
};

// One round (block-uniform control flow; every block returns normally).
__device__ __forceinline__ void wround_body(const WArgs& A, int32_t r, Stage& S, uint32_t* smax, uint64_t* Wloc,
                                            int32_t* wcount) {
    const uint32_t* __restrict__ rp = A.rp;
    const int32_t* __restrict__ col = A.col;
    const int32_t* __restrict__ wt = A.wt;
    const int64_t n = A.n;
    uint32_t* Dt = A.Dt;
    uint32_t* fbit = A.fbit;
    uint64_t* N0 = A.N0;
    uint64_t* N1 = A.N1;
    uint64_t* F0 = A.F0;
    uint64_t* F1 = A.F1;
    const int64_t cap = A.cap;
    WDev* dev = A.dev;
    const uint32_t delta = A.delta;
    // ---- control for this round, from what round r-1 left
    WState c;
    c.hi = __hip_atomic_load(&dev->ctl[(r + 2) % 3].hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.epoch = __hip_atomic_load(&dev->ctl[(r + 2) % 3].epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.done = __hip_atomic_load(&dev->ctl[(r + 2) % 3].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.pad = 0;
    if (c.done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) dev->ctl[r % 3] = c;  // keep the flag moving round to round
        return;
    }
    // counts can exceed the pile capacity only after an overflow (flagged to
    // the host); never read past the piles
    const int32_t n_in = (int32_t)std::min<int64_t>(
        __hip_atomic_load(&dev->ncnt[(r + 2) % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), cap);
    const int32_t ep = c.epoch;
    const int32_t f_in = (int32_t)std::min<int64_t>(
        __hip_atomic_load(&dev->fcnt[ep % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), cap);
    const bool split = n_in == 0;
    uint32_t hi = c.hi;
    if (split) {
        if (f_in == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) dev->ctl[r % 3] = WState{hi, ep, 1, 0};
            return;
        }
        const uint32_t mf = __hip_atomic_load(&dev->minfar[ep % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t next = ((uint64_t)mf / delta + 1) * (uint64_t)delta;
        const uint64_t step = (uint64_t)hi + delta;
        const uint64_t h = next > step ? next : step;
        hi = h > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)h;
    }
    uint64_t* nin = (r - 1) % 2 == 0 ? N0 : N1;
    uint64_t* nout = r % 2 == 0 ? N0 : N1;
    int32_t* ncnt_out = &dev->ncnt[r % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dev->ctl[r % 3] = WState{hi, split ? ep + 1 : ep, 0, 0};
        dev->ncnt[(r + 1) % 3] = 0;  // output counter of round r+1 (read by round r-1, now idle)
        if (split) {                 // slot of epoch ep+2 (last used by epoch ep-1)
            dev->fcnt[(ep + 2) % 3] = 0;
            dev->minfar[(ep + 2) % 3] = kInf;
        }
    }
    const int64_t items = split ? f_in : n_in;
    const int64_t per_block = ((items + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = std::min<int64_t>(b0 + per_block, items);
    if (b0 >= b1) return;  // block-uniform: nothing for this block
    if (threadIdx.x == 0) {
        S.count[0] = 0;
        S.count[1] = 0;
    }
    __syncthreads();
    uint32_t lmin = kInf;
    // Far appends go to the pile of the round's epoch: a split round opens
    // epoch ep + 1, and the near rounds after it append there too.
    const int32_t epa = split ? ep + 1 : ep;
    uint64_t* fpile = epa % 2 == 0 ? F0 : F1;
    int32_t* fcnt_cur = &dev->fcnt[epa % 3];
    // near round: relax every pair of the near pile; kPairLanes lanes per
    // pair, each taking every kPairLanes-th arc, so a round costs about one
    // chain of dependent atomics instead of one per arc.  Pairs a block finds
    // below the bound are then relaxed by the same block from its stage for up
    // to local_passes more passes before anything is flushed: relaxations may
    // run in any order (label correcting), and improvements travel many hops
    // per launch instead of one.  A split round relaxes the far pairs that fall
    // below its new bound at once, the same way, instead of handing them to
    // the next round.
    constexpr int kPairLanes = 8;
    const int sub = threadIdx.x & (kPairLanes - 1);
    auto relax_batch = [&](auto fetch, int64_t lo, int64_t hi_ix) {
        for (int64_t base = lo; base < hi_ix; base += kBlock / kPairLanes) {
            const int64_t t = base + threadIdx.x / kPairLanes;
            int32_t j = 0, v = 0;
            uint32_t d = kInf, b = 0, e = 0;
            if (t < hi_ix) {
                const uint64_t item = fetch(t);
                j = (int32_t)(item >> 32);
                v = (int32_t)(uint32_t)item;
                const int64_t bit = (int64_t)j * n + v;
                if (sub == 0) d = atomicOr(&Dt[bit], 1u) >> 1;  // leave the pile, read the distance
                b = rp[v];
                e = rp[v + 1];
            }
            d = (uint32_t)__shfl((int)d, lane_id() & ~(kPairLanes - 1));
            uint32_t* drow = Dt + (int64_t)j * n;
            uint32_t mx = e - b;
            for (int off = 32; off > 0; off >>= 1) {
                const uint32_t o = (uint32_t)__shfl_xor((int)mx, off);
                mx = o > mx ? o : mx;
            }
            if (lane_id() == 0) smax[threadIdx.x >> 6] = mx;
            __syncthreads();
            uint32_t maxlen = 0;
            for (int w = 0; w < kBlock / 64; w++) maxlen = smax[w] > maxlen ? smax[w] : maxlen;
            __syncthreads();
            for (uint32_t s0 = 0; s0 < maxlen; s0 += kPairLanes) {
                const uint32_t s = s0 + sub;
                bool to_near = false, to_far = false;
                uint64_t item = 0;
                if (s < e - b) {
                    const int32_t u = col[b + s];
                    const uint64_t cand64 = (uint64_t)d + (uint32_t)wt[b + s];
                    const uint32_t cand = cand64 > kMaxDist ? kMaxDist : (uint32_t)cand64;
                    if (cand64 > kMaxDist) dev->overflow = 1;
                    // a stale cached word only overstates the distance: the
                    // atomic below decides
                    if (cand < (drow[u] >> 1)) {
                        item = pair_of(j, u);
                        if (cand < hi) {
                            const uint32_t enc = cand << 1;  // flag 0: in a near pile
                            const uint32_t old = atomicMin(&drow[u], enc);
                            to_near = (old & 1u) && enc < old;  // this min cleared the flag
                        } else {
                            const uint32_t old = atomicMin(&drow[u], (cand << 1) | 1u);
                            if (cand < (old >> 1)) {
                                const int64_t bit = (int64_t)j * n + u;
                                const uint32_t ob = atomicOr(&fbit[bit >> 5], 1u << (bit & 31));
                                to_far = !(ob & (1u << (bit & 31)));
                                lmin = cand < lmin ? cand : lmin;
                            }
                        }
                    }
                }
                stage_put(S, 0, to_near, item);
                stage_put(S, 1, to_far, item);
                stage_maybe_flush(S, nout, ncnt_out, fpile, fcnt_cur, cap, &dev->overflow);
            }
        }
    };
    if (split) {
        // far pile of epoch ep: pairs below hi not yet in a near pile are
        // relaxed here (chunk by chunk, gathered in Wloc); the rest move to
        // the pile of epoch ep + 1.  Other blocks relax meanwhile, so a word
        // may only drop below what is read here; an improver that lands below
        // hi queues the pair itself.
        uint64_t* fin = ep % 2 == 0 ? F0 : F1;
        for (int64_t c0 = b0; c0 < b1; c0 += kStage) {
            const int64_t c1 = std::min<int64_t>(c0 + kStage, b1);
            __syncthreads();  // every thread has read the last chunk's count
            if (threadIdx.x == 0) *wcount = 0;
            __syncthreads();
            for (int64_t base = c0; base < c1; base += kBlock) {
                const int64_t t = base + threadIdx.x;
                uint64_t item = 0;
                bool take = false, to_far = false;
                if (t < c1) {
                    item = fin[t];
                    const int64_t bit = (int64_t)(item >> 32) * n + (uint32_t)item;
                    atomicAnd(&fbit[bit >> 5], ~(1u << (bit & 31)));
                    const uint32_t e = __hip_atomic_load(&Dt[bit], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t d = e >> 1;
                    if (d < hi) {
                        take = (e & 1u) != 0;  // not in a near pile: relax it now
                    } else {
                        const uint32_t old = atomicOr(&fbit[bit >> 5], 1u << (bit & 31));
                        to_far = !(old & (1u << (bit & 31)));
                        if (to_far) lmin = d < lmin ? d : lmin;
                    }
                }
                const uint64_t m = __ballot(take);
                if (m) {
                    int at = 0;
                    if (lane_id() == 0) at = atomicAdd(wcount, (int)__popcll(m));
                    at = __shfl(at, 0);
                    if (take) Wloc[at + (int)__popcll(m & lanemask_lt())] = item;
                }
                stage_put(S, 1, to_far, item);
                stage_maybe_flush(S, nout, ncnt_out, fpile, fcnt_cur, cap, &dev->overflow);
            }
            __syncthreads();
            const int32_t cnt = *wcount;
            relax_batch([&](int64_t t) { return Wloc[t]; }, 0, cnt);
        }
    } else {
        relax_batch([&](int64_t t) { return nin[t]; }, b0, b1);
    }
    for (int li = 0; li < A.local_passes; li++) {
        __syncthreads();
        const int32_t cnt = S.count[0];
        if (cnt == 0) break;  // block-uniform
        for (int t = threadIdx.x; t < cnt; t += kBlock) Wloc[t] = S.item[0][t];
        __syncthreads();
        if (threadIdx.x == 0) S.count[0] = 0;
        __syncthreads();
        relax_batch([&](int64_t t) { return Wloc[t]; }, 0, cnt);
    }
    stage_flush(S, nout, ncnt_out, fpile, fcnt_cur, cap, &dev->overflow);
    // the smallest far distance: one atomic per block, not per wave, on an
    // address that every block of the round updates
    lmin = wave_min_u32(lmin);
    __syncthreads();  // smax is free again
    if (lane_id() == 0) smax[threadIdx.x >> 6] = lmin;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = kInf;
        for (int w = 0; w < kBlock / 64; w++) m = smax[w] < m ? smax[w] : m;
        if (m != kInf) atomicMin(&dev->minfar[epa % 3], m);
    }
}

__global__ __launch_bounds__(kBlock) void k_wround(WArgs A, int32_t r) {
    __shared__ Stage S;
    __shared__ uint32_t smax[kBlock / 64];
    __shared__ uint64_t Wloc[kStage];
    __shared__ int32_t wcount;
    wround_body(A, r, S, smax, Wloc, &wcount);
}

// Rewrites the search's words 2d + f as plain distances (kInf stays) and
// finds the largest distance and whether any pair was left unreached.
__global__ void k_wmax(uint32_t* Dt, int64_t count, uint32_t* out, int32_t* unreached) {
    __shared__ uint32_t bm[4];
    uint32_t m = 0;
    bool un = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = Dt[t];
        if (e == kInf) {
            un = true;
        } else {
            const uint32_t d = e >> 1;
            Dt[t] = d;
            m = d > m ? d : m;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, off);
        m = o > m ? o : m;
    }
    if (lane_id() == 0) bm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = bm[w] > m ? bm[w] : m;
        m = bm[0] > m ? bm[0] : m;
        atomicMax(out, m);
    }
    if (un) *unreached = 1;
}

// ---------------------------------------------------------------- one workgroup per sample
//
// The batched path runs every sample's search in its own workgroup of one
// launch: near/far delta-stepping on one sample's row, with the near pile,
// the far pile and their counters owned by the workgroup.  Rounds are
// separated by workgroup barriers instead of launches, and the k searches run
// side by side without any host round trip or cross-workgroup
// synchronisation.  A weighted search on a grid takes thousands of rounds
// with frontiers of a few hundred to a few thousand nodes, all on one CU, so
// what a round costs is the CU's memory requests: kGroup lanes take one node
// (its arcs are one or two cache lines), and a node costs one atomic to leave
// the pile, its arc range, its arcs and one atomic minimum per arc.
// Each node has one 64-bit word W = 4d + f: bit 0 set while the node is in a
// near pile, bit 1 set while it is in the far pile.  An improver's atomic
// minimum with 4c + 1 (near) or 4c + 2 (far) changes the word exactly when
// c < d (an equal distance never queues a node again), and the old word's
// bit tells it whether it was the one to put the node in that pile.
constexpr int kSBlock = 1024;   // threads per sample's workgroup
constexpr int kGroup = 8;       // lanes per node: lane s of a group takes arcs s, s + 8, ...
constexpr int kUnroll = 4;      // nodes a group has in flight at once
constexpr int kLq = 6144;       // near-pile entries kept in LDS (more spill to device memory)
constexpr uint64_t kInfW = ~0ull << 2;  // unreached: largest d, in no pile

struct SearchBufs {
    uint64_t* W;      // [kg][n] words 4d + f
    int32_t* near;    // [kg][2][n] near piles beyond the LDS part
    int32_t* far;     // [kg][2][n] far piles
    int32_t* status;  // [kg]: 0 done, 4 distance overflow, 5 time limit
    int32_t* rounds;  // [kg]: rounds run
    int64_t* work;    // [kg][2]: nodes taken from near piles, arcs relaxed
};

// A sample's words are touched by its own workgroup only, and its phases are
// ordered by workgroup barriers: workgroup-scope atomics suffice.
__device__ __forceinline__ uint64_t wg_min(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t wg_and(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t wg_xor(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int wave_append(int32_t* cnt_lds, bool pred) {
    const uint64_t m = __ballot(pred);
    if (!m) return -1;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt_lds, (int32_t)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + (int)__popcll(m & lanemask_lt()) : -1;
}

__global__ __launch_bounds__(kSBlock) void k_wsearch(const uint32_t* __restrict__ rp, const int2* __restrict__ cw,
                                                      int64_t n,
                                                      const int32_t* __restrict__ samples, SearchBufs B, uint32_t delta,
                                                      uint64_t time_limit) {
    const int32_t j = blockIdx.x;
    uint64_t* W = B.W + (int64_t)j * n;
    int32_t* nsp = B.near + (int64_t)j * 2 * n;
    int32_t* fsp = B.far + (int64_t)j * 2 * n;
    __shared__ int32_t lq[2][kLq];
    __shared__ int32_t s_cnt[2];  // entries of the next near pile; of the current far pile (cumulative)
    __shared__ int32_t s_nq, s_nf, s_qsel, s_fsel, s_stop, s_rounds, s_ovf;
    __shared__ unsigned long long s_taken, s_relaxed;
    __shared__ uint32_t s_hi;
    __shared__ uint32_t s_min[kSBlock / 64];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int sub = lane & (kGroup - 1), glane = lane & ~(kGroup - 1);
    auto put_near = [&](int p, int32_t pos, int32_t v) {
        if (pos < kLq) lq[p][pos] = v;
        else nsp[(int64_t)p * n + pos] = v;
    };
    if (threadIdx.x == 0) {
        const int32_t src = samples[j];
        W[src] = 1;  // distance 0, in the first near pile
        put_near(0, 0, src);
        s_nq = 1;
        s_nf = 0;
        s_qsel = 0;
        s_fsel = 0;
        s_hi = delta;
        s_stop = 0;
        s_ovf = 0;
        s_rounds = 0;
        s_cnt[0] = s_cnt[1] = 0;
        s_taken = s_relaxed = 0;
    }
    __syncthreads();
    const uint64_t t0 = wall_clock64();
    constexpr int kPerWave = 64 / kGroup;  // nodes a wave takes at a time
    uint64_t my_taken = 0, my_relaxed = 0;  // work counters (the roofline's bytes)
    for (;;) {
        const int32_t nq = s_nq;
        const uint32_t hi = s_hi;
        const int pin = s_qsel, pout = s_qsel ^ 1;
        int32_t* fpile = fsp + (int64_t)s_fsel * n;
        if (nq > 0) {
            // ---- a near round: relax every node of the pile, kGroup lanes per node and
            // kUnroll nodes per group at a time, so that the takes, the arc loads and the
            // atomic minima of kUnroll nodes are in flight together
            for (int32_t base = wave * kPerWave * kUnroll; base < nq; base += (kSBlock / 64) * kPerWave * kUnroll) {
                int32_t v[kUnroll];
                uint64_t d[kUnroll];
                uint32_t b[kUnroll], e[kUnroll];
                bool valid[kUnroll];
#pragma unroll
                for (int r = 0; r < kUnroll; r++) {
                    const int32_t t = base + r * kPerWave + lane / kGroup;
                    valid[r] = t < nq;
                    v[r] = valid[r] ? (t < kLq ? lq[pin][t] : nsp[(int64_t)pin * n + t]) : 0;
                    d[r] = 0;
                    b[r] = e[r] = 0;
                }
#pragma unroll
                for (int r = 0; r < kUnroll; r++) {
                    // lane 0 of the group leaves the pile (reading d), lanes 1, 2 read the arc range
                    if (valid[r]) {
                        if (sub == 0) {
                            d[r] = wg_and(&W[v[r]], ~1ull) >> 2;
                            my_taken++;
                        }
                        else if (sub == 1) b[r] = rp[v[r]];
                        else if (sub == 2) e[r] = rp[v[r] + 1];
                    }
                }
                uint32_t trips = 0;
#pragma unroll
                for (int r = 0; r < kUnroll; r++) {
                    d[r] = (uint64_t)__shfl((long long)d[r], glane);
                    b[r] = (uint32_t)__shfl((int)b[r], glane + 1);
                    e[r] = (uint32_t)__shfl((int)e[r], glane + 2);
                    if (valid[r]) trips = max(trips, (e[r] - b[r] + kGroup - 1) / kGroup);
                }
                // the wave's trip count: its longest arc list (every lane takes part in the appends)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) trips = max(trips, (uint32_t)__shfl_xor((int)trips, off));
                for (uint32_t it = 0; it < trips; it++) {
                    int32_t u[kUnroll];
                    uint64_t c[kUnroll], o[kUnroll];
#pragma unroll
                    for (int r = 0; r < kUnroll; r++) {
                        const uint32_t a = b[r] + it * kGroup + sub;
                        u[r] = -1;
                        c[r] = 0;
                        if (valid[r] && a < e[r]) {
                            const int2 x = cw[a];  // the arc's end and length, one 8-byte load
                            u[r] = x.x;
                            c[r] = d[r] + (uint32_t)x.y;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kUnroll; r++) {
                        o[r] = 0;
                        if (u[r] >= 0) {
                            my_relaxed++;
                            if (c[r] > kMaxDist) s_ovf = 1;
                            o[r] = wg_min(&W[u[r]], (c[r] << 2) | (c[r] < hi ? 1ull : 2ull));
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kUnroll; r++) {
                        const bool better = u[r] >= 0 && c[r] < (o[r] >> 2);
                        const bool nr = c[r] < hi;
                        const int pn = wave_append(&s_cnt[0], better && nr && !(o[r] & 1ull));  // this minimum queued it
                        if (pn >= 0) put_near(pout, pn, u[r]);
                        const int pf = wave_append(&s_cnt[1], better && !nr && !(o[r] & 2ull));
                        if (pf >= 0) fpile[pf] = u[r];
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_nq = s_cnt[0];
                s_nf = s_cnt[1];
                s_cnt[0] = 0;
                s_qsel ^= 1;
                s_rounds++;
                if (s_ovf || wall_clock64() - t0 > time_limit) s_stop = 1;
            }
            __syncthreads();
            if (s_stop) break;
            continue;
        }
        // ---- the near pile is empty: split the far pile at the next bucket
        const int32_t nf = s_nf;
        if (nf == 0) break;  // uniform: the search is over
        // the least far distance not below hi (entries below hi were settled
        // in the rounds of this bucket)
        uint64_t m = kMaxDist + 1ull;
        for (int32_t t = threadIdx.x; t < nf; t += kSBlock) {
            const uint64_t dv = __hip_atomic_load(&W[fpile[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 2;
            if (dv >= hi && dv < m) m = dv;
        }
        uint32_t m32 = (uint32_t)m;
        m32 = wave_min_u32(m32);
        if (lane == 0) s_min[wave] = m32;
        if (threadIdx.x == 0) s_cnt[1] = 0;  // the far pile is rebuilt from here
        __syncthreads();
        uint32_t mm = kInf;
        for (int w = 0; w < kSBlock / 64; w++) mm = s_min[w] < mm ? s_min[w] : mm;
        const uint64_t nh = mm > kMaxDist ? (uint64_t)hi : ((uint64_t)mm / delta + 1) * (uint64_t)delta;
        const uint32_t nhi = nh > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)nh;
        int32_t* fnext = fsp + (int64_t)(s_fsel ^ 1) * n;
        for (int32_t base = wave * 64; base < nf; base += kSBlock) {
            const int32_t t = base + lane;
            const bool valid = t < nf;
            const int32_t v = valid ? fpile[t] : 0;
            bool to_near = false, keep = false;
            if (valid) {
                const uint64_t dv = __hip_atomic_load(&W[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 2;
                if (dv >= nhi) keep = true;
                else if (dv >= hi) to_near = (wg_xor(&W[v], 3ull) & 3ull) == 2ull;  // far pile -> near pile
                // else settled in an earlier bucket: dropped
            }
            const int pn = wave_append(&s_cnt[0], to_near);
            if (pn >= 0) put_near(pin, pn, v);  // the near pile is empty: refill it
            const int pk = wave_append(&s_cnt[1], keep);
            if (pk >= 0) fnext[pk] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_nq = s_cnt[0];
            s_nf = s_cnt[1];
            s_cnt[0] = 0;
            s_fsel ^= 1;
            s_hi = nhi;
            if (wall_clock64() - t0 > time_limit) s_stop = 1;
        }
        __syncthreads();
        if (s_stop) break;
    }
    atomicAdd(&s_taken, (unsigned long long)my_taken);
    atomicAdd(&s_relaxed, (unsigned long long)my_relaxed);
    __syncthreads();
    if (threadIdx.x == 0) {
        B.status[j] = s_ovf ? 4 : (s_stop ? 5 : 0);
        B.rounds[j] = s_rounds;
        B.work[2 * j] = (int64_t)s_taken;
        B.work[2 * j + 1] = (int64_t)s_relaxed;
    }
}

// The searches' words as plain distances into Dt (kInf = unreached), the
// largest distance and whether any node was left unreached.
__global__ void k_wdecode(const uint64_t* __restrict__ W, uint32_t* Dt, int64_t count, uint32_t* out,
                          int32_t* unreached) {
    __shared__ uint32_t bm[4];
    uint32_t m = 0;
    bool un = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = W[t];
        if (x == kInfW) {
            un = true;
            Dt[t] = kInf;
        } else {
            const uint32_t d = (uint32_t)(x >> 2);
            Dt[t] = d;
            m = d > m ? d : m;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, off);
        m = o > m ? o : m;
    }
    if (lane_id() == 0) bm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = bm[w] > m ? bm[w] : m;
        m = bm[0] > m ? bm[0] : m;
        atomicMax(out, m);
    }
    if (un) *unreached = 1;
}

__global__ void k_wfill64(uint64_t* p, int64_t count, uint64_t value) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = value;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t sssp_weighted_scratch(int64_t n, int32_t kg) {
    const int64_t pairs = n * kg;
    return align256(sizeof(WDev)) + align256((size_t)((pairs + 31) / 32) * 4) + 4 * align256((size_t)pairs * 8) +
           align256(16) + 1024;
}

__global__ void k_zip_arcs(const int32_t* __restrict__ col, const int32_t* __restrict__ w, int64_t arcs, int2* out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < arcs; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = make_int2(col[e], w[e]);
}

void zip_arcs(hipStream_t st, const int32_t* col, const int32_t* w, int64_t arcs, int2* out) {
    if (arcs <= 0) return;
    hipLaunchKernelGGL(k_zip_arcs, dim3((unsigned)std::min<int64_t>((arcs + 255) / 256, 65536)), dim3(256), 0, st, col, w,
                       arcs, out);
}

size_t sssp_wsearch_scratch(int64_t n, int32_t kg) {
    return align256((size_t)kg * n * 8) + 2 * align256((size_t)kg * 2 * n * 4) + 2 * align256((size_t)kg * 4) +
           align256((size_t)kg * 16) + align256(16) + 1024;
}

// A captured estimate's searches: the launches of sssp_weighted_batched
// without its host reads.  The searches' status and the decode's largest
// distance and unreached flag are folded on the device into the job's flags
// and *maxd_out, which a replay reads back.
__global__ void k_wfold(const int32_t* __restrict__ status, int32_t kg, const uint32_t* __restrict__ mx,
                        DevFlags* flags, uint32_t* maxd_out) {
    for (int32_t q = threadIdx.x; q < kg; q += blockDim.x) {
        const int32_t st = status[q];
        if (st == 4) flags->overflow = 1;
        else if (st == 5) flags->timeout = 1;
    }
    if (threadIdx.x == 0) {
        if (mx[1]) flags->disconnected = 1;
        *maxd_out = mx[0];
    }
}

static SearchBufs carve_search(void* scratch, int64_t n, int32_t kg, uint32_t** mx) {
    char* p = (char*)scratch;
    SearchBufs B;
    B.W = (uint64_t*)p;
    p += align256((size_t)n * kg * 8);
    B.near = (int32_t*)p;
    p += align256((size_t)kg * 2 * n * 4);
    B.far = (int32_t*)p;
    p += align256((size_t)kg * 2 * n * 4);
    B.status = (int32_t*)p;
    p += align256((size_t)kg * 4);
    B.rounds = (int32_t*)p;
    p += align256((size_t)kg * 4);
    B.work = (int64_t*)p;
    p += align256((size_t)kg * 16);
    *mx = (uint32_t*)p;
    return B;
}

static uint64_t search_time_limit() {
    int rate_khz = 0, device = 0;
    CCG_HIP(hipGetDevice(&device));
    CCG_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device));
    return (uint64_t)std::max(rate_khz, 1) * 120000ull;  // two minutes
}

void sssp_weighted_batched_enqueue(hipStream_t st, const uint32_t* rp, const int2* cw, int64_t n,
                                   const int32_t* samples_dev, int32_t kg, uint32_t* Dt, uint32_t delta,
                                   void* scratch, size_t scratch_size, DevFlags* flags, uint32_t* maxd_out) {
    if (scratch_size < sssp_wsearch_scratch(n, kg)) throw HipError{hipErrorOutOfMemory, "sssp_weighted_batched scratch"};
    if (delta < 1) delta = 1;
    uint32_t* mx = nullptr;
    const SearchBufs B = carve_search(scratch, n, kg, &mx);
    const int64_t pairs = n * kg;
    const unsigned gz = (unsigned)std::min<int64_t>((pairs + 255) / 256, 65536);
    hipLaunchKernelGGL(k_wfill64, dim3(gz), dim3(256), 0, st, B.W, pairs, kInfW);
    hipLaunchKernelGGL(k_wsearch, dim3((unsigned)kg), dim3(kSBlock), 0, st, rp, cw, n, samples_dev, B, delta,
                       search_time_limit());
    hipLaunchKernelGGL(k_wzero, dim3(1), dim3(64), 0, st, mx, (int64_t)2);
    hipLaunchKernelGGL(k_wdecode, dim3((unsigned)std::min<int64_t>(gz, 1024)), dim3(256), 0, st, B.W, Dt, pairs, mx,
                       (int32_t*)(mx + 1));
    hipLaunchKernelGGL(k_wfold, dim3(1), dim3(256), 0, st, (const int32_t*)B.status, kg, (const uint32_t*)mx, flags,
                       maxd_out);
    CCG_HIP(hipGetLastError());
}

// The k searches of a batched estimate, one workgroup each (k_wsearch), into
// Dt[j][v] (device, source-major rows of length n).  Returns 0 = done, 2 =
// unreached node, 4 = a distance beyond 2^31 - 2, 5 = the time limit expired.
int sssp_weighted_batched(hipStream_t st, const uint32_t* rp, const int2* cw, int64_t n, const int32_t* samples_dev,
                          int32_t kg, uint32_t* Dt, uint32_t delta, void* scratch, size_t scratch_size, int64_t* maxd,
                          TravStats* stats) {
    if (scratch_size < sssp_wsearch_scratch(n, kg)) throw HipError{hipErrorOutOfMemory, "sssp_weighted_batched scratch"};
    if (delta < 1) delta = 1;
    uint32_t* mx = nullptr;
    const SearchBufs B = carve_search(scratch, n, kg, &mx);
    const int64_t pairs = n * kg;
    const unsigned gz = (unsigned)std::min<int64_t>((pairs + 255) / 256, 65536);
    hipLaunchKernelGGL(k_wfill64, dim3(gz), dim3(256), 0, st, B.W, pairs, kInfW);
    // a search that has not finished after two minutes is stopped and reported
    const uint64_t limit = search_time_limit();
    KernelTimer kt;
    kt.start(st);
    hipLaunchKernelGGL(k_wsearch, dim3((unsigned)kg), dim3(kSBlock), 0, st, rp, cw, n, samples_dev, B, delta, limit);
    CCG_HIP(hipGetLastError());
    kt.stop(st);
    std::vector<int32_t> hs((size_t)kg * 2);
    std::vector<int64_t> hw((size_t)kg * 2);
    CCG_HIP(hipMemcpyAsync(hs.data(), B.status, sizeof(int32_t) * kg, hipMemcpyDeviceToHost, st));
    CCG_HIP(hipMemcpyAsync(hs.data() + kg, B.rounds, sizeof(int32_t) * kg, hipMemcpyDeviceToHost, st));
    CCG_HIP(hipMemcpyAsync(hw.data(), B.work, sizeof(int64_t) * kg * 2, hipMemcpyDeviceToHost, st));
    CCG_HIP(hipStreamSynchronize(st));
    for (int32_t q = 0; q < kg; q++) {
        stats->nodes_visited += hw[(size_t)2 * q];
        stats->arcs_scanned += hw[(size_t)2 * q + 1];
    }
    stats->kernel_ms += kt.ms();
    stats->kernel_launches += 1;
    stats->launches += 3;
    int32_t rmax = 0, bad = 0;
    for (int32_t q = 0; q < kg; q++) {
        rmax = std::max(rmax, hs[(size_t)kg + q]);
        if (hs[(size_t)q] != 0) bad = hs[(size_t)q];
    }
    stats->levels += rmax;
    if (bad) return bad;
    hipLaunchKernelGGL(k_wzero, dim3(1), dim3(64), 0, st, mx, (int64_t)2);
    hipLaunchKernelGGL(k_wdecode, dim3((unsigned)std::min<int64_t>(gz, 1024)), dim3(256), 0, st, B.W, Dt, pairs, mx,
                       (int32_t*)(mx + 1));
    uint32_t hm[2];
    CCG_HIP(hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, st));
    CCG_HIP(hipStreamSynchronize(st));
    *maxd = std::max<int64_t>(*maxd, hm[0]);
    return hm[1] ? 2 : 0;
}

// Distances from samples[0..kg) (device, internal ids) into Dt[j][v] (device,
// source-major rows of length n), every round a launch over the whole device
// (the plain path: one sample per call).  Returns 0 = done, 2 = unreached
// node, 4 = overflow (distance or pile capacity).
int sssp_weighted(hipStream_t st, const uint32_t* rp, const int32_t* col, const int32_t* w, int64_t n,
                  const int32_t* samples_dev, int32_t kg, uint32_t* Dt, const WeightedShape& shape, void* scratch,
                  size_t scratch_size, int64_t* maxd, TravStats* stats) {
    uint32_t delta = shape.delta;
    if (scratch_size < sssp_weighted_scratch(n, kg)) throw HipError{hipErrorOutOfMemory, "sssp_weighted scratch"};
    const int64_t pairs = n * kg;
    char* p = (char*)scratch;
    WDev* dev = (WDev*)p;
    p += align256(sizeof(WDev));
    uint32_t* fbit = (uint32_t*)p;
    p += align256((size_t)((pairs + 31) / 32) * 4);
    uint64_t* N0 = (uint64_t*)p;
    p += align256((size_t)pairs * 8);
    uint64_t* N1 = (uint64_t*)p;
    p += align256((size_t)pairs * 8);
    uint64_t* F0 = (uint64_t*)p;
    p += align256((size_t)pairs * 8);
    uint64_t* F1 = (uint64_t*)p;
    p += align256((size_t)pairs * 8);
    uint32_t* mx = (uint32_t*)p;
    if (delta < 1) delta = 1;

    const int64_t words = (pairs + 31) / 32;
    const unsigned gz = (unsigned)std::min<int64_t>((pairs + 255) / 256, 65536);
    hipLaunchKernelGGL(k_winit, dim3(gz), dim3(256), 0, st, Dt, pairs);
    hipLaunchKernelGGL(k_wzero, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 65536)), dim3(256), 0, st, fbit,
                       words);
    hipLaunchKernelGGL(k_wseed, dim3((kg + 63) / 64), dim3(64), 0, st, samples_dev, kg, n, Dt, N0, dev, delta);
    stats->launches += 3;

    WArgs A{rp, col, w, n, Dt, fbit, N0, N1, F0, F1, pairs, dev, delta, std::max(0, shape.local_passes)};
    const unsigned round_blocks = (unsigned)std::max(1, shape.round_blocks);
    WDev host;
    KernelTimer kt;
    // every round settles or moves at least one pair; far more rounds than
    // pairs means the control state is broken -- stop instead of spinning
    const int64_t max_rounds = std::min<int64_t>(4 * n + 10000, (int64_t)1 << 22);

    {
    int32_t r = 1;
    int batch = 16;
    for (;;) {
        kt.start(st);
        for (int q = 0; q < batch; q++, r++) {
            hipLaunchKernelGGL(k_wround, dim3(round_blocks), dim3(kBlock), 0, st, A, r);
        }
        CCG_HIP(hipGetLastError());
        kt.stop(st);
        CCG_HIP(hipMemcpyAsync(&host, dev, sizeof(WDev), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        stats->kernel_ms += kt.ms();
        stats->kernel_launches += batch;
        stats->launches += batch;
        if (host.overflow) return 4;
        if (host.ctl[(r + 2) % 3].done) break;  // the last round enqueued found nothing to do
        if (r > max_rounds) return 4;
        if (batch < 256) batch *= 2;
    }
    stats->levels += r - 1;
    }
    hipLaunchKernelGGL(k_wzero, dim3(1), dim3(64), 0, st, mx, (int64_t)2);
    hipLaunchKernelGGL(k_wmax, dim3((unsigned)std::min<int64_t>(gz, 1024)), dim3(256), 0, st, Dt, pairs, mx,
                       (int32_t*)(mx + 1));
    uint32_t hm[2];
    CCG_HIP(hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, st));
    CCG_HIP(hipStreamSynchronize(st));
    *maxd = std::max<int64_t>(*maxd, hm[0]);
    return hm[1] ? 2 : 0;
}

}  // namespace ccg
