// Outbound / inbound reachability sampling (Sec. 6.2, Algorithm 4) on graphs
// with unit arc lengths.
//
// For every node v the estimate needs the bottom-k sample of its reachability
// set R(v) (the nodes u != v that v reaches, outbound, or that reach v,
// inbound) under a uniformly random rank order of the nodes: the k members of
// R(v) ranked first, their distance sum, and the position T of the k-th among
// V \ {v}.  As in Algorithm 4, sources are taken in rank order and each one's
// search runs on the transposed direction (outbound: from u to the nodes that
// reach u), adding u to the sample of every node it meets; a node that holds
// enough lower-ranked members stops the search.
//
// Batched here: up to 64W sources of consecutive ranks advance together as
// one bit-parallel BFS (bit b = the b-th source of the batch, so bit order is
// rank order).  The first batches are smaller (128, 256, then 512 sources): while
// every node still collects, each extra word costs on every arc, whereas the
// later batches touch few nodes and are bound by the fixed cost of a cycle,
// so fewer, larger batches pay off there.  Kernels touch only the words the
// current batch uses.  The stopping rule is the exact one, not Algorithm 4's
// printed count-equals-k test (which loses members a node reaching x needs): a node x
// stops source u when x holds at least k + 1 members ranked before u,
// counting x itself when it ranks before u -- then every node reaching x has k
// such members other than itself and none of them needs u.  Inside a batch x
// counts only the bits it has already seen, so it may stop later than the
// sequential searches would, never earlier.  Nodes that hold more than k such
// members from earlier batches take no part.
//
// A source that already holds more than k members of its own, or that has no
// propagation arc (outbound: no node has an arc into it), can pass its bit to
// nobody, so it is skipped: a batch takes the next sources in rank order that
// can still pass their bit (bit order stays rank order, and every source
// skipped between them would have reached no node).
//
// Batches run as a state machine over three kernels that the host enqueues in
// cycles without reading anything back: push (frontier nodes OR their
// allowed bits into their neighbours' pending words), merge (new bits, their
// BFS level, the bits each node passes on next), account (after the last
// level: each touched node takes the first bits it still needs, in rank order,
// and adds their levels; then its last block picks and starts the next
// batch).  The control block says which kernel has work; the others return at
// once.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr int32_t kFirstBatch = 128;  // sources in the first batch; doubled per batch up to 64W
// Frontier entries are chunks of at most kChunk propagation arcs of a node
// (node << 32 | offset of the chunk's first arc), so a node with a huge
// degree is spread over many waves instead of holding up the level in one.
constexpr uint32_t kChunk = 256;

__host__ __device__ inline int64_t frontier_cap(int64_t n, int64_t arcs) { return n + arcs / kChunk + 1; }

enum : int32_t { kLevel = 1, kAccount = 2, kFinished = 3 };

struct ReachCtl {
    int32_t phase;
    int32_t batch;
    int64_t t0;      // rank of the batch's first source
    int64_t tnext;   // first entry of the list of sources with propagation arcs not yet looked at
    int32_t nsrc;    // sources in the batch
    int32_t level;   // BFS level of the bits the next merge records
    int32_t gl;      // global level stamp (first touch of a node per level)
    int32_t fsel;    // current frontier buffer
    int32_t nf;      // frontier size
    int32_t nfn;     // next frontier size
    int32_t nc;      // candidates of this level
    int32_t nt;      // nodes touched in this batch
    uint32_t ticket;
    int32_t overflow;  // a recorded level above 65535
    int32_t nw;        // words the current batch uses
    int64_t levels;  // levels run, all batches
    int64_t nact;    // sources with propagation arcs (the list's length)
};

struct ReachView {
    int64_t n;
    int64_t nsrc;  // ranked sources (n, or the nodes of positive weight)
    int32_t k;
    const uint32_t* rp;   // propagation arcs: from a node to the nodes its bits move to
    const int32_t* col;
    const int32_t* rank;         // internal id -> rank
    const int32_t* src_by_rank;  // rank -> internal id
    int32_t* act_src;            // [nsrc] the sources that have propagation arcs, in rank order
    int32_t* act_rank;           // [nsrc] their ranks
    int32_t* act_blk;            // per-chunk counts of such sources, then the chunks' offsets
    int32_t* src_rank;           // [64W] rank of each bit's source in the current batch
    int32_t* sbit;               // [n] the node's bit when it is a source of the current batch, else -1
    int32_t* cnt;       // members counted so far (exact up to k)
    int64_t* dsum;      // distance sum of the first min(k, cnt) members
    int64_t* tk;        // T once the k-th member is found
    uint64_t* seen;     // [n][W] bits of this batch at the node
    uint64_t* nx;       // [n][W] pending bits of this level
    uint64_t* fr;       // [n][W] bits the node passes on next level
    uint16_t* lev;      // [n][64W] level at which each bit arrived (open nodes)
    int32_t* stamp;     // batch that last touched the node
    int32_t* lmark;     // level stamp that last queued the node
    uint64_t* flist;    // [2][fcap] frontier chunk lists
    int64_t fcap;
    int32_t* cand;      // [n] nodes with pending bits this level
    int32_t* touched;   // [n] nodes touched in this batch
    // node-weighted sampling (Algorithm 5): the first k-1 members of each
    // node's sample and their distances (null for Algorithm 4)
    int32_t* mem_id;    // [n][k-1]
    uint16_t* mem_d;    // [n][k-1]
};

// Members ranked before the current batch that x holds, plus one when x
// itself ranks before the batch (every node ranked before it was a source of
// an earlier batch or was skipped).
__device__ __forceinline__ int64_t held_before(const ReachView& V, int64_t x, int64_t t0) {
    return (int64_t)V.cnt[x] + (V.rank[x] < t0 ? 1 : 0);
}

// The q lowest set bits of the W-word set s (all of them when s has fewer).
template <int W>
__device__ __forceinline__ void first_bits(const uint64_t (&s)[W], int64_t q, uint64_t (&out)[W]) {
#pragma unroll
    for (int j = 0; j < W; j++) {
        const uint64_t x = s[j];
        const int pc = __popcll(x);
        if (q <= 0) {
            out[j] = 0;
        } else if (q >= pc) {
            out[j] = x;
            q -= pc;
        } else {
            // position of the q-th set bit: halve the window while the low half holds fewer than q
            uint64_t y = x;
            int pos = 0;
            int r = (int)q;
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) {
                const int c = __popcll(y & ((1ull << sh) - 1));
                if (c < r) {
                    r -= c;
                    y >>= sh;
                    pos += sh;
                }
            }
            out[j] = x & (pos == 63 ? ~0ull : ((2ull << pos) - 1));
            q = 0;
        }
    }
}

// List appends staged per wave in LDS: one global atomic per flush instead of
// one per wave and call (hundreds of thousands of waves appending to one
// counter serialise on it).  put() and flush() are called with every lane of
// the wave active, so the count stays the same in all lanes.
constexpr int kWaveStage = 512;

struct WaveList {
    int32_t* items;  // this wave's LDS segment of kWaveStage entries
    int32_t* gcount;
    int32_t* glist;
    int32_t count;
    __device__ __forceinline__ void flush() {
        if (count == 0) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(gcount, count);
        base = __shfl(base, 0);
        for (int t = lane_id(); t < count; t += 64) glist[base + t] = items[t];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        count = 0;
    }
    __device__ __forceinline__ void put(bool pred, int32_t x) {
        const uint64_t m = __ballot(pred);
        if (!m) return;
        const int c = (int)__popcll(m);
        if (count + c > kWaveStage) flush();
        if (pred) items[count + (int)__popcll(m & lanemask_lt())] = x;
        count += c;
    }
};

template <int W>
__global__ __launch_bounds__(kBlock) void k_rch_push(ReachCtl* ctl, ReachView V) {
    if (ctl->phase != kLevel) return;
    const int32_t nf = ctl->nf;
    const uint64_t* F = V.flist + (int64_t)ctl->fsel * V.fcap;
    const int32_t gl = ctl->gl;
    const int64_t t0 = ctl->t0;
    const int32_t nwa = ctl->nw;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    __shared__ int32_t stage[kBlock / 64][kWaveStage];
    WaveList cand{stage[wave], &ctl->nc, V.cand, 0};
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t e = (int64_t)blockIdx.x * (kBlock / 64) + wave; e < nf; e += nwaves) {
        const uint64_t ent = F[e];
        const int64_t v = (int64_t)(ent >> 32);
        uint64_t f[W];
#pragma unroll
        for (int j = 0; j < W; j++) f[j] = j < nwa ? V.fr[v * W + j] : 0ull;
        const uint32_t a0 = V.rp[v] + (uint32_t)ent, a1 = min(V.rp[v + 1], a0 + kChunk);
        for (uint32_t base = a0; base < a1; base += 64) {  // same trip count in every lane
            const uint32_t a = base + lane;
            int64_t w = 0;
            bool first = false;
            if (a < a1) w = V.col[a];
            // a node holding more than k earlier members takes no part
            if (a < a1 && held_before(V, w, t0) <= V.k) {
                uint64_t any = 0;
#pragma unroll
                for (int j = 0; j < W; j++) {
                    if (!f[j]) continue;
                    const uint64_t b = f[j] & ~V.seen[w * W + j];
                    if (!b) continue;
                    any |= b;
                    // only bits not already pending need the atomic, so a popular
                    // target stops taking atomics once it holds the level's bits
                    // (a stale read only lets a redundant atomic through)
                    const uint64_t r =
                        b & ~__hip_atomic_load(&V.nx[w * W + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (r) atomicOr((unsigned long long*)&V.nx[w * W + j], (unsigned long long)r);
                }
                if (any && V.lmark[w] != gl) first = atomicExch(&V.lmark[w], gl) != gl;
            }
            cand.put(first, (int32_t)w);
        }
    }
    cand.flush();
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_rch_merge(ReachCtl* ctl, ReachView V) {
    if (ctl->phase != kLevel) return;
    const int32_t nc = ctl->nc;
    const int32_t level = ctl->level;
    const int32_t batch = ctl->batch;
    const int64_t t0 = ctl->t0;
    const int32_t nwa = ctl->nw;
    uint64_t* Fn = V.flist + (int64_t)(ctl->fsel ^ 1) * V.fcap;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    __shared__ int32_t stage[kBlock / 64][kWaveStage];
    WaveList tl{stage[wave], &ctl->nt, V.touched, 0};
    bool ovf = false;
    // same trip count in every lane of a block (the lists are appended to with every lane active)
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < nc; i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
        bool touch = false, pass = false;
        const int64_t w = i < nc ? V.cand[i] : 0;
        if (i < nc) {
            uint64_t nw[W], s[W];
            uint64_t any = 0;
#pragma unroll
            for (int j = 0; j < W; j++) {
                nw[j] = 0;
                s[j] = 0;
                if (j >= nwa) continue;
                const uint64_t p = V.nx[w * W + j];
                const uint64_t old = V.seen[w * W + j];
                nw[j] = p & ~old;
                s[j] = old | nw[j];
                if (p) V.nx[w * W + j] = 0;
                if (nw[j]) V.seen[w * W + j] = s[j];
                any |= nw[j];
            }
            if (V.stamp[w] != batch) {  // each candidate appears once per level
                V.stamp[w] = batch;
                touch = true;
            }
            if (any) {
                const int64_t held = held_before(V, w, t0);
                if (V.cnt[w] < V.k) {  // still collecting members: remember when each bit arrived
                    if (level > 65535) ovf = true;
#pragma unroll
                    for (int j = 0; j < W; j++) {
                        uint64_t x = nw[j];
                        while (x) {
                            const int b = __ffsll((unsigned long long)x) - 1;
                            x &= x - 1;
                            V.lev[w * (64 * W) + j * 64 + b] = (uint16_t)level;
                        }
                    }
                }
                // bit b moves on while the members ranked before it number at most k
                uint64_t keep[W];
                first_bits<W>(s, (int64_t)V.k - held + 1, keep);
                uint64_t fa = 0;
#pragma unroll
                for (int j = 0; j < W; j++) {
                    if (j >= nwa) continue;
                    const uint64_t f = nw[j] & keep[j];
                    V.fr[w * W + j] = f;
                    fa |= f;
                }
                pass = fa != 0;
            }
        }
        tl.put(touch, (int32_t)w);
        // the next frontier: the node's propagation arcs in chunks (none if it has no arcs)
        uint32_t c = 0;
        if (pass) c = (V.rp[w + 1] - V.rp[w] + kChunk - 1) / kChunk;
        uint32_t incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
            if (lane >= off) incl += y;
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, 63);
        int32_t base = 0;
        if (lane == 0 && total) base = atomicAdd(&ctl->nfn, (int32_t)total);
        base = __shfl(base, 0);
        for (uint32_t q = 0; q < c; q++) Fn[base + (incl - c) + q] = ((uint64_t)w << 32) | (q * kChunk);
    }
    tl.flush();
    if (ovf) ctl->overflow = 1;
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        ctl->ticket = 0;
        const int32_t nn = atomicAdd(&ctl->nfn, 0);
        ctl->nf = nn;
        ctl->nfn = 0;
        ctl->nc = 0;
        ctl->fsel ^= 1;
        ctl->level = level + 1;
        ctl->gl = ctl->gl + 1;
        ctl->levels = ctl->levels + 1;
        if (nn == 0) ctl->phase = kAccount;
        __threadfence();
    }
}

// The last block of account starts the next batch: it scans ranks from tnext
// for up to cap sources that can still pass their bit, in rank order.
template <int W>
__device__ void start_batch(ReachCtl* ctl, const ReachView& V) {
    __shared__ int32_t wcount[kBlock / 64];
    __shared__ int32_t got;
    __shared__ int64_t scan, first_rank, last_idx;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int32_t batch = ctl->batch;  // 1 for the first batch
    const int32_t cap = (int32_t)std::min<int64_t>(64 * W, (int64_t)kFirstBatch << std::min(batch - 1, 16));
    uint64_t* F = V.flist + (int64_t)ctl->fsel * V.fcap;
    if (threadIdx.x == 0) {
        got = 0;
        scan = ctl->tnext;
    }
    __syncthreads();
    constexpr int kPer = 16;  // ranks per thread and window
    // the scan runs over the sources that have propagation arcs (listed once
    // per estimate, in rank order): a source without any passes its bit to no one
    const int64_t nact = ctl->nact;
    while (got < cap && scan < nact) {
        // kPer x 256 entries per window from `scan` rounded down to a multiple of
        // kPer (entries before `scan` are not taken); thread t takes entries
        // w0 + t*kPer .. +kPer-1, 16-byte loads, so the window stays in rank order
        const int64_t w0 = scan & ~(int64_t)(kPer - 1);
        const int64_t i0 = w0 + (int64_t)threadIdx.x * kPer;
        int64_t s[kPer];
        int32_t rk[kPer];
        bool take[kPer];
        int32_t mine = 0;
        if (i0 + kPer <= nact) {  // the lists are 256-byte aligned and i0 is a multiple of kPer
#pragma unroll
            for (int c = 0; c < kPer / 4; c++) {
                const int4 a = *(const int4*)(V.act_src + i0 + 4 * c);
                const int4 b = *(const int4*)(V.act_rank + i0 + 4 * c);
                s[4 * c] = a.x, s[4 * c + 1] = a.y, s[4 * c + 2] = a.z, s[4 * c + 3] = a.w;
                rk[4 * c] = b.x, rk[4 * c + 1] = b.y, rk[4 * c + 2] = b.z, rk[4 * c + 3] = b.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                s[q] = i0 + q < nact ? V.act_src[i0 + q] : -1;
                rk[q] = i0 + q < nact ? V.act_rank[i0 + q] : 0;
            }
        }
#pragma unroll
        for (int q = 0; q < kPer; q++)
            if (i0 + q < scan) s[q] = -1;
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            take[q] = s[q] >= 0 && V.cnt[s[q]] <= V.k;
            mine += take[q] ? 1 : 0;
        }
        // exclusive prefix of `mine` over the block
        int32_t incl = mine;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wcount[wave] = incl;
        __syncthreads();
        int32_t b = got + incl - mine;
        for (int w = 0; w < wave; w++) b += wcount[w];
        int32_t total = got;
        for (int w = 0; w < kBlock / 64; w++) total += wcount[w];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            if (!take[q]) continue;
            if (b < cap) {
                const int64_t x = s[q];
                const uint64_t bit = 1ull << (b & 63);
                if (b == 0) first_rank = rk[q];
                if (b == cap - 1) last_idx = i0 + q;
                V.src_rank[b] = rk[q];
                V.sbit[x] = b;
                V.seen[x * W + (b >> 6)] = bit;
                V.stamp[x] = batch;
                V.fr[x * W + (b >> 6)] = bit;
                V.touched[b] = (int32_t)x;
            }
            b++;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (total >= cap) {  // the batch is full: continue after its last source
                scan = last_idx + 1;
                got = cap;
            } else {
                scan = w0 + (int64_t)kBlock * kPer;
                got = total;
            }
        }
        __syncthreads();
    }
    // the first frontier: the sources' propagation arcs in chunks, in source
    // order; thread t takes sources t*kSrc .. +kSrc-1 (64W <= kSrc * kBlock)
    constexpr int kSrc = (64 * W + kBlock - 1) / kBlock;
    const int32_t S = got;
    int64_t xs[kSrc];
    uint32_t cs[kSrc];
    uint32_t mine_c = 0;
#pragma unroll
    for (int q = 0; q < kSrc; q++) {
        const int32_t b = threadIdx.x * kSrc + q;
        xs[q] = b < S ? V.touched[b] : 0;
        cs[q] = b < S ? (V.rp[xs[q] + 1] - V.rp[xs[q]] + kChunk - 1) / kChunk : 0;
        mine_c += cs[q];
    }
    uint32_t incl = mine_c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wcount[wave] = (int32_t)incl;
    __syncthreads();
    int32_t nfe = 0, pos = (int32_t)(incl - mine_c);
    for (int w = 0; w < kBlock / 64; w++) {
        if (w < wave) pos += wcount[w];
        nfe += wcount[w];
    }
#pragma unroll
    for (int q = 0; q < kSrc; q++)
        for (uint32_t c = 0; c < cs[q]; c++) F[pos++] = ((uint64_t)xs[q] << 32) | (c * kChunk);
    if (threadIdx.x == 0) {
        ctl->tnext = scan < nact ? scan : nact;
        ctl->nsrc = S;
        ctl->nw = (S + 63) / 64;
        ctl->nt = S;
        ctl->nf = nfe;
        ctl->nfn = 0;
        ctl->nc = 0;
        ctl->level = 1;
        ctl->t0 = S > 0 ? first_rank : V.n;
        ctl->phase = S > 0 ? kLevel : kFinished;
        __threadfence();
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_rch_account(ReachCtl* ctl, ReachView V) {
    if (ctl->phase != kAccount) return;
    const int32_t nt = ctl->nt;
    const int32_t k = V.k;
    const int32_t nwa = ctl->nw;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nt; i += (int64_t)gridDim.x * kBlock) {
        const int64_t w = V.touched[i];
        uint64_t s[W];
#pragma unroll
        for (int j = 0; j < W; j++) {  // fr is a subset of seen: clear both where seen has bits
            s[j] = j < nwa ? V.seen[w * W + j] : 0ull;
            if (s[j]) {
                V.seen[w * W + j] = 0;
                V.fr[w * W + j] = 0;
            }
        }
        const int64_t r = V.rank[w];
        const int32_t own = V.sbit[w];
        if (own >= 0) {  // its own bit counts nothing for itself
            s[own >> 6] &= ~(1ull << (own & 63));
            V.sbit[w] = -1;
        }
        int32_t pc = 0;
#pragma unroll
        for (int j = 0; j < W; j++) pc += __popcll(s[j]);
        const int32_t c = V.cnt[w];
        if (c < k) {  // members in rank order until it holds k
            const int32_t need = k - c;
            uint64_t take[W];
            first_bits<W>(s, need, take);
            int32_t taken = 0;
            int64_t sum = 0, last_rk = -1;
#pragma unroll
            for (int j = 0; j < W; j++) {
                uint64_t x = take[j];
                while (x) {
                    // up to eight members at a time, their loads in flight together
                    int32_t bb[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        bb[u] = x ? __ffsll((unsigned long long)x) - 1 : -1;
                        x &= x - 1;
                    }
                    uint16_t lv[8];
                    int32_t rk[8], src[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        lv[u] = bb[u] >= 0 ? V.lev[w * (64 * W) + j * 64 + bb[u]] : (uint16_t)0;
                        rk[u] = bb[u] >= 0 ? V.src_rank[j * 64 + bb[u]] : 0;
                    }
                    if (V.mem_id) {
#pragma unroll
                        for (int u = 0; u < 8; u++) src[u] = bb[u] >= 0 ? V.src_by_rank[rk[u]] : 0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        if (bb[u] < 0) continue;
                        sum += lv[u];
                        if (V.mem_id) {  // Algorithm 5: keep the member, or the k-th's id
                            const int32_t slot = c + taken;
                            if (slot < k - 1) {
                                V.mem_id[w * (k - 1) + slot] = src[u];
                                V.mem_d[w * (k - 1) + slot] = lv[u];
                            } else {
                                V.tk[w] = src[u];
                            }
                        }
                        taken++;
                        last_rk = rk[u];
                    }
                }
            }
            if (taken == need && !V.mem_id) V.tk[w] = (last_rk + 1) - (r < last_rk ? 1 : 0);
            V.dsum[w] += sum;
        }
        V.cnt[w] = c + pc;
    }
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) {
            ctl->ticket = 0;
            ctl->batch = ctl->batch + 1;
        }
        __syncthreads();
        start_batch<W>(ctl, V);
    }
}

__global__ void k_rch_out(ReachView V, const int32_t* __restrict__ orig, int32_t* count, int64_t* distsum,
                          int64_t* T, double* B, double* R) {
    const int64_t n = V.n;
    const int32_t k = V.k;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = orig[v];
        const int32_t c = V.cnt[v] < k ? V.cnt[v] : k;
        const int64_t ds = V.dsum[v];
        const int64_t t = c == k ? V.tk[v] : 0;
        if (count) count[o] = c;
        if (distsum) distsum[o] = ds;
        if (T) T[o] = t;
        if (B) B[o] = c > 0 ? (double)ds / (double)c : 0.0;
        if (R) {
            double r;
            if (c < k) r = (double)c;
            else if (k == 1) r = 1.0;
            else r = 1.0 + (double)((int64_t)(k - 1) * (n - 2)) / (double)(t - 1);
            R[o] = r;
        }
    }
}

// Algorithm 5's estimates from the kept members: fewer than k, their exact
// weighted sums; else priority sampling's weights max(beta, 1/T) for the
// first k-1 members, T the rank U_k / (2^53 beta_k) of the k-th.
// Member distances are u16 levels (unit lengths) or u32 distances (arc
// lengths); with arc lengths a weighted sum that leaves int64 sets *ovf.
template <typename DT>
__global__ void k_rch_out_beta(ReachView V, const DT* __restrict__ mem_d, const int32_t* __restrict__ orig,
                               const uint32_t* __restrict__ beta, const uint64_t* __restrict__ U, int32_t* count,
                               int32_t* kth, double* S, double* R, int32_t* ovf) {
    const int64_t n = V.n;
    const int32_t k = V.k;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = orig[v];
        const int32_t c = V.cnt[v] < k ? V.cnt[v] : k;
        const int32_t* mi = V.mem_id + v * (k - 1);
        const DT* md = mem_d + v * (k - 1);
        bool bad = false;
        double s, r;
        int32_t q = -1;
        if (c < k) {
            int64_t ss = 0, rr = 0;
            for (int32_t j = 0; j < c; j++) {
                const int64_t b = beta[mi[j]];
                int64_t t;
                bad |= __builtin_mul_overflow(b, (int64_t)md[j], &t);
                bad |= __builtin_add_overflow(ss, t, &ss);
                rr += b;
            }
            s = (double)ss;
            r = (double)rr;
        } else {
            q = (int32_t)V.tk[v];
            const uint64_t Uk = U[q];
            const uint64_t bk = beta[q];
            const double tau = ldexp((double)bk, 53) / (double)Uk;
            int64_t hs = 0, hr = 0, ls = 0, lc = 0;
            for (int32_t j = 0; j < k - 1; j++) {
                const uint64_t b = beta[mi[j]];
                if ((unsigned __int128)b * Uk >= ((unsigned __int128)bk << 53)) {  // heavy: its own weight
                    int64_t t;
                    bad |= __builtin_mul_overflow((int64_t)b, (int64_t)md[j], &t);
                    bad |= __builtin_add_overflow(hs, t, &hs);
                    hr += (int64_t)b;
                } else {
                    ls += md[j];
                    lc += 1;
                }
            }
            s = (double)hs + tau * (double)ls;
            r = (double)hr + tau * (double)lc;
        }
        if (bad) *ovf = 1;
        if (count) count[o] = c;
        if (kth) kth[o] = q >= 0 ? orig[q] : -1;
        if (S) S[o] = s;
        if (R) R[o] = r;
    }
}

__global__ void k_rch_set_phase(ReachCtl* ctl, int32_t phase) { ctl->phase = phase; }

// The sources that have propagation arcs, listed in rank order once per
// estimate, so that picking a batch reads one count per candidate: per-chunk
// counts, one block's exclusive scan of them (which also stores the list's
// length), then each chunk writes its entries in order.
constexpr int kActPer = 16;                                  // ranks per thread
constexpr int64_t kActChunk = (int64_t)kBlock * kActPer;     // ranks per block

__device__ __forceinline__ bool has_arcs(const ReachView& V, int64_t r, int32_t& s) {
    if (r >= V.nsrc) return false;
    s = V.src_by_rank[r];
    return V.rp[s + 1] > V.rp[s];
}

__global__ __launch_bounds__(kBlock) void k_rch_act_count(ReachView V) {
    __shared__ int32_t total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kActChunk + (int64_t)threadIdx.x * kActPer;
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < kActPer; q++) {
        int32_t s;
        c += has_arcs(V, base + q, s) ? 1 : 0;
    }
    atomicAdd(&total, c);
    __syncthreads();
    if (threadIdx.x == 0) V.act_blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_rch_act_scan(ReachCtl* ctl, ReachView V, int32_t nb) {
    __shared__ int32_t wcount[kBlock / 64];
    __shared__ int64_t carry;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t t0 = 0; t0 < nb; t0 += kBlock) {
        const int32_t i = t0 + (int32_t)threadIdx.x;
        const int32_t v = i < nb ? V.act_blk[i] : 0;
        int32_t incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wcount[wave] = incl;
        __syncthreads();
        int64_t before = carry;
        int64_t tile = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            if (w < wave) before += wcount[w];
            tile += wcount[w];
        }
        if (i < nb) V.act_blk[i] = (int32_t)(before + incl - v);
        __syncthreads();
        if (threadIdx.x == 0) carry += tile;
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->nact = carry;
}

__global__ __launch_bounds__(kBlock) void k_rch_act_put(ReachView V) {
    __shared__ int32_t wcount[kBlock / 64];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kActChunk + (int64_t)threadIdx.x * kActPer;
    int32_t s[kActPer];
    bool f[kActPer];
    int32_t mine = 0;
#pragma unroll
    for (int q = 0; q < kActPer; q++) {
        s[q] = 0;
        f[q] = has_arcs(V, base + q, s[q]);
        mine += f[q] ? 1 : 0;
    }
    int32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wcount[wave] = incl;
    __syncthreads();
    int64_t pos = (int64_t)V.act_blk[blockIdx.x] + incl - mine;
    for (int w = 0; w < wave; w++) pos += wcount[w];
#pragma unroll
    for (int q = 0; q < kActPer; q++) {
        if (!f[q]) continue;
        V.act_src[pos] = s[q];
        V.act_rank[pos] = (int32_t)(base + q);
        pos++;
    }
}

__global__ void k_rch_rank(const int32_t* __restrict__ order_internal, int64_t n, int32_t* __restrict__ rank) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        rank[order_internal[r]] = (int32_t)r;
}


// ---- Algorithms 4 and 5 on graphs with arc lengths -------------------------
//
// The listing runs a pruned Dijkstra from each source in rank order.  Here a
// batch of sources of consecutive ranks (those that can still pass their
// membership on, as above) searches at once, one workgroup per source: the
// near/far delta-stepping of the estimate's weighted searches on the
// source's own row of 64-bit words 4d + flags (bit 0: in a near pile, bit 1:
// in the far pile).  A search does not enter a node that holds more than k
// members ranked before the batch (counting the node itself when it ranks
// before it): every node that reaches such a node through it has k members
// ranked before every source of the batch, so it needs none of them, and
// the shortest path from a source to a node that needs it never passes such
// a node.  Inside a batch a node counts only the earlier batches' members,
// so a search may run on where the sequential searches would stop, never the
// other way.  A node entered by a source for the first time joins the
// batch's touched list once (a batch stamp per node).
// Then one thread per touched node reads the batch's words at the node in
// rank order, takes the first sources it still needs (its own aside), adds
// their distances (or keeps them, Algorithm 5) and clears the words; the
// last block picks the next batch.
constexpr int kLBlock = 1024;  // threads per source's workgroup
constexpr int kLGroup = 8;     // lanes per node
constexpr int kLUnroll = 4;    // nodes a lane group has in flight
constexpr int kLLq = 4096;     // near-pile entries kept in LDS
constexpr int32_t kLFirstBatch = 128;
constexpr uint64_t kLInfW = ~0ull << 2;
constexpr uint64_t kLMaxDist = 0x7FFFFFFEull;
enum : int32_t { kLSearch = 1, kLFinished = 3 };

struct LenCtl {
    ReachCtl rc;          // phase, batch, t0, tnext, nsrc, nt, ticket, overflow, levels, nact
    int32_t timeout;      // a search ran past its time limit
    int32_t pad;
    uint64_t relaxed;     // arcs relaxed, all searches
};

struct LenView {
    int64_t n;
    int32_t k;
    int32_t smax;                // sources per batch at most (workgroups per search launch)
    const uint32_t* rp;          // propagation arcs
    const int2* cw;              // their (end, length) pairs
    const int32_t* rank;         // internal id -> rank (INT32_MAX: never a source)
    const int32_t* act_src;      // sources with propagation arcs, in rank order
    const int32_t* act_rank;
    int32_t* cnt;                // members counted so far (exact up to k)
    int64_t* dsum;
    int64_t* tk;
    uint64_t* W;                 // [smax][n] words, all 4d + flags = kLInfW between batches
    int32_t* near;               // [smax][2][n]
    int32_t* far;                // [smax][2][n]
    int32_t* bsrc;               // [smax] the batch's sources in rank order
    int32_t* brank;              // [smax] their ranks
    int32_t* sbit;               // [n] index of the node in the batch when it is one of its sources, else -1
    int32_t* stamp;              // [n] batch that last touched the node
    int32_t* touched;            // [n] nodes touched in this batch
    int32_t* mem_id;             // Algorithm 5: [n][k-1] the first k-1 members
    uint32_t* mem_d;             // and their distances
    uint32_t delta;
    uint64_t time_limit;         // wall-clock ticks per search
};

__device__ __forceinline__ uint64_t rl_min(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t rl_and(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t rl_xor(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// First touch of node u by a search of this batch: the node joins the list.
__device__ __forceinline__ void rl_touch(LenCtl* lc, const LenView& V, int32_t batch, bool first, int32_t u) {
    bool ins = false;
    if (first) ins = atomicExch(&V.stamp[u], batch) != batch;
    const int pos = wave_append(&lc->rc.nt, ins);
    if (pos >= 0) V.touched[pos] = u;
}

__global__ __launch_bounds__(kLBlock) void k_rl_search(LenCtl* lc, LenView V) {
    ReachCtl* ctl = &lc->rc;
    if (ctl->phase != kLSearch) return;
    const int32_t j = blockIdx.x;
    if (j >= ctl->nsrc) return;
    const int64_t n = V.n;
    const int64_t t0 = ctl->t0;
    const int32_t batch = ctl->batch;
    const int64_t k = V.k;
    const uint32_t delta = V.delta;
    uint64_t* W = V.W + (int64_t)j * n;
    int32_t* nsp = V.near + (int64_t)j * 2 * n;
    int32_t* fsp = V.far + (int64_t)j * 2 * n;
    __shared__ int32_t lq[2][kLLq];
    __shared__ int32_t s_cnt[2];  // entries of the next near pile; of the far pile being built
    __shared__ int32_t s_nq, s_nf, s_qsel, s_fsel, s_stop, s_ovf, s_phases;
    __shared__ uint32_t s_hi;
    __shared__ uint32_t s_min[kLBlock / 64];
    __shared__ unsigned long long s_relaxed;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int sub = lane & (kLGroup - 1), glane = lane & ~(kLGroup - 1);
    auto put_near = [&](int p, int32_t pos, int32_t v) {
        if (pos < kLLq) lq[p][pos] = v;
        else nsp[(int64_t)p * n + pos] = v;
    };
    if (threadIdx.x == 0) {
        const int32_t src = V.bsrc[j];
        W[src] = 1;  // distance 0, in the first near pile
        put_near(0, 0, src);
        s_nq = 1;
        s_nf = 0;
        s_qsel = 0;
        s_fsel = 0;
        s_hi = delta;
        s_stop = 0;
        s_ovf = 0;
        s_phases = 0;
        s_cnt[0] = s_cnt[1] = 0;
        s_relaxed = 0;
    }
    if (wave == 0) rl_touch(lc, V, batch, lane == 0, V.bsrc[j]);  // its word is cleared by the account
    __syncthreads();
    const uint64_t c0 = wall_clock64();
    constexpr int kPerWave = 64 / kLGroup;
    uint64_t my_relaxed = 0;
    for (;;) {
        const int32_t nq = s_nq;
        const uint32_t hi = s_hi;
        const int pin = s_qsel, pout = s_qsel ^ 1;
        int32_t* fpile = fsp + (int64_t)s_fsel * n;
        if (nq > 0) {
            for (int32_t base = wave * kPerWave * kLUnroll; base < nq; base += (kLBlock / 64) * kPerWave * kLUnroll) {
                int32_t v[kLUnroll];
                uint64_t d[kLUnroll];
                uint32_t b[kLUnroll], e[kLUnroll];
                bool valid[kLUnroll];
#pragma unroll
                for (int r = 0; r < kLUnroll; r++) {
                    const int32_t t = base + r * kPerWave + lane / kLGroup;
                    valid[r] = t < nq;
                    v[r] = valid[r] ? (t < kLLq ? lq[pin][t] : nsp[(int64_t)pin * n + t]) : 0;
                    d[r] = 0;
                    b[r] = e[r] = 0;
                }
#pragma unroll
                for (int r = 0; r < kLUnroll; r++) {
                    if (valid[r]) {
                        if (sub == 0) d[r] = rl_and(&W[v[r]], ~1ull) >> 2;  // leaves the near pile
                        else if (sub == 1) b[r] = V.rp[v[r]];
                        else if (sub == 2) e[r] = V.rp[v[r] + 1];
                    }
                }
                uint32_t trips = 0;
#pragma unroll
                for (int r = 0; r < kLUnroll; r++) {
                    d[r] = (uint64_t)__shfl((long long)d[r], glane);
                    b[r] = (uint32_t)__shfl((int)b[r], glane + 1);
                    e[r] = (uint32_t)__shfl((int)e[r], glane + 2);
                    if (valid[r]) trips = max(trips, (e[r] - b[r] + kLGroup - 1) / kLGroup);
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) trips = max(trips, (uint32_t)__shfl_xor((int)trips, off));
                for (uint32_t it = 0; it < trips; it++) {
                    int32_t u[kLUnroll];
                    uint64_t c[kLUnroll], o[kLUnroll];
#pragma unroll
                    for (int r = 0; r < kLUnroll; r++) {
                        const uint32_t a = b[r] + it * kLGroup + sub;
                        u[r] = -1;
                        c[r] = 0;
                        if (valid[r] && a < e[r]) {
                            const int2 x = V.cw[a];
                            u[r] = x.x;
                            c[r] = d[r] + (uint32_t)x.y;
                        }
                    }
                    // a node holding more than k members ranked before the batch takes no part
#pragma unroll
                    for (int r = 0; r < kLUnroll; r++)
                        if (u[r] >= 0 && (int64_t)V.cnt[u[r]] + (V.rank[u[r]] < t0 ? 1 : 0) > k) u[r] = -1;
#pragma unroll
                    for (int r = 0; r < kLUnroll; r++) {
                        o[r] = 0;
                        if (u[r] >= 0) {
                            my_relaxed++;
                            if (c[r] > kLMaxDist) s_ovf = 1;
                            o[r] = rl_min(&W[u[r]], (c[r] << 2) | (c[r] < hi ? 1ull : 2ull));
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kLUnroll; r++) {
                        const bool better = u[r] >= 0 && c[r] < (o[r] >> 2);
                        const bool nr = c[r] < hi;
                        const int pn = wave_append(&s_cnt[0], better && nr && !(o[r] & 1ull));
                        if (pn >= 0) put_near(pout, pn, u[r]);
                        const int pf = wave_append(&s_cnt[1], better && !nr && !(o[r] & 2ull));
                        if (pf >= 0) fpile[pf] = u[r];
                        rl_touch(lc, V, batch, better && o[r] == kLInfW, u[r]);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_nq = s_cnt[0];
                s_nf = s_cnt[1];
                s_cnt[0] = 0;
                s_qsel ^= 1;
                s_phases++;
                if (s_ovf || wall_clock64() - c0 > V.time_limit) s_stop = 1;
            }
            __syncthreads();
            if (s_stop) break;
            continue;
        }
        // the near pile is empty: the next bucket from the far pile
        const int32_t nf = s_nf;
        if (nf == 0) break;
        uint64_t m = kLMaxDist + 1ull;
        for (int32_t t = threadIdx.x; t < nf; t += kLBlock) {
            const uint64_t dv = __hip_atomic_load(&W[fpile[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 2;
            if (dv >= hi && dv < m) m = dv;
        }
        uint32_t m32 = (uint32_t)m;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t y = (uint32_t)__shfl_xor((int)m32, off);
            m32 = y < m32 ? y : m32;
        }
        if (lane == 0) s_min[wave] = m32;
        if (threadIdx.x == 0) s_cnt[1] = 0;
        __syncthreads();
        uint32_t mm = 0xFFFFFFFFu;
        for (int w = 0; w < kLBlock / 64; w++) mm = s_min[w] < mm ? s_min[w] : mm;
        const uint64_t nh = mm > kLMaxDist ? (uint64_t)hi : ((uint64_t)mm / delta + 1) * (uint64_t)delta;
        const uint32_t nhi = nh > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)nh;
        int32_t* fnext = fsp + (int64_t)(s_fsel ^ 1) * n;
        for (int32_t base = wave * 64; base < nf; base += kLBlock) {
            const int32_t t = base + lane;
            const bool ok = t < nf;
            const int32_t v = ok ? fpile[t] : 0;
            bool to_near = false, keep = false;
            if (ok) {
                const uint64_t dv = __hip_atomic_load(&W[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 2;
                if (dv >= nhi) keep = true;
                else if (dv >= hi) to_near = (rl_xor(&W[v], 3ull) & 3ull) == 2ull;  // far pile -> near pile
            }
            const int pn = wave_append(&s_cnt[0], to_near);
            if (pn >= 0) put_near(pin, pn, v);
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
            if (wall_clock64() - c0 > V.time_limit) s_stop = 1;
        }
        __syncthreads();
        if (s_stop) break;
    }
    atomicAdd(&s_relaxed, (unsigned long long)my_relaxed);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&lc->relaxed, s_relaxed);
        atomicAdd((unsigned long long*)&ctl->levels, (unsigned long long)s_phases);
        if (s_ovf) atomicOr(&ctl->overflow, 1);
        else if (s_stop) atomicOr(&lc->timeout, 1);
    }
}

// The last block of the account picks the next batch: up to cap sources of
// the list of sources with propagation arcs, from tnext on, that hold at most
// k members (the others can pass their membership to nobody), in rank order.
__device__ void rl_start_batch(LenCtl* lc, const LenView& V) {
    ReachCtl* ctl = &lc->rc;
    __shared__ int32_t wcount[kBlock / 64];
    __shared__ int32_t got;
    __shared__ int64_t scan, next_scan;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int32_t batch = ctl->batch;  // 1 for the first batch
    const int32_t cap = (int32_t)std::min<int64_t>(V.smax, (int64_t)kLFirstBatch << std::min(batch - 1, 16));
    const int64_t nact = ctl->nact;
    if (threadIdx.x == 0) {
        got = 0;
        scan = ctl->tnext;
    }
    __syncthreads();
    while (got < cap && scan < nact) {
        const int64_t i = scan + threadIdx.x;
        int32_t s = -1, rk = 0;
        bool take = false;
        if (i < nact) {
            s = V.act_src[i];
            rk = V.act_rank[i];
            take = V.cnt[s] <= V.k;
        }
        const uint64_t m = __ballot(take);
        if (lane == 0) wcount[wave] = (int32_t)__popcll(m);
        if (threadIdx.x == 0) next_scan = scan + kBlock;
        __syncthreads();
        int32_t pos = got + (int32_t)__popcll(m & lanemask_lt());
        int32_t total = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            if (w < wave) pos += wcount[w];
            total += wcount[w];
        }
        if (take && pos < cap) {
            V.bsrc[pos] = s;
            V.brank[pos] = rk;
            V.sbit[s] = pos;
        }
        if (take && pos == cap - 1) next_scan = i + 1;  // the batch is full: go on after its last source
        __syncthreads();
        if (threadIdx.x == 0) {
            got = got + total < cap ? got + total : cap;
            scan = next_scan;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->tnext = scan < nact ? scan : nact;
        ctl->nsrc = got;
        ctl->nt = 0;
        ctl->t0 = got > 0 ? V.brank[0] : V.n;
        ctl->phase = got > 0 ? kLSearch : kLFinished;
        __threadfence();
    }
}

// Runs after every search launch: the batch that launch searched (none
// before the first) is accounted, then the next one is picked.
__global__ __launch_bounds__(kBlock) void k_rl_account(LenCtl* lc, LenView V) {
    ReachCtl* ctl = &lc->rc;
    if (ctl->phase != kLSearch) return;
    const int32_t nt = ctl->nt;
    const int32_t S = ctl->nsrc;
    const int32_t k = V.k;
    const int64_t n = V.n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nt; i += (int64_t)gridDim.x * kBlock) {
        const int64_t y = V.touched[i];
        const int32_t own = V.sbit[y];
        if (own >= 0) V.sbit[y] = -1;  // its own search counts nothing for itself
        const int32_t c = V.cnt[y];
        const int64_t r = V.rank[y];
        int32_t pc = 0, taken = 0;
        int64_t sum = 0, last_rk = -1;
        for (int32_t j0 = 0; j0 < S; j0 += 8) {
            uint64_t x[8];
#pragma unroll
            for (int q = 0; q < 8; q++) x[q] = j0 + q < S ? V.W[(int64_t)(j0 + q) * n + y] : kLInfW;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                if (x[q] == kLInfW) continue;
                const int32_t jj = j0 + q;
                V.W[(int64_t)jj * n + y] = kLInfW;
                if (jj == own) continue;
                pc++;
                if (c + taken < k) {  // the members it still needs, in rank order
                    const uint32_t dd = (uint32_t)(x[q] >> 2);
                    sum += dd;
                    if (V.mem_id) {  // Algorithm 5: keep the member, or the k-th's id
                        const int32_t slot = c + taken;
                        if (slot < k - 1) {
                            V.mem_id[y * (k - 1) + slot] = V.bsrc[jj];
                            V.mem_d[y * (k - 1) + slot] = dd;
                        } else {
                            V.tk[y] = V.bsrc[jj];
                        }
                    }
                    taken++;
                    last_rk = V.brank[jj];
                }
            }
        }
        if (c < k) {
            if (c + taken == k && !V.mem_id) V.tk[y] = (last_rk + 1) - (r < last_rk ? 1 : 0);
            V.dsum[y] += sum;
        }
        V.cnt[y] = c + pc;
    }
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&ctl->ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) {
            ctl->ticket = 0;
            ctl->batch = ctl->batch + 1;
        }
        __syncthreads();
        rl_start_batch(lc, V);
    }
}

__global__ void k_rl_fill64(uint64_t* p, int64_t count, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

size_t reach_scratch_bytes(int64_t n, int64_t arcs, int32_t k_weighted) {
    constexpr int W = kReachWords;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t i32 = al(sizeof(int32_t) * n), i64 = al(sizeof(int64_t) * n);
    const size_t kw = (size_t)std::max(1, k_weighted - 1);
    const size_t nb = (size_t)((n + kActChunk - 1) / kActChunk) + 1;
    return al(sizeof(ReachCtl)) + 2 * i32 /* rank, src_by_rank */ + 2 * i32 /* act_src, act_rank */ +
           al(sizeof(int32_t) * nb) /* act_blk */ + i32 + 2 * i64 /* cnt, dsum, tk */ +
           3 * al(sizeof(uint64_t) * n * W) /* seen, nx, fr */ + al(sizeof(uint16_t) * n * 64 * W) /* lev */ +
           3 * i32 /* stamp, lmark, sbit */ + al(sizeof(int32_t) * 64 * W) /* src_rank */ +
           (k_weighted > 0 ? al(sizeof(int32_t) * n * kw) + al(sizeof(uint16_t) * n * kw) : 0) +
           al(sizeof(uint64_t) * 2 * (size_t)frontier_cap(n, arcs)) /* flist */ + 2 * i32 /* cand, touched */ + 1024;
}

size_t reach_len_scratch_bytes(int64_t n, int32_t sources, int32_t k_weighted) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t i32 = al(sizeof(int32_t) * n), i64 = al(sizeof(int64_t) * n);
    const size_t kw = (size_t)std::max(1, k_weighted - 1);
    const size_t nb = (size_t)((n + kActChunk - 1) / kActChunk) + 1;
    const size_t S = (size_t)std::max(1, sources);
    return al(sizeof(LenCtl)) + 4 * i32 /* rank, src_by_rank, act_src, act_rank */ + al(sizeof(int32_t) * nb) +
           i32 + 2 * i64 /* cnt, dsum, tk */ + al(sizeof(uint64_t) * S * n) /* W */ +
           2 * al(sizeof(int32_t) * S * 2 * n) /* near, far */ + 2 * al(sizeof(int32_t) * S) /* bsrc, brank */ +
           3 * i32 /* sbit, stamp, touched */ +
           (k_weighted > 0 ? al(sizeof(int32_t) * n * kw) + al(sizeof(uint32_t) * n * kw) : 0) + 1024;
}

// Algorithms 4 and 5 with arc lengths (the kernels above): batches of
// searches, one workgroup per source, then the account, enqueued in cycles
// that read nothing back until a chunk of them has run.
static void run_reach_lengths(hipStream_t st, const ReachArgs& a, void* scratch, size_t scratch_size,
                              ReachStats* stats) {
    const int64_t n = a.n;
    const bool weighted = a.beta != nullptr;
    const int32_t S = std::max(1, a.len_sources);
    if (scratch_size < reach_len_scratch_bytes(n, S, weighted ? a.k : 0))
        throw HipError{hipErrorOutOfMemory, "reach (arc lengths) scratch"};
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char* p = (char*)scratch;
    auto take = [&](size_t bytes) {
        char* q = p;
        p += al(bytes);
        return (void*)q;
    };
    LenCtl* lc = (LenCtl*)take(sizeof(LenCtl));
    LenView V{};
    V.n = n;
    V.k = a.k;
    V.smax = S;
    V.rp = a.rp;
    V.cw = a.cw;
    V.delta = std::max<uint32_t>(1, a.delta);
    int32_t* rank = (int32_t*)take(sizeof(int32_t) * n);
    int32_t* sbr = (int32_t*)take(sizeof(int32_t) * n);
    int32_t* act_src = (int32_t*)take(sizeof(int32_t) * n);
    int32_t* act_rank = (int32_t*)take(sizeof(int32_t) * n);
    int32_t* act_blk = (int32_t*)take(sizeof(int32_t) * ((size_t)((n + kActChunk - 1) / kActChunk) + 1));
    V.rank = rank;
    V.act_src = act_src;
    V.act_rank = act_rank;
    V.cnt = (int32_t*)take(sizeof(int32_t) * n);
    V.dsum = (int64_t*)take(sizeof(int64_t) * n);
    V.tk = (int64_t*)take(sizeof(int64_t) * n);
    V.W = (uint64_t*)take(sizeof(uint64_t) * (size_t)S * n);
    V.near = (int32_t*)take(sizeof(int32_t) * (size_t)S * 2 * n);
    V.far = (int32_t*)take(sizeof(int32_t) * (size_t)S * 2 * n);
    V.bsrc = (int32_t*)take(sizeof(int32_t) * S);
    V.brank = (int32_t*)take(sizeof(int32_t) * S);
    V.sbit = (int32_t*)take(sizeof(int32_t) * n);
    V.stamp = (int32_t*)take(sizeof(int32_t) * n);
    V.touched = (int32_t*)take(sizeof(int32_t) * n);
    if (weighted) {
        V.mem_id = (int32_t*)take(sizeof(int32_t) * n * std::max(1, a.k - 1));
        V.mem_d = (uint32_t*)take(sizeof(uint32_t) * n * std::max(1, a.k - 1));
    }
    int rate_khz = 0, device = 0;
    CCG_HIP(hipGetDevice(&device));
    CCG_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device));
    V.time_limit = (uint64_t)std::max(rate_khz, 1) * 120000ull;  // two minutes per search

    // the rank order and the list of sources with propagation arcs, as in the unit-length path
    ReachView R{};
    R.n = n;
    R.nsrc = a.nsrc > 0 ? a.nsrc : n;
    R.k = a.k;
    R.rp = a.rp;
    R.rank = rank;
    R.src_by_rank = sbr;
    R.act_src = act_src;
    R.act_rank = act_rank;
    R.act_blk = act_blk;
    R.cnt = V.cnt;
    R.dsum = V.dsum;
    R.tk = V.tk;
    R.mem_id = V.mem_id;
    if (a.order_dev)
        CCG_HIP(hipMemcpyAsync(sbr, a.order_dev, sizeof(int32_t) * R.nsrc, hipMemcpyDeviceToDevice, st));
    else
        CCG_HIP(hipMemcpyAsync(sbr, a.order, sizeof(int32_t) * R.nsrc, hipMemcpyHostToDevice, st));
    const unsigned gn = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    fill_u32(st, rank, 0x7FFFFFFFu, (size_t)n);
    hipLaunchKernelGGL(k_rch_rank, dim3(gn), dim3(256), 0, st, (const int32_t*)sbr, R.nsrc, rank);
    fill_u32(st, V.cnt, 0u, (size_t)n);
    fill_u32(st, V.dsum, 0u, (size_t)n * 2);
    fill_u32(st, V.tk, 0u, (size_t)n * 2);
    fill_u32(st, V.sbit, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, V.stamp, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, lc, 0u, sizeof(LenCtl) / 4);
    const int64_t words = (int64_t)S * n;
    hipLaunchKernelGGL(k_rl_fill64, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((words + 255) / 256, 65536))),
                       dim3(256), 0, st, V.W, words, kLInfW);
    const int32_t nb = (int32_t)((R.nsrc + kActChunk - 1) / kActChunk);
    if (nb > 0) {
        hipLaunchKernelGGL(k_rch_act_count, dim3((unsigned)nb), dim3(kBlock), 0, st, R);
        hipLaunchKernelGGL(k_rch_act_scan, dim3(1), dim3(kBlock), 0, st, &lc->rc, R, nb);
        hipLaunchKernelGGL(k_rch_act_put, dim3((unsigned)nb), dim3(kBlock), 0, st, R);
    }
    // start with an empty batch: the first search launch finds nothing to do and
    // the account after it picks the first batch
    hipLaunchKernelGGL(k_rch_set_phase, dim3(1), dim3(1), 0, st, &lc->rc, (int32_t)kLSearch);
    CCG_HIP(hipGetLastError());

    const unsigned ga = (unsigned)std::max(1, a.account_blocks);
    const int64_t max_cycles = R.nsrc + 4;  // every batch but the last takes at least one source
    int64_t cycles = 0;
    int32_t chunk = 4;
    LenCtl hc{};
    for (;;) {
        for (int32_t c = 0; c < chunk; c++) {
            hipLaunchKernelGGL(k_rl_search, dim3((unsigned)S), dim3(kLBlock), 0, st, lc, V);
            hipLaunchKernelGGL(k_rl_account, dim3(ga), dim3(kBlock), 0, st, lc, V);
        }
        CCG_HIP(hipGetLastError());
        cycles += chunk;
        CCG_HIP(hipMemcpyAsync(&hc, lc, sizeof(hc), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        if (hc.rc.phase == kLFinished || hc.rc.overflow || hc.timeout) break;
        if (cycles > max_cycles) throw HipError{hipErrorLaunchTimeOut, "reachability sampling did not finish"};
        if (chunk < 64) chunk *= 2;
    }
    if (!hc.rc.overflow && !hc.timeout) {
        if (weighted)
            hipLaunchKernelGGL(k_rch_out_beta<uint32_t>, dim3(gn), dim3(256), 0, st, R, (const uint32_t*)V.mem_d,
                               a.orig, a.beta, a.U, a.count, a.kth, a.S_w, a.R, &lc->rc.overflow);
        else
            hipLaunchKernelGGL(k_rch_out, dim3(gn), dim3(256), 0, st, R, a.orig, a.count, a.distsum, a.T, a.B, a.R);
        CCG_HIP(hipGetLastError());
        CCG_HIP(hipMemcpyAsync(&hc, lc, sizeof(hc), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
    }
    if (stats) {
        stats->cycles = cycles;
        stats->batches = hc.rc.batch;
        stats->levels = hc.rc.levels;
        stats->overflow = hc.rc.overflow != 0;
        stats->timeout = hc.timeout != 0;
        stats->relaxed = (int64_t)hc.relaxed;
    }
}

void run_reach(hipStream_t st, const ReachArgs& a, void* scratch, size_t scratch_size, ReachStats* stats) {
    if (a.cw) {
        run_reach_lengths(st, a, scratch, scratch_size, stats);
        return;
    }
    constexpr int W = kReachWords;
    const int64_t n = a.n;
    const bool weighted = a.beta != nullptr;
    if (scratch_size < reach_scratch_bytes(n, a.arcs, weighted ? a.k : 0))
        throw HipError{hipErrorOutOfMemory, "reach scratch"};
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char* p = (char*)scratch;
    auto take = [&](size_t bytes) {
        char* q = p;
        p += al(bytes);
        return (void*)q;
    };
    ReachCtl* ctl = (ReachCtl*)take(sizeof(ReachCtl));
    ReachView V{};
    V.n = n;
    V.nsrc = a.nsrc > 0 ? a.nsrc : n;
    V.k = a.k;
    V.rp = a.rp;
    V.col = a.col;
    int32_t* rank = (int32_t*)take(sizeof(int32_t) * n);
    int32_t* sbr = (int32_t*)take(sizeof(int32_t) * n);
    V.rank = rank;
    V.src_by_rank = sbr;
    const int32_t nb = (int32_t)((V.nsrc + kActChunk - 1) / kActChunk);
    V.act_src = (int32_t*)take(sizeof(int32_t) * n);
    V.act_rank = (int32_t*)take(sizeof(int32_t) * n);
    V.act_blk = (int32_t*)take(sizeof(int32_t) * ((size_t)((n + kActChunk - 1) / kActChunk) + 1));
    V.cnt = (int32_t*)take(sizeof(int32_t) * n);
    V.dsum = (int64_t*)take(sizeof(int64_t) * n);
    V.tk = (int64_t*)take(sizeof(int64_t) * n);
    V.seen = (uint64_t*)take(sizeof(uint64_t) * n * W);
    V.nx = (uint64_t*)take(sizeof(uint64_t) * n * W);
    V.fr = (uint64_t*)take(sizeof(uint64_t) * n * W);
    V.lev = (uint16_t*)take(sizeof(uint16_t) * n * 64 * W);
    V.stamp = (int32_t*)take(sizeof(int32_t) * n);
    V.lmark = (int32_t*)take(sizeof(int32_t) * n);
    V.sbit = (int32_t*)take(sizeof(int32_t) * n);
    V.src_rank = (int32_t*)take(sizeof(int32_t) * 64 * W);
    if (weighted) {
        V.mem_id = (int32_t*)take(sizeof(int32_t) * n * std::max(1, a.k - 1));
        V.mem_d = (uint16_t*)take(sizeof(uint16_t) * n * std::max(1, a.k - 1));
    }
    V.fcap = frontier_cap(n, a.arcs);
    V.flist = (uint64_t*)take(sizeof(uint64_t) * 2 * (size_t)V.fcap);
    V.cand = (int32_t*)take(sizeof(int32_t) * n);
    V.touched = (int32_t*)take(sizeof(int32_t) * n);

    if (a.order_dev)
        CCG_HIP(hipMemcpyAsync(sbr, a.order_dev, sizeof(int32_t) * V.nsrc, hipMemcpyDeviceToDevice, st));
    else
        CCG_HIP(hipMemcpyAsync(sbr, a.order, sizeof(int32_t) * V.nsrc, hipMemcpyHostToDevice, st));
    const unsigned gn = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    fill_u32(st, rank, 0x7FFFFFFFu, (size_t)n);  // nodes that are never sources rank after all
    hipLaunchKernelGGL(k_rch_rank, dim3(gn), dim3(256), 0, st, (const int32_t*)sbr, V.nsrc, rank);
    fill_u32(st, V.cnt, 0u, (size_t)n);
    fill_u32(st, V.dsum, 0u, (size_t)n * 2);
    fill_u32(st, V.tk, 0u, (size_t)n * 2);
    fill_u32(st, V.seen, 0u, (size_t)n * W * 2);
    fill_u32(st, V.nx, 0u, (size_t)n * W * 2);
    fill_u32(st, V.fr, 0u, (size_t)n * W * 2);
    fill_u32(st, V.stamp, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, V.lmark, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, V.sbit, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, ctl, 0u, sizeof(ReachCtl) / 4);
    if (nb > 0) {
        hipLaunchKernelGGL(k_rch_act_count, dim3((unsigned)nb), dim3(kBlock), 0, st, V);
        hipLaunchKernelGGL(k_rch_act_scan, dim3(1), dim3(kBlock), 0, st, ctl, V, nb);
        hipLaunchKernelGGL(k_rch_act_put, dim3((unsigned)nb), dim3(kBlock), 0, st, V);
    }
    // start in the account phase with nothing touched: its last block picks the first batch
    hipLaunchKernelGGL(k_rch_set_phase, dim3(1), dim3(1), 0, st, ctl, (int32_t)kAccount);
    CCG_HIP(hipGetLastError());

    const unsigned gp = (unsigned)a.push_blocks, gm = (unsigned)a.merge_blocks, ga = (unsigned)a.account_blocks;
    const int64_t nbatches = (V.nsrc + kFirstBatch - 1) / kFirstBatch + 1;
    const int64_t max_cycles = nbatches * (n + 2);
    int64_t cycles = 0;
    int32_t chunk = 16;
    ReachCtl hc{};
    for (;;) {
        for (int32_t c = 0; c < chunk; c++) {
            hipLaunchKernelGGL((k_rch_push<W>), dim3(gp), dim3(kBlock), 0, st, ctl, V);
            hipLaunchKernelGGL((k_rch_merge<W>), dim3(gm), dim3(kBlock), 0, st, ctl, V);
            hipLaunchKernelGGL((k_rch_account<W>), dim3(ga), dim3(kBlock), 0, st, ctl, V);
        }
        CCG_HIP(hipGetLastError());
        cycles += chunk;
        CCG_HIP(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        if (hc.phase == kFinished) break;
        if (cycles > max_cycles) throw HipError{hipErrorLaunchTimeOut, "reachability sampling did not finish"};
        if (chunk < 256) chunk *= 2;
    }
    if (weighted)
        hipLaunchKernelGGL(k_rch_out_beta<uint16_t>, dim3(gn), dim3(256), 0, st, V, (const uint16_t*)V.mem_d, a.orig,
                           a.beta, a.U, a.count, a.kth, a.S_w, a.R, &ctl->overflow);
    else
        hipLaunchKernelGGL(k_rch_out, dim3(gn), dim3(256), 0, st, V, a.orig, a.count, a.distsum, a.T, a.B, a.R);
    CCG_HIP(hipGetLastError());
    if (stats) {
        stats->cycles = cycles;
        stats->batches = hc.batch;
        stats->levels = hc.levels;
        stats->overflow = hc.overflow != 0;
    }
}

}  // namespace ccg
