// Estimator epilogue working directly on the per-level seen masks written by
// the batched BFS (S_L(v) = {i : d(c_i, v) <= L}, L = 0..lmax), so the
// distance matrix is never stored.  For a node v:
//   d(c_i, v)        = #{L < lmax : i not in S_L(v)}      (levels still missing i)
//   Delta(v)         = first L with S_L(v) non-empty, pivot = its lowest bit
//                      (the lowest sample index among the nearest, Sec. 2 / Alg. 2)
//   sum_i d(c_i, v)  = sum_{L < lmax} (k - |S_L(v)|)
//   L cap C (Eq. 6)  = Lmask[p][t] = {i : d(c_p, c_i) <= t}, t = floor(Delta*den/num)
//   sum_{L cap C} d  = sum_{L < lmax} |Lmask & ~S_L(v)|
// and |H|, sum_H from the per-sample tail tables (see k_suffix), as in the
// distance-matrix epilogue.  A group of 64 nodes stops writing masks after
// the level recorded in fill_level[g]; later masks are all-ones.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;

template <int W>
__device__ __forceinline__ uint64_t full_word(int w, uint64_t lastmask) {
    return w == W - 1 ? lastmask : ~0ull;
}

// One graph's part of the snapshot rows: the rows of nodes noff.. and, in
// each row of rs words, the W words from wo on (a single graph: noff = 0,
// wo = 0, rs = W; a batch of graphs shares one set of rows).
struct SnapView {
    const uint64_t* snap;
    size_t plane;  // words per level
    int32_t rs;    // words per row
    int32_t wo;    // first word of this graph's samples
    int64_t noff;  // first row of this graph's nodes
    const int32_t* fill_level;  // per 64 rows: last level written
    __device__ __forceinline__ const uint64_t* row(int32_t L, int64_t v) const {
        return snap + (size_t)L * plane + (size_t)(noff + v) * rs + wo;
    }
    __device__ __forceinline__ int32_t fill(int64_t v) const { return fill_level[(noff + v) >> 6]; }
};

// Mask of node v at level L: this graph's words, the last one cut to its
// samples (a batch keeps other graphs' bits set in every row).
template <int W>
__device__ __forceinline__ void mask_at(const SnapView& sv, int32_t L, int32_t fl, int64_t v, uint64_t lastmask,
                                        uint64_t s[W]) {
    if (L <= fl) {
        const uint64_t* row = sv.row(L, v);
#pragma unroll
        for (int p = 0; p < (W + 1) / 2; p++) {
            if (2 * p + 1 < W) {
                const uint4 q = *(const uint4*)(row + 2 * p);
                s[2 * p] = ((uint64_t)q.y << 32) | q.x;
                s[2 * p + 1] = ((uint64_t)q.w << 32) | q.z;
            } else {
                s[2 * p] = row[2 * p];
            }
        }
        s[W - 1] &= lastmask;
    } else {
#pragma unroll
        for (int w = 0; w < W; w++) s[w] = full_word<W>(w, lastmask);
    }
}

// first level at which bit i is in the mask of node v
template <int W>
__device__ __forceinline__ int32_t level_of(const SnapView& sv, int32_t lmax, int32_t fl, int64_t v, int32_t i) {
    for (int32_t L = 0; L <= lmax; L++) {
        if (L > fl) return L;
        const uint64_t x = sv.row(L, v)[i >> 6];
        if ((x >> (i & 63)) & 1ull) return L;
    }
    return -1;  // never reached
}

template <int W, typename MT>
__global__ void k_dmat_bits(SnapView sv, int32_t lmax, const int32_t* __restrict__ samples, int32_t k,
                            int32_t* __restrict__ dmat, MT* __restrict__ dmat_c, DevFlags* flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)k * k) return;
    const int32_t i = (int32_t)(t / k), j = (int32_t)(t % k);
    const int64_t cj = samples[j];
    const int32_t d = level_of<W>(sv, lmax, sv.fill(cj), cj, i);
    if (d < 0) flags->disconnected = 1;
    dmat[t] = d;
    dmat_c[t] = (MT)(d < 0 ? 0 : d);
}

// Lmask[p][t] = {i : dmat[p][i] <= t} for t = 0..lmax; one wave per p
template <int W, typename MT>
__global__ void k_lmask(const MT* __restrict__ dmat_c, int32_t k, int32_t lmax, uint64_t* __restrict__ lmask) {
    const int32_t p = blockIdx.x;
    const int lane = lane_id();
    for (int32_t t = 0; t <= lmax; t++) {
#pragma unroll
        for (int w = 0; w < W; w++) {
            const int32_t i = w * 64 + lane;
            const bool in = i < k && (int32_t)dmat_c[(int64_t)p * k + i] <= t;
            const uint64_t m = __ballot(in);
            if (lane == 0) lmask[((int64_t)p * (lmax + 1) + t) * W + w] = m;
        }
    }
}

// Everything the estimate needs per sample, one block per sample i, for
// searches of at most kBlock - 2 levels: row i of the sample distance matrix
// (the level at which each sample node gains bit i), the L masks of i as a
// pivot (Lmask[i][t] = {j : d(c_i, c_j) <= t}), the tail tables of its
// level histogram (summed over the histogram's slots) and the exact S(c_i).
// The same results as k_dmat_bits, k_lmask and k_suffix, in one launch.
template <int W, typename MT>
__global__ __launch_bounds__(kBlock) void k_sample_tables(
    SnapView sv, int32_t lmax, const int32_t* __restrict__ samples, int32_t k, const int32_t* __restrict__ hist,
    int32_t nslots, int32_t hrows, int64_t hlen, int32_t* __restrict__ dmat, MT* __restrict__ dmat_c,
    uint64_t* __restrict__ lmask, int32_t* __restrict__ Tcnt, int64_t* __restrict__ Tsum, int64_t* __restrict__ src_sum,
    DevFlags* flags) {
    __shared__ int32_t row[64 * W];
    __shared__ unsigned long long hsm[kBlock];
    __shared__ long long part[kBlock / 64];
    const int32_t i = blockIdx.x;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int32_t D = lmax + 1;  // distances 0..lmax
    // the row, and the histogram summed over its slots (kBlock / D threads per distance)
    long long rs = 0;
    bool bad = false;
    for (int32_t j = threadIdx.x; j < k; j += kBlock) {
        const int64_t cj = samples[j];
        const int32_t d = level_of<W>(sv, lmax, sv.fill(cj), cj, i);
        bad = bad || d < 0;
        dmat[(int64_t)i * k + j] = d;
        dmat_c[(int64_t)i * k + j] = (MT)(d < 0 ? 0 : d);
        row[j] = d < 0 ? 0 : d;
        rs += d;
    }
    if (bad) flags->disconnected = 1;
    hsm[threadIdx.x] = 0;
    __syncthreads();
    {
        const int32_t G = kBlock / D, dd = (int32_t)threadIdx.x % D, g = (int32_t)threadIdx.x / D;
        if (g < G && dd < hlen) {
            unsigned long long c = 0;
            for (int32_t s = g; s < nslots; s += G) c += (unsigned long long)hist[((int64_t)s * hrows + i) * hlen + dd];
            if (c) atomicAdd(&hsm[dd], c);
        }
    }
    rs = (long long)wave_sum64((int64_t)rs);
    if (lane == 0) part[wave] = rs;
    __syncthreads();
    // L masks of i as a pivot: wave w takes thresholds w, w + 4, ...
    for (int32_t t = wave; t <= lmax; t += kBlock / 64) {
#pragma unroll
        for (int w = 0; w < W; w++) {
            const int32_t j = w * 64 + lane;
            const uint64_t m = __ballot(j < k && row[j] <= t);
            if (lane == 0) lmask[((int64_t)i * (lmax + 1) + t) * W + w] = m;
        }
    }
    // tail tables: T_cnt[i][t] = sum_{d >= t} h[d], T_sum[i][t] = sum_{d >= t} d h[d]
    const int64_t tlen = (int64_t)lmax + 2;
    if (threadIdx.x < tlen) {
        int64_t c = 0, sm = 0;
        for (int32_t d = (int32_t)threadIdx.x; d < D; d++) {
            c += (int64_t)hsm[d];
            sm += (int64_t)d * (int64_t)hsm[d];
        }
        Tcnt[(int64_t)i * tlen + threadIdx.x] = (int32_t)c;
        Tsum[(int64_t)i * tlen + threadIdx.x] = sm;
        // S(c_i) = (sum over non-sampled u of d(c_i, u)) + sum_j d(c_i, c_j)
        if (threadIdx.x == 0) {
            long long tot = 0;
            for (int w = 0; w < kBlock / 64; w++) tot += part[w];
            src_sum[i] = sm + (int64_t)tot;
        }
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_estimate_bits(
    SnapView sv, int32_t lmax, int64_t n, int32_t k, uint64_t lastmask, const int32_t* __restrict__ sidx,
    int32_t bit_base, const int32_t* __restrict__ orig,
    const uint64_t* __restrict__ lmask, const int32_t* __restrict__ Tcnt, const int64_t* __restrict__ Tsum,
    int64_t tlen, const int64_t* __restrict__ src_sum, int64_t en, int64_t ed, double* S_hyb, double* S_samp,
    int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out, int32_t* delta_out, int64_t* sampsum_out,
    uint4* __restrict__ stage, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    bool any_ovf = false, any_unreached = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int32_t fl = sv.fill(v);
        const int32_t j = sidx[sv.noff + v] >= 0 ? sidx[sv.noff + v] - bit_base : -1;
        // One pass over the levels.  The pivot and Delta are known at the
        // first non-empty level, and with them the pivot's L mask, so the sum
        // over L cap C is taken in the same pass: every earlier level is empty
        // and adds |Lmask| (each of those samples is still missing there).
        int32_t delta = -1, p = 0, last = 0, lcnum = 0;
        int64_t sum = 0, lcsum = 0;
        uint64_t lm[W];
#pragma unroll
        for (int w = 0; w < W; w++) lm[w] = 0;
        auto take_lmask = [&](int32_t d, int32_t piv) {
            int64_t t = (int64_t)d * ed / en;
            if (t > lmax) t = lmax;
            lcnum = 0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                lm[w] = lmask[((int64_t)piv * (lmax + 1) + t) * W + w];
                lcnum += __popcll(lm[w]);
            }
            lcsum = (int64_t)d * lcnum;
        };
        for (int32_t L = 0; L <= lmax; L++) {
            uint64_t s[W];
            mask_at<W>(sv, L, fl, v, lastmask, s);
            int32_t c = 0;
#pragma unroll
            for (int w = 0; w < W; w++) c += __popcll(s[w]);
            if (delta < 0 && c > 0) {
                delta = L;
#pragma unroll
                for (int w = W - 1; w >= 0; w--)
                    if (s[w]) p = w * 64 + __ffsll((unsigned long long)s[w]) - 1;
                if (j < 0) take_lmask(delta, p);
            }
            if (L < lmax) {
                sum += k - c;
                if (delta >= 0) {
#pragma unroll
                    for (int w = 0; w < W; w++) lcsum += __popcll(lm[w] & ~s[w]);
                }
            }
            last = c;
        }
        const bool unreached = last != k;
        double hyb, samp;
        int64_t piv, pub;
        bool ovf = false;
        if (delta < 0) {  // no sample reaches v: pivot 0 at Delta 0, every level empty
            delta = 0;
            if (j < 0) {
                take_lmask(0, 0);
                lcsum = (int64_t)lmax * lcnum;
            }
        }
        if (j >= 0) {
            const int64_t S = src_sum[j];
            hyb = samp = (double)S;
            piv = pub = S;
            ovf = S >= LIM;
        } else {
            const int64_t thr = (int64_t)delta * ed;
            const int64_t tix = thr / en + 1;  // d > floor(Delta/eps)  <=>  d >= tix
            int64_t hnum = 0, hsum = 0;
            if (tix < tlen) {
                hnum = Tcnt[(int64_t)p * tlen + tix];
                hsum = Tsum[(int64_t)p * tlen + tix];
            }
            const int64_t hcsum = sum - lcsum;
            const int64_t lnum = (n - 1) - hnum - (int64_t)(k - lcnum);
            const int64_t a = hsum + hcsum;
            int64_t t1 = 0, t2 = 0, N = 0, ss = 0;
            ovf = __builtin_mul_overflow(a, (int64_t)lcnum, &t1) || __builtin_mul_overflow(lcsum, lnum, &t2) ||
                  __builtin_add_overflow(t1, t2, &N) || N >= LIM || lcnum < 1 || lnum < lcnum;
            hyb = (double)N / (double)lcnum;
            ovf = ovf || __builtin_mul_overflow(n - 1, sum, &ss) || ss >= LIM;
            samp = (double)ss / (double)k;
            piv = src_sum[p];
            pub = piv + (n - 1) * (int64_t)delta;
        }
        if (stage) {  // one 64-byte record per node, in internal order (coalesced)
            const uint64_t hb = (uint64_t)__double_as_longlong(hyb), sb = (uint64_t)__double_as_longlong(samp);
            uint4* r = stage + v * 4;
            r[0] = make_uint4((uint32_t)hb, (uint32_t)(hb >> 32), (uint32_t)sb, (uint32_t)(sb >> 32));
            r[1] = make_uint4((uint32_t)piv, (uint32_t)((uint64_t)piv >> 32), (uint32_t)pub, (uint32_t)((uint64_t)pub >> 32));
            r[2] = make_uint4((uint32_t)sum, (uint32_t)((uint64_t)sum >> 32), (uint32_t)p, (uint32_t)delta);
        } else {
            const int64_t o = orig[v];
            if (S_hyb) S_hyb[o] = hyb;
            if (S_samp) S_samp[o] = samp;
            if (S_piv) S_piv[o] = piv;
            if (S_pub) S_pub[o] = pub;
            if (pivot_out) pivot_out[o] = p;
            if (delta_out) delta_out[o] = delta;
            if (sampsum_out) sampsum_out[o] = sum;
        }
        any_ovf = any_ovf || ovf;
        any_unreached = any_unreached || unreached;
    }
    if (any_ovf) flags->overflow = 1;
    if (any_unreached) flags->disconnected = 1;
}

// The staged records written out in the caller's order: thread o reads the
// record of its internal node inv[o] (one 64-byte line) and writes each
// requested output at o, coalesced across the wave.
__global__ __launch_bounds__(kBlock) void k_put_outputs(int64_t n, const int32_t* __restrict__ inv,
                                                        const uint4* __restrict__ stage, double* S_hyb, double* S_samp,
                                                        int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out,
                                                        int32_t* delta_out, int64_t* sampsum_out) {
    for (int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x; o < n; o += (int64_t)gridDim.x * kBlock) {
        const uint4* r = stage + (int64_t)inv[o] * 4;
        const uint4 a = r[0], b = r[1], c = r[2];
        if (S_hyb) S_hyb[o] = __longlong_as_double((long long)(((uint64_t)a.y << 32) | a.x));
        if (S_samp) S_samp[o] = __longlong_as_double((long long)(((uint64_t)a.w << 32) | a.z));
        if (S_piv) S_piv[o] = (int64_t)(((uint64_t)b.y << 32) | b.x);
        if (S_pub) S_pub[o] = (int64_t)(((uint64_t)b.w << 32) | b.z);
        if (sampsum_out) sampsum_out[o] = (int64_t)(((uint64_t)c.y << 32) | c.x);
        if (pivot_out) pivot_out[o] = (int32_t)c.z;
        if (delta_out) delta_out[o] = (int32_t)c.w;
    }
}

// Distances from the masks: thread per (node, sample).  out_internal (DT,
// node-major, columns src_base..) or out_i32 at the caller's node ids.
template <int W, typename DT>
__global__ void k_materialize(SnapView sv, int32_t lmax, int64_t n, int32_t kg, int32_t src_base, int32_t k,
                              DT* __restrict__ out_internal, const int32_t* __restrict__ orig,
                              int32_t* __restrict__ out_i32, DevFlags* flags) {
    const int64_t count = n * kg;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / kg;
        const int32_t i = (int32_t)(t % kg);
        const int32_t d = level_of<W>(sv, lmax, sv.fill(v), v, i);
        if (d < 0) flags->disconnected = 1;
        if (out_internal) out_internal[v * k + src_base + i] = (DT)(d < 0 ? DistT<DT>::never : (uint32_t)d);
        if (out_i32) out_i32[(int64_t)orig[v] * k + src_base + i] = d;
    }
}

// Spreads the 8 bits of b over the 8 bytes of a word (byte j = bit j of b).
__device__ __forceinline__ uint64_t spread8(uint32_t b) {
    const uint64_t z = ((uint64_t)b * 0x0101010101010101ull) & 0x8040201008040201ull;
    return (((z + 0x7F7F7F7F7F7F7F7Full) | z) & 0x8080808080808080ull) >> 7;
}

// Distances from the masks, one thread per (node, 64-sample word): the
// distance of sample i is the number of levels 0..min(fill, lmax) whose mask
// lacks bit i (masks only grow, and the node is full after its fill level).
// Byte counters, eight samples per 64-bit accumulator, need lmax < 255.
// Output DT (u8 internal, node-major columns src_base..) or int32 at the
// caller's node ids; 16-byte stores when the row offsets allow.
template <int W, typename OT>
__global__ __launch_bounds__(kBlock) void k_materialize_words(
    SnapView sv, int32_t lmax, int64_t n, int32_t kg, int32_t src_base, int32_t k, OT* __restrict__ out,
    const int32_t* __restrict__ orig, int vec, DevFlags* flags, int add) {
    const int64_t count = n * W;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / W;
        const int w = (int)(t % W);
        const int nb = min(64, kg - w * 64);  // samples in this word
        if (nb <= 0) continue;
        const uint64_t valid = nb >= 64 ? ~0ull : ((1ull << nb) - 1);
        const int32_t last = min(sv.fill(v), lmax);
        uint64_t acc[8];
#pragma unroll
        for (int q = 0; q < 8; q++) acc[q] = 0;
        uint64_t miss = valid;
        for (int32_t L = 0; L <= last; L++) {
            miss = ~sv.row(L, v)[w] & valid;
            if (!miss) break;
#pragma unroll
            for (int q = 0; q < 8; q++) acc[q] += spread8((uint32_t)(miss >> (8 * q)) & 0xFFu);
        }
        if (miss) flags->disconnected = 1;  // a bit still unset when the node stopped changing
        const int64_t row = orig ? (int64_t)orig[v] : v;
        OT* dst = out + row * k + src_base + (int64_t)w * 64;
        if (vec && nb == 64) {
            if constexpr (sizeof(OT) == 1) {
                uint4* d4 = reinterpret_cast<uint4*>(dst);
                if (add) {  // the other direction's distances are there: bytewise sums (the host checked they fit)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const uint4 o = d4[q];
                        acc[2 * q] += ((uint64_t)o.y << 32) | o.x;
                        acc[2 * q + 1] += ((uint64_t)o.w << 32) | o.z;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; q++)
                    d4[q] = make_uint4((uint32_t)acc[2 * q], (uint32_t)(acc[2 * q] >> 32), (uint32_t)acc[2 * q + 1],
                                       (uint32_t)(acc[2 * q + 1] >> 32));
            } else {
                int4* d4 = reinterpret_cast<int4*>(dst);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const uint64_t a = acc[q];
                    d4[2 * q] = make_int4((int)(a & 0xFF), (int)((a >> 8) & 0xFF), (int)((a >> 16) & 0xFF),
                                          (int)((a >> 24) & 0xFF));
                    d4[2 * q + 1] = make_int4((int)((a >> 32) & 0xFF), (int)((a >> 40) & 0xFF),
                                              (int)((a >> 48) & 0xFF), (int)((a >> 56) & 0xFF));
                }
            }
        } else {
            for (int i = 0; i < nb; i++) {
                const OT d = (OT)((acc[i >> 3] >> (8 * (i & 7))) & 0xFF);
                dst[i] = add ? (OT)(dst[i] + d) : d;
            }
        }
    }
}

// Round-trip distances of one group of samples (one-byte rows, whole 64-bit
// words) from both directions' masks in one pass, one thread per (node, word):
// the forward and the reverse level counts, summed (the host checked that
// the largest sums fit a byte), written once.  Materialising the forward
// distances first and adding the reverse ones in place wrote the rows twice
// and read them back once.
template <int W>
__global__ __launch_bounds__(kBlock) void k_materialize_round_trip(SnapView fw, int32_t lmax_f, SnapView rv,
                                                                   int32_t lmax_r, int64_t n, int32_t k,
                                                                   uint8_t* __restrict__ out, DevFlags* flags) {
    const int64_t count = n * W;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / W;
        const int w = (int)(t % W);
        uint64_t acc[8];
#pragma unroll
        for (int q = 0; q < 8; q++) acc[q] = 0;
        bool unreached = false;
#pragma unroll
        for (int dir = 0; dir < 2; dir++) {
            const SnapView& sv = dir == 0 ? fw : rv;
            const int32_t last = min(sv.fill(v), dir == 0 ? lmax_f : lmax_r);
            uint64_t miss = ~0ull;
            for (int32_t L = 0; L <= last; L++) {
                miss = ~sv.row(L, v)[w];
                if (!miss) break;
#pragma unroll
                for (int q = 0; q < 8; q++) acc[q] += spread8((uint32_t)(miss >> (8 * q)) & 0xFFu);
            }
            unreached = unreached || miss != 0;
        }
        if (unreached) flags->disconnected = 1;  // a bit still unset when the node stopped changing
        uint4* d4 = reinterpret_cast<uint4*>(out + v * k + (int64_t)w * 64);
#pragma unroll
        for (int q = 0; q < 4; q++)
            d4[q] = make_uint4((uint32_t)acc[2 * q], (uint32_t)(acc[2 * q] >> 32), (uint32_t)acc[2 * q + 1],
                               (uint32_t)(acc[2 * q + 1] >> 32));
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline unsigned grid_for(int64_t items, int64_t cap) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <int W, typename MT>
void bits_t(hipStream_t st, const BitsEpilogueArgs& a, void* scratch, DevFlags* flags) {
    const int64_t n = a.n;
    const int32_t k = a.k;
    const int32_t lmax = a.lmax;
    const int64_t tlen = (int64_t)lmax + 2;
    const int rem = k - (W - 1) * 64;
    const uint64_t lastmask = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
    char* p = (char*)scratch;
    const bool staged = a.inv && (a.S_hyb || a.S_samp || a.S_piv || a.S_pub || a.pivot || a.delta || a.sampsum);
    uint4* stage = staged ? (uint4*)p : nullptr;  // 64 bytes per node, first in the scratch
    if (staged) p += align256((size_t)n * 64);
    int32_t* Tcnt = (int32_t*)p;
    p += align256(sizeof(int32_t) * k * tlen);
    int64_t* Tsum = (int64_t*)p;
    p += align256(sizeof(int64_t) * k * tlen);
    MT* dmat_c = (MT*)p;
    p += align256(sizeof(MT) * (size_t)k * k);
    uint64_t* lmask = (uint64_t*)p;

    const SnapView sv{a.snap, a.plane, a.row_words > 0 ? a.row_words : W, a.word_off, a.node_off, a.fill_level};
    const int32_t hrows = a.hist_rows > 0 ? a.hist_rows : k;
    const int64_t kk = (int64_t)k * k;
    if (lmax + 2 <= kBlock) {  // the tail tables' lmax + 2 entries, one thread each
        hipLaunchKernelGGL((k_sample_tables<W, MT>), dim3(k), dim3(kBlock), 0, st, sv, lmax, a.samples, k,
                           a.hist + (int64_t)a.bit_base * a.hist_len, a.hist_slots, hrows, a.hist_len, a.dmat, dmat_c,
                           lmask, Tcnt, Tsum, a.src_sum, flags);
    } else {
        hipLaunchKernelGGL((k_dmat_bits<W, MT>), dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, st, sv, lmax,
                           a.samples, k, a.dmat, dmat_c, flags);
        run_suffix(st, a.hist + (int64_t)a.bit_base * a.hist_len, a.hist_slots, k, hrows, a.hist_len, lmax, a.dmat,
                   Tcnt, Tsum, a.src_sum, nullptr);
        hipLaunchKernelGGL((k_lmask<W, MT>), dim3(k), dim3(64), 0, st, dmat_c, k, lmax, lmask);
    }
    hipLaunchKernelGGL((k_estimate_bits<W>), dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, sv, lmax, n, k, lastmask,
                       a.sidx, a.bit_base, a.orig, lmask, Tcnt, Tsum, tlen, a.src_sum, a.eps_num, a.eps_den, a.S_hyb,
                       a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, stage, flags);
    if (staged)
        hipLaunchKernelGGL(k_put_outputs, dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, n, a.inv,
                           (const uint4*)stage, a.S_hyb, a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum);
    CCG_HIP(hipGetLastError());
    if (a.Dout) {
        if (lmax < 255) {
            hipLaunchKernelGGL((k_materialize_words<W, int32_t>), dim3(grid_for(n * W, 65536)), dim3(kBlock), 0, st,
                               sv, lmax, n, k, 0, k, a.Dout, a.orig, (int)(k % 4 == 0), flags, 0);
        } else {
            hipLaunchKernelGGL((k_materialize<W, uint8_t>), dim3(grid_for(n * k, 65536)), dim3(256), 0, st, sv, lmax,
                               n, k, 0, k, (uint8_t*)nullptr, a.orig, a.Dout, flags);
        }
    }
    if (a.S_err || a.S_ad || a.S_ad_err || a.S_sweep || a.S_sweep_err) {
        // Sec. 4 and the threshold sweep need each node's distance row:
        // materialise it (after the tables above in the scratch), then the
        // shared error pass; the sweep's tables follow the rows
        char* dq = (char*)lmask + align256(sizeof(uint64_t) * (size_t)k * (lmax + 1) * W);
        ErrArgs ea;
        ea.D = dq;
        ea.n = n;
        ea.k = k;
        ea.sidx = a.sidx + a.node_off;
        ea.bit_base = a.bit_base;
        ea.orig = a.orig;
        ea.dmat_c = dmat_c;
        ea.mt_bytes = (int)sizeof(MT);
        ea.Tcnt = Tcnt;
        ea.Tsum = Tsum;
        ea.tlen = tlen;
        ea.src_sum = a.src_sum;
        ea.eps_num = a.eps_num;
        ea.eps_den = a.eps_den;
        ea.S_err = a.S_err;
        ea.S_ad = a.S_ad;
        ea.S_ad_err = a.S_ad_err;
        ea.S_sweep = a.S_sweep;
        ea.S_sweep_err = a.S_sweep_err;
        const size_t db = lmax < 255 ? 1 : (lmax < 65535 ? 2 : 4);
        ea.sweep_scratch = dq + align256((size_t)n * k * db);
        if (lmax < 255) {
            ea.dk = DistKind::U8;
            hipLaunchKernelGGL((k_materialize_words<W, uint8_t>), dim3(grid_for(n * W, 65536)), dim3(kBlock), 0, st,
                               sv, lmax, n, k, 0, k, (uint8_t*)dq, (const int32_t*)nullptr, (int)(k % 16 == 0), flags,
                               0);
        } else if (lmax < 65535) {
            ea.dk = DistKind::U16;
            hipLaunchKernelGGL((k_materialize<W, uint16_t>), dim3(grid_for(n * k, 65536)), dim3(256), 0, st, sv,
                               lmax, n, k, 0, k, (uint16_t*)dq, (const int32_t*)nullptr, (int32_t*)nullptr, flags);
        } else {
            ea.dk = DistKind::U32;
            hipLaunchKernelGGL((k_materialize<W, uint32_t>), dim3(grid_for(n * k, 65536)), dim3(256), 0, st, sv,
                               lmax, n, k, 0, k, (uint32_t*)dq, (const int32_t*)nullptr, (int32_t*)nullptr, flags);
        }
        run_errest(st, ea, flags);
    }
}

template <int W>
void bits_mt(hipStream_t st, const BitsEpilogueArgs& a, void* scratch, DevFlags* flags) {
    if (a.lmax < 255) bits_t<W, uint8_t>(st, a, scratch, flags);
    else if (a.lmax < 65535) bits_t<W, uint16_t>(st, a, scratch, flags);
    else bits_t<W, uint32_t>(st, a, scratch, flags);
}

template <int W, typename DT>
void materialize_t(hipStream_t st, const uint64_t* snap, size_t plane, int32_t lmax, const int32_t* fill_level,
                   int64_t n, int32_t kg, int32_t src_base, int32_t k, void* D, DevFlags* flags, bool add) {
    const SnapView sv{snap, plane, W, 0, 0, fill_level};
    if constexpr (sizeof(DT) == 1) {
        if (lmax < 255) {
            const int vec = (k % 16 == 0) && (src_base % 16 == 0);
            hipLaunchKernelGGL((k_materialize_words<W, uint8_t>), dim3(grid_for(n * W, 65536)), dim3(kBlock), 0, st,
                               sv, lmax, n, kg, src_base, k, (uint8_t*)D, (const int32_t*)nullptr, vec, flags,
                               add ? 1 : 0);
            return;
        }
    }
    if (add) throw HipError{hipErrorInvalidValue, "summed distances need one-byte rows"};
    hipLaunchKernelGGL((k_materialize<W, DT>), dim3(grid_for(n * kg, 65536)), dim3(256), 0, st, sv, lmax, n, kg,
                       src_base, k, (DT*)D, (const int32_t*)nullptr, (int32_t*)nullptr, flags);
}

template <int W>
void materialize_w(hipStream_t st, const uint64_t* snap, size_t plane, int32_t lmax, const int32_t* fill_level,
                   int64_t n, int32_t kg, int32_t src_base, int32_t k, void* D, DistKind dk, DevFlags* flags, bool add) {
    switch (dk) {
        case DistKind::U8: materialize_t<W, uint8_t>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, flags, add); break;
        case DistKind::U16: materialize_t<W, uint16_t>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, flags, add); break;
        default: materialize_t<W, uint32_t>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, flags, add); break;
    }
}

}  // namespace

size_t bits_epilogue_scratch(int32_t k, int32_t lmax, int64_t err_rows, bool err, int64_t stage_rows) {
    const int64_t tlen = (int64_t)lmax + 2;
    const int W = (k + 63) / 64;
    const size_t db = lmax < 255 ? 1 : (lmax < 65535 ? 2 : 4);
    return align256(sizeof(int32_t) * k * tlen) + align256(sizeof(int64_t) * k * tlen) +
           align256(sizeof(uint32_t) * (size_t)k * k) + align256(sizeof(uint64_t) * (size_t)k * (lmax + 1) * W) +
           align256((size_t)err_rows * k * db) + (err ? sweep_scratch_bytes(err_rows, k) : 0) +
           align256((size_t)stage_rows * 64) + 1024;
}

void run_bits_epilogue(hipStream_t st, const BitsEpilogueArgs& a, void* scratch, size_t scratch_size,
                       DevFlags* flags) {
    const bool want_err = a.S_err || a.S_ad || a.S_ad_err || a.S_sweep || a.S_sweep_err;
    const bool staged = a.inv && (a.S_hyb || a.S_samp || a.S_piv || a.S_pub || a.pivot || a.delta || a.sampsum);
    if (scratch_size < bits_epilogue_scratch(a.k, a.lmax, want_err ? a.n : 0, want_err, staged ? a.n : 0))
        throw HipError{hipErrorOutOfMemory, "bits epilogue scratch"};
    switch ((a.k + 63) / 64) {
        case 1: bits_mt<1>(st, a, scratch, flags); break;
        case 2: bits_mt<2>(st, a, scratch, flags); break;
        case 3: bits_mt<3>(st, a, scratch, flags); break;
        default: bits_mt<4>(st, a, scratch, flags); break;
    }
}

void materialize_distances(hipStream_t st, const uint64_t* snap, size_t plane, int32_t lmax, const int32_t* fill_level,
                           int64_t n, int32_t kg, int32_t src_base, int32_t k, void* D, DistKind dk, DevFlags* flags,
                           bool add) {
    switch ((kg + 63) / 64) {
        case 1: materialize_w<1>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, dk, flags, add); break;
        case 2: materialize_w<2>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, dk, flags, add); break;
        case 3: materialize_w<3>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, dk, flags, add); break;
        default: materialize_w<4>(st, snap, plane, lmax, fill_level, n, kg, src_base, k, D, dk, flags, add); break;
    }
    CCG_HIP(hipGetLastError());
}

void materialize_round_trip(hipStream_t st, const uint64_t* snap_f, const int32_t* fill_f, int32_t lmax_f,
                            const uint64_t* snap_r, const int32_t* fill_r, int32_t lmax_r, int64_t n, int32_t k,
                            void* D, DevFlags* flags) {
    if (k % 64 != 0 || k > 256 || lmax_f + lmax_r > 254)
        throw HipError{hipErrorInvalidValue, "round-trip rows need whole words and byte sums"};
    const int W = k / 64;
    const size_t plane = (size_t)n * W;
    const SnapView fw{snap_f, plane, W, 0, 0, fill_f}, rv{snap_r, plane, W, 0, 0, fill_r};
    const dim3 grid(grid_for(n * W, 65536));
    switch (W) {
        case 1: hipLaunchKernelGGL((k_materialize_round_trip<1>), grid, dim3(kBlock), 0, st, fw, lmax_f, rv, lmax_r, n, k, (uint8_t*)D, flags); break;
        case 2: hipLaunchKernelGGL((k_materialize_round_trip<2>), grid, dim3(kBlock), 0, st, fw, lmax_f, rv, lmax_r, n, k, (uint8_t*)D, flags); break;
        case 3: hipLaunchKernelGGL((k_materialize_round_trip<3>), grid, dim3(kBlock), 0, st, fw, lmax_f, rv, lmax_r, n, k, (uint8_t*)D, flags); break;
        default: hipLaunchKernelGGL((k_materialize_round_trip<4>), grid, dim3(kBlock), 0, st, fw, lmax_f, rv, lmax_r, n, k, (uint8_t*)D, flags); break;
    }
    CCG_HIP(hipGetLastError());
}

void put_outputs(hipStream_t st, int64_t n, const int32_t* inv, const void* stage, double* S_hyb, double* S_samp,
                 int64_t* S_piv, int64_t* S_pub, int32_t* pivot, int32_t* delta, int64_t* sampsum) {
    hipLaunchKernelGGL(k_put_outputs, dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, n, inv, (const uint4*)stage, S_hyb,
                       S_samp, S_piv, S_pub, pivot, delta, sampsum);
    CCG_HIP(hipGetLastError());
}

}  // namespace ccg
