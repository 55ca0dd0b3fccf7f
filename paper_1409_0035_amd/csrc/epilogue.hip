// Estimator epilogue: from the node-major distance matrix D[v][i] = d(c_i, v)
// (internal, degree-sorted node ids) to every estimate of Sec. 2 of the
// paper, for every node, written at the caller's node ids.
//
//   k_reduce    (when the traversal did not count it) per-sample histogram
//               hist[i][d] = #{u not in C : d(c_i,u) = d}, one lane per node.
//   k_dmat      sample-to-sample distances dmat[i][j] = d(c_i, c_j) = D[c_j][i],
//               as int32 for the caller and in a compact width for k_estimate.
//   k_suffix    per sample, T_cnt[i][t] = sum_{d >= t} hist[i][d] and
//               T_sum[i][t] = sum_{d >= t} d * hist[i][d] -- the tail counts and
//               sums Alg. 1 builds with its Thresh/bin arrays, here for every
//               integer threshold -- and the exact sum of the sample,
//               S(c_i) = T_sum[i][0] + sum_j dmat[i][j].
//   k_estimate  one lane per node: pivot (argmin of the row, lowest index on
//               ties), Delta, sum of the row; the samples split into L cap C
//               and HC by dmat[pivot][i] * num <= Delta * den (eps = num/den);
//               |H| and sum_H from the tail tables at floor(Delta*den/num)+1;
//               |L| = n-1-|H|-|HC| (Alg. 1 finalisation); Eq. (6) as the exact
//               integer N = (sum_H + sum_HC)*|L cap C| + |L|*sum_{L cap C},
//               divided once by |L cap C| in IEEE double.
// For directed graphs the distances are round-trip: D + Dr (Sec. 6.1).
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
// the row estimate with its tables in LDS: block size, largest table copy,
// blocks per launch (two per CU of the 256)
constexpr int kEstBlock = 512;
constexpr size_t kEstTableLds = 64 * 1024;
constexpr int64_t kEstTableBlocks = 512;
// row pieces each lane of the histogram keeps in flight (four measured the
// same as two on the round trip of rmat22dir, and three in the estimate)
constexpr int kRowsInFlight = 2;

// Reads element i of a distance row; with RT the reverse row is added.
template <typename DT, bool RT>
__device__ __forceinline__ uint32_t dist_at(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t off) {
    uint32_t a = (uint32_t)D[off];
    if (RT) a += (uint32_t)Dr[off];
    return a;
}

template <typename DT, bool RT>
__device__ __forceinline__ bool unreached_at(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t off) {
    bool u = (uint32_t)D[off] == DistT<DT>::never;
    if (RT) u = u || (uint32_t)Dr[off] == DistT<DT>::never;
    return u;
}

// Visits row[0..k) of D (+Dr) calling f(i, d).  Uses 16-byte loads when the
// row length in bytes is a multiple of 16.
template <typename DT, bool RT, typename F>
__device__ __forceinline__ void for_row(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t v, int32_t k,
                                        F&& f) {
    constexpr int per = 16 / sizeof(DT);
    const int64_t base = v * k;
    if (((int64_t)k * sizeof(DT)) % 16 == 0) {
        const uint4* a = (const uint4*)(D + base);
        const uint4* b = RT ? (const uint4*)(Dr + base) : nullptr;
        for (int32_t c = 0; c < k / per; c++) {
            const uint4 va = a[c];
            uint4 vb = make_uint4(0, 0, 0, 0);
            if (RT) vb = b[c];
            const uint32_t wa[4] = {va.x, va.y, va.z, va.w};
            const uint32_t wb[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
#pragma unroll
                for (int e = 0; e < 4 / (int)sizeof(DT); e++) {
                    const int sh = e * 8 * (int)sizeof(DT);
                    const uint32_t mask = sizeof(DT) == 4 ? 0xFFFFFFFFu : ((1u << (8 * sizeof(DT))) - 1);
                    uint32_t d = (wa[q] >> sh) & mask;
                    if (RT) d += (wb[q] >> sh) & mask;
                    f(c * per + q * (4 / (int)sizeof(DT)) + e, d);
                }
            }
        }
    } else {
        for (int32_t i = 0; i < k; i++) f(i, dist_at<DT, RT>(D, Dr, base + i));
    }
}

// histogram over non-sampled nodes, one lane per node; LDS copy while it fits
template <typename DT, bool RT>
__global__ __launch_bounds__(kBlock) void k_reduce(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n,
                                                   int32_t k, const int32_t* __restrict__ sidx, int64_t hlen,
                                                   int32_t* __restrict__ hist, int use_lds, DevFlags* flags) {
    extern __shared__ int32_t lds_hist[];  // [k][hlen] when use_lds
    if (use_lds) {
        for (int64_t t = threadIdx.x; t < (int64_t)k * hlen; t += kBlock) lds_hist[t] = 0;
        __syncthreads();
    }
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        if (sidx[v] >= 0) continue;
        for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
            if ((int64_t)d >= hlen) {
                bad = true;
            } else if (use_lds) {
                atomicAdd(&lds_hist[(int64_t)i * hlen + d], 1);
            } else {
                atomicAdd(&hist[(int64_t)i * hlen + d], 1);
            }
        });
    }
    if (bad) flags->disconnected = 1;  // an unreached entry (or a distance beyond the bound)
    if (use_lds) {
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)k * hlen; t += kBlock) {
            const int32_t c = lds_hist[t];
            if (c) atomicAdd(&hist[t], c);
        }
    }
}

// ---- row-cooperative variants: G lanes per node, lane j of a node holding
// the j-th 16 bytes of its row (and of the reverse row), so a wave's loads are
// consecutive bytes and each row is read once.  For rows of 16 * G bytes,
// G in {1, 2, 4, 8, 16}.

template <typename DT, bool RT>
struct RowPiece {
    static constexpr int PER = 16 / (int)sizeof(DT);
    uint32_t d[PER];
    bool unreached = false;
    // the lane's 16 bytes of the row (a) and of the reverse row (b)
    __device__ __forceinline__ void decode(const uint4 a, const uint4 b) {
        const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
        const uint32_t wb[4] = {b.x, b.y, b.z, b.w};
        constexpr uint32_t mask = sizeof(DT) == 4 ? 0xFFFFFFFFu : ((1u << (8 * sizeof(DT))) - 1);
#pragma unroll
        for (int q = 0; q < 4; q++) {
#pragma unroll
            for (int e = 0; e < 4 / (int)sizeof(DT); e++) {
                const int sh = e * 8 * (int)sizeof(DT);
                const uint32_t x = (wa[q] >> sh) & mask;
                uint32_t y = 0;
                if (RT) y = (wb[q] >> sh) & mask;
                unreached = unreached || x == DistT<DT>::never || (RT && y == DistT<DT>::never);
                d[q * (4 / (int)sizeof(DT)) + e] = x + y;
            }
        }
    }
};

// A lane's undecoded piece of a node's row and the node's sample index, so
// the next node's loads can be in flight while this one is worked on.
// The loads are unconditional, of node min(v, n - 1) (n >= 1): a refill past
// the end reads the last node again and its values go unused, and the
// registers never merge old and new values (such a merge makes the compiler
// wait for the loads in flight).
template <typename DT, bool RT>
struct RawPiece {
    uint4 a, b;
    uint4 ax[3];  // the further 16-byte parts of a wider piece (the estimate's wide lanes)
    int32_t j;
    __device__ __forceinline__ void fetch(const DT* __restrict__ D, const DT* __restrict__ Dr,
                                          const int32_t* __restrict__ sidx, int64_t v, int64_t n, int32_t k, int sub) {
        const int64_t vc = v < n ? v : n - 1;
        a = ((const uint4*)(D + vc * k))[sub];
        b = make_uint4(0, 0, 0, 0);
        if (RT) b = ((const uint4*)(Dr + vc * k))[sub];
        j = sidx[vc];
    }
};

// Byte j of the result is byte (j + b) mod 16 of x, for 0 <= b < 16.
__device__ __forceinline__ uint4 rotate_bytes(const uint4 x, uint32_t b) {
    uint32_t w0 = x.x, w1 = x.y, w2 = x.z, w3 = x.w;
    if (b & 4) {
        const uint32_t t = w0;
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = t;
    }
    if (b & 8) {
        const uint32_t t0 = w0, t1 = w1;
        w0 = w2;
        w1 = w3;
        w2 = t0;
        w3 = t1;
    }
    const uint32_t s = b & 3;  // alignbyte(hi, lo, s): bytes s .. s+3 of the pair (lo, hi)
    return make_uint4(__builtin_amdgcn_alignbyte(w1, w0, s), __builtin_amdgcn_alignbyte(w2, w1, s),
                      __builtin_amdgcn_alignbyte(w3, w2, s), __builtin_amdgcn_alignbyte(w0, w3, s));
}

// ---- byte-packed helpers for rows of u8 distances (a lane's 16-byte piece
// as four words).  Zero-byte test: (t - 0x01..01) & ~t & 0x80..80 is nonzero
// iff some byte of t is zero, and its lowest set flag marks the lowest zero
// byte (a borrow only carries upwards from a zero byte).

__device__ __forceinline__ uint32_t zero_byte_flags(uint32_t t) { return (t - 0x01010101u) & ~t & 0x80808080u; }

// any byte equal to 0xFF (an unreached entry)
__device__ __forceinline__ bool any_byte_ff(const uint4 a) {
    return (zero_byte_flags(~a.x) | zero_byte_flags(~a.y) | zero_byte_flags(~a.z) | zero_byte_flags(~a.w)) != 0;
}

// sum of the 16 bytes plus acc (v_sad_u8 against zero adds a word's four bytes)
__device__ __forceinline__ uint32_t bytes_sum(const uint4 a, uint32_t acc) {
    acc = __builtin_amdgcn_sad_u8(a.x, 0u, acc);
    acc = __builtin_amdgcn_sad_u8(a.y, 0u, acc);
    acc = __builtin_amdgcn_sad_u8(a.z, 0u, acc);
    return __builtin_amdgcn_sad_u8(a.w, 0u, acc);
}

// smallest of the 16 bytes
__device__ __forceinline__ uint32_t bytes_min(const uint4 a) {
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
    uint32_t m = 0xFFu;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t b0 = w[q] & 0xFFu, b1 = (w[q] >> 8) & 0xFFu, b2 = (w[q] >> 16) & 0xFFu, b3 = w[q] >> 24;
        m = min(m, min(min(b0, b1), min(b2, b3)));
    }
    return m;
}

// index (0..15) of the first byte equal to m, which must occur
__device__ __forceinline__ uint32_t bytes_first_eq(const uint4 a, uint32_t m) {
    const uint32_t mb = m * 0x01010101u;
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
    uint32_t idx = 0;
#pragma unroll
    for (int q = 3; q >= 0; q--) {
        const uint32_t z = zero_byte_flags(w[q] ^ mb);
        if (z) idx = 4u * (uint32_t)q + ((uint32_t)__builtin_ctz(z) >> 3);
    }
    return idx;
}

// index (0 .. 16 PC - 1) of the first byte equal to m in the parts p[0] (low) .. p[PC - 1]
template <int PC>
__device__ __forceinline__ uint32_t bytes_first_eq_n(const uint4 (&p)[PC], uint32_t m) {
    const uint32_t mb = m * 0x01010101u;
    uint32_t idx = 0;
#pragma unroll
    for (int q = 4 * PC - 1; q >= 0; q--) {
        const uint4 x = p[q >> 2];
        const uint32_t w = (q & 3) == 0 ? x.x : (q & 3) == 1 ? x.y : (q & 3) == 2 ? x.z : x.w;
        const uint32_t z = zero_byte_flags(w ^ mb);
        if (z) idx = 4u * (uint32_t)q + ((uint32_t)__builtin_ctz(z) >> 3);
    }
    return idx;
}

// For the bytes y_b of dm (entries of a row of the sample distance matrix,
// each < 255) that are <= L (L <= 255): the sum of the matching bytes of d
// is added to sum and their number to cnt.  Even and odd bytes are compared
// as 16-bit halves: 0x100 + L - y has bit 8 set iff y <= L, and never borrows
// across halves.
__device__ __forceinline__ void bytes_sum_le(const uint4 d, const uint4 dm, uint32_t L, uint32_t& sum,
                                             uint32_t& cnt) {
    const uint32_t C = 0x01000100u + L * 0x00010001u;
    const uint32_t dw[4] = {d.x, d.y, d.z, d.w}, yw[4] = {dm.x, dm.y, dm.z, dm.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t fe = (C - (yw[q] & 0x00FF00FFu)) & 0x01000100u;          // even bytes 0, 2
        const uint32_t fo = (C - ((yw[q] >> 8) & 0x00FF00FFu)) & 0x01000100u;   // odd bytes 1, 3
        const uint32_t mask = ((fe >> 8) * 0xFFu) | (((fo >> 8) * 0xFFu) << 8);
        sum = __builtin_amdgcn_sad_u8(dw[q] & mask, 0u, sum);
        cnt += (uint32_t)__builtin_popcount(fe | (fo << 1));
    }
}

// Value of the partner lane at step s of a reduction over aligned groups of
// up to 16 lanes, by DPP lane permutations inside a row: swap neighbours,
// swap pairs, then mirror the half row and the row.  After steps 0 .. lg-1
// combining x with its partner, every lane holds its 2^lg-lane group's total
// (mirroring pairs each lane with one of the other half, which by then holds
// that half's total).
__device__ __forceinline__ uint32_t dpp_partner(uint32_t x, int s) {
    switch (s) {
        case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
        default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false); // row_mirror
    }
}

// Group sums and minima over aligned groups of G <= 16 lanes (all lanes active).
template <int G>
__device__ __forceinline__ uint32_t group_sum32(uint32_t x) {
    static_assert(G <= 16, "groups of at most 16 lanes");
#pragma unroll
    for (int s = 0; (1 << s) < G; s++) x += dpp_partner(x, s);
    return x;
}

template <int G>
__device__ __forceinline__ int64_t group_sum64(int64_t x) {
    static_assert(G <= 16, "groups of at most 16 lanes");
#pragma unroll
    for (int s = 0; (1 << s) < G; s++) {
        const uint64_t lo = dpp_partner((uint32_t)x, s), hi = dpp_partner((uint32_t)((uint64_t)x >> 32), s);
        x += (int64_t)((hi << 32) | lo);
    }
    return x;
}

template <int G>
__device__ __forceinline__ uint32_t group_min32(uint32_t x) {
    static_assert(G <= 16, "groups of at most 16 lanes");
#pragma unroll
    for (int s = 0; (1 << s) < G; s++) x = min(x, dpp_partner(x, s));
    return x;
}

// Row stride of the LDS histogram of k_reduce_rows: hlen made odd, so that
// counters (i, d) of samples that differ mod 64 sit in different banks when d
// is the same.
__host__ __device__ inline int64_t hist_stride(int64_t hlen) { return hlen | 1; }

// histogram over non-sampled nodes (as k_reduce).  With LDS the block's copy
// is [k][hist_stride(hlen)], and each lane takes its piece rotated so that the
// 64 lanes of one update count 64 samples that differ mod 64 (when k allows):
// without the rotation the node slots of a wave (neighbouring nodes, which
// mostly share a distance) would all add to the same counter.  (Measured on
// the round trip of the directed R-MAT scale-22 graph, k = 128: 179 us per
// launch without the rotation, 84 us rotating by the node slot alone, 64 us
// as here; a [d][i] layout was slower, 157 us.)  kRowsInFlight pieces are
// refilled in turn, so the next trips' loads are in flight while one is
// counted.
template <typename DT, bool RT, int G, bool USE_LDS>
__global__ __launch_bounds__(kBlock) void k_reduce_rows(const DT* __restrict__ D, const DT* __restrict__ Dr,
                                                        int64_t n, int32_t k, const int32_t* __restrict__ sidx,
                                                        int64_t hlen, int32_t* __restrict__ hist, DevFlags* flags) {
    extern __shared__ int32_t lds_hist[];  // [k][hist_stride(hlen)] with USE_LDS
    if (n < 1) return;
    const int64_t hs = hist_stride(hlen);
    if (USE_LDS) {
        for (int64_t t = threadIdx.x; t < (int64_t)k * hs; t += kBlock) lds_hist[t] = 0;
        __syncthreads();
    }
    constexpr int PER = RowPiece<DT, RT>::PER;
    constexpr int NPW = 64 / G;    // node slots per wave
    constexpr int SPB = 64 / PER;  // lane pieces per 64 samples
    const int sub = lane_id() & (G - 1);
    const uint32_t rot = (uint32_t)((lane_id() / G + NPW * (sub / SPB)) & (PER - 1));
    const uint32_t hlen32 = (uint32_t)min<int64_t>(hlen, 0xFFFFFFFFll);
    const int64_t stride = (int64_t)gridDim.x * (kBlock / G);
    bool bad = false;
    // LDS row starts of the lane's samples in rotated order (u8 rows)
    uint32_t lbase[sizeof(DT) == 1 ? 16 : 1];
    if constexpr (sizeof(DT) == 1) {
#pragma unroll
        for (int e = 0; e < 16; e++) lbase[e] = ((uint32_t)sub * 16u + ((e + rot) & 15u)) * (uint32_t)hs;
    }
    // counts the piece in rp (node v), then refills rp with node v + kRowsInFlight * stride
    auto step = [&](RawPiece<DT, RT>& rp, int64_t v) {
        const int32_t j = rp.j;
        if constexpr (sizeof(DT) == 1 && !RT && USE_LDS) {
            // u8 rows of one direction: one packed test for an unreached entry
            // or a distance past the bound (either fails the estimate, so the
            // node is not counted), then a byte extract and an add per entry
            const uint4 a = rotate_bytes(rp.a, rot);
            rp.fetch(D, Dr, sidx, v + kRowsInFlight * stride, n, k, sub);
            if (j >= 0) return;
            uint32_t le = 0, dummy = 0;
            bytes_sum_le(make_uint4(0, 0, 0, 0), a, (uint32_t)min<int64_t>(hlen - 1, 255), dummy, le);
            if (any_byte_ff(a) || le != 16u) {
                bad = true;
                return;
            }
            const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const uint32_t d = (w[e >> 2] >> (8 * (e & 3))) & 0xFFu;
                atomicAdd(&lds_hist[lbase[e] + d], 1);
            }
            return;
        }
        RowPiece<DT, RT> r;
        r.decode(rotate_bytes(rp.a, rot * (uint32_t)sizeof(DT)),
                 RT ? rotate_bytes(rp.b, rot * (uint32_t)sizeof(DT)) : rp.b);
        rp.fetch(D, Dr, sidx, v + kRowsInFlight * stride, n, k, sub);
        if (j >= 0) return;
        if (r.unreached) {
            bad = true;
            return;
        }
#pragma unroll
        for (int e = 0; e < PER; e++) {
            const uint32_t i = (uint32_t)sub * PER + ((e + rot) & (PER - 1));
            const uint32_t d = r.d[e];
            if (d >= hlen32) {
                bad = true;
            } else if (USE_LDS) {
                atomicAdd(&lds_hist[__umul24(i, (uint32_t)hs) + d], 1);
            } else {
                atomicAdd(&hist[(int64_t)i * hlen + d], 1);
            }
        }
    };
    const int64_t v0 = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
    RawPiece<DT, RT> pp[kRowsInFlight];
#pragma unroll
    for (int u = 0; u < kRowsInFlight; u++) pp[u].fetch(D, Dr, sidx, v0 + u * stride, n, k, sub);
    for (int64_t v = v0; v < n; v += kRowsInFlight * stride) {
#pragma unroll
        for (int u = 0; u < kRowsInFlight; u++)
            if (v + u * stride < n) step(pp[u], v + u * stride);
    }
    if (bad) flags->disconnected = 1;
    if (USE_LDS) {
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)k * hs; t += kBlock) {
            const int64_t i = t / hs, d = t - i * hs;
            const int32_t c = lds_hist[t];
            if (c && d < hlen) atomicAdd(&hist[i * hlen + d], c);
        }
    }
}

// Bytes of the estimate's small tables when copied to LDS: Tsum (k x tlen
// int64), src_sum (k int64), Tcnt (k x tlen int32), then dmat_c (k x k MT) at
// a 16-byte boundary.
inline size_t est_table_bytes(int32_t k, int64_t tlen, size_t mt_bytes) {
    const size_t head = (size_t)k * (size_t)tlen * 12 + (size_t)k * 8;
    return ((head + 15) & ~size_t(15)) + (size_t)k * (size_t)k * mt_bytes;
}

// The lane's PER entries of a row of dmat_c, one 16-byte load when the piece
// is a multiple of 16 bytes (then the row start is aligned too: k * sizeof(DT)
// is a multiple of 16, so k is a multiple of PER).
template <typename MT, int PER>
__device__ __forceinline__ void load_mt_piece(const MT* row, int sub, uint32_t (&m)[PER]) {
    constexpr int BYTES = PER * (int)sizeof(MT);
    if constexpr (BYTES % 16 == 0) {
        constexpr uint32_t mask = sizeof(MT) == 4 ? 0xFFFFFFFFu : ((1u << (8 * sizeof(MT))) - 1);
        const uint4* p = (const uint4*)row + (int64_t)sub * (BYTES / 16);
#pragma unroll
        for (int c = 0; c < BYTES / 16; c++) {
            const uint4 x = p[c];
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int e = 0; e < 4 / (int)sizeof(MT); e++)
                    m[c * (16 / (int)sizeof(MT)) + q * (4 / (int)sizeof(MT)) + e] =
                        (w[q] >> (e * 8 * (int)sizeof(MT))) & mask;
        }
    } else {
#pragma unroll
        for (int e = 0; e < PER; e++) m[e] = row[(int64_t)sub * PER + e];
    }
}

// the estimators (as k_estimate).  A wave takes rounds of 64 consecutive
// positions o: caller ids when inv is set (the node is v = inv[o], and the
// outputs go to o, so a wave's stores are consecutive; a row is whole cache
// lines, so reading rows in this order wastes nothing), else internal ids
// (outputs to orig[v]).  Round r of wave gw starts at 64 (gw + r nw), its
// trip t takes positions t * 64/G + q, one per group q of G lanes; a round's
// internal ids are loaded a round ahead, one per lane, and handed to the
// groups by a lane shuffle.  A node is sample c_j exactly when its distance to
// c_j is 0 (lengths are positive), so the argmin tells sampled nodes apart.
// With LT the small tables (dmat_c, Tcnt, Tsum, src_sum) are copied to LDS
// first.  Two row pieces are refilled in turn, so the next trip's loads are in
// flight while one is worked on; a lane of each group keeps its node's totals
// until the round ends, and then all 64 lanes finish their nodes at once.
template <typename DT, bool RT, typename MT, int G, int PC, bool LT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_estimate_rows(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ orig,
    const int32_t* __restrict__ inv, const MT* __restrict__ dmat_c, const int32_t* __restrict__ Tcnt,
    const int64_t* __restrict__ Tsum, int64_t tlen, const int64_t* __restrict__ src_sum, int64_t en, int64_t ed,
    double* S_hyb, double* S_samp, int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out, int32_t* delta_out,
    int64_t* sampsum_out, DevFlags* flags) {
    static_assert(G >= 2 && G <= 16, "two to sixteen lanes per node");
    static_assert(PC == 1 || ((PC == 2 || PC == 4) && sizeof(DT) == 1 && !RT && sizeof(MT) == 1),
                  "32- and 64-byte lanes for u8 rows of one direction");
    extern __shared__ __align__(16) unsigned char lds_tab[];
    if (n < 1) return;
    constexpr int PER = RowPiece<DT, RT>::PER;
    constexpr int NPW = 64 / G;  // nodes per wave and trip
    // row sums: a u8 row (either direction) sums below 2^32 for any k < 2^23
    using AT = typename std::conditional<sizeof(DT) == 1, uint32_t, int64_t>::type;
    const int64_t LIM = (int64_t)1 << 53;
    constexpr bool kPacked = sizeof(DT) == 1 && !RT && sizeof(MT) == 1;
    int64_t* l_ts = (int64_t*)lds_tab;
    int64_t* l_ss = l_ts + (int64_t)k * tlen;
    int32_t* l_tc = (int32_t*)(l_ss + k);
    MT* l_dm = (MT*)(lds_tab + ((((size_t)k * (size_t)tlen * 12 + (size_t)k * 8) + 15) & ~size_t(15)));
    if constexpr (LT) {
        const int64_t kt = (int64_t)k * tlen;
        for (int64_t t = threadIdx.x; t < kt; t += BLOCK) {
            l_ts[t] = Tsum[t];
            l_tc[t] = Tcnt[t];
        }
        for (int64_t t = threadIdx.x; t < k; t += BLOCK) l_ss[t] = src_sum[t];
        const int64_t kk = (int64_t)k * k;
        if ((kk * (int64_t)sizeof(MT)) % 4 == 0) {
            const uint32_t* s4 = (const uint32_t*)dmat_c;
            uint32_t* d4 = (uint32_t*)l_dm;
            for (int64_t t = threadIdx.x; t < kk * (int64_t)sizeof(MT) / 4; t += BLOCK) d4[t] = s4[t];
        } else {
            for (int64_t t = threadIdx.x; t < kk; t += BLOCK) l_dm[t] = dmat_c[t];
        }
        __syncthreads();
    }
    const int lane = lane_id();
    const int sub = lane & (G - 1);
    const int q = lane / G;
    bool any_ovf = false, any_unreached = false;
    const int64_t gw = (int64_t)blockIdx.x * (BLOCK / 64) + threadIdx.x / 64;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    const int64_t rounds = (n + 63) / 64;
    const int64_t my_rounds = gw < rounds ? (rounds - 1 - gw) / nw + 1 : 0;
    const int64_t trips = my_rounds * G;  // the same for every lane of the wave
    // a round's internal ids, one per lane (positions past the end read the last one)
    auto load_ids = [&](int64_t r) -> int32_t {
        const int64_t o = min((gw + r * nw) * 64 + lane, n - 1);
        return inv ? inv[o] : (int32_t)o;
    };
    int32_t ids_cur = load_ids(0), ids_nxt = load_ids(1);
    // the piece of trip s (s at most one round ahead of the trip in hand):
    // unconditional, so the registers never merge old and new values
    auto fetch = [&](RawPiece<DT, RT>& rp, int64_t s, int64_t r_now) {
        const int32_t ids = (s / G == r_now) ? ids_cur : ids_nxt;
        const int64_t v = __shfl(ids, (int)(s % G) * NPW + q);
        rp.a = ((const uint4*)(D + v * k))[sub * PC];
#pragma unroll
        for (int i = 1; i < PC; i++) rp.ax[i - 1] = ((const uint4*)(D + v * k))[sub * PC + i];
        rp.b = make_uint4(0, 0, 0, 0);
        if (RT) rp.b = ((const uint4*)(Dr + v * k))[sub];
    };
    // a node's totals, held by one lane of its group until the round's end
    int64_t ho = -1, hv = 0;
    int32_t hp = 0;
    uint32_t hdelta = 0, hlcnum = 0;
    AT hrowsum = 0, hlcsum = 0;
    bool hunr = false;
    // the end of Algorithm 1 for the nodes the lanes hold, all lanes at once
    auto finish = [&]() {
        if (ho < 0) return;
        const int64_t o = ho, v = hv;
        ho = -1;
        const int p = hp;
        const int64_t delta = hdelta;
        const int64_t lim = en == 1 ? delta * ed : delta * ed / en;
        double hyb, samp;
        int64_t piv, pub;
        bool ovf = false;
        const int64_t sum64 = (int64_t)hrowsum, lcsum64 = (int64_t)hlcsum, lcnum64 = (int64_t)hlcnum;
        if (delta == 0) {  // the node is sample c_p: its exact sum
            const int64_t S = LT ? l_ss[p] : src_sum[p];
            hyb = samp = (double)S;
            piv = pub = S;
            ovf = S >= LIM;
        } else {
            const int64_t tix = lim + 1;  // d > floor(Delta/eps)  <=>  d >= tix
            int64_t hnum = 0, hsum = 0;
            if (tix < tlen) {
                if constexpr (LT) {
                    hnum = l_tc[(uint32_t)p * (uint32_t)tlen + (uint32_t)tix];
                    hsum = l_ts[(uint32_t)p * (uint32_t)tlen + (uint32_t)tix];
                } else {
                    hnum = Tcnt[(int64_t)p * tlen + tix];
                    hsum = Tsum[(int64_t)p * tlen + tix];
                }
            }
            const int64_t hcsum = sum64 - lcsum64;
            const int64_t lnum = (n - 1) - hnum - (int64_t)(k - lcnum64);
            const int64_t a = hsum + hcsum;
            int64_t t1 = 0, t2 = 0, N = 0, ss = 0;
            ovf = __builtin_mul_overflow(a, lcnum64, &t1) || __builtin_mul_overflow(lcsum64, lnum, &t2) ||
                  __builtin_add_overflow(t1, t2, &N) || N >= LIM || lcnum64 < 1 || lnum < lcnum64;
            hyb = (double)N / (double)lcnum64;
            ovf = ovf || __builtin_mul_overflow(n - 1, sum64, &ss) || ss >= LIM;
            samp = (double)ss / (double)k;
            piv = LT ? l_ss[p] : src_sum[p];
            pub = piv + (n - 1) * delta;
        }
        const int64_t out = inv ? o : (int64_t)orig[v];
        if (S_hyb) S_hyb[out] = hyb;
        if (S_samp) S_samp[out] = samp;
        if (S_piv) S_piv[out] = piv;
        if (S_pub) S_pub[out] = pub;
        if (pivot_out) pivot_out[out] = p;
        if (delta_out) delta_out[out] = (int32_t)delta;
        if (sampsum_out) sampsum_out[out] = sum64;
        any_ovf = any_ovf || ovf;
        any_unreached = any_unreached || hunr;
    };
    auto step = [&](RawPiece<DT, RT>& rp, int64_t s) {
        const int t = (int)(s % G);
        const int64_t r = s / G;
        if (t == 0 && r > 0) {  // a new round: its ids were loaded a round ago
            ids_cur = ids_nxt;
            ids_nxt = load_ids(r + 1);
        }
        const int64_t o = (gw + r * nw) * 64 + t * NPW + q;
        const bool valid = o < n;
        const int64_t v = __shfl(ids_cur, t * NPW + q);
        uint32_t best;
        int32_t bi;
        AT sum, lcsum = 0;
        uint32_t lcnum = 0;
        bool unr;
        if constexpr (kPacked) {
            // u8 rows, one direction, u8 sample distances: byte-packed arithmetic
            // on the lane's PC pieces of 16 bytes
            uint4 pc[PC];
            pc[0] = rp.a;
#pragma unroll
            for (int i = 1; i < PC; i++) pc[i] = rp.ax[i - 1];
            fetch(rp, s + 2, r);
            bool ff = false;
            uint32_t m = 0xFFu, rs = 0;
#pragma unroll
            for (int i = 0; i < PC; i++) {
                ff = ff || any_byte_ff(pc[i]);
                m = min(m, bytes_min(pc[i]));
                rs = bytes_sum(pc[i], rs);
            }
            unr = valid && ff;
            const uint32_t at = bytes_first_eq_n<PC>(pc, m);
            const uint32_t key = group_min32<G>(valid ? ((m << 16) | ((uint32_t)sub * PER * PC + at)) : 0xFFFFFFFFu);
            best = key >> 16;  // the lowest index among equal minima
            bi = (int32_t)(key & 0xFFFFu);
            sum = group_sum32<G>(valid ? rs : 0u);
            const int64_t lim = en == 1 ? (int64_t)best * ed : (int64_t)best * ed / en;
            if (valid && best != 0) {
                const uint4* dmr = LT ? (const uint4*)(l_dm + (uint32_t)bi * (uint32_t)k)
                                      : (const uint4*)(dmat_c + (int64_t)bi * k);
                const uint32_t L8 = lim >= 255 ? 255u : (uint32_t)lim;
#pragma unroll
                for (int i = 0; i < PC; i++) bytes_sum_le(pc[i], dmr[sub * PC + i], L8, lcsum, lcnum);
            }
        } else {
            RowPiece<DT, RT> rw;
            rw.decode(rp.a, rp.b);
            fetch(rp, s + 2, r);
            if (!valid) {
#pragma unroll
                for (int e = 0; e < PER; e++) rw.d[e] = 0xFFFFFFFFu;
                rw.unreached = false;
            }
            unr = rw.unreached;
            // argmin (lowest index among equal minima) and sum
            best = 0xFFFFFFFFu;
            bi = 0;
            sum = 0;
#pragma unroll
            for (int e = 0; e < PER; e++) {
                if (rw.d[e] < best) {
                    best = rw.d[e];
                    bi = sub * PER + e;
                }
                sum += valid ? (AT)rw.d[e] : (AT)0;
            }
            if constexpr (sizeof(DT) == 1) {
                // one key: distance (< 2^9, an all-ones placeholder for a masked
                // node) above the index (k <= 256 for rows of at most 256 bytes)
                const uint32_t key = group_min32<G>(valid ? ((best << 16) | (uint32_t)bi) : 0xFFFFFFFFu);
                best = key >> 16;
                bi = (int32_t)(key & 0xFFFFu);
            } else {
#pragma unroll
                for (int st = 0; (1 << st) < G; st++) {
                    const uint32_t ob = dpp_partner(best, st);
                    const int32_t oi = (int32_t)dpp_partner((uint32_t)bi, st);
                    if (ob < best || (ob == best && oi < bi)) {
                        best = ob;
                        bi = oi;
                    }
                }
            }
            if constexpr (sizeof(AT) == 4) sum = group_sum32<G>(sum);
            else sum = group_sum64<G>(sum);
            // the L cap C split against the pivot's row of the sample distances:
            // dmat * num <= Delta * den  <=>  dmat <= floor(Delta * den / num)
            const int64_t thr = (int64_t)best * ed;
            const int64_t lim = en == 1 ? thr : thr / en;
            const uint32_t lim32 = (uint32_t)min<int64_t>(lim, 0xFFFFFFFFll);
            if (valid && best != 0) {
                uint32_t m[PER];
                if constexpr (LT) load_mt_piece<MT, PER>(l_dm + (uint32_t)bi * (uint32_t)k, sub, m);
                else load_mt_piece<MT, PER>(dmat_c + (int64_t)bi * k, sub, m);
#pragma unroll
                for (int e = 0; e < PER; e++) {
                    if (m[e] <= lim32) {
                        lcsum += (AT)rw.d[e];
                        lcnum += 1;
                    }
                }
            }
        }
        if constexpr (sizeof(AT) == 4) lcsum = group_sum32<G>(lcsum);
        else lcsum = group_sum64<G>(lcsum);
        lcnum = group_sum32<G>(lcnum);
        const bool unreached = group_sum32<G>(unr ? 1u : 0u) != 0;
        // every lane of the group now holds the node's totals: the lane whose
        // sub index is this trip's number in the round keeps them
        if (sub == t) {
            ho = valid ? o : -1;
            hv = v;
            hp = bi;
            hdelta = best;
            hrowsum = sum;
            hlcsum = lcsum;
            hlcnum = lcnum;
            hunr = unreached;
        }
        if (t == G - 1) finish();
    };
    RawPiece<DT, RT> pa, pb;
    fetch(pa, 0, 0);
    fetch(pb, 1, 0);
    for (int64_t s = 0; s < trips; s += 2) {
        step(pa, s);
        if (s + 1 < trips) step(pb, s + 1);
    }
    if (any_ovf) flags->overflow = 1;
    if (any_unreached) flags->disconnected = 1;
}

template <typename DT, bool RT, typename MT>
__global__ void k_dmat(const DT* __restrict__ D, const DT* __restrict__ Dr, const int32_t* __restrict__ samples,
                       int32_t k, int32_t* __restrict__ dmat_out, MT* __restrict__ dmat_c, DevFlags* flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)k * k) return;
    const int32_t i = (int32_t)(t / k), j = (int32_t)(t % k);
    const int64_t off = (int64_t)samples[j] * k + i;
    if (unreached_at<DT, RT>(D, Dr, off)) flags->disconnected = 1;
    const uint32_t d = dist_at<DT, RT>(D, Dr, off);
    dmat_out[t] = (int32_t)d;
    dmat_c[t] = (MT)d;
}

// One block per sample: sums the histogram copies, reverse inclusive scan
// into T[i][t] for t = 0..maxd+1 (T[i][maxd+1] = 0), then S(c_i).
__global__ __launch_bounds__(kBlock) void k_suffix(const int32_t* __restrict__ hist, int32_t nslots, int32_t k,
                                                   int32_t hrows, int64_t hlen, int64_t maxd, const int32_t* __restrict__ dmat,
                                                   int32_t* __restrict__ Tcnt, int64_t* __restrict__ Tsum,
                                                   int64_t* __restrict__ src_sum) {
    __shared__ int64_t wc[kBlock / 64], ws[kBlock / 64];
    const int32_t i = blockIdx.x;
    const int64_t tlen = maxd + 2;
    int32_t* tc = Tcnt + (int64_t)i * tlen;
    int64_t* ts = Tsum + (int64_t)i * tlen;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t carry_c = 0, carry_s = 0;
    if (threadIdx.x == 0) {
        tc[maxd + 1] = 0;
        ts[maxd + 1] = 0;
    }
    // short tables (BFS levels): the slots are summed first by all threads,
    // kBlock / (maxd + 1) of them per distance
    __shared__ unsigned long long hsm[kBlock];
    const bool small = maxd + 1 <= kBlock;
    if (small) {
        const int32_t D = (int32_t)(maxd + 1), G = kBlock / D;
        hsm[threadIdx.x] = 0;
        __syncthreads();
        const int32_t dd = (int32_t)threadIdx.x % D, g = (int32_t)threadIdx.x / D;
        if (g < G && dd < hlen) {
            unsigned long long c = 0;
            for (int32_t s = g; s < nslots; s += G) c += (unsigned long long)hist[((int64_t)s * hrows + i) * hlen + dd];
            if (c) atomicAdd(&hsm[dd], c);
        }
        __syncthreads();
    }
    for (int64_t top = maxd; top >= 0; top -= kBlock) {
        const int64_t d = top - threadIdx.x;
        int64_t c = 0;
        if (d >= 0 && d < hlen) {
            if (small)
                c = (int64_t)hsm[d];
            else
                for (int32_t s = 0; s < nslots; s++) c += hist[((int64_t)s * hrows + i) * hlen + d];
        }
        int64_t s = c * (d >= 0 ? d : 0);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t yc = __shfl_up(c, off);
            const int64_t ys = __shfl_up(s, off);
            if (lane >= off) {
                c += yc;
                s += ys;
            }
        }
        if (lane == 63) {
            wc[wave] = c;
            ws[wave] = s;
        }
        __syncthreads();
        int64_t pc = carry_c, ps = carry_s;
        for (int w = 0; w < wave; w++) {
            pc += wc[w];
            ps += ws[w];
        }
        if (d >= 0) {
            tc[d] = (int32_t)(pc + c);
            ts[d] = ps + s;
        }
        for (int w = 0; w < kBlock / 64; w++) {
            carry_c += wc[w];
            carry_s += ws[w];
        }
        __syncthreads();
    }
    // S(c_i) = (sum over non-sampled u of d(c_i,u)) + sum_j d(c_i,c_j)
    int64_t rs = 0;
    for (int32_t j = threadIdx.x; j < k; j += kBlock) rs += dmat[(int64_t)i * k + j];
    rs = wave_sum64(rs);
    __syncthreads();
    if (lane == 0) wc[wave] = rs;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < kBlock / 64; w++) tot += wc[w];
        src_sum[i] = carry_s + tot;
    }
}

// Long histograms (weighted distances): the same tail tables in three
// parallel steps over chunks of kChunk entries.
constexpr int64_t kChunk = 4096;

__global__ __launch_bounds__(kBlock) void k_chunk_sums(const int32_t* __restrict__ hist, int32_t nslots, int32_t k,
                                                       int32_t hrows, int64_t hlen, int64_t* __restrict__ csum_c,
                                                       int64_t* __restrict__ csum_s, int64_t nchunks) {
    __shared__ int64_t wc[kBlock / 64], ws[kBlock / 64];
    const int64_t c = blockIdx.x;
    const int32_t i = blockIdx.y;
    int64_t cc = 0, cs = 0;
    for (int64_t d = c * kChunk + threadIdx.x; d < (c + 1) * kChunk && d < hlen; d += kBlock) {
        int64_t h = 0;
        for (int32_t s = 0; s < nslots; s++) h += hist[((int64_t)s * hrows + i) * hlen + d];
        cc += h;
        cs += h * d;
    }
    cc = wave_sum64(cc);
    cs = wave_sum64(cs);
    if (lane_id() == 0) {
        wc[threadIdx.x >> 6] = cc;
        ws[threadIdx.x >> 6] = cs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0, b = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            a += wc[w];
            b += ws[w];
        }
        csum_c[(int64_t)i * nchunks + c] = a;
        csum_s[(int64_t)i * nchunks + c] = b;
    }
}

// per sample: carry[c] = totals of the chunks above c (one thread per sample)
__global__ void k_chunk_carry(int64_t* csum_c, int64_t* csum_s, int32_t k, int64_t nchunks) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    int64_t a = 0, b = 0;
    for (int64_t c = nchunks - 1; c >= 0; c--) {
        const int64_t x = csum_c[(int64_t)i * nchunks + c], y = csum_s[(int64_t)i * nchunks + c];
        csum_c[(int64_t)i * nchunks + c] = a;
        csum_s[(int64_t)i * nchunks + c] = b;
        a += x;
        b += y;
    }
}

__global__ __launch_bounds__(kBlock) void k_chunk_suffix(const int32_t* __restrict__ hist, int32_t nslots, int32_t k,
                                                         int32_t hrows, int64_t hlen, int64_t maxd, const int64_t* __restrict__ carry_c,
                                                         const int64_t* __restrict__ carry_s, int64_t nchunks,
                                                         int32_t* __restrict__ Tcnt, int64_t* __restrict__ Tsum) {
    __shared__ int64_t wc[kBlock / 64], ws[kBlock / 64];
    const int64_t ch = blockIdx.x;
    const int32_t i = blockIdx.y;
    const int64_t tlen = maxd + 2;
    int32_t* tc = Tcnt + (int64_t)i * tlen;
    int64_t* ts = Tsum + (int64_t)i * tlen;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t carry_cc = carry_c[(int64_t)i * nchunks + ch], carry_ss = carry_s[(int64_t)i * nchunks + ch];
    if (ch == 0 && threadIdx.x == 0) {
        tc[maxd + 1] = 0;
        ts[maxd + 1] = 0;
    }
    const int64_t lo = ch * kChunk;
    const int64_t hi_ = std::min<int64_t>((ch + 1) * kChunk, maxd + 1);
    for (int64_t top = hi_ - 1; top >= lo; top -= kBlock) {
        const int64_t d = top - threadIdx.x;
        int64_t c = 0;
        if (d >= lo && d < hlen)
            for (int32_t s = 0; s < nslots; s++) c += hist[((int64_t)s * hrows + i) * hlen + d];
        int64_t sm = c * (d >= 0 ? d : 0);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t yc = __shfl_up(c, off);
            const int64_t ys = __shfl_up(sm, off);
            if (lane >= off) {
                c += yc;
                sm += ys;
            }
        }
        if (lane == 63) {
            wc[wave] = c;
            ws[wave] = sm;
        }
        __syncthreads();
        int64_t pc = carry_cc, ps = carry_ss;
        for (int w = 0; w < wave; w++) {
            pc += wc[w];
            ps += ws[w];
        }
        if (d >= lo) {
            tc[d] = (int32_t)(pc + c);
            ts[d] = ps + sm;
        }
        for (int w = 0; w < kBlock / 64; w++) {
            carry_cc += wc[w];
            carry_ss += ws[w];
        }
        __syncthreads();
    }
}

__global__ void k_src_sum(const int64_t* __restrict__ Tsum, int64_t tlen, const int32_t* __restrict__ dmat, int32_t k,
                          int64_t* __restrict__ src_sum) {
    const int32_t i = blockIdx.x;
    int64_t rs = 0;
    for (int32_t j = threadIdx.x; j < k; j += 64) rs += dmat[(int64_t)i * k + j];
    rs = wave_sum64(rs);
    if (threadIdx.x == 0) src_sum[i] = Tsum[(int64_t)i * tlen] + rs;
}

template <typename DT, bool RT, typename MT>
__global__ __launch_bounds__(kBlock) void k_estimate(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ sidx,
    const int32_t* __restrict__ orig, const MT* __restrict__ dmat_c, const int32_t* __restrict__ Tcnt,
    const int64_t* __restrict__ Tsum, int64_t tlen, const int64_t* __restrict__ src_sum, int64_t en, int64_t ed,
    double* S_hyb, double* S_samp, int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out, int32_t* delta_out,
    int64_t* sampsum_out, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    bool any_ovf = false, any_unreached = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        uint32_t best = 0xFFFFFFFFu;
        int32_t p = 0;
        int64_t sum = 0;
        bool unreached = false;
        for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
            if (d < best) {  // strict: ties keep the lower sample index
                best = d;
                p = i;
            }
            sum += d;
        });
        const int64_t delta = best;
        if (RT) {
            // an unreached entry is the maximal code in either direction
            unreached = unreached_at<DT, RT>(D, Dr, v * k + p);
        } else {
            unreached = best == DistT<DT>::never;
        }
        const int32_t j = sidx[v];
        double hyb, samp;
        int64_t piv, pub;
        bool ovf = false;
        if (j >= 0) {
            const int64_t S = src_sum[j];
            hyb = samp = (double)S;
            piv = pub = S;
            ovf = S >= LIM;
        } else {
            const int64_t thr = delta * ed;
            const MT* drow = dmat_c + (int64_t)p * k;
            int64_t lcsum = 0;
            int32_t lcnum = 0;
            for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
                if ((int64_t)drow[i] * en <= thr) {
                    lcsum += d;
                    lcnum += 1;
                }
            });
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
            pub = piv + (n - 1) * delta;
        }
        const int64_t o = orig[v];
        if (S_hyb) S_hyb[o] = hyb;
        if (S_samp) S_samp[o] = samp;
        if (S_piv) S_piv[o] = piv;
        if (S_pub) S_pub[o] = pub;
        if (pivot_out) pivot_out[o] = p;
        if (delta_out) delta_out[o] = (int32_t)delta;
        if (sampsum_out) sampsum_out[o] = sum;
        any_ovf = any_ovf || ovf;
        any_unreached = any_unreached || unreached;
    }
    if (any_ovf) flags->overflow = 1;
    if (any_unreached) flags->disconnected = 1;
}

// Sec. 4 / Algorithm 2 (Sec. 4.2), step 1: each sample's row of the sample
// distance matrix in increasing order -- perm[p][j] is the sample of rank j
// by distance from c_p (index order among equal distances), ds[p][j] that
// distance (32-bit whatever the width of dmat_c); rows of kp = k rounded up
// to 8 entries, padded with index 0 and distance ~0.  One block per sample;
// bitonic sort of the keys (distance << 12 | index) in LDS, k2 = the power of
// two >= k (<= 4096).
template <typename MT>
__global__ __launch_bounds__(kBlock) void k_sort_rows(const MT* __restrict__ dmat_c, int32_t k, int32_t k2,
                                                      int32_t kp, uint32_t* __restrict__ perm,
                                                      uint32_t* __restrict__ ds) {
    extern __shared__ uint64_t skey[];
    const int64_t p = blockIdx.x;
    for (int32_t i = threadIdx.x; i < k2; i += kBlock)
        skey[i] = i < k ? ((uint64_t)dmat_c[p * k + i] << 12) | (uint64_t)i : ~0ull;
    __syncthreads();
    for (int32_t size = 2; size <= k2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = threadIdx.x; t < k2 / 2; t += kBlock) {
                const int32_t lo = 2 * t - (t & (stride - 1));  // pairs (lo, lo + stride), bit `stride` of lo clear
                const int32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = skey[lo], b = skey[hi];
                if ((a > b) == up) {
                    skey[lo] = b;
                    skey[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t j = threadIdx.x; j < kp; j += kBlock) {
        const uint64_t x = j < k ? skey[j] : ~0ull;
        perm[p * kp + j] = j < k ? (uint32_t)(x & 0xFFF) : 0u;
        ds[p * kp + j] = j < k ? (uint32_t)(x >> 12) : ~0u;
    }
}

// Sec. 4 and Algorithm 2 (Sec. 4.2): every candidate estimate has Eq. (6)'s
// form with L cap C a prefix of the samples ranked by distance from the
// node's pivot c_p (k_sort_rows), so all of them come from prefix sums along
// those ranks.  With LC the first lc ranks, HC the others and H, |H| the
// nodes outside C beyond the candidate's threshold:
//   N   = (sum_H d(c_p,u) + sum_HC d(v,c_i)) * lc + |L| * sum_LC d(v,c_i), estimate N / lc
//   err = ((lc * sum_LC d^2 - (sum_LC d)^2) / lc^3) * |L| + (sum_F (d - d_p)^2 / |F|) * |H|
// with F = HC, or, when HC is empty, F = the samples at the largest distance
// from c_p (Sec. 4.1's "suffix" of the farthest samples: the last ranks), and
// |L| = n-1-|H|-|HC|, in exactly this order of double operations on exact
// integers (d = d(v,c_i), d_p = d(c_p,c_i)).
//   * hybrid, eps = num/den (the call's, then each of the adaptive list): LC =
//     {i : d_p <= floor(Delta*den/num)}, H beyond that threshold (tail tables);
//     S_err is the call's error, S_ad the first smallest error over the list.
//   * threshold sweep: pure pivoting, S(c_p) with error (sum_i (d - d_p)^2 / k)
//     * (n-1-k), then for every distinct d_p = T, increasing, LC = the ranks at
//     distance <= T and H the nodes outside C beyond T other than v itself
//     (beyond T when Delta > T); the smallest error wins, the first on ties.
// The ranks, and so the candidate thresholds, depend on the pivot alone:
// nodes are grouped by pivot and a wavefront takes up to 64 nodes of one
// pivot, one per lane, walking the ranks in step (uniform loads of the sorted
// row, uniform tail lookups, every lane evaluating its own node's candidate
// at each distinct distance).  Each lane's distance row is staged in LDS when
// 64 rows fit.
constexpr int kErrEps = 8;             // the call's eps + up to 7 listed ones
constexpr int kErrBucketBlocks = 512;  // blocks of the bucketing kernels
struct ErrEps {
    int32_t count;  // entries used; entry 0 is the call's eps
    int64_t num[kErrEps], den[kErrEps];
};

__device__ __forceinline__ void prefix_candidate(int64_t n, int32_t k, int64_t lc, int64_t lcsum, uint64_t lcsq,
                                                 int64_t hcsum, uint64_t fsq, int64_t fnum, int64_t hnum,
                                                 int64_t hsum, double& est, double& err, bool& eo) {
    const int64_t LIM = (int64_t)1 << 53;
    const int64_t hcnum = k - lc;
    const int64_t lnum = (n - 1) - hnum - hcnum;
    int64_t t1 = 0, t2 = 0, N = 0, vn1 = 0, vn2 = 0, varnum = 0;
    bool e = __builtin_mul_overflow(hsum + hcsum, lc, &t1) || __builtin_mul_overflow(lcsum, lnum, &t2) ||
             __builtin_add_overflow(t1, t2, &N) || N >= LIM || lc < 1 || lnum < lc || hnum < 0;
    e = e || __builtin_mul_overflow(lc, (int64_t)lcsq, &vn1) || __builtin_mul_overflow(lcsum, lcsum, &vn2) ||
        __builtin_sub_overflow(vn1, vn2, &varnum);
    eo = eo || e;
    est = (double)N / (double)lc;
    const double tL = ((double)varnum / (double)(lc * lc * lc)) * (double)lnum;
    const double tH = ((double)(int64_t)fsq / (double)fnum) * (double)hnum;
    err = tL + tH;
}

// Per node: the pivot of an unsampled node (lowest index among the nearest
// samples), its row sum and its total squared pivot error
// sum_i (d(v,c_i) - d(c_p,c_i))^2; sampled nodes get their outputs here (the
// exact sum, error 0) and pivot -1.  Each block counts its nodes per pivot in
// LDS, keeps its counts (bcnt[block][p]) and adds them to the totals: one
// global atomic per (block, pivot) instead of one per node on a few hot
// pivots.
template <typename DT, bool RT, typename MT>
__global__ __launch_bounds__(kBlock) void k_err_pivot(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n,
                                                      int32_t k, const int32_t* __restrict__ sidx, int32_t bit_base,
                                                      const int32_t* __restrict__ orig, const MT* __restrict__ dmat_c,
                                                      const int64_t* __restrict__ src_sum, int32_t* __restrict__ piv,
                                                      int64_t* __restrict__ vsum, uint64_t* __restrict__ vsq,
                                                      int32_t* __restrict__ cnt, int32_t* __restrict__ bcnt,
                                                      double* S_err, double* S_ad, double* S_ad_err, double* S_sweep,
                                                      double* S_sweep_err, DevFlags* flags) {
    extern __shared__ int32_t lcnt[];
    bool big = false;
    for (int32_t p = threadIdx.x; p < k; p += kBlock) lcnt[p] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int32_t js = sidx[v];
        if (js >= 0) {
            const int64_t o = orig[v];
            const double ex = (double)src_sum[js - bit_base];
            if (S_err) S_err[o] = 0.0;
            if (S_ad) S_ad[o] = ex;
            if (S_ad_err) S_ad_err[o] = 0.0;
            if (S_sweep) S_sweep[o] = ex;
            if (S_sweep_err) S_sweep_err[o] = 0.0;
            piv[v] = -1;
            continue;
        }
        uint32_t best = 0xFFFFFFFFu;
        int32_t p = 0;
        int64_t sum = 0;
        for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
            if (d < best) {
                best = d;
                p = i;
            }
            sum += d;
        });
        const MT* drow = dmat_c + (int64_t)p * k;
        uint64_t sq = 0;
        for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
            const int64_t dl = drow[i];
            big = big || d >= (1u << 25) || dl >= (1 << 25);  // squares summed over k <= 4096 stay below 2^62
            const int64_t df = (int64_t)d - dl;
            sq += (uint64_t)(df * df);
        });
        piv[v] = p;
        vsum[v] = sum;
        vsq[v] = sq;
        atomicAdd(&lcnt[p], 1);
    }
    if (big) flags->overflow = 1;
    __syncthreads();
    for (int32_t p = threadIdx.x; p < k; p += kBlock) {
        const int32_t c = lcnt[p];
        bcnt[(int64_t)blockIdx.x * k + p] = c;
        if (c) atomicAdd(&cnt[p], c);
    }
}

// One block: exclusive prefix sums of the per-pivot counts (node offsets) and
// of ceil(count / 64) (wavefront tasks), each with its total at entry k.
__global__ __launch_bounds__(kBlock) void k_err_buckets(const int32_t* __restrict__ cnt, int32_t k,
                                                        int32_t* __restrict__ start, int32_t* __restrict__ tstart) {
    __shared__ int32_t wa[kBlock / 64], wb[kBlock / 64];
    const int32_t per = (k + kBlock - 1) / kBlock;
    const int32_t lo = threadIdx.x * per;
    int32_t sa = 0, sb = 0;
    for (int32_t i = lo; i < lo + per && i < k; i++) {
        sa += cnt[i];
        sb += (cnt[i] + 63) / 64;
    }
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int32_t ia = sa, ib = sb;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t ya = __shfl_up(ia, off), yb = __shfl_up(ib, off);
        if (lane >= off) {
            ia += ya;
            ib += yb;
        }
    }
    if (lane == 63) {
        wa[wave] = ia;
        wb[wave] = ib;
    }
    __syncthreads();
    int32_t ba = 0, bb = 0;
    for (int w = 0; w < wave; w++) {
        ba += wa[w];
        bb += wb[w];
    }
    int32_t ra = ba + ia - sa, rb = bb + ib - sb;  // exclusive
    for (int32_t i = lo; i < lo + per && i < k; i++) {
        start[i] = ra;
        tstart[i] = rb;
        ra += cnt[i];
        rb += (cnt[i] + 63) / 64;
    }
    if (threadIdx.x == kBlock - 1) {
        start[k] = ra;
        tstart[k] = rb;
    }
}

// Places the nodes in their pivot's bucket: the same blocks over the same
// nodes as k_err_pivot reserve their share of each bucket with one atomic per
// pivot, then hand out slots from LDS (order within a bucket is arbitrary).
__global__ __launch_bounds__(kBlock) void k_err_fill(const int32_t* __restrict__ piv, int64_t n, int32_t k,
                                                     const int32_t* __restrict__ start,
                                                     const int32_t* __restrict__ bcnt, int32_t* __restrict__ fill,
                                                     int32_t* __restrict__ order) {
    extern __shared__ int32_t lpos[];
    for (int32_t p = threadIdx.x; p < k; p += kBlock) {
        const int32_t c = bcnt[(int64_t)blockIdx.x * k + p];
        lpos[p] = c ? start[p] + atomicAdd(&fill[p], c) : 0;
    }
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int32_t p = piv[v];
        if (p >= 0) order[atomicAdd(&lpos[p], 1)] = (int32_t)v;
    }
}

// One wavefront (block of 64) per task: up to 64 unsampled nodes of one
// pivot.  AT: the prefix accumulators' type (32-bit when every square and
// its sum over k <= 4096 ranks fits, as for distances below 2^9).
template <typename DT, bool RT, bool STAGED, typename AT>
__global__ __launch_bounds__(64) void k_errsweep(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, int32_t kp,
    const int32_t* __restrict__ orig, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ ds,
    const int64_t* __restrict__ vsum, const uint64_t* __restrict__ vsq, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ start, const int32_t* __restrict__ tstart, const int32_t* __restrict__ order,
    int32_t stride, const int32_t* __restrict__ Tcnt, const int64_t* __restrict__ Tsum, int64_t tlen,
    const int64_t* __restrict__ src_sum, ErrEps E, double* S_err, double* S_ad, double* S_ad_err, double* S_sweep,
    double* S_sweep_err, DevFlags* flags) {
    extern __shared__ uint32_t stage_words[];
    const int32_t task = blockIdx.x;
    if (task >= tstart[k]) return;
    // the pivot whose tasks include this one: the last p with tstart[p] <= task
    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (tstart[mid] <= task) lo = mid;
        else hi = mid - 1;
    }
    const int32_t p = __builtin_amdgcn_readfirstlane(lo);
    const int lane = threadIdx.x;
    const int32_t first = start[p] + (task - tstart[p]) * 64;
    const bool active = first + lane < start[p] + cnt[p];
    const int64_t v = active ? order[first + lane] : 0;
    const int64_t row = v * k;
    const bool want_eps = S_err || S_ad || S_ad_err;
    const bool want_sw = S_sweep || S_sweep_err;
    const DT* srow = nullptr;
    const DT* srow_r = nullptr;
    if (STAGED) {
        // this lane's row (and reverse row) into its LDS slot
        uint8_t* slot = (uint8_t*)stage_words + (size_t)lane * stride;
        const int32_t bytes = k * (int32_t)sizeof(DT);
        if (active) {
            const uint8_t* g = (const uint8_t*)(D + row);
            const uint8_t* gr = RT ? (const uint8_t*)(Dr + row) : nullptr;
            if (bytes % 16 == 0) {
                for (int32_t b = 0; b < bytes; b += 16) {
                    const uint4 x = *(const uint4*)(g + b);
                    uint32_t* w = (uint32_t*)(slot + b);
                    w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
                    if (RT) {
                        const uint4 y = *(const uint4*)(gr + b);
                        uint32_t* wr = (uint32_t*)(slot + bytes + b);
                        wr[0] = y.x; wr[1] = y.y; wr[2] = y.z; wr[3] = y.w;
                    }
                }
            } else {
                for (int32_t i = 0; i < k; i++) {
                    ((DT*)slot)[i] = D[row + i];
                    if (RT) ((DT*)(slot + bytes))[i] = Dr[row + i];
                }
            }
        }
        srow = (const DT*)slot;
        srow_r = (const DT*)(slot + bytes);
    }
    // every lane reads its own slot (or row 0 of D when inactive): in bounds
    // without a branch; inactive lanes then see 0
    auto dist = [&](int32_t i) -> uint32_t {
        uint32_t a;
        if (STAGED) {
            a = (uint32_t)srow[i];
            if (RT) a += (uint32_t)srow_r[i];
        } else {
            a = dist_at<DT, RT>(D, Dr, row + i);
        }
        return active ? a : 0u;
    };
    const uint32_t* pr = perm + (int64_t)p * kp;
    const uint32_t* dr = ds + (int64_t)p * kp;
    const int32_t* tc = Tcnt + (int64_t)p * tlen;
    const int64_t* ts = Tsum + (int64_t)p * tlen;
    // the sorted row in groups of kRun ranks: uniform loads first, then the
    // lanes' row reads, then the arithmetic
    constexpr int kRun = 8;
    uint32_t ri[kRun], rd[kRun];
    int64_t rl[kRun];
    auto load_run = [&](int32_t j0) {  // rows are padded to a multiple of kRun
#pragma unroll
        for (int t = 0; t < kRun; t++) {
            ri[t] = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)pr[j0 + t]);
            rl[t] = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)dr[j0 + t]);
        }
#pragma unroll
        for (int t = 0; t < kRun; t++) rd[t] = dist((int32_t)ri[t]);
    };
    // the row sum and the total squared pivot error, from the pivot pass
    const int64_t sum = active ? vsum[v] : 0;
    const uint64_t sq_all = active ? vsq[v] : 0;
    const int64_t delta = dist(p);
    // the hybrid thresholds floor(Delta/eps), their tails, and the prefix
    // state at each one's candidate rank
    int64_t thr[kErrEps], ehn[kErrEps], ehs[kErrEps], elc[kErrEps], ec1[kErrEps];
    uint64_t ec2[kErrEps], ece[kErrEps];
#pragma unroll
    for (int e = 0; e < kErrEps; e++) {
        thr[e] = -1;
        ehn[e] = ehs[e] = elc[e] = ec1[e] = 0;
        ec2[e] = ece[e] = 0;
        if (want_eps && e < E.count) {
            thr[e] = delta * E.den[e] / E.num[e];
            if (thr[e] + 1 < tlen) {
                ehn[e] = tc[thr[e] + 1];
                ehs[e] = ts[thr[e] + 1];
            }
        }
    }
    // prefix sums along the ranks; candidates at each distinct distance
    using UAT = typename std::make_unsigned<AT>::type;
    AT c1 = 0;
    UAT c2 = 0, ce = 0;
    // the prefix state at the previous distinct distance, and the squared
    // pivot errors of the last ranks (the farthest samples) with their count
    UAT ce_last = 0;
    int64_t lc_last = 0, suf_cnt = 1;
    uint64_t suf_sq = 0;
    double berr = __builtin_inf(), best_est = 0.0;
    bool eo = false;
    for (int32_t j0 = 0; j0 < k; j0 += kRun) {
        load_run(j0);
        const int64_t after =
            j0 + kRun < k ? (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)dr[j0 + kRun]) : INT64_MAX;
#pragma unroll
        for (int t = 0; t < kRun; t++) {
            const int32_t j = j0 + t;
            if (j >= k) break;  // uniform
            const int64_t dl = rl[t];
            const int64_t nx = j + 1 < k ? (t + 1 < kRun ? rl[t + 1] : after) : INT64_MAX;
            const uint32_t d = rd[t];
            const AT df = (AT)d - (AT)dl;
            c1 += (AT)d;
            c2 += (UAT)d * (UAT)d;
            ce += (UAT)(df * df);
            if (nx == dl) continue;  // not the last rank at this distance (uniform)
            const int64_t lc = j + 1;
            if (lc == k) {  // the farthest distance: its ranks are the suffix
                suf_sq = (uint64_t)(UAT)(ce - ce_last);
                suf_cnt = lc - lc_last;
            }
            if (want_sw) {
                int64_t hn = 0, hs = 0;
                if (dl + 1 < tlen) {
                    hn = tc[dl + 1];
                    hs = ts[dl + 1];
                }
                if (dl < delta) {  // v itself is beyond T
                    hn -= 1;
                    hs -= delta;
                }
                double est, err;
                const bool hc = lc < k;
                prefix_candidate(n, k, lc, (int64_t)c1, (uint64_t)c2, sum - (int64_t)c1,
                                 hc ? sq_all - (uint64_t)ce : suf_sq, hc ? k - lc : suf_cnt, hn, hs, est, err, eo);
                if (err < berr) {
                    berr = err;
                    best_est = est;
                }
            }
            if (want_eps) {
#pragma unroll
                for (int e = 0; e < kErrEps; e++) {
                    if (dl <= thr[e] && thr[e] < nx) {
                        elc[e] = lc;
                        ec1[e] = (int64_t)c1;
                        ec2[e] = (uint64_t)c2;
                        ece[e] = (uint64_t)ce;
                    }
                }
            }
            ce_last = ce;
            lc_last = lc;
        }
    }
    if (!active) return;
    const int64_t o = orig[v];
    if (want_eps) {
        double err0 = 0.0, ad = 0.0, ad_err = 0.0;
#pragma unroll
        for (int e = 0; e < kErrEps; e++) {
            if (e < E.count) {
                double est, err;
                const bool hc = elc[e] < k;
                prefix_candidate(n, k, elc[e], ec1[e], ec2[e], sum - ec1[e], hc ? sq_all - ece[e] : suf_sq,
                                 hc ? k - elc[e] : suf_cnt, ehn[e], ehs[e], est, err, eo);
                if (e == 0) {
                    err0 = err;
                } else if (e == 1 || err < ad_err) {
                    ad = est;
                    ad_err = err;
                }
            }
        }
        if (S_err) S_err[o] = err0;
        if (S_ad) S_ad[o] = ad;
        if (S_ad_err) S_ad_err[o] = ad_err;
    }
    if (want_sw) {
        const double pure = ((double)(int64_t)sq_all / (double)k) * (double)(n - 1 - k);
        const bool thr_wins = berr < pure;
        if (S_sweep) S_sweep[o] = thr_wins ? best_est : (double)src_sum[p];
        if (S_sweep_err) S_sweep_err[o] = thr_wins ? berr : pure;
        eo = eo || src_sum[p] >= ((int64_t)1 << 53);
    }
    if (eo) flags->overflow = 1;
}

template <typename DT, bool RT>
__global__ void k_to_i32(const DT* __restrict__ D, const DT* __restrict__ Dr, const int32_t* __restrict__ orig,
                         int64_t n, int32_t k, int32_t* __restrict__ out) {
    const int64_t count = n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / k, i = t % k;
        out[(int64_t)orig[v] * k + i] = (int32_t)dist_at<DT, RT>(D, Dr, t);
    }
}

__global__ void k_sidx(const int32_t* __restrict__ samples, int32_t k, int32_t* __restrict__ sidx) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k && samples[i] >= 0) sidx[samples[i]] = i;  // negative: a bit position no sample uses
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        p[t] = value;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline unsigned grid_for(int64_t items, int64_t cap) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// lanes per node of the row-cooperative kernels (16 bytes each), or 0 when the
// row is not 16 * G bytes for G in {1, 2, 4, 8, 16}
template <typename DT>
int row_lanes(int32_t k) {
    const int64_t bytes = (int64_t)k * (int64_t)sizeof(DT);
    if (bytes % 16 != 0) return 0;
    const int64_t g = bytes / 16;
    return (g == 1 || g == 2 || g == 4 || g == 8 || g == 16) ? (int)g : 0;
}

template <typename DT, bool RT, typename MT>
void epilogue_t(hipStream_t st, const EpilogueArgs& a, void* scratch, DevFlags* flags) {
    const int64_t n = a.n;
    const int32_t k = a.k;
    const int64_t maxd = a.maxd;
    const int64_t tlen = maxd + 2;
    char* p = (char*)scratch;
    int32_t* Tcnt = (int32_t*)p;
    p += align256(sizeof(int32_t) * k * tlen);
    int64_t* Tsum = (int64_t*)p;
    p += align256(sizeof(int64_t) * k * tlen);
    MT* dmat_c = (MT*)p;
    p += align256(sizeof(MT) * (size_t)k * k);
    int64_t* chunks = (int64_t*)p;
    p += align256(suffix_chunk_scratch(k, maxd));
    int32_t* hist = a.hist;
    int32_t nslots = a.hist_slots;
    int64_t hlen = a.hist_len;
    if (!a.hist_done) {
        // histogram by a pass over D
        hist = (int32_t*)p;
        hlen = maxd + 1;
        nslots = 1;
        fill_u32(st, hist, 0u, (size_t)(k * hlen));
        const int G = row_lanes<DT>(k);
        // LDS copy of the histogram: [k][hlen] for k_reduce, [k][hist_stride(hlen)] for the row variant
        const size_t lds = sizeof(int32_t) * (size_t)k * (size_t)(G > 0 ? hist_stride(hlen) : hlen);
        const int use_lds = lds <= 48 * 1024 ? 1 : 0;
        const unsigned rb = grid_for(n, use_lds ? 1024 : 8192);
        const size_t lb = use_lds ? lds : 0;
        const DT* Dp = (const DT*)a.D;
        const DT* Drp = (const DT*)a.Dr;
        switch (G) {
            case 1:
                if (use_lds) hipLaunchKernelGGL((k_reduce_rows<DT, RT, 1, true>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                else hipLaunchKernelGGL((k_reduce_rows<DT, RT, 1, false>), dim3(rb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                break;
            case 2:
                if (use_lds) hipLaunchKernelGGL((k_reduce_rows<DT, RT, 2, true>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                else hipLaunchKernelGGL((k_reduce_rows<DT, RT, 2, false>), dim3(rb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                break;
            case 4:
                if (use_lds) hipLaunchKernelGGL((k_reduce_rows<DT, RT, 4, true>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                else hipLaunchKernelGGL((k_reduce_rows<DT, RT, 4, false>), dim3(rb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                break;
            case 8:
                if (use_lds) hipLaunchKernelGGL((k_reduce_rows<DT, RT, 8, true>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                else hipLaunchKernelGGL((k_reduce_rows<DT, RT, 8, false>), dim3(rb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                break;
            case 16:
                if (use_lds) hipLaunchKernelGGL((k_reduce_rows<DT, RT, 16, true>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                else hipLaunchKernelGGL((k_reduce_rows<DT, RT, 16, false>), dim3(rb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx, hlen, hist, flags);
                break;
            default:
                hipLaunchKernelGGL((k_reduce<DT, RT>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist,
                                   use_lds, flags);
        }
        CCG_HIP(hipGetLastError());
    }
    const int64_t kk = (int64_t)k * k;
    hipLaunchKernelGGL((k_dmat<DT, RT, MT>), dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, st, (const DT*)a.D,
                       (const DT*)a.Dr, a.samples, k, a.dmat, dmat_c, flags);
    run_suffix(st, hist, nslots, k, k, hlen, maxd, a.dmat, Tcnt, Tsum, a.src_sum, chunks);
    {
        const DT* Dp = (const DT*)a.D;
        const DT* Drp = (const DT*)a.Dr;
        const int G = row_lanes<DT>(k);
        // the row kernel: 64 positions per wave and round; small tables in
        // LDS when they fit (blocks of 512 threads, two per CU: a block copies
        // the tables once, so the grid stays at a few blocks per CU)
        const int64_t rounds = (n + 63) / 64;
        const size_t tb = est_table_bytes(k, tlen, sizeof(MT));
        const bool lt = tb <= kEstTableLds;
        const unsigned ebl = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(kEstTableBlocks, (rounds + kEstBlock / 64 - 1) / (kEstBlock / 64)));
        const unsigned eb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (rounds + kBlock / 64 - 1) / (kBlock / 64)));
#define CCG_EST_ROWS(GG, PP)                                                                                           \
    do {                                                                                                               \
        if (lt)                                                                                                        \
            hipLaunchKernelGGL((k_estimate_rows<DT, RT, MT, GG, PP, true, kEstBlock>), dim3(ebl), dim3(kEstBlock), tb, \
                               st, Dp, Drp, n, k, a.orig, a.inv, dmat_c, Tcnt, Tsum, tlen, a.src_sum, a.eps_num,       \
                               a.eps_den, a.S_hyb, a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, flags);    \
        else                                                                                                           \
            hipLaunchKernelGGL((k_estimate_rows<DT, RT, MT, GG, PP, false, kBlock>), dim3(eb), dim3(kBlock), 0, st,    \
                               Dp, Drp, n, k, a.orig, a.inv, dmat_c, Tcnt, Tsum, tlen, a.src_sum, a.eps_num,           \
                               a.eps_den, a.S_hyb, a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, flags);    \
    } while (0)
        // byte-packed rows take 32 bytes per lane from 64-byte rows up, 64 bytes from 128-byte rows up
        constexpr bool kPk = sizeof(DT) == 1 && !RT && sizeof(MT) == 1;
        switch (G) {
            case 2: CCG_EST_ROWS(2, 1); break;
            case 4:
                if constexpr (kPk) CCG_EST_ROWS(2, 2);
                else CCG_EST_ROWS(4, 1);
                break;
            case 8:
                if constexpr (kPk) CCG_EST_ROWS(2, 4);
                else CCG_EST_ROWS(8, 1);
                break;
            case 16:
                if constexpr (kPk) CCG_EST_ROWS(4, 4);
                else CCG_EST_ROWS(16, 1);
                break;
            default:
                hipLaunchKernelGGL((k_estimate<DT, RT, MT>), dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, Dp, Drp, n, k,
                                   a.sidx, a.orig, dmat_c, Tcnt, Tsum, tlen, a.src_sum, a.eps_num, a.eps_den, a.S_hyb,
                                   a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, flags);
        }
#undef CCG_EST_ROWS
        CCG_HIP(hipGetLastError());
    }
    CCG_HIP(hipGetLastError());
    if (a.Dout) {
        hipLaunchKernelGGL((k_to_i32<DT, RT>), dim3(grid_for(n * k, 65536)), dim3(256), 0, st, (const DT*)a.D,
                           (const DT*)a.Dr, a.orig, n, k, a.Dout);
    }
    if (a.S_err || a.S_ad || a.S_ad_err || a.S_sweep || a.S_sweep_err) {
        ErrArgs ea;
        ea.D = a.D;
        ea.Dr = a.Dr;
        ea.dk = a.dk;
        ea.n = n;
        ea.k = k;
        ea.sidx = a.sidx;
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
        // after the tables above and the histogram this pass may have counted
        ea.sweep_scratch = p + (a.hist_done ? 0 : align256(sizeof(int32_t) * k * (maxd + 1)));
        run_errest(st, ea, flags);
    }
}

template <typename DT, bool RT>
void epilogue_mt(hipStream_t st, const EpilogueArgs& a, void* scratch, DevFlags* flags) {
    if (a.maxd < 255) epilogue_t<DT, RT, uint8_t>(st, a, scratch, flags);
    else if (a.maxd < 65535) epilogue_t<DT, RT, uint16_t>(st, a, scratch, flags);
    else epilogue_t<DT, RT, uint32_t>(st, a, scratch, flags);
}

}  // namespace

namespace {

// LDS bytes per lane for a staged row (and reverse row): a multiple of 4
// with an odd number of words, so that lanes reading the same offset of their
// rows hit different banks
inline int32_t stage_stride(int32_t k, int dt_bytes, bool rt) {
    int32_t b = k * dt_bytes * (rt ? 2 : 1);
    b = (b + 3) & ~3;
    if ((b / 4) % 2 == 0) b += 4;
    return b;
}

template <typename DT, bool RT, typename MT>
void errest_t(hipStream_t st, const ErrArgs& a, DevFlags* flags) {
    ErrEps E{};
    E.count = 1;
    E.num[0] = a.eps_num;
    E.den[0] = a.eps_den;
    for (int32_t e = 0; e < kAdaptiveEps && E.count < kErrEps; e++) {
        E.num[E.count] = kAdaptiveEpsNum[e];
        E.den[E.count] = kAdaptiveEpsDen[e];
        E.count++;
    }
    if (!a.sweep_scratch) throw HipError{hipErrorInvalidValue, "error-estimate scratch"};
    const int32_t k = a.k;
    const int64_t n = a.n;
    char* q = (char*)a.sweep_scratch;
    const int32_t kp = (k + 7) & ~7;
    uint32_t* perm = (uint32_t*)q;
    q += align256(sizeof(uint32_t) * (size_t)k * kp);
    uint32_t* ds = (uint32_t*)q;
    q += align256(sizeof(uint32_t) * (size_t)k * kp);
    int32_t* piv = (int32_t*)q;
    q += align256(sizeof(int32_t) * (size_t)n);
    int64_t* vsum = (int64_t*)q;
    q += align256(sizeof(int64_t) * (size_t)n);
    uint64_t* vsq = (uint64_t*)q;
    q += align256(sizeof(uint64_t) * (size_t)n);
    int32_t* bcnt = (int32_t*)q;  // per block of the bucketing kernels: its count per pivot
    q += align256(sizeof(int32_t) * (size_t)kErrBucketBlocks * k);
    int32_t* order = (int32_t*)q;
    q += align256(sizeof(int32_t) * (size_t)n);
    int32_t* cnt = (int32_t*)q;  // cnt, fill: k each; start, tstart: k + 1 each
    int32_t* fill = cnt + k;
    int32_t* start = fill + k;
    int32_t* tstart = start + (k + 1);
    int32_t k2 = 1;
    while (k2 < k) k2 <<= 1;
    hipLaunchKernelGGL((k_sort_rows<MT>), dim3((unsigned)k), dim3(kBlock), sizeof(uint64_t) * (size_t)k2, st,
                       (const MT*)a.dmat_c, k, k2, kp, perm, ds);
    fill_u32(st, cnt, 0u, (size_t)2 * k);
    const unsigned bb = grid_for(n, kErrBucketBlocks);
    hipLaunchKernelGGL((k_err_pivot<DT, RT, MT>), dim3(bb), dim3(kBlock), sizeof(int32_t) * (size_t)k, st,
                       (const DT*)a.D, (const DT*)a.Dr, n, k, a.sidx, a.bit_base, a.orig, (const MT*)a.dmat_c,
                       a.src_sum, piv, vsum, vsq, cnt, bcnt, a.S_err, a.S_ad, a.S_ad_err, a.S_sweep, a.S_sweep_err,
                       flags);
    hipLaunchKernelGGL(k_err_buckets, dim3(1), dim3(kBlock), 0, st, (const int32_t*)cnt, k, start, tstart);
    hipLaunchKernelGGL(k_err_fill, dim3(bb), dim3(kBlock), sizeof(int32_t) * (size_t)k, st, (const int32_t*)piv, n, k,
                       (const int32_t*)start, (const int32_t*)bcnt, fill, order);
    // tasks: at most one partial wavefront per pivot beyond n / 64 full ones
    const unsigned tasks = (unsigned)((n + 63) / 64 + k);
    const int32_t stride = stage_stride(k, (int)sizeof(DT), RT);
    const size_t lds = (size_t)64 * stride;
    using AT = typename std::conditional<sizeof(DT) == 1, int32_t, int64_t>::type;  // d < 2^9: squares fit 32 bits
#define CCG_ERRSWEEP(STG, LDSB)                                                                                        \
    hipLaunchKernelGGL((k_errsweep<DT, RT, STG, AT>), dim3(tasks), dim3(64), LDSB, st, (const DT*)a.D, (const DT*)a.Dr, \
                       n, k, kp, a.orig, (const uint32_t*)perm, (const uint32_t*)ds, (const int64_t*)vsum,             \
                       (const uint64_t*)vsq, (const int32_t*)cnt,                                                     \
                       (const int32_t*)start, (const int32_t*)tstart, (const int32_t*)order, stride, a.Tcnt, a.Tsum,  \
                       a.tlen, a.src_sum, E, a.S_err, a.S_ad, a.S_ad_err, a.S_sweep, a.S_sweep_err, flags)
    if (lds <= 32 * 1024) CCG_ERRSWEEP(true, lds);
    else CCG_ERRSWEEP(false, 0);
#undef CCG_ERRSWEEP
}

template <typename DT, bool RT>
void errest_m(hipStream_t st, const ErrArgs& a, DevFlags* flags) {
    switch (a.mt_bytes) {
        case 1: errest_t<DT, RT, uint8_t>(st, a, flags); break;
        case 2: errest_t<DT, RT, uint16_t>(st, a, flags); break;
        default: errest_t<DT, RT, uint32_t>(st, a, flags); break;
    }
}

template <typename DT>
void errest_r(hipStream_t st, const ErrArgs& a, DevFlags* flags) {
    if (a.Dr) errest_m<DT, true>(st, a, flags);
    else errest_m<DT, false>(st, a, flags);
}

}  // namespace

size_t sweep_scratch_bytes(int64_t n, int32_t k) {
    const size_t kp = ((size_t)k + 7) & ~(size_t)7;
    return 2 * align256(sizeof(uint32_t) * (size_t)k * kp) + 2 * align256(sizeof(int32_t) * (size_t)n) +
           2 * align256(sizeof(int64_t) * (size_t)n) + align256(sizeof(int32_t) * (size_t)kErrBucketBlocks * k) +
           align256(sizeof(int32_t) * (4 * (size_t)k + 2));
}

void run_errest(hipStream_t st, const ErrArgs& a, DevFlags* flags) {
    if (!a.S_err && !a.S_ad && !a.S_ad_err && !a.S_sweep && !a.S_sweep_err) return;
    switch (a.dk) {
        case DistKind::U8: errest_r<uint8_t>(st, a, flags); break;
        case DistKind::U16: errest_r<uint16_t>(st, a, flags); break;
        default: errest_r<uint32_t>(st, a, flags); break;
    }
    CCG_HIP(hipGetLastError());
}

void fill_u32(hipStream_t st, void* p, uint32_t value, size_t count) {
    if (count == 0) return;
    size_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, (uint32_t*)p, value, count);
}

void compute_sidx(hipStream_t st, const int32_t* samples, int32_t k, int32_t* sidx, int64_t n) {
    fill_u32(st, sidx, 0xFFFFFFFFu, (size_t)n);
    hipLaunchKernelGGL(k_sidx, dim3((k + 255) / 256), dim3(256), 0, st, samples, k, sidx);
}

void run_suffix(hipStream_t st, const int32_t* hist, int32_t nslots, int32_t k, int32_t hist_rows, int64_t hlen,
                int64_t maxd,
                const int32_t* dmat, int32_t* Tcnt, int64_t* Tsum, int64_t* src_sum, int64_t* chunk_scratch) {
    const int64_t nchunks = (maxd + 1 + kChunk - 1) / kChunk;
    if (nchunks <= 1 || chunk_scratch == nullptr) {
        hipLaunchKernelGGL(k_suffix, dim3(k), dim3(kBlock), 0, st, hist, nslots, k, hist_rows, hlen, maxd, dmat, Tcnt,
                           Tsum,
                           src_sum);
    } else {
        int64_t* cc = chunk_scratch;
        int64_t* cs = chunk_scratch + (int64_t)k * nchunks;
        hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)nchunks, k), dim3(kBlock), 0, st, hist, nslots, k, hist_rows,
                           hlen, cc, cs,
                           nchunks);
        hipLaunchKernelGGL(k_chunk_carry, dim3((k + 63) / 64), dim3(64), 0, st, cc, cs, k, nchunks);
        hipLaunchKernelGGL(k_chunk_suffix, dim3((unsigned)nchunks, k), dim3(kBlock), 0, st, hist, nslots, k, hist_rows,
                           hlen, maxd,
                           cc, cs, nchunks, Tcnt, Tsum);
        hipLaunchKernelGGL(k_src_sum, dim3(k), dim3(64), 0, st, Tsum, maxd + 2, dmat, k, src_sum);
    }
    CCG_HIP(hipGetLastError());
}

size_t suffix_chunk_scratch(int32_t k, int64_t maxd) {
    const int64_t nchunks = (maxd + 1 + kChunk - 1) / kChunk;
    return sizeof(int64_t) * 2 * (size_t)k * (size_t)nchunks + 256;
}

size_t epilogue_scratch(int64_t n, int32_t k, int64_t maxd, bool hist_done, bool err) {
    const int64_t tlen = maxd + 2;
    size_t s = align256(sizeof(int32_t) * k * tlen) + align256(sizeof(int64_t) * k * tlen) +
               align256(sizeof(uint32_t) * (size_t)k * k) + align256(suffix_chunk_scratch(k, maxd)) + 1024;
    if (!hist_done) s += align256(sizeof(int32_t) * k * (maxd + 1));
    if (err) s += align256(sweep_scratch_bytes(n, k));
    return s;
}

void run_epilogue(hipStream_t st, const EpilogueArgs& a, void* scratch, size_t scratch_size, DevFlags* flags) {
    const bool want_err = a.S_err || a.S_ad || a.S_ad_err || a.S_sweep || a.S_sweep_err;
    if (scratch_size < epilogue_scratch(a.n, a.k, a.maxd, a.hist_done, want_err))
        throw HipError{hipErrorOutOfMemory, "epilogue scratch"};
    const bool rt = a.Dr != nullptr;
    switch (a.dk) {
        case DistKind::U8:
            rt ? epilogue_mt<uint8_t, true>(st, a, scratch, flags) : epilogue_mt<uint8_t, false>(st, a, scratch, flags);
            break;
        case DistKind::U16:
            rt ? epilogue_mt<uint16_t, true>(st, a, scratch, flags) : epilogue_mt<uint16_t, false>(st, a, scratch, flags);
            break;
        default:
            rt ? epilogue_mt<uint32_t, true>(st, a, scratch, flags) : epilogue_mt<uint32_t, false>(st, a, scratch, flags);
            break;
    }
}

}  // namespace ccg
