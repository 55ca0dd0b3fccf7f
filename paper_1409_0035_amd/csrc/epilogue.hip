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
    __device__ __forceinline__ void load(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t v, int32_t k,
                                         int sub) {
        const uint4 a = ((const uint4*)(D + v * k))[sub];
        uint4 b = make_uint4(0, 0, 0, 0);
        if (RT) b = ((const uint4*)(Dr + v * k))[sub];
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

template <int G>
__device__ __forceinline__ int64_t group_sum64(int64_t x) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// histogram over non-sampled nodes (as k_reduce)
template <typename DT, bool RT, int G>
__global__ __launch_bounds__(kBlock) void k_reduce_rows(const DT* __restrict__ D, const DT* __restrict__ Dr,
                                                        int64_t n, int32_t k, const int32_t* __restrict__ sidx,
                                                        int64_t hlen, int32_t* __restrict__ hist, int use_lds,
                                                        DevFlags* flags) {
    extern __shared__ int32_t lds_hist[];  // [k][hlen] when use_lds
    if (use_lds) {
        for (int64_t t = threadIdx.x; t < (int64_t)k * hlen; t += kBlock) lds_hist[t] = 0;
        __syncthreads();
    }
    constexpr int PER = RowPiece<DT, RT>::PER;
    const int sub = lane_id() & (G - 1);
    const int64_t per_block = kBlock / G;
    bool bad = false;
    for (int64_t v0 = (int64_t)blockIdx.x * per_block; v0 < n; v0 += (int64_t)gridDim.x * per_block) {
        const int64_t v = v0 + threadIdx.x / G;
        if (v >= n || sidx[v] >= 0) continue;
        RowPiece<DT, RT> r;
        r.load(D, Dr, v, k, sub);
#pragma unroll
        for (int e = 0; e < PER; e++) {
            const int64_t i = (int64_t)sub * PER + e;
            const uint32_t d = r.d[e];
            if ((int64_t)d >= hlen || r.unreached) {
                bad = true;
            } else if (use_lds) {
                atomicAdd(&lds_hist[i * hlen + d], 1);
            } else {
                atomicAdd(&hist[i * hlen + d], 1);
            }
        }
    }
    if (bad) flags->disconnected = 1;
    if (use_lds) {
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)k * hlen; t += kBlock) {
            const int32_t c = lds_hist[t];
            if (c) atomicAdd(&hist[t], c);
        }
    }
}

// the estimators (as k_estimate)
template <typename DT, bool RT, typename MT, int G>
__global__ __launch_bounds__(kBlock) void k_estimate_rows(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ sidx,
    const int32_t* __restrict__ orig, const MT* __restrict__ dmat_c, const int32_t* __restrict__ Tcnt,
    const int64_t* __restrict__ Tsum, int64_t tlen, const int64_t* __restrict__ src_sum, int64_t en, int64_t ed,
    double* S_hyb, double* S_samp, int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out, int32_t* delta_out,
    int64_t* sampsum_out, DevFlags* flags) {
    constexpr int PER = RowPiece<DT, RT>::PER;
    const int64_t LIM = (int64_t)1 << 53;
    const int sub = lane_id() & (G - 1);
    const int64_t per_block = kBlock / G;
    bool any_ovf = false, any_unreached = false;
    // every lane runs the same number of iterations (the group shuffles need
    // all lanes); nodes past the end are masked, not skipped
    const int64_t steps = (n + per_block - 1) / per_block;
    for (int64_t s0 = blockIdx.x; s0 < steps; s0 += gridDim.x) {
        const int64_t v = s0 * per_block + threadIdx.x / G;
        const bool valid = v < n;
        RowPiece<DT, RT> r;
        if (valid) {
            r.load(D, Dr, v, k, sub);
        } else {
#pragma unroll
            for (int e = 0; e < PER; e++) r.d[e] = 0xFFFFFFFFu;
        }
        // argmin (lowest index among equal minima) and sum
        uint32_t best = 0xFFFFFFFFu;
        int32_t bi = 0;
        int64_t sum = 0;
#pragma unroll
        for (int e = 0; e < PER; e++) {
            if (r.d[e] < best) {
                best = r.d[e];
                bi = sub * PER + e;
            }
            sum += valid ? r.d[e] : 0;
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const uint32_t ob = (uint32_t)__shfl_xor((int)best, off);
            const int32_t oi = __shfl_xor(bi, off);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        sum = group_sum64<G>(sum);
        const int p = bi;
        const int64_t delta = best;
        const int32_t j = valid ? sidx[v] : 0;
        // the L cap C split against the pivot's row of the sample distances
        const int64_t thr = delta * ed;
        const MT* drow = dmat_c + (int64_t)p * k;
        int64_t lcsum = 0, lcnum = 0;
        if (valid && j < 0) {
#pragma unroll
            for (int e = 0; e < PER; e++) {
                if ((int64_t)drow[sub * PER + e] * en <= thr) {
                    lcsum += r.d[e];
                    lcnum += 1;
                }
            }
        }
        lcsum = group_sum64<G>(lcsum);
        lcnum = group_sum64<G>(lcnum);
        bool unreached = r.unreached;
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) unreached = unreached || __shfl_xor((int)unreached, off);
        if (!valid || sub != 0) continue;
        double hyb, samp;
        int64_t piv, pub;
        bool ovf = false;
        if (j >= 0) {
            const int64_t S = src_sum[j];
            hyb = samp = (double)S;
            piv = pub = S;
            ovf = S >= LIM;
        } else {
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
            ovf = __builtin_mul_overflow(a, lcnum, &t1) || __builtin_mul_overflow(lcsum, lnum, &t2) ||
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
    for (int64_t top = maxd; top >= 0; top -= kBlock) {
        const int64_t d = top - threadIdx.x;
        int64_t c = 0;
        if (d >= 0 && d < hlen)
            for (int32_t s = 0; s < nslots; s++) c += hist[((int64_t)s * hrows + i) * hlen + d];
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

// Sec. 4: the estimated squared error of the hybrid estimate for the call's
// eps, and the adaptive estimate -- for each eps of a fixed list, the hybrid
// estimate and its estimated error, the first smallest error kept.  One lane
// per node, one pass over its distance row for all eps at once.  For one eps,
// with L cap C = {i : dmat[p][i] * num <= Delta * den} and HC the other
// samples:
//   err = ((LCnum * LCsumsq - LCsum^2) / LCnum^3) * Lnum + (HCsqerr / HCnum) * Hnum
// (second term 0 without HC), HCsqerr = sum over HC of (d(v,c_i) - d(c_p,c_i))^2,
// in exactly this order of double operations on exact integers.
constexpr int kErrEps = 8;  // the call's eps + up to 7 listed ones
struct ErrEps {
    int32_t count;  // entries used; entry 0 is the call's eps
    int64_t num[kErrEps], den[kErrEps];
};

template <typename DT, bool RT, typename MT>
__global__ __launch_bounds__(kBlock) void k_errest(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ sidx,
    int32_t bit_base, const int32_t* __restrict__ orig, const MT* __restrict__ dmat_c, const int32_t* __restrict__ Tcnt,
    const int64_t* __restrict__ Tsum, int64_t tlen, const int64_t* __restrict__ src_sum, ErrEps E, double* S_err,
    double* S_ad, double* S_ad_err, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    bool any_ovf = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int64_t o = orig[v];
        const int32_t js = sidx[v];
        if (js >= 0) {  // a sample: its exact sum, no error
            if (S_err) S_err[o] = 0.0;
            if (S_ad) S_ad[o] = (double)src_sum[js - bit_base];
            if (S_ad_err) S_ad_err[o] = 0.0;
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
        const int64_t delta = best;
        const MT* drow = dmat_c + (int64_t)p * k;
        int32_t lcnum[kErrEps];
        int64_t lcsum[kErrEps];
        uint64_t lcsq[kErrEps], hcsq[kErrEps];
#pragma unroll
        for (int e = 0; e < kErrEps; e++) {
            lcnum[e] = 0;
            lcsum[e] = 0;
            lcsq[e] = 0;
            hcsq[e] = 0;
        }
        bool big = false;
        for_row<DT, RT>(D, Dr, v, k, [&](int32_t i, uint32_t d) {
            const int64_t dl = drow[i];
            const uint64_t dd = (uint64_t)d * d;
            const int64_t diff = (int64_t)d - dl;
            const uint64_t ee = (uint64_t)(diff * diff);
            big = big || d >= (1u << 25) || dl >= (1 << 25);  // squares summed over k <= 4096 stay below 2^62
#pragma unroll
            for (int e = 0; e < kErrEps; e++) {
                if (e >= E.count) break;
                if (dl * E.num[e] <= delta * E.den[e]) {
                    lcnum[e] += 1;
                    lcsum[e] += d;
                    lcsq[e] += dd;
                } else {
                    hcsq[e] += ee;
                }
            }
        });
        bool ovf = big;
        double ad = 0.0, ad_err = 0.0, err0 = 0.0;
#pragma unroll
        for (int e = 0; e < kErrEps; e++) {
            if (e >= E.count) break;
            const int64_t thr = delta * E.den[e];
            const int64_t tix = thr / E.num[e] + 1;  // d > floor(Delta/eps)  <=>  d >= tix
            int64_t hnum = 0, hsum = 0;
            if (tix < tlen) {
                hnum = Tcnt[(int64_t)p * tlen + tix];
                hsum = Tsum[(int64_t)p * tlen + tix];
            }
            const int64_t lc = lcnum[e];
            const int64_t hcnum = k - lc;
            const int64_t hcsum = sum - lcsum[e];
            const int64_t lnum = (n - 1) - hnum - hcnum;
            int64_t t1 = 0, t2 = 0, N = 0, vn1 = 0, vn2 = 0, varnum = 0;
            bool eo = __builtin_mul_overflow(hsum + hcsum, lc, &t1) || __builtin_mul_overflow(lcsum[e], lnum, &t2) ||
                      __builtin_add_overflow(t1, t2, &N) || N >= LIM || lc < 1 || lnum < lc;
            eo = eo || __builtin_mul_overflow(lc, (int64_t)lcsq[e], &vn1) ||
                 __builtin_mul_overflow(lcsum[e], lcsum[e], &vn2) || __builtin_sub_overflow(vn1, vn2, &varnum);
            ovf = ovf || eo;
            const double est = (double)N / (double)lc;
            const double tL = ((double)varnum / (double)(lc * lc * lc)) * (double)lnum;
            const double tH = hcnum > 0 ? ((double)(int64_t)hcsq[e] / (double)hcnum) * (double)hnum : 0.0;
            const double err = tL + tH;
            if (e == 0) {
                err0 = err;
            } else if (e == 1 || err < ad_err) {
                ad = est;
                ad_err = err;
            }
        }
        if (S_err) S_err[o] = err0;
        if (S_ad) S_ad[o] = ad;
        if (S_ad_err) S_ad_err[o] = ad_err;
        any_ovf = any_ovf || ovf;
    }
    if (any_ovf) flags->overflow = 1;
}

// Algorithm 2 / Sec. 4.2 (threshold sweep), step 1: each sample's row of the
// sample distance matrix in increasing order -- perm[p][j] is the sample of
// rank j by distance from c_p (index order among equal distances), ds[p][j]
// that distance.  One block per sample; bitonic sort of the keys
// (distance << 12 | index) in LDS, k2 = the power of two >= k (<= 4096).
template <typename MT>
__global__ __launch_bounds__(kBlock) void k_sort_rows(const MT* __restrict__ dmat_c, int32_t k, int32_t k2,
                                                      uint16_t* __restrict__ perm, MT* __restrict__ ds) {
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
    for (int32_t j = threadIdx.x; j < k; j += kBlock) {
        const uint64_t x = skey[j];
        perm[p * k + j] = (uint16_t)(x & 0xFFF);
        ds[p * k + j] = (MT)(x >> 12);
    }
}

// Step 2, one wavefront per node v outside C.  Candidates, compared in this
// order: pure pivoting, S(c_p) with error (sum_i (d(v,c_i) - d(c_p,c_i))^2 / k)
// * (n-1-k); then, for every distinct distance T from the pivot c_p to a
// sample, increasing, the estimate of the threshold T over V \ {v}:
//   L = {u : d(c_p,u) <= T}, HC = samples beyond T, H = other nodes beyond T,
//   N = (sum_H d(c_p,u) + sum_HC d(v,u)) * |L cap C| + |L| * sum_{L cap C} d(v,u),
//   estimate N / |L cap C|, error as in Sec. 4.1 with these sets.
// |H| and sum_H come from the tail tables at T + 1, less v itself when
// Delta > T (v lies beyond T from its pivot but is no term of its own sum);
// |L| = n-1-|H|-|HC|.  The smallest error wins, the first candidate on ties.
// Lane l walks the sorted ranks [l*P, l*P + P): a first pass sums its ranks,
// a wave scan gives each lane the sums of the ranks before it, a second pass
// evaluates the candidates at the last rank of each distinct distance; a wave
// reduction picks (error, rank).
template <typename DT, bool RT, typename MT>
__global__ __launch_bounds__(kBlock) void k_sweep(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ sidx,
    int32_t bit_base, const int32_t* __restrict__ orig, const uint16_t* __restrict__ perm, const MT* __restrict__ ds,
    const int32_t* __restrict__ Tcnt, const int64_t* __restrict__ Tsum, int64_t tlen, const int64_t* __restrict__ src_sum,
    double* S_sweep, double* S_sweep_err, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    const int32_t P = (k + 63) / 64;
    const int32_t j0 = lane * P < k ? lane * P : k;
    const int32_t j1 = j0 + P < k ? j0 + P : k;
    bool ovf = false;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < n; v += nwaves) {
        const int64_t o = orig[v];
        const int32_t js = sidx[v];
        if (js >= 0) {  // a sample: its exact sum, no error
            if (lane == 0) {
                if (S_sweep) S_sweep[o] = (double)src_sum[js - bit_base];
                if (S_sweep_err) S_sweep_err[o] = 0.0;
            }
            continue;
        }
        const int64_t row = v * k;
        // pivot (lowest index among the nearest samples), Delta, row sum
        uint32_t best = 0xFFFFFFFFu;
        int32_t bi = k;
        int64_t sum = 0;
        for (int32_t i = lane; i < k; i += 64) {
            const uint32_t d = dist_at<DT, RT>(D, Dr, row + i);
            if (d < best) {
                best = d;
                bi = i;
            }
            sum += d;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t ob = __shfl_xor(best, off);
            const int32_t oi = __shfl_xor(bi, off);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        sum = wave_sum64(sum);
        const int32_t p = bi;
        const int64_t delta = best;
        const uint16_t* pr = perm + (int64_t)p * k;
        const MT* dr = ds + (int64_t)p * k;
        // pass 1: this lane's sums over its ranks
        int64_t a1 = 0;
        uint64_t a2 = 0, ae = 0;
        bool big = false;
        for (int32_t j = j0; j < j1; j++) {
            const uint32_t d = dist_at<DT, RT>(D, Dr, row + pr[j]);
            const int64_t dl = dr[j];
            big = big || d >= (1u << 25) || dl >= (1 << 25);  // squares summed over k <= 4096 stay below 2^62
            const int64_t df = (int64_t)d - dl;
            a1 += d;
            a2 += (uint64_t)d * d;
            ae += (uint64_t)(df * df);
        }
        int64_t s1 = a1;
        uint64_t s2 = a2, se = ae;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y1 = __shfl_up(s1, off);
            const uint64_t y2 = __shfl_up(s2, off), ye = __shfl_up(se, off);
            if (lane >= off) {
                s1 += y1;
                s2 += y2;
                se += ye;
            }
        }
        const uint64_t sq_all = __shfl(se, 63);
        int64_t c1 = s1 - a1;  // sums over the ranks before this lane's
        uint64_t c2 = s2 - a2, ce = se - ae;
        // pass 2: the candidates whose threshold is a distance of this lane's ranks
        double lerr = __builtin_inf(), lest = 0.0;
        int32_t lpos = k;
        bool eo = false;
        for (int32_t j = j0; j < j1; j++) {
            const uint32_t d = dist_at<DT, RT>(D, Dr, row + pr[j]);
            const int64_t dl = dr[j];
            const int64_t df = (int64_t)d - dl;
            c1 += d;
            c2 += (uint64_t)d * d;
            ce += (uint64_t)(df * df);
            if (j + 1 < k && (int64_t)dr[j + 1] == dl) continue;  // not the last rank at this distance
            const int64_t lc = j + 1;
            const int64_t hcnum = k - lc;
            const int64_t hcsum = sum - c1;
            const uint64_t hcsq = sq_all - ce;
            int64_t hnum = 0, hsum = 0;
            if (dl + 1 < tlen) {
                hnum = Tcnt[(int64_t)p * tlen + dl + 1];
                hsum = Tsum[(int64_t)p * tlen + dl + 1];
            }
            if (dl < delta) {  // v itself is beyond T
                hnum -= 1;
                hsum -= delta;
            }
            const int64_t lnum = (n - 1) - hnum - hcnum;
            int64_t t1 = 0, t2 = 0, N = 0, vn1 = 0, vn2 = 0, varnum = 0;
            bool e = __builtin_mul_overflow(hsum + hcsum, lc, &t1) || __builtin_mul_overflow(c1, lnum, &t2) ||
                     __builtin_add_overflow(t1, t2, &N) || N >= LIM || lnum < lc || hnum < 0;
            e = e || __builtin_mul_overflow(lc, (int64_t)c2, &vn1) || __builtin_mul_overflow(c1, c1, &vn2) ||
                __builtin_sub_overflow(vn1, vn2, &varnum);
            eo = eo || e;
            const double est = (double)N / (double)lc;
            const double tL = ((double)varnum / (double)(lc * lc * lc)) * (double)lnum;
            const double tH = hcnum > 0 ? ((double)(int64_t)hcsq / (double)hcnum) * (double)hnum : 0.0;
            const double err = tL + tH;
            if (err < lerr) {
                lerr = err;
                lest = est;
                lpos = j;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double oe = __shfl_xor(lerr, off), os = __shfl_xor(lest, off);
            const int32_t op = __shfl_xor(lpos, off);
            if (oe < lerr || (oe == lerr && op < lpos)) {
                lerr = oe;
                lest = os;
                lpos = op;
            }
        }
        const double pure = ((double)(int64_t)sq_all / (double)k) * (double)(n - 1 - k);
        if (lane == 0) {
            const bool thr = lerr < pure;
            if (S_sweep) S_sweep[o] = thr ? lest : (double)src_sum[p];
            if (S_sweep_err) S_sweep_err[o] = thr ? lerr : pure;
        }
        ovf = ovf || big || eo || src_sum[p] >= LIM;
    }
    if (ovf) flags->overflow = 1;
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
        const size_t lds = sizeof(int32_t) * (size_t)k * hlen;
        const int use_lds = lds <= 48 * 1024 ? 1 : 0;
        const int G = row_lanes<DT>(k);
        const unsigned rb = grid_for(n, use_lds ? 1024 : 8192);
        const size_t lb = use_lds ? lds : 0;
        const DT* Dp = (const DT*)a.D;
        const DT* Drp = (const DT*)a.Dr;
        switch (G) {
            case 1: hipLaunchKernelGGL((k_reduce_rows<DT, RT, 1>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, use_lds, flags); break;
            case 2: hipLaunchKernelGGL((k_reduce_rows<DT, RT, 2>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, use_lds, flags); break;
            case 4: hipLaunchKernelGGL((k_reduce_rows<DT, RT, 4>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, use_lds, flags); break;
            case 8: hipLaunchKernelGGL((k_reduce_rows<DT, RT, 8>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, use_lds, flags); break;
            case 16: hipLaunchKernelGGL((k_reduce_rows<DT, RT, 16>), dim3(rb), dim3(kBlock), lb, st, Dp, Drp, n, k, a.sidx, hlen, hist, use_lds, flags); break;
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
        const unsigned eb = grid_for(n * (G > 0 ? G : 1), 8192);
#define CCG_EST_ROWS(GG)                                                                                            \
    hipLaunchKernelGGL((k_estimate_rows<DT, RT, MT, GG>), dim3(eb), dim3(kBlock), 0, st, Dp, Drp, n, k, a.sidx,       \
                       a.orig, dmat_c, Tcnt, Tsum, tlen, a.src_sum, a.eps_num, a.eps_den, a.S_hyb, a.S_samp, a.S_piv, \
                       a.S_pub, a.pivot, a.delta, a.sampsum, flags)
        switch (G) {
            case 1: CCG_EST_ROWS(1); break;
            case 2: CCG_EST_ROWS(2); break;
            case 4: CCG_EST_ROWS(4); break;
            case 8: CCG_EST_ROWS(8); break;
            case 16: CCG_EST_ROWS(16); break;
            default:
                hipLaunchKernelGGL((k_estimate<DT, RT, MT>), dim3(grid_for(n, 4096)), dim3(kBlock), 0, st, Dp, Drp, n, k,
                                   a.sidx, a.orig, dmat_c, Tcnt, Tsum, tlen, a.src_sum, a.eps_num, a.eps_den, a.S_hyb,
                                   a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, flags);
        }
#undef CCG_EST_ROWS
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
    if (a.S_err || a.S_ad || a.S_ad_err) {
        const int64_t g = std::max<int64_t>(1, std::min<int64_t>((a.n + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL((k_errest<DT, RT, MT>), dim3((unsigned)g), dim3(kBlock), 0, st, (const DT*)a.D,
                           (const DT*)a.Dr, a.n, a.k, a.sidx, a.bit_base, a.orig, (const MT*)a.dmat_c, a.Tcnt, a.Tsum,
                           a.tlen, a.src_sum, E, a.S_err, a.S_ad, a.S_ad_err, flags);
    }
    if (a.S_sweep || a.S_sweep_err) {
        if (!a.sweep_scratch) throw HipError{hipErrorInvalidValue, "threshold sweep scratch"};
        const int32_t k = a.k;
        int32_t k2 = 1;
        while (k2 < k) k2 <<= 1;
        uint16_t* perm = (uint16_t*)a.sweep_scratch;
        MT* ds = (MT*)((char*)a.sweep_scratch + align256(sizeof(uint16_t) * (size_t)k * k));
        hipLaunchKernelGGL((k_sort_rows<MT>), dim3((unsigned)k), dim3(kBlock), sizeof(uint64_t) * (size_t)k2, st,
                           (const MT*)a.dmat_c, k, k2, perm, ds);
        const int64_t g = std::max<int64_t>(1, std::min<int64_t>((a.n + 3) / 4, 16384));
        hipLaunchKernelGGL((k_sweep<DT, RT, MT>), dim3((unsigned)g), dim3(kBlock), 0, st, (const DT*)a.D,
                           (const DT*)a.Dr, a.n, k, a.sidx, a.bit_base, a.orig, (const uint16_t*)perm, (const MT*)ds,
                           a.Tcnt, a.Tsum, a.tlen, a.src_sum, a.S_sweep, a.S_sweep_err, flags);
    }
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

size_t sweep_scratch_bytes(int32_t k) {
    return align256(sizeof(uint16_t) * (size_t)k * k) + align256(sizeof(uint32_t) * (size_t)k * k);
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

size_t epilogue_scratch(int64_t n, int32_t k, int64_t maxd, bool hist_done, bool sweep) {
    const int64_t tlen = maxd + 2;
    size_t s = align256(sizeof(int32_t) * k * tlen) + align256(sizeof(int64_t) * k * tlen) +
               align256(sizeof(uint32_t) * (size_t)k * k) + align256(suffix_chunk_scratch(k, maxd)) + 1024;
    if (!hist_done) s += align256(sizeof(int32_t) * k * (maxd + 1));
    if (sweep) s += sweep_scratch_bytes(k);
    (void)n;
    return s;
}

void run_epilogue(hipStream_t st, const EpilogueArgs& a, void* scratch, size_t scratch_size, DevFlags* flags) {
    if (scratch_size < epilogue_scratch(a.n, a.k, a.maxd, a.hist_done, a.S_sweep || a.S_sweep_err))
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
