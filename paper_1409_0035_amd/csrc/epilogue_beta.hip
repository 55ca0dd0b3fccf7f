// Node-weighted hybrid estimate (Sec. 5, Algorithm 3) from the int32 distance
// rows D[v][i] = d(c_i, v) at the caller's node ids, the sample distance
// matrix and the node weights beta.
//
// The sample has adjusted weights beta^(c) = max(tau, beta(c)), tau = R/m:
// light samples weigh tau, heavy ones their own weight.  For v outside C,
// with the pivot, Delta and the sets L, HC, H of Eq. (6):
//   S_beta^(v) = sum_H beta(u) d(c(v),u) + sum_HC beta(u) d(v,u) + sum_{L cap C} beta^(u) d(v,u)
// as N / m with N = (sum_H + sum_HC + sum_{heavy L cap C}) * m + R * sum_{light L cap C} d,
// exact integers and one division; the variance estimate of the L term,
// sum over light L cap C of d^2 (tau - beta) tau, as t * (t * A - B), t = R/m.
// sum_H comes from beta-weighted tail tables: per sample, the beta mass of
// the nodes outside C at each distance (k_beta_hist), suffix-summed with the
// distance (k_beta_suffix), read at floor(Delta/eps) + 1.
//
//   k_beta_maxd      largest distance (the tables' length), when the traversal
//                    gives no bound on it
//   k_beta_hist      hw[i][d] = sum of beta(u) over u outside C with d(c_i,u) = d,
//                    per block in LDS when the table fits
//   k_beta_suffix    WT[i][t] = sum_{d >= t} d * hw[i][d] and WC[i][t] = sum_{d >= t}
//                    hw[i][d]; exact S_beta(c_i) = WT[i][0] + sum_j beta(c_j) d(c_i, c_j);
//                    the samples at the largest distance from c_i, listed
// The error estimate (Sec. 4.1 with beta masses, Sec. 5) adds to the variance
// estimate beta(H) (from WC) times the beta-weighted mean over HC of
// (d(v,c_i) - d(c(v),c_i))^2.  When HC has no weight the mean is over the
// samples at the largest distance from the pivot (Sec. 4.1's suffix of the
// farthest samples, read from the pivot's list), and 0 if those weigh
// nothing either.
//   k_beta_estimate  one lane per node: pivot, Delta, the split of the samples,
//                    the estimate and the variance estimate (k_beta_estimate_rows:
//                    G lanes per node, for rows of a multiple of 16 bytes)
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;

__global__ void k_beta_maxd(const int32_t* __restrict__ D, int64_t count, int32_t* __restrict__ out) {
    int32_t m = 0;
    const int64_t q = count / 4;  // 16-byte pieces, then the tail
    const int4* D4 = (const int4*)D;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < q; t += (int64_t)gridDim.x * blockDim.x) {
        const int4 x = D4[t];
        m = max(max(m, x.x), max(x.y, max(x.z, x.w)));
    }
    for (int64_t t = q * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        m = max(m, D[t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (lane_id() == 0) atomicMax(out, m);
}

__global__ __launch_bounds__(kBlock) void k_beta_hist(const int32_t* __restrict__ D, int64_t n, int32_t k,
                                                      const int32_t* __restrict__ sidx,
                                                      const uint32_t* __restrict__ beta, int64_t hlen,
                                                      unsigned long long* __restrict__ hw, int use_lds) {
    extern __shared__ unsigned long long lh[];
    const int64_t cells = (int64_t)k * hlen;
    if (use_lds) {
        for (int64_t c = threadIdx.x; c < cells; c += kBlock) lh[c] = 0;
        __syncthreads();
    }
    const int64_t count = n * k;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < count; t += (int64_t)gridDim.x * kBlock) {
        const int64_t u = t / k;
        const int32_t i = (int32_t)(t - u * k);
        const uint32_t b = beta[u];
        const int32_t d = D[t];
        // the caller has ruled out unreached entries; the bound keeps the tables safe regardless
        if (b == 0 || sidx[u] >= 0 || d < 0 || d >= hlen) continue;
        const int64_t cell = (int64_t)i * hlen + d;
        if (use_lds) atomicAdd(&lh[cell], (unsigned long long)b);
        else atomicAdd(&hw[cell], (unsigned long long)b);
    }
    if (use_lds) {
        __syncthreads();
        for (int64_t c = threadIdx.x; c < cells; c += kBlock)
            if (lh[c]) atomicAdd(&hw[c], lh[c]);
    }
}

// One block per sample: reverse inclusive scan of d * hw[i][d].
__global__ __launch_bounds__(kBlock) void k_beta_suffix(const unsigned long long* __restrict__ hw, int32_t k,
                                                        int64_t hlen, const int32_t* __restrict__ dmat,
                                                        const int32_t* __restrict__ samples,
                                                        const uint32_t* __restrict__ beta, int64_t* __restrict__ WT,
                                                        int64_t* __restrict__ WC, int64_t* __restrict__ Sx,
                                                        int32_t* __restrict__ farP, int32_t* __restrict__ farCnt,
                                                        int32_t* __restrict__ farIdx, uint32_t* __restrict__ farB,
                                                        DevFlags* flags) {
    __shared__ int64_t ws[kBlock / 64], wc[kBlock / 64];
    const int32_t i = blockIdx.x;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t* wt = WT + (int64_t)i * hlen;
    int64_t* wcn = WC + (int64_t)i * hlen;
    int64_t carry = 0, carry_c = 0;
    bool ovf = false;
    for (int64_t top = hlen - 1; top >= 0; top -= kBlock) {
        const int64_t d = top - threadIdx.x;
        int64_t s = 0, c = 0;
        if (d >= 0) {
            const unsigned long long h = hw[(int64_t)i * hlen + d];
            unsigned long long prod = 0;
            const bool o = __builtin_mul_overflow(h, (unsigned long long)d, &prod);
            ovf = ovf || o || prod > (unsigned long long)INT64_MAX;
            s = (int64_t)prod;
            c = (int64_t)h;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(s, off), z = __shfl_up(c, off);
            if (lane >= off) {
                s += y;
                c += z;
            }
        }
        if (lane == 63) {
            ws[wave] = s;
            wc[wave] = c;
        }
        __syncthreads();
        int64_t pre = carry, pre_c = carry_c;
        for (int w = 0; w < wave; w++) {
            pre += ws[w];
            pre_c += wc[w];
        }
        if (d >= 0) {
            wt[d] = pre + s;
            wcn[d] = pre_c + c;
        }
        for (int w = 0; w < kBlock / 64; w++) {
            carry += ws[w];
            carry_c += wc[w];
        }
        __syncthreads();
    }
    // the samples' own part: sum_j beta(c_j) d(c_i, c_j); and the largest
    // d(c_i, c_j), the distance of the samples that stand in for an empty HC
    // when c_i is the pivot
    int64_t sj = 0;
    int32_t far = INT32_MIN;
    for (int32_t j = threadIdx.x; j < k; j += kBlock) {
        const int32_t d = dmat[(int64_t)i * k + j];
        sj += (int64_t)beta[samples[j]] * d;
        far = max(far, d);
    }
    sj = wave_sum64(sj);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) far = max(far, __shfl_xor(far, off));
    __shared__ int32_t wf[kBlock / 64];
    if (lane == 0) {
        ws[wave] = sj;
        wf[wave] = far;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = carry;
        int32_t f = INT32_MIN;
        for (int w = 0; w < kBlock / 64; w++) {
            tot += ws[w];
            f = max(f, wf[w]);
        }
        Sx[i] = tot;
        farP[i] = f;
        wf[0] = f;
        if (carry < 0 || tot < 0) ovf = true;
    }
    // the samples at that distance, listed (in any order) for the estimate
    __shared__ int32_t nfar;
    if (threadIdx.x == 0) nfar = 0;
    __syncthreads();
    const int32_t fmax = wf[0];
    for (int32_t j = threadIdx.x; j < k; j += kBlock)
        if (dmat[(int64_t)i * k + j] == fmax) {
            const int32_t t = atomicAdd(&nfar, 1);
            farIdx[(int64_t)i * k + t] = j;
            farB[(int64_t)i * k + t] = beta[samples[j]];
        }
    __syncthreads();
    if (threadIdx.x == 0) farCnt[i] = nfar;
    if (ovf) flags->overflow = 1;
}

__global__ __launch_bounds__(kBlock) void k_beta_estimate(
    const int32_t* __restrict__ D, int64_t n, int32_t k, const int32_t* __restrict__ dmat,
    const int32_t* __restrict__ sidx, const int32_t* __restrict__ samples, const uint32_t* __restrict__ beta,
    const uint8_t* __restrict__ light, int64_t R, int32_t m, int64_t num, int64_t den, const int64_t* __restrict__ WT,
    const int64_t* __restrict__ WC, int64_t hlen, const int64_t* __restrict__ Sx, const int32_t* __restrict__ farP,
    const int32_t* __restrict__ farCnt, const int32_t* __restrict__ farIdx, const uint32_t* __restrict__ farB,
    double* S, double* var, double* err, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    bool ovf = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int32_t js = sidx[v];
        if (js >= 0) {  // a sample: its exact weighted sum
            const int64_t x = Sx[js];
            ovf = ovf || x >= LIM;
            if (S) S[v] = (double)x;
            if (var) var[v] = 0.0;
            if (err) err[v] = 0.0;
            continue;
        }
        const int32_t* row = D + v * k;
        int32_t best = INT32_MAX, p = 0;
        for (int32_t i = 0; i < k; i++) {
            const int32_t d = row[i];
            if (d < best) {
                best = d;
                p = i;
            }
        }
        const int64_t delta = best;
        const int32_t* drow = dmat + (int64_t)p * k;
        int64_t HC = 0, Lb = 0, Ls = 0, A = 0, B = 0, HCb = 0, HCsq = 0;
        bool e = false;
        for (int32_t i = 0; i < k; i++) {
            const int64_t d = row[i];
            const int64_t b = beta[samples[i]];
            int64_t t = 0;
            if ((int64_t)drow[i] * num <= delta * den) {  // L cap C
                if (light[i]) {
                    Ls += d;
                    int64_t dd = 0;
                    e = e || __builtin_mul_overflow(d, d, &dd) || __builtin_add_overflow(A, dd, &A) ||
                        __builtin_mul_overflow(dd, b, &t) || __builtin_add_overflow(B, t, &B);
                } else {
                    e = e || __builtin_mul_overflow(b, d, &t) || __builtin_add_overflow(Lb, t, &Lb);
                }
            } else {  // HC
                const int64_t df = d - drow[i];
                int64_t q = 0;
                HCb += b;
                e = e || __builtin_mul_overflow(b, d, &t) || __builtin_add_overflow(HC, t, &HC) ||
                    __builtin_mul_overflow(df * df, b, &q) || __builtin_add_overflow(HCsq, q, &HCsq);
            }
        }
        if (err && HCb == 0) {  // the samples farthest from the pivot stand in for HC (the pivot's list)
            const int32_t far = farP[p], cnt = farCnt[p];
            for (int32_t t = 0; t < cnt; t++) {
                const int32_t i = farIdx[(int64_t)p * k + t];
                const int64_t b = farB[(int64_t)p * k + t], df = (int64_t)row[i] - far;
                int64_t q = 0;
                HCb += b;
                e = e || __builtin_mul_overflow(df * df, b, &q) || __builtin_add_overflow(HCsq, q, &HCsq);
            }
        }
        const int64_t thr = delta * den / num;  // H: nodes outside C at distance > floor(Delta/eps)
        const int64_t H = thr + 1 < hlen ? WT[(int64_t)p * hlen + thr + 1] : 0;
        const int64_t Hb = thr + 1 < hlen ? WC[(int64_t)p * hlen + thr + 1] : 0;
        int64_t s1 = 0, s2 = 0, s3 = 0, N = 0;
        e = e || __builtin_add_overflow(H, HC, &s1) || __builtin_add_overflow(s1, Lb, &s1) ||
            __builtin_mul_overflow(s1, (int64_t)m, &s2) || __builtin_mul_overflow(Ls, R, &s3) ||
            __builtin_add_overflow(s2, s3, &N) || N >= LIM;
        ovf = ovf || e;
        if (S) S[v] = (double)N / (double)m;
        const double tt = (double)R / (double)m;
        const double vv = tt * (tt * (double)A - (double)B);
        if (var) var[v] = vv;
        if (err) err[v] = vv + (HCb > 0 ? ((double)HCsq / (double)HCb) * (double)Hb : 0.0);
    }
    if (ovf) flags->overflow = 1;
}

// The same estimate with G lanes per node, each taking every G-th 16-byte
// piece of the node's row (rows of k int32, k a multiple of 4): the pivot
// by a group argmin (lowest index on ties), then the group sums.
template <int G>
__global__ __launch_bounds__(kBlock) void k_beta_estimate_rows(
    const int32_t* __restrict__ D, int64_t n, int32_t k, const int32_t* __restrict__ dmat,
    const int32_t* __restrict__ sidx, const int32_t* __restrict__ samples, const uint32_t* __restrict__ beta,
    const uint8_t* __restrict__ light, int64_t R, int32_t m, int64_t num, int64_t den, const int64_t* __restrict__ WT,
    const int64_t* __restrict__ WC, int64_t hlen, const int64_t* __restrict__ Sx, const int32_t* __restrict__ farP,
    const int32_t* __restrict__ farCnt, const int32_t* __restrict__ farIdx, const uint32_t* __restrict__ farB,
    double* S, double* var, double* err, DevFlags* flags) {
    const int64_t LIM = (int64_t)1 << 53;
    const int g = threadIdx.x & (G - 1);
    const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
    const int32_t pieces = k / 4;
    bool ovf = false;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G; v < n; v += groups) {
        const int32_t js = sidx[v];
        if (js >= 0) {
            if (g == 0) {
                const int64_t x = Sx[js];
                ovf = ovf || x >= LIM;
                if (S) S[v] = (double)x;
                if (var) var[v] = 0.0;
                if (err) err[v] = 0.0;
            }
            continue;
        }
        const int4* row = (const int4*)(D + v * k);
        int32_t best = INT32_MAX, bi = k;
        for (int32_t c = g; c < pieces; c += G) {
            const int4 x = row[c];
            const int32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (w[q] < best) {
                    best = w[q];
                    bi = 4 * c + q;
                }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const int32_t ob = __shfl_xor(best, off, G), oi = __shfl_xor(bi, off, G);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int32_t p = bi < k ? bi : k - 1;  // a row with no finite entry (an error the traversal reports) stays in bounds
        const int64_t delta = best;
        const int32_t* drow = dmat + (int64_t)p * k;
        int64_t HC = 0, Lb = 0, Ls = 0, A = 0, B = 0, HCb = 0, HCsq = 0;
        bool e = false;
        for (int32_t c = g; c < pieces; c += G) {
            const int4 x = row[c];
            const int32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int32_t i = 4 * c + q;
                const int64_t d = w[q];
                const int64_t b = beta[samples[i]];
                int64_t t = 0;
                if ((int64_t)drow[i] * num <= delta * den) {
                    if (light[i]) {
                        Ls += d;
                        int64_t dd = 0;
                        e = e || __builtin_mul_overflow(d, d, &dd) || __builtin_add_overflow(A, dd, &A) ||
                            __builtin_mul_overflow(dd, b, &t) || __builtin_add_overflow(B, t, &B);
                    } else {
                        e = e || __builtin_mul_overflow(b, d, &t) || __builtin_add_overflow(Lb, t, &Lb);
                    }
                } else {
                    const int64_t df = d - drow[i];
                    int64_t qq = 0;
                    HCb += b;
                    e = e || __builtin_mul_overflow(b, d, &t) || __builtin_add_overflow(HC, t, &HC) ||
                        __builtin_mul_overflow(df * df, b, &qq) || __builtin_add_overflow(HCsq, qq, &HCsq);
                }
            }
        }
        // group sums; overflow of a sum shows as a partial sum out of range,
        // so each partial stays below 2^62 and the total is checked
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const int64_t a1 = __shfl_xor(HC, off, G), a2 = __shfl_xor(Lb, off, G), a3 = __shfl_xor(Ls, off, G);
            const int64_t a4 = __shfl_xor(A, off, G), a5 = __shfl_xor(B, off, G);
            const int64_t a6 = __shfl_xor(HCb, off, G), a7 = __shfl_xor(HCsq, off, G);
            e = e || __builtin_add_overflow(HC, a1, &HC) || __builtin_add_overflow(Lb, a2, &Lb) ||
                __builtin_add_overflow(Ls, a3, &Ls) || __builtin_add_overflow(A, a4, &A) ||
                __builtin_add_overflow(B, a5, &B) || __builtin_add_overflow(HCb, a6, &HCb) ||
                __builtin_add_overflow(HCsq, a7, &HCsq);
        }
        if (err && HCb == 0) {  // HC has no weight (HCb is the group's total): the samples farthest from the pivot
            // instead, from the pivot's list; the terms are non-negative, so a
            // sum overflows in some grouping exactly when the total does
            const int32_t far = farP[p], cnt = farCnt[p];
            for (int32_t t = g; t < cnt; t += G) {
                const int32_t i = farIdx[(int64_t)p * k + t];
                const int64_t b = farB[(int64_t)p * k + t], df = (int64_t)D[v * k + i] - far;
                int64_t qq = 0;
                HCb += b;
                e = e || __builtin_mul_overflow(df * df, b, &qq) || __builtin_add_overflow(HCsq, qq, &HCsq);
            }
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const int64_t a6 = __shfl_xor(HCb, off, G), a7 = __shfl_xor(HCsq, off, G);
                e = e || __builtin_add_overflow(HCb, a6, &HCb) || __builtin_add_overflow(HCsq, a7, &HCsq);
            }
        }
        if (g == 0) {
            const int64_t thr = delta * den / num;
            const int64_t H = thr + 1 < hlen ? WT[(int64_t)p * hlen + thr + 1] : 0;
            const int64_t Hb = thr + 1 < hlen ? WC[(int64_t)p * hlen + thr + 1] : 0;
            int64_t s1 = 0, s2 = 0, s3 = 0, N = 0;
            e = e || __builtin_add_overflow(H, HC, &s1) || __builtin_add_overflow(s1, Lb, &s1) ||
                __builtin_mul_overflow(s1, (int64_t)m, &s2) || __builtin_mul_overflow(Ls, R, &s3) ||
                __builtin_add_overflow(s2, s3, &N) || N >= LIM;
            if (S) S[v] = (double)N / (double)m;
            const double tt = (double)R / (double)m;
            const double vv = tt * (tt * (double)A - (double)B);
            if (var) var[v] = vv;
            if (err) err[v] = vv + (HCb > 0 ? ((double)HCsq / (double)HCb) * (double)Hb : 0.0);
        }
        ovf = ovf || e;
    }
    if (ovf) flags->overflow = 1;
}

}  // namespace

void run_beta_epilogue(hipStream_t st, const BetaArgs& a, DevFlags* flags) {
    const int64_t n = a.n;
    const int32_t k = a.k;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    // the tables' length: the largest distance, or a bound on it the
    // traversal already knows (entries past the largest distance stay zero)
    const int64_t cells = n * k;
    int64_t maxd = a.maxd;
    if (maxd < 0) {
        int32_t* dmax = (int32_t*)a.small_scratch;
        fill_u32(st, dmax, 0u, 1);
        hipLaunchKernelGGL(k_beta_maxd,
                           dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((cells + 255) / 256, 8192))), dim3(256),
                           0, st, a.D, cells, dmax);
        int32_t hm = 0;
        CCG_HIP(hipMemcpyAsync(&hm, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CCG_HIP(hipStreamSynchronize(st));
        maxd = hm;
    }
    const int64_t hlen = maxd + 2;
    const size_t need = al(sizeof(uint64_t) * (size_t)k * hlen) * 3 + al(sizeof(int64_t) * (size_t)k) +
                        al(sizeof(int32_t) * (size_t)k) * 2 + al(sizeof(int32_t) * (size_t)k * k) * 2;
    void* scr = a.get_scratch(need);
    char* q = (char*)scr;
    unsigned long long* hw = (unsigned long long*)q;
    q += al(sizeof(uint64_t) * (size_t)k * hlen);
    int64_t* WT = (int64_t*)q;
    q += al(sizeof(uint64_t) * (size_t)k * hlen);
    int64_t* WC = (int64_t*)q;
    q += al(sizeof(uint64_t) * (size_t)k * hlen);
    int64_t* Sx = (int64_t*)q;
    q += al(sizeof(int64_t) * (size_t)k);
    int32_t* farP = (int32_t*)q;
    q += al(sizeof(int32_t) * (size_t)k);
    int32_t* farCnt = (int32_t*)q;
    q += al(sizeof(int32_t) * (size_t)k);
    int32_t* farIdx = (int32_t*)q;
    q += al(sizeof(int32_t) * (size_t)k * k);
    uint32_t* farB = (uint32_t*)q;
    fill_u32(st, hw, 0u, (size_t)k * hlen * 2);
    const size_t lds = sizeof(uint64_t) * (size_t)k * hlen;
    const int use_lds = lds <= 48 * 1024 ? 1 : 0;
    const unsigned hb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cells + kBlock - 1) / kBlock, use_lds ? 1024 : 8192));
    hipLaunchKernelGGL(k_beta_hist, dim3(hb), dim3(kBlock), use_lds ? lds : 0, st, a.D, n, k, a.sidx, a.beta, hlen, hw,
                       use_lds);
    hipLaunchKernelGGL(k_beta_suffix, dim3((unsigned)k), dim3(kBlock), 0, st, (const unsigned long long*)hw, k, hlen,
                       a.dmat, a.samples, a.beta, WT, WC, Sx, farP, farCnt, farIdx, farB, flags);
    const int32_t pieces = k % 4 == 0 ? k / 4 : 0;
    const int G = pieces >= 16 ? 16 : (pieces >= 8 ? 8 : (pieces >= 4 ? 4 : 0));
    const unsigned eb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n * (G ? G : 1) + kBlock - 1) / kBlock, 16384));
#define CCG_BETA_ROWS(GG)                                                                                            \
    hipLaunchKernelGGL((k_beta_estimate_rows<GG>), dim3(eb), dim3(kBlock), 0, st, a.D, n, k, a.dmat, a.sidx,          \
                       a.samples, a.beta, a.light, a.R, a.m, a.eps_num, a.eps_den, (const int64_t*)WT,                 \
                       (const int64_t*)WC, hlen, (const int64_t*)Sx, (const int32_t*)farP,      \
                       (const int32_t*)farCnt, (const int32_t*)farIdx, (const uint32_t*)farB, a.S, a.var, a.err, flags)
    switch (G) {
        case 16: CCG_BETA_ROWS(16); break;
        case 8: CCG_BETA_ROWS(8); break;
        case 4: CCG_BETA_ROWS(4); break;
        default:
            hipLaunchKernelGGL(k_beta_estimate, dim3(eb), dim3(kBlock), 0, st, a.D, n, k, a.dmat, a.sidx, a.samples,
                               a.beta, a.light, a.R, a.m, a.eps_num, a.eps_den, (const int64_t*)WT,
                               (const int64_t*)WC, hlen, (const int64_t*)Sx, (const int32_t*)farP,
                               (const int32_t*)farCnt, (const int32_t*)farIdx, (const uint32_t*)farB, a.S, a.var,
                               a.err, flags);
    }
#undef CCG_BETA_ROWS
    CCG_HIP(hipGetLastError());
}

}  // namespace ccg
