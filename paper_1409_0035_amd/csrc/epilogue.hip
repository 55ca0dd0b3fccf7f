// Estimator epilogue: from the node-major distance matrix D[v][i] = d(c_i, v)
// to every estimate of Sec. 2 of the paper, for every node.
//
//   k_reduce    one streaming pass over D: per-sample sums S(c_i) = sum_v D[v][i]
//               (exact centrality of the samples) and, per sample, the histogram
//               hist[i][d] = #{u not in C : d(c_i,u) = d}.
//   k_dmat      sample-to-sample distances dmat[i][j] = d(c_i, c_j) = D[c_j][i].
//   k_suffix    per sample, T_cnt[i][t] = sum_{d >= t} hist[i][d] and
//               T_sum[i][t] = sum_{d >= t} d * hist[i][d]: the tail counts and
//               sums that Alg. 1 builds with its Thresh/bin arrays, here for
//               every integer threshold at once.
//   k_estimate  one wave per node: pivot (argmin of the row, lowest index on
//               ties), Delta, sum of the row, split of the samples into L cap C
//               and HC by dmat[pivot][i] * num <= Delta * den (eps = num/den),
//               |H| and sum_H from the tail tables at t = floor(Delta*den/num)+1,
//               |L| = n-1-|H|-|HC| (Alg. 1 finalisation), and Eq. (6) as the
//               exact integer N = (sum_H + sum_HC)*|L cap C| + |L|*sum_{L cap C}
//               divided once by |L cap C| in IEEE double.
// For directed graphs the distances are round-trip: D + Dr (Sec. 6.1).
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr int64_t kLdsHistMax = 256;  // LDS histogram used while maxd < 256

template <typename DT, bool RT>
__device__ __forceinline__ int64_t load_dist(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t off,
                                             bool& unreached) {
    const uint32_t a = (uint32_t)D[off];
    if (a == DistT<DT>::never) unreached = true;
    int64_t d = a;
    if (RT) {
        const uint32_t b = (uint32_t)Dr[off];
        if (b == DistT<DT>::never) unreached = true;
        d += b;
    }
    return d;
}

// grid.y = column block of 64 samples; lane j handles sample cb*64 + j for a
// contiguous range of nodes per wave.
template <typename DT, bool RT>
__global__ __launch_bounds__(kBlock) void k_reduce(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n,
                                                   int32_t k, const int32_t* __restrict__ sidx, int64_t maxd,
                                                   int32_t* __restrict__ hist, unsigned long long* __restrict__ src_sum,
                                                   int use_lds, DevFlags* flags) {
    extern __shared__ int32_t lds_hist[];  // [(maxd+1)][64] when use_lds
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int32_t cb = blockIdx.y;
    const int32_t i = cb * 64 + lane;
    const bool vi = i < k;
    const int64_t hlen = maxd + 1;
    if (use_lds) {
        for (int64_t t = threadIdx.x; t < hlen * 64; t += kBlock) lds_hist[t] = 0;
        __syncthreads();
    }
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    const int64_t chunk = (n + waves - 1) / waves;
    const int64_t v0 = wid * chunk;
    const int64_t v1 = v0 + chunk < n ? v0 + chunk : n;
    int64_t sum = 0;
    bool unreached = false;
    bool too_far = false;
    for (int64_t v = v0; v < v1; ++v) {
        if (!vi) continue;
        const int64_t d = load_dist<DT, RT>(D, Dr, v * k + i, unreached);
        sum += d;
        if (sidx[v] < 0) {
            if (d > maxd) {
                too_far = true;
            } else if (use_lds) {
                atomicAdd(&lds_hist[d * 64 + lane], 1);
            } else {
                atomicAdd(&hist[(int64_t)i * hlen + d], 1);
            }
        }
    }
    if (vi && sum) atomicAdd(&src_sum[i], (unsigned long long)sum);
    if (unreached) flags->disconnected = 1;
    if (too_far) flags->overflow = 1;
    if (use_lds) {
        __syncthreads();
        for (int64_t t = threadIdx.x; t < hlen * 64; t += kBlock) {
            const int32_t c = lds_hist[t];
            const int32_t ii = cb * 64 + (int32_t)(t & 63);
            if (c && ii < k) atomicAdd(&hist[(int64_t)ii * hlen + (t >> 6)], c);
        }
    }
}

template <typename DT, bool RT>
__global__ void k_dmat(const DT* __restrict__ D, const DT* __restrict__ Dr, const int32_t* __restrict__ samples,
                       int32_t k, int32_t* __restrict__ dmat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)k * k) return;
    const int32_t i = (int32_t)(t / k), j = (int32_t)(t % k);
    bool unreached = false;
    dmat[t] = (int32_t)load_dist<DT, RT>(D, Dr, (int64_t)samples[j] * k + i, unreached);
}

template <typename DT, bool RT>
__global__ void k_to_i32(const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t count, int32_t* __restrict__ out) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        bool unreached = false;
        out[t] = (int32_t)load_dist<DT, RT>(D, Dr, t, unreached);
    }
}

// one block per sample: reverse inclusive scan of hist[i][0..maxd] into
// T[i][t] for t = 0..maxd+1 (T[i][maxd+1] = 0)
__global__ __launch_bounds__(kBlock) void k_suffix(const int32_t* __restrict__ hist, int64_t maxd,
                                                   int32_t* __restrict__ Tcnt, int64_t* __restrict__ Tsum) {
    __shared__ int64_t wc[kBlock / 64], ws[kBlock / 64];
    const int32_t i = blockIdx.x;
    const int64_t hlen = maxd + 1, tlen = maxd + 2;
    const int32_t* h = hist + (int64_t)i * hlen;
    int32_t* tc = Tcnt + (int64_t)i * tlen;
    int64_t* ts = Tsum + (int64_t)i * tlen;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t carry_c = 0, carry_s = 0;
    if (threadIdx.x == 0) {
        tc[maxd + 1] = 0;
        ts[maxd + 1] = 0;
    }
    // chunks of kBlock entries from the top: thread j takes d = top - j
    for (int64_t top = maxd; top >= 0; top -= kBlock) {
        const int64_t d = top - threadIdx.x;
        int64_t c = d >= 0 ? h[d] : 0;
        int64_t s = c * (d >= 0 ? d : 0);
        // inclusive scan within the wave
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
}

template <typename DT, bool RT>
__global__ __launch_bounds__(kBlock) void k_estimate(
    const DT* __restrict__ D, const DT* __restrict__ Dr, int64_t n, int32_t k, const int32_t* __restrict__ sidx,
    const int32_t* __restrict__ dmat, const int32_t* __restrict__ Tcnt, const int64_t* __restrict__ Tsum,
    int64_t tlen, const unsigned long long* __restrict__ src_sum, int64_t en, int64_t ed, double* S_hyb,
    double* S_samp, int64_t* S_piv, int64_t* S_pub, int32_t* pivot_out, int32_t* delta_out, int64_t* sampsum_out,
    DevFlags* flags) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t LIM = (int64_t)1 << 53;
    for (int64_t v = wid; v < n; v += waves) {
        bool unreached = false;
        uint64_t best = ~0ull;
        int64_t sum = 0;
        for (int32_t i = lane; i < k; i += 64) {
            const int64_t d = load_dist<DT, RT>(D, Dr, v * k + i, unreached);
            const uint64_t key = ((uint64_t)d << 32) | (uint32_t)i;
            best = key < best ? key : best;
            sum += d;
        }
        best = wave_min64(best);
        sum = wave_sum64(sum);
        const int32_t p = (int32_t)(best & 0xffffffffu);
        const int64_t delta = (int64_t)(best >> 32);
        const int32_t j = sidx[v];
        double hyb, samp;
        int64_t piv, pub;
        bool ovf = false;
        if (j >= 0) {
            // sampled node: exact S(v) for every estimator
            const int64_t S = (int64_t)src_sum[j];
            hyb = samp = (double)S;
            piv = pub = S;
            ovf = S >= LIM;
        } else {
            const int64_t thr = delta * ed;
            int64_t lcsum = 0;
            int32_t lcnum = 0;
            const int32_t* drow = dmat + (int64_t)p * k;
            for (int32_t i = lane; i < k; i += 64) {
                if ((int64_t)drow[i] * en <= thr) {
                    bool u2 = false;
                    lcsum += load_dist<DT, RT>(D, Dr, v * k + i, u2);
                    lcnum += 1;
                }
            }
            lcsum = wave_sum64(lcsum);
            lcnum = wave_sum32(lcnum);
            const int64_t tix = thr / en + 1;  // d > floor(Delta/eps)  <=>  d >= tix
            int64_t hnum = 0, hsum = 0;
            if (tix < tlen) {
                hnum = Tcnt[(int64_t)p * tlen + tix];
                hsum = Tsum[(int64_t)p * tlen + tix];
            }
            const int64_t hcsum = sum - lcsum;
            const int64_t lnum = (n - 1) - hnum - (int64_t)(k - lcnum);
            const int64_t a = hsum + hcsum;
            int64_t t1 = 0, t2 = 0, N = 0;
            ovf = __builtin_mul_overflow(a, (int64_t)lcnum, &t1) || __builtin_mul_overflow(lcsum, lnum, &t2) ||
                  __builtin_add_overflow(t1, t2, &N) || N >= LIM || lcnum < 1 || lnum < lcnum;
            hyb = (double)N / (double)lcnum;
            int64_t ss = 0;
            ovf = ovf || __builtin_mul_overflow(n - 1, sum, &ss) || ss >= LIM;
            samp = (double)ss / (double)k;
            piv = (int64_t)src_sum[p];
            pub = piv + (n - 1) * delta;
        }
        if (lane == 0) {
            if (S_hyb) S_hyb[v] = hyb;
            if (S_samp) S_samp[v] = samp;
            if (S_piv) S_piv[v] = piv;
            if (S_pub) S_pub[v] = pub;
            if (pivot_out) pivot_out[v] = p;
            if (delta_out) delta_out[v] = (int32_t)delta;
            if (sampsum_out) sampsum_out[v] = sum;
            if (ovf) flags->overflow = 1;
        }
        if (unreached) flags->disconnected = 1;
    }
}

__global__ void k_sidx(const int32_t* __restrict__ samples, int32_t k, int32_t* __restrict__ sidx, int64_t n,
                       DevFlags* flags) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int32_t v = samples[i];
    if (v < 0 || v >= n) {
        flags->bad_sample = 1;
        return;
    }
    sidx[v] = i;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        p[t] = value;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename DT, bool RT>
void epilogue_t(hipStream_t st, const EpilogueArgs& a, void* scratch, DevFlags* flags) {
    const int64_t n = a.n;
    const int32_t k = a.k;
    const int64_t hlen = a.maxd + 1, tlen = a.maxd + 2;
    char* p = (char*)scratch;
    int32_t* sidx = (int32_t*)p;
    p += align256(sizeof(int32_t) * n);
    int32_t* hist = (int32_t*)p;
    p += align256(sizeof(int32_t) * k * hlen);
    int32_t* Tcnt = (int32_t*)p;
    p += align256(sizeof(int32_t) * k * tlen);
    int64_t* Tsum = (int64_t*)p;

    const DT* D = (const DT*)a.D;
    const DT* Dr = (const DT*)a.Dr;
    fill_u32(st, sidx, 0xFFFFFFFFu, (size_t)n);
    fill_u32(st, hist, 0u, (size_t)(k * hlen));
    fill_u32(st, a.src_sum, 0u, (size_t)k * 2);
    hipLaunchKernelGGL(k_sidx, dim3((k + 255) / 256), dim3(256), 0, st, a.samples, k, sidx, n, flags);

    const int use_lds = a.maxd < kLdsHistMax ? 1 : 0;
    const size_t lds = use_lds ? sizeof(int32_t) * 64 * hlen : 0;
    int64_t gx = (n + 255) / 256;
    if (gx > 1024) gx = 1024;
    if (gx < 1) gx = 1;
    dim3 grid((unsigned)gx, (unsigned)((k + 63) / 64));
    hipLaunchKernelGGL((k_reduce<DT, RT>), grid, dim3(kBlock), lds, st, D, Dr, n, k, sidx, a.maxd, hist,
                       (unsigned long long*)a.src_sum, use_lds, flags);
    CCG_HIP(hipGetLastError());
    const int64_t kk = (int64_t)k * k;
    hipLaunchKernelGGL((k_dmat<DT, RT>), dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, st, D, Dr, a.samples, k,
                       a.dmat);
    hipLaunchKernelGGL(k_suffix, dim3(k), dim3(kBlock), 0, st, hist, a.maxd, Tcnt, Tsum);
    int64_t ge = (n + 3) / 4;
    if (ge > 8192) ge = 8192;
    if (ge < 1) ge = 1;
    hipLaunchKernelGGL((k_estimate<DT, RT>), dim3((unsigned)ge), dim3(kBlock), 0, st, D, Dr, n, k, sidx, a.dmat,
                       Tcnt, Tsum, tlen, (const unsigned long long*)a.src_sum, a.eps_num, a.eps_den, a.S_hyb,
                       a.S_samp, a.S_piv, a.S_pub, a.pivot, a.delta, a.sampsum, flags);
    CCG_HIP(hipGetLastError());
    if (a.Dout) {
        const int64_t cnt = n * k;
        int64_t g = (cnt + 255) / 256;
        if (g > 65536) g = 65536;
        hipLaunchKernelGGL((k_to_i32<DT, RT>), dim3((unsigned)g), dim3(256), 0, st, D, Dr, cnt, a.Dout);
    }
}

}  // namespace

void fill_u32(hipStream_t st, void* p, uint32_t value, size_t count) {
    if (count == 0) return;
    size_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, (uint32_t*)p, value, count);
}

size_t epilogue_scratch(int64_t n, int32_t k, int64_t maxd) {
    const int64_t hlen = maxd + 1, tlen = maxd + 2;
    return align256(sizeof(int32_t) * n) + align256(sizeof(int32_t) * k * hlen) + align256(sizeof(int32_t) * k * tlen) +
           align256(sizeof(int64_t) * k * tlen) + 1024;
}

void run_epilogue(hipStream_t st, const EpilogueArgs& a, void* scratch, size_t scratch_size, DevFlags* flags) {
    if (scratch_size < epilogue_scratch(a.n, a.k, a.maxd)) throw HipError{hipErrorOutOfMemory, "epilogue scratch"};
    const bool rt = a.Dr != nullptr;
    switch (a.dk) {
        case DistKind::U8:
            rt ? epilogue_t<uint8_t, true>(st, a, scratch, flags) : epilogue_t<uint8_t, false>(st, a, scratch, flags);
            break;
        case DistKind::U16:
            rt ? epilogue_t<uint16_t, true>(st, a, scratch, flags) : epilogue_t<uint16_t, false>(st, a, scratch, flags);
            break;
        default:
            rt ? epilogue_t<uint32_t, true>(st, a, scratch, flags) : epilogue_t<uint32_t, false>(st, a, scratch, flags);
            break;
    }
}

}  // namespace ccg
