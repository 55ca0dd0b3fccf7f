// Priority ranks of node-weighted reachability sampling (Sec. 6.2,
// Algorithm 5) on the device.
//
// Node u of positive weight beta(u) gets the rank U(u) / (2^53 beta(u)), with
// U(u) = (x_u >> 11) + 1 and x_u the (u+1)-th output of SplitMix64 from the
// seed; the sources are taken in increasing rank.  SplitMix64's i-th output
// depends on i alone (its state after i steps is seed + i * gamma), so every
// node draws its own U.
//
// Order: U / beta rounded to double is monotone in the exact rank, so
// different doubles order as the exact ranks do, and positive doubles order
// as their bit patterns.  An LSD radix sort (four stable passes of 8 bits)
// orders the nodes by the upper 32 bits of the double; then each run of equal
// upper halves is sorted by the whole double, equal doubles by the exact
// cross products U(a) beta(b) vs U(b) beta(a), and equal ranks by node id.
#include "internal.h"

namespace ccg {

namespace {

constexpr int kBlock = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kBlock * kPerThread;  // elements per block in a radix pass
constexpr int kDigits = 256;

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per internal node v (caller id orig[v]): its weight and U at internal ids,
// and, for positive weights, the sort key appended to the lists.
__global__ void k_prio_init(int64_t n, uint64_t seed, const uint32_t* __restrict__ beta_c,
                            const int32_t* __restrict__ orig, uint32_t* __restrict__ beta_i, uint64_t* __restrict__ U_i,
                            uint64_t* __restrict__ key, uint32_t* __restrict__ hi, uint32_t* __restrict__ pos,
                            int32_t* __restrict__ vals, int32_t* count) {
    for (int64_t v0 = (int64_t)blockIdx.x * kBlock; v0 < n; v0 += (int64_t)gridDim.x * kBlock) {
        const int64_t v = v0 + threadIdx.x;
        bool take = false;
        uint64_t U = 0, bits = 0;
        if (v < n) {
            const int64_t u = orig[v];
            const uint32_t b = beta_c[u];
            U = (splitmix_at(seed, (uint64_t)u + 1) >> 11) + 1;
            beta_i[v] = b;
            U_i[v] = U;
            if (b > 0) {
                const double kd = (double)U / (double)b;  // both exact; one IEEE division
                bits = (uint64_t)__double_as_longlong(kd);
                take = true;
            }
        }
        const int idx = wave_append(count, take);
        if (take) {
            key[idx] = bits;
            hi[idx] = (uint32_t)(bits >> 32);
            pos[idx] = (uint32_t)idx;
            vals[idx] = (int32_t)v;
        }
    }
}

// Digit counts of each block's tile: hist[d * nblocks + b].
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ hi, int64_t m, int shift,
                                                       int32_t* __restrict__ hist) {
    __shared__ int32_t c[kDigits];
    c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int q = 0; q < kPerThread; q++) {
        const int64_t i = t0 + (int64_t)q * kBlock + threadIdx.x;
        if (i < m) atomicAdd(&c[(hi[i] >> shift) & (kDigits - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = c[threadIdx.x];
}

// Exclusive prefix sum over the whole digit-major table (one block).
__global__ __launch_bounds__(1024) void k_radix_scan(int32_t* hist, int64_t count) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int64_t base = 0; base < count; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t x = i < count ? hist[i] : 0;
        int32_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < wave; w++) before += wsum[w];
        if (i < count) hist[i] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 16; w++) carry += wsum[w];
        __syncthreads();
    }
}

// Stable scatter of each block's tile by digit: the tile is read in rounds
// of 256 elements in order; inside a round, an element's place among equal
// digits comes from its wave's peers (eight ballots) and the earlier waves.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* __restrict__ hi_in,
                                                          const uint32_t* __restrict__ pos_in, int64_t m, int shift,
                                                          const int32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ hi_out, uint32_t* __restrict__ pos_out) {
    __shared__ int32_t base[kDigits];
    __shared__ int32_t wcnt[kBlock / 64][kDigits];
    const int wave = threadIdx.x >> 6;
    base[threadIdx.x] = hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    for (int w = 0; w < kBlock / 64; w++) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int q = 0; q < kPerThread; q++) {
        const int64_t i = t0 + (int64_t)q * kBlock + threadIdx.x;
        const bool valid = i < m;
        uint32_t h = 0, p = 0;
        int d = 0;
        if (valid) {
            h = hi_in[i];
            p = pos_in[i];
            d = (int)((h >> shift) & (kDigits - 1));
        }
        // lanes of this wave with the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t ones = __ballot(((d >> b) & 1) != 0);
            peers &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank = (int)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[wave][d] = (int)__popcll(peers);
        __syncthreads();
        if (valid) {
            int at = base[d] + rank;
            for (int w = 0; w < wave; w++) at += wcnt[w][d];
            hi_out[at] = h;
            pos_out[at] = p;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            add += wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = 0;
        }
        base[threadIdx.x] += add;
        __syncthreads();
    }
}

// Runs of equal upper halves, each sorted by its first thread (insertion
// sort: runs are short), then written out as internal node ids by rank.
__global__ void k_prio_runs(int64_t m, const uint32_t* __restrict__ hi, uint32_t* __restrict__ pos,
                            const uint64_t* __restrict__ key, const int32_t* __restrict__ vals,
                            const uint64_t* __restrict__ U_i, const uint32_t* __restrict__ beta_i,
                            const int32_t* __restrict__ orig, int32_t* __restrict__ by_rank) {
    auto less = [&](uint32_t a, uint32_t b) {
        if (key[a] != key[b]) return key[a] < key[b];
        const int32_t x = vals[a], y = vals[b];
        const unsigned __int128 lx = (unsigned __int128)U_i[x] * beta_i[y];
        const unsigned __int128 ly = (unsigned __int128)U_i[y] * beta_i[x];
        if (lx != ly) return lx < ly;
        return orig[x] < orig[y];
    };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        if (i > 0 && hi[i] == hi[i - 1]) continue;  // not the first of its run
        int64_t j = i + 1;
        while (j < m && hi[j] == hi[i]) j++;
        for (int64_t a = i + 1; a < j; a++) {
            const uint32_t x = pos[a];
            int64_t b = a - 1;
            while (b >= i && less(x, pos[b])) {
                pos[b + 1] = pos[b];
                b--;
            }
            pos[b + 1] = x;
        }
        for (int64_t a = i; a < j; a++) by_rank[a] = vals[pos[a]];
    }
}

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t priority_scratch_bytes(int64_t n) {
    const int64_t blocks = (n + kTile - 1) / kTile;
    return al256(sizeof(uint64_t) * n) + 4 * al256(sizeof(uint32_t) * n) + al256(sizeof(int32_t) * n) +
           al256(sizeof(int32_t) * kDigits * (size_t)std::max<int64_t>(blocks, 1)) + al256(sizeof(int32_t)) + 1024;
}

void priority_order(hipStream_t st, int64_t n, int64_t m, uint64_t seed, const uint32_t* beta_c,
                    const int32_t* orig, uint32_t* beta_i, uint64_t* U_i, int32_t* by_rank, void* scratch,
                    size_t scratch_size) {
    if (scratch_size < priority_scratch_bytes(n)) throw HipError{hipErrorOutOfMemory, "priority order scratch"};
    char* p = (char*)scratch;
    auto take = [&](size_t bytes) {
        char* q = p;
        p += al256(bytes);
        return (void*)q;
    };
    uint64_t* key = (uint64_t*)take(sizeof(uint64_t) * n);
    uint32_t* hi0 = (uint32_t*)take(sizeof(uint32_t) * n);
    uint32_t* hi1 = (uint32_t*)take(sizeof(uint32_t) * n);
    uint32_t* pos0 = (uint32_t*)take(sizeof(uint32_t) * n);
    uint32_t* pos1 = (uint32_t*)take(sizeof(uint32_t) * n);
    int32_t* vals = (int32_t*)take(sizeof(int32_t) * n);
    const int64_t blocks = std::max<int64_t>(1, (m + kTile - 1) / kTile);
    int32_t* hist = (int32_t*)take(sizeof(int32_t) * kDigits * (size_t)blocks);
    int32_t* count = (int32_t*)take(sizeof(int32_t));
    fill_u32(st, count, 0u, 1);
    const unsigned gn = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 65536));
    hipLaunchKernelGGL(k_prio_init, dim3(gn), dim3(kBlock), 0, st, n, seed, beta_c, orig, beta_i, U_i, key, hi0, pos0,
                       vals, count);
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const uint32_t*)hi0, m, shift,
                           hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, hist, (int64_t)kDigits * blocks);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const uint32_t*)hi0,
                           (const uint32_t*)pos0, m, shift, (const int32_t*)hist, hi1, pos1);
        std::swap(hi0, hi1);
        std::swap(pos0, pos1);
    }
    const unsigned gm = (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + kBlock - 1) / kBlock, 65536));
    hipLaunchKernelGGL(k_prio_runs, dim3(gm), dim3(kBlock), 0, st, m, (const uint32_t*)hi0, pos0,
                       (const uint64_t*)key, (const int32_t*)vals, (const uint64_t*)U_i, (const uint32_t*)beta_i, orig,
                       by_rank);
    CCG_HIP(hipGetLastError());
}

}  // namespace ccg
