// Stable least-significant-digit radix sort of 64-bit keys carrying a 32-bit value,
// 8-bit digits, deterministic (no atomics decide a position).
//
// Used where the library must return a set in canonical order or pick the top entries
// of a list: the sorted unique P = C(S) \ S (Eq. 1) and its H_PS rows, the exported keys
// of the PT2 reduce, and the top-|psi| selection of the outer loop.
//
// One pass per digit:
//   count    one workgroup per tile of kSortTile keys: a 256-bin histogram of the
//            digit (LDS adds: a count does not depend on their order), written
//            digit-major, counts[d * nblocks + block];
//   scan     exclusive scan of the counts (launch_exclusive_scan): the output position
//            of the first key with digit d of each tile;
//   scatter  the tile is walked in order, 256 keys at a time; a key's rank among the
//            keys of its digit is the number of equal digits in earlier waves of the
//            same step (per-wave digit counts in LDS) plus those in lower lanes of its
//            own wave (eight ballots give the lanes whose digit equals this lane's), so
//            equal digits keep their input order.
#include <utility>

#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kSortThreads = 256;
constexpr int kSortPer = 16;
constexpr int kSortTile = kSortThreads * kSortPer;
constexpr int kSortWaves = kSortThreads / kWave;

int64_t sort_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                             int64_t nblk, int32_t *__restrict__ counts) {
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int k = 0; k < kSortPer; ++k) {
        const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = (int32_t)hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t *__restrict__ kin,
                                                               const int32_t *__restrict__ vin, int64_t n, int shift,
                                                               int64_t nblk, const int64_t *__restrict__ offs,
                                                               uint64_t *__restrict__ kout,
                                                               int32_t *__restrict__ vout) {
    __shared__ int64_t run[256];
    __shared__ uint32_t wcnt[kSortWaves][256];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    run[t] = offs[(int64_t)t * nblk + blockIdx.x];
    for (int w = 0; w < kSortWaves; ++w) wcnt[w][t] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int k = 0; k < kSortPer; ++k) {
        const int64_t i = base + (int64_t)k * kSortThreads + t;
        const bool have = i < n;
        uint64_t key = 0ull;
        int32_t val = 0;
        uint32_t d = 256u;  // no key: a digit no real key has
        if (have) {
            key = kin[i];
            val = vin[i];
            d = (uint32_t)(key >> shift) & 255u;
        }
        // lanes of this wave holding the same digit (absent lanes match no present lane)
        uint64_t peers = __ballot(have);
        if (!have) peers = ~peers;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (have && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (have) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            const int64_t pos = run[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            tot += wcnt[w][t];
            wcnt[w][t] = 0u;
        }
        run[t] += tot;
        __syncthreads();
    }
}

__global__ void k_iota_i32(int32_t *__restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

void launch_iota_i32(hipStream_t st, int32_t *v, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, n);
}

size_t sort_scratch_counts(int64_t n) { return (size_t)256 * (size_t)sort_blocks(n); }

void launch_radix_sort(hipStream_t st, uint64_t *keys, int32_t *vals, int64_t n, int bits, const SortScratch &w) {
    if (n <= 1 || bits <= 0) return;
    const int64_t nblk = sort_blocks(n);
    uint64_t *ka = keys, *kb = w.keys;
    int32_t *va = vals, *vb = w.vals;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        hipLaunchKernelGGL(k_sort_count, dim3((unsigned)nblk), dim3(kSortThreads), 0, st, ka, n, shift, nblk,
                           w.counts);
        launch_exclusive_scan(st, w.counts, 256 * nblk, w.offs, w.bsum, w.total);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nblk), dim3(kSortThreads), 0, st, ka, va, n, shift, nblk,
                           w.offs, kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (passes & 1) {
        (void)hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    }
}

// ------------------------------------------------------------------ determinant keys
// Canonical order of determinants is ascending (alpha, beta) as unsigned integers.  For
// M <= 32 one 64-bit sort key (alpha << M | beta) orders them; otherwise two stable
// sorts (by beta, then by alpha) do.
__global__ void k_det_sortkey(const uint64_t *__restrict__ dets, const int32_t *__restrict__ perm, int64_t n, int M,
                              int word, uint64_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm ? perm[i] : i;
    if (word < 0)
        key[i] = (dets[2 * j] << M) | dets[2 * j + 1];
    else
        key[i] = dets[2 * j + word];
}

__global__ void k_gather_u64(const uint64_t *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                             uint64_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

void launch_gather_u64(hipStream_t st, const uint64_t *src, const int32_t *perm, int64_t n, uint64_t *dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, n, dst);
}

// dst[i] = src[perm[i]] for records of `words` 64-bit words
__global__ void k_permute_words(const uint64_t *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                                int words, uint64_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    for (int w = 0; w < words; ++w) dst[i * words + w] = src[j * words + w];
}

void launch_permute_words(hipStream_t st, const uint64_t *src, const int32_t *perm, int64_t n, int words,
                          uint64_t *dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_permute_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, n, words,
                       dst);
}

void launch_sort_dets(hipStream_t st, const uint64_t *dets, int64_t n, int M, int32_t *perm, uint64_t *key,
                      const SortScratch &w) {
    if (n <= 0) return;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    launch_iota_i32(st, perm, n);
    if (M <= 32) {
        hipLaunchKernelGGL(k_det_sortkey, g, b, 0, st, dets, (const int32_t *)nullptr, n, M, -1, key);
        launch_radix_sort(st, key, perm, n, 2 * M, w);
        return;
    }
    hipLaunchKernelGGL(k_det_sortkey, g, b, 0, st, dets, (const int32_t *)nullptr, n, M, 1, key);
    launch_radix_sort(st, key, perm, n, M, w);
    hipLaunchKernelGGL(k_det_sortkey, g, b, 0, st, dets, perm, n, M, 0, key);
    launch_radix_sort(st, key, perm, n, M, w);
}

}  // namespace dnqs
