// Hamiltonian-side kernels: integral staging, hash set of S, validation, the FP64
// diagonal, and the H_SS builder.
//
// H_SS builder.  S is small enough (|S| <= a few 1e6) that comparing every pair of
// determinants is cheaper than probing a hash table with every excitation: a pair
// test is two 64-bit XORs, two popcounts and a compare (about 10 VALU ops), while the
// excitation route needs |S| * n_exc probes of a random 16-byte slot (n_exc = 30,723
// at M = 28, 7+7).  Each workgroup owns a block of RB rows; each of its waves sweeps
// its own contiguous range of columns y, 64 at a time (one y per lane, coalesced
// 16-byte loads), and tests every row of the block against them.  The row dets are
// wave-uniform (scalar loads).  Hits are compacted in lane order with ballot/mbcnt,
// so each row's columns come out in ascending order without a sort:
//   pass 1 counts hits per (row, column range), an exclusive scan gives offsets,
//   pass 2 repeats the sweep and writes the columns,
//   pass 3 evaluates the couplings, one wave per row over its entries.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

// ------------------------------------------------------------------ integral staging
__global__ void k_stage_integrals(int M, const double *__restrict__ eri64, float *__restrict__ eri32,
                                  double *__restrict__ J, double *__restrict__ K) {
    size_t n4 = (size_t)M * M * M * M;
    size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = tid; i < n4; i += stride) eri32[i] = (float)eri64[i];
    for (size_t i = tid; i < (size_t)M * M; i += stride) {
        int p = (int)(i / M), q = (int)(i % M);
        J[i] = eri64[eri_index(M, p, p, q, q)];
        K[i] = eri64[eri_index(M, p, q, q, p)];
    }
}

// packed[tri(tri(p,q), tri(r,s))] = (pq|rs) for the canonical p>=q, r>=s, pq>=rs
__global__ void k_pack_eri(int M, const double *__restrict__ eri64, double *__restrict__ pk) {
    size_t n4 = (size_t)M * M * M * M;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(i % M), r = (int)((i / M) % M), q = (int)((i / M / M) % M), p = (int)(i / M / M / M);
        if (p < q || r < s) continue;
        const int pq = tri_index(p, q), rs = tri_index(r, s);
        if (pq < rs) continue;
        pk[tri_index(pq, rs)] = eri64[i];
    }
}

size_t packed_eri_size(int M) {
    size_t np = (size_t)M * (M + 1) / 2;
    return np * (np + 1) / 2;
}

void launch_pack_eri(hipStream_t st, int M, const double *eri64, double *pk) {
    size_t n4 = (size_t)M * M * M * M;
    int blocks = (int)((n4 + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pack_eri, dim3(blocks), dim3(256), 0, st, M, eri64, pk);
}

void launch_stage_integrals(hipStream_t st, int M, const double *eri64, float *eri32, double *J, double *K) {
    size_t n4 = (size_t)M * M * M * M;
    int blocks = (int)((n4 + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_stage_integrals, dim3(blocks), dim3(256), 0, st, M, eri64, eri32, J, K);
}

// ------------------------------------------------------------------ validation
// err[0] |= 1: wrong electron count; 2: not strictly ascending; 4: bits above M.
__global__ void k_validate_dets(const uint64_t *__restrict__ dets, int64_t n, int M, int na, int nb, int check_order,
                                int *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t a = dets[2 * i], b = dets[2 * i + 1];
    int e = 0;
    if (popc64(a) != na || popc64(b) != nb) e |= 1;
    if (M < 64 && ((a >> M) != 0 || (b >> M) != 0)) e |= 4;
    if (check_order && i > 0) {
        uint64_t pa = dets[2 * i - 2], pb = dets[2 * i - 1];
        if (!(pa < a || (pa == a && pb < b))) e |= 2;
    }
    if (e) atomicOr(err, e);
}

void launch_validate_dets(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, int check_order,
                          int *err) {
    hipLaunchKernelGGL(k_validate_dets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dets, n, M, na, nb,
                       check_order, err);
}

// ------------------------------------------------------------------ hash set of S
__global__ void k_fill_u64(uint64_t *__restrict__ p, size_t n, uint64_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

void launch_fill_u64(hipStream_t st, uint64_t *p, size_t n, uint64_t v) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

__global__ void k_detset_insert(const uint64_t *__restrict__ dets, int64_t n, unsigned long long *keys,
                                int32_t *__restrict__ idx, uint64_t mask) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t a = dets[2 * i], b = dets[2 * i + 1];
    uint64_t h = key_hash(a, b) & mask;
    for (;;) {
        unsigned long long prev = atomicCAS(&keys[2 * h], (unsigned long long)kEmptyKey, (unsigned long long)a);
        if (prev == kEmptyKey) {
            keys[2 * h + 1] = b;
            idx[h] = (int32_t)i;
            return;
        }
        h = (h + 1) & mask;
    }
}

void launch_detset_insert(hipStream_t st, const uint64_t *dets, int64_t n, uint64_t *keys, int32_t *idx,
                          uint64_t mask) {
    hipLaunchKernelGGL(k_detset_insert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dets, n,
                       (unsigned long long *)keys, idx, mask);
}

// ------------------------------------------------------------------ diagonal
__global__ void k_diag(Ham H, const uint64_t *__restrict__ dets, int64_t n, double *__restrict__ diag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    diag[i] = h_diag(H, dets[2 * i], dets[2 * i + 1]);
}

void launch_diag(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, double *diag) {
    hipLaunchKernelGGL(k_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, H, dets, n, diag);
}

// ------------------------------------------------------------------ H_SS all-pairs
constexpr int kRowBlock = 256;   // rows per workgroup
constexpr int kWavesPerBlock = 4;

// y range of column sub-range `sub` out of nsub, each a multiple of 64 long
__device__ __forceinline__ void sub_range(int64_t n, int nsub, int sub, int64_t &y0, int64_t &y1) {
    int64_t len = (n + nsub - 1) / nsub;
    len = (len + 63) & ~(int64_t)63;
    y0 = (int64_t)sub * len;
    y1 = y0 + len;
    if (y0 > n) y0 = n;
    if (y1 > n) y1 = n;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_hss_pairs(Ham H, const uint64_t *__restrict__ dets, int64_t n, int nsub,
                                                   int32_t *__restrict__ counts, const int64_t *__restrict__ offs,
                                                   int32_t *__restrict__ col, float *__restrict__ val) {
    __shared__ int64_t cursor[kWavesPerBlock][kRowBlock];
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t row0 = (int64_t)blockIdx.x * kRowBlock;
    const int nrows = (int)((n - row0) < kRowBlock ? (n - row0) : kRowBlock);
    const int sub = blockIdx.y * kWavesPerBlock + wave;
    int64_t y0, y1;
    sub_range(n, nsub, sub, y0, y1);
    for (int r = lane; r < nrows; r += kWave)
        cursor[wave][r] = FILL ? offs[(row0 + r) * nsub + sub] : 0;
    __syncthreads();
    for (int64_t yb = y0; yb < y1; yb += kWave) {
        const int64_t y = yb + lane;
        const bool valid = y < y1;
        const uint64_t ya = valid ? dets[2 * y] : 0ull;
        const uint64_t ybb = valid ? dets[2 * y + 1] : 0ull;
        for (int r = 0; r < nrows; ++r) {
            const int64_t xr = row0 + r;
            const uint64_t xa = dets[2 * xr];
            const uint64_t xb = dets[2 * xr + 1];
            const int d = popc64(xa ^ ya) + popc64(xb ^ ybb);
            const bool hit = valid && (d == 2 || d == 4);
            const uint64_t m = ballot(hit);
            if (m) {
                if (FILL) {
                    if (hit) col[cursor[wave][r] + mbcnt(m)] = (int32_t)y;
                }
                if (lane == 0) cursor[wave][r] += __popcll(m);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    if (!FILL) {
        __builtin_amdgcn_wave_barrier();
        for (int r = lane; r < nrows; r += kWave) counts[(row0 + r) * nsub + sub] = (int32_t)cursor[wave][r];
    }
}

int hss_nsub(int64_t n) {
    // enough workgroups to fill 256 CUs several times over
    int64_t row_blocks = (n + kRowBlock - 1) / kRowBlock;
    int splits = 1;
    while (row_blocks * splits < 2048 && splits < 64 && (int64_t)splits * kWavesPerBlock * 64 * 2 < n) splits *= 2;
    return splits * kWavesPerBlock;
}

void launch_hss_count(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, int nsub, int32_t *counts) {
    dim3 grid((unsigned)((n + kRowBlock - 1) / kRowBlock), (unsigned)(nsub / kWavesPerBlock));
    hipLaunchKernelGGL(k_hss_pairs<false>, grid, dim3(256), 0, st, H, dets, n, nsub, counts, nullptr, nullptr,
                       nullptr);
}

void launch_hss_fill(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, int nsub, const int64_t *offs,
                     int32_t *col, float *val) {
    dim3 grid((unsigned)((n + kRowBlock - 1) / kRowBlock), (unsigned)(nsub / kWavesPerBlock));
    hipLaunchKernelGGL(k_hss_pairs<true>, grid, dim3(256), 0, st, H, dets, n, nsub, nullptr, offs, col, val);
}

// Values of H_SS after the structure is known: one wave per row, its lanes over the
// row's entries, so that every lane of a wave evaluates a coupling (in the sweep only the
// one or two lanes of a hit would be active).  The row's determinant is wave-uniform.
__global__ __launch_bounds__(256) void k_hss_values(Ham H, const uint64_t *__restrict__ dets, int64_t n,
                                                    const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, float *__restrict__ val) {
    const int lane = threadIdx.x % kWave;
    const int64_t x = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (x >= n) return;
    const uint64_t xa = dets[2 * x], xb = dets[2 * x + 1];
    const int64_t b = row_ptr[x], e = row_ptr[x + 1];
    const EriPacked eri{H.eri_pk};
    for (int64_t j = b + lane; j < e; j += kWave) {
        const int64_t y = col[j];
        val[j] = (float)h_offdiag(H, eri, xa, xb, dets[2 * y], dets[2 * y + 1]);
    }
}

void launch_hss_values(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const int64_t *row_ptr,
                       const int32_t *col, float *val) {
    hipLaunchKernelGGL(k_hss_values, dim3((unsigned)((n * kWave + 255) / 256)), dim3(256), 0, st, H, dets, n, row_ptr,
                       col, val);
}

// row_ptr[i] = offs[i*nsub], row_ptr[n] = total
__global__ void k_row_ptr(const int64_t *__restrict__ offs, int64_t n, int nsub, int64_t total,
                          int64_t *__restrict__ row_ptr) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) row_ptr[i] = offs[i * nsub];
    if (i == n) row_ptr[n] = total;
}

void launch_row_ptr(hipStream_t st, const int64_t *offs, int64_t n, int nsub, int64_t total, int64_t *row_ptr) {
    hipLaunchKernelGGL(k_row_ptr, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, offs, n, nsub, total,
                       row_ptr);
}

// ------------------------------------------------------------------ exclusive scan (int32 -> int64)
// Three phases: per-block sums, a single-block scan of the block sums, per-block scan.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;  // items per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wave] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        if (w < wave) pre += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                            int64_t *__restrict__ bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_bsums(int64_t *__restrict__ bsum, int64_t nb,
                                                           int64_t *__restrict__ total) {
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                           const int64_t *__restrict__ bsum,
                                                           int64_t *__restrict__ out) {
    // each thread owns kScanItems consecutive items
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t loc[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        loc[k] = i < n ? in[i] : 0;
        s += loc[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += loc[k];
    }
}

int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

void launch_exclusive_scan(hipStream_t st, const int32_t *in, int64_t n, int64_t *out, int64_t *bsum,
                           int64_t *total) {
    int64_t nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanBlock), 0, st, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum, out);
}

}  // namespace dnqs
