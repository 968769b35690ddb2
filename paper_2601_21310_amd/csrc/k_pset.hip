// The connected set outside S (Eq. 1): P = C(S) \ S written out in canonical order, its
// diagonal H_aa, the order-free fingerprint of P, and the rows H_PS (a in P, columns in S).
//
//   1. every excitation a of every x in S (one wavefront per x, closed-form unranking of
//      the excitation ids as in the PT2 pass) is probed in the hash set of S; those not
//      in S (and, for the heat-bath-screened set of Eq. 14, with |<a|H|x> psi_x| at the
//      threshold or above) are counted per x, and after an exclusive scan written out in
//      excitation order (ballot + mbcnt ranks: no atomics decide a position);
//   2. the candidates are sorted (stable radix sort, k_sort.hip) and duplicates dropped,
//      which leaves P sorted and unique;
//   3. for each a in P (one wavefront per a) its excitations are probed in S again; the
//      hits are the columns of row a of H_PS, with <a|H|x> by the Slater-Condon rules
//      (FP64, stored FP32 like H_SS), counted, scanned, written in excitation order and
//      then sorted by column within the row.
#include <utility>

#include "dnqs_device.h"
#include "dnqs_excite.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kPsThreads = 256;
constexpr int kPsWaves = kPsThreads / kWave;

// The lists a wave wrote to LDS are read by its other lanes: order the accesses.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sort key of a determinant in canonical order (M <= 32: one word).
__device__ __forceinline__ uint64_t det_key(uint64_t a, uint64_t b, int M) { return (a << M) | b; }

// Pass 1: per x, the excitations that are not in S.  FILL = false writes cnt[x];
// FILL = true writes the targets at off[x] on: one sort key per target (M <= 32) or the
// alpha and beta words in two arrays.  With psi given and hb_eps > 0, only the targets
// a with |<a|H|x> psi_x| >= hb_eps sqrt(norm2[0]) (the heat-bath screen of Eq. 14, psi
// normalised); a kept a then appears at least once (from its strongest x).
template <bool FILL>
__global__ __launch_bounds__(kPsThreads) void k_pc_pass(Ham H, const uint64_t *__restrict__ dets, int64_t n,
                                                        DetSet S, const double *__restrict__ psi, double hb_eps,
                                                        const double *__restrict__ norm2, int32_t *__restrict__ cnt,
                                                        const int64_t *__restrict__ off, uint64_t *__restrict__ ka,
                                                        uint64_t *__restrict__ kb) {
    __shared__ uint8_t lists[kPsWaves][4][64];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int M = H.M;
    const EriPacked eri{H.eri_pk};
    const bool screen = psi != nullptr && hb_eps > 0.0;
    const double thr = screen ? hb_eps * sqrt(norm2[0]) : 0.0;
    for (int64_t x = (int64_t)blockIdx.x * kPsWaves + wave; x < n; x += (int64_t)gridDim.x * kPsWaves) {
        const uint64_t xa = dets[2 * x], xb = dets[2 * x + 1];
        const double px = screen ? psi[x] : 1.0;
        wave_build_lists(lists[wave], M, xa, xb);
        wave_lds_sync();
        const ExcLists c = make_exc_lists(lists[wave], M, H.na, H.nb);
        int64_t pos = FILL ? off[x] : 0;
        int count = 0;
        // with the screen, a determinant of zero amplitude couples to nothing
        const int total = (screen && px == 0.0) ? 0 : c.total;
        for (int e0 = 0; e0 < total; e0 += kWave) {
            const int e = e0 + lane;
            bool out = false;
            uint64_t a = xa, b = xb;
            if (e < total) {
                apply_positions(excitation_positions(c, e), a, b);
                out = detset_find(S, a, b) < 0;
                if (out && screen) out = fabs(h_offdiag(H, eri, a, b, xa, xb) * px) >= thr;
            }
            const uint64_t m = __ballot(out);
            if (FILL && out) {
                const int64_t p = pos + mbcnt(m);
                if (M <= 32) {
                    ka[p] = det_key(a, b, M);
                } else {
                    ka[p] = a;
                    kb[p] = b;
                }
            }
            pos += __popcll(m);
            count += __popcll(m);
        }
        if (!FILL && lane == 0) cnt[x] = count;
        wave_lds_sync();
    }
}

// flag[i] = 1 where sorted candidate i starts a run of equal keys
__global__ void k_unique_flag(const uint64_t *__restrict__ ka, const uint64_t *__restrict__ kb,
                              const int32_t *__restrict__ perm, int64_t m, bool two, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    bool first = i == 0;
    if (!first) {
        if (two) {
            const int32_t p = perm[i], q = perm[i - 1];
            first = ka[p] != ka[q] || kb[p] != kb[q];
        } else {
            first = ka[i] != ka[i - 1];
        }
    }
    flag[i] = first ? 1 : 0;
}

// P[k] = the k-th distinct candidate, as {alpha, beta}
__global__ void k_unique_write(const uint64_t *__restrict__ ka, const uint64_t *__restrict__ kb,
                               const int32_t *__restrict__ perm, int64_t m, bool two, int M,
                               const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                               uint64_t *__restrict__ p_dets) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || !flag[i]) return;
    const int64_t k = pos[i];
    if (two) {
        p_dets[2 * k] = ka[perm[i]];
        p_dets[2 * k + 1] = kb[perm[i]];
    } else {
        const uint64_t mask = M == 64 ? ~0ull : ((1ull << M) - 1ull);
        p_dets[2 * k] = ka[i] >> M;
        p_dets[2 * k + 1] = ka[i] & mask;
    }
}

// fp[0] += sum of key_hash(a) (mod 2^64), fp[1] ^= XOR of key_hash(a): order-free
__global__ __launch_bounds__(256) void k_fingerprint(const uint64_t *__restrict__ p, int64_t m,
                                                     unsigned long long *__restrict__ fp) {
    unsigned long long s = 0ull, x = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t h = key_hash(p[2 * i], p[2 * i + 1]);
        s += h;
        x ^= h;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        x ^= __shfl_xor(x, o, 64);
    }
    if (threadIdx.x % kWave == 0) {
        atomicAdd(&fp[0], s);
        atomicXor(&fp[1], x);
    }
}

// H_PS rows.  FILL = false: cnt[a] = number of x in S connected to a; FILL = true: the
// columns and values from off[a] on, in excitation order.
template <bool FILL>
__global__ __launch_bounds__(kPsThreads) void k_hps_pass(Ham H, const uint64_t *__restrict__ pd, int64_t m, DetSet S,
                                                         int32_t *__restrict__ cnt, const int64_t *__restrict__ off,
                                                         int32_t *__restrict__ col, float *__restrict__ val) {
    __shared__ uint8_t lists[kPsWaves][4][64];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const EriPacked eri{H.eri_pk};
    for (int64_t r = (int64_t)blockIdx.x * kPsWaves + wave; r < m; r += (int64_t)gridDim.x * kPsWaves) {
        const uint64_t ra = pd[2 * r], rb = pd[2 * r + 1];
        wave_build_lists(lists[wave], H.M, ra, rb);
        wave_lds_sync();
        const ExcLists c = make_exc_lists(lists[wave], H.M, H.na, H.nb);
        int64_t pos = FILL ? off[r] : 0;
        int count = 0;
        for (int e0 = 0; e0 < c.total; e0 += kWave) {
            const int e = e0 + lane;
            int32_t j = -1;
            uint64_t a = ra, b = rb;
            if (e < c.total) {
                apply_positions(excitation_positions(c, e), a, b);
                j = detset_find(S, a, b);
            }
            const uint64_t hm = __ballot(j >= 0);
            if (FILL && j >= 0) {
                const int64_t p = pos + mbcnt(hm);
                col[p] = j;
                val[p] = (float)h_offdiag(H, eri, ra, rb, a, b);
            }
            pos += __popcll(hm);
            count += __popcll(hm);
        }
        if (!FILL && lane == 0) cnt[r] = count;
        wave_lds_sync();
    }
}

// columns of each row ascending (insertion sort by one thread per row; rows of H_PS
// hold a handful of entries)
__global__ void k_sort_rows(const int64_t *__restrict__ row_ptr, int64_t m, int32_t *__restrict__ col,
                            float *__restrict__ val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int64_t b = row_ptr[r], e = row_ptr[r + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t c = col[i];
        const float v = val[i];
        int64_t j = i - 1;
        while (j >= b && col[j] > c) {
            col[j + 1] = col[j];
            val[j + 1] = val[j];
            --j;
        }
        col[j + 1] = c;
        val[j + 1] = v;
    }
}

// row_ptr[r] = off[r] (r < m), row_ptr[m] = total
__global__ void k_rows_from_offsets(const int64_t *__restrict__ off, int64_t m, const int64_t *__restrict__ total,
                                    int64_t *__restrict__ row_ptr) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) row_ptr[r] = off[r];
    if (r == m) row_ptr[m] = *total;
}

static unsigned grid_for(int64_t items, int per_block, unsigned cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_pc_pass(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const DetSet &S,
                    const double *psi, double hb_eps, const double *norm2, int32_t *cnt, const int64_t *off,
                    uint64_t *ka, uint64_t *kb, bool fill) {
    const dim3 g(grid_for(n, kPsWaves, 65535u)), b(kPsThreads);
    if (fill)
        hipLaunchKernelGGL(k_pc_pass<true>, g, b, 0, st, H, dets, n, S, psi, hb_eps, norm2, cnt, off, ka, kb);
    else
        hipLaunchKernelGGL(k_pc_pass<false>, g, b, 0, st, H, dets, n, S, psi, hb_eps, norm2, cnt, off, ka, kb);
}

// Sort key of a selection by |psi|: descending log|psi| (order-preserving bits of the
// double, inverted; sign 0 / -inf last), taken for the determinants in the order perm.
__global__ void k_topk_key(const double *__restrict__ la, const int8_t *__restrict__ sg,
                           const int32_t *__restrict__ perm, int64_t n, uint64_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    double v = la[j];
    if ((sg && sg[j] == 0) || !(v > -INFINITY)) v = -INFINITY;
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t asc = (u >> 63) ? ~u : (u | (1ull << 63));
    key[i] = ~asc;
}

void launch_topk_key(hipStream_t st, const double *la, const int8_t *sg, const int32_t *perm, int64_t n,
                     uint64_t *key) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_topk_key, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, la, sg, perm, n, key);
}

void launch_unique(hipStream_t st, const uint64_t *ka, const uint64_t *kb, const int32_t *perm, int64_t m, bool two,
                   int M, int32_t *flag, int64_t *pos, int64_t *bsum, int64_t *total, uint64_t *p_dets, bool write) {
    if (m <= 0) return;
    const dim3 g((unsigned)((m + 255) / 256)), b(256);
    if (!write) {
        hipLaunchKernelGGL(k_unique_flag, g, b, 0, st, ka, kb, perm, m, two, flag);
        launch_exclusive_scan(st, flag, m, pos, bsum, total);
    } else {
        hipLaunchKernelGGL(k_unique_write, g, b, 0, st, ka, kb, perm, m, two, M, flag, pos, p_dets);
    }
}

void launch_fingerprint(hipStream_t st, const uint64_t *p, int64_t m, unsigned long long *fp) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_fingerprint, dim3(grid_for(m, 256, 1024u)), dim3(256), 0, st, p, m, fp);
}

void launch_hps_pass(hipStream_t st, const Ham &H, const uint64_t *pd, int64_t m, const DetSet &S, int32_t *cnt,
                     const int64_t *off, int32_t *col, float *val, bool fill) {
    if (m <= 0) return;
    const dim3 g(grid_for(m, kPsWaves, 65535u)), b(kPsThreads);
    if (fill)
        hipLaunchKernelGGL(k_hps_pass<true>, g, b, 0, st, H, pd, m, S, cnt, off, col, val);
    else
        hipLaunchKernelGGL(k_hps_pass<false>, g, b, 0, st, H, pd, m, S, cnt, off, col, val);
}

void launch_row_ptr_from_offsets(hipStream_t st, const int64_t *off, int64_t m, const int64_t *total,
                                 int64_t *row_ptr) {
    hipLaunchKernelGGL(k_rows_from_offsets, dim3((unsigned)((m + 1 + 255) / 256)), dim3(256), 0, st, off, m, total,
                       row_ptr);
}

void launch_rows_finish(hipStream_t st, const int64_t *off, int64_t m, const int64_t *total, int64_t *row_ptr,
                        int32_t *col, float *val) {
    const dim3 g((unsigned)((m + 1 + 255) / 256)), b(256);
    hipLaunchKernelGGL(k_rows_from_offsets, g, b, 0, st, off, m, total, row_ptr);
    if (m > 0) hipLaunchKernelGGL(k_sort_rows, dim3((unsigned)((m + 255) / 256)), b, 0, st, row_ptr, m, col, val);
}

}  // namespace dnqs
