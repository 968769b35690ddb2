// Epstein-Nesbet PT2 (Eq. 13), external sum, by partitioning instead of global atomics.
//
// The reduce-by-key w_a = sum_x H_ax psi_x runs over |S| * n_exc pairs (3.1e9 at
// M = 28, 7+7, |S| = 1e5) into ~9e8 unique keys: only ~3.4 pairs per key, so an
// on-chip pre-aggregation saves little and a global hash table is bound by atomic
// throughput.  Instead the pairs are streamed through two hash partitions into
// sub-buckets small enough to reduce in LDS:
//
//   L1  one wave per determinant enumerates its excitations; each pair is written as
//       an 8-byte descriptor [x index: 24 bits | four 7-bit flipped spin-orbital
//       positions: 28 bits | the 12 hash bits after the L1 bits: 12 bits] to one of K1
//       buckets by the top bits of the target's key hash.  A count pass
//       and an exclusive scan in bucket-major order give every workgroup a private,
//       contiguous run per bucket (no global atomics; writes of a run coalesce in L2).
//   L2  each L1 bucket is cut into chunks; the same count -> scan -> scatter splits it
//       into K2 sub-buckets by the hash bits carried in the descriptor (a pure stream:
//       no gathers, no rehashing).
//   R   one workgroup per sub-bucket decodes each descriptor (x XOR positions),
//       recomputes H_ax exactly (FP64 integrals), accumulates w_a in an LDS hash table
//       (64-bit CAS + FP64 add in LDS), then for every key not in S adds
//       w_a^2 / (E - H_aa) (FP64) to its partial sum.  Membership in S is known
//       without probing the global hash set: the members of S that hash into the
//       sub-bucket (grouped once per call by k_s_sub_*) are inserted first and
//       flagged.  H_aa is the diagonal rule over a table of h_pp and
//       V(p,q) = J_pq - d_s K_pq staged in LDS (M <= 32).  A sub-bucket whose keys do not
//       fit the table raises a flag and the host repeats L2 + R with twice as many
//       sub-buckets.
#include "dnqs_device.h"
#include "dnqs_excite.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kL1Waves = 4;
constexpr int kL1XPerWave = 4;
constexpr int kL1XPerGroup = kL1Waves * kL1XPerWave;
constexpr int kMaxK1 = 1024;
constexpr int kMaxK2 = 4096;
constexpr int kRedThreads = 512;
constexpr int kRedTab = 4096;  // LDS hash-table slots per sub-bucket

__device__ __forceinline__ uint32_t l1_bucket(uint64_t h, int s1) { return s1 ? (uint32_t)(h >> (64 - s1)) : 0u; }

__device__ __forceinline__ uint32_t l2_bucket(uint64_t h, int s1, int s2) {
    return s2 ? (uint32_t)((h << s1) >> (64 - s2)) : 0u;
}

int64_t pt2_l1_groups(int64_t n) { return (n + kL1XPerGroup - 1) / kL1XPerGroup; }

constexpr int kDescXBits = 24;
constexpr int kDescHashBits = 12;

__device__ __forceinline__ uint64_t make_desc(int64_t x, uint32_t pos, uint64_t h, int s1) {
    const uint64_t l2b = (h << s1) >> (64 - kDescHashBits);
    return (uint64_t)x | ((uint64_t)pos << kDescXBits) | (l2b << (kDescXBits + 28));
}
__device__ __forceinline__ int64_t desc_x(uint64_t d) { return (int64_t)(d & ((1ull << kDescXBits) - 1)); }
__device__ __forceinline__ uint32_t desc_pos(uint64_t d) { return (uint32_t)((d >> kDescXBits) & 0xfffffffull); }
__device__ __forceinline__ uint32_t desc_sub(uint64_t d, int s2) {
    return s2 ? (uint32_t)(d >> (64 - s2)) : 0u;
}

int pt2_max_dets() { return 1 << kDescXBits; }

// ------------------------------------------------------------------ L1
template <bool FILL, bool PACKED>
__global__ __launch_bounds__(256) void k_pt2_l1(Ham H, const uint64_t *__restrict__ dets, int64_t n,
                                                const double *__restrict__ psi, int s1, int64_t nwg,
                                                uint32_t *__restrict__ counts, const int64_t *__restrict__ offs,
                                                uint64_t *__restrict__ desc) {
    __shared__ uint8_t lists[kL1Waves][4][64];
    __shared__ uint32_t cur[kMaxK1];
    __shared__ int64_t base[FILL ? kMaxK1 : 1];
    const int K1 = 1 << s1;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t wg = blockIdx.x;
    for (int b = threadIdx.x; b < K1; b += blockDim.x) {
        cur[b] = 0u;
        if (FILL) base[b] = offs[(int64_t)b * nwg + wg];
    }
    for (int k = 0; k < kL1XPerWave; ++k) {
        const int64_t x = wg * kL1XPerGroup + (int64_t)wave * kL1XPerWave + k;
        const bool live = x < n && psi[x] != 0.0;
        const uint64_t xa = live ? dets[2 * x] : 0ull, xb = live ? dets[2 * x + 1] : 0ull;
        __syncthreads();  // previous x's lists are no longer read
        wave_build_lists(lists[wave], H.M, xa, xb);
        __syncthreads();
        if (!live) continue;
        const ExcLists c = make_exc_lists(lists[wave], H.M, H.na, H.nb);
        for (int64_t e = lane; e < c.total; e += kWave) {
            const uint32_t pos = excitation_positions(c, e);
            uint64_t ka = xa, kb = xb;
            apply_positions(pos, ka, kb);
            const uint64_t h = target_hash<PACKED>(ka, kb);
            const uint32_t b = l1_bucket(h, s1);
            const uint32_t r = atomicAdd(&cur[b], 1u);
            if (FILL) desc[base[b] + r] = make_desc(x, pos, h, s1);
        }
    }
    if (!FILL) {
        __syncthreads();
        for (int b = threadIdx.x; b < K1; b += blockDim.x) counts[wg * K1 + b] = cur[b];
    }
}

void launch_pt2_l1(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const double *psi, int s1,
                   int64_t nwg, uint32_t *counts, const int64_t *offs, uint64_t *desc, bool fill, bool packed) {
    dim3 grid((unsigned)nwg), blk(kL1Waves * kWave);
    if (fill) {
        if (packed)
            hipLaunchKernelGGL((k_pt2_l1<true, true>), grid, blk, 0, st, H, dets, n, psi, s1, nwg, counts, offs, desc);
        else
            hipLaunchKernelGGL((k_pt2_l1<true, false>), grid, blk, 0, st, H, dets, n, psi, s1, nwg, counts, offs, desc);
    } else {
        if (packed)
            hipLaunchKernelGGL((k_pt2_l1<false, true>), grid, blk, 0, st, H, dets, n, psi, s1, nwg, counts, offs, desc);
        else
            hipLaunchKernelGGL((k_pt2_l1<false, false>), grid, blk, 0, st, H, dets, n, psi, s1, nwg, counts, offs,
                               desc);
    }
}

// out[c * R + r] = in[r * C + c]
__global__ void k_transpose_u32(const uint32_t *__restrict__ in, int64_t R, int64_t C, int32_t *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * C) return;
    const int64_t r = i / C, c = i % C;
    out[c * R + r] = (int32_t)in[i];
}

void launch_transpose_u32(hipStream_t st, const uint32_t *in, int64_t R, int64_t C, int32_t *out) {
    hipLaunchKernelGGL(k_transpose_u32, dim3((unsigned)((R * C + 255) / 256)), dim3(256), 0, st, in, R, C, out);
}

// bucket_start[b] = offs[b * nwg] (b < K1), bucket_start[K1] = total
__global__ void k_gather_starts(const int64_t *__restrict__ offs, int K, int64_t stride, const int64_t *__restrict__ total,
                                int64_t *__restrict__ starts) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < K) starts[b] = offs[(int64_t)b * stride];
    if (b == K) starts[K] = *total;
}

void launch_gather_starts(hipStream_t st, const int64_t *offs, int K, int64_t stride, const int64_t *total,
                          int64_t *starts) {
    hipLaunchKernelGGL(k_gather_starts, dim3((K + 1 + 255) / 256), dim3(256), 0, st, offs, K, stride, total, starts);
}

// ------------------------------------------------------------------ L2
// Chunk c covers desc1[start, start + len) inside L1 bucket b1; the L2 counts of the
// chunks of bucket b1 are laid out as [b2][chunk] after position cb0 * K2, so that one
// exclusive scan orders the output by (b1, b2, chunk).
__device__ __forceinline__ int64_t l2_tpos(const PT2Chunk &ch, int64_t c, int b2, int K2) {
    return ch.cb0 * (int64_t)K2 + (int64_t)b2 * ch.nc + (c - ch.cb0);
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_pt2_l2(const uint64_t *__restrict__ desc1, const PT2Chunk *__restrict__ chunks,
                                                int s2, uint32_t *__restrict__ counts, const int64_t *__restrict__ offs,
                                                uint64_t *__restrict__ desc2) {
    __shared__ uint32_t cur[kMaxK2];
    __shared__ int64_t base[FILL ? kMaxK2 : 1];
    const int K2 = 1 << s2;
    const int64_t c = blockIdx.x;
    const PT2Chunk ch = chunks[c];
    for (int b = threadIdx.x; b < K2; b += blockDim.x) {
        cur[b] = 0u;
        if (FILL) base[b] = offs[l2_tpos(ch, c, b, K2)];
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < ch.len; i += blockDim.x) {
        const uint64_t d = desc1[ch.start + i];
        const uint32_t b = desc_sub(d, s2);
        const uint32_t r = atomicAdd(&cur[b], 1u);
        if (FILL) desc2[base[b] + r] = d;
    }
    if (!FILL) {
        __syncthreads();
        for (int b = threadIdx.x; b < K2; b += blockDim.x) counts[c * K2 + b] = cur[b];
    }
}

void launch_pt2_l2(hipStream_t st, const uint64_t *desc1, const PT2Chunk *chunks, int64_t nchunk, int s2,
                   uint32_t *counts, const int64_t *offs, uint64_t *desc2, bool fill) {
    dim3 grid((unsigned)nchunk), blk(256);
    if (fill)
        hipLaunchKernelGGL(k_pt2_l2<true>, grid, blk, 0, st, desc1, chunks, s2, counts, offs, desc2);
    else
        hipLaunchKernelGGL(k_pt2_l2<false>, grid, blk, 0, st, desc1, chunks, s2, counts, offs, desc2);
}

// counts[c * K2 + b2] -> out[l2_tpos(c, b2)]
__global__ void k_l2_transpose(const uint32_t *__restrict__ counts, const PT2Chunk *__restrict__ chunks, int64_t nchunk,
                               int K2, int32_t *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchunk * K2) return;
    const int64_t c = i / K2;
    const int b = (int)(i % K2);
    out[l2_tpos(chunks[c], c, b, K2)] = (int32_t)counts[i];
}

void launch_l2_transpose(hipStream_t st, const uint32_t *counts, const PT2Chunk *chunks, int64_t nchunk, int K2,
                         int32_t *out) {
    hipLaunchKernelGGL(k_l2_transpose, dim3((unsigned)((nchunk * K2 + 255) / 256)), dim3(256), 0, st, counts, chunks,
                       nchunk, K2, out);
}

// sub-bucket starts: sb[b1 * K2 + b2]; empty L1 buckets take their L1 start
__global__ void k_sub_starts(const int64_t *__restrict__ offs2, const int64_t *__restrict__ bstart,
                             const int64_t *__restrict__ bcb0, const int64_t *__restrict__ bnc, int K1, int K2,
                             int64_t *__restrict__ sb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ns = (int64_t)K1 * K2;
    if (i > ns) return;
    if (i == ns) {
        sb[ns] = bstart[K1];
        return;
    }
    const int b1 = (int)(i / K2), b2 = (int)(i % K2);
    sb[i] = bnc[b1] > 0 ? offs2[bcb0[b1] * K2 + (int64_t)b2 * bnc[b1]] : bstart[b1];
}

void launch_sub_starts(hipStream_t st, const int64_t *offs2, const int64_t *bstart, const int64_t *bcb0,
                       const int64_t *bnc, int K1, int K2, int64_t *sb) {
    int64_t ns = (int64_t)K1 * K2 + 1;
    hipLaunchKernelGGL(k_sub_starts, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, offs2, bstart, bcb0, bnc, K1,
                       K2, sb);
}

// ------------------------------------------------------------------ reduce
__device__ inline void red_block(double &s, double &mn, double &np, double &nt) {
    __shared__ double sh[4][kRedThreads / kWave];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        np += __shfl_xor(np, o, 64);
        nt += __shfl_xor(nt, o, 64);
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) {
        sh[0][wave] = s;
        sh[1][wave] = mn;
        sh[2][wave] = np;
        sh[3][wave] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
            sh[0][0] += sh[0][w];
            sh[1][0] = fmin(sh[1][0], sh[1][w]);
            sh[2][0] += sh[2][w];
            sh[3][0] += sh[3][w];
        }
        s = sh[0][0];
        mn = sh[1][0];
        np = sh[2][0];
        nt = sh[3][0];
    }
}

// Coulomb minus same-spin exchange between spin-orbitals s, t (alpha s < M, beta M + p)
__device__ __forceinline__ double v_so(const Ham &H, int s, int t) {
    const int M = H.M;
    const bool sa = s < M, ta = t < M;
    const int i = sa ? s : s - M, j = ta ? t : t - M;
    double v = H.J[i * M + j];
    if (sa == ta) v -= H.K[i * M + j];
    return v;
}

// Diagonal table for M <= 32: vt[p] = h_pp for the 2M spin-orbitals, then
// vt[2M + q(q-1)/2 + p] = V(p, q) for p < q, so that
// H_aa = E_core + sum_{q in a} (vt[q] + sum_{p in a, p < q} vt[2M + q(q-1)/2 + p]).
// 2M + M(2M-1) doubles: 12.8 KB at M = 28, 16.6 KB at M = 32.

__global__ void k_diag_table(Ham H, double *__restrict__ vt) {
    const int No = 2 * H.M;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < No) {
        const int sp = t < H.M ? t : t - H.M;
        vt[t] = H.h64[sp * H.M + sp];
        return;
    }
    const int u = t - No;
    if (u >= No * (No - 1) / 2) return;
    int q = (int)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
    while (q * (q - 1) / 2 > u) --q;
    while ((q + 1) * q / 2 <= u) ++q;
    const int p = u - q * (q - 1) / 2;
    vt[t] = v_so(H, p, q);
}

int pt2_diag_table_size(int M) { return 2 * M + (2 * M) * (2 * M - 1) / 2; }

void launch_diag_table(hipStream_t st, const Ham &H, double *vt) {
    const int total = pt2_diag_table_size(H.M);
    hipLaunchKernelGGL(k_diag_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, H, vt);
}

// ------------------------------------------------------------------ S by sub-bucket
// The keys of S grouped by the sub-bucket their hash falls in (top sbits bits, the
// concatenated L1 and L2 bucket indices), so that each reduce workgroup can mark the
// members of S among its keys without probing the global hash set.
template <bool PACKED>
__device__ __forceinline__ int64_t s_sub(uint64_t a, uint64_t b, int sbits) {
    return sbits ? (int64_t)(target_hash<PACKED>(a, b) >> (64 - sbits)) : 0;
}

template <bool PACKED>
__global__ void k_s_sub_count(const uint64_t *__restrict__ dets, int64_t n, int sbits, int32_t *__restrict__ cnt) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    atomicAdd(&cnt[s_sub<PACKED>(dets[2 * x], dets[2 * x + 1], sbits)], 1);
}

template <bool PACKED>
__global__ void k_s_sub_fill(const uint64_t *__restrict__ dets, int64_t n, int sbits, const int64_t *__restrict__ offs,
                             int32_t *__restrict__ cur, uint64_t *__restrict__ skeys) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t a = dets[2 * x], b = dets[2 * x + 1];
    const int64_t s = s_sub<PACKED>(a, b, sbits);
    const int64_t pos = offs[s] + atomicAdd(&cur[s], 1);
    skeys[2 * pos] = a;
    skeys[2 * pos + 1] = b;
}

void launch_s_sub(hipStream_t st, const uint64_t *dets, int64_t n, int sbits, bool packed, int32_t *cnt,
                  const int64_t *offs, uint64_t *skeys, bool fill) {
    if (n == 0) return;
    dim3 grid((unsigned)((n + 255) / 256)), blk(256);
    if (fill) {
        if (packed)
            hipLaunchKernelGGL(k_s_sub_fill<true>, grid, blk, 0, st, dets, n, sbits, offs, cnt, skeys);
        else
            hipLaunchKernelGGL(k_s_sub_fill<false>, grid, blk, 0, st, dets, n, sbits, offs, cnt, skeys);
    } else {
        if (packed)
            hipLaunchKernelGGL(k_s_sub_count<true>, grid, blk, 0, st, dets, n, sbits, cnt);
        else
            hipLaunchKernelGGL(k_s_sub_count<false>, grid, blk, 0, st, dets, n, sbits, cnt);
    }
}

// ------------------------------------------------------------------ reduce kernel
// Insert (a, b) into the LDS table; returns the slot or -1 when the table is full.
template <bool PACKED>
__device__ __forceinline__ int red_insert(unsigned long long *ka_t, unsigned long long *kb_t, uint64_t a, uint64_t b) {
    uint32_t s = (uint32_t)target_hash<PACKED>(a, b) & (kRedTab - 1);
    for (int p = 0; p < kRedTab; ++p) {
        if (PACKED) {
            const unsigned long long k = pack_key(a, b);
            const unsigned long long prev = atomicCAS(&ka_t[s], (unsigned long long)kEmptyKey, k);
            if (prev == kEmptyKey || prev == k) return (int)s;
        } else {
            const unsigned long long pa = atomicCAS(&ka_t[s], (unsigned long long)kEmptyKey, (unsigned long long)a);
            if (pa == kEmptyKey || pa == a) {
                const unsigned long long pb =
                    atomicCAS(&kb_t[s], (unsigned long long)kEmptyKey, (unsigned long long)b);
                if (pb == kEmptyKey || pb == b) return (int)s;
            }
        }
        s = (s + 1) & (kRedTab - 1);
    }
    return -1;
}

template <bool PACKED>
__global__ __launch_bounds__(kRedThreads) void k_pt2_reduce(Ham H, const uint64_t *__restrict__ dets,
                                                            const double *__restrict__ psi,
                                                            const uint64_t *__restrict__ desc,
                                                            const int64_t *__restrict__ sb,
                                                            const uint64_t *__restrict__ skeys,
                                                            const int64_t *__restrict__ soffs, int64_t n_s,
                                                            int64_t nsb, const double *__restrict__ vt,
                                                            const double *__restrict__ energy, uint64_t sample_mask,
                                                            PT2Export ex, double *__restrict__ part,
                                                            int *__restrict__ overflow) {
    __shared__ unsigned long long ka_t[kRedTab];
    __shared__ unsigned long long kb_t[PACKED ? 1 : kRedTab];
    __shared__ double w_t[kRedTab];
    __shared__ uint32_t in_s[kRedTab / 32];
    extern __shared__ double vt_s[];  // diagonal table (PACKED), sized at launch
    for (int t = threadIdx.x; t < kRedTab; t += blockDim.x) {
        ka_t[t] = kEmptyKey;
        if (!PACKED) kb_t[t] = kEmptyKey;
        w_t[t] = 0.0;
    }
    for (int t = threadIdx.x; t < kRedTab / 32; t += blockDim.x) in_s[t] = 0u;
    const int No = 2 * H.M;
    if (PACKED)
        for (int t = threadIdx.x; t < No + No * (No - 1) / 2; t += blockDim.x) vt_s[t] = vt[t];
    __syncthreads();
    bool lost = false;
    // members of S that hash into this sub-bucket: in the table, marked
    const int64_t q0 = soffs[blockIdx.x], q1 = blockIdx.x + 1 < nsb ? soffs[blockIdx.x + 1] : n_s;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const int s = red_insert<PACKED>(ka_t, kb_t, skeys[2 * q], skeys[2 * q + 1]);
        if (s < 0)
            lost = true;
        else
            atomicOr(&in_s[s >> 5], 1u << (s & 31));
    }
    __syncthreads();
    const int64_t s0 = sb[blockIdx.x], s1 = sb[blockIdx.x + 1];
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const uint64_t d = desc[i];
        const int64_t x = desc_x(d);
        const uint64_t xa = dets[2 * x], xb = dets[2 * x + 1];
        uint64_t a = xa, b = xb;
        apply_positions(desc_pos(d), a, b);
        const double v = h_offdiag(H, EriPacked{H.eri_pk}, a, b, xa, xb) * psi[x];
        const int s = red_insert<PACKED>(ka_t, kb_t, a, b);
        if (s < 0)
            lost = true;
        else
            atomicAdd(&w_t[s], v);
    }
    if (lost) atomicOr(overflow, 1);
    __syncthreads();
    const double E = energy[0];
    double sum = 0.0, mn = INFINITY, np = 0.0, nt = 0.0;
    for (int t = threadIdx.x; t < kRedTab; t += blockDim.x) {
        uint64_t a, b;
        if (PACKED) {
            const unsigned long long k = ka_t[t];
            if (k == kEmptyKey) continue;
            a = k & 0xffffffffull;
            b = k >> 32;
        } else {
            if (kb_t[t] == kEmptyKey) continue;
            a = ka_t[t];
            b = kb_t[t];
        }
        if ((in_s[t >> 5] >> (t & 31)) & 1u) continue;
        if (sample_mask && (key_hash(a, b) & sample_mask)) continue;
        const double w = w_t[t];
        double haa;
        if (PACKED) {
            const uint64_t occ = a | (b << H.M);
            haa = H.ecore;
            uint64_t rest = occ;
            while (rest) {
                const int qo = ctz64(rest);
                rest &= rest - 1;
                double e = vt_s[qo];
                const double *row = vt_s + No + qo * (qo - 1) / 2;
                uint64_t below = occ & ((1ull << qo) - 1ull);
                while (below) {
                    e += row[ctz64(below)];
                    below &= below - 1;
                }
                haa += e;
            }
        } else {
            haa = h_diag(H, a, b);
        }
        const double den = E - haa;
        np += 1.0;
        mn = fmin(mn, fabs(den));
        if (fabs(den) < 1e-8) nt += 1.0;
        if (w != 0.0) sum += w * w / den;
        if (ex.cap > 0) {
            const unsigned long long k = atomicAdd((unsigned long long *)ex.count, 1ull);
            if ((int64_t)k < ex.cap) {
                ex.keys[2 * k] = a;
                ex.keys[2 * k + 1] = b;
                ex.w[k] = w;
                ex.haa[k] = haa;
            }
        }
    }
    red_block(sum, mn, np, nt);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = sum;
        part[4 * blockIdx.x + 1] = mn;
        part[4 * blockIdx.x + 2] = np;
        part[4 * blockIdx.x + 3] = nt;
    }
}

void launch_pt2_reduce(hipStream_t st, const Ham &H, const uint64_t *dets, const double *psi, const uint64_t *desc,
                       const int64_t *sb, int64_t nsb, const uint64_t *skeys, const int64_t *soffs, int64_t n_s,
                       const double *vt, const double *energy, uint64_t sample_mask, const PT2Export &ex, double *part,
                       int *overflow, bool packed) {
    dim3 grid((unsigned)nsb), blk(kRedThreads);
    if (packed)
        hipLaunchKernelGGL(k_pt2_reduce<true>, grid, blk, sizeof(double) * pt2_diag_table_size(H.M), st, H, dets, psi, desc, sb, skeys, soffs, n_s, nsb, vt,
                           energy, sample_mask, ex, part, overflow);
    else
        hipLaunchKernelGGL(k_pt2_reduce<false>, grid, blk, 0, st, H, dets, psi, desc, sb, skeys, soffs, n_s, nsb, vt,
                           energy, sample_mask, ex, part, overflow);
}

int pt2_red_tab() { return kRedTab; }
int pt2_max_k1() { return kMaxK1; }
int pt2_max_k2() { return kMaxK2; }

}  // namespace dnqs
