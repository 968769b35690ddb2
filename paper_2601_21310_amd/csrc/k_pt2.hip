// Epstein-Nesbet PT2 (Eq. 13).
//
// Generation: one wavefront per determinant x of S.  The wave lists the occupied and
// empty orbitals of each spin string in LDS, then its lanes walk the excitation ids
// e in [0, n_exc) 64 at a time, unranking each id in closed form into
//   [alpha singles | beta singles | alpha-alpha doubles | beta-beta doubles | alpha-beta doubles]
// and computing the target key a and H_ax (FP64 integral table and arithmetic: the
// PT2 sum reaches tens of Ha on strongly coupled inputs, where FP32 couplings alone
// would cost ~1e-6 Ha).
// Reduce-by-key: the pair (a, H_ax psi_x) is added into an open-addressing hash table
// in device memory with a 64-bit CAS on the key and a native FP64 atomic add on the
// value.  Keys of S are kept too and dropped in the finalize pass (one probe of the S
// set per unique key instead of one per pair).  Work can be split into passes by a
// hash of the key so that each pass's table fits a memory budget.
// Finalize: for every unique a not in S, H_aa in FP64 and w_a^2 / (E - H_aa),
// summed in FP64 per block and then in a fixed order.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kMaxProbe = 1 << 14;

// pair index t over n items (i < j), ordered by j then i: t = j(j-1)/2 + i
__device__ __forceinline__ void unrank_pair(int t, int &i, int &j) {
    int jj = (int)((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
    while (jj * (jj - 1) / 2 > t) --jj;
    while ((jj + 1) * jj / 2 <= t) ++jj;
    j = jj;
    i = t - jj * (jj - 1) / 2;
}

__device__ __forceinline__ uint64_t pass_hash(uint64_t h) { return h >> 44; }

__device__ __forceinline__ uint64_t pack_key(uint64_t a, uint64_t b) { return a | (b << 32); }

template <bool PACKED>
__device__ __forceinline__ void table_add(const PT2Table &T, uint64_t a, uint64_t b, uint64_t h, double val) {
    uint64_t s = h & T.mask;
    if (PACKED) {
        const unsigned long long key = pack_key(a, b);
        Slot16 *slots = (Slot16 *)T.slots;
        for (int probe = 0; probe < kMaxProbe; ++probe) {
            unsigned long long cur = __hip_atomic_load(&slots[s].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == key) {
                unsafeAtomicAdd(&slots[s].w, val);
                return;
            }
            if (cur == kEmptyKey) {
                unsigned long long prev = atomicCAS(&slots[s].key, (unsigned long long)kEmptyKey, key);
                if (prev == kEmptyKey) {
                    atomicAdd(T.n_unique, 1ull);
                    unsafeAtomicAdd(&slots[s].w, val);
                    return;
                }
                if (prev == key) {
                    unsafeAtomicAdd(&slots[s].w, val);
                    return;
                }
            }
            s = (s + 1) & T.mask;
        }
    } else {
        Slot32 *slots = (Slot32 *)T.slots;
        for (int probe = 0; probe < kMaxProbe; ++probe) {
            unsigned long long ka = __hip_atomic_load(&slots[s].ka, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ka == kEmptyKey) ka = atomicCAS(&slots[s].ka, (unsigned long long)kEmptyKey, (unsigned long long)a);
            if (ka == kEmptyKey || ka == a) {
                // alpha word is ours (or already a): settle the beta word
                unsigned long long kb =
                    __hip_atomic_load(&slots[s].kb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (kb == kEmptyKey) {
                    kb = atomicCAS(&slots[s].kb, (unsigned long long)kEmptyKey, (unsigned long long)b);
                    if (kb == kEmptyKey) {
                        atomicAdd(T.n_unique, 1ull);
                        unsafeAtomicAdd(&slots[s].w, val);
                        return;
                    }
                }
                if (kb == b) {
                    unsafeAtomicAdd(&slots[s].w, val);
                    return;
                }
            }
            s = (s + 1) & T.mask;
        }
    }
    atomicOr(T.overflow, 1);
}

constexpr int kGenWaves = 4;

template <bool PACKED>
__global__ __launch_bounds__(256) void k_pt2_gen(Ham H, const uint64_t *__restrict__ dets, int64_t n,
                                                 const double *__restrict__ psi, int npass, int pass, PT2Table T) {
    __shared__ uint8_t lists[kGenWaves][4][64];  // occ_a, vir_a, occ_b, vir_b
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int M = H.M, na = H.na, nb = H.nb;
    const int64_t x = (int64_t)blockIdx.x * kGenWaves + wave;
    const bool live = x < n;
    const uint64_t xa = live ? dets[2 * x] : 0ull, xb = live ? dets[2 * x + 1] : 0ull;
    {
        const bool in = lane < M;
        const bool ba = in && ((xa >> lane) & 1ull), bb = in && ((xb >> lane) & 1ull);
        const uint64_t moa = ballot(ba), mva = ballot(in && !ba), mob = ballot(bb), mvb = ballot(in && !bb);
        if (ba) lists[wave][0][mbcnt(moa)] = (uint8_t)lane;
        if (in && !ba) lists[wave][1][mbcnt(mva)] = (uint8_t)lane;
        if (bb) lists[wave][2][mbcnt(mob)] = (uint8_t)lane;
        if (in && !bb) lists[wave][3][mbcnt(mvb)] = (uint8_t)lane;
    }
    __syncthreads();
    if (!live) return;
    const double px = psi[x];
    if (px == 0.0) return;
    const uint8_t *oa = lists[wave][0], *va = lists[wave][1], *ob = lists[wave][2], *vb = lists[wave][3];
    const int nva = M - na, nvb = M - nb;
    const int64_t nsa = (int64_t)na * nva, nsb = (int64_t)nb * nvb;
    const int64_t pva = (int64_t)nva * (nva - 1) / 2, pvb = (int64_t)nvb * (nvb - 1) / 2;
    const int64_t ndaa = (int64_t)na * (na - 1) / 2 * pva, ndbb = (int64_t)nb * (nb - 1) / 2 * pvb;
    const int64_t c1 = nsa, c2 = c1 + nsb, c3 = c2 + ndaa, c4 = c3 + ndbb, total = c4 + nsa * nsb;
    for (int64_t e = lane; e < total; e += kWave) {
        uint64_t ka = xa, kb = xb;
        if (e < c1) {
            const int t = (int)e;
            ka ^= (1ull << oa[t / nva]) | (1ull << va[t % nva]);
        } else if (e < c2) {
            const int t = (int)(e - c1);
            kb ^= (1ull << ob[t / nvb]) | (1ull << vb[t % nvb]);
        } else if (e < c3) {
            const int64_t t = e - c2;
            int i, j, a, b;
            unrank_pair((int)(t / pva), i, j);
            unrank_pair((int)(t % pva), a, b);
            ka ^= (1ull << oa[i]) | (1ull << oa[j]) | (1ull << va[a]) | (1ull << va[b]);
        } else if (e < c4) {
            const int64_t t = e - c3;
            int i, j, a, b;
            unrank_pair((int)(t / pvb), i, j);
            unrank_pair((int)(t % pvb), a, b);
            kb ^= (1ull << ob[i]) | (1ull << ob[j]) | (1ull << vb[a]) | (1ull << vb[b]);
        } else {
            const int64_t t = e - c4;
            const int sa = (int)(t / nsb), sb = (int)(t % nsb);
            ka ^= (1ull << oa[sa / nva]) | (1ull << va[sa % nva]);
            kb ^= (1ull << ob[sb / nvb]) | (1ull << vb[sb % nvb]);
        }
        const uint64_t hk = PACKED ? mix64(pack_key(ka, kb)) : key_hash(ka, kb);
        if (npass > 1 && (int)(pass_hash(hk) % (uint64_t)npass) != pass) continue;
        const double hv = h_offdiag(H, H.eri64, ka, kb, xa, xb);
        table_add<PACKED>(T, ka, kb, hk, hv * px);
    }
}

void launch_pt2_gen(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const double *psi, int npass,
                    int pass, const PT2Table &T, bool packed) {
    dim3 grid((unsigned)((n + kGenWaves - 1) / kGenWaves));
    if (packed)
        hipLaunchKernelGGL(k_pt2_gen<true>, grid, dim3(256), 0, st, H, dets, n, psi, npass, pass, T);
    else
        hipLaunchKernelGGL(k_pt2_gen<false>, grid, dim3(256), 0, st, H, dets, n, psi, npass, pass, T);
}

// clear a table: keys to kEmptyKey, values to 0
__global__ void k_pt2_clear(PT2Table T, int packed) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t cap = T.mask + 1;
    if (packed) {
        Slot16 *s = (Slot16 *)T.slots;
        for (; i < cap; i += stride) {
            s[i].key = kEmptyKey;
            s[i].w = 0.0;
        }
    } else {
        Slot32 *s = (Slot32 *)T.slots;
        for (; i < cap; i += stride) {
            s[i].ka = kEmptyKey;
            s[i].kb = kEmptyKey;
            s[i].w = 0.0;
            s[i].pad = 0.0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *T.n_unique = 0ull;
        *T.overflow = 0;
    }
}

void launch_pt2_clear(hipStream_t st, const PT2Table &T, bool packed) {
    uint64_t cap = T.mask + 1;
    uint64_t blocks = (cap + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_pt2_clear, dim3((unsigned)blocks), dim3(256), 0, st, T, packed ? 1 : 0);
}

constexpr int kFinBlock = 256;

__device__ inline void block_sum_min(double &s, double &mn, unsigned long long &np, unsigned long long &nt) {
    __shared__ double ss[kFinBlock / kWave], sm[kFinBlock / kWave];
    __shared__ unsigned long long sp[kFinBlock / kWave], st[kFinBlock / kWave];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        np += __shfl_xor(np, o, 64);
        nt += __shfl_xor(nt, o, 64);
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) {
        ss[wave] = s;
        sm[wave] = mn;
        sp[wave] = np;
        st[wave] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFinBlock / kWave; ++w) {
            ss[0] += ss[w];
            sm[0] = fmin(sm[0], sm[w]);
            sp[0] += sp[w];
            st[0] += st[w];
        }
        s = ss[0];
        mn = sm[0];
        np = sp[0];
        nt = st[0];
    }
}

template <bool PACKED>
__global__ __launch_bounds__(kFinBlock) void k_pt2_finalize(Ham H, PT2Table T, DetSet S,
                                                            const double *__restrict__ energy, uint64_t sample_mask,
                                                            PT2Export ex, double *__restrict__ part) {
    const double E = energy[0];
    const uint64_t cap = T.mask + 1;
    double s = 0.0, mn = INFINITY;
    unsigned long long np = 0, nt = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t a, b;
        double w;
        if (PACKED) {
            const Slot16 sl = ((const Slot16 *)T.slots)[i];
            if (sl.key == kEmptyKey) continue;
            a = sl.key & 0xffffffffull;
            b = sl.key >> 32;
            w = sl.w;
        } else {
            const Slot32 sl = ((const Slot32 *)T.slots)[i];
            if (sl.kb == kEmptyKey) continue;
            a = sl.ka;
            b = sl.kb;
            w = sl.w;
        }
        if (sample_mask && (key_hash(a, b) & sample_mask)) continue;
        if (detset_find(S, a, b) >= 0) continue;
        const double haa = h_diag(H, a, b);
        const double den = E - haa;
        ++np;
        mn = fmin(mn, fabs(den));
        if (fabs(den) < 1e-8) ++nt;
        if (w != 0.0) s += w * w / den;
        if (ex.cap > 0) {
            unsigned long long k = atomicAdd((unsigned long long *)ex.count, 1ull);
            if ((int64_t)k < ex.cap) {
                ex.keys[2 * k] = a;
                ex.keys[2 * k + 1] = b;
                ex.w[k] = w;
                ex.haa[k] = haa;
            }
        }
    }
    block_sum_min(s, mn, np, nt);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = s;
        part[4 * blockIdx.x + 1] = mn;
        part[4 * blockIdx.x + 2] = (double)np;
        part[4 * blockIdx.x + 3] = (double)nt;
    }
}

int pt2_fin_blocks(uint64_t cap) {
    uint64_t b = (cap + kFinBlock - 1) / kFinBlock;
    if (b > 2048) b = 2048;
    return (int)b;
}

// acc[0] += ext sum, acc[1] = min(acc[1], min den), acc[2] += |P|, acc[3] += tiny; fixed order
__global__ __launch_bounds__(kFinBlock) void k_pt2_accumulate(const double *__restrict__ part, int nb,
                                                              double *__restrict__ acc) {
    double s = 0.0, mn = INFINITY;
    unsigned long long np = 0, nt = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        s += part[4 * i];
        mn = fmin(mn, part[4 * i + 1]);
        np += (unsigned long long)part[4 * i + 2];
        nt += (unsigned long long)part[4 * i + 3];
    }
    block_sum_min(s, mn, np, nt);
    if (threadIdx.x == 0) {
        acc[0] += s;
        acc[1] = fmin(acc[1], mn);
        acc[2] += (double)np;
        acc[3] += (double)nt;
    }
}

void launch_pt2_finalize(hipStream_t st, const Ham &H, const PT2Table &T, bool packed, const DetSet &S,
                         const double *energy, uint64_t sample_mask, const PT2Export &ex, double *part,
                         double *acc) {
    int nb = pt2_fin_blocks(T.mask + 1);
    if (packed)
        hipLaunchKernelGGL(k_pt2_finalize<true>, dim3(nb), dim3(kFinBlock), 0, st, H, T, S, energy, sample_mask, ex,
                           part);
    else
        hipLaunchKernelGGL(k_pt2_finalize<false>, dim3(nb), dim3(kFinBlock), 0, st, H, T, S, energy, sample_mask,
                           ex, part);
    hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, nb, acc);
}

// internal term over S: sum (v - E psi)^2 / (E - diag), terms with zero numerator skipped
__global__ __launch_bounds__(kFinBlock) void k_pt2_internal(const double *__restrict__ psi,
                                                            const double *__restrict__ v,
                                                            const double *__restrict__ diag, int64_t n,
                                                            const double *__restrict__ energy,
                                                            double *__restrict__ part) {
    const double E = energy[0];
    double s = 0.0, mn = INFINITY;
    unsigned long long np = 0, nt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double r = v[i] - E * psi[i];
        const double den = E - diag[i];
        mn = fmin(mn, fabs(den));
        if (fabs(den) < 1e-8) ++nt;
        const double num = r * r;
        if (num != 0.0) s += num / den;
    }
    block_sum_min(s, mn, np, nt);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = s;
        part[4 * blockIdx.x + 1] = mn;
        part[4 * blockIdx.x + 2] = 0.0;
        part[4 * blockIdx.x + 3] = (double)nt;
    }
}

__global__ void k_pt2_init_acc(double *acc) {
    acc[0] = 0.0;
    acc[1] = INFINITY;
    acc[2] = 0.0;
    acc[3] = 0.0;
}

void launch_pt2_internal(hipStream_t st, const double *psi, const double *v, const double *diag, int64_t n,
                         const double *energy, double *part, double *acc_int) {
    int64_t nb = (n + kFinBlock - 1) / kFinBlock;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_pt2_init_acc, dim3(1), dim3(1), 0, st, acc_int);
    hipLaunchKernelGGL(k_pt2_internal, dim3((unsigned)nb), dim3(kFinBlock), 0, st, psi, v, diag, n, energy, part);
    hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, (int)nb, acc_int);
}

void launch_pt2_init_acc(hipStream_t st, double *acc) {
    hipLaunchKernelGGL(k_pt2_init_acc, dim3(1), dim3(1), 0, st, acc);
}

// out = {(int + ext)/norm, int, ext, min den}; counts[1] = |P|, counts[2] = tiny
__global__ void k_pt2_final(const double *__restrict__ acc_int, const double *__restrict__ acc_ext,
                            const double *__restrict__ stats, double *__restrict__ out, int64_t *__restrict__ counts,
                            int64_t pairs, int64_t passes) {
    const double norm = stats[0];
    out[0] = norm > 0.0 ? (acc_int[0] + acc_ext[0]) / norm : NAN;
    out[1] = acc_int[0];
    out[2] = acc_ext[0];
    out[3] = fmin(acc_int[1], acc_ext[1]);
    counts[0] = pairs;
    counts[1] = (int64_t)acc_ext[2];
    counts[2] = (int64_t)(acc_int[3] + acc_ext[3]);
    counts[3] = passes;
}

void launch_pt2_final(hipStream_t st, const double *acc_int, const double *acc_ext, const double *stats,
                      double *out, int64_t *counts, int64_t pairs, int64_t passes) {
    hipLaunchKernelGGL(k_pt2_final, dim3(1), dim3(1), 0, st, acc_int, acc_ext, stats, out, counts, pairs, passes);
}

}  // namespace dnqs
