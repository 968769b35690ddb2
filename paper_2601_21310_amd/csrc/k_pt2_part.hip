// Epstein-Nesbet PT2 (Eq. 13), external sum, by partitioning instead of global atomics.
//
// The reduce-by-key w_a = sum_x H_ax psi_x runs over |S| * n_exc pairs (3.1e9 at
// M = 28, 7+7, |S| = 1e5) into ~9e8 unique keys: only ~3.4 pairs per key, so an
// on-chip pre-aggregation saves little and a global hash table is bound by atomic
// throughput.  Instead the pairs are streamed through two hash partitions into
// sub-buckets small enough to reduce in LDS:
//
//   L1  a workgroup enumerates the excitations of 64 determinants (closed-form
//       unranking); each pair becomes an 8-byte descriptor [x index: 24 bits | four
//       7-bit flipped spin-orbital positions: 28 bits | the 12 hash bits after the L1
//       bits: 12 bits] bound for one of K1 buckets by the top bits of the target's key
//       hash.  A count pass and an exclusive scan in bucket-major order give every
//       workgroup a private, contiguous run per bucket (no global atomics); the fill
//       pass sorts each round of 8192 descriptors by bucket in LDS so that runs are
//       written in whole lines.
//   L2  each L1 bucket is cut into chunks; the same count -> scan -> sorted scatter
//       splits it into K2 sub-buckets by the hash bits carried in the descriptor (a
//       pure stream: no gathers, no rehashing).
//   R   (k_pt2_reduce.hip) one workgroup per sub-bucket decodes each descriptor (x XOR positions),
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

#include "dnqs_pt2.h"

namespace dnqs {

// Determinants per L1 workgroup (at most kL1XPerGroup).  A workgroup's LDS fills a CU, so
// the groups run in waves of one per CU; the group size is chosen so that the last wave
// is (nearly) full rather than a few groups running alone on an idle chip.
int pt2_l1_xper(int64_t n) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t per_wave = (int64_t)kL1XPerGroup * cus;
    const int64_t waves = std::max<int64_t>(1, (n + per_wave - 1) / per_wave);
    const int64_t xper = (n + waves * cus - 1) / (waves * cus);
    return (int)std::min<int64_t>(std::max<int64_t>(xper, 1), kL1XPerGroup);
}

int64_t pt2_l1_groups(int64_t n) {
    const int xper = pt2_l1_xper(n);
    return (n + xper - 1) / xper;
}
int pt2_max_dets() { return 1 << kDescXBits; }

// ------------------------------------------------------------------ block scan
// Exclusive scan of cnt[0..count) into out (count <= 2 * blockDim.x, blockDim.x a
// multiple of 64); returns nothing, out is complete after the call (which syncs).
__device__ inline void block_exclusive_scan(const uint32_t *cnt, uint32_t *out, int count, uint32_t *wsum) {
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave, nw = blockDim.x / kWave;
    const uint32_t a0 = 2 * t < count ? cnt[2 * t] : 0u, a1 = 2 * t + 1 < count ? cnt[2 * t + 1] : 0u;
    uint32_t v = a0 + a1;  // inclusive scan of the pair sums across the wave
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    if (lane == kWave - 1) wsum[wave] = v;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < nw; ++w) {
            const uint32_t x = wsum[w];
            wsum[w] = acc;
            acc += x;
        }
    }
    __syncthreads();
    const uint32_t excl = wsum[wave] + v - (a0 + a1);
    if (2 * t < count) out[2 * t] = excl;
    if (2 * t + 1 < count) out[2 * t + 1] = excl + a0;
    __syncthreads();
}

// ------------------------------------------------------------------ L1
// One 1024-thread workgroup per xper (<= kL1XPerGroup) determinants.  The workgroup's pairs are
// numbered q = (determinant in the group) * n_exc + excitation and produced in rounds of
// kL1Round (8 per thread).  Count pass (FILL = false): per-bucket totals of the group.
// Fill pass: each round is sorted by bucket in LDS (histogram with ranks, scan, place)
// and written out so that consecutive lanes write consecutive descriptors of one
// bucket's run: whole lines instead of one 8-byte write per open run.  Pairs of dead
// determinants (psi = 0) go to bucket K1, which is never written.
// Key-space slice (ss > 0): only targets whose top ss hash bits equal `slice` are kept,
// and the bucket bits are taken from the hash shifted past the slice bits.
template <bool FILL, bool PACKED>
__global__ __launch_bounds__(kL1Threads) void k_pt2_l1(Ham H, const uint64_t *__restrict__ dets, int64_t n,
                                                       const double *__restrict__ psi, int s1, int xper, int64_t nwg,
                                                       uint32_t *__restrict__ counts, const int64_t *__restrict__ offs,
                                                       uint64_t *__restrict__ desc, int ss, uint32_t slice,
                                                       unsigned long long *__restrict__ cur1, int64_t cap1,
                                                       int *__restrict__ ovf) {
    __shared__ uint8_t lists[kL1XPerGroup][4][64];
    __shared__ uint64_t xs[kL1XPerGroup][2];
    __shared__ uint32_t live_s[kL1XPerGroup];
    __shared__ uint32_t hist[kMaxK1 + 1];
    __shared__ uint32_t bst[FILL ? kMaxK1 + 1 : 1];
    __shared__ uint32_t cur[FILL ? kMaxK1 : 1];
    __shared__ int64_t base[FILL ? kMaxK1 : 1];
    __shared__ uint64_t srt[FILL ? kL1Round : 1];
    __shared__ uint16_t sbk[FILL ? kL1Round : 1];
    __shared__ uint32_t wsum[kL1Threads / kWave];
    const int K1 = 1 << s1;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t wg = blockIdx.x;
    constexpr int kWavesL1 = kL1Threads / kWave;
    for (int xl = wave; xl < xper; xl += kWavesL1) {
        const int64_t x = wg * xper + xl;
        const bool live = x < n && psi[x] != 0.0;
        const uint64_t xa = live ? dets[2 * x] : 0ull, xb = live ? dets[2 * x + 1] : 0ull;
        wave_build_lists(lists[xl], H.M, xa, xb);
        if (lane == 0) {
            xs[xl][0] = xa;
            xs[xl][1] = xb;
            live_s[xl] = live ? 1u : 0u;
        }
    }
    for (int b = threadIdx.x; b <= K1; b += blockDim.x) {
        hist[b] = 0u;
        if (FILL && b < K1) {
            cur[b] = 0u;
            base[b] = cur1 ? 0 : offs[(int64_t)b * nwg + wg];
        }
    }
    __syncthreads();
    const ExcLists proto = make_exc_lists(lists[0], H.M, H.na, H.nb);  // class sizes: the same for every det
    const int T = proto.total;
    const int64_t total = (int64_t)xper * T;
    for (int64_t r0 = 0; r0 < total; r0 += kL1Round) {
        uint64_t d[kL1Round / kL1Threads];
        uint32_t bk[kL1Round / kL1Threads], rk[kL1Round / kL1Threads];
        int64_t q = r0 + threadIdx.x;
        int xl = (int)(q / T);
        int e = (int)(q - (int64_t)xl * T);
#pragma unroll
        for (int j = 0; j < kL1Round / kL1Threads; ++j) {
            bk[j] = (uint32_t)K1;
            d[j] = 0ull;
            if (q < total && live_s[xl]) {
                ExcLists c = proto;
                c.oa = lists[xl][0];
                c.va = lists[xl][1];
                c.ob = lists[xl][2];
                c.vb = lists[xl][3];
                const uint32_t pos = excitation_positions(c, e);
                uint64_t ka = xs[xl][0], kb = xs[xl][1];
                apply_positions(pos, ka, kb);
                uint64_t h = target_hash<PACKED>(ka, kb);
                const bool in_slice = ss == 0 || (uint32_t)(h >> (64 - ss)) == slice;
                if (ss) h <<= ss;
                if (in_slice) {
                    bk[j] = l1_bucket(h, s1);
                    d[j] = make_desc(wg * xper + xl, pos, h, s1);
                }
            }
            rk[j] = atomicAdd(&hist[bk[j]], 1u);
            q += blockDim.x;
            e += blockDim.x;
            while (e >= T) {
                e -= T;
                ++xl;
            }
        }
        if (!FILL) continue;
        __syncthreads();
        block_exclusive_scan(hist, bst, K1 + 1, wsum);
#pragma unroll
        for (int j = 0; j < kL1Round / kL1Threads; ++j)
            if (bk[j] < (uint32_t)K1) {
                const uint32_t sp = bst[bk[j]] + rk[j];
                srt[sp] = d[j];
                sbk[sp] = (uint16_t)bk[j];
            }
        if (cur1) {
            // fixed-capacity bucket regions: this round's run of bucket b is reserved at
            // the region's cursor (one 64-bit atomic per non-empty bucket and round), so no
            // count pass is needed; a region that would overflow raises *ovf and the
            // caller repeats the pass with counted offsets
            for (int b = threadIdx.x; b < K1; b += blockDim.x) {
                const uint32_t c = hist[b];
                int64_t r = -1;
                if (c) {
                    r = (int64_t)atomicAdd(&cur1[b], (unsigned long long)c);
                    if (r + (int64_t)c > cap1) {
                        atomicOr(ovf, 1);
                        r = -1;
                    } else {
                        r += (int64_t)b * cap1;
                    }
                }
                base[b] = r;
            }
        }
        __syncthreads();
        const uint32_t nvalid = bst[K1];
        for (uint32_t sp = threadIdx.x; sp < nvalid; sp += blockDim.x) {
            const uint32_t b = sbk[sp];
            if (!cur1)
                desc[base[b] + cur[b] + (sp - bst[b])] = srt[sp];
            else if (base[b] >= 0)
                desc[base[b] + (sp - bst[b])] = srt[sp];
        }
        __syncthreads();
        for (int b = threadIdx.x; b <= K1; b += blockDim.x) {
            if (b < K1) cur[b] += hist[b];
            hist[b] = 0u;
        }
        __syncthreads();
    }
    if (!FILL) {
        __syncthreads();
        for (int b = threadIdx.x; b < K1; b += blockDim.x) counts[wg * K1 + b] = hist[b];
    }
}

void launch_pt2_l1(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const double *psi, int s1,
                   int64_t nwg, uint32_t *counts, const int64_t *offs, uint64_t *desc, bool fill, bool packed, int ss,
                   uint32_t slice, uint64_t *cur1, int64_t cap1, int *ovf) {
    dim3 grid((unsigned)nwg), blk(kL1Threads);
    const int xper = pt2_l1_xper(n);  // nwg = pt2_l1_groups(n) comes from the same choice
    unsigned long long *c1 = reinterpret_cast<unsigned long long *>(cur1);
    if (fill) {
        if (packed)
            hipLaunchKernelGGL((k_pt2_l1<true, true>), grid, blk, 0, st, H, dets, n, psi, s1, xper, nwg, counts, offs, desc,
                               ss, slice, c1, cap1, ovf);
        else
            hipLaunchKernelGGL((k_pt2_l1<true, false>), grid, blk, 0, st, H, dets, n, psi, s1, xper, nwg, counts, offs, desc,
                               ss, slice, c1, cap1, ovf);
    } else {
        if (packed)
            hipLaunchKernelGGL((k_pt2_l1<false, true>), grid, blk, 0, st, H, dets, n, psi, s1, xper, nwg, counts, offs,
                               desc, ss, slice, c1, cap1, ovf);
        else
            hipLaunchKernelGGL((k_pt2_l1<false, false>), grid, blk, 0, st, H, dets, n, psi, s1, xper, nwg, counts, offs,
                               desc, ss, slice, c1, cap1, ovf);
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

__global__ void k_pt2_l2_staged(const uint64_t *__restrict__ desc1, const PT2Chunk *__restrict__ chunks, int s2,
                                const int64_t *__restrict__ offs, uint64_t *__restrict__ desc2);

void launch_pt2_l2(hipStream_t st, const uint64_t *desc1, const PT2Chunk *chunks, int64_t nchunk, int s2,
                   uint32_t *counts, const int64_t *offs, uint64_t *desc2, bool fill) {
    dim3 grid((unsigned)nchunk), blk(256);
    if (fill && (1 << s2) <= kMaxK2Staged)
        hipLaunchKernelGGL(k_pt2_l2_staged, grid, dim3(kL2Threads), 0, st, desc1, chunks, s2, offs, desc2);
    else if (fill)
        hipLaunchKernelGGL(k_pt2_l2<true>, grid, blk, 0, st, desc1, chunks, s2, counts, offs, desc2);
    else
        hipLaunchKernelGGL(k_pt2_l2<false>, grid, blk, 0, st, desc1, chunks, s2, counts, offs, desc2);
}

// Staged L2 fill (K2 <= kMaxK2Staged): rounds of kL2Round descriptors of a chunk are
// sorted by sub-bucket in LDS and written out run by run, as in the L1 fill.
__global__ __launch_bounds__(kL2Threads) void k_pt2_l2_staged(const uint64_t *__restrict__ desc1,
                                                              const PT2Chunk *__restrict__ chunks, int s2,
                                                              const int64_t *__restrict__ offs,
                                                              uint64_t *__restrict__ desc2) {
    __shared__ uint64_t srt[kL2Round];
    __shared__ uint32_t hist[kMaxK2Staged], bst[kMaxK2Staged], cur[kMaxK2Staged];
    __shared__ int64_t base[kMaxK2Staged];
    __shared__ uint32_t wsum[kL2Threads / kWave];
    const int K2 = 1 << s2;
    const int64_t c = blockIdx.x;
    const PT2Chunk ch = chunks[c];
    for (int b = threadIdx.x; b < K2; b += blockDim.x) {
        hist[b] = 0u;
        cur[b] = 0u;
        base[b] = offs[l2_tpos(ch, c, b, K2)];
    }
    __syncthreads();
    constexpr int PER = kL2Round / kL2Threads;
    for (int64_t r0 = 0; r0 < ch.len; r0 += kL2Round) {
        const int nr = (int)(ch.len - r0 < kL2Round ? ch.len - r0 : kL2Round);
        uint64_t d[PER];
        uint32_t bk[PER], rk[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = j * kL2Threads + threadIdx.x;
            bk[j] = 0xffffffffu;
            if (i < nr) {
                d[j] = desc1[ch.start + r0 + i];
                bk[j] = desc_sub(d[j], s2);
                rk[j] = atomicAdd(&hist[bk[j]], 1u);
            }
        }
        __syncthreads();
        block_exclusive_scan(hist, bst, K2, wsum);
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (bk[j] != 0xffffffffu) srt[bst[bk[j]] + rk[j]] = d[j];
        __syncthreads();
        for (int sp = threadIdx.x; sp < nr; sp += blockDim.x) {
            const uint64_t v = srt[sp];
            const uint32_t b = desc_sub(v, s2);
            desc2[base[b] + cur[b] + (sp - bst[b])] = v;
        }
        __syncthreads();
        for (int b = threadIdx.x; b < K2; b += blockDim.x) {
            cur[b] += hist[b];
            hist[b] = 0u;
        }
        __syncthreads();
    }
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

int pt2_max_k1() { return kMaxK1; }
int pt2_max_k2() { return kMaxK2; }

}  // namespace dnqs
