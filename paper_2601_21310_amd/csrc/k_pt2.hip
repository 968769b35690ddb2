// Epstein-Nesbet PT2 (Eq. 13): the internal term over S, fixed-order accumulation of
// per-workgroup partial sums, and the final combination.  The external sum over P is
// in k_pt2_part.hip.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

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

// acc[0] += ext sum, acc[1] = min(acc[1], min den), acc[2] += |P|, acc[3] += tiny; fixed order
__global__ __launch_bounds__(kFinBlock) void k_pt2_accumulate(const double *__restrict__ part, int64_t nb,
                                                              double *__restrict__ acc) {
    double s = 0.0, mn = INFINITY;
    unsigned long long np = 0, nt = 0;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
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
    hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, nb, acc_int);
}

// Contiguous chunks of the partials summed by many workgroups (fixed order within a
// chunk, then over the chunks), for the ~5e5 partials of the external sum.
constexpr int kAccBlocks = 1024;

__global__ __launch_bounds__(kFinBlock) void k_pt2_accumulate_chunks(const double *__restrict__ part, int64_t nb,
                                                                     double *__restrict__ out) {
    const int64_t chunk = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < nb ? lo + chunk : nb;
    double s = 0.0, mn = INFINITY;
    unsigned long long np = 0, nt = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        s += part[4 * i];
        mn = fmin(mn, part[4 * i + 1]);
        np += (unsigned long long)part[4 * i + 2];
        nt += (unsigned long long)part[4 * i + 3];
    }
    block_sum_min(s, mn, np, nt);
    if (threadIdx.x == 0) {
        out[4 * blockIdx.x + 0] = s;
        out[4 * blockIdx.x + 1] = mn;
        out[4 * blockIdx.x + 2] = (double)np;
        out[4 * blockIdx.x + 3] = (double)nt;
    }
}

void launch_pt2_accumulate(hipStream_t st, const double *part, int64_t nb, double *acc, double *scratch) {
    if (scratch && nb > 4 * kAccBlocks) {
        hipLaunchKernelGGL(k_pt2_accumulate_chunks, dim3(kAccBlocks), dim3(kFinBlock), 0, st, part, nb, scratch);
        hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, scratch, (int64_t)kAccBlocks, acc);
    } else {
        hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, nb, acc);
    }
}

int pt2_accumulate_scratch() { return 4 * kAccBlocks; }

void launch_pt2_init_acc(hipStream_t st, double *acc) {
    hipLaunchKernelGGL(k_pt2_init_acc, dim3(1), dim3(1), 0, st, acc);
}

__global__ void k_pt2_merge(double *acc, const double *part) {
    acc[0] += part[0];
    acc[1] = fmin(acc[1], part[1]);
    acc[2] += part[2];
    acc[3] += part[3];
}

void launch_pt2_merge(hipStream_t st, double *acc, const double *part) {
    hipLaunchKernelGGL(k_pt2_merge, dim3(1), dim3(1), 0, st, acc, part);
}

// Source records of the reduce's per-pair gather, one cache line each: for M <= 32
// (packed) rec[2x .. 2x+1] = {alpha | beta << 32, bits of psi_x} (16 bytes: with the
// integrals the table stays resident in each XCD's L2), else rec[4x .. 4x+3] = {alpha,
// beta, bits of psi_x, 0}.
__global__ void k_pt2_records(const uint64_t *__restrict__ dets, const double *__restrict__ psi, int64_t n,
                              bool packed, uint64_t *__restrict__ rec) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t pb = (uint64_t)__double_as_longlong(psi[x]);
    if (packed) {
        rec[2 * x + 0] = dets[2 * x] | (dets[2 * x + 1] << 32);
        rec[2 * x + 1] = pb;
    } else {
        rec[4 * x + 0] = dets[2 * x];
        rec[4 * x + 1] = dets[2 * x + 1];
        rec[4 * x + 2] = pb;
        rec[4 * x + 3] = 0ull;
    }
}

void launch_pt2_records(hipStream_t st, const uint64_t *dets, const double *psi, int64_t n, bool packed,
                        uint64_t *rec) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pt2_records, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dets, psi, n, packed,
                       rec);
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
