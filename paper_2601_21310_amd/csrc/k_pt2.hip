// Epstein-Nesbet PT2 (Eq. 13): the fixed-order sum of the internal terms over S, the
// fixed-order accumulation of per-sub-bucket partial records, and the final combination.
// The pair partition is in k_pt2_part.hip, the per-sub-bucket reduce in k_pt2_reduce.hip.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kFinBlock = 256;
constexpr int kRec = 8;  // doubles per partial record (kRedPart)

// One partial record: {sum, min |E - H_aa|, |P|, tiny, fingerprint sum bits, fingerprint
// XOR bits, 0, 0}.  Counts and the fingerprint are integers (exact in any order); the
// sums of records are taken in a fixed order.
struct Rec {
    double s, mn;
    unsigned long long np, nt, fs, fx;
};

__device__ __forceinline__ Rec rec_zero() { return Rec{0.0, INFINITY, 0ull, 0ull, 0ull, 0ull}; }

__device__ __forceinline__ void rec_add(Rec &r, const double *p) {
    r.s += p[0];
    r.mn = fmin(r.mn, p[1]);
    r.np += (unsigned long long)p[2];
    r.nt += (unsigned long long)p[3];
    r.fs += (unsigned long long)__double_as_longlong(p[4]);
    r.fx ^= (unsigned long long)__double_as_longlong(p[5]);
}

__device__ __forceinline__ void rec_store(const Rec &r, double *p) {
    p[0] = r.s;
    p[1] = r.mn;
    p[2] = (double)r.np;
    p[3] = (double)r.nt;
    p[4] = __longlong_as_double((long long)r.fs);
    p[5] = __longlong_as_double((long long)r.fx);
    p[6] = 0.0;
    p[7] = 0.0;
}

// block reduction of a record (fixed order: lanes by xor butterfly, then waves in order)
__device__ inline void block_rec(Rec &r) {
    __shared__ double ss[kFinBlock / kWave], sm[kFinBlock / kWave];
    __shared__ unsigned long long sp[kFinBlock / kWave], st[kFinBlock / kWave], sf[kFinBlock / kWave],
        sx[kFinBlock / kWave];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r.s += __shfl_xor(r.s, o, 64);
        r.mn = fmin(r.mn, __shfl_xor(r.mn, o, 64));
        r.np += __shfl_xor(r.np, o, 64);
        r.nt += __shfl_xor(r.nt, o, 64);
        r.fs += __shfl_xor(r.fs, o, 64);
        r.fx ^= __shfl_xor(r.fx, o, 64);
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) {
        ss[wave] = r.s;
        sm[wave] = r.mn;
        sp[wave] = r.np;
        st[wave] = r.nt;
        sf[wave] = r.fs;
        sx[wave] = r.fx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFinBlock / kWave; ++w) {
            ss[0] += ss[w];
            sm[0] = fmin(sm[0], sm[w]);
            sp[0] += sp[w];
            st[0] += st[w];
            sf[0] += sf[w];
            sx[0] ^= sx[w];
        }
        r.s = ss[0];
        r.mn = sm[0];
        r.np = sp[0];
        r.nt = st[0];
        r.fs = sf[0];
        r.fx = sx[0];
    }
}

// acc (one record) += the records part[0 .. nb), in a fixed order
__global__ __launch_bounds__(kFinBlock) void k_pt2_accumulate(const double *__restrict__ part, int64_t nb,
                                                              double *__restrict__ acc) {
    Rec r = rec_zero();
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) rec_add(r, part + kRec * i);
    block_rec(r);
    if (threadIdx.x == 0) {
        Rec a = rec_zero();
        rec_add(a, acc);
        a.s += r.s;
        a.mn = fmin(a.mn, r.mn);
        a.np += r.np;
        a.nt += r.nt;
        a.fs += r.fs;
        a.fx ^= r.fx;
        rec_store(a, acc);
    }
}

// Internal term over S (Eq. 13, first sum): the terms term[i] were formed by the reduce
// from exact FP64 couplings; here they are summed in a fixed order, with the minimum of
// |E - H_ii| and the count of |E - H_ii| < 1e-8 over S.
__global__ __launch_bounds__(kFinBlock) void k_pt2_internal(const double *__restrict__ term,
                                                            const double *__restrict__ diag, int64_t n,
                                                            const double *__restrict__ energy,
                                                            double *__restrict__ part) {
    const double E = energy[0];
    Rec r = rec_zero();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double den = E - diag[i];
        r.mn = fmin(r.mn, fabs(den));
        if (fabs(den) < 1e-8) ++r.nt;
        r.s += term[i];
    }
    block_rec(r);
    if (threadIdx.x == 0) {
        r.np = 0ull;
        r.fs = 0ull;
        r.fx = 0ull;
        rec_store(r, part + kRec * blockIdx.x);
    }
}

__global__ void k_pt2_init_acc(double *acc) {
    const Rec r = rec_zero();
    rec_store(r, acc);
}

void launch_pt2_internal(hipStream_t st, const double *term, const double *diag, int64_t n, const double *energy,
                         double *part, double *acc_int) {
    int64_t nb = (n + kFinBlock - 1) / kFinBlock;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_pt2_init_acc, dim3(1), dim3(1), 0, st, acc_int);
    hipLaunchKernelGGL(k_pt2_internal, dim3((unsigned)nb), dim3(kFinBlock), 0, st, term, diag, n, energy, part);
    hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, nb, acc_int);
}

// Contiguous chunks of the partials summed by many workgroups (fixed order within a
// chunk, then over the chunks), for the ~5e5 partials of the external sum.
constexpr int kAccBlocks = 1024;

__global__ __launch_bounds__(kFinBlock) void k_pt2_accumulate_chunks(const double *__restrict__ part, int64_t nb,
                                                                     double *__restrict__ out) {
    const int64_t chunk = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < nb ? lo + chunk : nb;
    Rec r = rec_zero();
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) rec_add(r, part + kRec * i);
    block_rec(r);
    if (threadIdx.x == 0) rec_store(r, out + kRec * blockIdx.x);
}

void launch_pt2_accumulate(hipStream_t st, const double *part, int64_t nb, double *acc, double *scratch) {
    if (scratch && nb > 4 * kAccBlocks) {
        hipLaunchKernelGGL(k_pt2_accumulate_chunks, dim3(kAccBlocks), dim3(kFinBlock), 0, st, part, nb, scratch);
        hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, scratch, (int64_t)kAccBlocks, acc);
    } else {
        hipLaunchKernelGGL(k_pt2_accumulate, dim3(1), dim3(kFinBlock), 0, st, part, nb, acc);
    }
}

int pt2_accumulate_scratch() { return kRec * kAccBlocks; }

void launch_pt2_init_acc(hipStream_t st, double *acc) {
    hipLaunchKernelGGL(k_pt2_init_acc, dim3(1), dim3(1), 0, st, acc);
}

__global__ void k_pt2_merge(double *acc, const double *part) {
    Rec a = rec_zero();
    rec_add(a, acc);
    rec_add(a, part);
    rec_store(a, acc);
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

// out = {(int + ext)/norm, int, ext, min den};
// counts = {pairs, |P|, tiny, sub-buckets, fingerprint sum, fingerprint XOR}
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
    counts[4] = (int64_t)__double_as_longlong(acc_ext[4]);
    counts[5] = (int64_t)__double_as_longlong(acc_ext[5]);
}

void launch_pt2_final(hipStream_t st, const double *acc_int, const double *acc_ext, const double *stats,
                      double *out, int64_t *counts, int64_t pairs, int64_t passes) {
    hipLaunchKernelGGL(k_pt2_final, dim3(1), dim3(1), 0, st, acc_int, acc_ext, stats, out, counts, pairs, passes);
}

}  // namespace dnqs
