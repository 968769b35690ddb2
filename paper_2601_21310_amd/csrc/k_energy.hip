// Energy kernels (Eq. 11): global scale removal, v = H_SS psi, and the FP64 reductions
// psi^T v and psi^T psi.  All reductions run in a fixed order (per-block partials,
// then one block), so E is bit-reproducible for a given psi.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kRedBlock = 256;

__device__ inline double block_reduce_max(double v) {
    __shared__ double sm[kRedBlock / kWave];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double r = sm[0];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) r = fmax(r, sm[w]);
    __syncthreads();
    return r;
}

__device__ inline double block_reduce_sum(double v) {
    __shared__ double sm[kRedBlock / kWave];
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double r = sm[0];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) r += sm[w];
    __syncthreads();
    return r;
}

// partial[b] = max over the block's items of logabs (sign 0 items are -inf already)
__global__ __launch_bounds__(kRedBlock) void k_max_partial(const double *__restrict__ la, int64_t n,
                                                           double *__restrict__ part) {
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, la[i]);
    m = block_reduce_max(m);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(kRedBlock) void k_max_final(const double *__restrict__ part, int nb,
                                                         double *__restrict__ out) {
    double m = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
    m = block_reduce_max(m);
    if (threadIdx.x == 0) out[0] = m;
}

// psi[x] = sign[x] * exp(la[x] - lmax)
__global__ void k_psi(const double *__restrict__ la, const int8_t *__restrict__ sg, int64_t n,
                      const double *__restrict__ lmax, double *__restrict__ psi) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = lmax[0];
    const int s = sg[i];
    psi[i] = (s == 0 || !isfinite(m)) ? 0.0 : (double)s * exp(la[i] - m);
}

int reduce_blocks(int64_t n) {
    int64_t b = (n + kRedBlock - 1) / kRedBlock;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

// lmax_out[0] = max logabs; psi = scaled amplitudes
void launch_scale_psi(hipStream_t st, const double *la, const int8_t *sg, int64_t n, double *part,
                      double *lmax_out, double *psi) {
    int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_max_partial, dim3(nb), dim3(kRedBlock), 0, st, la, n, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kRedBlock), 0, st, part, nb, lmax_out);
    hipLaunchKernelGGL(k_psi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, la, sg, n, lmax_out, psi);
}

// One wave per row: v[x] = diag[x] psi[x] + sum_j val[j] psi[col[j]] (FP64 accumulation).
// Block partials: part_pv[b] = sum psi v, part_pp[b] = sum psi^2 over the block's rows.
constexpr int kSpmvRowsPerBlock = kRedBlock / kWave;

__global__ __launch_bounds__(kRedBlock) void k_spmv(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, const float *__restrict__ val,
                                                    const double *__restrict__ diag, const double *__restrict__ psi,
                                                    int64_t n, double *__restrict__ v, double *__restrict__ part_pv,
                                                    double *__restrict__ part_pp) {
    __shared__ double s_pv[kSpmvRowsPerBlock], s_pp[kSpmvRowsPerBlock];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t x = (int64_t)blockIdx.x * kSpmvRowsPerBlock + wave;
    double pv = 0.0, pp = 0.0;
    if (x < n) {
        const double s = wave_sum(row_dot_lane(row_ptr, col, val, psi, x, lane));
        const double px = psi[x];
        const double vx = s + diag[x] * px;
        if (lane == 0) v[x] = vx;
        pv = px * vx;
        pp = px * px;
    }
    if (lane == 0) {
        s_pv[wave] = pv;
        s_pp[wave] = pp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kSpmvRowsPerBlock; ++w) {
            a += s_pv[w];
            c += s_pp[w];
        }
        part_pv[blockIdx.x] = a;
        part_pp[blockIdx.x] = c;
    }
}

// stats[0] = psi^T psi, stats[2] = psi^T v (stats[1] = l_max written earlier); E.
__global__ __launch_bounds__(kRedBlock) void k_energy_final(const double *__restrict__ part_pv,
                                                            const double *__restrict__ part_pp, int64_t nb,
                                                            double *__restrict__ stats,
                                                            double *__restrict__ energy) {
    // each thread's partials in the same order as a plain strided loop, eight of each
    // read together per step rather than one memory round trip per partial
    double a = 0.0, c = 0.0;
    const int64_t bs = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 7 * bs < nb; i += 8 * bs) {
        double va[8], vc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            va[u] = part_pv[i + u * bs];
            vc[u] = part_pp[i + u * bs];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a += va[u];
            c += vc[u];
        }
    }
    for (; i < nb; i += bs) {
        a += part_pv[i];
        c += part_pp[i];
    }
    a = block_reduce_sum(a);
    c = block_reduce_sum(c);
    if (threadIdx.x == 0) {
        stats[0] = c;
        stats[2] = a;
        energy[0] = c > 0.0 ? a / c : NAN;
    }
}

int64_t spmv_blocks(int64_t n) { return (n + kSpmvRowsPerBlock - 1) / kSpmvRowsPerBlock; }

void launch_spmv_energy(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *diag, const double *psi, int64_t n, double *v, double *part_pv,
                        double *part_pp, double *stats, double *energy) {
    int64_t nb = spmv_blocks(n);
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)nb), dim3(kRedBlock), 0, st, row_ptr, col, val, diag, psi, n, v,
                       part_pv, part_pp);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedBlock), 0, st, part_pv, part_pp, nb, stats, energy);
}

void launch_energy_final(hipStream_t st, const double *part_pv, const double *part_pp, int64_t nb, double *stats,
                         double *energy) {
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedBlock), 0, st, part_pv, part_pp, nb, stats, energy);
}

__global__ void k_set_f64(double *p, double v) { p[0] = v; }

void launch_set_f64(hipStream_t st, double *p, double v) {
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, st, p, v);
}

__global__ void k_copy_f64(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

void launch_copy_f64(hipStream_t st, const double *a, double *b, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

}  // namespace dnqs
