// Lanczos iteration on H_SS for its lowest eigenpair: E_diag = lambda_min(H_SS), the
// variational-space diagnostic of the post-optimisation analysis (Sec. 2.4), and the
// converged reference vector at which PT2 is evaluated when the network is not used.
//
// Device side: the sparse product is the energy SpMV (k_energy.hip: FP32 off-diagonal
// values, FP64 diagonal and accumulation); the Krylov vectors are FP64 and every new
// vector is orthogonalised against all earlier ones twice (classical Gram-Schmidt,
// repeated), with every dot product a fixed-order reduction, so the iteration is
// reproducible to the bit.  Host side: the lowest eigenpair of the small tridiagonal
// matrix (bisection on the Sturm count, then inverse iteration), and the stopping test.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kLzBlock = 256;
constexpr int kLzDotBlocks = 64;  // partial sums per dot product

__device__ inline double lz_block_sum(double v) {
    __shared__ double sm[kLzBlock / kWave];
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kLzBlock / kWave; ++w) r += sm[w];
    __syncthreads();
    return r;
}

// part[k * kLzDotBlocks + b] = sum over block b's share of V[k] . w, for k < m
__global__ __launch_bounds__(kLzBlock) void k_lz_dots(const double *__restrict__ V, int64_t ldv, int m,
                                                      const double *__restrict__ w, int64_t n,
                                                      double *__restrict__ part) {
    const int k = blockIdx.y, b = blockIdx.x;
    const double *vk = V + (int64_t)k * ldv;
    double s = 0.0;
    for (int64_t i = (int64_t)b * kLzBlock + threadIdx.x; i < n; i += (int64_t)kLzDotBlocks * kLzBlock)
        s += vk[i] * w[i];
    s = lz_block_sum(s);
    if (threadIdx.x == 0) part[(int64_t)k * kLzDotBlocks + b] = s;
}

// c[k] (+)= sum of the kLzDotBlocks partials of dot k, in order
__global__ void k_lz_dots_final(const double *__restrict__ part, int m, double *__restrict__ c, int accumulate) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double s = 0.0;
    for (int b = 0; b < kLzDotBlocks; ++b) s += part[(int64_t)k * kLzDotBlocks + b];
    c[k] = accumulate ? c[k] + s : s;
}

// w[i] -= sum_k c[k] V[k][i] (k ascending); part[b] = block b's share of |w|^2
__global__ __launch_bounds__(kLzBlock) void k_lz_orth(const double *__restrict__ V, int64_t ldv, int m,
                                                      const double *__restrict__ c, double *__restrict__ w,
                                                      int64_t n, double *__restrict__ part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kLzBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLzBlock) {
        double x = w[i];
        for (int k = 0; k < m; ++k) x -= c[k] * V[(int64_t)k * ldv + i];
        w[i] = x;
        s += x * x;
    }
    s = lz_block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sqrt(sum of nb partials): each thread sums a fixed strided share, then the
// block sum in a fixed order (one workgroup; the same bits on every call)
__global__ __launch_bounds__(kLzBlock) void k_lz_norm(const double *__restrict__ part, int nb,
                                                      double *__restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kLzBlock) s += part[b];
    s = lz_block_sum(s);
    if (threadIdx.x == 0) out[0] = sqrt(s);
}

// dst[i] = src[i] / nrm[0]
__global__ void k_lz_scale(const double *__restrict__ src, int64_t n, const double *__restrict__ nrm,
                           double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] / nrm[0];
}

// out[i] = sum_k y[k] V[k][i] (k ascending)
__global__ void k_lz_combine(const double *__restrict__ V, int64_t ldv, int m, const double *__restrict__ y,
                             int64_t n, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += y[k] * V[(int64_t)k * ldv + i];
    out[i] = s;
}

// start vector when the caller gives none: the determinants with the lowest diagonal
// weighted up, plus a SplitMix64-based deterministic spread so that no eigenvector is
// orthogonal to it by symmetry
__global__ void k_lz_start(const double *__restrict__ diag, int64_t n, const double *__restrict__ dmin,
                           double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = (double)(mix64((uint64_t)i + 0x9e3779b97f4a7c15ull) >> 11) * 0x1.0p-53;
    v[i] = exp(-(diag[i] - dmin[0])) + 1e-3 * (u - 0.5);
}

__global__ __launch_bounds__(kLzBlock) void k_lz_min(const double *__restrict__ d, int64_t n, double *__restrict__ out) {
    __shared__ double sm[kLzBlock];
    double m = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += kLzBlock) m = fmin(m, d[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < kLzBlock; ++t) m = fmin(m, sm[t]);
        out[0] = m;
    }
}

static unsigned lz_grid(int64_t n) {
    int64_t g = (n + kLzBlock - 1) / kLzBlock;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (unsigned)g;
}

int lanczos_dot_blocks() { return kLzDotBlocks; }
int lanczos_norm_blocks(int64_t n) { return (int)lz_grid(n); }

void launch_lz_dots(hipStream_t st, const double *V, int64_t ldv, int m, const double *w, int64_t n, double *part,
                    double *c, bool accumulate) {
    hipLaunchKernelGGL(k_lz_dots, dim3(kLzDotBlocks, (unsigned)m), dim3(kLzBlock), 0, st, V, ldv, m, w, n, part);
    hipLaunchKernelGGL(k_lz_dots_final, dim3((unsigned)((m + 63) / 64)), dim3(64), 0, st, part, m, c,
                       accumulate ? 1 : 0);
}

void launch_lz_orth(hipStream_t st, const double *V, int64_t ldv, int m, const double *c, double *w, int64_t n,
                    double *part, double *nrm) {
    const unsigned g = lz_grid(n);
    hipLaunchKernelGGL(k_lz_orth, dim3(g), dim3(kLzBlock), 0, st, V, ldv, m, c, w, n, part);
    hipLaunchKernelGGL(k_lz_norm, dim3(1), dim3(kLzBlock), 0, st, part, (int)g, nrm);
}

void launch_lz_norm(hipStream_t st, const double *w, int64_t n, double *part, double *nrm) {
    // |w| with no vectors to remove
    const unsigned g = lz_grid(n);
    hipLaunchKernelGGL(k_lz_orth, dim3(g), dim3(kLzBlock), 0, st, w, n, 0, (const double *)nullptr,
                       const_cast<double *>(w), n, part);
    hipLaunchKernelGGL(k_lz_norm, dim3(1), dim3(kLzBlock), 0, st, part, (int)g, nrm);
}

void launch_lz_scale(hipStream_t st, const double *src, int64_t n, const double *nrm, double *dst) {
    hipLaunchKernelGGL(k_lz_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n, nrm, dst);
}

void launch_lz_combine(hipStream_t st, const double *V, int64_t ldv, int m, const double *y, int64_t n,
                       double *out) {
    hipLaunchKernelGGL(k_lz_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, V, ldv, m, y, n, out);
}

void launch_lz_start(hipStream_t st, const double *diag, int64_t n, double *tmp1, double *v) {
    hipLaunchKernelGGL(k_lz_min, dim3(1), dim3(kLzBlock), 0, st, diag, n, tmp1);
    hipLaunchKernelGGL(k_lz_start, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, diag, n, tmp1, v);
}

}  // namespace dnqs
