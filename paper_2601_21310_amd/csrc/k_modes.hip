// The target-set objectives of Sec. 2.3 on T = [V; P]: the proxy Hamiltonian of Eq. 8 as
// one CSR matrix over T (assembled from H_VV, H_PV and its transpose H_VP, and the
// diagonal of P), and the Asymmetric objective's sparse product (Eq. 6) with the vector
// whose residual drives the adjoint of either its exact gradient or the Eq. 7 estimator.
//
// Every energy and gradient then runs through the same kernels as the variational mode:
// amplitudes over T, this product, the fixed-order FP64 reductions and the adjoint.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kMdBlock = 256;

// count of the determinants p[0..m) that are members of S
__global__ void k_count_in_set(const uint64_t *__restrict__ p, int64_t m, DetSet S, int *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && detset_find(S, p[2 * i], p[2 * i + 1]) >= 0) atomicAdd(count, 1);
}

void launch_count_in_set(hipStream_t st, const uint64_t *p, int64_t m, const DetSet &S, int *count) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_count_in_set, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, p, m, S, count);
}

// entries per column of a CSR matrix (the row lengths of its transpose)
__global__ void k_col_count(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, int64_t m,
                            int32_t *__restrict__ cnt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    for (int64_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) atomicAdd(&cnt[col[j]], 1);
}

// the transpose's entries, each row's in arbitrary order (sorted afterwards by column)
__global__ void k_transpose_fill(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                 const float *__restrict__ val, int64_t m, const int64_t *__restrict__ off,
                                 int32_t *__restrict__ cur, int32_t *__restrict__ tcol, float *__restrict__ tval) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    for (int64_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
        const int32_t c = col[j];
        const int64_t q = off[c] + atomicAdd(&cur[c], 1);
        tcol[q] = (int32_t)r;
        tval[q] = val[j];
    }
}

void launch_csr_transpose(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val, int64_t m,
                          int64_t ncols, int32_t *cnt, int64_t *off, int64_t *bsum, int64_t *total,
                          int64_t *t_row_ptr, int32_t *t_col, float *t_val, bool fill) {
    const dim3 g((unsigned)((m + 255) / 256)), b(256);
    if (!fill) {
        if (m > 0) hipLaunchKernelGGL(k_col_count, g, b, 0, st, row_ptr, col, m, cnt);
        launch_exclusive_scan(st, cnt, ncols, off, bsum, total);
        return;
    }
    // cnt is reused as the cursors (zeroed by the caller)
    if (m > 0) hipLaunchKernelGGL(k_transpose_fill, g, b, 0, st, row_ptr, col, val, m, off, cnt, t_col, t_val);
    launch_rows_finish(st, off, ncols, total, t_row_ptr, t_col, t_val);
}

// row lengths of the proxy matrix over T: V rows hold H_VV then H_VP, P rows hold H_PV
__global__ void k_target_len(const int64_t *__restrict__ vv, const int64_t *__restrict__ vp, int64_t nv,
                             const int64_t *__restrict__ pv, int64_t np, int32_t *__restrict__ len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nv)
        len[r] = (int32_t)((vv[r + 1] - vv[r]) + (vp[r + 1] - vp[r]));
    else if (r < nv + np)
        len[r] = (int32_t)(pv[r - nv + 1] - pv[r - nv]);
}

// copy the rows into place; H_VP's columns shift by nv (P's positions in T)
__global__ void k_target_fill(const int64_t *__restrict__ vv, const int32_t *__restrict__ vvc,
                              const float *__restrict__ vvv, const int64_t *__restrict__ vp,
                              const int32_t *__restrict__ vpc, const float *__restrict__ vpv,
                              const int64_t *__restrict__ pv, const int32_t *__restrict__ pvc,
                              const float *__restrict__ pvv, int64_t nv, int64_t np,
                              const int64_t *__restrict__ off, int32_t *__restrict__ col, float *__restrict__ val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nv + np) return;
    int64_t q = off[r];
    if (r < nv) {
        for (int64_t j = vv[r]; j < vv[r + 1]; ++j, ++q) {
            col[q] = vvc[j];
            val[q] = vvv[j];
        }
        for (int64_t j = vp[r]; j < vp[r + 1]; ++j, ++q) {
            col[q] = (int32_t)(nv + vpc[j]);
            val[q] = vpv[j];
        }
    } else {
        const int64_t a = r - nv;
        for (int64_t j = pv[a]; j < pv[a + 1]; ++j, ++q) {
            col[q] = pvc[j];
            val[q] = pvv[j];
        }
    }
}

void launch_target_assemble(hipStream_t st, const int64_t *vv, const int32_t *vvc, const float *vvv,
                            const int64_t *vp, const int32_t *vpc, const float *vpv, const int64_t *pv,
                            const int32_t *pvc, const float *pvv, int64_t nv, int64_t np, int32_t *len,
                            int64_t *off, int64_t *bsum, int64_t *total, int32_t *col, float *val, bool fill) {
    const int64_t nt = nv + np;
    const dim3 g((unsigned)((nt + 255) / 256)), b(256);
    if (!fill) {
        hipLaunchKernelGGL(k_target_len, g, b, 0, st, vv, vp, nv, pv, np, len);
        launch_exclusive_scan(st, len, nt, off, bsum, total);
    } else {
        hipLaunchKernelGGL(k_target_fill, g, b, 0, st, vv, vvc, vvv, vp, vpc, vpv, pv, pvc, pvv, nv, np, off, col,
                           val);
    }
}

// ---------------------------------------------------------------- Asymmetric objective
// One wave per row of the proxy matrix over T.  For x in V: sV = (H_VV psi_V)_x (diagonal
// included), sP = (H_VP psi_P)_x, u[x] = sV + sP (= (H_VT psi_T)_x, the numerator of
// E_loc(x) psi(x)); for a in P: u[a] = (H_PV psi_V)_a (no diagonal).  Block partials of
// psi_x u_x and psi_x^2 over V only; k_asym_vec later turns u into the vector v' for
// which 2 (v' - E psi) / psi_V^T psi_V is the adjoint's coefficient.
constexpr int kMdRows = kMdBlock / kWave;

__global__ __launch_bounds__(kMdBlock) void k_spmv_asym(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const float *__restrict__ val,
                                                        const double *__restrict__ diag,
                                                        const double *__restrict__ psi, int64_t n, int64_t nv,
                                                        double *__restrict__ u, double *__restrict__ up,
                                                        double *__restrict__ part_pv, double *__restrict__ part_pp) {
    __shared__ double s_pv[kMdRows], s_pp[kMdRows];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t x = (int64_t)blockIdx.x * kMdRows + wave;
    double pv = 0.0, pp = 0.0;
    if (x < n) {
        const int64_t b = row_ptr[x], e = row_ptr[x + 1];
        double sv = 0.0, sp = 0.0;
        for (int64_t j = b + lane; j < e; j += kWave) {
            const int32_t c = col[j];
            const double t = (double)val[j] * psi[c];
            if (c < nv)
                sv += t;
            else
                sp += t;
        }
        sv = wave_sum(sv);
        sp = wave_sum(sp);
        const double px = psi[x];
        if (x < nv) {
            sv += diag[x] * px;
            if (lane == 0) {
                u[x] = sv + sp;
                up[x] = sp;
            }
            pv = px * (sv + sp);
            pp = px * px;
        } else if (lane == 0) {
            u[x] = sv;
            up[x] = 0.0;
        }
    }
    if (lane == 0) {
        s_pv[wave] = pv;
        s_pp[wave] = pp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kMdRows; ++w) {
            a += s_pv[w];
            c += s_pp[w];
        }
        part_pv[blockIdx.x] = a;
        part_pp[blockIdx.x] = c;
    }
}

// v' for the adjoint: exact gradient of Eq. 6: V rows u - sP / 2 (the H_VP part enters
// the derivative once, H_VV twice), P rows u / 2 + E psi (no normalisation term);
// estimator of Eq. 7: V rows u, P rows E psi (no coefficient on P)
__global__ void k_asym_vec(const double *__restrict__ u, const double *__restrict__ up,
                           const double *__restrict__ psi, int64_t n, int64_t nv, const double *__restrict__ energy,
                           int estimator, double *__restrict__ v) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const double E = energy[0];
    if (x < nv)
        v[x] = estimator ? u[x] : u[x] - 0.5 * up[x];
    else
        v[x] = estimator ? E * psi[x] : 0.5 * u[x] + E * psi[x];
}

void launch_energy_asym(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *diag, const double *psi, int64_t n, int64_t nv, double *u, double *up,
                        double *part_pv, double *part_pp, double *stats, double *energy, int estimator, double *v) {
    const int64_t nb = (n + kMdRows - 1) / kMdRows;
    hipLaunchKernelGGL(k_spmv_asym, dim3((unsigned)nb), dim3(kMdBlock), 0, st, row_ptr, col, val, diag, psi, n, nv, u,
                       up, part_pv, part_pp);
    launch_energy_final(st, part_pv, part_pp, nb, stats, energy);
    hipLaunchKernelGGL(k_asym_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, u, up, psi, n, nv, energy,
                       estimator, v);
}

int64_t asym_blocks(int64_t n) { return (n + kMdRows - 1) / kMdRows; }

}  // namespace dnqs
