// Kernels for batched problems (one geometry each: its own integrals, S, theta and
// H_SS), run together so that every stage of a step is one launch over all problems.
//
// Layout: the problems' determinants are concatenated, each problem's rows padded to a
// multiple of 128 so that every 128-row GEMM tile belongs to one problem.  Padding
// rows repeat the problem's first determinant (valid input for the network) and are
// given psi = 0 and an empty H_SS row, so they contribute nothing.  Reductions are
// segmented per problem, one workgroup per problem, in a fixed order.
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kSegBlock = 256;

// ---------------------------------------------------------------- layout
// Copy one problem's dets into rows [off, off + n) and fill padding rows [off + n, end)
// with its first det; pid[row] = g for every row of the span; diag and CSR likewise
// (column indices shifted by off, padding rows empty).
__global__ void k_cat_problem(int g, int64_t off, int64_t n, int64_t end, const uint64_t *__restrict__ dets,
                              const int64_t *__restrict__ row_ptr, const double *__restrict__ diag, int64_t nnz_off,
                              uint64_t *__restrict__ dets_cat, int32_t *__restrict__ pid,
                              int64_t *__restrict__ row_ptr_cat, double *__restrict__ diag_cat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < end - off;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = off + i;
        const int64_t src = i < n ? i : 0;
        dets_cat[2 * r] = dets[2 * src];
        dets_cat[2 * r + 1] = dets[2 * src + 1];
        pid[r] = g;
        row_ptr_cat[r] = nnz_off + row_ptr[i < n ? i : n];
        diag_cat[r] = i < n ? diag[i] : 0.0;
    }
}

__global__ void k_cat_cols(int64_t nnz, int64_t off, const int32_t *__restrict__ col, const float *__restrict__ val,
                           int64_t nnz_off, int32_t *__restrict__ col_cat, float *__restrict__ val_cat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        col_cat[nnz_off + i] = (int32_t)(col[i] + off);
        val_cat[nnz_off + i] = val[i];
    }
}

__global__ void k_set_i64(int64_t *p, int64_t v) { p[0] = v; }

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_cat_problem(hipStream_t st, int g, int64_t off, int64_t n, int64_t end, const uint64_t *dets,
                        const int64_t *row_ptr, const int32_t *col, const float *val, const double *diag, int64_t nnz,
                        int64_t nnz_off, uint64_t *dets_cat, int32_t *pid, int64_t *row_ptr_cat, int32_t *col_cat,
                        float *val_cat, double *diag_cat) {
    hipLaunchKernelGGL(k_cat_problem, dim3(grid_for(end - off)), dim3(256), 0, st, g, off, n, end, dets, row_ptr, diag,
                       nnz_off, dets_cat, pid, row_ptr_cat, diag_cat);
    if (nnz > 0)
        hipLaunchKernelGGL(k_cat_cols, dim3(grid_for(nnz)), dim3(256), 0, st, nnz, off, col, val, nnz_off, col_cat,
                           val_cat);
}

void launch_set_i64(hipStream_t st, int64_t *p, int64_t v) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, p, v);
}

// ---------------------------------------------------------------- segmented reductions
__device__ inline double seg_block_max(double v) {
    __shared__ double sm[kSegBlock / kWave];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (threadIdx.x % kWave == 0) sm[threadIdx.x / kWave] = v;
    __syncthreads();
    double r = sm[0];
    for (int w = 1; w < kSegBlock / kWave; ++w) r = fmax(r, sm[w]);
    __syncthreads();
    return r;
}

__device__ inline double seg_block_sum(double v) {
    __shared__ double sm[kSegBlock / kWave];
    v = wave_sum(v);
    if (threadIdx.x % kWave == 0) sm[threadIdx.x / kWave] = v;
    __syncthreads();
    double r = sm[0];
    for (int w = 1; w < kSegBlock / kWave; ++w) r += sm[w];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- per-item reductions
// The per-problem reductions are cut into work items {problem, first row, rows} of at
// most 4096 rows, listed in layout order, largest problem first, and launched one
// workgroup per item: the dispatcher starts workgroups in index order, so it hands out
// the items largest problem first and the short problems fill the tail, with no
// software queue.  Each item's partial result goes to its own slot and the slots of a
// problem are combined in item order, so the results do not depend on which CU ran which
// item.  (A persistent form that pulled items from an atomic head was miscompiled: with
// the head read by one lane and broadcast through LDS, the compiler split the loop so that
// the other lanes repeated the barrier-and-read part without the lane that takes the next
// item, and the workgroups spun.)

// ipart[2 item] = max of log|psi| over the item's rows
__global__ __launch_bounds__(kSegBlock) void k_item_lmax(const double *__restrict__ la, const int4 *__restrict__ items,
                                                         double *__restrict__ ipart) {
    const int it = blockIdx.x;
    const int4 w = items[it];
    double m = -INFINITY;
    for (int i = threadIdx.x; i < w.z; i += blockDim.x) m = fmax(m, la[(int64_t)w.y + i]);
    m = seg_block_max(m);
    if (threadIdx.x == 0) ipart[2 * it] = m;
}

// ipart[2 item] = sum of psi v, ipart[2 item + 1] = sum of psi^2 over the item's rows
__global__ __launch_bounds__(kSegBlock) void k_item_energy(const double *__restrict__ pv, const double *__restrict__ pp,
                                                           const int4 *__restrict__ items, double *__restrict__ ipart) {
    const int it = blockIdx.x;
    const int4 w = items[it];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < w.z; i += blockDim.x) {
        a += pv[(int64_t)w.y + i];
        c += pp[(int64_t)w.y + i];
    }
    a = seg_block_sum(a);
    c = seg_block_sum(c);
    if (threadIdx.x == 0) {
        ipart[2 * it] = a;
        ipart[2 * it + 1] = c;
    }
}

// one thread per problem: combine its items in order (items of a problem are contiguous)
__global__ void k_q_finish(const int4 *__restrict__ items, int nitems, const double *__restrict__ ipart,
                           const ProbDev *__restrict__ P, int G, int energy) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    double a = energy ? 0.0 : -INFINITY, c = 0.0;
    for (int it = 0; it < nitems; ++it) {
        if (items[it].x != g) continue;
        if (energy) {
            a += ipart[2 * it];
            c += ipart[2 * it + 1];
        } else {
            a = fmax(a, ipart[2 * it]);
        }
    }
    const ProbDev p = P[g];
    if (!energy) {
        p.stats[1] = a;
        return;
    }
    p.stats[0] = c;
    p.stats[2] = a;
    p.energy[0] = c > 0.0 ? a / c : NAN;
}

// psi[x] = sign exp(la - lmax of its problem); 0 on padding rows
__global__ void k_psi_grouped(const double *__restrict__ la, const int8_t *__restrict__ sg, int64_t ntot,
                              RowProblems rp, double *__restrict__ psi) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ntot) return;
    const ProbDev &p = rp.P[rp.pid[x]];
    const double m = p.stats[1];
    const int s = sg[x];
    psi[x] = (x - p.off >= p.n || s == 0 || !isfinite(m)) ? 0.0 : (double)s * exp(la[x] - m);
}

// one wave per row: v[x] = diag psi + sum val psi[col]; pv[x] = psi v, pp[x] = psi^2
__global__ __launch_bounds__(256) void k_spmv_rows(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                   const float *__restrict__ val, const double *__restrict__ diag,
                                                   const double *__restrict__ psi, int64_t n, double *__restrict__ v,
                                                   double *__restrict__ pv, double *__restrict__ pp) {
    const int lane = threadIdx.x % kWave;
    const int64_t x = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (x >= n) return;
    const double s = wave_sum(row_dot_lane(row_ptr, col, val, psi, x, lane));
    if (lane == 0) {
        const double px = psi[x];
        const double vx = s + diag[x] * px;
        v[x] = vx;
        pv[x] = px * vx;
        pp[x] = px * px;
    }
}

void launch_energy_grouped(hipStream_t st, const double *la, const int8_t *sg, int64_t ntot, int G, RowProblems rp,
                           const int64_t *row_ptr, const int32_t *col, const float *val, const double *diag,
                           double *psi, double *v, double *pv, double *pp, const int4 *items, int nitems,
                           double *ipart) {
    const unsigned fg = (unsigned)((G + 63) / 64);
    if (nitems > 0) hipLaunchKernelGGL(k_item_lmax, dim3((unsigned)nitems), dim3(kSegBlock), 0, st, la, items, ipart);
    hipLaunchKernelGGL(k_q_finish, dim3(fg), dim3(64), 0, st, items, nitems, ipart, rp.P, G, 0);
    hipLaunchKernelGGL(k_psi_grouped, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st, la, sg, ntot, rp, psi);
    hipLaunchKernelGGL(k_spmv_rows, dim3((unsigned)((ntot * kWave + 255) / 256)), dim3(256), 0, st, row_ptr, col, val,
                       diag, psi, ntot, v, pv, pp);
    if (nitems > 0)
        hipLaunchKernelGGL(k_item_energy, dim3((unsigned)nitems), dim3(kSegBlock), 0, st, pv, pp, items, ipart);
    hipLaunchKernelGGL(k_q_finish, dim3(fg), dim3(64), 0, st, items, nitems, ipart, rp.P, G, 1);
}

// ---------------------------------------------------------------- gradients
// grad_g[off + i] = sum over z in [zrange[g].x, zrange[g].y) of part[z * cnt + i]  (fixed order)
__global__ void k_reduce_splits_grouped(const float *__restrict__ part, const int2 *__restrict__ zrange, int64_t cnt,
                                        const ProbDev *__restrict__ P, int64_t off) {
    const int g = blockIdx.y;
    float *out = P[g].grad + off;
    const int z0 = zrange[g].x, z1 = zrange[g].y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        int z = z0;
        for (; z + 8 <= z1; z += 8) {  // eight reads in flight, added in z order
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * cnt + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; z < z1; ++z) s += part[(int64_t)z * cnt + i];
        out[i] = s;
    }
}

void launch_reduce_splits_grouped(hipStream_t st, const float *part, const int2 *zrange, int64_t cnt, int G,
                                  const ProbDev *P, int64_t off) {
    int64_t bx = (cnt + 255) / 256;
    if (bx > 256) bx = 256;
    hipLaunchKernelGGL(k_reduce_splits_grouped, dim3((unsigned)bx, G), dim3(256), 0, st, part, zrange, cnt, P, off);
}

// grad_g[dst + i] = grad_g[src + i]
__global__ void k_copy_grouped(const ProbDev *__restrict__ P, int64_t src, int64_t dst, int64_t cnt) {
    float *gr = P[blockIdx.y].grad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        gr[dst + i] = gr[src + i];
}

void launch_copy_grouped(hipStream_t st, const ProbDev *P, int G, int64_t src, int64_t dst, int64_t cnt) {
    int64_t bx = (cnt + 255) / 256;
    if (bx > 64) bx = 64;
    hipLaunchKernelGGL(k_copy_grouped, dim3((unsigned)bx, G), dim3(256), 0, st, P, src, dst, cnt);
}

// AdamW over every problem's parameters; moments stored problem-major [G][nparam]
__global__ void k_adamw_grouped(const ProbDev *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                                int64_t np, AdamCfg c, const int *__restrict__ step) {
    const int g = blockIdx.y;
    float *theta = (float *)P[g].theta;
    const float *grad = P[g].grad;
    float *mg = m + (int64_t)g * np, *vg = v + (int64_t)g * np;
    const int t = step[0] + 1;
    const double tc = (double)(t < c.decay_steps ? t : c.decay_steps);
    const float lr = (float)(c.lr_min + 0.5 * (c.lr_max - c.lr_min) *
                                            (1.0 + cos(3.14159265358979323846 * tc / (double)c.decay_steps)));
    const float bc1 = 1.0f - powf(c.beta1, (float)t), bc2 = 1.0f - powf(c.beta2, (float)t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const float gr = grad[i];
        const float mi = c.beta1 * mg[i] + (1.0f - c.beta1) * gr;
        const float vi = c.beta2 * vg[i] + (1.0f - c.beta2) * gr * gr;
        mg[i] = mi;
        vg[i] = vi;
        theta[i] -= lr * ((mi / bc1) / (sqrtf(vi / bc2) + c.eps) + c.weight_decay * theta[i]);
    }
}

__global__ void k_step_incr_b(int *step) { step[0] += 1; }

void launch_adamw_grouped(hipStream_t st, const ProbDev *P, int G, float *m, float *v, int64_t np, const AdamCfg &c,
                          int *step) {
    int64_t bx = (np + 255) / 256;
    if (bx > 512) bx = 512;
    hipLaunchKernelGGL(k_adamw_grouped, dim3((unsigned)bx, G), dim3(256), 0, st, P, m, v, np, c, step);
    hipLaunchKernelGGL(k_step_incr_b, dim3(1), dim3(1), 0, st, step);
}

}  // namespace dnqs
