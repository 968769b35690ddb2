// Occupied-row form of the orbital output layer (Eqs. 3-4).
//
// The determinant of x reads only the rows of Phi(x) at the occupied spin-orbitals, so
// only N_e of the N_o row blocks of the output layer are needed per configuration.
// For a variational set grown around a reference determinant, the reference orbitals
// are occupied in most of S and every other orbital in a few percent of it.  The output
// layer is therefore split by orbital:
//   dense  orbitals (occupied in a large share of S): one GEMM over their N_e-wide
//          column blocks for every configuration (rows of unoccupied orbitals unused);
//   sparse orbitals: one "entry" per (configuration, occupied sparse orbital), its N_e
//          outputs computed from that configuration's last hidden layer.
// Entries are grouped by orbital, each group in ascending configuration order, built
// without atomics so that every sum below has a fixed order.  The data gradient of the
// sparse rows is formed by orbital (its weight block read once per tile of entries) and
// then summed per configuration in row order.
//
//   k_os_count      occupancy count of every spin-orbital over S
//   k_os_bcount     per block of 256 configurations: sparse entries per orbital
//   k_os_scan       entry offsets per (block, orbital)
//   k_os_fill       entry -> (configuration, occupied row), and (configuration, row) ->
//                   entry (-1 for a dense orbital)
//   k_os_gather_w   the dense orbitals' columns of W_L and b_L, [W_D; b_D]
//   k_os_fwd        O_sp[e][k] = b_L[p N_e + k] + sum_h h[x_e][h] W_L[h][p N_e + k]
//   k_os_trans_w    W_L as [orbital][electron][hidden]
//   k_os_drows      C[e][h] = sum_k dO_sp[e][k] W_L[h][p_e N_e + k]
//   k_os_dsum       delta[x][h] = (delta_D[x][h] + sum_{sparse rows e of x} C[e][h])
//                   (1 - h[x][h]^2)
//   k_os_wgrad      partial dW_L, db_L of the sparse orbitals over chunks of entries
//   k_os_wgrad_sum  fixed-order sum of the chunk partials into the gradient columns
//   k_os_scatter    dense orbitals' [dW_D; db_D] into the gradient columns
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

constexpr int kOsBlock = 256;  // configurations per block in the entry build

__device__ __forceinline__ bool so_occupied(uint64_t a, uint64_t b, int M, int p) {
    return p < M ? ((a >> p) & 1ull) : ((b >> (p - M)) & 1ull);
}

// row of spin-orbital p (occupied) in A(x): alpha orbitals first, ascending
__device__ __forceinline__ int so_row(uint64_t a, uint64_t b, int M, int na, int p) {
    return p < M ? popc64(a & ((1ull << p) - 1ull)) : na + popc64(b & ((1ull << (p - M)) - 1ull));
}

__global__ void k_os_count(const uint64_t *__restrict__ dets, int64_t n, int M, unsigned long long *__restrict__ cnt) {
    __shared__ unsigned int h[128];
    const int No = 2 * M;
    for (int p = threadIdx.x; p < No; p += blockDim.x) h[p] = 0u;
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) {
        uint64_t a = dets[2 * x], b = dets[2 * x + 1];
        while (a) {
            atomicAdd(&h[ctz64(a)], 1u);
            a &= a - 1;
        }
        while (b) {
            atomicAdd(&h[M + ctz64(b)], 1u);
            b &= b - 1;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < No; p += blockDim.x)
        if (h[p]) atomicAdd(&cnt[p], (unsigned long long)h[p]);
}

__global__ void k_os_bcount(const uint64_t *__restrict__ dets, int64_t n, int M, const int *__restrict__ dpos,
                            int *__restrict__ bcnt) {
    __shared__ unsigned int h[128];
    const int No = 2 * M;
    for (int p = threadIdx.x; p < No; p += blockDim.x) h[p] = 0u;
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * kOsBlock + threadIdx.x;
    if (x < n) {
        uint64_t a = dets[2 * x], b = dets[2 * x + 1];
        while (a) {
            const int p = ctz64(a);
            a &= a - 1;
            if (dpos[p] < 0) atomicAdd(&h[p], 1u);
        }
        while (b) {
            const int p = M + ctz64(b);
            b &= b - 1;
            if (dpos[p] < 0) atomicAdd(&h[p], 1u);
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < No; p += blockDim.x) bcnt[(int64_t)blockIdx.x * No + p] = (int)h[p];
}

// one thread per orbital: boff[blk][p] = eoff[p] + sum_{b < blk} bcnt[b][p]
__global__ void k_os_scan(const int *__restrict__ bcnt, int64_t nblk, int No, const int64_t *__restrict__ eoff,
                          int64_t *__restrict__ boff) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= No) return;
    int64_t s = eoff[p];
    for (int64_t b = 0; b < nblk; ++b) {
        boff[b * No + p] = s;
        s += bcnt[b * No + p];
    }
}

// One thread per configuration, kOsBlock per block.  For every orbital in turn the
// block ranks its configurations holding that sparse orbital (ascending x).
__global__ __launch_bounds__(kOsBlock) void k_os_fill(const uint64_t *__restrict__ dets, int64_t n, int M, int na,
                                                      int Ne, const int *__restrict__ dpos,
                                                      const int64_t *__restrict__ boff, int32_t *__restrict__ ex,
                                                      int32_t *__restrict__ ej, int32_t *__restrict__ idx) {
    __shared__ int wsum[kOsBlock / kWave];
    const int No = 2 * M;
    const int64_t x = (int64_t)blockIdx.x * kOsBlock + threadIdx.x;
    const bool live = x < n;
    const uint64_t a = live ? dets[2 * x] : 0ull, b = live ? dets[2 * x + 1] : 0ull;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    for (int p = 0; p < No; ++p) {
        const bool occ = live && so_occupied(a, b, M, p);
        const bool sp = occ && dpos[p] < 0;
        const int j = occ ? so_row(a, b, M, na, p) : 0;
        const uint64_t bal = __ballot(sp);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        before += __popcll(bal & ((1ull << lane) - 1ull));
        if (sp) {
            const int64_t e = boff[(int64_t)blockIdx.x * No + p] + before;
            ex[e] = (int32_t)x;
            ej[e] = j;
            idx[x * Ne + j] = (int32_t)e;
        } else if (occ) {
            idx[x * Ne + j] = -1;
        }
        __syncthreads();
    }
}

// WD[h][t] = W[h][dorb[t / Ne] Ne + t % Ne] (h < din), WD[din][t] = b[...]
__global__ void k_os_gather_w(const float *__restrict__ W, const float *__restrict__ bias, int din, int width,
                              int Ne, int nd, const int *__restrict__ dorb, float *__restrict__ WD) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wd = nd * Ne;
    if (i >= (int64_t)(din + 1) * wd) return;
    const int h = (int)(i / wd), t = (int)(i % wd);
    const int col = dorb[t / Ne] * Ne + t % Ne;
    WD[i] = h < din ? W[(int64_t)h * width + col] : bias[col];
}

// Entry tiles: {orbital, first entry, count <= kOsTile}.  A tile is a small dense product,
// [entries x din] (the entries' h_{L-1} rows) times the orbital's [din x Ne] column block
// of W_L, done on v_mfma_f32_16x16x4f32: each wave takes 16 entries, NP/16 output blocks
// of 16 columns.  A workgroup takes kOsFwdTiles consecutive tiles (the tiles of one
// orbital are consecutive) and stages the column block in LDS once per orbital run, as
// [din][NP + 4] (the padding puts the four k rows one B fragment reads on distinct banks).
// MFMA 16x16x4 lane layout: A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k, D[i][j] at
// lane j + 16 (i / 4), element i % 4.  Each lane loads four consecutive h values of its
// entry (64 contiguous bytes per entry and K step of 16), so MFMA m of a step takes
// k = k0 + 4 (lane / 16) + m: the k order within a dot product is permuted, which only
// reorders the FP32 sum.
constexpr int kOsTile = 64, kOsFwdTiles = 4;

typedef float v4f_os __attribute__((ext_vector_type(4)));

template <int NP>
__device__ __forceinline__ void os_stage_w(float *Ws, const float *__restrict__ W, int din, int width, int Ne, int p) {
    // eight reads in flight per thread (clamped to valid addresses, padding columns zeroed)
    constexpr int S = NP + 4;
    const int tot = din * NP;
    for (int i0 = threadIdx.x; i0 < tot; i0 += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            const int h = i / NP, c = i % NP;
            v[u] = W[(int64_t)(h < din ? h : 0) * width + p * Ne + (c < Ne ? c : 0)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < tot) Ws[(i / NP) * S + i % NP] = i % NP < Ne ? v[u] : 0.0f;
        }
    }
}

template <int NP>
__global__ __launch_bounds__(256) void k_os_fwd(const float *__restrict__ hL, int din, const float *__restrict__ W,
                                                const float *__restrict__ bias, int width, int Ne,
                                                const int4 *__restrict__ tiles, int64_t ntiles,
                                                const int32_t *__restrict__ ex, float *__restrict__ Osp) {
    constexpr int S = NP + 4, JB = NP / 16;
    extern __shared__ float Ws[];  // [din][S]
    const int64_t t0 = (int64_t)blockIdx.x * kOsFwdTiles;
    const int64_t t1 = t0 + kOsFwdTiles < ntiles ? t0 + kOsFwdTiles : ntiles;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, kg = lane >> 4;
    int staged = -1;
    for (int64_t t = t0; t < t1; ++t) {
        const int4 tl = tiles[t];
        const int p = tl.x;
        if (p != staged) {  // uniform over the workgroup
            __syncthreads();
            os_stage_w<NP>(Ws, W, din, width, Ne, p);
            __syncthreads();
            staged = p;
        }
        const int le = 16 * wave + li;  // this lane's A row (entry) within the tile
        // a row past the tile reads the tile's first entry; its outputs are not stored
        const int64_t e = (int64_t)tl.y + (le < tl.z ? le : 0);
        const float *hr = hL + (int64_t)ex[e] * din + 4 * kg;
        v4f_os acc[JB];
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) acc[jb] = v4f_os{0.0f, 0.0f, 0.0f, 0.0f};
        if (16 * wave < tl.z) {  // uniform per wave
            int k0 = 0;
            for (; k0 + 128 <= din; k0 += 128) {
                v4f_os a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = *reinterpret_cast<const v4f_os *>(hr + k0 + 16 * u);
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const float *wr = Ws + (k0 + 16 * u + 4 * kg + m) * S + li;
#pragma unroll
                        for (int jb = 0; jb < JB; ++jb)
                            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][m], wr[16 * jb], acc[jb], 0, 0, 0);
                    }
            }
            for (; k0 < din; k0 += 16) {
                const v4f_os av = *reinterpret_cast<const v4f_os *>(hr + k0);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float *wr = Ws + (k0 + 4 * kg + m) * S + li;
#pragma unroll
                    for (int jb = 0; jb < JB; ++jb)
                        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m], wr[16 * jb], acc[jb], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
            const int col = 16 * jb + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int er = 16 * wave + 4 * kg + r;
                if (er < tl.z && col < Ne) {
                    const int64_t ee = (int64_t)tl.y + er;
                    Osp[ee * Ne + col] = bias[p * Ne + col] + acc[jb][r];
                }
            }
        }
    }
}

// WT[p][k][h] = W[h][p Ne + k]
__global__ void k_os_trans_w(const float *__restrict__ W, int din, int width, float *__restrict__ WT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)din * width) return;
    const int col = (int)(i / din), h = (int)(i % din);
    WT[i] = W[(int64_t)h * width + col];
}

// Data gradient of the sparse rows, by orbital: Cr[e][h] = sum_k dO_sp[e][k] W[h][p Ne + k]
// for the entries e of one tile (orbital p); thread h keeps W's Ne values for its h in
// registers, the tile's dO rows are staged in LDS.
template <int NP>
__global__ __launch_bounds__(256) void k_os_drows(const float *__restrict__ WT, int din, int Ne,
                                                  const int4 *__restrict__ tiles, const float *__restrict__ dOsp,
                                                  float *__restrict__ Cr) {
    __shared__ float gs[kOsTile * NP];
    const int4 tl = tiles[blockIdx.x];
    const int p = tl.x;
    // reads issued unconditionally (clamped indices) so that they overlap; padding zeroed
    for (int i = threadIdx.x; i < tl.z * NP; i += blockDim.x) {
        const int e = i / NP, k = i % NP;
        const float v = dOsp[((int64_t)tl.y + e) * Ne + (k < Ne ? k : 0)];
        gs[i] = k < Ne ? v : 0.0f;
    }
    __syncthreads();
    for (int h = threadIdx.x; h < din; h += blockDim.x) {
        float w[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) w[k] = WT[((int64_t)p * Ne + (k < Ne ? k : 0)) * din + h];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (k >= Ne) w[k] = 0.0f;
        for (int e = 0; e < tl.z; ++e) {
            const float4 *g4 = reinterpret_cast<const float4 *>(gs + e * NP);
            float s = 0.0f;
#pragma unroll
            for (int q = 0; q < NP / 4; ++q) {
                const float4 g = g4[q];
                s = fmaf(g.x, w[4 * q + 0], s);
                s = fmaf(g.y, w[4 * q + 1], s);
                s = fmaf(g.z, w[4 * q + 2], s);
                s = fmaf(g.w, w[4 * q + 3], s);
            }
            Cr[((int64_t)tl.y + e) * din + h] = s;
        }
    }
}

// delta[x][h] = (dD[x][h] + sum of Cr[e][h] over x's sparse rows e in row order)
//               * (1 - hL[x][h]^2); four configurations per workgroup, one wave each.
// dD (the dense part) may be null (no dense orbital).
__global__ __launch_bounds__(256) void k_os_dsum(int64_t n, int Ne, int din, const float *__restrict__ dD,
                                                 const float *__restrict__ Cr, const int32_t *__restrict__ idx,
                                                 const float *__restrict__ hL, float *__restrict__ delta) {
    __shared__ int es[4][32];
    __shared__ int nes[4];
    const int sl = threadIdx.x / 64, lt = threadIdx.x % 64;
    const int64_t x = (int64_t)blockIdx.x * 4 + sl;
    const bool live = x < n;
    const int e = (live && lt < Ne) ? idx[x * Ne + lt] : -1;
    const uint64_t bal = __ballot(e >= 0);
    if (e >= 0) es[sl][__popcll(bal & ((1ull << lt) - 1ull))] = e;
    if (lt == 0) nes[sl] = __popcll(bal);
    __syncthreads();
    if (!live) return;
    const int cnt = nes[sl];
    // four h per lane and four sparse rows at a time, all reads of a batch in flight
    // together (clamped to valid addresses); each sum in the order dD, then the rows
    for (int h0 = lt; h0 < din; h0 += 256) {
        int hh[4];
        float s[4], hv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            hh[u] = h0 + 64 * u < din ? h0 + 64 * u : h0;
            s[u] = dD ? dD[x * din + hh[u]] : 0.0f;
            hv[u] = hL[x * din + hh[u]];
        }
        for (int r0 = 0; r0 < cnt; r0 += 4) {
            float c[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float *cr = Cr + (int64_t)es[sl][r0 + q < cnt ? r0 + q : r0] * din;
#pragma unroll
                for (int u = 0; u < 4; ++u) c[q][u] = cr[hh[u]];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (r0 + q < cnt) s[u] += c[q][u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (h0 + 64 * u < din) delta[x * din + h0 + 64 * u] = s[u] * (1.0f - hv[u] * hv[u]);
    }
}

// Partial weight / bias gradients of the sparse orbitals.  Work item {orbital, first
// entry, count <= kOsItemMax}; its entries' dO (rows padded to NP values) and
// configurations are staged in LDS; thread h in [0, din] (h = din: the bias row)
// accumulates the Ne outputs over the item's entries in order into part[item][h][k].
constexpr int kOsItemMax = 512;

template <int NP>
__global__ __launch_bounds__(256) void k_os_wgrad(const float *__restrict__ hL, int din, int Ne,
                                                  const int4 *__restrict__ items, const int32_t *__restrict__ ex,
                                                  const float *__restrict__ dOsp, float *__restrict__ part) {
    extern __shared__ float gs[];  // [kOsItemMax][NP], then kOsItemMax configuration indices
    int *xs = reinterpret_cast<int *>(gs + kOsItemMax * NP);
    const int4 it = items[blockIdx.x];
    // staging with eight reads in flight per thread (clamped addresses, padding zeroed)
    const int tot = it.z * NP;
    for (int i0 = threadIdx.x; i0 < tot; i0 += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            const int e = i < tot ? i / NP : 0, k = i % NP;
            v[u] = dOsp[((int64_t)it.y + e) * Ne + (k < Ne ? k : 0)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < tot) gs[i] = i % NP < Ne ? v[u] : 0.0f;
        }
    }
    for (int i = threadIdx.x; i < it.z; i += blockDim.x) xs[i] = ex[(int64_t)it.y + i];
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * (din + 1) * Ne;
    for (int h = blockIdx.y * blockDim.x + threadIdx.x; h <= din; h += gridDim.y * blockDim.x) {
        float acc[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = 0.0f;
        // eight entries' h values read together (row din, the bias row, is 1; its lanes
        // read a valid element and discard it), then accumulated in entry order
        const int hc = h < din ? h : din - 1;
        int i = 0;
        for (; i + 8 <= it.z; i += 8) {
            float hv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) hv[u] = hL[(int64_t)xs[i + u] * din + hc];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float hu = h < din ? hv[u] : 1.0f;
                const float4 *g4 = reinterpret_cast<const float4 *>(gs + (i + u) * NP);
#pragma unroll
                for (int q = 0; q < NP / 4; ++q) {
                    const float4 g = g4[q];
                    acc[4 * q + 0] = fmaf(hu, g.x, acc[4 * q + 0]);
                    acc[4 * q + 1] = fmaf(hu, g.y, acc[4 * q + 1]);
                    acc[4 * q + 2] = fmaf(hu, g.z, acc[4 * q + 2]);
                    acc[4 * q + 3] = fmaf(hu, g.w, acc[4 * q + 3]);
                }
            }
        }
        for (; i < it.z; ++i) {
            const float hv = h < din ? hL[(int64_t)xs[i] * din + hc] : 1.0f;
            const float4 *g4 = reinterpret_cast<const float4 *>(gs + i * NP);
#pragma unroll
            for (int q = 0; q < NP / 4; ++q) {
                const float4 g = g4[q];
                acc[4 * q + 0] = fmaf(hv, g.x, acc[4 * q + 0]);
                acc[4 * q + 1] = fmaf(hv, g.y, acc[4 * q + 1]);
                acc[4 * q + 2] = fmaf(hv, g.z, acc[4 * q + 2]);
                acc[4 * q + 3] = fmaf(hv, g.w, acc[4 * q + 3]);
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (k < Ne) out[(int64_t)h * Ne + k] = acc[k];
    }
}

// grad[h][p Ne + k] (h <= din; row din is the bias) = sum over the orbital's items in
// order; zero for a sparse orbital without entries.  One thread per (h, p, k).
__global__ void k_os_wgrad_sum(const float *__restrict__ part, int din, int Ne, int No, const int *__restrict__ dpos,
                               const int *__restrict__ ifirst, const int *__restrict__ icount,
                               float *__restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int width = No * Ne;
    if (i >= (int64_t)(din + 1) * width) return;
    const int h = (int)(i / width), col = (int)(i % width);
    const int p = col / Ne, k = col % Ne;
    if (dpos[p] >= 0) return;
    float s = 0.0f;
    for (int q = 0; q < icount[p]; ++q) s += part[((int64_t)(ifirst[p] + q) * (din + 1) + h) * Ne + k];
    grad[i] = s;
}

// grad[h][dorb[t / Ne] Ne + t % Ne] = GD[h][t] for h <= din
__global__ void k_os_scatter(const float *__restrict__ GD, int din, int Ne, int nd, int width,
                             const int *__restrict__ dorb, float *__restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wd = nd * Ne;
    if (i >= (int64_t)(din + 1) * wd) return;
    const int h = (int)(i / wd), t = (int)(i % wd);
    grad[(int64_t)h * width + dorb[t / Ne] * Ne + t % Ne] = GD[i];
}

// ------------------------------------------------------------------ launches
static unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_os_count(hipStream_t st, const uint64_t *dets, int64_t n, int M, unsigned long long *cnt) {
    hipLaunchKernelGGL(k_os_count, dim3(g1(n)), dim3(256), 0, st, dets, n, M, cnt);
}

int64_t os_blocks(int64_t n) { return (n + kOsBlock - 1) / kOsBlock; }

void launch_os_build(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int Ne, const int *dpos,
                     const int64_t *eoff, int *bcnt, int64_t *boff, int32_t *ex, int32_t *ej, int32_t *idx) {
    const int64_t nb = os_blocks(n);
    const int No = 2 * M;
    hipLaunchKernelGGL(k_os_bcount, dim3((unsigned)nb), dim3(kOsBlock), 0, st, dets, n, M, dpos, bcnt);
    hipLaunchKernelGGL(k_os_scan, dim3(1), dim3(128), 0, st, bcnt, nb, No, eoff, boff);
    hipLaunchKernelGGL(k_os_fill, dim3((unsigned)nb), dim3(kOsBlock), 0, st, dets, n, M, na, Ne, dpos, boff, ex, ej,
                       idx);
}

void launch_os_gather_w(hipStream_t st, const float *W, const float *bias, int din, int width, int Ne, int nd,
                        const int *dorb, float *WD) {
    const int64_t tot = (int64_t)(din + 1) * nd * Ne;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_os_gather_w, dim3(g1(tot)), dim3(256), 0, st, W, bias, din, width, Ne, nd, dorb, WD);
}

int os_tile() { return kOsTile; }

// k_os_fwd stages the orbital's din x NP weight block in LDS
// (and reads h_{L-1} rows as 16-byte vectors, whole K steps of 16)
bool os_fwd_fits(int din, int Ne) {
    return din % 16 == 0 && (size_t)din * (Ne <= 16 ? 20 : 36) * sizeof(float) <= 160 * 1024;
}
int os_item() { return kOsItemMax; }

void launch_os_fwd(hipStream_t st, const float *hL, int din, const float *W, const float *bias, int width, int Ne,
                   const int4 *tiles, int64_t ntiles, const int32_t *ex, float *Osp) {
    if (ntiles == 0) return;
    const unsigned blocks = (unsigned)((ntiles + kOsFwdTiles - 1) / kOsFwdTiles);
    if (Ne <= 16)
        hipLaunchKernelGGL(k_os_fwd<16>, dim3(blocks), dim3(256), sizeof(float) * din * 20, st, hL, din, W, bias,
                           width, Ne, tiles, ntiles, ex, Osp);
    else
        hipLaunchKernelGGL(k_os_fwd<32>, dim3(blocks), dim3(256), sizeof(float) * din * 36, st, hL, din, W, bias,
                           width, Ne, tiles, ntiles, ex, Osp);
}

void launch_os_trans_w(hipStream_t st, const float *W, int din, int width, float *WT) {
    const int64_t tot = (int64_t)din * width;
    hipLaunchKernelGGL(k_os_trans_w, dim3(g1(tot)), dim3(256), 0, st, W, din, width, WT);
}

void launch_os_dgrad(hipStream_t st, int64_t n, int Ne, int din, const float *WT, const int4 *tiles, int64_t ntiles,
                     const float *dOsp, float *Cr, const float *dD, const int32_t *idx, const float *hL,
                     float *delta) {
    if (ntiles > 0) {
        if (Ne <= 16)
            hipLaunchKernelGGL(k_os_drows<16>, dim3((unsigned)ntiles), dim3(256), 0, st, WT, din, Ne, tiles, dOsp, Cr);
        else
            hipLaunchKernelGGL(k_os_drows<32>, dim3((unsigned)ntiles), dim3(256), 0, st, WT, din, Ne, tiles, dOsp, Cr);
    }
    hipLaunchKernelGGL(k_os_dsum, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, Ne, din, dD, Cr, idx, hL,
                       delta);
}

void launch_os_wgrad(hipStream_t st, const float *hL, int din, int Ne, const int4 *items, int64_t nitems,
                     const int32_t *ex, const float *dOsp, float *part, const int *dpos, const int *ifirst,
                     const int *icount, int No, float *grad) {
    if (nitems > 0) {
        const unsigned gy = (unsigned)((din + 1 + 255) / 256);
        if (Ne <= 16)
            hipLaunchKernelGGL(k_os_wgrad<16>, dim3((unsigned)nitems, gy), dim3(256),
                               (sizeof(float) * 16 + sizeof(int)) * kOsItemMax, st, hL, din, Ne, items, ex, dOsp, part);
        else
            hipLaunchKernelGGL(k_os_wgrad<32>, dim3((unsigned)nitems, gy), dim3(256),
                               (sizeof(float) * 32 + sizeof(int)) * kOsItemMax, st, hL, din, Ne, items, ex, dOsp, part);
    }
    const int64_t tot = (int64_t)(din + 1) * No * Ne;
    hipLaunchKernelGGL(k_os_wgrad_sum, dim3(g1(tot)), dim3(256), 0, st, part, din, Ne, No, dpos, ifirst, icount,
                       grad);
}

void launch_os_scatter(hipStream_t st, const float *GD, int din, int Ne, int nd, int width, const int *dorb,
                       float *grad) {
    const int64_t tot = (int64_t)(din + 1) * nd * Ne;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_os_scatter, dim3(g1(tot)), dim3(256), 0, st, GD, din, Ne, nd, width, dorb, grad);
}

}  // namespace dnqs
