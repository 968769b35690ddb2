// Network kernels for the neural backflow amplitude (Eqs. 2-4) and its adjoint.
//
//   k_embed     h1 = tanh(b1 + sum_{p in occ(x)} W1[p,:])      (layer 1 on 0/1 input;
//               k_embed_tiled for one weight set, LDS-staged)
//   k_gemm_f32  C = epi(A B) on MFMA v_mfma_f32_32x32x2f32, 128x128 tiles, fused
//               epilogues: +bias, tanh(+bias), *(1 - h^2); split-K for weight grads
//   k_orb_lu    A(x) = Phi0[occ] + O[x, occ] -> Gauss-Jordan with partial pivoting,
//               row per lane (rows stay put, positions are exchanged), log|det| in
//               FP64, sign, and A^-1 for the adjoint
//   k_det_bwd   dL/dO[x, p*Ne+k] = c_x (A_x^-T)[j,k] for p = i_j, 0 elsewhere,
//               c_x = 2 (v_x - E psi_x) psi_x / psi^T psi            (Eq. 12)
//   (both also take the occupied-row layout of the output layer, k_outsplit.hip)
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ embedding
constexpr int kEmbedCfg = 4;  // configurations per workgroup

__global__ __launch_bounds__(256) void k_embed(const uint64_t *__restrict__ dets, int64_t n, int M, int d1,
                                               const float *__restrict__ W1g, const float *__restrict__ b1g,
                                               float *__restrict__ h1, float *__restrict__ U, RowProblems rp,
                                               int64_t offW1, int64_t offb1) {
    const int No = 2 * M;
    for (int i = 0; i < kEmbedCfg; ++i) {
        const int64_t x = (int64_t)blockIdx.x * kEmbedCfg + i;
        if (x >= n) return;
        const float *W1 = W1g, *b1 = b1g;
        if (rp.pid) {
            const float *th = rp.P[rp.pid[x]].theta;
            W1 = th + offW1;
            b1 = th + offb1;
        }
        const uint64_t a = dets[2 * x], b = dets[2 * x + 1];
        for (int c = threadIdx.x; c < d1; c += blockDim.x) {
            // rows of the occupied spin-orbitals, ascending (alpha, then beta), eight
            // reads in flight at a time (an exhausted slot reads row 0 and is not added)
            float s = b1[c];
            uint64_t t = a;
            int base = 0;
            for (int half = 0; half < 2; ++half) {
                while (t) {
                    int pp[8];
                    bool ok[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        ok[u] = t != 0;
                        pp[u] = ok[u] ? base + ctz64(t) : 0;
                        t &= t - 1;
                    }
                    float v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = W1[(size_t)pp[u] * d1 + c];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (ok[u]) s += v[u];
                }
                t = b;
                base = M;
            }
            h1[x * d1 + c] = tanhf(s);
        }
        if (U) {
            for (int p = threadIdx.x; p < No; p += blockDim.x) {
                uint64_t w = p < M ? a : b;
                int q = p < M ? p : p - M;
                U[x * No + p] = (float)((w >> q) & 1ull);
            }
        }
    }
}

// One weight set: a workgroup takes 128 columns of h1 for kEmbedTileCfg configurations and
// stages those columns of W1 (N_o x 128) in LDS once, so that W1 is read from L2 once per
// workgroup rather than once per configuration; each wave takes one configuration at a
// time (its occupied orbitals are uniform over the wave), two adjacent columns per lane
// (the kernel is VALU-bound: the per-configuration gather arithmetic is shared by two
// outputs).  Same sums, same order as k_embed.
constexpr int kEmbedTileCols = 128, kEmbedTileCfg = 64;  // two columns per lane

__global__ __launch_bounds__(256) void k_embed_tiled(const uint64_t *__restrict__ dets, int64_t n, int M, int d1,
                                                     const float *__restrict__ W1, const float *__restrict__ b1,
                                                     float *__restrict__ h1, float *__restrict__ U) {
    extern __shared__ float Ws[];  // [N_o][128]
    __shared__ uint64_t Ds[2 * kEmbedTileCfg];
    __shared__ unsigned char Ps[kEmbedTileCfg][128];  // occupied spin-orbitals, ascending
    const int No = 2 * M;
    const int c0 = blockIdx.y * kEmbedTileCols;
    const int64_t x0 = (int64_t)blockIdx.x * kEmbedTileCfg;
    // the tile's configurations and W1 columns, eight reads in flight per thread
    for (int i = threadIdx.x; i < 2 * kEmbedTileCfg; i += blockDim.x)
        Ds[i] = x0 + i / 2 < n ? dets[2 * x0 + i] : 0ull;
    const int tot = No * kEmbedTileCols;
    for (int i0 = threadIdx.x; i0 < tot; i0 += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            const int p = i / kEmbedTileCols, c = c0 + i % kEmbedTileCols;
            v[u] = W1[(size_t)(i < tot ? p : 0) * d1 + (c < d1 ? c : 0)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < tot) Ws[i] = c0 + i % kEmbedTileCols < d1 ? v[u] : 0.0f;
        }
    }
    __syncthreads();
    // occupied lists by rank, one (configuration, spin-orbital) pair per thread (vector
    // work: a scalar bit loop per configuration would queue on the CU's one scalar unit);
    // the occupation vector U is written here too
    for (int i = threadIdx.x; i < kEmbedTileCfg * No; i += blockDim.x) {
        const int j = i / No, p = i % No;
        if (x0 + j >= n) continue;
        const uint64_t a = Ds[2 * j], b = Ds[2 * j + 1];
        const uint64_t w = p < M ? a : b;
        const int q = p < M ? p : p - M;
        const bool occ = (w >> q) & 1ull;
        if (occ) {
            const uint64_t below = (1ull << q) - 1ull;
            const int rank = p < M ? popc64(a & below) : popc64(a) + popc64(b & below);
            Ps[j][rank] = (unsigned char)p;
        }
        if (U && blockIdx.y == 0) U[(x0 + j) * No + p] = occ ? 1.0f : 0.0f;
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int c = c0 + 2 * lane;  // this lane's two columns c, c + 1 (d1 is even)
    const float bc0 = c < d1 ? b1[c] : 0.0f, bc1 = c + 1 < d1 ? b1[c + 1] : 0.0f;
    for (int j = wave; j < kEmbedTileCfg; j += blockDim.x / kWave) {
        const int64_t x = x0 + j;
        if (x >= n) break;
        const int ne = popc64(Ds[2 * j]) + popc64(Ds[2 * j + 1]);
        // occupied rows ascending (alpha, then beta), eight LDS reads in flight at a time
        float s0 = bc0, s1 = bc1;
        for (int r0 = 0; r0 < ne; r0 += 8) {
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = *reinterpret_cast<const float2 *>(
                    Ws + (r0 + u < ne ? Ps[j][r0 + u] : 0) * kEmbedTileCols + 2 * lane);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (r0 + u < ne) {
                    s0 += v[u].x;
                    s1 += v[u].y;
                }
        }
        if (c + 1 < d1) {
            *reinterpret_cast<float2 *>(h1 + x * d1 + c) = make_float2(tanhf(s0), tanhf(s1));
        } else if (c < d1) {
            h1[x * d1 + c] = tanhf(s0);
        }
    }
}

void launch_embed(hipStream_t st, const uint64_t *dets, int64_t n, int M, int d1, const float *W1, const float *b1,
                  float *h1, float *U, RowProblems rp, int64_t offW1, int64_t offb1) {
    if (n <= 0) return;
    if (!rp.pid && d1 % 2 == 0) {
        dim3 grid((unsigned)((n + kEmbedTileCfg - 1) / kEmbedTileCfg),
                  (unsigned)((d1 + kEmbedTileCols - 1) / kEmbedTileCols));
        hipLaunchKernelGGL(k_embed_tiled, grid, dim3(256), sizeof(float) * 2 * M * kEmbedTileCols, st, dets, n, M, d1,
                           W1, b1, h1, U);
        return;
    }
    dim3 grid((unsigned)((n + kEmbedCfg - 1) / kEmbedCfg));
    hipLaunchKernelGGL(k_embed, grid, dim3(256), 0, st, dets, n, M, d1, W1, b1, h1, U, rp, offW1, offb1);
}

// ------------------------------------------------------------------ FP32 MFMA GEMM
constexpr int BN = 128, BK = 16;
constexpr int LDS_B = BN + 4;

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap the linear id so that
// consecutive logical tiles (which share an A row-tile) land on the same XCD and hit
// its L2.
__device__ __forceinline__ int xcd_remap(int L, int total) {
    const int nx = 8;
    int full = (total / nx) * nx;
    if (L >= full) return L;
    int per = total / nx;
    return (L % nx) * per + (L / nx);
}

// 8 consecutive floats at p; `ok(j)` says whether element j is in range.  Vector loads
// when all 8 are in range and the address is 16-byte aligned.
template <typename OK>
__device__ __forceinline__ void load8(const float *p, bool full, OK ok, float (&r)[8]) {
    if (full && ((((uintptr_t)p) & 15) == 0)) {
        const v4f u = *(const v4f *)p, w = *(const v4f *)(p + 4);
        r[0] = u[0]; r[1] = u[1]; r[2] = u[2]; r[3] = u[3];
        r[4] = w[0]; r[5] = w[1]; r[6] = w[2]; r[7] = w[3];
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = ok(j) ? p[j] : 0.0f;
    }
}

// A tile (TM rows m x BK k) into registers: threads t < 2*TM take 8 elements each.
template <bool A_KCONTIG, int TM>
__device__ __forceinline__ void load_a_tile(const GemmArgs &g, int m0, int k0, int kend, float (&r)[8]) {
    const int t = threadIdx.x;
    if (t >= 2 * TM) return;
    const int mload = g.ones_row >= 0 ? g.ones_row : g.M;
    const float *A = (const float *)g.A;
    if (A_KCONTIG) {  // A[m*lda + k]; thread: one m, 8 consecutive k
        const int m = m0 + (t >> 1), k = k0 + (t & 1) * 8;
        const float *p = A + (int64_t)m * g.lda + k;
        const bool full = m < mload && k + 8 <= kend && (g.lda & 3) == 0;
        load8(p, full, [&](int j) { return m < mload && k + j < kend; }, r);
        if (m == g.ones_row) {
#pragma unroll
            for (int j = 0; j < 8; ++j) r[j] = (k + j < kend) ? 1.0f : 0.0f;
        }
    } else {  // A[k*lda + m]; thread: one k, 8 consecutive m
        const int k = k0 + t / (TM / 8), m = m0 + (t % (TM / 8)) * 8;
        const float *p = A + (int64_t)k * g.lda + m;
        const bool full = k < kend && m + 8 <= mload && (g.lda & 3) == 0;
        load8(p, full, [&](int j) { return k < kend && m + j < mload; }, r);
        if (g.ones_row >= 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (m + j == g.ones_row) r[j] = k < kend ? 1.0f : 0.0f;
        }
    }
}

template <bool A_KCONTIG, int TM>
__device__ __forceinline__ void store_a_tile(float (*As)[TM + 4], const float (&r)[8]) {
    const int t = threadIdx.x;
    if (t >= 2 * TM) return;
    if (A_KCONTIG) {
        const int m = t >> 1, k = (t & 1) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) As[k + j][m] = r[j];
    } else {
        const int k = t / (TM / 8), m = (t % (TM / 8)) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) As[k][m + j] = r[j];
    }
}

template <bool B_NCONTIG>
__device__ __forceinline__ void load_b_tile(const GemmArgs &g, int n0, int k0, int kend, float (&r)[8]) {
    const int t = threadIdx.x;
    const float *B = (const float *)g.B;
    if (B_NCONTIG) {  // B[k*ldb + n]
        const int k = k0 + (t >> 4), n = n0 + (t & 15) * 8;
        const float *p = B + (int64_t)k * g.ldb + n;
        const bool full = k < kend && n + 8 <= g.N && (g.ldb & 3) == 0;
        load8(p, full, [&](int j) { return k < kend && n + j < g.N; }, r);
    } else {  // B[n*ldb + k]
        const int n = n0 + (t >> 1), k = k0 + (t & 1) * 8;
        const float *p = B + (int64_t)n * g.ldb + k;
        const bool full = n < g.N && k + 8 <= kend && (g.ldb & 3) == 0;
        load8(p, full, [&](int j) { return n < g.N && k + j < kend; }, r);
    }
}

template <bool B_NCONTIG>
__device__ __forceinline__ void store_b_tile(float (*Bs)[LDS_B], const float (&r)[8]) {
    const int t = threadIdx.x;
    if (B_NCONTIG) {
        const int k = t >> 4, n = (t & 15) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[k][n + j] = r[j];
    } else {
        const int n = t >> 1, k = (t & 1) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[k + j][n] = r[j];
    }
}

// FP32 MFMA GEMM, operands and output in FP32.  Tile TM x 128 (TM = 128 or 64); the
// four waves are 2 x 2, each (TM/2) x 64 = WI x 2 MFMA blocks of 32 x 32.
template <bool A_KCONTIG, bool B_NCONTIG, int EPI, int TM>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g0) {
    constexpr int WI = TM / 64;
    GemmArgs g = g0;
    __shared__ float As[BK][TM + 4];
    __shared__ float Bs[BK][LDS_B];
    const int tiles_n = (g.N + BN - 1) / BN;
    const int tiles_m = (g.M + TM - 1) / TM;
    const int L = xcd_remap(blockIdx.x, tiles_n * tiles_m);
    const int m0 = (L / tiles_n) * TM, n0 = (L % tiles_n) * BN;
    if (g.tile_pid) {
        const int pg = g.tile_pid[(int64_t)(L / tiles_n) * TM / 128];
        g.B = g.Bg[pg];
        if (g.biasg) g.bias = g.biasg[pg];
    }
    int kbeg = blockIdx.z * g.k_chunk;
    int kend = kbeg + g.k_chunk;
    if (g.ksplit) {
        kbeg = g.ksplit[blockIdx.z].x;
        kend = g.ksplit[blockIdx.z].y;
    }
    if (kend > g.K) kend = g.K;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 64;
    const int li = lane & 31, lk = lane >> 5;

    v16f acc[WI][2];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    float ra[8], rb[8];
    if (kbeg < kend) {
        load_a_tile<A_KCONTIG, TM>(g, m0, kbeg, kend, ra);
        load_b_tile<B_NCONTIG>(g, n0, kbeg, kend, rb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store_a_tile<A_KCONTIG, TM>(As, ra);
        store_b_tile<B_NCONTIG>(Bs, rb);
        __syncthreads();
        if (k0 + BK < kend) {
            load_a_tile<A_KCONTIG, TM>(g, m0, k0 + BK, kend, ra);
            load_b_tile<B_NCONTIG>(g, n0, k0 + BK, kend, rb);
        }
#pragma unroll
        for (int kk = 0; kk < BK / 2; ++kk) {
            float a[WI];
#pragma unroll
            for (int i = 0; i < WI; ++i) a[i] = As[2 * kk + lk][wm + 32 * i + li];
            const float b0 = Bs[2 * kk + lk][wn + li];
            const float b1 = Bs[2 * kk + lk][wn + 32 + li];
#pragma unroll
            for (int i = 0; i < WI; ++i) {
                acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b0, acc[i][0], 0, 0, 0);
                acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b1, acc[i][1], 0, 0, 0);
            }
        }
    }
    float *C = (float *)g.C + (int64_t)blockIdx.z * g.c_split_stride;
    const float *act = (const float *)g.act;
    if (m0 + TM <= g.M && n0 + BN <= g.N) {
        // interior tile (uniform): no bounds tests; each lane's 16 rows of a block sit at
        // fixed multiples of ld from its first row, so only one 64-bit address per block
        const int64_t ldc = g.ldc, lda_ = g.ldact;
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = n0 + wn + j * 32 + li;
                const int64_t row0 = m0 + wm + i * 32 + 4 * lk;
                float fac[16];
                if (EPI == EPI_DTANH) {
                    const float *ap = act + row0 * lda_ + col;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float hv = ap[(int64_t)(8 * (r >> 2) + (r & 3)) * lda_];
                        fac[r] = 1.0f - hv * hv;
                    }
                }
                const float bias = (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) ? g.bias[col] : 0.0f;
                float *cp = C + row0 * ldc + col;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float v = acc[i][j][r];
                    if (EPI == EPI_BIAS) v += bias;
                    if (EPI == EPI_BIAS_TANH) v = tanhf(v + bias);
                    if (EPI == EPI_DTANH) v *= fac[r];
                    cp[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] = v;
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn + j * 32 + li;
            // tanh' factors first, as one batch of in-range loads (clamped indices), so
            // that the 16 reads overlap instead of each waiting before its store
            float fac[16];
            if (EPI == EPI_DTANH) {
                const int cc = col < g.N ? col : g.N - 1;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                    const float hv = act[(int64_t)(row < g.M ? row : g.M - 1) * g.ldact + cc];
                    fac[r] = 1.0f - hv * hv;
                }
            }
            if (col >= g.N) continue;
            float bias = (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) ? g.bias[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (row >= g.M) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_BIAS) v += bias;
                if (EPI == EPI_BIAS_TANH) v = tanhf(v + bias);
                if (EPI == EPI_DTANH) v *= fac[r];
                C[(int64_t)row * g.ldc + col] = v;
            }
        }
}

template <bool AK, bool BN_, int EPI, int TM>
static void launch_gemm_t(hipStream_t st, const GemmArgs &g, int splits) {
    int tiles = ((g.M + TM - 1) / TM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((k_gemm_f32<AK, BN_, EPI, TM>), dim3(tiles, 1, splits), dim3(256), 0, st, g);
}

static int split_chunk(int K, int splits) {
    int chunk = (K + splits - 1) / splits;
    chunk = (chunk + BK - 1) / BK * BK;
    return chunk > 0 ? chunk : BK;
}

void launch_gemm_f32(hipStream_t st, const GemmArgs &g0, bool a_kcontig, bool b_ncontig, int epi, int splits,
                     int tm) {
    GemmArgs g = g0;
    if (splits < 1) splits = 1;
    // a chunk given by the caller (a multiple of BK) fixes the split ranges
    g.k_chunk = g0.k_chunk > 0 ? g0.k_chunk : split_chunk(g.K, splits);
#define DISPATCH_TM(AK, BNC, EPI)                                           \
    if (tm == 64)                                                           \
        launch_gemm_t<AK, BNC, EPI, 64>(st, g, splits);                     \
    else                                                                    \
        launch_gemm_t<AK, BNC, EPI, 128>(st, g, splits);
#define DISPATCH(AK, BNC)                                                   \
    switch (epi) {                                                          \
        case EPI_STORE: DISPATCH_TM(AK, BNC, EPI_STORE) break;              \
        case EPI_BIAS: DISPATCH_TM(AK, BNC, EPI_BIAS) break;                \
        case EPI_BIAS_TANH: DISPATCH_TM(AK, BNC, EPI_BIAS_TANH) break;      \
        case EPI_DTANH: DISPATCH_TM(AK, BNC, EPI_DTANH) break;              \
    }
    if (a_kcontig && b_ncontig) { DISPATCH(true, true) }
    else if (a_kcontig && !b_ncontig) { DISPATCH(true, false) }
    else if (!a_kcontig && b_ncontig) { DISPATCH(false, true) }
    else { DISPATCH(false, false) }
#undef DISPATCH
#undef DISPATCH_TM
}

// out[i] = sum_z part[z*count + i], fixed order
__global__ void k_reduce_splits(const float *__restrict__ part, int splits, int64_t count, float *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        // eight partials read together, then added in split order (the same sum as a
        // plain loop over z, without one memory round trip per split)
        float s = 0.0f;
        int z = 0;
        for (; z + 8 <= splits; z += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * count + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; z < splits; ++z) s += part[(int64_t)z * count + i];
        out[i] = s;
    }
}

void launch_reduce_splits(hipStream_t st, const float *part, int splits, int64_t count, float *out) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)blocks), dim3(256), 0, st, part, splits, count, out);
}

// out[i] (+)= the splits' partials added in split order onto out[i] (0 for the first
// fold): folding the splits block by block gives the bits of one k_reduce_splits over
// all of them, since that sum is also taken left to right starting from 0.
__global__ void k_fold_splits(const float *__restrict__ part, int splits, int64_t count, float *__restrict__ out,
                              int accumulate) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        float s = accumulate ? out[i] : 0.0f;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
        out[i] = s;
    }
}

void launch_fold_splits(hipStream_t st, const float *part, int splits, int64_t count, float *out, bool accumulate) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fold_splits, dim3((unsigned)blocks), dim3(256), 0, st, part, splits, count, out,
                       accumulate ? 1 : 0);
}

// ------------------------------------------------------------------ orbital rows + LU
// spin-orbital index of the r-th occupied spin-orbital (ascending), alpha block first
__device__ __forceinline__ int occupied_so(uint64_t a, uint64_t b, int M, int na, int r) {
    uint64_t s = r < na ? a : b;
    int k = r < na ? r : r - na;
    for (int i = 0; i < k; ++i) s &= s - 1;
    int p = ctz64(s);
    return r < na ? p : M + p;
}

// G lanes per configuration; lane r of a group holds row r of [A | I] (its row position
// changes with the pivoting, the data stays in the lane).
template <int G>
__global__ __launch_bounds__(256) void k_orb_lu(const uint64_t *__restrict__ dets, int64_t n, int M, int na, int nb,
                                                const float *__restrict__ O, const float *__restrict__ Phi0g,
                                                double *__restrict__ logabs, int8_t *__restrict__ sign,
                                                float *__restrict__ Ainv, RowProblems rp, int64_t offPhi0,
                                                OutSplit os) {
    const int Ne = na + nb, No = 2 * M;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t x = gt / G;
    const int r = (int)(gt % G);
    const bool live = x < n;
    const bool row_live = live && r < Ne;
    float a[G], inv[G];
#pragma unroll
    for (int c = 0; c < G; ++c) {
        a[c] = 0.0f;
        inv[c] = (c == r && row_live) ? 1.0f : 0.0f;
    }
    if (row_live) {
        const uint64_t da = dets[2 * x], db = dets[2 * x + 1];
        const int p = occupied_so(da, db, M, na, r);
        const float *orow;
        if (os.idx) {
            const int dp = os.dpos[p];
            orow = dp >= 0 ? os.OD + x * (int64_t)(os.nd * Ne) + (int64_t)dp * Ne
                           : os.Osp + (int64_t)os.idx[x * Ne + r] * Ne;
        } else {
            orow = O + x * (int64_t)(No * Ne) + (int64_t)p * Ne;
        }
        const float *Phi0 = rp.pid ? rp.P[rp.pid[x]].theta + offPhi0 : Phi0g;
        const float *prow = Phi0 + (int64_t)p * Ne;
#pragma unroll
        for (int c = 0; c < G; ++c)
            if (c < Ne) a[c] = prow[c] + orow[c];
    }
    // Rows stay in their lanes: vpos is the row position a lane would hold after the
    // partial-pivoting row exchanges, and only vpos is exchanged (the pivot row is
    // broadcast from wherever it lives).  Same pivots, same arithmetic as exchanging the
    // rows; half the cross-lane traffic.  |det| is kept as an FP64 mantissa and binary
    // exponent (one log at the end).
    int vpos = r;
    double mant = 1.0;
    int expo = 0;
    int sgn = 1;
    bool singular = false;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        if (k >= Ne) continue;  // uniform; keeps the loop fully unrolled
        // partial pivoting: largest |a[k]| among rows at positions >= k, lowest position on
        // ties; key = position * 64 + lane
        float cand = (vpos >= k && vpos < Ne) ? fabsf(a[k]) : -1.0f;
        int ci = vpos * 64 + r;
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) {
            float oc = __shfl_xor(cand, o, G);
            int oi = __shfl_xor(ci, o, G);
            if (oc > cand || (oc == cand && oi < ci)) {
                cand = oc;
                ci = oi;
            }
        }
        const int pv = ci >> 6, plane = ci & 63;  // pivot row's position and lane
        if (pv != k) sgn = -sgn;
        if (r == plane) vpos = k;
        else if (vpos == k) vpos = pv;
        float pa[G], pi[G];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            pa[c] = __shfl(a[c], plane, G);
            pi[c] = __shfl(inv[c], plane, G);
        }
        float d = pa[k];
        if (d == 0.0f) {
            singular = true;
            d = 1.0f;
        } else {
            mant *= fabs((double)d);
            int e;
            mant = frexp(mant, &e);
            expo += e;
            if (d < 0.0f) sgn = -sgn;
        }
        const float rd = 1.0f / d;
        if (r == plane) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                a[c] = pa[c] * rd;
                inv[c] = pi[c] * rd;
            }
        } else {
            const float f = a[k] * rd;
#pragma unroll
            for (int c = 0; c < G; ++c) {
                a[c] = fmaf(-f, pa[c], a[c]);
                inv[c] = fmaf(-f, pi[c], inv[c]);
            }
        }
    }
    if (live && r == 0) {
        logabs[x] = singular ? -INFINITY : log(mant) + (double)expo * 0.69314718055994530942;
        sign[x] = singular ? (int8_t)0 : (int8_t)sgn;
    }
    if (Ainv && row_live) {  // row vpos of A^-1
        float *out = Ainv + x * (int64_t)(Ne * Ne) + (int64_t)vpos * Ne;
#pragma unroll
        for (int c = 0; c < G; ++c)
            if (c < Ne) out[c] = singular ? 0.0f : inv[c];
    }
}

int orb_lu_group(int ne) { return ne <= 8 ? 8 : ne <= 16 ? 16 : ne <= 32 ? 32 : 0; }

void launch_orb_lu(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const float *O,
                   const float *Phi0, double *logabs, int8_t *sign, float *Ainv, RowProblems rp, int64_t offPhi0,
                   OutSplit os) {
    const int G = orb_lu_group(na + nb);
    const int64_t threads = n * G;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (G == 8)
        hipLaunchKernelGGL(k_orb_lu<8>, dim3(blocks), dim3(256), 0, st, dets, n, M, na, nb, O, Phi0, logabs, sign,
                           Ainv, rp, offPhi0, os);
    else if (G == 16)
        hipLaunchKernelGGL(k_orb_lu<16>, dim3(blocks), dim3(256), 0, st, dets, n, M, na, nb, O, Phi0, logabs, sign,
                           Ainv, rp, offPhi0, os);
    else
        hipLaunchKernelGGL(k_orb_lu<32>, dim3(blocks), dim3(256), 0, st, dets, n, M, na, nb, O, Phi0, logabs, sign,
                           Ainv, rp, offPhi0, os);
}

// ------------------------------------------------------------------ det backward + scatter
// dO[x][p*Ne+k] = c_x * Ainv_x[k][j] if p = i_j is occupied, else 0
constexpr int kBwdCfg = 4;

__global__ __launch_bounds__(256) void k_det_bwd(const uint64_t *__restrict__ dets, int64_t n, int M, int na,
                                                 int nb, const double *__restrict__ psi,
                                                 const double *__restrict__ v, const double *__restrict__ energy,
                                                 const double *__restrict__ stats, const float *__restrict__ Ainv,
                                                 float *__restrict__ dO, RowProblems rp, OutSplit os) {
    const int Ne = na + nb, No = 2 * M;
    const int width = No * Ne, wd = os.nd * Ne;
    // the block's configurations' bit strings, psi and v read together up front (index
    // clamped to the last configuration), rather than one round trip per configuration
    uint64_t da[kBwdCfg], db[kBwdCfg];
    double pxs[kBwdCfg], vs[kBwdCfg];
#pragma unroll
    for (int i = 0; i < kBwdCfg; ++i) {
        const int64_t x = (int64_t)blockIdx.x * kBwdCfg + i;
        const int64_t xc = x < n ? x : n - 1;
        da[i] = dets[2 * xc];
        db[i] = dets[2 * xc + 1];
        pxs[i] = psi[xc];
        vs[i] = v[xc];
    }
#pragma unroll
    for (int i = 0; i < kBwdCfg; ++i) {
        const int64_t x = (int64_t)blockIdx.x * kBwdCfg + i;
        if (x >= n) return;
        double E, norm;
        bool pad = false;
        if (rp.pid) {
            const ProbDev &P = rp.P[rp.pid[x]];
            E = P.energy[0];
            norm = P.stats[0];
            pad = x - P.off >= P.n;
        } else {
            E = energy[0];
            norm = stats[0];
        }
        const bool ok = norm > 0.0 && isfinite(E) && !pad;
        const uint64_t a = da[i], b = db[i];
        const double px = pxs[i];
        const float c = ok ? (float)(2.0 * (vs[i] - E * px) * px / norm) : 0.0f;
        const float *ai = Ainv + x * (int64_t)(Ne * Ne);
        if (os.idx) {
            // sparse rows: dOsp[e][k] = c Ainv[k][j] for row j held as entry e
            for (int t = threadIdx.x; t < Ne * Ne; t += blockDim.x) {
                const int j = t / Ne, k = t % Ne;
                const int e = os.idx[x * Ne + j];
                if (e >= 0) os.dOsp[(int64_t)e * Ne + k] = c * ai[k * Ne + j];
            }
        }
        if (os.idx) {
            // the dense orbitals' columns, compact
            for (int t = threadIdx.x; t < wd; t += blockDim.x) {
                const int p = os.dorb[t / Ne], k = t % Ne;
                float out = 0.0f;
                const uint64_t s = p < M ? a : b;
                const int q = p < M ? p : p - M;
                if ((s >> q) & 1ull) {
                    const int j = (p < M ? 0 : na) + popc64(s & ((1ull << q) - 1ull));
                    out = c * ai[k * Ne + j];
                }
                os.dOD[x * wd + t] = out;
            }
        }
        if (!dO) continue;
        for (int t = threadIdx.x; t < width; t += blockDim.x) {
            const int p = t / Ne, k = t % Ne;
            float out = 0.0f;
            const uint64_t s = p < M ? a : b;
            const int q = p < M ? p : p - M;
            if ((s >> q) & 1ull) {
                const int j = (p < M ? 0 : na) + popc64(s & ((1ull << q) - 1ull));
                out = c * ai[k * Ne + j];
            }
            dO[x * width + t] = out;
        }
    }
}

void launch_det_bwd(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const double *psi,
                    const double *v, const double *energy, const double *stats, const float *Ainv, float *dO,
                    RowProblems rp, OutSplit os) {
    hipLaunchKernelGGL(k_det_bwd, dim3((unsigned)((n + kBwdCfg - 1) / kBwdCfg)), dim3(256), 0, st, dets, n, M, na,
                       nb, psi, v, energy, stats, Ainv, dO, rp, os);
}

// y[i] = x[i]
__global__ void k_copy_f32(const float *__restrict__ x, float *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

void launch_copy_f32(hipStream_t st, const float *x, float *y, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
}

}  // namespace dnqs
