// Split-BF16 MFMA GEMM for the mixed-precision form: C = epi(A B) with A, B and C in FP32
// in HBM, computed on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
//
// Each operand value x is split when it is staged into LDS as x_hi = bf16(x) and
// x_lo = bf16(x - x_hi), so x = x_hi + x_lo to about 2^-17 relative.  A product is taken
// as a_lo b_hi + a_hi b_lo + a_hi b_hi (the a_lo b_lo term, ~2^-18 relative, is dropped):
// three BF16 MFMAs per operand pair, FP32 accumulation.  A single BF16 product (operands
// rounded to 2^-9) moves the variational energy by a few 1e-5 Ha at the headline size;
// the split form keeps it near 1e-7 Ha at a sixth of the BF16 MFMA peak, which is still
// more than five times the FP32 MFMA peak.
//
// Tiles: TM x 128 per workgroup (TM = 128 or 64), K step 32; 4 waves as 2 x 2, each
// (TM/2) x 64 = WI x 2 MFMA tiles.  LDS holds the hi and lo parts of both operands
// k-contiguous ([row][k], rows padded by 8 bf16 so a wave's 16-byte fragment reads are
// free of bank conflicts); 40 KB per workgroup at TM = 128.  MFMA lane layout: A[i][k]
// comes from lane i + 32*(k/8), element k%8; B[k][j] from lane j + 32*(k/8); C/D rows
// 8*(r/4) + 4*(lane/32) + r%4, column lane%32.
//
// Operands are FP32 in either orientation: "k-contiguous" (row r, k at r*ld + k) or
// "row-contiguous" (k at k*ld + r).  The epilogues and the split-K / grouped-problem
// arguments are those of the FP32 MFMA GEMM (GemmArgs).
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

typedef float v16f_x __attribute__((ext_vector_type(16)));
typedef float v4f_x __attribute__((ext_vector_type(4)));
typedef __bf16 bf16_t;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));

constexpr int XBN = 128, XBK = 32, XPAD = 8;
constexpr int XLD = XBK + XPAD;  // bf16 per LDS row

__device__ __forceinline__ int xcd_remap_x(int L, int total) {
    const int nx = 8;
    int full = (total / nx) * nx;
    if (L >= full) return L;
    int per = total / nx;
    return (L % nx) * per + (L / nx);
}

__device__ __forceinline__ void split_bf16(float x, bf16_t &hi, bf16_t &lo) {
    hi = (bf16_t)x;
    lo = (bf16_t)(x - (float)hi);
}

// One operand tile: ROWS rows x 32 k of an FP32 matrix P into registers r[16]; threads
// t < 2*ROWS take part.
//   KC (k-contiguous, P[row*ld + k]):   thread = (row t/2, k 16*(t%2) .. +15)
//   !KC (row-contiguous, P[k*ld + row]): thread = (rows 4*(t%(ROWS/4)) .. +3,
//                                        k 4*(t/(ROWS/4)) .. +3), r[4*kk + rr] = P[k+kk][row+rr]
// Rows >= rows_ld and k >= kend read as 0; row `ones` (if >= 0) reads as 1 for k < kend.
template <bool KC, int ROWS>
__device__ __forceinline__ void xload(const float *__restrict__ P, int ld, int r0, int rows_ld, int ones, int k0,
                                      int kend, float (&r)[16]) {
    const int t = threadIdx.x;
    if (t >= 2 * ROWS) return;
    if (KC) {
        const int row = r0 + (t >> 1), k = k0 + (t & 1) * 16;
        const float *p = P + (int64_t)row * ld + k;
        if (row < rows_ld && k + 16 <= kend && (ld & 3) == 0 && ((((uintptr_t)p) & 15) == 0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const v4f_x u = *(const v4f_x *)(p + 4 * q);
                r[4 * q + 0] = u[0];
                r[4 * q + 1] = u[1];
                r[4 * q + 2] = u[2];
                r[4 * q + 3] = u[3];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) r[j] = (row < rows_ld && k + j < kend) ? p[j] : 0.0f;
        }
        if (row == ones) {
#pragma unroll
            for (int j = 0; j < 16; ++j) r[j] = (k + j < kend) ? 1.0f : 0.0f;
        }
    } else {
        const int row = r0 + 4 * (t % (ROWS / 4)), k = k0 + 4 * (t / (ROWS / 4));
        const bool vec = row + 4 <= rows_ld && (ld & 3) == 0 && ((((uintptr_t)(P + row)) & 15) == 0);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const float *p = P + (int64_t)(k + kk) * ld + row;
            if (k + kk < kend && vec) {
                const v4f_x u = *(const v4f_x *)p;
                r[4 * kk + 0] = u[0];
                r[4 * kk + 1] = u[1];
                r[4 * kk + 2] = u[2];
                r[4 * kk + 3] = u[3];
            } else {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) r[4 * kk + rr] = (k + kk < kend && row + rr < rows_ld) ? p[rr] : 0.0f;
            }
        }
        if (ones >= row && ones < row + 4) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) r[4 * kk + (ones - row)] = (k + kk < kend) ? 1.0f : 0.0f;
        }
    }
}

// Split the tile in r into the hi / lo LDS arrays ([row][k]).
template <bool KC, int ROWS>
__device__ __forceinline__ void xstore(bf16_t (*Hs)[XLD], bf16_t (*Ls)[XLD], const float (&r)[16]) {
    const int t = threadIdx.x;
    if (t >= 2 * ROWS) return;
    if (KC) {
        const int row = t >> 1, k = (t & 1) * 16;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            bf16x8_t h, l;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                bf16_t a, b;
                split_bf16(r[8 * q + j], a, b);
                h[j] = a;
                l[j] = b;
            }
            *(bf16x8_t *)&Hs[row][k + 8 * q] = h;
            *(bf16x8_t *)&Ls[row][k + 8 * q] = l;
        }
    } else {
        const int row = 4 * (t % (ROWS / 4)), k = 4 * (t / (ROWS / 4));
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            bf16x4_t h, l;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                bf16_t a, b;
                split_bf16(r[4 * kk + rr], a, b);
                h[kk] = a;
                l[kk] = b;
            }
            *(bf16x4_t *)&Hs[row + rr][k] = h;
            *(bf16x4_t *)&Ls[row + rr][k] = l;
        }
    }
}

// AK: A k-contiguous (A[m*lda + k]) else A[k*lda + m].  BNC: B n-contiguous
// (B[k*ldb + n], i.e. row-contiguous in the [n][k] view) else B[n*ldb + k].
template <bool AK, bool BNC, int EPI, int TM>
__global__ __launch_bounds__(256) void k_gemm_x3(GemmArgs g0) {
    constexpr int WI = TM / 64;
    GemmArgs g = g0;
    __shared__ __attribute__((aligned(16))) bf16_t Ah[TM][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Al[TM][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bh[XBN][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bl[XBN][XLD];
    const int tiles_n = (g.N + XBN - 1) / XBN;
    const int tiles_m = (g.M + TM - 1) / TM;
    const int L = xcd_remap_x(blockIdx.x, tiles_n * tiles_m);
    const int m0 = (L / tiles_n) * TM, n0 = (L % tiles_n) * XBN;
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
    const float *A = (const float *)g.A;
    const float *B = (const float *)g.B;
    const int mload = g.ones_row >= 0 ? g.ones_row : g.M;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 64;
    const int li = lane & 31, lk = (lane >> 5) * 8;

    v16f_x acc[WI][2];
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    float ra[16], rb[16];
    if (kbeg < kend) {
        xload<AK, TM>(A, g.lda, m0, mload, g.ones_row, kbeg, kend, ra);
        xload<!BNC, XBN>(B, g.ldb, n0, g.N, -1, kbeg, kend, rb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += XBK) {
        __syncthreads();
        xstore<AK, TM>(Ah, Al, ra);
        xstore<!BNC, XBN>(Bh, Bl, rb);
        __syncthreads();
        if (k0 + XBK < kend) {
            xload<AK, TM>(A, g.lda, m0, mload, g.ones_row, k0 + XBK, kend, ra);
            xload<!BNC, XBN>(B, g.ldb, n0, g.N, -1, k0 + XBK, kend, rb);
        }
#pragma unroll
        for (int ks = 0; ks < XBK; ks += 16) {
            bf16x8_t ah[WI], al[WI], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < WI; ++i) {
                ah[i] = *(const bf16x8_t *)&Ah[wm + 32 * i + li][ks + lk];
                al[i] = *(const bf16x8_t *)&Al[wm + 32 * i + li][ks + lk];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bh[j] = *(const bf16x8_t *)&Bh[wn + 32 * j + li][ks + lk];
                bl[j] = *(const bf16x8_t *)&Bl[wn + 32 * j + li][ks + lk];
            }
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
    }
    float *C = (float *)g.C + (int64_t)blockIdx.z * g.c_split_stride;
    const float *act = (const float *)g.act;
    const int lrow = (lane >> 5) * 4;
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn + j * 32 + li;
            if (col >= g.N) continue;
            const float bias = (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) ? g.bias[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + i * 32 + 8 * (r >> 2) + lrow + (r & 3);
                if (row >= g.M) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_BIAS) v += bias;
                if (EPI == EPI_BIAS_TANH) v = tanhf(v + bias);
                if (EPI == EPI_DTANH) {
                    const float hv = act[(int64_t)row * g.ldact + col];
                    v *= (1.0f - hv * hv);
                }
                C[(int64_t)row * g.ldc + col] = v;
            }
        }
}

template <bool AK, bool BNC, int EPI, int TM>
static void launch_x(hipStream_t st, GemmArgs g, int splits) {
    const int tiles = ((g.M + TM - 1) / TM) * ((g.N + XBN - 1) / XBN);
    hipLaunchKernelGGL((k_gemm_x3<AK, BNC, EPI, TM>), dim3(tiles, 1, splits), dim3(256), 0, st, g);
}

int gemm_x3_kstep() { return XBK; }

void launch_gemm_x3(hipStream_t st, const GemmArgs &g0, bool a_kcontig, bool b_ncontig, int epi, int splits,
                    int tm) {
    GemmArgs g = g0;
    if (splits < 1) splits = 1;
    int chunk = (g.K + splits - 1) / splits;
    chunk = (chunk + XBK - 1) / XBK * XBK;
    g.k_chunk = chunk > 0 ? chunk : XBK;
#define DISPATCH_TM(AK, BNC, EPI)                    \
    if (tm == 64)                                    \
        launch_x<AK, BNC, EPI, 64>(st, g, splits);   \
    else                                             \
        launch_x<AK, BNC, EPI, 128>(st, g, splits);
#define DISPATCH(AK, BNC)                                              \
    switch (epi) {                                                     \
        case EPI_STORE: DISPATCH_TM(AK, BNC, EPI_STORE) break;         \
        case EPI_BIAS: DISPATCH_TM(AK, BNC, EPI_BIAS) break;           \
        case EPI_BIAS_TANH: DISPATCH_TM(AK, BNC, EPI_BIAS_TANH) break; \
        case EPI_DTANH: DISPATCH_TM(AK, BNC, EPI_DTANH) break;         \
    }
    if (a_kcontig && b_ncontig) { DISPATCH(true, true) }
    else if (a_kcontig && !b_ncontig) { DISPATCH(true, false) }
    else if (!a_kcontig && b_ncontig) { DISPATCH(false, true) }
    else { DISPATCH(false, false) }
#undef DISPATCH
#undef DISPATCH_TM
}

}  // namespace dnqs
