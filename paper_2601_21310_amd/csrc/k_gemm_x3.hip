// Split-BF16 MFMA GEMM for the mixed-precision form: C = epi(A B) with A, B and C in FP32
// in HBM, computed on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
//
// Each operand value x is split as x_hi = bf16(x) and x_lo = bf16(x - x_hi), so
// x = x_hi + x_lo to about 2^-17 relative.  A product is taken as
// a_lo b_hi + a_hi b_lo + a_hi b_hi (the a_lo b_lo term, ~2^-18 relative, is dropped):
// three BF16 MFMAs per operand pair, FP32 accumulation.  A single BF16 product (operands
// rounded to 2^-9) moves the variational energy by a few 1e-5 Ha at the headline size;
// the split form keeps it near 1e-7 Ha at a sixth of the BF16 MFMA peak, which is still
// more than five times the FP32 MFMA peak.
//
// Tiles: TM x 128 per workgroup (TM = 128 or 64), K step 32; 4 waves as 2 x 2, each
// (TM/2) x 64 = WI x 2 MFMA tiles.  LDS holds the hi and lo parts of both operands
// k-contiguous ([row][k], rows padded by 8 bf16 so a wave's 16-byte fragment reads are
// free of bank conflicts), double-buffered: 80 KB per workgroup at TM = 128, one
// barrier per K step; global loads are issued two K steps before their data is staged,
// so that a step's MFMAs (768 cycles per wave) hide most of the memory latency.
// MFMA lane layout: A[i][k] comes from lane i + 32*(k/8), element k%8; B[k][j] from lane
// j + 32*(k/8); C/D rows 8*(r/4) + 4*(lane/32) + r%4, column lane%32.
//
// Operands are FP32 in either orientation, "k-contiguous" (row r, k at r*ld + k) or
// "row-contiguous" (k at k*ld + r), split while staged into LDS; or, for B only, BF16
// hi / lo planes split once beforehand (weights), staged by plain copies.  The epilogues
// and the split-K / grouped-problem arguments are those of the FP32 MFMA GEMM.
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

// tanh for the mixed form's hidden layers: tanh x = sign(x) (1 - e) / (1 + e) with
// e = exp(-2|x|) = 2^(-2 log2(e) |x|) in (0, 1], on the hardware exp2 and reciprocal
// (about 1 ulp each), so the absolute error stays near 1e-7, well below the 2^-17
// relative error of the split products that consume it.
__device__ __forceinline__ float tanh_mixed(float x) {
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(x));
    return copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
}

__device__ __forceinline__ void split_bf16(float x, bf16_t &hi, bf16_t &lo) {
    hi = (bf16_t)x;
    lo = (bf16_t)(x - (float)hi);
}

// One FP32 operand tile: ROWS rows x 32 k of P into registers r[16]; threads t < 2*ROWS
// take part.
//   KC (k-contiguous, P[row*ld + k]):   thread = (row t/2, k 16*(t%2) .. +15)
//   !KC (row-contiguous, P[k*ld + row]): thread = (rows 4*(t/8) .. +3, k 4*(t%8) .. +3),
//                                        r[4*kk + rr] = P[k+kk][row+rr]
// (in the !KC mapping eight consecutive lanes cover the 32 k of four rows, so their
// 8-byte LDS writes fall on distinct banks.)
// Rows >= rows_ld and k >= kend read as 0; row `ones` (if >= 0) reads as 1 for k < kend.
template <bool KC, int ROWS>
__device__ __forceinline__ void xload(const float *__restrict__ P, int64_t ld, int r0, int rows_ld, int ones, int k0,
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
        const int row = r0 + 4 * (t >> 3), k = k0 + 4 * (t & 7);
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
        const int row = 4 * (t >> 3), k = 4 * (t & 7);
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

// A pre-split B tile (128 rows n x 32 k of the hi and lo planes): thread = (n t/2,
// k 16*(t%2) .. +15), 16 hi and 16 lo values.
struct PreTile {
    bf16x8_t h0, h1, l0, l1;
};

__device__ __forceinline__ void pload(const bf16_t *__restrict__ hi, const bf16_t *__restrict__ lo, int64_t ld,
                                      int n0, int N, int k0, int kend, PreTile &r) {
    const int t = threadIdx.x;
    const int n = n0 + (t >> 1), k = k0 + (t & 1) * 16;
    const int64_t off = (int64_t)n * ld + k;
    if (n < N && k + 16 <= kend && (ld & 7) == 0 && (((uintptr_t)(hi + off)) & 15) == 0 &&
        (((uintptr_t)(lo + off)) & 15) == 0) {
        r.h0 = *(const bf16x8_t *)(hi + off);
        r.h1 = *(const bf16x8_t *)(hi + off + 8);
        r.l0 = *(const bf16x8_t *)(lo + off);
        r.l1 = *(const bf16x8_t *)(lo + off + 8);
    } else {
        const bf16_t z = (bf16_t)0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool ok0 = n < N && k + j < kend, ok1 = n < N && k + 8 + j < kend;
            r.h0[j] = ok0 ? hi[off + j] : z;
            r.l0[j] = ok0 ? lo[off + j] : z;
            r.h1[j] = ok1 ? hi[off + 8 + j] : z;
            r.l1[j] = ok1 ? lo[off + 8 + j] : z;
        }
    }
}

__device__ __forceinline__ void pstore(bf16_t (*Hs)[XLD], bf16_t (*Ls)[XLD], const PreTile &r) {
    const int t = threadIdx.x;
    const int n = t >> 1, k = (t & 1) * 16;
    *(bf16x8_t *)&Hs[n][k] = r.h0;
    *(bf16x8_t *)&Hs[n][k + 8] = r.h1;
    *(bf16x8_t *)&Ls[n][k] = r.l0;
    *(bf16x8_t *)&Ls[n][k + 8] = r.l1;
}

// ---------------------------------------------------------------- clamped-load form
// The bounds-checked loads above branch per lane, and the skipped prefetches past the
// last step branch per workgroup; the compiler then has to wait for every load in flight
// (vmcnt(0)) before each LDS staging, which takes away the second step of lookahead.  In
// the clamped form every thread issues the same vector loads for every step: a row past
// the operand reads a valid row, k past kend reads k = 0, and the staging zeroes what is
// out of range.  It needs (checked on the host) k0 % 16 == 0, kend % 4 == 0 (% 8 for the
// pre-split planes), ld % 4 == 0 (% 8), 16-byte aligned operands, and in the
// row-contiguous form rows_ld % 4 == 0, so that each 16-byte load is either wholly
// in range or wholly out.  The tile is spread over all 256 threads: PER = ROWS*32/256
// values each (16 at 128 rows, 8 at 64).
//   KC:  thread = (row t/(32/PER), k PER*(t%(32/PER)) .. +PER-1), r[j] = P[row][k+j]
//   !KC: thread = (rows 4*(t/(128/PER)) .. +3, k (PER/4)*(t%(128/PER)) .. +PER/4-1),
//        r[4*kk + rr] = P[k+kk][row+rr]
template <bool KC, int ROWS>
__device__ __forceinline__ void xload_cl(const float *__restrict__ P, int64_t ld, int r0, int rows_ld, int k0,
                                         int kend, float (&r)[16]) {
    constexpr int PER = ROWS * XBK / 256;
    const int t = threadIdx.x;
    if (KC) {
        constexpr int TPR = XBK / PER;
        const int row = r0 + t / TPR, k = k0 + (t % TPR) * PER;
        const int rc = row < rows_ld ? row : rows_ld - 1;
        const float *prow = P + (int64_t)rc * ld;
#pragma unroll
        for (int q = 0; q < PER / 4; ++q) {
            const int kq = k + 4 * q;
            const v4f_x u = *(const v4f_x *)(prow + (kq < kend ? kq : 0));
            r[4 * q + 0] = u[0];
            r[4 * q + 1] = u[1];
            r[4 * q + 2] = u[2];
            r[4 * q + 3] = u[3];
        }
    } else {
        constexpr int KPT = PER / 4, TPG = XBK / KPT;
        const int row = r0 + 4 * (t / TPG), k = k0 + KPT * (t % TPG);
        const int rc = row < rows_ld ? row : 0;
#pragma unroll
        for (int kk = 0; kk < KPT; ++kk) {
            const int kc = k + kk < kend ? k + kk : 0;
            const v4f_x u = *(const v4f_x *)(P + (int64_t)kc * ld + rc);
            r[4 * kk + 0] = u[0];
            r[4 * kk + 1] = u[1];
            r[4 * kk + 2] = u[2];
            r[4 * kk + 3] = u[3];
        }
    }
}

// Stage a clamped-form tile: zero what lies past rows_ld or kend, ones in row `ones`,
// split into the hi / lo LDS arrays.
template <bool KC, int ROWS>
__device__ __forceinline__ void xstore_cl(bf16_t (*Hs)[XLD], bf16_t (*Ls)[XLD], const float (&r)[16], int r0,
                                          int rows_ld, int ones, int k0, int kend) {
    constexpr int PER = ROWS * XBK / 256;
    const int t = threadIdx.x;
    // a tile wholly in range (the common case, uniform over the workgroup) is split as is
    if (r0 + ROWS <= rows_ld && k0 + XBK <= kend && (ones < r0 || ones >= r0 + ROWS)) {
        if (KC) {
            constexpr int TPR = XBK / PER;
            const int lr = t / TPR, lk = (t % TPR) * PER;
#pragma unroll
            for (int q = 0; q < PER / 8; ++q) {
                bf16x8_t h, l;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    bf16_t a, b;
                    split_bf16(r[8 * q + j], a, b);
                    h[j] = a;
                    l[j] = b;
                }
                *(bf16x8_t *)&Hs[lr][lk + 8 * q] = h;
                *(bf16x8_t *)&Ls[lr][lk + 8 * q] = l;
            }
        } else {
            constexpr int KPT = PER / 4, TPG = XBK / KPT;
            const int lr = 4 * (t / TPG), lk = KPT * (t % TPG);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                typedef __bf16 bfk_t __attribute__((ext_vector_type(KPT)));
                bfk_t h, l;
#pragma unroll
                for (int kk = 0; kk < KPT; ++kk) {
                    bf16_t a, b;
                    split_bf16(r[4 * kk + rr], a, b);
                    h[kk] = a;
                    l[kk] = b;
                }
                *(bfk_t *)&Hs[lr + rr][lk] = h;
                *(bfk_t *)&Ls[lr + rr][lk] = l;
            }
        }
        return;
    }
    if (KC) {
        constexpr int TPR = XBK / PER;
        const int lr = t / TPR, lk = (t % TPR) * PER;
        const int row = r0 + lr, k = k0 + lk;
        const bool rin = row < rows_ld, one = row == ones;
#pragma unroll
        for (int q = 0; q < PER / 8; ++q) {
            bf16x8_t h, l;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool kin = k + 8 * q + j < kend;
                const float v = one ? (kin ? 1.0f : 0.0f) : (rin && kin ? r[8 * q + j] : 0.0f);
                bf16_t a, b;
                split_bf16(v, a, b);
                h[j] = a;
                l[j] = b;
            }
            *(bf16x8_t *)&Hs[lr][lk + 8 * q] = h;
            *(bf16x8_t *)&Ls[lr][lk + 8 * q] = l;
        }
    } else {
        constexpr int KPT = PER / 4, TPG = XBK / KPT;
        const int lr = 4 * (t / TPG), lk = KPT * (t % TPG);
        const int row = r0 + lr, k = k0 + lk;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const bool rin = row + rr < rows_ld, one = row + rr == ones;
            typedef __bf16 bfk_t __attribute__((ext_vector_type(KPT)));
            bfk_t h, l;
#pragma unroll
            for (int kk = 0; kk < KPT; ++kk) {
                const bool kin = k + kk < kend;
                const float v = one ? (kin ? 1.0f : 0.0f) : (rin && kin ? r[4 * kk + rr] : 0.0f);
                bf16_t a, b;
                split_bf16(v, a, b);
                h[kk] = a;
                l[kk] = b;
            }
            *(bfk_t *)&Hs[lr + rr][lk] = h;
            *(bfk_t *)&Ls[lr + rr][lk] = l;
        }
    }
}

// Clamped form of pload / pstore (conditions as for xload_cl, with ld % 8 == 0).
__device__ __forceinline__ void pload_cl(const bf16_t *__restrict__ hi, const bf16_t *__restrict__ lo, int64_t ld,
                                         int n0, int N, int k0, int kend, PreTile &r) {
    const int t = threadIdx.x;
    const int n = n0 + (t >> 1), k = k0 + (t & 1) * 16;
    const int64_t nrow = (int64_t)(n < N ? n : N - 1) * ld;
    const int64_t o0 = nrow + (k < kend ? k : 0), o1 = nrow + (k + 8 < kend ? k + 8 : 0);
    r.h0 = *(const bf16x8_t *)(hi + o0);
    r.h1 = *(const bf16x8_t *)(hi + o1);
    r.l0 = *(const bf16x8_t *)(lo + o0);
    r.l1 = *(const bf16x8_t *)(lo + o1);
}

__device__ __forceinline__ void pstore_cl(bf16_t (*Hs)[XLD], bf16_t (*Ls)[XLD], const PreTile &r, int n0, int N,
                                          int k0, int kend) {
    const int t = threadIdx.x;
    const int n = t >> 1, k = (t & 1) * 16;
    if (n0 + XBN <= N && k0 + XBK <= kend) {
        pstore(Hs, Ls, r);
        return;
    }
    const bool in0 = n0 + n < N && k0 + k < kend, in1 = n0 + n < N && k0 + k + 8 < kend;
    const bf16x8_t z = {};
    *(bf16x8_t *)&Hs[n][k] = in0 ? r.h0 : z;
    *(bf16x8_t *)&Hs[n][k + 8] = in1 ? r.h1 : z;
    *(bf16x8_t *)&Ls[n][k] = in0 ? r.l0 : z;
    *(bf16x8_t *)&Ls[n][k + 8] = in1 ? r.l1 : z;
}

// AK: A k-contiguous (A[m*lda + k]) else A[k*lda + m].  BNC: B n-contiguous
// (B[k*ldb + n], i.e. row-contiguous in the [n][k] view) else B[n*ldb + k].  BPRE: B
// from the pre-split planes g.bsplit (BNC ignored).  CL: the clamped-load form.
template <bool AK, bool BNC, int EPI, int TM, bool BPRE, bool CL>
__global__ __launch_bounds__(256, 2) void k_gemm_x3(GemmArgs g0) {
    constexpr int WI = TM / 64;
    GemmArgs g = g0;
    __shared__ __attribute__((aligned(16))) bf16_t Ah[2][TM][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Al[2][TM][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bh[2][XBN][XLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bl[2][XBN][XLD];
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
    // the clamped form has no per-tile B: the kernel argument keeps it a global pointer
    const float *B = (const float *)(CL ? g0.B : g.B);
    const bf16_t *Bhi = (const bf16_t *)g.bsplit;
    const bf16_t *Blo = BPRE ? Bhi + g.bs_plane : nullptr;
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

    // Global loads run two K steps ahead: register set 0 holds the even steps, set 1
    // the odd ones; the loop is unrolled by two so that the sets stay static.
    float ra0[16], rb0[16], ra1[16], rb1[16];
    PreTile pb0, pb1;
    auto load = [&](int step, float (&ra)[16], float (&rb)[16], PreTile &pb) {
        const int k0 = kbeg + step * XBK;
        if (CL) {
            __builtin_amdgcn_sched_barrier(0);
            xload_cl<AK, TM>(A, g.lda, m0, mload, k0, kend, ra);
            if (BPRE)
                pload_cl(Bhi, Blo, g.ldbs, n0, g.N, k0, kend, pb);
            else
                xload_cl<!BNC, XBN>(B, g.ldb, n0, g.N, k0, kend, rb);
            // keep each step's loads together and in program order, so that the wait
            // before a staging covers only the older step
            __builtin_amdgcn_sched_barrier(0);
            return;
        }
        xload<AK, TM>(A, g.lda, m0, mload, g.ones_row, k0, kend, ra);
        if (BPRE)
            pload(Bhi, Blo, g.ldbs, n0, g.N, k0, kend, pb);
        else
            xload<!BNC, XBN>(B, g.ldb, n0, g.N, -1, k0, kend, rb);
    };
    auto store = [&](int buf, int step, const float (&ra)[16], const float (&rb)[16], const PreTile &pb) {
        if (CL) {
            __builtin_amdgcn_sched_barrier(0);
            const int k0 = kbeg + step * XBK;
            xstore_cl<AK, TM>(Ah[buf], Al[buf], ra, m0, mload, g.ones_row, k0, kend);
            if (BPRE)
                pstore_cl(Bh[buf], Bl[buf], pb, n0, g.N, k0, kend);
            else
                xstore_cl<!BNC, XBN>(Bh[buf], Bl[buf], rb, n0, g.N, -1, k0, kend);
            __builtin_amdgcn_sched_barrier(0);
            return;
        }
        xstore<AK, TM>(Ah[buf], Al[buf], ra);
        if (BPRE)
            pstore(Bh[buf], Bl[buf], pb);
        else
            xstore<!BNC, XBN>(Bh[buf], Bl[buf], rb);
    };
    auto compute = [&](int cur) {
#pragma unroll
        for (int ks = 0; ks < XBK; ks += 16) {
            bf16x8_t ah[WI], al[WI], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < WI; ++i) {
                ah[i] = *(const bf16x8_t *)&Ah[cur][wm + 32 * i + li][ks + lk];
                al[i] = *(const bf16x8_t *)&Al[cur][wm + 32 * i + li][ks + lk];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bh[j] = *(const bf16x8_t *)&Bh[cur][wn + 32 * j + li][ks + lk];
                bl[j] = *(const bf16x8_t *)&Bl[cur][wn + 32 * j + li][ks + lk];
            }
            // three passes over the WI x 2 accumulators, so that consecutive MFMAs never
            // depend on each other (a dependent MFMA waits for the previous result)
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    };
    const int nk = kend > kbeg ? (kend - kbeg + XBK - 1) / XBK : 0;
    // step s lives in register set s % 2 and LDS buffer s % 2.  In the clamped form the
    // loads and stagings past the last step run too (they read valid addresses and stage
    // zeros), so that every path through the loop issues the same loads.
    if (nk > 0) {
        load(0, ra0, rb0, pb0);
        store(0, 0, ra0, rb0, pb0);
        if (CL || nk > 1) load(1, ra1, rb1, pb1);
        if (CL || nk > 2) load(2, ra0, rb0, pb0);
    }
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
        // even step it: LDS buffer 0; stage step it+1 (set 1) into buffer 1
        compute(0);
        if (CL || it + 1 < nk) {
            store(1, it + 1, ra1, rb1, pb1);
            if (CL || it + 3 < nk) load(it + 3, ra1, rb1, pb1);
        }
        __syncthreads();
        // the clamped form runs an odd nk's last pair through: the step past the end was
        // staged as zeros and adds exact zeros, and the loop body stays one block
        if (!CL && it + 1 >= nk) break;
        // odd step it+1: LDS buffer 1; stage step it+2 (set 0) into buffer 0
        compute(1);
        if (CL || it + 2 < nk) {
            store(0, it + 2, ra0, rb0, pb0);
            if (CL || it + 4 < nk) load(it + 4, ra0, rb0, pb0);
        }
        __syncthreads();
    }
    float *C = (float *)g.C + (int64_t)blockIdx.z * g.c_split_stride;
    const float *act = (const float *)g.act;
    const int lrow = (lane >> 5) * 4;
    if (m0 + TM <= g.M && n0 + XBN <= g.N) {
        // interior tile (uniform): no bounds tests; each lane's 16 rows of a block sit at
        // fixed multiples of ld from its first row, so only one 64-bit address per block
        const int64_t ldc = g.ldc, lda_ = g.ldact;
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = n0 + wn + j * 32 + li;
                const int64_t row0 = m0 + wm + i * 32 + lrow;
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
                    if (EPI == EPI_BIAS_TANH) v = tanh_mixed(v + bias);
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
                    const int row = m0 + wm + i * 32 + 8 * (r >> 2) + lrow + (r & 3);
                    const float hv = act[(int64_t)(row < g.M ? row : g.M - 1) * g.ldact + cc];
                    fac[r] = 1.0f - hv * hv;
                }
            }
            if (col >= g.N) continue;
            const float bias = (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) ? g.bias[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + i * 32 + 8 * (r >> 2) + lrow + (r & 3);
                if (row >= g.M) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_BIAS) v += bias;
                if (EPI == EPI_BIAS_TANH) v = tanh_mixed(v + bias);
                if (EPI == EPI_DTANH) v *= fac[r];
                C[(int64_t)row * g.ldc + col] = v;
            }
        }
}

static bool al16(const void *p) { return (((uintptr_t)p) & 15) == 0; }

// Whether the clamped-load form applies (its conditions are stated above xload_cl).
template <bool AK, bool BNC, bool BPRE>
static bool clamped_ok(const GemmArgs &g) {
    if (g.ksplit || g.tile_pid || g.k_chunk % XBK) return false;
    const int mload = g.ones_row >= 0 ? g.ones_row : g.M;
    if (mload < 1 || g.N < 1 || g.K < 1) return false;
    // k-contiguous operands need kend % 4 == 0 (pre-split planes % 8); chunks are whole steps
    if ((AK || (!BPRE && !BNC)) && g.K % 4) return false;
    if (BPRE && g.K % 8) return false;
    if (g.lda % 4 || !al16(g.A) || (!AK && mload % 4)) return false;
    if (BPRE) return g.ldbs % 8 == 0 && g.bs_plane % 8 == 0 && al16(g.bsplit);
    return g.ldb % 4 == 0 && al16(g.B) && (!BNC || g.N % 4 == 0);
}

template <bool AK, bool BNC, int EPI, int TM, bool BPRE>
static void launch_x(hipStream_t st, GemmArgs g, int splits) {
    const int tiles = ((g.M + TM - 1) / TM) * ((g.N + XBN - 1) / XBN);
    if (clamped_ok<AK, BNC, BPRE>(g))
        hipLaunchKernelGGL((k_gemm_x3<AK, BNC, EPI, TM, BPRE, true>), dim3(tiles, 1, splits), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((k_gemm_x3<AK, BNC, EPI, TM, BPRE, false>), dim3(tiles, 1, splits), dim3(256), 0, st, g);
}

void launch_gemm_x3(hipStream_t st, const GemmArgs &g0, bool a_kcontig, bool b_ncontig, int epi, int splits,
                    int tm) {
    GemmArgs g = g0;
    if (splits < 1) splits = 1;
    int chunk = (g.K + splits - 1) / splits;
    chunk = (chunk + XBK - 1) / XBK * XBK;
    // a chunk given by the caller (a multiple of XBK) fixes the split ranges
    g.k_chunk = g0.k_chunk > 0 ? g0.k_chunk : (chunk > 0 ? chunk : XBK);
    if (g.bsplit && a_kcontig) {  // weights as B: pre-split planes
#define DISPATCH_PRE(EPI)                                    \
    if (tm == 64)                                            \
        launch_x<true, false, EPI, 64, true>(st, g, splits);  \
    else                                                     \
        launch_x<true, false, EPI, 128, true>(st, g, splits);
        switch (epi) {
            case EPI_STORE: DISPATCH_PRE(EPI_STORE) break;
            case EPI_BIAS: DISPATCH_PRE(EPI_BIAS) break;
            case EPI_BIAS_TANH: DISPATCH_PRE(EPI_BIAS_TANH) break;
            case EPI_DTANH: DISPATCH_PRE(EPI_DTANH) break;
        }
#undef DISPATCH_PRE
        return;
    }
    g.bsplit = nullptr;
#define DISPATCH_TM(AK, BNC, EPI)                          \
    if (tm == 64)                                          \
        launch_x<AK, BNC, EPI, 64, false>(st, g, splits);  \
    else                                                   \
        launch_x<AK, BNC, EPI, 128, false>(st, g, splits);
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

// hi / lo planes of a row-major R x C FP32 matrix: out[c][r] (transpose) or out[r][c]
__global__ void k_split_planes(const float *__restrict__ W, int R, int C, bool transpose, bf16_t *__restrict__ hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)R * C;
    if (i >= total) return;
    const int r = (int)(i / C), c = (int)(i % C);
    bf16_t h, l;
    split_bf16(W[i], h, l);
    const int64_t o = transpose ? (int64_t)c * R + r : i;
    hi[o] = h;
    hi[total + o] = l;
}

void launch_split_planes(hipStream_t st, const float *W, int R, int C, bool transpose, void *planes) {
    const int64_t total = (int64_t)R * C;
    if (total == 0) return;
    hipLaunchKernelGGL(k_split_planes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, W, R, C, transpose,
                       (bf16_t *)planes);
}

}  // namespace dnqs
