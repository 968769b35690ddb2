// Epstein-Nesbet PT2 (Eq. 13), external sum: the per-sub-bucket reduce that follows the
// partition passes of k_pt2_part.hip.
//
// One workgroup per sub-bucket (~6000 pairs, ~1700 unique keys at the benchmark size):
//   1. stage the diagonal table (h_pp, V(p,q) = J_pq - d_s K_pq; M <= 62) in LDS;
//   2. insert the members of S that hash into this sub-bucket, flagged (S is grouped by
//      the same hash bits once per call, k_s_sub_*), so no key is probed in the global
//      hash set of S;
//   3. decode every pair descriptor (x XOR flipped positions), recompute H_ax exactly in
//      FP64 from the packed integrals and accumulate w_a = sum_x H_ax psi_x in a 3072-slot
//      LDS table (64-bit CAS on the key; the sum in fixed point, 64 + 32-bit integer
//      adds, so that it does not depend on the order of the adds); the source
//      determinant and psi_x come from one 16-byte (M <= 32) or 32-byte record, and
//      single excitations are queued and done last;
//   4. for the members a of S: the internal term of Eq. 13 from v_a = w_a + H_aa psi_a;
//   5. compact the keys not in S to the front of the table, then for each form
//      w_a^2 / (E - H_aa) in FP64, H_aa from the LDS table by the diagonal rule, and
//      sum them exactly over the workgroup (integer limbs below the largest term), so
//      the result of a call is reproducible to the bit.
// A sub-bucket whose keys do not fit the table raises a flag and the host repeats the L2
// split and the reduce with twice as many sub-buckets.
#include "dnqs_device.h"
#include "dnqs_excite.h"
#include "dnqs_kernels.h"
#include "dnqs_pt2.h"

namespace dnqs {

// ------------------------------------------------------------------ reduce
// Wave reductions: two quad permutations and two rotations within each row of 16 lanes
// by DPP leave every lane with its row's result, and the four rows' results are read out
// (readlane) and combined in a fixed order, (r0 op r1) op (r2 op r3).  Every lane of the
// wave must be active.  (Cross-lane moves on the VALU: the generic shuffle goes through
// the LDS crossbar, one round trip per step.)
// a 64-bit value of lane l, as two 32-bit reads (the readlane builtin is 32-bit: a wider
// argument is narrowed to its low half)
__device__ __forceinline__ long long readlane64(long long v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (long long)(((uint64_t)hi << 32) | lo);
}

template <int CTRL, int ROW>
__device__ __forceinline__ long long dpp_ll(long long id, long long v) {
    return __builtin_amdgcn_update_dpp(id, v, CTRL, ROW, 0xf, false);
}

template <typename T>
__device__ __forceinline__ long long to_ll(T v) {
    if constexpr (sizeof(T) == 8 && __is_same(T, double)) return __double_as_longlong(v);
    else return (long long)v;
}

template <typename T>
__device__ __forceinline__ T from_ll(long long v) {
    if constexpr (__is_same(T, double)) return __longlong_as_double(v);
    else return (T)v;
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T id, Op op) {
    const long long i = to_ll(id);
    v = op(v, from_ll<T>(dpp_ll<0xB1, 0xf>(i, to_ll(v))));   // quad_perm [1,0,3,2]
    v = op(v, from_ll<T>(dpp_ll<0x4E, 0xf>(i, to_ll(v))));   // quad_perm [2,3,0,1]
    v = op(v, from_ll<T>(dpp_ll<0x124, 0xf>(i, to_ll(v))));  // row_ror:4
    v = op(v, from_ll<T>(dpp_ll<0x128, 0xf>(i, to_ll(v))));  // row_ror:8
    const long long b = to_ll(v);
    const T r0 = from_ll<T>(readlane64(b, 0)), r1 = from_ll<T>(readlane64(b, 16));
    const T r2 = from_ll<T>(readlane64(b, 32)), r3 = from_ll<T>(readlane64(b, 48));
    return op(op(r0, r1), op(r2, r3));
}

// Coulomb minus same-spin exchange between spin-orbitals s, t (alpha s < M, beta M + p)
__device__ __forceinline__ double v_so(const Ham &H, int s, int t) {
    const int M = H.M;
    const bool sa = s < M, ta = t < M;
    const int i = sa ? s : s - M, j = ta ? t : t - M;
    double v = H.J[i * M + j];
    if (sa == ta) v -= H.K[i * M + j];
    return v;
}

// Diagonal table for M <= 32: vt[p] = h_pp for the 2M spin-orbitals, then
// vt[2M + q(q-1)/2 + p] = V(p, q) for p < q, so that
// H_aa = E_core + sum_{q in a} (vt[q] + sum_{p in a, p < q} vt[2M + q(q-1)/2 + p]).
// 2M + M(2M-1) doubles: 12.8 KB at M = 28, 16.6 KB at M = 32.

__global__ void k_diag_table(Ham H, double *__restrict__ vt) {
    const int No = 2 * H.M;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < No) {
        const int sp = t < H.M ? t : t - H.M;
        vt[t] = H.h64[sp * H.M + sp];
        return;
    }
    const int u = t - No;
    if (u >= No * (No - 1) / 2) return;
    int q = (int)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
    while (q * (q - 1) / 2 > u) --q;
    while ((q + 1) * q / 2 <= u) ++q;
    const int p = u - q * (q - 1) / 2;
    vt[t] = v_so(H, p, q);
}

int pt2_diag_table_size(int M) { return 2 * M + (2 * M) * (2 * M - 1) / 2; }

// 128-bit-key reduce: 3 x 32 KB of tables, flags and the singles queue; the diagonal table must fit the
// remaining LDS of a CU (M <= 62)
bool pt2_diag_table_fits(int M) {
    return 3 * 32768 + 1024 + sizeof(uint64_t) * kRedSingles + sizeof(double) * pt2_diag_table_size(M) <= 160 * 1024;
}

void launch_diag_table(hipStream_t st, const Ham &H, double *vt) {
    const int total = pt2_diag_table_size(H.M);
    hipLaunchKernelGGL(k_diag_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, H, vt);
}

// ------------------------------------------------------------------ S by sub-bucket
// The keys of S grouped by the sub-bucket their hash falls in (top sbits bits, the
// concatenated L1 and L2 bucket indices), so that each reduce workgroup can mark the
// members of S among its keys without probing the global hash set.
// sub-bucket of a member of S in key-space slice `slice` (-1: another slice)
template <bool PACKED>
__device__ __forceinline__ int64_t s_sub(uint64_t a, uint64_t b, int sbits, int ss, uint32_t slice) {
    uint64_t h = target_hash<PACKED>(a, b);
    if (ss) {
        if ((uint32_t)(h >> (64 - ss)) != slice) return -1;
        h <<= ss;
    }
    return sbits ? (int64_t)(h >> (64 - sbits)) : 0;
}

template <bool PACKED>
__global__ void k_s_sub_count(const uint64_t *__restrict__ dets, int64_t n, int sbits, int ss, uint32_t slice,
                              int32_t *__restrict__ cnt) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t s = s_sub<PACKED>(dets[2 * x], dets[2 * x + 1], sbits, ss, slice);
    if (s >= 0) atomicAdd(&cnt[s], 1);
}

template <bool PACKED>
__global__ void k_s_sub_fill(const uint64_t *__restrict__ dets, int64_t n, int sbits, int ss, uint32_t slice,
                             const int64_t *__restrict__ offs, int32_t *__restrict__ cur,
                             uint64_t *__restrict__ skeys, int32_t *__restrict__ sidx) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint64_t a = dets[2 * x], b = dets[2 * x + 1];
    const int64_t s = s_sub<PACKED>(a, b, sbits, ss, slice);
    if (s < 0) return;
    const int64_t pos = offs[s] + atomicAdd(&cur[s], 1);
    skeys[2 * pos] = a;
    skeys[2 * pos + 1] = b;
    sidx[pos] = (int32_t)x;
}

void launch_s_sub(hipStream_t st, const uint64_t *dets, int64_t n, int sbits, bool packed, int32_t *cnt,
                  const int64_t *offs, uint64_t *skeys, int32_t *sidx, bool fill, int ss, uint32_t slice) {
    if (n == 0) return;
    dim3 grid((unsigned)((n + 255) / 256)), blk(256);
    if (fill) {
        if (packed)
            hipLaunchKernelGGL(k_s_sub_fill<true>, grid, blk, 0, st, dets, n, sbits, ss, slice, offs, cnt, skeys, sidx);
        else
            hipLaunchKernelGGL(k_s_sub_fill<false>, grid, blk, 0, st, dets, n, sbits, ss, slice, offs, cnt, skeys, sidx);
    } else {
        if (packed)
            hipLaunchKernelGGL(k_s_sub_count<true>, grid, blk, 0, st, dets, n, sbits, ss, slice, cnt);
        else
            hipLaunchKernelGGL(k_s_sub_count<false>, grid, blk, 0, st, dets, n, sbits, ss, slice, cnt);
    }
}

// ------------------------------------------------------------------ reduce kernel
// Probe sequence of a key in the LDS table (double hashing).  The key is folded to 32
// bits (f = a XOR b * odd constant) and multiplied by a second odd constant; the top 22
// bits of the product map onto the kRedTab slots (start = floor(top22 * 3 / 2^12), near
// uniform), and seven low bits give the step 6k + 1, which is odd and not a multiple of 3,
// so coprime with kRedTab = 3 * 2^10: the sequence visits every slot.  Two 32-bit
// multiplies and a 24-bit one: the hash is computed for every pair, and a full
// integer-hash finaliser cost more than the probes it saved.  Independent of the
// partition hash, whose top bits chose the sub-bucket.  Double hashing rather than linear
// probing: its probe counts have a shorter tail at the same load (no clustering), and a
// wave waits for its longest probe sequence.
static_assert(kRedTab == 3072, "the probe step is coprime with 3 * 2^10");

struct Probe {
    uint32_t s, step;
};

template <bool PACKED>
__device__ __forceinline__ Probe red_probe(uint64_t a, uint64_t b) {
    uint32_t f = (uint32_t)a ^ ((uint32_t)b * 0x9e3779b1u);
    if (!PACKED) f ^= ((uint32_t)(a >> 32) * 0x85ebca6bu) ^ ((uint32_t)(b >> 32) * 0xc2b2ae35u);
    const uint32_t h = (f ^ (f >> 16)) * 0x7feb352du;
    Probe p;
    p.s = __umul24(h >> 10, 3u) >> 12;           // [0, 3072)
    p.step = __umul24((h >> 3) & 127u, 6u) + 1u;  // 6k + 1 <= 763
    return p;
}

__device__ __forceinline__ void red_step(Probe &p) {
    p.s += p.step;
    if (p.s >= (uint32_t)kRedTab) p.s -= (uint32_t)kRedTab;
}

// A pass is redone with more sub-buckets when a table fills up.  "Full" is decided by a
// count of the occupied slots: past 7/8 of the slots the pass is marked lost, so no lane
// keeps probing an (almost) full table; at the table's working load (about 0.55) the
// longest probe sequence over millions of tables stays far below kRedProbe, the hard
// bound on a probe sequence.  In the pair loop each wave adds its newly claimed slots
// with one atomic (a ballot), and the loop checks the count once per iteration.
constexpr int kRedFillMax = kRedTab / 8 * 7;
constexpr int kRedProbe = 1024;

// Insert (a, b) into the LDS table (linear probing); returns the slot, or -1 when no free
// slot or matching key is found within kRedProbe probes.  claimed: this call took an
// empty slot.
template <bool PACKED>
__device__ __forceinline__ int red_insert(unsigned long long *ka_t, unsigned long long *kb_t, uint64_t a, uint64_t b,
                                          bool &claimed) {
    Probe pr = red_probe<PACKED>(a, b);
    for (int p = 0; p < kRedProbe; ++p) {
        const uint32_t s = pr.s;
        if (PACKED) {
            const unsigned long long k = pack_key(a, b);
            const unsigned long long prev = atomicCAS(&ka_t[s], (unsigned long long)kEmptyKey, k);
            if (prev == kEmptyKey || prev == k) {
                claimed = prev == kEmptyKey;
                return (int)s;
            }
        } else {
            const unsigned long long pa = atomicCAS(&ka_t[s], (unsigned long long)kEmptyKey, (unsigned long long)a);
            if (pa == kEmptyKey) claimed = true;
            if (pa == kEmptyKey || pa == a) {
                const unsigned long long pb =
                    atomicCAS(&kb_t[s], (unsigned long long)kEmptyKey, (unsigned long long)b);
                if (pb == kEmptyKey || pb == b) return (int)s;
            }
        }
        red_step(pr);
    }
    return -1;
}

// Slot of a key already in the table (after every insertion is done), -1 if absent.
template <bool PACKED>
__device__ __forceinline__ int red_find(const unsigned long long *ka_t, const unsigned long long *kb_t, uint64_t a,
                                        uint64_t b) {
    Probe pr = red_probe<PACKED>(a, b);
    for (int p = 0; p < kRedProbe; ++p) {
        const uint32_t s = pr.s;
        if (PACKED) {
            const unsigned long long k = ka_t[s];
            if (k == pack_key(a, b)) return (int)s;
            if (k == kEmptyKey) return -1;
        } else {
            if (ka_t[s] == a && kb_t[s] == b) return (int)s;
            if (kb_t[s] == kEmptyKey) return -1;
        }
        red_step(pr);
    }
    return -1;
}

// ------------------------------------------------------------------ exact sums
// w_a is accumulated in fixed point, so that the sum does not depend on the order in
// which lanes and waves add their terms (integer addition is associative): each term
// t = H_ax psi_x, |t| <= 2^wexp, is scaled to y = t 2^(62 - cb - wexp), where 2^cb exceeds
// the number of pairs of the sub-bucket and cb >= 11 (so |y| <= 2^51 and neither sum can
// overflow), rounded to the nearest integer (the 64-bit part), and the remainder
// (|r| <= 1/2) is scaled by 2^(30 - cb) and truncated into a 32-bit part.  About
// 90 - 2 cb bits below 2^wexp are kept: 2^(wexp-64) or finer for sub-buckets of up to 2^13
// pairs, far below the FP64 rounding of w_a itself.
//
// Rounding to an integer uses the FP64 adder: for |y| < 2^51, y + 1.5 2^52 lies in
// [2^52, 2^53), where the spacing is 1, so the sum is 1.5 2^52 + round(y) exactly and
// round(y) is the difference of the two bit patterns as 64-bit integers; y - round(y) is
// exact.  Two instructions where a double-to-int64 conversion takes about a dozen.
constexpr double kRoundMagic = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ long long round_split(double y, double &rem) {
    const double m = y + kRoundMagic;
    rem = y - (m - kRoundMagic);
    return __double_as_longlong(m) - __double_as_longlong(kRoundMagic);
}

struct FixQ {
    double up1, up2;    // 2^(62 - cb - wexp), 2^(30 - cb)
    double dn1, dn2;    // inverses
};

__device__ __forceinline__ FixQ make_fixq(int wexp, int64_t npairs) {
    int cb = 11;
    while (cb < 30 && ((int64_t)1 << cb) <= npairs) ++cb;
    FixQ q;
    q.up1 = ldexp(1.0, 62 - cb - wexp);
    q.up2 = ldexp(1.0, 30 - cb);
    q.dn1 = ldexp(1.0, wexp + cb - 62);
    q.dn2 = ldexp(1.0, wexp + cb - 62 - (30 - cb));
    return q;
}

__device__ __forceinline__ void fix_split(const FixQ &q, double t, long long &hi, int &lo) {
    double r;
    hi = round_split(t * q.up1, r);
    lo = __double2int_rz(r * q.up2);
}

__device__ __forceinline__ double fix_join(const FixQ &q, long long hi, int lo) {
    return (double)hi * q.dn1 + (double)lo * q.dn2;
}

// The workgroup's outputs, to part[0..8) by thread 0:
//   [0] the exact sum of every thread's values v[0..cnt): the workgroup's largest |v|
//       fixes the scale 2^e, every value is cut into three 40-bit integer limbs below it
//       (nearest-integer limbs, so a limb may be negative) and the limbs are summed as
//       integers (at most 2^12 values per thread group: no overflow), so the result does
//       not depend on how the values are spread over the threads; the FP64 result is the
//       exact sum up to the limbs' 2^(e-120) grid, rounded once.  Values that are not
//       finite are summed in FP64 (their sum is inf or NaN in any order).
//   [1] min of mn, [2] sum of np, [3] sum of nt, [4], [5] (bits) sum mod 2^64 and XOR of
//       fs, fx; [6], [7] zero.  Each is exact in any order.
// Two barriers: the maximum and the other reductions together, then the limbs.  Every
// thread of the block must call it.
template <int K>
__device__ inline void red_final(const double (&v)[K], int cnt, double mn, double np, double nt,
                                 unsigned long long fs, unsigned long long fx, double *__restrict__ out) {
    constexpr int NW = kRedThreads / kWave;
    __shared__ double s_d[4][NW];              // max |v|, min, np, nt
    __shared__ unsigned long long s_u[3][NW];  // fs, fx, non-finite flag
    __shared__ long long s_l[3][NW];           // limb sums (or the FP64 sum's bits)
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double mx = 0.0;
    unsigned long long bad = 0ull;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < cnt) {
            if (isfinite(v[j]))
                mx = fmax(mx, fabs(v[j]));
            else
                bad = 1ull;
        }
    const auto dmax = [](double a, double b) { return fmax(a, b); };
    const auto dmin = [](double a, double b) { return fmin(a, b); };
    const auto dadd = [](double a, double b) { return a + b; };
    const auto uadd = [](unsigned long long a, unsigned long long b) { return a + b; };
    const auto uxor = [](unsigned long long a, unsigned long long b) { return a ^ b; };
    const auto uor = [](unsigned long long a, unsigned long long b) { return a | b; };
    const auto ladd = [](long long a, long long b) { return a + b; };
    mx = wave_reduce(mx, 0.0, dmax);
    mn = wave_reduce(mn, (double)INFINITY, dmin);
    np = wave_reduce(np, 0.0, dadd);
    nt = wave_reduce(nt, 0.0, dadd);
    fs = wave_reduce(fs, 0ull, uadd);
    fx = wave_reduce(fx, 0ull, uxor);
    bad = wave_reduce(bad, 0ull, uor);
    if (lane == 0) {
        s_d[0][wave] = mx;
        s_d[1][wave] = mn;
        s_d[2][wave] = np;
        s_d[3][wave] = nt;
        s_u[0][wave] = fs;
        s_u[1][wave] = fx;
        s_u[2][wave] = bad;
    }
    __syncthreads();
    mx = 0.0;
    bad = 0ull;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mx = fmax(mx, s_d[0][w]);
        bad |= s_u[2][w];
    }
    double sum = 0.0;
    if (bad) {
        // inf / NaN present: an FP64 sum (non-finite in any order)
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < cnt) t += v[j];
        t = wave_reduce(t, 0.0, dadd);
        if (lane == 0) s_l[0][wave] = __double_as_longlong(t);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < NW; ++w) sum += __longlong_as_double(s_l[0][w]);
    } else if (mx != 0.0) {
        int e;
        (void)frexp(mx, &e);  // mx < 2^e
        const double up = ldexp(1.0, 40 - e), sh = 1099511627776.0;  // 2^40
        long long l2 = 0, l1 = 0, l0 = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < cnt) {
                // nearest-integer limbs: |a2| <= 2^40, |a1|, |a0| <= 2^39 (remainders are exact)
                double r;
                const long long a2 = round_split(v[j] * up, r);
                const long long a1 = round_split(r * sh, r);
                const long long a0 = round_split(r * sh, r);
                l2 += a2;
                l1 += a1;
                l0 += a0;
            }
        l2 = wave_reduce(l2, 0ll, ladd);
        l1 = wave_reduce(l1, 0ll, ladd);
        l0 = wave_reduce(l0, 0ll, ladd);
        if (lane == 0) {
            s_l[0][wave] = l2;
            s_l[1][wave] = l1;
            s_l[2][wave] = l0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long L2 = 0, L1 = 0, L0 = 0;
            for (int w = 0; w < NW; ++w) {
                L2 += s_l[0][w];
                L1 += s_l[1][w];
                L0 += s_l[2][w];
            }
            // carry the lower limbs up; the conversion is a fixed formula of the integers
            const long long c0 = L0 / 1099511627776ll;
            L0 -= c0 * 1099511627776ll;
            L1 += c0;
            const long long c1 = L1 / 1099511627776ll;
            L1 -= c1 * 1099511627776ll;
            L2 += c1;
            sum = ldexp((double)L2 + ((double)L1 + (double)L0 / sh) / sh, e - 40);
        }
    }
    if (threadIdx.x == 0) {
        double m = s_d[1][0], p = s_d[2][0], q = s_d[3][0];
        unsigned long long a = s_u[0][0], x = s_u[1][0];
        for (int w = 1; w < NW; ++w) {
            m = fmin(m, s_d[1][w]);
            p += s_d[2][w];
            q += s_d[3][w];
            a += s_u[0][w];
            x ^= s_u[1][w];
        }
        out[0] = sum;
        out[1] = m;
        out[2] = p;
        out[3] = q;
        out[4] = __longlong_as_double((long long)a);
        out[5] = __longlong_as_double((long long)x);
        out[6] = 0.0;
        out[7] = 0.0;
    }
}

// H_aa by the diagonal rule from the LDS table, with the loops unrolled over at most
// kHaaOcc electrons per spin.  Every key of the sector has na alpha and nb beta electrons,
// so the trip counts are the same on every lane and the occupied indices stay in
// registers.  W: 32-bit strings (M <= 32) or 64-bit.
constexpr int kHaaOcc = 16;

__device__ __forceinline__ int low_bit(uint32_t m) { return __builtin_ctz(m); }
__device__ __forceinline__ int low_bit(uint64_t m) { return ctz64(m); }

template <typename W>
__device__ __forceinline__ double haa_unrolled(const double *vt, int No, int M, int na, int nb, W a, W b,
                                               double ecore) {
    int oa[kHaaOcc], ob[kHaaOcc];
#pragma unroll
    for (int k = 0; k < kHaaOcc; ++k) {
        oa[k] = 0;
        ob[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < kHaaOcc; ++k)
        if (k < na) {
            oa[k] = low_bit(a);
            a &= a - 1;
        }
#pragma unroll
    for (int k = 0; k < kHaaOcc; ++k)
        if (k < nb) {
            ob[k] = M + low_bit(b);
            b &= b - 1;
        }
    double e0 = ecore, e1 = 0.0, e2 = 0.0;
#pragma unroll
    for (int q = 0; q < kHaaOcc; ++q)
        if (q < na) {
            const double *row = vt + No + oa[q] * (oa[q] - 1) / 2;
            e0 += vt[oa[q]];
#pragma unroll
            for (int p = 0; p < q; ++p) e1 += row[oa[p]];
        }
#pragma unroll
    for (int q = 0; q < kHaaOcc; ++q)
        if (q < nb) {
            const double *row = vt + No + ob[q] * (ob[q] - 1) / 2;
            e0 += vt[ob[q]];
#pragma unroll
            for (int p = 0; p < kHaaOcc; ++p)
                if (p < na) e2 += row[oa[p]];
#pragma unroll
            for (int p = 0; p < q; ++p) e1 += row[ob[p]];
        }
    return e0 + (e1 + e2);
}

// H_aa by the diagonal rule with the alpha count NA fixed at compile time, row by row of
// the table (a row: the pairs (p, q) of one occupied spin-orbital q with the occupied p
// below it): the alpha rows and the alpha part of every beta row are straight-line code,
// so their reads are issued together and waited for together, where the loops bounded by
// the runtime counts wait once per read.  The beta rows are a loop that is not unrolled,
// which keeps the registers in flight to one row.  Each row is summed before it is added,
// a fixed order, so the result is reproducible to the bit.
template <int NA, typename W>
__device__ __forceinline__ double haa_rows(const double *vt, int No, int M, int nb, W a, W b, double ecore) {
    int oa[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        oa[k] = low_bit(a);
        a &= a - 1;
    }
    double e = ecore;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const double *row = vt + No + oa[q] * (oa[q] - 1) / 2;
        double r = vt[oa[q]];
#pragma unroll
        for (int p = 0; p < q; ++p) r += row[oa[p]];
        e += r;
    }
    W prev = 0;
#pragma unroll 1
    for (int q = 0; q < nb; ++q) {
        const int sq = M + low_bit(b);
        b &= b - 1;
        const double *row = vt + No + sq * (sq - 1) / 2;
        double r = vt[sq];
#pragma unroll
        for (int p = 0; p < NA; ++p) r += row[oa[p]];
        for (W pb = prev; pb; pb &= pb - 1) r += row[M + low_bit(pb)];
        prev |= (W)1 << (sq - M);
        e += r;
    }
    return e;
}

// the alpha counts of the workloads measured here get the row form; others the generic
// unrolled loops (a wave-uniform branch: na and nb are kernel arguments)
template <typename W>
__device__ __forceinline__ double haa_lds(const double *vt, int No, int M, int na, int nb, W a, W b, double ecore) {
    if (sizeof(W) == 4) {  // M <= 32
        if (na == 7) return haa_rows<7, W>(vt, No, M, nb, a, b, ecore);
        if (na == 6) return haa_rows<6, W>(vt, No, M, nb, a, b, ecore);
        if (na == 5) return haa_rows<5, W>(vt, No, M, nb, a, b, ecore);
        if (na == 4) return haa_rows<4, W>(vt, No, M, nb, a, b, ecore);
    } else if (na == 12) {
        return haa_rows<12, W>(vt, No, M, nb, a, b, ecore);
    }
    return haa_unrolled<W>(vt, No, M, na, nb, a, b, ecore);
}

// exclusive scan of one count per thread across the workgroup; total to every thread.
// The wave's inclusive scan by DPP: row shifts by 1, 2 and 3 of the original values give
// sums of four, row shifts by 4 and 8 (on the upper banks) complete each row of 16, and
// the totals of the rows below (read out of lanes 15, 31, 47) are added.
__device__ inline uint32_t red_scan(uint32_t v, uint32_t &total) {
    __shared__ uint32_t wsum[kRedThreads / kWave];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int x = (int)v;
    int inc = x + __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    inc += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);         // row_shr:2
    inc += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xf, 0xf, false);         // row_shr:3
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x114, 0xf, 0xe, false);       // row_shr:4, banks 1-3
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x118, 0xf, 0xc, false);       // row_shr:8, banks 2-3
    const int t0 = __builtin_amdgcn_readlane(inc, 15), t1 = __builtin_amdgcn_readlane(inc, 31);
    const int t2 = __builtin_amdgcn_readlane(inc, 47);
    const int row = lane >> 4;
    inc += (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
    if (lane == kWave - 1) wsum[wave] = (uint32_t)inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int w = 0; w < kRedThreads / kWave; ++w) {
        const uint32_t y = wsum[w];
        if (w < wave) before += y;
        total += y;
    }
    return before + (uint32_t)inc - v;
}

// (-1)^(occupied orbitals of s strictly between p and q); 32-bit strings when M <= 32
template <bool PACKED>
__device__ __forceinline__ int red_phase(uint64_t s, int p, int q) {
    if (PACKED) {
        const int lo = min(p, q), hi = max(p, q);
        const uint32_t m = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
        return (__popc((uint32_t)s & m) & 1) ? -1 : 1;
    }
    return phase_between(s, p, q);
}

// Pair index (p|q) -> p(p+1)/2 + q for p >= q, with a 24-bit product: p, q < 2^11 (orbital
// pairs of M <= 64), so p(p+1) < 2^24.
// (v_mul_u32_u24 written out: left to itself the compiler fuses the product and the index's
// widening into a 64-bit multiply-add, which issues at a quarter of the rate)
__device__ __forceinline__ int tri24(int p, int q) {
    const uint32_t hi = (uint32_t)max(p, q), lo = (uint32_t)min(p, q);
    uint32_t pr;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(pr) : "v"(hi), "v"(hi + 1u));
    return (int)((pr >> 1) + lo);
}

// H_ax psi_x for one pair descriptor.  The descriptor's flipped positions give the
// excitation directly (holes of x, then particles; ascending within a spin), so the
// class, the orbitals and the target are read off it; the values and phases are those of
// the Slater-Condon rules with ascending hole/particle pairing (h_offdiag).
// the source record of a pair: x's strings and psi_x
struct SrcRec {
    uint4 s;      // alpha (x, y), beta (z, w) as 32-bit halves
    uint64_t p;   // bits of psi_x
};

// Records are 16 bytes when M <= 32 ({alpha | beta << 32, bits of psi_x}: the table stays
// resident in each XCD's L2 next to the integrals) and 32 bytes otherwise ({alpha, beta,
// bits of psi_x, 0}); see launch_pt2_records.
template <bool PACKED>
__device__ __forceinline__ SrcRec load_src(const uint64_t *__restrict__ rec, uint64_t d) {
    const int64_t x = desc_x(d);
    if (PACKED) {
        const uint4 v = *reinterpret_cast<const uint4 *>(rec + 2 * x);
        return SrcRec{make_uint4(v.x, 0u, v.y, 0u), ((uint64_t)v.w << 32) | v.z};
    }
    return SrcRec{*reinterpret_cast<const uint4 *>(rec + 4 * x), rec[4 * x + 2]};
}

// A pair's target (a, b) and the factors of H_ax psi_x = (-1)^phase (e1 - e2) psi_x; the
// phase is kept as the FP64 sign bit (sgn = 0 or 2^63) and applied with an XOR, which is
// exact.  The integrals are kept as loaded and combined in red_add, after the loop has
// issued its prefetches, so that the wait for them does not cover the prefetches.
struct PairVal {
    uint64_t a, b;
    double e1, e2, px;
    uint64_t sgn;
};

__device__ __forceinline__ uint64_t sign_bit(int ph) { return ph < 0 ? 0x8000000000000000ull : 0ull; }

__device__ __forceinline__ double pair_term(const PairVal &pv) {
    return __longlong_as_double((long long)((uint64_t)__double_as_longlong((pv.e1 - pv.e2) * pv.px) ^ pv.sgn));
}

__device__ __forceinline__ uint64_t src_alpha(const SrcRec &sr) { return ((uint64_t)sr.s.y << 32) | sr.s.x; }
__device__ __forceinline__ uint64_t src_beta(const SrcRec &sr) { return ((uint64_t)sr.s.w << 32) | sr.s.z; }

// Double excitations.  The descriptor's flipped positions give the excitation directly
// (holes of x, then particles; ascending within a spin), so the class, the orbitals and
// the target are read off it; values and phases are those of the Slater-Condon rules with
// ascending hole/particle pairing (h_offdiag).  One code path for both classes (a wave
// nearly always holds both); the exchange integral is loaded for same-spin pairs only:
//   alpha-beta: i -> r (alpha), j -> t (beta), value (ri|tj)
//   same-spin:  holes i < j, particles r < t, value (ri|tj) - (rj|ti)
// Called on every descriptor of the sub-bucket, singles included.
template <bool PACKED>
__device__ __forceinline__ PairVal double_value(const Ham &H, const SrcRec &sr, uint64_t d) {
    const uint32_t pos = desc_pos(d);
    const int p0 = (int)(pos & 127u), p1 = (int)((pos >> 7) & 127u);
    // A single's last two positions are kNoPos: it is called on singles too (their result
    // is discarded), so use its two real positions there to keep every index in the table.
    const bool single = ((pos >> 14) & 127u) == kNoPos;
    const int p2 = single ? p0 : (int)((pos >> 14) & 127u), p3 = single ? p1 : (int)((pos >> 21) & 127u);
    const bool ab = p0 < 64 && p2 >= 64, beta = p0 >= 64;
    const int i = p0 & 63, t = p3 & 63;
    const int r = ab ? p1 : (p2 & 63), j = ab ? (p2 - 64) : (p1 & 63);
    const int ri = tri24(r, i), tj = tri24(t, j);
    const int rj = tri24(r, j), ti = tri24(t, i);
    const double *e = H.eri_pk;
    PairVal pv;
    pv.e1 = e[tri24(ri, tj)];
    pv.e2 = 0.0;
    if (!ab) pv.e2 = e[tri24(rj, ti)];  // same-spin doubles only: fewer L1/L2 requests
    pv.px = __longlong_as_double((long long)sr.p);
    int par;
    if (PACKED) {
        // M <= 32: 32-bit strings, masks and phases
        const uint32_t xa = sr.s.x, xb = sr.s.z;
        const uint32_t f_ir = (1u << i) | (1u << r), f_jt = (1u << j) | (1u << t);
        const uint32_t s1 = beta ? xb : xa;                                  // holds i and r
        const uint32_t s2 = ab ? xb : ((s1 & ~(1u << i)) | (1u << r));  // holds j and t
        pv.a = xa ^ (ab ? f_ir : (beta ? 0u : (f_ir | f_jt)));
        pv.b = xb ^ (ab ? f_jt : (beta ? (f_ir | f_jt) : 0u));
        // occupied orbitals strictly between the hole and the particle, for both moves
        const uint32_t m1 = ((1u << max(i, r)) - 1u) & ~((2u << min(i, r)) - 1u);
        const uint32_t m2 = ((1u << max(j, t)) - 1u) & ~((2u << min(j, t)) - 1u);
        par = (__popc(s1 & m1) + __popc(s2 & m2)) & 1;
    } else {
        const uint64_t xa = src_alpha(sr), xb = src_beta(sr);
        const uint64_t f_ir = (1ull << i) | (1ull << r), f_jt = (1ull << j) | (1ull << t);
        const uint64_t s1 = beta ? xb : xa;
        const uint64_t s2 = ab ? xb : ((s1 & ~(1ull << i)) | (1ull << r));
        pv.a = xa ^ (ab ? f_ir : (beta ? 0ull : (f_ir | f_jt)));
        pv.b = xb ^ (ab ? f_jt : (beta ? (f_ir | f_jt) : 0ull));
        par = (phase_between(s1, i, r) * phase_between(s2, j, t)) < 0 ? 1 : 0;
    }
    pv.sgn = (uint64_t)par << 63;
    return pv;
}

// Single-excitation value (as single_value: h_pq + sum over the occupied r != q of
// (pq|rr) - [same spin] (pr|rq), same spin first, both in ascending r, so the result is
// the same to the bit) with the integral loads issued eight orbitals at a time: a single
// costs a few load latencies instead of one per occupied orbital.
__device__ __forceinline__ double single_value_grouped(const Ham &H, int p, int q, uint64_t same, uint64_t other) {
    const double *e = H.eri_pk;
    const int pq = tri_index(p, q);
    double v = H.h64[p * H.M + q];
    uint64_t s = same & ~(1ull << q), o = other;
    while (s | o) {
        double c[8], x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            c[k] = 0.0;
            x[k] = 0.0;
            if (s) {
                const int r = ctz64(s);
                s &= s - 1;
                c[k] = e[tri_index(pq, tri_index(r, r))];
                x[k] = e[tri_index(tri_index(p, r), tri_index(r, q))];
            } else if (o) {
                const int r = ctz64(o);
                o &= o - 1;
                c[k] = e[tri_index(pq, tri_index(r, r))];
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) v += c[k] - x[k];
    }
    return v;
}

// Single excitation (hole p0, particle p1): the value sums over the occupied orbitals.
template <bool PACKED>
__device__ __forceinline__ PairVal single_pair(const Ham &H, const SrcRec &sr, uint64_t d) {
    const uint64_t xa = src_alpha(sr), xb = src_beta(sr);
    const uint32_t pos = desc_pos(d);
    const int p0 = (int)(pos & 127u), p1 = (int)((pos >> 7) & 127u);
    const bool beta = p0 >= 64;
    const int q = p0 & 63, p = p1 & 63;
    const uint64_t same = beta ? xb : xa, other = beta ? xa : xb;
    const uint64_t flip = (1ull << q) | (1ull << p);
    PairVal pv;
    pv.a = beta ? xa : (xa ^ flip);
    pv.b = beta ? (xb ^ flip) : xb;
    pv.e1 = single_value_grouped(H, p, q, same, other);
    pv.e2 = 0.0;
    pv.px = __longlong_as_double((long long)sr.p);
    pv.sgn = sign_bit(red_phase<PACKED>(same, p, q));
    return pv;
}

// One lane's share of a single (hole p0, particle p1) spread over eight lanes; the
// returned e1 holds h_pq, and the caller adds the eight parts.
//   M <= 32: lane l takes the orbitals r = l, l + 8, l + 16, l + 24 and adds, for each,
//   (pq|rr) once per electron occupying r (q excluded on the same spin) minus (pr|rq) when
//   r is occupied on the same spin (the weights 0, 1, 2 and the products are exact).  Its
//   loads go out together, so a single costs one integral latency; the order of the adds
//   is fixed.
//   Otherwise: lane l sums the terms of the occupied orbitals r != q numbered l, l + 8, ...
//   (same spin first, ascending).
template <bool PACKED>
__device__ __forceinline__ PairVal single_part(const Ham &H, const SrcRec &sr, uint64_t d, int l, double &part) {
    const uint64_t xa = src_alpha(sr), xb = src_beta(sr);
    const uint32_t pos = desc_pos(d);
    const int p0 = (int)(pos & 127u), p1 = (int)((pos >> 7) & 127u);
    const bool beta = p0 >= 64;
    const int q = p0 & 63, p = p1 & 63;
    const uint64_t same = beta ? xb : xa, other = beta ? xa : xb;
    const uint64_t flip = (1ull << q) | (1ull << p);
    const double *e = H.eri_pk;
    if (PACKED) {
        const int pq = tri24(p, q);
        const uint32_t sm = (uint32_t)same & ~(1u << q), om = (uint32_t)other;
        double c[4], x[4], nc[4], nx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // every load is issued (index clamped into the table), then weighted by the
            // occupation: no branches, so the eight loads go out back to back
            const int r = l + 8 * k;  // < 32; strings hold no bits at or above M
            const int rl = min(r, H.M - 1);
            const uint32_t bit = 1u << r;
            nc[k] = (double)(((sm & bit) ? 1 : 0) + ((om & bit) ? 1 : 0));
            nx[k] = (sm & bit) ? 1.0 : 0.0;
            c[k] = e[tri24(pq, tri24(rl, rl))];
            x[k] = e[tri24(tri24(p, rl), tri24(rl, q))];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) part += nc[k] * c[k] - nx[k] * x[k];
    } else {
        const int pq = tri_index(p, q);
        uint64_t sm = same & ~(1ull << q), om = other;
        const int ns = popc64(sm);
        // this lane's orbitals: entries l, l + 8, ... of (same-spin list, other-spin list)
        for (int idx = 0;; idx += 8) {
            const int n = idx + l;
            if (n >= ns + popc64(om)) break;
            if (n < ns) {
                uint64_t m = sm;
                for (int c = 0; c < n; ++c) m &= m - 1;
                const int r = ctz64(m);
                part += e[tri_index(pq, tri_index(r, r))] - e[tri_index(tri_index(p, r), tri_index(r, q))];
            } else {
                uint64_t m = om;
                for (int c = 0; c < n - ns; ++c) m &= m - 1;
                const int r = ctz64(m);
                part += e[tri_index(pq, tri_index(r, r))];
            }
        }
    }
    PairVal pv;
    pv.a = beta ? xa : (xa ^ flip);
    pv.b = beta ? (xb ^ flip) : xb;
    pv.e1 = H.h64[p * H.M + q];
    pv.e2 = 0.0;
    pv.px = __longlong_as_double((long long)sr.p);
    pv.sgn = sign_bit(red_phase<PACKED>(same, p, q));
    return pv;
}

__device__ __forceinline__ bool is_single(uint64_t d) { return ((desc_pos(d) >> 14) & 127u) == kNoPos; }

// adds H_ax psi_x to w_a; hb_thr > 0: also marks a when |H_ax psi_x| >= hb_thr (the
// heat-bath screen of Eq. 14: a key enters the external sum only if some coupling
// reaches the threshold)
template <bool PACKED>
__device__ __forceinline__ bool red_add(const PairVal &pv, unsigned long long *ka_t, unsigned long long *kb_t,
                                        long long *w_hi, int *w_lo, const FixQ &fq, double hb_thr,
                                        uint32_t *hb_ok, bool &claimed) {
    const int s = red_insert<PACKED>(ka_t, kb_t, pv.a, pv.b, claimed);
    if (s < 0) return false;
    long long hi;
    int lo;
    const double t = pair_term(pv);
    fix_split(fq, t, hi, lo);
    atomicAdd(reinterpret_cast<unsigned long long *>(&w_hi[s]), (unsigned long long)hi);  // two's complement
    atomicAdd(&w_lo[s], lo);
    if (hb_thr > 0.0 && fabs(t) >= hb_thr) atomicOr(&hb_ok[s >> 5], 1u << (s & 31));
    return true;
}

// H_aa of a key from the LDS diagonal table (or the global tables when it is absent).
template <bool PACKED>
__device__ __forceinline__ double red_haa(const Ham &H, const double *vt_s, bool lds_vt, int No, uint64_t a,
                                          uint64_t b) {
    if (PACKED && H.na <= kHaaOcc && H.nb <= kHaaOcc)
        return haa_lds<uint32_t>(vt_s, No, H.M, H.na, H.nb, (uint32_t)a, (uint32_t)b, H.ecore);
    if (!PACKED && lds_vt && H.na <= kHaaOcc && H.nb <= kHaaOcc)
        return haa_lds<uint64_t>(vt_s, No, H.M, H.na, H.nb, a, b, H.ecore);
    if (PACKED) {
        const uint64_t occ = a | (b << H.M);
        double haa = H.ecore;
        uint64_t rest = occ;
        while (rest) {
            const int qo = ctz64(rest);
            rest &= rest - 1;
            double e = vt_s[qo];
            const double *row = vt_s + No + qo * (qo - 1) / 2;
            uint64_t below = occ & ((1ull << qo) - 1ull);
            while (below) {
                e += row[ctz64(below)];
                below &= below - 1;
            }
            haa += e;
        }
        return haa;
    }
    if (lds_vt) {
        // 128-bit keys: alpha p -> p, beta p -> M + p; every pair (p, q) of occupied
        // spin-orbitals once, from the row of the larger index
        double haa = H.ecore;
        uint64_t ra = a;
        while (ra) {
            const int q = ctz64(ra);
            ra &= ra - 1;
            double e = vt_s[q];
            const double *row = vt_s + No + q * (q - 1) / 2;
            uint64_t below = a & ((1ull << q) - 1ull);
            while (below) {
                e += row[ctz64(below)];
                below &= below - 1;
            }
            haa += e;
        }
        uint64_t rb = b;
        while (rb) {
            const int q = ctz64(rb);
            rb &= rb - 1;
            const int qs = H.M + q;
            double e = vt_s[qs];
            const double *row = vt_s + No + qs * (qs - 1) / 2;
            uint64_t al = a;
            while (al) {
                e += row[ctz64(al)];
                al &= al - 1;
            }
            uint64_t below = b & ((1ull << q) - 1ull);
            while (below) {
                e += row[H.M + ctz64(below)];
                below &= below - 1;
            }
            haa += e;
        }
        return haa;
    }
    return h_diag(H, a, b);
}

// Key count of sampled sub-buckets, before the reduce: workgroup i inserts the keys of
// sub-bucket i * stride (its members of S, then every pair's target) into an LDS table
// like the reduce's and stops once the table passes the reduce's fill limit.  *maxkeys
// receives the largest count.  The host uses it to cut the key space finer before the
// reduce runs, instead of after a reduce pass whose tables overflowed (few pairs per
// key: many keys per sub-bucket).
template <bool PACKED>
__global__ __launch_bounds__(kRedThreads) void k_pt2_keycount(const uint64_t *__restrict__ rec,
                                                              const uint64_t *__restrict__ desc,
                                                              const int64_t *__restrict__ sb, int64_t nsb,
                                                              int64_t stride, const uint64_t *__restrict__ skeys,
                                                              const int64_t *__restrict__ soffs, int64_t n_s,
                                                              int *__restrict__ maxkeys) {
    __shared__ unsigned long long ka_t[kRedTab];
    __shared__ unsigned long long kb_t[PACKED ? 1 : kRedTab];
    __shared__ int s_fill;
    const int64_t i = (int64_t)blockIdx.x * stride;
    if (i >= nsb) return;
    for (int t = threadIdx.x; t < kRedTab; t += blockDim.x) {
        ka_t[t] = kEmptyKey;
        if (!PACKED) kb_t[t] = kEmptyKey;
    }
    if (threadIdx.x == 0) s_fill = 0;
    __syncthreads();
    const int lane = (int)(threadIdx.x % kWave);
    auto count = [&](bool claimed) {
        const uint64_t m = __ballot(claimed);
        if (m && lane == __ffsll((unsigned long long)m) - 1) atomicAdd(&s_fill, __popcll(m));
    };
    const int64_t q0 = soffs[i], q1 = i + 1 < nsb ? soffs[i + 1] : n_s;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        bool claimed = false;
        (void)red_insert<PACKED>(ka_t, kb_t, skeys[2 * q], skeys[2 * q + 1], claimed);
        count(claimed);
    }
    __syncthreads();
    const int64_t s0 = sb[i], s1 = sb[i + 1];
    for (int64_t k0 = s0; k0 < s1; k0 += blockDim.x) {
        if (__hip_atomic_load(&s_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > kRedFillMax) break;
        const int64_t k = k0 + threadIdx.x;
        bool claimed = false;
        if (k < s1) {
            // the target: x with the descriptor's positions flipped (alpha p, beta 64 + p)
            const uint64_t d = desc[k];
            const SrcRec sr = load_src<PACKED>(rec, d);
            uint64_t a = src_alpha(sr), b = src_beta(sr);
            const uint32_t pos = desc_pos(d);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t p = (pos >> (7 * u)) & 127u;
                if (p == kNoPos) continue;
                if (p < 64)
                    a ^= 1ull << p;
                else
                    b ^= 1ull << (p - 64);
            }
            (void)red_insert<PACKED>(ka_t, kb_t, a, b, claimed);
        }
        count(claimed);
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(maxkeys, s_fill);
}

void launch_pt2_keycount(hipStream_t st, const uint64_t *rec, const uint64_t *desc, const int64_t *sb, int64_t nsb,
                         int64_t nsample, const uint64_t *skeys, const int64_t *soffs, int64_t n_s, int *maxkeys,
                         bool packed) {
    if (nsb <= 0 || nsample <= 0) return;
    const int64_t stride = std::max<int64_t>(1, nsb / nsample);
    const int64_t nwg = (nsb + stride - 1) / stride;
    if (packed)
        hipLaunchKernelGGL(k_pt2_keycount<true>, dim3((unsigned)nwg), dim3(kRedThreads), 0, st, rec, desc, sb, nsb,
                           stride, skeys, soffs, n_s, maxkeys);
    else
        hipLaunchKernelGGL(k_pt2_keycount<false>, dim3((unsigned)nwg), dim3(kRedThreads), 0, st, rec, desc, sb, nsb,
                           stride, skeys, soffs, n_s, maxkeys);
}

int pt2_red_fill_max() { return kRedFillMax; }

// Per sub-bucket output part[kRedPart * sub-bucket]:
//   [0] external sum over its keys of P (exact workgroup sum, see red_final)
//   [1] min |E - H_aa| over those keys      [2] their number     [3] those with |E - H_aa| < 1e-8
//   [4], [5] (bits) sum mod 2^64 and XOR of key_hash(a) over those keys (order-free
//   fingerprint of P)
// and, for each member a of S in the sub-bucket, int_term[index of a] =
// (v_a - E psi_a)^2 / (E - H_aa) with v_a = w_a + H_aa psi_a (w_a: the off-diagonal
// part of (H_SS psi)_a, summed exactly from FP64 couplings like the external w_a).
template <bool PACKED>
__global__ __launch_bounds__(kRedThreads) void k_pt2_reduce(Ham H, const uint64_t *__restrict__ rec,
                                                            const uint64_t *__restrict__ desc,
                                                            const int64_t *__restrict__ sb,
                                                            const uint64_t *__restrict__ skeys,
                                                            const int32_t *__restrict__ sidx,
                                                            const int64_t *__restrict__ soffs, int64_t n_s,
                                                            int64_t nsb, const double *__restrict__ vt,
                                                            const double *__restrict__ energy, uint64_t sample_mask,
                                                            int wexp, double hb_eps,
                                                            const double *__restrict__ norm2, PT2Export ex,
                                                            double *__restrict__ part,
                                                            double *__restrict__ int_term,
                                                            int *__restrict__ overflow) {
    __shared__ unsigned long long ka_t[kRedTab];
    __shared__ unsigned long long kb_t[PACKED ? 1 : kRedTab];
    __shared__ long long w_hi[kRedTab];
    __shared__ int w_lo[kRedTab];
    __shared__ uint32_t in_s[kRedTab / 32];
    __shared__ uint32_t hb_ok[kRedTab / 32];  // heat-bath screen passed (hb_eps > 0)
    __shared__ uint64_t sq[kRedSingles];  // single excitations, deferred
    __shared__ int nsq;
    __shared__ int s_lost;  // a key did not fit: this pass is redone, so stop early
    __shared__ int s_fill;  // occupied slots
    extern __shared__ double vt_s[];  // diagonal table, sized at launch (empty: global tables)
    for (int t = threadIdx.x; t < kRedTab; t += blockDim.x) {
        ka_t[t] = kEmptyKey;
        if (!PACKED) kb_t[t] = kEmptyKey;
        w_hi[t] = 0;
        w_lo[t] = 0;
    }
    for (int t = threadIdx.x; t < kRedTab / 32; t += blockDim.x) {
        in_s[t] = 0u;
        hb_ok[t] = 0u;
    }
    if (threadIdx.x == 0) {
        nsq = 0;
        s_lost = 0;
        s_fill = 0;
    }
    // |H_ax psi_x| >= hb_eps ||psi||_2 (psi in any scale: the threshold is on the normalised psi)
    const double hb_thr = hb_eps > 0.0 ? hb_eps * sqrt(norm2[0]) : 0.0;
    const int No = 2 * H.M;
    const bool lds_vt = vt != nullptr;  // else (M > 62) H_aa from the global J, K tables
    if (lds_vt)
        for (int t = threadIdx.x; t < No + No * (No - 1) / 2; t += blockDim.x) vt_s[t] = vt[t];
    __syncthreads();
    // s_lost and s_fill are read while other waves update them: relaxed LDS atomics (a
    // volatile pointer would become a generic one, whose loads wait for every load in flight)
    auto set_lost = [&]() { __hip_atomic_store(&s_lost, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
    // members of S that hash into this sub-bucket: in the table, marked
    const int64_t q0 = soffs[blockIdx.x], q1 = blockIdx.x + 1 < nsb ? soffs[blockIdx.x + 1] : n_s;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        bool claimed = false;
        const int s = red_insert<PACKED>(ka_t, kb_t, skeys[2 * q], skeys[2 * q + 1], claimed);
        if (claimed) atomicAdd(&s_fill, 1);
        if (s < 0)
            set_lost();
        else
            atomicOr(&in_s[s >> 5], 1u << (s & 31));
    }
    __syncthreads();
    const int64_t s0 = sb[blockIdx.x], s1 = sb[blockIdx.x + 1], step = blockDim.x;
    const FixQ fq = make_fixq(wexp, s1 - s0);
    // Doubles first.  A single excitation's value sums over all occupied orbitals
    // (~3 N_e integral loads against 1-2 for a double); at ~1% of the pairs in random
    // order, handled inline they would stall about half of the waves, so they are queued
    // and done together after the doubles.
    // The per-pair work is a chain of dependent loads (descriptor from HBM, then the source
    // record, then the integrals, from L2), so the loop is software-pipelined: the
    // descriptor of pair k + 4 and the source record of pair k + 1 are loaded while pair k
    // is done.  The loop is unrolled over a ring of four descriptor and two record
    // registers (no register moves, which would wait for the newest load), the loads are
    // unconditional (index clamped into the sub-bucket) and come after the current pair's
    // integral loads, so that every wait is for a count of loads and never for a
    // prefetch.  Singles go to the LDS queue; if it fills up they are all redone by a
    // rescan instead.
    if (s1 > s0) {
        // in-bucket offsets in 32 bits (a sub-bucket holds far fewer than 2^31 pairs)
        const uint64_t *dsb = desc + s0;
        const int nsub = (int)(s1 - s0), base = (int)threadIdx.x, stp = (int)step;
        auto ld_desc = [&](int k) { return dsb[min(base + k * stp, nsub - 1)]; };
        uint64_t D0 = ld_desc(0), D1 = ld_desc(1), D2 = ld_desc(2), D3 = ld_desc(3);
        SrcRec R0 = load_src<PACKED>(rec, D0), R1{};
        // pair k: descriptor Dk, record Rk; loads the record of pair k + 1 (from Dn) into
        // Rn and the descriptor of pair k + 4 into Dk
        auto stage = [&](int k, uint64_t &Dk, const SrcRec &Rk, const uint64_t &Dn, SrcRec &Rn) {
            const uint64_t d = Dk;
            const PairVal pv = double_value<PACKED>(H, Rk, d);
            Rn = load_src<PACKED>(rec, Dn);
            Dk = ld_desc(k + 4);
            bool claimed = false;
            if (base + k * stp < nsub) {
                if (is_single(d)) {
                    const int q = atomicAdd(&nsq, 1);
                    if (q < kRedSingles) sq[q] = d;
                } else if (!red_add<PACKED>(pv, ka_t, kb_t, w_hi, w_lo, fq, hb_thr, hb_ok, claimed)) {
                    set_lost();
                }
            }
            // the wave's newly claimed slots, one atomic (no return value)
            const uint64_t m = __ballot(claimed);
            if (m && (int)(threadIdx.x % kWave) == __ffsll((unsigned long long)m) - 1) atomicAdd(&s_fill, __popcll(m));
        };
        for (int k = 0; base + k * stp < nsub; k += 4) {
            const int lost_now = __hip_atomic_load(&s_lost, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int fill_now = __hip_atomic_load(&s_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lost_now | (fill_now > kRedFillMax)) break;  // per wave; the workgroup leaves together below
            stage(k, D0, R0, D1, R1);
            stage(k + 1, D1, R1, D2, R0);
            stage(k + 2, D2, R0, D3, R1);
            stage(k + 3, D3, R1, D0, R0);
        }
    }
    __syncthreads();
    // the same values on every thread after the barrier
    if (__builtin_amdgcn_readfirstlane(s_lost) | (__builtin_amdgcn_readfirstlane(s_fill) > kRedFillMax)) {
        if (threadIdx.x == 0) atomicOr(overflow, 1);
        return;
    }
    if (nsq <= kRedSingles) {
        // eight lanes per queued single, each summing every eighth occupied orbital
        for (int k0 = 0; k0 < nsq; k0 += kRedThreads / 8) {
            const int k = k0 + (int)(threadIdx.x >> 3), l = (int)(threadIdx.x & 7);
            const bool have = k < nsq;
            PairVal pv{};
            double part_v = 0.0;
            if (have) pv = single_part<PACKED>(H, load_src<PACKED>(rec, sq[k]), sq[k], l, part_v);
            part_v += __shfl_xor(part_v, 1, 8);
            part_v += __shfl_xor(part_v, 2, 8);
            part_v += __shfl_xor(part_v, 4, 8);
            if (have && l == 0) {
                pv.e1 += part_v;
                bool claimed = false;
                if (!red_add<PACKED>(pv, ka_t, kb_t, w_hi, w_lo, fq, hb_thr, hb_ok, claimed)) set_lost();
                if (claimed) atomicAdd(&s_fill, 1);
            }
        }
    } else {
        for (int64_t i = s0 + threadIdx.x; i < s1; i += step) {
            const uint64_t d = desc[i];
            bool claimed = false;
            if (is_single(d) &&
                !red_add<PACKED>(single_pair<PACKED>(H, load_src<PACKED>(rec, d), d), ka_t, kb_t, w_hi, w_lo, fq, hb_thr,
                                 hb_ok, claimed))
                set_lost();
            if (claimed) atomicAdd(&s_fill, 1);
        }
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_lost) | (__builtin_amdgcn_readfirstlane(s_fill) > kRedFillMax)) {
        if (threadIdx.x == 0) atomicOr(overflow, 1);
        return;
    }
    const double E = energy[0];
    // internal term of the members of S in this sub-bucket (few per sub-bucket)
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const uint64_t a = skeys[2 * q], b = skeys[2 * q + 1];
        const int s = red_find<PACKED>(ka_t, kb_t, a, b);
        if (s < 0) continue;  // not reached: every member was inserted
        const int32_t xi = sidx[q];
        const double pa = __longlong_as_double((long long)(PACKED ? rec[2 * (int64_t)xi + 1] : rec[4 * (int64_t)xi + 2]));
        const double w = fix_join(fq, w_hi[s], w_lo[s]);
        const double haa = red_haa<PACKED>(H, vt_s, lds_vt, No, a, b);
        const double r = w + (haa - E) * pa;
        const double num = r * r;
        int_term[xi] = num != 0.0 ? num / (E - haa) : 0.0;
    }
    // compact the keys that enter the sum (not in S, in the sample) to the front of the
    // table, so that every lane of the H_aa loop below has a key
    constexpr int kPer = kRedTab / kRedThreads;
    unsigned long long ck[kPer], cb[kPer];
    double cw[kPer];
    uint32_t live = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = threadIdx.x + j * kRedThreads;
        ck[j] = ka_t[t];
        cb[j] = PACKED ? 0ull : kb_t[t];
        cw[j] = fix_join(fq, w_hi[t], w_lo[t]);
        bool ok = (PACKED ? ck[j] : cb[j]) != kEmptyKey && !((in_s[t >> 5] >> (t & 31)) & 1u);
        if (hb_thr > 0.0) ok = ok && ((hb_ok[t >> 5] >> (t & 31)) & 1u);
        if (ok && sample_mask) {
            const uint64_t a = PACKED ? (ck[j] & 0xffffffffull) : ck[j], b = PACKED ? (ck[j] >> 32) : cb[j];
            ok = !(key_hash(a, b) & sample_mask);
        }
        live |= (ok ? 1u : 0u) << j;
    }
    uint32_t n_live = 0;
    uint32_t pos = red_scan((uint32_t)__popc(live), n_live);
    __syncthreads();
    double *w_t = reinterpret_cast<double *>(w_hi);  // the fixed-point table is read out: reuse it
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if ((live >> j) & 1u) {
            ka_t[pos] = ck[j];
            if (!PACKED) kb_t[pos] = cb[j];
            w_t[pos] = cw[j];
            ++pos;
        }
    __syncthreads();
    // one pass over the live keys (a plain loop, so H_aa's code appears once): the term
    // w_a^2 / (E - H_aa) replaces w_a in its slot
    double mn = INFINITY, np = 0.0, nt = 0.0;
    unsigned long long fsum = 0ull, fxor = 0ull;
    for (int t = threadIdx.x; t < (int)n_live; t += kRedThreads) {
        uint64_t a, b;
        if (PACKED) {
            const unsigned long long k = ka_t[t];
            a = k & 0xffffffffull;
            b = k >> 32;
        } else {
            a = ka_t[t];
            b = kb_t[t];
        }
        const double w = w_t[t];
        const double haa = red_haa<PACKED>(H, vt_s, lds_vt, No, a, b);
        const double den = E - haa;
        np += 1.0;
        mn = fmin(mn, fabs(den));
        if (fabs(den) < 1e-8) nt += 1.0;
        w_t[t] = w != 0.0 ? w * w / den : 0.0;
        const uint64_t kh = key_hash(a, b);
        fsum += kh;
        fxor ^= kh;
        if (ex.cap > 0) {
            const unsigned long long k = atomicAdd((unsigned long long *)ex.count, 1ull);
            if ((int64_t)k < ex.cap) {
                ex.keys[2 * k] = a;
                ex.keys[2 * k + 1] = b;
                ex.w[k] = w;
                ex.haa[k] = haa;
            }
        }
    }
    // this thread's terms (its own slots, written above) into registers for the exact sum
    double terms[kPer];
    int nterm = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = threadIdx.x + j * kRedThreads;
        terms[j] = t < (int)n_live ? w_t[t] : 0.0;
        if (t < (int)n_live) nterm = j + 1;
    }
    red_final<kPer>(terms, nterm, mn, np, nt, fsum, fxor, part + (int64_t)kRedPart * blockIdx.x);
}

void launch_pt2_reduce(hipStream_t st, const Ham &H, const uint64_t *rec, const uint64_t *desc,
                       const int64_t *sb, int64_t nsb, const uint64_t *skeys, const int32_t *sidx,
                       const int64_t *soffs, int64_t n_s, const double *vt, const double *energy,
                       uint64_t sample_mask, int wexp, double hb_eps, const double *norm2, const PT2Export &ex,
                       double *part, double *int_term, int *overflow, bool packed) {
    dim3 grid((unsigned)nsb), blk(kRedThreads);
    const size_t vt_bytes = sizeof(double) * pt2_diag_table_size(H.M);
    if (packed)
        hipLaunchKernelGGL(k_pt2_reduce<true>, grid, blk, vt_bytes, st, H, rec, desc, sb, skeys, sidx, soffs, n_s,
                           nsb, vt, energy, sample_mask, wexp, hb_eps, norm2, ex, part, int_term, overflow);
    else if (pt2_diag_table_fits(H.M))
        hipLaunchKernelGGL(k_pt2_reduce<false>, grid, blk, vt_bytes, st, H, rec, desc, sb, skeys, sidx, soffs, n_s,
                           nsb, vt, energy, sample_mask, wexp, hb_eps, norm2, ex, part, int_term, overflow);
    else
        hipLaunchKernelGGL(k_pt2_reduce<false>, grid, blk, 0, st, H, rec, desc, sb, skeys, sidx, soffs, n_s, nsb,
                           (const double *)nullptr, energy, sample_mask, wexp, hb_eps, norm2, ex, part, int_term, overflow);
}

int pt2_red_tab() { return kRedTab; }
int pt2_red_part() { return kRedPart; }

}  // namespace dnqs
