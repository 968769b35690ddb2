// Enumeration of the single and double excitations of one determinant by a wavefront.
//
// The wave writes the occupied and empty orbitals of each spin string to LDS once;
// lanes then map excitation ids e in [0, n_exc) in closed form onto
//   [alpha singles | beta singles | alpha-alpha doubles | beta-beta doubles | alpha-beta doubles]
// and return the flipped spin-orbitals as four 7-bit positions (alpha p -> p,
// beta p -> 64 + p, unused -> 127).  The target is x XOR those bits.
#pragma once
#include "dnqs_device.h"

namespace dnqs {

constexpr uint32_t kNoPos = 127u;

// a * b for a, b < 2^24 with a product below 2^32, as v_mul_u32_u24 (full rate; a 32-bit
// integer multiply issues at a quarter of the rate), written out so that the compiler
// keeps it
__device__ __forceinline__ int mul24(int a, int b) {
    int p;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(p) : "v"(a), "v"(b));
    return p;
}

// n / d and n % d for 0 <= n, d < 2^24: a float-reciprocal estimate (off by at most a
// few) corrected to the exact quotient with integer arithmetic.
struct FastDiv {
    int d;
    float r;
};

__device__ __forceinline__ FastDiv make_fastdiv(int d) { return FastDiv{d, 1.0f / (float)d}; }

__device__ __forceinline__ int fdiv(int n, const FastDiv &f, int &rem) {
    int q = (int)((float)n * f.r);
    int r = n - mul24(q, f.d);  // q d <= n + a few d < 2^25
    while (r < 0) {
        --q;
        r += f.d;
    }
    while (r >= f.d) {
        ++q;
        r -= f.d;
    }
    rem = r;
    return q;
}

// Excitation ids are below 2^24 (n_exc of any sector with M <= 64 is ~1.4e6 at most).
struct ExcLists {
    const uint8_t *oa, *va, *ob, *vb;  // occupied / empty orbitals per spin string
    FastDiv nva, nvb, pva, pvb, nsb;   // class sizes used as divisors
    int c1, c2, c3, c4, total;         // class boundaries
};

// pair index t over n items (i < j), ordered by j then i: t = j(j-1)/2 + i
__device__ __forceinline__ void unrank_pair(int t, int &i, int &j) {
    int jj = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
    while (mul24(jj, jj - 1) / 2 > t) --jj;  // jj < 2^13
    while (mul24(jj + 1, jj) / 2 <= t) ++jj;
    j = jj;
    i = t - mul24(jj, jj - 1) / 2;
}

// Fill lists[4][64] for det (xa, xb) with one wavefront (lanes 0..M-1 take part).
__device__ inline void wave_build_lists(uint8_t (*lists)[64], int M, uint64_t xa, uint64_t xb) {
    const int lane = __lane_id();
    const bool in = lane < M;
    const bool ba = in && ((xa >> lane) & 1ull), bb = in && ((xb >> lane) & 1ull);
    const uint64_t moa = __ballot(ba), mva = __ballot(in && !ba), mob = __ballot(bb), mvb = __ballot(in && !bb);
    if (ba) lists[0][mbcnt(moa)] = (uint8_t)lane;
    if (in && !ba) lists[1][mbcnt(mva)] = (uint8_t)lane;
    if (bb) lists[2][mbcnt(mob)] = (uint8_t)lane;
    if (in && !bb) lists[3][mbcnt(mvb)] = (uint8_t)lane;
}

__device__ inline ExcLists make_exc_lists(const uint8_t (*lists)[64], int M, int na, int nb) {
    ExcLists c;
    c.oa = lists[0];
    c.va = lists[1];
    c.ob = lists[2];
    c.vb = lists[3];
    const int nva = M - na, nvb = M - nb;
    const int nsa = na * nva, nsb = nb * nvb;
    const int pva = nva * (nva - 1) / 2, pvb = nvb * (nvb - 1) / 2;
    // a size-0 class is never divided by; keep its divisor at 1
    c.nva = make_fastdiv(nva > 0 ? nva : 1);
    c.nvb = make_fastdiv(nvb > 0 ? nvb : 1);
    c.pva = make_fastdiv(pva > 0 ? pva : 1);
    c.pvb = make_fastdiv(pvb > 0 ? pvb : 1);
    c.nsb = make_fastdiv(nsb > 0 ? nsb : 1);
    const int ndaa = na * (na - 1) / 2 * pva, ndbb = nb * (nb - 1) / 2 * pvb;
    c.c1 = nsa;
    c.c2 = c.c1 + nsb;
    c.c3 = c.c2 + ndaa;
    c.c4 = c.c3 + ndbb;
    c.total = c.c4 + nsa * nsb;
    return c;
}

__device__ __forceinline__ uint32_t pack_pos(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3) {
    return p0 | (p1 << 7) | (p2 << 14) | (p3 << 21);
}

// flipped positions of excitation e (0 <= e < total)
__device__ inline uint32_t excitation_positions(const ExcLists &c, int e) {
    int r;
    if (e < c.c1) {
        const int q = fdiv(e, c.nva, r);
        return pack_pos(c.oa[q], c.va[r], kNoPos, kNoPos);
    }
    if (e < c.c2) {
        const int q = fdiv(e - c.c1, c.nvb, r);
        return pack_pos(64u + c.ob[q], 64u + c.vb[r], kNoPos, kNoPos);
    }
    if (e < c.c3) {
        int i, j, a, b;
        const int q = fdiv(e - c.c2, c.pva, r);
        unrank_pair(q, i, j);
        unrank_pair(r, a, b);
        return pack_pos(c.oa[i], c.oa[j], c.va[a], c.va[b]);
    }
    if (e < c.c4) {
        int i, j, a, b;
        const int q = fdiv(e - c.c3, c.pvb, r);
        unrank_pair(q, i, j);
        unrank_pair(r, a, b);
        return pack_pos(64u + c.ob[i], 64u + c.ob[j], 64u + c.vb[a], 64u + c.vb[b]);
    }
    int sb;
    const int sa = fdiv(e - c.c4, c.nsb, sb);
    int ra, rb;
    const int qa = fdiv(sa, c.nva, ra), qb = fdiv(sb, c.nvb, rb);
    return pack_pos(c.oa[qa], c.va[ra], 64u + c.ob[qb], 64u + c.vb[rb]);
}

// target = x with the bits at the packed positions flipped
__device__ __forceinline__ void apply_positions(uint32_t pos, uint64_t &a, uint64_t &b) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t p = (pos >> (7 * k)) & 127u;
        if (p == kNoPos) continue;
        if (p < 64u)
            a ^= 1ull << p;
        else
            b ^= 1ull << (p - 64u);
    }
}

__device__ __forceinline__ uint64_t pack_key(uint64_t a, uint64_t b) { return a | (b << 32); }

// key hash of a target; packed keys (M <= 32) hash the packed word
template <bool PACKED>
__device__ __forceinline__ uint64_t target_hash(uint64_t a, uint64_t b) {
    return PACKED ? mix64(pack_key(a, b)) : key_hash(a, b);
}

}  // namespace dnqs
