// Device-side building blocks shared by the HIP kernels of the library.
// gfx950 only: wave64, MFMA, 160 KB LDS per CU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dnqs {

constexpr int kWave = 64;
constexpr uint64_t kEmptyKey = ~0ull;

// Integral tables of one geometry, all device pointers.
struct Ham {
    int M, na, nb;
    double ecore;
    const double *h64;    // [M*M]
    const double *eri64;  // [M^4], (pq|rs) at ((p*M+q)*M+r)*M+s
    const float *eri32;   // [M^4]
    const double *eri_pk; // 8-fold packed (pq|rs): index pair(pair(p,q), pair(r,s))
    const double *J;      // [M*M], (pp|qq)
    const double *K;      // [M*M], (pq|qp)
};

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }

// bits strictly between lo and hi (lo != hi, both in [0, 63])
__device__ __forceinline__ uint64_t between_mask(int p, int q) {
    int lo = p < q ? p : q, hi = p < q ? q : p;
    return ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
}

// (-1)^(occupied orbitals of s strictly between p and q), as +1/-1
__device__ __forceinline__ int phase_between(uint64_t s, int p, int q) {
    return (popc64(s & between_mask(p, q)) & 1) ? -1 : 1;
}

__device__ __forceinline__ size_t eri_index(int M, int p, int q, int r, int s) {
    return (((size_t)p * M + q) * M + r) * M + s;
}

// Slater-Condon rule 0: <x|H|x> in FP64.
__device__ inline double h_diag(const Ham &H, uint64_t a, uint64_t b) {
    const int M = H.M;
    double e = H.ecore;
    uint64_t ta = a;
    while (ta) {
        int p = ctz64(ta);
        ta &= ta - 1;
        e += H.h64[p * M + p];
        uint64_t ra = ta;  // alpha q > p
        while (ra) {
            int q = ctz64(ra);
            ra &= ra - 1;
            e += H.J[p * M + q] - H.K[p * M + q];
        }
        uint64_t rb = b;  // every beta q
        while (rb) {
            int q = ctz64(rb);
            rb &= rb - 1;
            e += H.J[p * M + q];
        }
    }
    uint64_t tb = b;
    while (tb) {
        int p = ctz64(tb);
        tb &= tb - 1;
        e += H.h64[p * M + p];
        uint64_t rb = tb;
        while (rb) {
            int q = ctz64(rb);
            rb &= rb - 1;
            e += H.J[p * M + q] - H.K[p * M + q];
        }
    }
    return e;
}

// index of an unordered pair (p, q) in the lower triangle
__device__ __forceinline__ int tri_index(int p, int q) { return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p; }

// (pq|rs) from the dense M^4 table
template <typename T>
struct EriDense {
    const T *e;
    int M;
    __device__ __forceinline__ double operator()(int p, int q, int r, int s) const {
        return (double)e[eri_index(M, p, q, r, s)];
    }
};

// (pq|rs) from the 8-fold packed FP64 table (M = 28: 661 KB, resident in L2)
struct EriPacked {
    const double *e;
    __device__ __forceinline__ double operator()(int p, int q, int r, int s) const {
        return e[tri_index(tri_index(p, q), tri_index(r, s))];
    }
};

// Single excitation q -> p on spin string `same` (the ket's string of that spin,
// q occupied, p empty); `other` is the ket's opposite-spin string.
// value (without phase) = h_pq + sum_{r in same, r != q} [(pq|rr) - (pr|rq)]
//                               + sum_{r in other} (pq|rr)
template <typename ERI>
__device__ inline double single_value(const Ham &H, const ERI &eri, int p, int q, uint64_t same, uint64_t other) {
    const int M = H.M;
    double v = H.h64[p * M + q];
    uint64_t s = same & ~(1ull << q);
    while (s) {
        int r = ctz64(s);
        s &= s - 1;
        v += eri(p, q, r, r) - eri(p, r, r, q);
    }
    uint64_t o = other;
    while (o) {
        int r = ctz64(o);
        o &= o - 1;
        v += eri(p, q, r, r);
    }
    return v;
}

// <x|H|y> for x != y of one sector, by comparing the strings.  Returns 0 for rank > 2.
// Holes (occupied in y only) and particles (occupied in x only) are paired in
// ascending order; the phase is that of applying the pairs one after the other.
template <typename ERI>
__device__ inline double h_offdiag(const Ham &H, const ERI &eri, uint64_t xa, uint64_t xb, uint64_t ya, uint64_t yb) {
    uint64_t da = xa ^ ya, db = xb ^ yb;
    int na = popc64(da), nb = popc64(db);
    if (na + nb == 2) {
        if (na == 2) {
            int q = ctz64(ya & da), p = ctz64(xa & da);
            return phase_between(ya, p, q) * single_value(H, eri, p, q, ya, yb);
        } else {
            int q = ctz64(yb & db), p = ctz64(xb & db);
            return phase_between(yb, p, q) * single_value(H, eri, p, q, yb, ya);
        }
    }
    if (na + nb != 4) return 0.0;
    if (na == 4 || nb == 4) {  // same-spin double
        uint64_t s = na == 4 ? ya : yb;
        uint64_t hole = s & (na == 4 ? da : db);
        uint64_t part = (na == 4 ? xa : xb) & (na == 4 ? da : db);
        int i = ctz64(hole);
        int j = ctz64(hole & (hole - 1));
        int a = ctz64(part);
        int b = ctz64(part & (part - 1));
        int s1 = phase_between(s, i, a);
        uint64_t s_1 = (s & ~(1ull << i)) | (1ull << a);
        int s2 = phase_between(s_1, j, b);
        double v = eri(a, i, b, j) - eri(a, j, b, i);
        return s1 * s2 * v;
    }
    // alpha-beta double
    int i = ctz64(ya & da), a = ctz64(xa & da);
    int j = ctz64(yb & db), b = ctz64(xb & db);
    int sg = phase_between(ya, i, a) * phase_between(yb, j, b);
    return sg * eri(a, i, b, j);
}

// SplitMix64 output function (Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

__device__ __forceinline__ uint64_t key_hash(uint64_t a, uint64_t b) { return mix64(a ^ mix64(b)); }

// ---------------------------------------------------------------- hash set of S
// Open addressing, linear probing, capacity a power of two.  keys[2*i], keys[2*i+1]
// hold (alpha, beta); kEmptyKey in the alpha word marks an empty slot.  idx[i] is the
// position of the det in S.
struct DetSet {
    const uint64_t *keys;
    const int32_t *idx;
    uint64_t mask;
};

__device__ inline int32_t detset_find(const DetSet &S, uint64_t a, uint64_t b) {
    uint64_t h = key_hash(a, b) & S.mask;
    for (;;) {
        uint64_t ka = S.keys[2 * h];
        if (ka == kEmptyKey) return -1;
        if (ka == a && S.keys[2 * h + 1] == b) return S.idx[h];
        h = (h + 1) & S.mask;
    }
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of mask below this lane
__device__ __forceinline__ int mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Off-diagonal part of row x of H_SS times psi by one wave (sum of the lanes' partial
// sums; the caller reduces across the wave).  Eight independent FP64 partial sums per
// lane, combined in a fixed order.
__device__ __forceinline__ double row_dot_lane(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                               const float *__restrict__ val, const double *__restrict__ psi,
                                               int64_t x, int lane) {
    // Eight elements per lane and step: the 16 index/value reads go out together, then the
    // 8 psi gathers, so a row of a few hundred elements costs a few memory round trips.
    // Slots past the row end read the row's first element and add 0.
    const int64_t b = row_ptr[x], e = row_ptr[x + 1];
    double s[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] = 0.0;
    for (int64_t j0 = b + lane; j0 < e; j0 += 8 * kWave) {
        int32_t c[8];
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t j = j0 + u * kWave;
            const int64_t jj = j < e ? j : b;
            c[u] = col[jj];
            v[u] = val[jj];
            if (j >= e) v[u] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += (double)v[u] * psi[c[u]];
    }
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace dnqs
