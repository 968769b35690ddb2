/*
 * FP64 CPU oracle: the combinatorial half of the deterministic NQS method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product path (the HIP library) never
 * links, loads or calls it, and shares no code with it.
 *
 * Everything here is written to be read against the paper, not to be fast:
 *   - operator algebra on Fock states: the dense second-quantised Hamiltonian built
 *     by applying creation/annihilation strings to basis states (a brute-force pin
 *     for the Slater-Condon rules, which the paper's discrete combinatorial kernel
 *     evaluates, Sec. 3.1);
 *   - the Slater-Condon matrix element <x|H|y> between two determinants, found by
 *     comparing the two occupation strings;
 *   - H_SS in CSR by its definition: for each row x, every y in S whose excitation
 *     rank relative to x is 1 or 2 (the off-diagonal part), plus the diagonal;
 *   - generation of all single and double excitations of x (the connected set C of
 *     Eq. 1, read structurally as excitation rank <= 2);
 *   - the external Epstein-Nesbet sum of Eq. 13 over P = C \ S;
 *   - w_a = sum_{x in S} H_ax psi_x for one given a, by enumerating the excitations
 *     of a and looking each one up in S.
 *
 * Conventions (the paper does not fix them; the HIP path uses the same ones):
 *   det = (alpha string, beta string), bit p = spatial orbital p, M <= 64;
 *   spin-orbital index: alpha p -> p, beta p -> M + p;
 *   |x> = a+_{i1} ... a+_{iN} |0> with i1 < ... < iN;
 *   a_k, a+_k carry the sign (-1)^(number of occupied spin-orbitals below k);
 *   H = E_core + sum h_pq a+_{p s} a_{q s} + 1/2 sum (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s},
 *   with (pq|rs) in chemists' notation, eri[((p*M+q)*M+r)*M+s].
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC sc_oracle.c -o libsc_oracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int M;
    const double *h;
    const double *eri;
    double ecore;
} ham_t;

static double ERI(const ham_t *H, int p, int q, int r, int s) {
    int M = H->M;
    return H->eri[(((size_t)p * M + q) * M + r) * M + s];
}

/* ------------------------------------------------------------------ Fock states */
/* A Fock state over 2M spin-orbitals, held as the two spin strings. */
typedef struct {
    uint64_t a, b;
} fock_t;

static int fock_bit(fock_t z, int M, int k) {
    return k < M ? (int)((z.a >> k) & 1u) : (int)((z.b >> (k - M)) & 1u);
}

static void fock_set(fock_t *z, int M, int k, int v) {
    uint64_t *w = k < M ? &z->a : &z->b;
    int bit = k < M ? k : k - M;
    if (v)
        *w |= (uint64_t)1 << bit;
    else
        *w &= ~((uint64_t)1 << bit);
}

/* number of occupied spin-orbitals with index < k */
static int fock_below(fock_t z, int M, int k) {
    int c = 0;
    for (int t = 0; t < k; ++t) c += fock_bit(z, M, t);
    return c;
}

/* apply a_k; returns sign (+1/-1) or 0 if the result vanishes */
static int op_annihilate(fock_t *z, int M, int k) {
    if (!fock_bit(*z, M, k)) return 0;
    int s = (fock_below(*z, M, k) & 1) ? -1 : 1;
    fock_set(z, M, k, 0);
    return s;
}

/* apply a+_k */
static int op_create(fock_t *z, int M, int k) {
    if (fock_bit(*z, M, k)) return 0;
    int s = (fock_below(*z, M, k) & 1) ? -1 : 1;
    fock_set(z, M, k, 1);
    return s;
}

static int cmp_det(uint64_t xa, uint64_t xb, uint64_t ya, uint64_t yb) {
    if (xa != ya) return xa < ya ? -1 : 1;
    if (xb != yb) return xb < yb ? -1 : 1;
    return 0;
}

/* index of (a,b) in the canonically sorted det list, or -1 */
static int64_t find_det(const uint64_t *dets, int64_t n, uint64_t a, uint64_t b) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_det(dets[2 * mid], dets[2 * mid + 1], a, b);
        if (c == 0) return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/*
 * Dense Hamiltonian over a basis (sorted canonical dets, all of one sector) by
 * operator algebra: H[r*n + c] = <basis_r| H |basis_c>.  Brute force: every term of
 * the second-quantised operator is applied to every basis state.
 */
int or_dense_opalg(int M, const double *h, const double *eri, double ecore, const uint64_t *basis,
                   int64_t n, double *Hout) {
    ham_t H = {M, h, eri, ecore};
    int No = 2 * M;
    memset(Hout, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t c = 0; c < n; ++c) {
        fock_t y = {basis[2 * c], basis[2 * c + 1]};
        Hout[c * n + c] += ecore;
        /* one-body: sum_{PQ, same spin} h_pq a+_P a_Q */
        for (int P = 0; P < No; ++P)
            for (int Q = 0; Q < No; ++Q) {
                if ((P < M) != (Q < M)) continue;
                fock_t z = y;
                int s = op_annihilate(&z, M, Q);
                if (!s) continue;
                s *= op_create(&z, M, P);
                if (!s) continue;
                int64_t r = find_det(basis, n, z.a, z.b);
                if (r < 0) return -1;
                Hout[r * n + c] += s * h[(P % M) * M + (Q % M)];
            }
        /* two-body: 1/2 sum (pq|rs) a+_P a+_R a_S a_Q, spin(P)=spin(Q), spin(R)=spin(S) */
        for (int P = 0; P < No; ++P)
            for (int Q = 0; Q < No; ++Q) {
                if ((P < M) != (Q < M)) continue;
                for (int R = 0; R < No; ++R)
                    for (int S = 0; S < No; ++S) {
                        if ((R < M) != (S < M)) continue;
                        fock_t z = y;
                        int s = op_annihilate(&z, M, Q);
                        if (!s) continue;
                        s *= op_annihilate(&z, M, S);
                        if (!s) continue;
                        s *= op_create(&z, M, R);
                        if (!s) continue;
                        s *= op_create(&z, M, P);
                        if (!s) continue;
                        int64_t r = find_det(basis, n, z.a, z.b);
                        if (r < 0) return -1;
                        Hout[r * n + c] += 0.5 * s * ERI(&H, P % M, Q % M, R % M, S % M);
                    }
            }
    }
    return 0;
}

/* ------------------------------------------------------------------ Slater-Condon */
static int popc64(uint64_t v) { return __builtin_popcountll(v); }

/* spin-orbital string as a 2M-long bit array; occupied count strictly between lo and hi */
static int occ_between(fock_t z, int M, int lo, int hi) {
    if (lo > hi) {
        int t = lo;
        lo = hi;
        hi = t;
    }
    int c = 0;
    for (int k = lo + 1; k < hi; ++k) c += fock_bit(z, M, k);
    return c;
}

/* list the spin-orbitals set in mask (a 2M string given as two words), ascending */
static int list_bits(uint64_t ma, uint64_t mb, int M, int *out) {
    int n = 0;
    for (int k = 0; k < 2 * M; ++k) {
        int bit = k < M ? (int)((ma >> k) & 1u) : (int)((mb >> (k - M)) & 1u);
        if (bit) out[n++] = k;
    }
    return n;
}

/* Slater-Condon rule 0: <y|H|y> */
double or_hdiag(int M, const double *h, const double *eri, double ecore, uint64_t ya, uint64_t yb) {
    ham_t H = {M, h, eri, ecore};
    int occ[128];
    int n = list_bits(ya, yb, M, occ);
    double e = ecore;
    for (int i = 0; i < n; ++i) {
        int p = occ[i] % M;
        e += h[p * M + p];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            int p = occ[i] % M, r = occ[j] % M;
            int same = (occ[i] < M) == (occ[j] < M);
            e += 0.5 * ERI(&H, p, p, r, r);
            if (same) e -= 0.5 * ERI(&H, p, r, r, p);
        }
    return e;
}

/*
 * <x|H|y> by the Slater-Condon rules.  Holes are the spin-orbitals occupied in y but
 * not in x, particles the reverse.  Excitation rank 0, 1 and 2 give the diagonal, a
 * single and a double; higher ranks give 0.  The phase is the sign of the operator
 * string that maps y to x, applied one hole/particle pair at a time (holes and
 * particles each in ascending order; the k-th hole goes to the k-th particle).
 */
double or_hxy(int M, const double *h, const double *eri, double ecore, uint64_t xa, uint64_t xb,
              uint64_t ya, uint64_t yb) {
    ham_t H = {M, h, eri, ecore};
    uint64_t ha = ya & ~xa, hb = yb & ~xb; /* holes */
    uint64_t pa = xa & ~ya, pb = xb & ~yb; /* particles */
    int nh = popc64(ha) + popc64(hb), np_ = popc64(pa) + popc64(pb);
    if (nh != np_) return 0.0;
    if (nh == 0) return or_hdiag(M, h, eri, ecore, ya, yb);
    if (nh > 2) return 0.0;
    int hole[2], part[2];
    list_bits(ha, hb, M, hole);
    list_bits(pa, pb, M, part);
    fock_t y = {ya, yb};
    if (nh == 1) {
        int q = hole[0], p = part[0];
        if ((q < M) != (p < M)) return 0.0;
        int sign = (occ_between(y, M, p, q) & 1) ? -1 : 1;
        double v = h[(p % M) * M + (q % M)];
        int occ[128];
        int n = list_bits(ya, yb, M, occ);
        for (int k = 0; k < n; ++k) {
            int r = occ[k];
            if (r == q) continue;
            v += ERI(&H, p % M, q % M, r % M, r % M);
            if ((r < M) == (p < M)) v -= ERI(&H, p % M, r % M, r % M, q % M);
        }
        return sign * v;
    }
    /* double: i -> a then j -> b */
    int i = hole[0], j = hole[1], a = part[0], b = part[1];
    int s1 = (occ_between(y, M, i, a) & 1) ? -1 : 1;
    fock_t y1 = y;
    fock_set(&y1, M, i, 0);
    fock_set(&y1, M, a, 1);
    int s2 = (occ_between(y1, M, j, b) & 1) ? -1 : 1;
    int si = i < M, sj = j < M, sa = a < M, sb = b < M;
    double v = 0.0;
    if (si == sa && sj == sb) v += ERI(&H, a % M, i % M, b % M, j % M);
    if (sj == sa && si == sb) v -= ERI(&H, a % M, j % M, b % M, i % M);
    return s1 * s2 * v;
}

/* excitation rank between two dets of one sector */
static int exc_rank(uint64_t xa, uint64_t xb, uint64_t ya, uint64_t yb) {
    return (popc64(xa ^ ya) + popc64(xb ^ yb)) / 2;
}

/* dense H over a basis by the Slater-Condon rules (for comparison with or_dense_opalg) */
int or_dense_sc(int M, const double *h, const double *eri, double ecore, const uint64_t *basis, int64_t n,
                double *Hout) {
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c)
            Hout[r * n + c] = or_hxy(M, h, eri, ecore, basis[2 * r], basis[2 * r + 1], basis[2 * c],
                                     basis[2 * c + 1]);
    return 0;
}

/*
 * H_SS rows by definition.  For each requested row x = dets[rows[k]], the columns are
 * every y in S (ascending canonical index) with excitation rank 1 or 2 relative to x.
 * Pass 1 (col == NULL): counts[k] = number of such y.  Pass 2: fills col/val at
 * offsets row_ptr[k] and the diagonal diag[k].
 */
int or_csr_rows(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                const int64_t *rows, int64_t n_rows, int64_t *counts, const int64_t *row_ptr, int32_t *col,
                double *val, double *diag) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_rows; ++k) {
        int64_t i = rows[k];
        uint64_t xa = dets[2 * i], xb = dets[2 * i + 1];
        int64_t c = 0, pos = row_ptr ? row_ptr[k] : 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            int r = exc_rank(xa, xb, dets[2 * j], dets[2 * j + 1]);
            if (r < 1 || r > 2) continue;
            if (col) {
                col[pos + c] = (int32_t)j;
                val[pos + c] = or_hxy(M, h, eri, ecore, xa, xb, dets[2 * j], dets[2 * j + 1]);
            }
            ++c;
        }
        if (counts) counts[k] = c;
        if (diag) diag[k] = or_hdiag(M, h, eri, ecore, xa, xb);
    }
    return 0;
}

/* ------------------------------------------------------------------ excitations */
/*
 * All single and double excitations of x within its (N_alpha, N_beta) sector, as a
 * list of dets out[2*k], out[2*k+1].  Written as plain loops over holes and particles:
 * alpha singles, beta singles, alpha-alpha doubles, beta-beta doubles, alpha-beta
 * doubles.  Returns the number written (at most cap), or the full count if out==NULL.
 */
int64_t or_excitations(int M, uint64_t xa, uint64_t xb, uint64_t *out, int64_t cap) {
    int oa[64], va[64], ob[64], vb[64];
    int noa = 0, nva = 0, nob = 0, nvb = 0;
    for (int p = 0; p < M; ++p) {
        if ((xa >> p) & 1u)
            oa[noa++] = p;
        else
            va[nva++] = p;
        if ((xb >> p) & 1u)
            ob[nob++] = p;
        else
            vb[nvb++] = p;
    }
    int64_t k = 0;
#define EMIT(A, B)                  \
    do {                            \
        if (out && k < cap) {       \
            out[2 * k] = (A);       \
            out[2 * k + 1] = (B);   \
        }                           \
        ++k;                        \
    } while (0)
    const uint64_t one = 1;
    for (int i = 0; i < noa; ++i)
        for (int a = 0; a < nva; ++a) EMIT((xa & ~(one << oa[i])) | (one << va[a]), xb);
    for (int i = 0; i < nob; ++i)
        for (int a = 0; a < nvb; ++a) EMIT(xa, (xb & ~(one << ob[i])) | (one << vb[a]));
    for (int i = 0; i < noa; ++i)
        for (int j = i + 1; j < noa; ++j)
            for (int a = 0; a < nva; ++a)
                for (int b = a + 1; b < nva; ++b)
                    EMIT((xa & ~(one << oa[i]) & ~(one << oa[j])) | (one << va[a]) | (one << va[b]), xb);
    for (int i = 0; i < nob; ++i)
        for (int j = i + 1; j < nob; ++j)
            for (int a = 0; a < nvb; ++a)
                for (int b = a + 1; b < nvb; ++b)
                    EMIT(xa, (xb & ~(one << ob[i]) & ~(one << ob[j])) | (one << vb[a]) | (one << vb[b]));
    for (int i = 0; i < noa; ++i)
        for (int a = 0; a < nva; ++a)
            for (int j = 0; j < nob; ++j)
                for (int b = 0; b < nvb; ++b)
                    EMIT((xa & ~(one << oa[i])) | (one << va[a]), (xb & ~(one << ob[j])) | (one << vb[b]));
#undef EMIT
    return k;
}

/* ------------------------------------------------------------------ PT2 */
/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), used only to
 * spread keys over threads and to pick a reproducible sampled subset of keys. */
static uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

/* key hash used for sampled subsets: mix64(alpha ^ mix64(beta)) */
uint64_t or_key_hash(uint64_t a, uint64_t b) { return mix64(a ^ mix64(b)); }

typedef struct {
    uint64_t a, b;
    double w;     /* sum of H_ax psi_x */
    double c;     /* sum of |H_ax psi_x| (bounds the rounding error of w) */
    double mx;    /* largest |H_ax psi_x| (the heat-bath measure of a, Eq. 14) */
    int64_t k;    /* number of contributions */
    int used;
} slot_t;

typedef struct {
    slot_t *s;
    size_t cap, n;
} map_t;

static void map_init(map_t *m, size_t cap) {
    m->cap = 1;
    while (m->cap < cap) m->cap <<= 1;
    m->s = (slot_t *)calloc(m->cap, sizeof(slot_t));
    m->n = 0;
}

static slot_t *map_slot(map_t *m, uint64_t a, uint64_t b);

static void map_grow(map_t *m) {
    map_t g;
    map_init(&g, m->cap * 2);
    for (size_t i = 0; i < m->cap; ++i)
        if (m->s[i].used) *map_slot(&g, m->s[i].a, m->s[i].b) = m->s[i];
    free(m->s);
    *m = g;
}

/* the slot of key (a, b), created empty (w = c = k = 0) if absent */
static slot_t *map_slot(map_t *m, uint64_t a, uint64_t b) {
    if (2 * (m->n + 1) > m->cap) map_grow(m);
    size_t i = (size_t)(or_key_hash(a, b) >> 7) & (m->cap - 1);
    for (;;) {
        slot_t *s = &m->s[i];
        if (!s->used) {
            memset(s, 0, sizeof *s);
            s->used = 1;
            s->a = a;
            s->b = b;
            m->n++;
            return s;
        }
        if (s->a == a && s->b == b) return s;
        i = (i + 1) & (m->cap - 1);
    }
}

static void map_add(map_t *m, uint64_t a, uint64_t b, double w) {
    slot_t *s = map_slot(m, a, b);
    s->w += w;
    s->c += fabs(w);
    if (fabs(w) > s->mx) s->mx = fabs(w);
    s->k += 1;
}

/*
 * External part of Eq. 13, unnormalised: sum over a in P = C(S) \ S of
 * w_a^2 / (E - H_aa), with w_a = sum_{x in S} H_ax psi_x.  Only keys whose
 * or_key_hash has (hash & sample_mask) == sample_val are kept (mask 0 keeps all), and
 * only keys whose largest single coupling max_x |H_ax psi_x| is at least eps_abs (the
 * heat-bath screen of Eq. 14 with the threshold in the scale of psi; 0 keeps all); w_a
 * of a kept key is its whole sum.
 * A term whose numerator is exactly 0 contributes 0.  Statistics out:
 *   stats_i[0] = (x, a) pairs generated, stats_i[1] = kept unique a,
 *   stats_i[2] = terms with |E - H_aa| < 1e-8,
 *   stats_i[3] = sum of or_key_hash(a) over the kept a (mod 2^64),
 *   stats_i[4] = xor of or_key_hash(a) over the kept a
 *     (with stats_i[1], an order-free fingerprint of the kept set);
 *   stats_d[0] = min |E - H_aa|,
 *   stats_d[1] = sum_a |t_a|, t_a = w_a^2 / (E - H_aa),
 *   stats_d[2] = sum_a 2 |w_a| c_a / |E - H_aa|, c_a = sum_x |H_ax psi_x|,
 *   stats_d[3] = sum_a 2 |w_a| k_a / |E - H_aa|, k_a = number of x with a pair to a,
 *   stats_d[4] = sum_a |t_a| (|E| + |H_aa|) / |E - H_aa|
 *     (first-order sensitivities of the sum to relative errors in the terms, to
 *     relative errors in the H_ax psi_x, to an absolute error per H_ax psi_x, and to
 *     relative errors in E and H_aa: error bars for another implementation).
 * Work is split over threads by key hash, so each thread owns a private map.
 */
double or_pt2_external_hb(int M, const double *h, const double *eri, double ecore, const uint64_t *dets,
                          int64_t n, const double *psi, double E, uint64_t sample_mask, uint64_t sample_val,
                          double eps_abs, int64_t *stats_i, double *stats_d) {
    int64_t n_pairs = 0, n_keys = 0, n_tiny = 0;
    uint64_t fp_sum = 0, fp_xor = 0;
    double total = 0.0, min_den = INFINITY, sens[4] = {0.0, 0.0, 0.0, 0.0};
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *part_sum = (double *)calloc((size_t)nthr, sizeof(double));
    double *part_min = (double *)malloc(sizeof(double) * (size_t)nthr);
    double *part_sens = (double *)calloc(4 * (size_t)nthr, sizeof(double));
    int64_t *part_keys = (int64_t *)calloc((size_t)nthr, sizeof(int64_t));
    int64_t *part_tiny = (int64_t *)calloc((size_t)nthr, sizeof(int64_t));
    int64_t *part_pairs = (int64_t *)calloc((size_t)nthr, sizeof(int64_t));
    uint64_t *part_fp = (uint64_t *)calloc(2 * (size_t)nthr, sizeof(uint64_t));
    for (int t = 0; t < nthr; ++t) part_min[t] = INFINITY;
#pragma omp parallel num_threads(nthr)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        map_t m;
        map_init(&m, 1024);
        int64_t cap = or_excitations(M, dets[0], dets[1], NULL, 0);
        uint64_t *ex = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(cap > 0 ? cap : 1));
        for (int64_t i = 0; i < n; ++i) {
            uint64_t xa = dets[2 * i], xb = dets[2 * i + 1];
            int64_t ne = or_excitations(M, xa, xb, ex, cap);
            if (t == 0) part_pairs[0] += ne;
            if (psi[i] == 0.0) continue;
            for (int64_t k = 0; k < ne; ++k) {
                uint64_t aa = ex[2 * k], ab = ex[2 * k + 1];
                uint64_t hk = or_key_hash(aa, ab);
                if ((int)(hk % (uint64_t)nthr) != t) continue;
                if ((hk & sample_mask) != sample_val) continue;
                if (find_det(dets, n, aa, ab) >= 0) continue;
                double hax = or_hxy(M, h, eri, ecore, aa, ab, xa, xb);
                map_add(&m, aa, ab, hax * psi[i]);
            }
        }
        double s = 0.0;
        for (size_t q = 0; q < m.cap; ++q) {
            if (!m.s[q].used) continue;
            if (m.s[q].mx < eps_abs) continue; /* screened out (Eq. 14) */
            part_keys[t]++;
            uint64_t hk = or_key_hash(m.s[q].a, m.s[q].b);
            part_fp[2 * t] += hk;
            part_fp[2 * t + 1] ^= hk;
            double haa = or_hdiag(M, h, eri, ecore, m.s[q].a, m.s[q].b);
            double den = E - haa;
            double ad = fabs(den);
            if (ad < part_min[t]) part_min[t] = ad;
            if (ad < 1e-8) part_tiny[t]++;
            double w = m.s[q].w;
            if (w != 0.0) {
                double term = w * w / den;
                s += term;
                part_sens[4 * t + 0] += fabs(term);
                part_sens[4 * t + 1] += 2.0 * fabs(w) * m.s[q].c / ad;
                part_sens[4 * t + 2] += 2.0 * fabs(w) * (double)m.s[q].k / ad;
                part_sens[4 * t + 3] += fabs(term) * (fabs(E) + fabs(haa)) / ad;
            }
        }
        part_sum[t] = s;
        free(ex);
        free(m.s);
    }
    for (int t = 0; t < nthr; ++t) {
        total += part_sum[t];
        n_keys += part_keys[t];
        n_tiny += part_tiny[t];
        fp_sum += part_fp[2 * t];
        fp_xor ^= part_fp[2 * t + 1];
        for (int k = 0; k < 4; ++k) sens[k] += part_sens[4 * t + k];
        if (part_min[t] < min_den) min_den = part_min[t];
    }
    n_pairs = part_pairs[0];
    if (stats_i) {
        stats_i[0] = n_pairs;
        stats_i[1] = n_keys;
        stats_i[2] = n_tiny;
        stats_i[3] = (int64_t)fp_sum;
        stats_i[4] = (int64_t)fp_xor;
    }
    if (stats_d) {
        stats_d[0] = min_den;
        for (int k = 0; k < 4; ++k) stats_d[1 + k] = sens[k];
    }
    free(part_sum);
    free(part_min);
    free(part_sens);
    free(part_keys);
    free(part_tiny);
    free(part_pairs);
    free(part_fp);
    return total;
}

double or_pt2_external(int M, const double *h, const double *eri, double ecore, const uint64_t *dets,
                       int64_t n, const double *psi, double E, uint64_t sample_mask, uint64_t sample_val,
                       int64_t *stats_i, double *stats_d) {
    return or_pt2_external_hb(M, h, eri, ecore, dets, n, psi, E, sample_mask, sample_val, 0.0, stats_i, stats_d);
}

/*
 * The set P = C(S) \ S of Eq. 1 written out: every determinant a of the sector that
 * is a single or double excitation of some x in S and is not itself in S, each once,
 * in canonical order (ascending alpha, then beta).  With psi given, also
 * w_a = sum_{x in S} H_ax psi_x and H_aa, and with eps_abs > 0 only the a whose
 * largest coupling max_x |H_ax psi_x| reaches eps_abs (the screened set of Eq. 14).  Single-threaded, for small S: returns |P|
 * and writes min(|P|, cap) entries (keys[2k], keys[2k+1]; w and haa may be NULL).
 */
static int cmp_key(const void *x, const void *y) {
    const uint64_t *u = (const uint64_t *)x, *v = (const uint64_t *)y;
    return cmp_det(u[0], u[1], v[0], v[1]);
}

int64_t or_pt2_plist_hb(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                        const double *psi, double eps_abs, uint64_t *keys, double *w_out, double *haa_out,
                        int64_t cap) {
    map_t m;
    map_init(&m, 1024);
    int64_t ecap = or_excitations(M, dets[0], dets[1], NULL, 0);
    uint64_t *ex = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(ecap > 0 ? ecap : 1));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t xa = dets[2 * i], xb = dets[2 * i + 1];
        int64_t ne = or_excitations(M, xa, xb, ex, ecap);
        for (int64_t k = 0; k < ne; ++k) {
            uint64_t aa = ex[2 * k], ab = ex[2 * k + 1];
            if (find_det(dets, n, aa, ab) >= 0) continue;
            double hax = psi ? or_hxy(M, h, eri, ecore, aa, ab, xa, xb) * psi[i] : 0.0;
            map_add(&m, aa, ab, hax);
        }
    }
    free(ex);
    /* (alpha, beta, index into the map) triples of the kept keys, sorted canonically */
    int64_t np_ = 0, j = 0;
    for (size_t q = 0; q < m.cap; ++q)
        if (m.s[q].used && m.s[q].mx >= eps_abs) ++np_;
    uint64_t *list = (uint64_t *)malloc(sizeof(uint64_t) * 3 * (size_t)(np_ > 0 ? np_ : 1));
    for (size_t q = 0; q < m.cap; ++q)
        if (m.s[q].used && m.s[q].mx >= eps_abs) {
            list[3 * j] = m.s[q].a;
            list[3 * j + 1] = m.s[q].b;
            list[3 * j + 2] = (uint64_t)q;
            ++j;
        }
    qsort(list, (size_t)np_, 3 * sizeof(uint64_t), cmp_key);
    for (int64_t k = 0; k < np_ && k < cap; ++k) {
        keys[2 * k] = list[3 * k];
        keys[2 * k + 1] = list[3 * k + 1];
        if (w_out) w_out[k] = m.s[list[3 * k + 2]].w;
        if (haa_out) haa_out[k] = or_hdiag(M, h, eri, ecore, list[3 * k], list[3 * k + 1]);
    }
    free(list);
    free(m.s);
    return np_;
}

int64_t or_pt2_plist(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                     const double *psi, uint64_t *keys, double *w_out, double *haa_out, int64_t cap) {
    return or_pt2_plist_hb(M, h, eri, ecore, dets, n, psi, 0.0, keys, w_out, haa_out, cap);
}

/*
 * w_a = sum_{x in S} H_ax psi_x for each of the given keys a (keys[2k], keys[2k+1]),
 * computed one by one: the excitations of a are enumerated and looked up in S.
 * Also returns H_aa.  psi is indexed like dets.
 */
int or_w_keys(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
              const double *psi, const uint64_t *keys, int64_t n_keys, double *w_out, double *haa_out) {
    if (n_keys <= 0) return 0;
    int64_t cap = or_excitations(M, keys[0], keys[1], NULL, 0);
#pragma omp parallel
    {
        uint64_t *ex = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(cap > 0 ? cap : 1));
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < n_keys; ++k) {
            uint64_t aa = keys[2 * k], ab = keys[2 * k + 1];
            int64_t ne = or_excitations(M, aa, ab, ex, cap);
            double w = 0.0;
            for (int64_t e = 0; e < ne; ++e) {
                int64_t j = find_det(dets, n, ex[2 * e], ex[2 * e + 1]);
                if (j < 0) continue;
                w += or_hxy(M, h, eri, ecore, aa, ab, ex[2 * e], ex[2 * e + 1]) * psi[j];
            }
            w_out[k] = w;
            if (haa_out) haa_out[k] = or_hdiag(M, h, eri, ecore, aa, ab);
        }
        free(ex);
    }
    return 0;
}

/* set the number of OpenMP threads the oracle uses (timing of the oracle on fewer cores) */
void or_set_num_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* number of OpenMP threads the oracle will use */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
