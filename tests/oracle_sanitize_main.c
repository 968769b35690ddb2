/* Drives the FP64 oracle's C part (oracle/sc_oracle.c) on a small sector so that it can be
 * built with AddressSanitizer and UndefinedBehaviorSanitizer on the host: every entry
 * point runs once on M = 8, 3 alpha + 2 beta electrons, with random integrals of the
 * 8-fold symmetry.  Prints OK and a checksum; any memory or UB error aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_dense_opalg(int M, const double *h, const double *eri, double ecore, const uint64_t *basis, int64_t n,
                   double *Hout);
int or_dense_sc(int M, const double *h, const double *eri, double ecore, const uint64_t *basis, int64_t n,
                double *Hout);
double or_hdiag(int M, const double *h, const double *eri, double ecore, uint64_t ya, uint64_t yb);
double or_hxy(int M, const double *h, const double *eri, double ecore, uint64_t xa, uint64_t xb, uint64_t ya,
              uint64_t yb);
int or_csr_rows(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                const int64_t *rows, int64_t n_rows, int64_t *counts, const int64_t *row_ptr, int32_t *col,
                double *val, double *diag);
int64_t or_excitations(int M, uint64_t xa, uint64_t xb, uint64_t *out, int64_t cap);
double or_pt2_external_hb(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                          const double *psi, double E, uint64_t sample_mask, uint64_t sample_val, double eps_abs,
                          int64_t *stats_i, double *stats_d);
int64_t or_pt2_plist_hb(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
                        const double *psi, double eps_abs, uint64_t *keys, double *w_out, double *haa_out,
                        int64_t cap);
int or_w_keys(int M, const double *h, const double *eri, double ecore, const uint64_t *dets, int64_t n,
              const double *psi, const uint64_t *keys, int64_t n_keys, double *w_out, double *haa_out);

static uint64_t lcg = 0x9e3779b97f4a7c15ull;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * 0x1.0p-53 - 0.5;
}

int main(void) {
    enum { M = 8, NA = 3, NB = 2 };
    double h[M * M], *eri = malloc(sizeof(double) * M * M * M * M);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q <= p; ++q) h[p * M + q] = h[q * M + p] = urand() + (p == q ? -2.0 * (M - p) : 0.0);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            for (int r = 0; r < M; ++r)
                for (int s = 0; s < M; ++s) eri[((p * M + q) * M + r) * M + s] = 0.0;
    /* (pq|rs) with the 8-fold symmetry */
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            for (int r = 0; r < M; ++r)
                for (int s = 0; s < M; ++s) {
                    const int a = p > q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
                    const int b = r > s ? r * (r + 1) / 2 + s : s * (s + 1) / 2 + r;
                    if (a < b) continue;
                    const double v = 0.1 * urand() + (p == q && r == s ? 0.3 : 0.0);
                    const int idx[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                                           {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
                    for (int k = 0; k < 8; ++k)
                        eri[((idx[k][0] * M + idx[k][1]) * M + idx[k][2]) * M + idx[k][3]] = v;
                }
    /* the full sector: C(8,3) * C(8,2) = 56 * 28 determinants, ascending (alpha, beta) */
    uint64_t al[64], be[64];
    int na = 0, nb = 0;
    for (uint64_t s = 0; s < (1u << M); ++s) {
        if (__builtin_popcountll(s) == NA) al[na++] = s;
        if (__builtin_popcountll(s) == NB) be[nb++] = s;
    }
    const int64_t n = (int64_t)na * nb;
    uint64_t *dets = malloc(sizeof(uint64_t) * 2 * n);
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            dets[2 * (i * nb + j)] = al[i];
            dets[2 * (i * nb + j) + 1] = be[j];
        }
    double *H1 = malloc(sizeof(double) * n * n), *H2 = malloc(sizeof(double) * n * n);
    if (or_dense_opalg(M, h, eri, 0.5, dets, n, H1) != 0) return 2;
    or_dense_sc(M, h, eri, 0.5, dets, n, H2);
    double dmax = 0.0, chk = 0.0;
    for (int64_t i = 0; i < n * n; ++i) {
        dmax = fmax(dmax, fabs(H1[i] - H2[i]));
        chk += H1[i];
    }
    chk += or_hdiag(M, h, eri, 0.5, dets[0], dets[1]) + or_hxy(M, h, eri, 0.5, dets[0], dets[1], dets[2], dets[3]);
    /* H_SS rows of a subset S (the first 300 determinants) */
    const int64_t ns = 300;
    int64_t rows[300], counts[300], row_ptr[301];
    for (int64_t i = 0; i < ns; ++i) rows[i] = i;
    or_csr_rows(M, h, eri, 0.5, dets, ns, rows, ns, counts, NULL, NULL, NULL, NULL);
    row_ptr[0] = 0;
    for (int64_t i = 0; i < ns; ++i) row_ptr[i + 1] = row_ptr[i] + counts[i];
    int32_t *col = malloc(sizeof(int32_t) * (row_ptr[ns] + 1));
    double *val = malloc(sizeof(double) * (row_ptr[ns] + 1)), diag[300];
    or_csr_rows(M, h, eri, 0.5, dets, ns, rows, ns, NULL, row_ptr, col, val, diag);
    for (int64_t i = 0; i < row_ptr[ns]; ++i) chk += val[i] * 1e-3 + col[i] * 1e-9;
    const int64_t ne = or_excitations(M, dets[0], dets[1], NULL, 0);
    uint64_t *ex = malloc(sizeof(uint64_t) * 2 * ne);
    or_excitations(M, dets[0], dets[1], ex, ne);
    /* PT2 pieces on S with a random psi */
    double psi[300], st_d[5];
    int64_t st_i[5];
    for (int64_t i = 0; i < ns; ++i) psi[i] = urand();
    chk += or_pt2_external_hb(M, h, eri, 0.5, dets, ns, psi, -5.0, 0, 0, 0.0, st_i, st_d);
    chk += or_pt2_external_hb(M, h, eri, 0.5, dets, ns, psi, -5.0, 3, 0, 1e-3, st_i, st_d);
    const int64_t np = or_pt2_plist_hb(M, h, eri, 0.5, dets, ns, psi, 0.0, NULL, NULL, NULL, 0);
    uint64_t *keys = malloc(sizeof(uint64_t) * 2 * (np + 1));
    double *w = malloc(sizeof(double) * (np + 1)), *haa = malloc(sizeof(double) * (np + 1));
    or_pt2_plist_hb(M, h, eri, 0.5, dets, ns, psi, 0.0, keys, w, haa, np);
    double *w2 = malloc(sizeof(double) * (np + 1)), *haa2 = malloc(sizeof(double) * (np + 1));
    or_w_keys(M, h, eri, 0.5, dets, ns, psi, keys, np, w2, haa2);
    double dw = 0.0;
    for (int64_t k = 0; k < np; ++k) dw = fmax(dw, fabs(w[k] - w2[k]) + fabs(haa[k] - haa2[k]));
    printf("OK n=%lld nnz=%lld n_exc=%lld |P|=%lld dense=%.3e w=%.3e checksum=%.6f\n", (long long)n,
           (long long)row_ptr[ns], (long long)ne, (long long)np, dmax, dw, chk);
    free(eri); free(dets); free(H1); free(H2); free(col); free(val); free(ex); free(keys); free(w); free(haa);
    free(w2); free(haa2);
    return (dmax < 1e-10 && dw < 1e-10) ? 0 : 3;
}
