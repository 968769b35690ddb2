// Launch functions of the library's kernels (host side), and the small structs the
// kernels take by value.  Internal to the library; the public ABI is include/dnqs.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dnqs {

struct Ham;
struct DetSet;

// ---------------------------------------------------------------- Hamiltonian side
void launch_stage_integrals(hipStream_t st, int M, const double *eri64, float *eri32, double *J, double *K);
void launch_validate_dets(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, int check_order,
                          int *err);
void launch_fill_u64(hipStream_t st, uint64_t *p, size_t n, uint64_t v);
void launch_detset_insert(hipStream_t st, const uint64_t *dets, int64_t n, uint64_t *keys, int32_t *idx,
                          uint64_t mask);
void launch_diag(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, double *diag);
int hss_nsub(int64_t n);
void launch_hss_count(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, int nsub, int32_t *counts);
void launch_hss_fill(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, int nsub, const int64_t *offs,
                     int32_t *col, float *val);
void launch_row_ptr(hipStream_t st, const int64_t *offs, int64_t n, int nsub, int64_t total, int64_t *row_ptr);
int64_t scan_blocks(int64_t n);
void launch_exclusive_scan(hipStream_t st, const int32_t *in, int64_t n, int64_t *out, int64_t *bsum,
                           int64_t *total);

// ---------------------------------------------------------------- network
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

// C[M x N] (+ split index * c_split_stride) = epi(A[M x K] * B[K x N])
//   A: a_kcontig ? A[m*lda + k] : A[k*lda + m]     (rows m >= ones_row >= 0 read as 1)
//   B: b_ncontig ? B[k*ldb + n] : B[n*ldb + k]
struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    const float *bias;
    const float *act;
    int64_t ldact;
    int ones_row;
    int k_chunk;
    int64_t c_split_stride;
};

void launch_embed(hipStream_t st, const uint64_t *dets, int64_t n, int M, int d1, const float *W1, const float *b1,
                  float *h1, float *U);
void launch_gemm_f32(hipStream_t st, const GemmArgs &g, bool a_kcontig, bool b_ncontig, int epi, int splits);
void launch_reduce_splits(hipStream_t st, const float *part, int splits, int64_t count, float *out);
int orb_lu_group(int ne);
void launch_orb_lu(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const float *O,
                   const float *Phi0, double *logabs, int8_t *sign, float *Ainv);
void launch_det_bwd(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const double *psi,
                    const double *v, const double *energy, const double *stats, const float *Ainv, float *dO);
void launch_copy_f32(hipStream_t st, const float *x, float *y, int64_t n);

// ---------------------------------------------------------------- energy
int reduce_blocks(int64_t n);
void launch_scale_psi(hipStream_t st, const double *la, const int8_t *sg, int64_t n, double *part, double *lmax_out,
                      double *psi);
int64_t spmv_blocks(int64_t n);
void launch_spmv_energy(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *diag, const double *psi, int64_t n, double *v, double *part_pv,
                        double *part_pp, double *stats, double *energy);
void launch_set_f64(hipStream_t st, double *p, double v);
void launch_copy_f64(hipStream_t st, const double *a, double *b, int64_t n);

// ---------------------------------------------------------------- PT2
struct Slot16 {
    unsigned long long key;
    double w;
};
struct Slot32 {
    unsigned long long ka, kb;
    double w, pad;
};
struct PT2Table {
    void *slots;
    uint64_t mask;  // capacity - 1
    unsigned long long *n_unique;
    int *overflow;
};
struct PT2Export {
    int64_t cap;
    uint64_t *keys;
    double *w;
    double *haa;
    int64_t *count;
};

void launch_pt2_gen(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const double *psi, int npass,
                    int pass, const PT2Table &T, bool packed);
void launch_pt2_clear(hipStream_t st, const PT2Table &T, bool packed);
int pt2_fin_blocks(uint64_t cap);
void launch_pt2_finalize(hipStream_t st, const Ham &H, const PT2Table &T, bool packed, const DetSet &S,
                         const double *energy, uint64_t sample_mask, const PT2Export &ex, double *part, double *acc);
void launch_pt2_internal(hipStream_t st, const double *psi, const double *v, const double *diag, int64_t n,
                         const double *energy, double *part, double *acc_int);
void launch_pt2_init_acc(hipStream_t st, double *acc);
void launch_pt2_final(hipStream_t st, const double *acc_int, const double *acc_ext, const double *stats,
                      double *out, int64_t *counts, int64_t pairs, int64_t passes);

}  // namespace dnqs
