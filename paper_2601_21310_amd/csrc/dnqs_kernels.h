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
size_t packed_eri_size(int M);
void launch_pack_eri(hipStream_t st, int M, const double *eri64, double *pk);
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
// val[j] = <x|H|col[j]> for the entries of every row x
void launch_hss_values(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const int64_t *row_ptr,
                       const int32_t *col, float *val);
int64_t scan_blocks(int64_t n);
void launch_exclusive_scan(hipStream_t st, const int32_t *in, int64_t n, int64_t *out, int64_t *bsum,
                           int64_t *total);

// ---------------------------------------------------------------- sort (k_sort.hip)
// Workspace of a radix sort of n keys: keys, vals [n]; counts, offs [sort_scratch_counts(n)];
// bsum [scan_blocks(sort_scratch_counts(n)) + 1]; total [1].
struct SortScratch {
    uint64_t *keys;
    int32_t *vals;
    int32_t *counts;
    int64_t *offs;
    int64_t *bsum;
    int64_t *total;
};
size_t sort_scratch_counts(int64_t n);
// stable ascending sort of keys[0..n) on their low `bits` bits, vals moved along
void launch_radix_sort(hipStream_t st, uint64_t *keys, int32_t *vals, int64_t n, int bits, const SortScratch &w);
void launch_iota_i32(hipStream_t st, int32_t *v, int64_t n);
void launch_gather_u64(hipStream_t st, const uint64_t *src, const int32_t *perm, int64_t n, uint64_t *dst);
// dst[i] = src[perm[i]], records of `words` 64-bit words
void launch_permute_words(hipStream_t st, const uint64_t *src, const int32_t *perm, int64_t n, int words,
                          uint64_t *dst);
// perm = the canonical order of dets[0..n) (key: n words of scratch)
void launch_sort_dets(hipStream_t st, const uint64_t *dets, int64_t n, int M, int32_t *perm, uint64_t *key,
                      const SortScratch &w);

// ---------------------------------------------------------------- P = C(S) \ S (k_pset.hip)
// psi (scaled, nullable) with hb_eps > 0: heat-bath screen against hb_eps sqrt(norm2[0])
void launch_pc_pass(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const DetSet &S,
                    const double *psi, double hb_eps, const double *norm2, int32_t *cnt, const int64_t *off,
                    uint64_t *ka, uint64_t *kb, bool fill);
// key[i]: descending log|psi| of determinant perm[i] (sign 0 last), for a radix sort
void launch_topk_key(hipStream_t st, const double *la, const int8_t *sg, const int32_t *perm, int64_t n,
                     uint64_t *key);
void launch_unique(hipStream_t st, const uint64_t *ka, const uint64_t *kb, const int32_t *perm, int64_t m, bool two,
                   int M, int32_t *flag, int64_t *pos, int64_t *bsum, int64_t *total, uint64_t *p_dets, bool write);
void launch_fingerprint(hipStream_t st, const uint64_t *p, int64_t m, unsigned long long *fp);
void launch_hps_pass(hipStream_t st, const Ham &H, const uint64_t *pd, int64_t m, const DetSet &S, int32_t *cnt,
                     const int64_t *off, int32_t *col, float *val, bool fill);
void launch_rows_finish(hipStream_t st, const int64_t *off, int64_t m, const int64_t *total, int64_t *row_ptr,
                        int32_t *col, float *val);
void launch_row_ptr_from_offsets(hipStream_t st, const int64_t *off, int64_t m, const int64_t *total,
                                 int64_t *row_ptr);

// ---------------------------------------------------------------- Lanczos (k_lanczos.hip)
int lanczos_dot_blocks();
int lanczos_norm_blocks(int64_t n);
// c[0..m) (+)= V[k] . w for the m vectors V[k] = V + k ldv; part: m * lanczos_dot_blocks()
void launch_lz_dots(hipStream_t st, const double *V, int64_t ldv, int m, const double *w, int64_t n, double *part,
                    double *c, bool accumulate);
// w -= sum_k c[k] V[k]; nrm[0] = |w| (part: lanczos_norm_blocks(n))
void launch_lz_orth(hipStream_t st, const double *V, int64_t ldv, int m, const double *c, double *w, int64_t n,
                    double *part, double *nrm);
void launch_lz_norm(hipStream_t st, const double *w, int64_t n, double *part, double *nrm);
void launch_lz_scale(hipStream_t st, const double *src, int64_t n, const double *nrm, double *dst);
void launch_lz_combine(hipStream_t st, const double *V, int64_t ldv, int m, const double *y, int64_t n,
                       double *out);
void launch_lz_start(hipStream_t st, const double *diag, int64_t n, double *tmp1, double *v);

// ---------------------------------------------------------------- network
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

// C[M x N] (+ split index * c_split_stride) = epi(A[M x K] * B[K x N])
//   A: a_kcontig ? A[m*lda + k] : A[k*lda + m]     (rows m >= ones_row >= 0 read as 1)
//   B: b_ncontig ? B[k*ldb + n] : B[n*ldb + k]
// Element types are fixed by the kernel that takes the struct; the pointers are untyped.
struct GemmArgs {
    int M, N, K;
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
    const float *bias;
    const void *act;
    int64_t ldact;
    int ones_row;
    int k_chunk;
    int64_t c_split_stride;
    // grouped launches over several problems (batched geometries), all optional:
    const int *tile_pid;        // problem of each 128-row tile: B = Bg[pid], bias = biasg[pid]
    const void *const *Bg;
    const float *const *biasg;
    const int2 *ksplit;         // k range [x, y) of each blockIdx.z (split-K over problems)
    // split-BF16 engine only, optional: B given as BF16 hi / lo planes, both [n][k]
    // (k-contiguous, leading dimension ldbs); the lo plane starts bs_plane elements
    // after the hi plane.  Used for weights, split once per call.
    const void *bsplit;
    int64_t ldbs, bs_plane;
};

// One problem of a batched launch (rows off .. off+n-1 of the concatenated layout;
// rows from off+n to the next problem's off are padding and contribute nothing).
struct ProbDev {
    const float *theta;
    float *grad;
    double *energy;
    double *stats;
    int64_t off, n;
};

// Optional per-row problem lookup: with pid != nullptr, row x belongs to problem
// pid[x] and its parameters are P[pid[x]].theta + the given offsets.
struct RowProblems {
    const int32_t *pid;
    const ProbDev *P;
};

void launch_embed(hipStream_t st, const uint64_t *dets, int64_t n, int M, int d1, const float *W1, const float *b1,
                  float *h1, float *U, RowProblems rp = {}, int64_t offW1 = 0, int64_t offb1 = 0);
// C = epi(A B): FP32 MFMA, or split-BF16 MFMA (three BF16 products per operand pair);
// same arguments and layouts for both.  Tiles of tm (128 or 64) x 128; split-K over
// `splits` chunks of K (or the ksplit table) into C + z * c_split_stride.
void launch_gemm_f32(hipStream_t st, const GemmArgs &g, bool a_kcontig, bool b_ncontig, int epi, int splits,
                     int tm = 128);
void launch_gemm_x3(hipStream_t st, const GemmArgs &g, bool a_kcontig, bool b_ncontig, int epi, int splits,
                    int tm = 128);
// hi = bf16(W), lo = bf16(W - hi) of a row-major R x C FP32 matrix, written as planes
// [C][R] (transpose) or [R][C]; lo = hi + R * C
void launch_split_planes(hipStream_t st, const float *W, int R, int C, bool transpose, void *planes);
void launch_reduce_splits(hipStream_t st, const float *part, int splits, int64_t count, float *out);
void launch_fold_splits(hipStream_t st, const float *part, int splits, int64_t count, float *out, bool accumulate);
int orb_lu_group(int ne);
// Output layer in the occupied-row form (k_outsplit.hip): the dense orbitals' column
// blocks in OD (ldd = nd * Ne per configuration, orbital p at dpos[p] * Ne), every other
// occupied row j of A(x) as entry e = idx[x * Ne + j] with its Ne values at Osp[e * Ne].
// In the backward, dOD / dOsp take the same layout (dorb lists the dense orbitals), and
// the full-width dO is written as well when given (the data gradient uses it).
struct OutSplit {
    const float *OD = nullptr;
    const float *Osp = nullptr;
    float *dOD = nullptr;
    float *dOsp = nullptr;
    const int *dpos = nullptr;
    const int *dorb = nullptr;
    const int32_t *idx = nullptr;
    int nd = 0;
};
void launch_orb_lu(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const float *O,
                   const float *Phi0, double *logabs, int8_t *sign, float *Ainv, RowProblems rp = {},
                   int64_t offPhi0 = 0, OutSplit os = {});
void launch_det_bwd(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int nb, const double *psi,
                    const double *v, const double *energy, const double *stats, const float *Ainv, float *dO,
                    RowProblems rp = {}, OutSplit os = {});
// occupied-row output layer (k_outsplit.hip)
void launch_os_count(hipStream_t st, const uint64_t *dets, int64_t n, int M, unsigned long long *cnt);
int64_t os_blocks(int64_t n);
void launch_os_build(hipStream_t st, const uint64_t *dets, int64_t n, int M, int na, int Ne, const int *dpos,
                     const int64_t *eoff, int *bcnt, int64_t *boff, int32_t *ex, int32_t *ej, int32_t *idx);
void launch_os_gather_w(hipStream_t st, const float *W, const float *bias, int din, int width, int Ne, int nd,
                        const int *dorb, float *WD);
int os_tile();
void launch_os_trans_w(hipStream_t st, const float *W, int din, int width, float *WT);
// data gradient of the output layer's sparse rows (Cr: entries x din scratch), added to
// the dense part dD (may be null) per configuration, times (1 - hL^2), into delta
void launch_os_dgrad(hipStream_t st, int64_t n, int Ne, int din, const float *WT, const int4 *tiles, int64_t ntiles,
                     const float *dOsp, float *Cr, const float *dD, const int32_t *idx, const float *hL,
                     float *delta);
bool os_fwd_fits(int din, int Ne);  // the occupied-row forward fits LDS for this layer
int os_item();  // entries per weight-gradient work item (at most)
void launch_os_fwd(hipStream_t st, const float *hL, int din, const float *W, const float *bias, int width, int Ne,
                   const int4 *tiles, int64_t ntiles, const int32_t *ex, float *Osp);
void launch_os_wgrad(hipStream_t st, const float *hL, int din, int Ne, const int4 *items, int64_t nitems,
                     const int32_t *ex, const float *dOsp, float *part, const int *dpos, const int *ifirst,
                     const int *icount, int No, float *grad);
void launch_os_scatter(hipStream_t st, const float *GD, int din, int Ne, int nd, int width, const int *dorb,
                       float *grad);
void launch_copy_f32(hipStream_t st, const float *x, float *y, int64_t n);

// ---------------------------------------------------------------- batched problems, optimiser
struct AdamCfg {
    float lr_max, lr_min;
    int decay_steps;
    float beta1, beta2, eps, weight_decay;
};
void launch_adamw(hipStream_t st, float *theta, const float *grad, float *m, float *v, int64_t n, const AdamCfg &c,
                  int *step);
void launch_cat_problem(hipStream_t st, int g, int64_t off, int64_t n, int64_t end, const uint64_t *dets,
                        const int64_t *row_ptr, const int32_t *col, const float *val, const double *diag, int64_t nnz,
                        int64_t nnz_off, uint64_t *dets_cat, int32_t *pid, int64_t *row_ptr_cat, int32_t *col_cat,
                        float *val_cat, double *diag_cat);
void launch_set_i64(hipStream_t st, int64_t *p, int64_t v);
// per problem: l_max, psi, v = H psi and E, the per-problem reductions one workgroup per
// (problem, row chunk) item, items largest problem first
void launch_energy_grouped(hipStream_t st, const double *la, const int8_t *sg, int64_t ntot, int G, RowProblems rp,
                           const int64_t *row_ptr, const int32_t *col, const float *val, const double *diag,
                           double *psi, double *v, double *pv, double *pp, const int4 *items, int nitems,
                           double *ipart);
void launch_reduce_splits_grouped(hipStream_t st, const float *part, const int2 *zrange, int64_t cnt, int G,
                                  const ProbDev *P, int64_t off);
void launch_copy_grouped(hipStream_t st, const ProbDev *P, int G, int64_t src, int64_t dst, int64_t cnt);
void launch_adamw_grouped(hipStream_t st, const ProbDev *P, int G, float *m, float *v, int64_t np, const AdamCfg &c,
                          int *step);

// ---------------------------------------------------------------- energy
int reduce_blocks(int64_t n);
void launch_scale_psi(hipStream_t st, const double *la, const int8_t *sg, int64_t n, double *part, double *lmax_out,
                      double *psi);
int64_t spmv_blocks(int64_t n);
void launch_spmv_energy(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *diag, const double *psi, int64_t n, double *v, double *part_pv,
                        double *part_pp, double *stats, double *energy);
void launch_set_f64(hipStream_t st, double *p, double v);
// stats[0] = sum of part_pp, stats[2] = sum of part_pv (fixed order), energy = ratio
void launch_energy_final(hipStream_t st, const double *part_pv, const double *part_pp, int64_t nb, double *stats,
                         double *energy);

// ---------------------------------------------------------------- target-set modes (k_modes.hip)
void launch_count_in_set(hipStream_t st, const uint64_t *p, int64_t m, const DetSet &S, int *count);
// transpose of an m-row CSR with ncols columns: pass 1 (fill = false) counts into cnt and
// scans into off / total; pass 2 (cnt zeroed) scatters and sorts each row by column
void launch_csr_transpose(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val, int64_t m,
                          int64_t ncols, int32_t *cnt, int64_t *off, int64_t *bsum, int64_t *total,
                          int64_t *t_row_ptr, int32_t *t_col, float *t_val, bool fill);
// proxy matrix over T = [V; P] from H_VV, H_VP, H_PV: pass 1 row lengths and offsets,
// pass 2 the entries
void launch_target_assemble(hipStream_t st, const int64_t *vv, const int32_t *vvc, const float *vvv,
                            const int64_t *vp, const int32_t *vpc, const float *vpv, const int64_t *pv,
                            const int32_t *pvc, const float *pvv, int64_t nv, int64_t np, int32_t *len,
                            int64_t *off, int64_t *bsum, int64_t *total, int32_t *col, float *val, bool fill);
int64_t asym_blocks(int64_t n);
// Asymmetric objective (Eq. 6) on the proxy matrix over T: E, stats (psi_V^T psi_V,
// psi_V^T H_VT psi_T) and the adjoint's vector v (exact gradient, or Eq. 7's estimator)
void launch_energy_asym(hipStream_t st, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *diag, const double *psi, int64_t n, int64_t nv, double *u, double *up,
                        double *part_pv, double *part_pp, double *stats, double *energy, int estimator, double *v);
void launch_copy_f64(hipStream_t st, const double *a, double *b, int64_t n);

// ---------------------------------------------------------------- PT2
struct PT2Export {
    int64_t cap;
    uint64_t *keys;
    double *w;
    double *haa;
    int64_t *count;
};
// one L2 chunk: desc1[start, start+len) in L1 bucket b1, whose chunks are cb0..cb0+nc-1
struct PT2Chunk {
    int64_t start, len, cb0, nc;
};

int64_t pt2_l1_groups(int64_t n);
int pt2_red_tab();
// the largest key count (members of S included) of the sub-buckets 0, stride, 2 stride, ...
// (stride = nsb / nsample), counted up to just past the reduce's fill limit
void launch_pt2_keycount(hipStream_t st, const uint64_t *rec, const uint64_t *desc, const int64_t *sb, int64_t nsb,
                         int64_t nsample, const uint64_t *skeys, const int64_t *soffs, int64_t n_s, int *maxkeys,
                         bool packed);
int pt2_red_fill_max();
int pt2_red_part();
int pt2_max_k1();
int pt2_max_k2();
// ss > 0: key-space slice `slice` of 2^ss (targets with those top hash bits only).
// Fill with cur1 != nullptr: no counts needed; bucket b's descriptors go to the region
// [b cap1, (b + 1) cap1) of desc, appended at the cursor cur1[b] (zeroed by the caller),
// and a region that would overflow sets *ovf (its excess is not written)
void launch_pt2_l1(hipStream_t st, const Ham &H, const uint64_t *dets, int64_t n, const double *psi, int s1,
                   int64_t nwg, uint32_t *counts, const int64_t *offs, uint64_t *desc, bool fill, bool packed, int ss,
                   uint32_t slice, uint64_t *cur1 = nullptr, int64_t cap1 = 0, int *ovf = nullptr);
void launch_transpose_u32(hipStream_t st, const uint32_t *in, int64_t R, int64_t C, int32_t *out);
void launch_gather_starts(hipStream_t st, const int64_t *offs, int K, int64_t stride, const int64_t *total,
                          int64_t *starts);
void launch_pt2_l2(hipStream_t st, const uint64_t *desc1, const PT2Chunk *chunks, int64_t nchunk, int s2,
                   uint32_t *counts, const int64_t *offs, uint64_t *desc2, bool fill);
int pt2_max_dets();
void launch_l2_transpose(hipStream_t st, const uint32_t *counts, const PT2Chunk *chunks, int64_t nchunk, int K2,
                         int32_t *out);
void launch_sub_starts(hipStream_t st, const int64_t *offs2, const int64_t *bstart, const int64_t *bcb0,
                       const int64_t *bnc, int K1, int K2, int64_t *sb);
int pt2_diag_table_size(int M);
void launch_diag_table(hipStream_t st, const Ham &H, double *vt);
// The members of S in key-space slice `slice` grouped by the reduce sub-bucket of their
// keys (sbits hash bits after the ss slice bits): count into cnt (fill == false), or
// place into skeys at offs[sub] + cursor (cnt used as cursors)
void launch_s_sub(hipStream_t st, const uint64_t *dets, int64_t n, int sbits, bool packed, int32_t *cnt,
                  const int64_t *offs, uint64_t *skeys, int32_t *sidx, bool fill, int ss, uint32_t slice);
// rec: the source records of launch_pt2_records (same packed flag); wexp: 2^wexp bounds
// |H_ax psi_x| (psi scaled to max |psi| = 1); part: kRedPart doubles per sub-bucket;
// int_term[x]: the internal term of each member x of S in the processed slice;
// hb_eps > 0: only keys with some |H_ax psi_x| >= hb_eps sqrt(norm2[0]) enter the external sum
void launch_pt2_reduce(hipStream_t st, const Ham &H, const uint64_t *rec, const uint64_t *desc,
                       const int64_t *sb, int64_t nsb, const uint64_t *skeys, const int32_t *sidx,
                       const int64_t *soffs, int64_t n_s, const double *vt, const double *energy,
                       uint64_t sample_mask, int wexp, double hb_eps, const double *norm2, const PT2Export &ex,
                       double *part, double *int_term, int *overflow, bool packed);
// acc (8 doubles) += the partial records part[8 nb] (sum, min, |P|, tiny, fingerprint sum and
// XOR), in a fixed order; scratch (if not null) holds pt2_accumulate_scratch() doubles
// for a two-level sum
void launch_pt2_accumulate(hipStream_t st, const double *part, int64_t nb, double *acc, double *scratch = nullptr);
int pt2_accumulate_scratch();
// acc_int (8 doubles) = fixed-order sum of term[0..n) with min |E - diag| and tiny count;
// part holds 8 * 2048 doubles
void launch_pt2_internal(hipStream_t st, const double *term, const double *diag, int64_t n, const double *energy,
                         double *part, double *acc_int);
void launch_pt2_init_acc(hipStream_t st, double *acc);
// acc += part (8-double records): a finished key-space slice into the external total
void launch_pt2_merge(hipStream_t st, double *acc, const double *part);
// per determinant of S: {alpha | beta << 32, psi bits} when packed (M <= 32), else
// {alpha, beta, psi bits, 0}; rec holds 4 n words
void launch_pt2_records(hipStream_t st, const uint64_t *dets, const double *psi, int64_t n, bool packed,
                        uint64_t *rec);
void launch_pt2_final(hipStream_t st, const double *acc_int, const double *acc_ext, const double *stats,
                      double *out, int64_t *counts, int64_t pairs, int64_t passes);

}  // namespace dnqs
