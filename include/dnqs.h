/*
 * dnqs.h -- C ABI of the MI355X (gfx950) hot path of the deterministic neural-network
 * quantum-state method for quantum chemistry (arXiv 2601.21310):
 *
 *   Slater-Condon matrix elements between bit-string determinants -> H_SS (CSR)
 *   neural backflow amplitude psi(x) = det A(x)                       (Eqs. 2-4)
 *   variational energy E = psi^T H_SS psi / psi^T psi and its gradient (Eqs. 11-12)
 *   Epstein-Nesbet PT2 correction over the connected set             (Eq. 13)
 *
 * Conventions
 *   Determinant: two uint64 words {alpha, beta}; bit p = spatial orbital p; M <= 64.
 *   Spin-orbital index: alpha p -> p, beta p -> M + p.  |x> = a+_{i1}...a+_{iN}|0>
 *   with i1 < ... < iN; a_k and a+_k carry (-1)^(occupied spin-orbitals below k).
 *   Determinant arrays are uint64[n][2], sorted ascending on (alpha, beta) as unsigned
 *   integers ("canonical order") and free of duplicates.
 *   Integrals: h[p*M+q] and eri[((p*M+q)*M+r)*M+s] = (pq|rs) (chemists' notation),
 *   real, with 8-fold symmetry; FP64 host arrays.
 *   Network: widths w[0] = 2M (occupation bits, spin-orbital order), w[1..L-1]
 *   hidden (tanh), w[L] = 2M * N_e (linear).  DeltaPhi[p][k] = o[p*N_e + k].
 *   theta (FP32, device) packs [W1 b1 W2 b2 ... WL bL Phi0]; W_l is row-major
 *   w[l-1] x w[l]; Phi0 is row-major 2M x N_e.  Gradients use the same packing.
 *
 * Pointers
 *   "dev" = device memory of the context's device, "host" = host memory.  The caller
 *   owns every pointer it passes; the library never frees them and never keeps them
 *   past the call, except where a call says otherwise.  The library owns the context
 *   and connection objects; the device memory behind them comes from the caller's
 *   allocator given to dnqs_create (or from hipMalloc when none is given).
 *
 * Streams and synchronisation
 *   Work is enqueued on the context's stream (dnqs_create / dnqs_set_stream).
 *   dnqs_amplitudes and dnqs_energy_and_grad enqueue and return without waiting;
 *   results that feed later calls (E, norms) stay in device memory.
 *   dnqs_set_integrals, dnqs_build_connections and dnqs_pt2 synchronise the stream
 *   (they size buffers from results computed on the device).
 *
 * Errors
 *   Every call returns a dnqs_status.  Arguments are validated on the host before
 *   any launch; on a non-zero status nothing was enqueued by that call unless the
 *   status is DNQS_EHIP or DNQS_EDOMAIN (the latter found from device results by the
 *   synchronising calls dnqs_lanczos and dnqs_pt2).  dnqs_last_error() gives a message for the last failure on
 *   a context.  No C++ exception crosses this boundary.
 */
#ifndef DNQS_H
#define DNQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dnqs_ctx dnqs_ctx;   /* device, stream, integral slots, workspaces */
typedef struct dnqs_conn dnqs_conn; /* a variational set S with its H_SS */

typedef enum {
    DNQS_OK = 0,
    DNQS_EINVAL = -1,    /* bad argument (size, pointer, sector, ordering) */
    DNQS_ENOMEM = -2,    /* device allocation failed */
    DNQS_EHIP = -3,      /* a HIP runtime call failed */
    DNQS_ECAPACITY = -4, /* a fixed-capacity structure would overflow */
    DNQS_ESTATE = -5,    /* call out of order (e.g. no integrals in the slot) */
    DNQS_EDOMAIN = -6    /* numerical domain error: psi^T psi or a start vector's norm is 0 or not finite */
} dnqs_status;

/* Arithmetic of the network GEMMs.  Activations, weights and gradients are FP32 in
 * memory in every form; the embedding, the LU and the orbital projection are FP32 and
 * every reduction (log|det|, psi^T psi, psi^T H psi, PT2) is FP64.
 * "Split BF16": each FP32 operand x is held as x_hi = bf16(x) plus x_lo = bf16(x - x_hi)
 * and a product is a_lo b_hi + a_hi b_lo + a_hi b_hi on BF16 MFMA with FP32
 * accumulation (relative error near 2^-17 per product instead of 2^-9 for one BF16
 * product). */
typedef enum {
    DNQS_FP32 = 0,      /* every network GEMM on FP32 MFMA */
    DNQS_MIXED = 1,     /* hidden-layer GEMMs in split BF16; orbital output layer on FP32 MFMA */
    DNQS_SPLIT_BF16 = 2 /* every network GEMM, the orbital output layer included, in split BF16 */
} dnqs_precision;

#define DNQS_MAX_LAYERS 8
#define DNQS_MAX_SLOTS 128

/* Network shape: n_layers linear maps, width[0..n_layers]. */
typedef struct {
    int n_layers;
    int width[DNQS_MAX_LAYERS + 1];
} dnqs_net;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`, enqueuing on `stream` (a hipStream_t;
 * NULL = the null stream).  *out receives the context.
 * Device memory: every buffer the library holds (staged integrals, connection objects,
 * workspaces) is obtained from alloc(bytes, user) and returned through release(p, user)
 * when both are given (e.g. a framework's caching allocator, which then stays the only
 * owner of device memory; the memory must be usable on `stream` and on a second stream
 * of the same device that the context creates, and is returned only after the work
 * queued on both has finished); alloc returns NULL on failure (the call then fails with
 * DNQS_ENOMEM; there is no fallback).  With both NULL the library uses hipMalloc /
 * hipFree.  The callbacks are called from the thread that makes the library call, only
 * outside dnqs_capture_begin / dnqs_capture_end, and must outlive the context and every
 * connection object made with it. */
dnqs_status dnqs_create(dnqs_ctx **out, int device, void *stream, void *(*alloc)(size_t bytes, void *user),
                        void (*release)(void *p, void *user), void *user);
void dnqs_destroy(dnqs_ctx *ctx);
dnqs_status dnqs_set_stream(dnqs_ctx *ctx, void *stream);
/* Message for the last failure on ctx (static storage owned by ctx); "" if none.
 * With ctx == NULL, the message of the last dnqs_create failure. */
const char *dnqs_last_error(const dnqs_ctx *ctx);

/* Number of FP32 entries of theta (and of the gradient) for a network on a system
 * with M spatial orbitals and n_alpha + n_beta electrons; -1 if the shape is invalid. */
int64_t dnqs_param_count(const dnqs_net *net, int M, int n_alpha, int n_beta);

/* ------------------------------------------------------------------ integrals
 * Stage the Hamiltonian of one geometry into `slot` (0 <= slot < DNQS_MAX_SLOTS):
 * the one- and two-electron integrals the paper reads from an FCIDUMP (Algorithm 1
 * input; Sec. 3.3).  h: host FP64 [M*M]; eri: host FP64 [M^4]; e_core adds to every
 * diagonal element.  1 <= M <= 64, 0 <= n_alpha, n_beta <= M, n_alpha+n_beta >= 1.
 * The library keeps device copies (FP64 and FP32 tables); the host arrays may be
 * freed after the call.  Synchronises the stream. */
dnqs_status dnqs_set_integrals(dnqs_ctx *ctx, int slot, int M, int n_alpha, int n_beta, const double *h,
                               const double *eri, double e_core);

/* ------------------------------------------------------------------ connections
 * Build H_SS for the variational set S = dets (dev uint64[n][2], canonical order,
 * unique, every det in the slot's (n_alpha, n_beta) sector), using the integrals of
 * `slot`.  H_SS[x][y] = <x|H|y> by the Slater-Condon rules; the off-diagonal pattern
 * is every pair of S at excitation rank 1 or 2 (the connected set of Eq. 1 read as
 * excitation rank <= 2, restricted to S).  The result keeps:
 *   row_ptr int64[n+1], col int32[nnz] (ascending within each row), val FP32[nnz]
 *   (off-diagonal only), diag FP64[n], and a copy of S.
 * flags: DNQS_VALIDATE checks ordering, uniqueness and sector on the device first
 * (DNQS_EINVAL on failure).  DNQS_EMIT_P also lists the rest of the connected set,
 * P = C(S) \ S (Eq. 1; Sec. 2.1's perturbative space), sorted in canonical order and
 * unique, with its diagonal H_aa (FP64) and an order-free fingerprint of P:
 * {sum over a in P of h(a) mod 2^64, XOR over a in P of h(a)} with the key hash
 * h(a) = mix(alpha ^ mix(beta)), mix the SplitMix64 output function (the same
 * fingerprint dnqs_pt2 reports for any size).  DNQS_EMIT_HPS (implies EMIT_P) also
 * keeps H_PS: row a of P holds <a|H|x> for the x in S at excitation rank 1 or 2 from
 * a, CSR with int64 row pointers, int32 columns ascending, FP32 values (the couplings
 * Sec. 2.3's proxy objective and Eq. 13 use).  Listing P holds every pair (x, a) once:
 * DNQS_ECAPACITY if |S| n_exc >= 2^31.  *out receives a new object owned by the caller
 * through dnqs_conn_free.  1 <= n < 2^31.  Synchronises the stream. */
#define DNQS_VALIDATE 1u
#define DNQS_EMIT_P 2u
#define DNQS_EMIT_HPS 4u
dnqs_status dnqs_build_connections(dnqs_ctx *ctx, int slot, const uint64_t *dets, int64_t n, unsigned flags,
                                   dnqs_conn **out);
/* Target set T = [V; P] of the target-space objectives (Sec. 2.3): V = the determinants of
 * cv (an ordinary set from dnqs_build_connections), P = p_dets (dev uint64[n_p][2],
 * canonical order, unique, none in V; DNQS_VALIDATE checks the order, the sector and
 * that no member of P is in V; e.g. the screened set of dnqs_heatbath_candidates).  The
 * result is a connection object over T, rows and amplitudes in the order V then P, whose
 * matrix is the proxy Hamiltonian of Eq. 8: H_VV, H_VP and H_PV exact (Slater-Condon,
 * FP32 values), the P-P block reduced to its FP64 diagonal.  dnqs_energy_and_grad on it
 * evaluates the Proxy objective (Eqs. 9-10) or, with DNQS_ASYM / DNQS_ASYM_ESTIMATOR, the
 * Asymmetric one (Eqs. 6-7).  The exact Rayleigh quotient over T that removes the proxy's
 * bias after optimisation (Sec. 2.4) is dnqs_build_connections on T in canonical order
 * (e.g. from dnqs_select_topk with K = |T|).  1 <= |V| + n_p < 2^31.  Synchronises the
 * stream. */
dnqs_status dnqs_build_target(dnqs_ctx *ctx, int slot, const dnqs_conn *cv, const uint64_t *p_dets, int64_t n_p,
                              unsigned flags, dnqs_conn **out);
/* n_dets, nnz (off-diagonal) of a connection object (host outputs, either may be NULL). */
dnqs_status dnqs_conn_info(const dnqs_conn *conn, int64_t *n_dets, int64_t *nnz);
/* |P|, nnz(H_PS) (-1 without DNQS_EMIT_HPS) and the fingerprint {sum, xor} of P (host
 * outputs, any may be NULL); DNQS_ESTATE if P was not built. */
dnqs_status dnqs_conn_p_info(const dnqs_conn *conn, int64_t *n_p, int64_t *nnz_ps, uint64_t *fingerprint);
/* Copy P and H_PS into caller buffers (dev): p_dets uint64[|P|][2] (canonical order),
 * p_diag FP64[|P|] (H_aa), row_ptr int64[|P|+1], col int32[nnz_ps], val FP32[nnz_ps];
 * any pointer may be NULL to skip it.  DNQS_ESTATE if the part asked for was not built.
 * Enqueued on the context's stream. */
dnqs_status dnqs_conn_export_p(dnqs_ctx *ctx, const dnqs_conn *conn, uint64_t *p_dets, double *p_diag,
                               int64_t *row_ptr, int32_t *col, float *val);
/* The occupied-row plan of the output layer kept with the connections (see
 * dnqs_energy_and_grad): n_dense = orbitals computed densely, or -1 when the full-width
 * layer is used; n_entries = (configuration, other occupied orbital) rows.  Host
 * outputs, either may be NULL. */
dnqs_status dnqs_conn_output_plan(const dnqs_conn *conn, int *n_dense, int64_t *n_entries);
/* Copy H_SS into caller buffers (dev): row_ptr[n+1], col[nnz], val[nnz], diag[n];
 * any pointer may be NULL to skip it.  Enqueued on the context's stream. */
dnqs_status dnqs_conn_export(dnqs_ctx *ctx, const dnqs_conn *conn, int64_t *row_ptr, int32_t *col, float *val,
                             double *diag);
void dnqs_conn_free(dnqs_conn *conn);

/* ------------------------------------------------------------------ amplitudes
 * log|psi(x)| (dev FP64[n]) and sign(psi(x)) (dev int8[n], -1/0/+1) for each det of
 * `dets` (dev uint64[n][2], any order, in the slot's sector), with
 * psi(x) = det A(x), A(x)[j][k] = Phi0[i_j][k] + DeltaPhi(x)[i_j][k] (Eqs. 2-4).
 * An exactly singular A(x) gives sign 0 and log|psi| = -inf.  n >= 1. */
dnqs_status dnqs_amplitudes(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta, const uint64_t *dets,
                            int64_t n, int precision, double *log_abs, int8_t *sign);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dnqs_amplitudes with every
 * workspace (the activations h_1 .. h_{L-1}, the output layer, the BF16 weight planes)
 * carved from a fixed 64 MiB scratch region that the library holds on each device for
 * the life of the process, so that the call allocates nothing.  Same arguments, same
 * kernels and the same results bit for bit as dnqs_amplitudes.  The region bounds n:
 * about 64 MiB / (4 (d_1 + ... + d_L)) configurations (7,000 for the 56-512-512-512-784
 * network); a larger n gives DNQS_ECAPACITY before any launch, outputs untouched.
 * Every context on a device shares that device's region and it keeps the last call's
 * contents (each workspace is written in full before it is read): calls that overlap
 * on one device, from any context or stream, race and must be serialised by the
 * caller.  No autotuning and no timing during the call. */
dnqs_status dnqs_amplitudes_noalloc(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta,
                                    const uint64_t *dets, int64_t n, int precision, double *log_abs, int8_t *sign);

/* ------------------------------------------------------------------ energy and gradient
 * One variational step's worth of work on S = conn's determinants (Eqs. 11-12):
 *   psi_x = sign_x exp(log|psi_x| - l_max)                (global scale removed)
 *   v = H_SS psi,  E = psi^T v / psi^T psi                 (FP64 reductions)
 *   grad = dE/dtheta = (2/psi^T psi) sum_x (v_x - E psi_x) d psi_x/d theta
 * Outputs (dev): energy FP64[1]; stats FP64[3] = {psi^T psi, l_max, psi^T v};
 * grad FP32[param_count] (NULL: no backward pass); v_out FP64[n] (NULL: not kept);
 * log_abs FP64[n] and sign int8[n] (NULL: not kept).  E is NaN and the call still
 * succeeds if psi^T psi underflows; grad is then zero.  Enqueued, does not wait.
 * The orbital output layer is computed for the occupied rows only where that pays:
 * when S is concentrated on some orbitals (as a set grown around a reference is), the
 * orbitals occupied in >= 35% of S take a dense GEMM and every other occupied row is
 * computed per configuration (the plan is built by dnqs_build_connections).  Results
 * equal the full-width layer up to FP32 summation order.  flags: DNQS_FULL_OUTPUT
 * forces the full-width layer (as in the batched call).  The weight gradients (and the
 * output layer's per-row products) run on a second stream of the context's device that
 * is forked from and joined back to the context's stream with events, so the call is
 * still ordered with that stream as a whole (no fork inside dnqs_capture_begin/end). */
#define DNQS_FULL_OUTPUT 1u
/* On a target set T = [V; P] (dnqs_build_target), the default objective is the Proxy mode
 * of Sec. 2.3: E = psi_T^T H~ psi_T / psi_T^T psi_T with the proxy Hamiltonian of Eq. 8,
 * and grad its exact gradient (Eq. 10).  DNQS_ASYM selects the Asymmetric objective
 * (Eq. 6), E = psi_V^T H_VT psi_T / psi_V^T psi_V (normalised on V, local energies over
 * T), with its exact gradient (every amplitude of T differentiated: the terms through
 * psi on P that Eq. 7 drops are included); DNQS_ASYM_ESTIMATOR the same energy with the
 * gradient estimator of Eq. 7, 2 sum_V p_V(x) (E_loc(x) - E) d ln|psi(x)| (not the
 * gradient of E: the paper's non-conservative field).  With either flag stats[0] is
 * psi_V^T psi_V, stats[2] is psi_V^T H_VT psi_T, and v_out holds the vector v' whose
 * residual 2 (v' - E psi) / psi_V^T psi_V is the derivative of E with respect to psi
 * (exact) or the estimator's coefficient. */
#define DNQS_ASYM 2u
#define DNQS_ASYM_ESTIMATOR 4u
/* DNQS_RECOMPUTE: keep only the last hidden layer h_{L-1} (the output layer reads it for
 * every configuration); the embedding's occupations and h_1 .. h_{L-2} are formed by
 * blocks of rows in the forward pass and formed again by block in the backward pass
 * (micro-batched gradient accumulation, Sec. 3.1), so their memory is that of one block.
 * The weight gradients' split-K partials fall on block boundaries, so the results equal
 * those without the flag bit for bit.  No effect for networks with one hidden layer. */
#define DNQS_RECOMPUTE 8u
dnqs_status dnqs_energy_and_grad(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta,
                                 const dnqs_conn *conn, int precision, unsigned flags, double *energy,
                                 double *stats, float *grad, double *v_out, double *log_abs, int8_t *sign);

/* ------------------------------------------------------------------ Lanczos
 * Lowest eigenpair of H_SS (conn) by the Lanczos iteration: E_diag = lambda_min(H_SS),
 * the exact energy within the variational space that the post-optimisation analysis
 * compares E with (Sec. 2.4), and its eigenvector, the converged psi at which Eq. 13 is
 * evaluated.  The matrix is H_SS as stored (FP32 off-diagonal values, FP64 diagonal);
 * Krylov vectors are FP64 and fully re-orthogonalised (two Gram-Schmidt rounds), every
 * reduction in a fixed order (reproducible to the bit).  start: dev FP64[n] initial
 * vector (NULL: the diagonal's lowest entries weighted up plus a fixed pseudo-random
 * spread).  Stops when the Ritz residual |H y - lambda y| <= tol max(1, |lambda|), at
 * max_iter (1..4096) vectors or on an invariant subspace.  energy: dev FP64[1]; vec:
 * dev FP64[n] unit Ritz vector (NULL: not formed); iters, residual: host (NULL: not
 * returned).  Holds (max_iter + 1) n FP64 values of workspace.  DNQS_EDOMAIN if the
 * start vector's norm is 0 or not finite (energy and vec untouched).  Synchronises the
 * stream. */
dnqs_status dnqs_lanczos(dnqs_ctx *ctx, const dnqs_conn *conn, int max_iter, double tol, const double *start,
                         double *energy, double *vec, int *iters, double *residual);

/* ------------------------------------------------------------------ PT2
 * Epstein-Nesbet correction of Eq. 13 for psi on S = conn's determinants, given
 * as (log_abs, sign) (dev, any global scale) and E (dev FP64[1]):
 *   dE = ( sum_{a in S} (v_a - E psi_a)^2 / (E - H_aa)
 *        + sum_{a in P} w_a^2 / (E - H_aa) ) / psi^T psi,
 *   v = H_SS psi, w_a = sum_{x in S} H_ax psi_x, P = C(S) \ S (unscreened).
 * Both sums use couplings computed in FP64 from the integrals (not the FP32 values of
 * H_SS): every pair (x, a) of S x C(S) is generated once, and w_a (a in P) and the
 * off-diagonal part of v_a (a in S) are summed from them.  A term whose numerator is
 * exactly 0 contributes 0.  The sums do not depend on the order of the work on the
 * device: w_a is accumulated in fixed point (integers), and each partial sum over keys
 * exactly (integer limbs) before a fixed-order FP64 sum, so repeated calls give the
 * same bits.  |S| <= 2^24 (DNQS_EINVAL otherwise).
 * out (dev FP64[4]) = {dE, internal sum, external sum, min|E-H_aa|}; the two sums are
 *   unnormalised and taken for psi scaled so that max_x |psi_x| = 1 (dE does not depend
 *   on the scale)
 * counts (dev int64[6]) = {(x,a) pairs generated, |P|, terms with |E-H_aa| < 1e-8,
 *                          sub-buckets of the on-chip reduction, fingerprint of P:
 *                          sum of h(a) mod 2^64, XOR of h(a) (as in dnqs_build_connections)}.
 * opts may be NULL.  With opts->sample_mask != 0 only keys a whose
 * SplitMix64-based key hash h(a) = mix(alpha ^ mix(beta)) has (h & sample_mask) == 0
 * enter the external sum, |P| and the fingerprint (the internal sum is always
 * complete).  With opts->export_cap > 0 up to export_cap kept keys are written to
 * export_keys (dev uint64[cap][2]) with export_w (w_a, for psi scaled so that
 * max_x |psi_x| = 1) and export_haa (H_aa) (dev FP64[cap]), and the number of kept keys
 * to export_count (dev int64[1]; may exceed export_cap).  When all kept keys fit
 * (count <= cap) they are in canonical order.
 * With opts->eps_hb > 0 the external sum, |P|, the fingerprint and the export cover only
 * the heat-bath-screened set of Eq. 14 (Sec. 3.2): the a in P whose largest coupling
 * max_x |H_ax psi_x| reaches eps_hb for psi normalised to ||psi||_2 = 1; each such a
 * with its whole w_a (eps_hb = 0: all of P).
 * Memory: the external sum materialises an 8-byte descriptor per (x, a) pair twice.
 * When 16 bytes x pairs exceed opts->max_pair_bytes (0: half of the free device memory
 * at the call), the key space is cut into 2^k slices by the top k bits of the key hash
 * and processed one slice after the other (S re-enumerated for each), so that any |S|
 * fits; the result does not depend on the slicing beyond FP64 summation order.
 * counts[3] then sums the sub-buckets over slices.  DNQS_EDOMAIN, before the sums and
 * with out and counts untouched, if log_abs has no finite maximum (psi^T psi after
 * scaling is 0 or not finite).  Synchronises the stream. */
typedef struct {
    uint64_t sample_mask;
    int64_t export_cap;
    uint64_t *export_keys;
    double *export_w;
    double *export_haa;
    int64_t *export_count;
    int64_t max_pair_bytes;
    double eps_hb;
} dnqs_pt2_opts;
dnqs_status dnqs_pt2(dnqs_ctx *ctx, int slot, const dnqs_conn *conn, const double *log_abs, const int8_t *sign,
                     const double *energy, const dnqs_pt2_opts *opts, double *out, int64_t *counts);

/* ------------------------------------------------------------------ subspace evolution
 * The two steps of Algorithm 1's outer loop that change the variational set.
 *
 * dnqs_heatbath_candidates: the screened perturbative set P_k of step 1 (Eq. 14,
 * Sec. 3.2) for psi on S = conn's determinants, given as (log_abs, sign) (dev, any
 * scale): every a outside S at excitation rank 1 or 2 from some x in S with
 * max_x |<a|H|x> psi_x| >= eps_hb for psi normalised to ||psi||_2 = 1 (eps_hb = 0: all of
 * P = C(S) \ S), sorted in canonical order and unique.  The first min(|P_k|, cap)
 * determinants go to out_dets (dev uint64[cap][2]); *n_out (host) = |P_k|, which may
 * exceed cap (call again with a larger buffer).  Every (x, a) candidate is held once:
 * DNQS_ECAPACITY if |S| n_exc >= 2^31.  Synchronises the stream.
 *
 * dnqs_select_topk: the Top-K selector of step 3 (Sec. 2.4, Fixed-Size Selection): of the
 * n determinants dets (dev uint64[n][2], any order, unique) with amplitudes
 * (log_abs, sign) (dev; sign NULL: all non-zero; sign 0 counts as the smallest), the
 * min(K, n) with the largest |psi| (equal |psi|: the lower determinant first), written in
 * canonical order to out_dets (dev uint64[K][2]); *n_out (host) = min(K, n).
 * Synchronises the stream. */
dnqs_status dnqs_heatbath_candidates(dnqs_ctx *ctx, int slot, const dnqs_conn *conn, const double *log_abs,
                                     const int8_t *sign, double eps_hb, int64_t cap, uint64_t *out_dets,
                                     int64_t *n_out);
dnqs_status dnqs_select_topk(dnqs_ctx *ctx, int slot, const uint64_t *dets, const double *log_abs,
                             const int8_t *sign, int64_t n, int64_t K, uint64_t *out_dets, int64_t *n_out);

/* ------------------------------------------------------------------ batched geometries
 * Several independent problems (e.g. the geometries of a dissociation curve), each with
 * its own integrals (slot), variational set and H_SS (conn), parameters and outputs,
 * evaluated together: every stage of energy_and_grad (embedding, each GEMM, LU, SpMV,
 * reductions, adjoint) is one launch over all problems, with work items ordered by
 * problem.  All problems share (M, n_alpha, n_beta) and the network shape.  The first
 * call with a new set of conns builds a plan (copies of S and H_SS in a concatenated
 * layout) and synchronises; later calls with the same conns and pointers only enqueue
 * (so they may be captured in a graph).  Per problem the results equal those of
 * dnqs_energy_and_grad up to the summation order of the weight gradients.
 * theta, grad, energy, stats: dev pointers as in dnqs_energy_and_grad (grad NULL for
 * every problem: no backward pass).  1 <= n_problems <= DNQS_MAX_SLOTS. */
typedef struct {
    int slot;
    const dnqs_conn *conn;
    float *theta;
    float *grad;
    double *energy;
    double *stats;
} dnqs_problem;
dnqs_status dnqs_energy_and_grad_batched(dnqs_ctx *ctx, const dnqs_net *net, int n_problems,
                                         const dnqs_problem *problems, int precision, unsigned flags);

/* AdamW (the inner-loop optimiser, Sec. 3.3) for every problem of a batch:
 * m, v: dev FP32 [n_problems * param_count] (problem-major, zero before the first step);
 * step: dev int32[1], read as t - 1 and incremented; lr follows the cosine decay
 * lr_min + (lr_max - lr_min) (1 + cos(pi min(t, decay_steps) / decay_steps)) / 2.
 * theta[i] -= lr (mhat / (sqrt(vhat) + eps) + weight_decay theta[i]).  Enqueue only. */
typedef struct {
    float lr_max, lr_min;
    int decay_steps;
    float beta1, beta2, eps, weight_decay;
} dnqs_adamw_cfg;
dnqs_status dnqs_adamw_batched(dnqs_ctx *ctx, const dnqs_net *net, int n_problems, const dnqs_problem *problems,
                               float *m, float *v, const dnqs_adamw_cfg *cfg, int *step);

/* HIP graph capture of the work a context enqueues between begin and end (the context's
 * stream must not be the null stream).  Only calls that do not synchronise may be made
 * in between: dnqs_energy_and_grad(_batched) after a first un-captured call with the
 * same arguments, dnqs_adamw_batched, dnqs_amplitudes.  dnqs_graph_launch replays the
 * graph on the context's stream. */
typedef struct dnqs_graph dnqs_graph;
dnqs_status dnqs_capture_begin(dnqs_ctx *ctx);
dnqs_status dnqs_capture_end(dnqs_ctx *ctx, dnqs_graph **out);
dnqs_status dnqs_graph_launch(dnqs_ctx *ctx, dnqs_graph *graph);
void dnqs_graph_free(dnqs_graph *graph);

/* ------------------------------------------------------------------ autotuner
 * Tile shapes of the network GEMMs (Sec. 3.3's batched inner loop is dominated by
 * them): each GEMM shape (engine, kind, M, N, K) has a configuration: tile height
 * (128 or 64 rows by 128 columns) and, for weight gradients, the split-K count.  With
 * tuning enabled, the first call that meets a shape times every candidate on the
 * context's stream (HIP events; one warm-up and three timed runs each) and keeps the
 * fastest for the context's lifetime; without it (the default) or during graph capture
 * a shape not in the table uses the default (128 rows, split-K for about 2048
 * workgroups).  Results do not depend on the tile height; the split-K count changes
 * the summation order of weight gradients only.
 * dnqs_tune_export writes the table as text, one line "engine kind M N K tm splits"
 * per shape (engine 0 FP32, 1 split BF16; kind 0 forward, 1 weight gradient, 2 data
 * gradient, 3 batched weight gradient with splits 0), NUL-terminated, at most cap
 * bytes, and returns the full length (-1 for a NULL ctx).  dnqs_tune_import merges
 * such text into the table (EINVAL on a malformed or out-of-range line, leaving the
 * table unchanged). */
dnqs_status dnqs_autotune(dnqs_ctx *ctx, int enable);
int64_t dnqs_tune_export(const dnqs_ctx *ctx, char *buf, int64_t cap);
dnqs_status dnqs_tune_import(dnqs_ctx *ctx, const char *text);

/* ------------------------------------------------------------------ timing
 * Average device time (ms) of the most recent launches of the named kernel family
 * recorded with HIP events on the context's stream since dnqs_timing_reset, and the
 * number of launches; families: "hss", "amp", "egrad", "pt2", "pt2_l1",
 * "pt2_l1_fill", "pt2_l2", "pt2_reduce".  Timing is
 * recorded only after dnqs_timing_enable(ctx, 1). */
dnqs_status dnqs_timing_enable(dnqs_ctx *ctx, int on);
dnqs_status dnqs_timing_reset(dnqs_ctx *ctx);
dnqs_status dnqs_timing_get(dnqs_ctx *ctx, const char *family, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* DNQS_H */
