// C ABI of the library (include/dnqs.h): argument validation, device memory,
// and the order of kernel launches for each call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dnqs.h"
#include "dnqs_device.h"
#include "dnqs_kernels.h"

using namespace dnqs;

namespace {

struct Slot {
    bool set = false;
    int M = 0, na = 0, nb = 0;
    double ecore = 0.0;
    double *h64 = nullptr, *eri64 = nullptr, *J = nullptr, *K = nullptr, *eri_pk = nullptr;
    float *eri32 = nullptr;
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct TimingRec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

thread_local std::string g_create_error;

}  // namespace

struct dnqs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Slot slots[DNQS_MAX_SLOTS];
    std::map<std::string, Buf> ws;
    bool timing = false;
    std::map<std::string, TimingRec> times;
    std::vector<hipEvent_t> event_pool;
};

struct dnqs_conn {
    int device = 0;
    int slot = 0;
    int M = 0, na = 0, nb = 0;
    int64_t n = 0, nnz = 0;
    uint64_t *dets = nullptr;
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    float *val = nullptr;
    double *diag = nullptr;
    uint64_t *set_keys = nullptr;
    int32_t *set_idx = nullptr;
    uint64_t set_mask = 0;
};

namespace {

dnqs_status fail(dnqs_ctx *ctx, dnqs_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return s;
}

#define HIPCHK(ctx, call)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return fail((ctx), e_ == hipErrorOutOfMemory ? DNQS_ENOMEM : DNQS_EHIP, "%s: %s (%s:%d)", #call, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                       \
    } while (0)

#define CHECK_LAUNCH(ctx) HIPCHK(ctx, hipGetLastError())

// Workspace buffer `name` of at least `bytes` bytes (grown, never shrunk).
dnqs_status ws_get(dnqs_ctx *ctx, const std::string &name, size_t bytes, void **out) {
    if (bytes == 0) bytes = 256;
    Buf &b = ctx->ws[name];
    if (b.bytes < bytes) {
        if (b.p) {
            // queued kernels may still use the old buffer
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            HIPCHK(ctx, hipFree(b.p));
        }
        b.p = nullptr;
        b.bytes = 0;
        size_t want = bytes + bytes / 8;
        want = (want + 255) & ~(size_t)255;
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            b.p = nullptr;
            (void)hipGetLastError();
            return fail(ctx, DNQS_ENOMEM, "workspace '%s': cannot allocate %zu bytes", name.c_str(), want);
        }
        b.bytes = want;
    }
    *out = b.p;
    return DNQS_OK;
}

template <typename T>
dnqs_status ws_t(dnqs_ctx *ctx, const std::string &name, size_t count, T **out) {
    void *p = nullptr;
    dnqs_status s = ws_get(ctx, name, count * sizeof(T), &p);
    *out = (T *)p;
    return s;
}

#define TRY(expr)                           \
    do {                                    \
        dnqs_status s_ = (expr);            \
        if (s_ != DNQS_OK) return s_;       \
    } while (0)

// ---------------------------------------------------------------- timing
hipEvent_t ev_take(dnqs_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timer {
    dnqs_ctx *ctx;
    const char *fam;
    hipEvent_t a = nullptr;
    Timer(dnqs_ctx *c, const char *f) : ctx(c), fam(f) {
        if (ctx->timing) {
            a = ev_take(ctx);
            if (a) (void)hipEventRecord(a, ctx->stream);
        }
    }
    void stop() {
        if (!a) return;
        hipEvent_t b = ev_take(ctx);
        if (b) {
            (void)hipEventRecord(b, ctx->stream);
            ctx->times[fam].ev.push_back({a, b});
        }
        a = nullptr;
    }
    ~Timer() { stop(); }
};

dnqs_status set_device(dnqs_ctx *ctx) {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return DNQS_OK;
}

Ham make_ham(const Slot &s) {
    Ham H;
    H.M = s.M;
    H.na = s.na;
    H.nb = s.nb;
    H.ecore = s.ecore;
    H.h64 = s.h64;
    H.eri64 = s.eri64;
    H.eri32 = s.eri32;
    H.eri_pk = s.eri_pk;
    H.J = s.J;
    H.K = s.K;
    return H;
}

dnqs_status check_slot(dnqs_ctx *ctx, int slot) {
    if (slot < 0 || slot >= DNQS_MAX_SLOTS) return fail(ctx, DNQS_EINVAL, "slot %d out of range", slot);
    if (!ctx->slots[slot].set) return fail(ctx, DNQS_ESTATE, "no integrals staged in slot %d", slot);
    return DNQS_OK;
}

int64_t n_excitations(int M, int na, int nb) {
    auto c2 = [](int64_t k) { return k * (k - 1) / 2; };
    int64_t sa = (int64_t)na * (M - na), sb = (int64_t)nb * (M - nb);
    return sa + sb + c2(na) * c2(M - na) + c2(nb) * c2(M - nb) + sa * sb;
}

struct NetView {
    int L;
    const int *w;
    int64_t offW[DNQS_MAX_LAYERS + 1], offb[DNQS_MAX_LAYERS + 1], offPhi0, total;
};

dnqs_status net_view(dnqs_ctx *ctx, const dnqs_net *net, int M, int na, int nb, NetView *v) {
    if (!net) return fail(ctx, DNQS_EINVAL, "net is NULL");
    const int L = net->n_layers;
    if (L < 2 || L > DNQS_MAX_LAYERS) return fail(ctx, DNQS_EINVAL, "n_layers = %d, need 2..%d", L, DNQS_MAX_LAYERS);
    const int No = 2 * M, Ne = na + nb;
    if (net->width[0] != No) return fail(ctx, DNQS_EINVAL, "width[0] = %d, need 2M = %d", net->width[0], No);
    if (net->width[L] != No * Ne)
        return fail(ctx, DNQS_EINVAL, "width[%d] = %d, need 2M*Ne = %d", L, net->width[L], No * Ne);
    for (int l = 0; l <= L; ++l)
        if (net->width[l] < 1 || net->width[l] > (1 << 20)) return fail(ctx, DNQS_EINVAL, "width[%d] invalid", l);
    v->L = L;
    v->w = net->width;
    int64_t off = 0;
    for (int l = 1; l <= L; ++l) {
        v->offW[l] = off;
        off += (int64_t)net->width[l - 1] * net->width[l];
        v->offb[l] = off;
        off += net->width[l];
    }
    v->offPhi0 = off;
    off += (int64_t)No * Ne;
    v->total = off;
    return DNQS_OK;
}

int splitk_splits(int M, int N, int64_t K) {
    int tiles = ((M + 127) / 128) * ((N + 127) / 128);
    int s = (2048 + tiles - 1) / tiles;
    int64_t maxs = K / 256;
    if (maxs < 1) maxs = 1;
    if (s > maxs) s = (int)maxs;
    if (s > 256) s = 256;
    if (s < 1) s = 1;
    return s;
}

// Forward pass: activations h_1..h_{L-1} kept in workspaces "h1".., output layer in "O",
// then orbital rows + LU.  With want_grad also U (occupations) and A^-1.
dnqs_status forward(dnqs_ctx *ctx, const Slot &sl, const NetView &nv, const float *theta, const uint64_t *dets,
                    int64_t n, int precision, bool want_grad, double *logabs, int8_t *sign, float **Ainv_out) {
    (void)precision;
    hipStream_t st = ctx->stream;
    const int M = sl.M, No = 2 * M, Ne = sl.na + sl.nb, L = nv.L;
    const int *w = nv.w;
    float *U = nullptr;
    if (want_grad) TRY(ws_t(ctx, "U", (size_t)n * No, &U));
    float *h = nullptr;
    TRY(ws_t(ctx, "h1", (size_t)n * w[1], &h));
    launch_embed(st, dets, n, M, w[1], theta + nv.offW[1], theta + nv.offb[1], h, U);
    CHECK_LAUNCH(ctx);
    float *prev = h;
    for (int l = 2; l <= L; ++l) {
        float *out = nullptr;
        if (l < L)
            TRY(ws_t(ctx, "h" + std::to_string(l), (size_t)n * w[l], &out));
        else
            TRY(ws_t(ctx, "O", (size_t)n * w[l], &out));
        GemmArgs g{};
        g.M = (int)n;
        g.N = w[l];
        g.K = w[l - 1];
        g.A = prev;
        g.lda = w[l - 1];
        g.B = theta + nv.offW[l];
        g.ldb = w[l];
        g.C = out;
        g.ldc = w[l];
        g.bias = theta + nv.offb[l];
        g.ones_row = -1;
        launch_gemm_f32(st, g, true, true, l < L ? EPI_BIAS_TANH : EPI_BIAS, 1);
        CHECK_LAUNCH(ctx);
        prev = out;
    }
    float *Ainv = nullptr;
    if (want_grad) TRY(ws_t(ctx, "Ainv", (size_t)n * Ne * Ne, &Ainv));
    launch_orb_lu(st, dets, n, M, sl.na, sl.nb, prev, theta + nv.offPhi0, logabs, sign, Ainv);
    CHECK_LAUNCH(ctx);
    if (Ainv_out) *Ainv_out = Ainv;
    return DNQS_OK;
}

dnqs_status validate_dets_dev(dnqs_ctx *ctx, const Slot &sl, const uint64_t *dets, int64_t n, bool order) {
    int *err = nullptr;
    TRY(ws_t(ctx, "valid_err", 1, &err));
    HIPCHK(ctx, hipMemsetAsync(err, 0, sizeof(int), ctx->stream));
    launch_validate_dets(ctx->stream, dets, n, sl.M, sl.na, sl.nb, order ? 1 : 0, err);
    CHECK_LAUNCH(ctx);
    int h = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (h & 1) return fail(ctx, DNQS_EINVAL, "a determinant has the wrong electron count for the slot's sector");
    if (h & 4) return fail(ctx, DNQS_EINVAL, "a determinant has bits set at or above M");
    if (h & 2) return fail(ctx, DNQS_EINVAL, "determinants are not in strictly ascending canonical order");
    return DNQS_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

dnqs_status dnqs_create(dnqs_ctx **out, int device, void *stream) {
    if (!out) {
        g_create_error = "out is NULL";
        return DNQS_EINVAL;
    }
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        g_create_error = "no HIP device";
        return DNQS_EHIP;
    }
    if (device < 0 || device >= count) {
        g_create_error = "device index out of range";
        return DNQS_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return DNQS_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        g_create_error = "hipGetDeviceProperties failed";
        return DNQS_EHIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
        return DNQS_EINVAL;
    }
    dnqs_ctx *c = new dnqs_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return DNQS_OK;
}

void dnqs_destroy(dnqs_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->ws)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (auto &s : ctx->slots) {
        if (!s.set) continue;
        (void)hipFree(s.h64);
        (void)hipFree(s.eri64);
        (void)hipFree(s.eri32);
        (void)hipFree(s.eri_pk);
        (void)hipFree(s.J);
        (void)hipFree(s.K);
    }
    for (auto &kv : ctx->times)
        for (auto &p : kv.second.ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
}

dnqs_status dnqs_set_stream(dnqs_ctx *ctx, void *stream) {
    if (!ctx) return DNQS_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return DNQS_OK;
}

const char *dnqs_last_error(const dnqs_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int64_t dnqs_param_count(const dnqs_net *net, int M, int n_alpha, int n_beta) {
    if (M < 1 || M > 64 || n_alpha < 0 || n_beta < 0 || n_alpha > M || n_beta > M) return -1;
    NetView v;
    if (net_view(nullptr, net, M, n_alpha, n_beta, &v) != DNQS_OK) return -1;
    return v.total;
}

dnqs_status dnqs_set_integrals(dnqs_ctx *ctx, int slot, int M, int n_alpha, int n_beta, const double *h,
                               const double *eri, double e_core) {
    if (!ctx) return DNQS_EINVAL;
    if (slot < 0 || slot >= DNQS_MAX_SLOTS) return fail(ctx, DNQS_EINVAL, "slot %d out of range", slot);
    if (M < 1 || M > 64) return fail(ctx, DNQS_EINVAL, "M = %d, need 1..64", M);
    if (n_alpha < 0 || n_beta < 0 || n_alpha > M || n_beta > M || n_alpha + n_beta < 1)
        return fail(ctx, DNQS_EINVAL, "electron counts (%d, %d) invalid for M = %d", n_alpha, n_beta, M);
    if (!h || !eri) return fail(ctx, DNQS_EINVAL, "h or eri is NULL");
    if (!std::isfinite(e_core)) return fail(ctx, DNQS_EINVAL, "e_core is not finite");
    TRY(set_device(ctx));
    Slot &s = ctx->slots[slot];
    if (s.set) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(s.h64);
        (void)hipFree(s.eri64);
        (void)hipFree(s.eri32);
        (void)hipFree(s.eri_pk);
        (void)hipFree(s.J);
        (void)hipFree(s.K);
        s = Slot();
    }
    const size_t m2 = (size_t)M * M, m4 = m2 * m2;
    HIPCHK(ctx, hipMalloc(&s.h64, m2 * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&s.eri64, m4 * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&s.eri32, m4 * sizeof(float)));
    HIPCHK(ctx, hipMalloc(&s.J, m2 * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&s.K, m2 * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&s.eri_pk, packed_eri_size(M) * sizeof(double)));
    HIPCHK(ctx, hipMemcpyAsync(s.h64, h, m2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(s.eri64, eri, m4 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    launch_stage_integrals(ctx->stream, M, s.eri64, s.eri32, s.J, s.K);
    launch_pack_eri(ctx->stream, M, s.eri64, s.eri_pk);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    s.M = M;
    s.na = n_alpha;
    s.nb = n_beta;
    s.ecore = e_core;
    s.set = true;
    return DNQS_OK;
}

void dnqs_conn_free(dnqs_conn *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->dets);
    (void)hipFree(c->row_ptr);
    (void)hipFree(c->col);
    (void)hipFree(c->val);
    (void)hipFree(c->diag);
    (void)hipFree(c->set_keys);
    (void)hipFree(c->set_idx);
    delete c;
}

dnqs_status dnqs_build_connections(dnqs_ctx *ctx, int slot, const uint64_t *dets, int64_t n, unsigned flags,
                                   dnqs_conn **out) {
    if (!ctx) return DNQS_EINVAL;
    if (!out) return fail(ctx, DNQS_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(check_slot(ctx, slot));
    if (!dets) return fail(ctx, DNQS_EINVAL, "dets is NULL");
    if (n < 1 || n >= (int64_t)1 << 31) return fail(ctx, DNQS_EINVAL, "n = %lld out of range", (long long)n);
    TRY(set_device(ctx));
    const Slot &sl = ctx->slots[slot];
    hipStream_t st = ctx->stream;
    if (flags & DNQS_VALIDATE) TRY(validate_dets_dev(ctx, sl, dets, n, true));
    Timer tm(ctx, "hss");
    dnqs_conn *c = new dnqs_conn();
    c->device = ctx->device;
    c->slot = slot;
    c->M = sl.M;
    c->na = sl.na;
    c->nb = sl.nb;
    c->n = n;
    auto cleanup = [&](dnqs_status s) {
        dnqs_conn_free(c);
        return s;
    };
#define CHK_C(call)                                                                                        \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? DNQS_ENOMEM : DNQS_EHIP, "%s: %s", #call,     \
                                hipGetErrorString(e_)));                                                   \
    } while (0)
    CHK_C(hipMalloc(&c->dets, (size_t)n * 16));
    CHK_C(hipMemcpyAsync(c->dets, dets, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
    // hash set of S at load <= 1/2
    uint64_t cap = 1024;
    while (cap < (uint64_t)(2 * n)) cap <<= 1;
    c->set_mask = cap - 1;
    CHK_C(hipMalloc(&c->set_keys, cap * 16));
    CHK_C(hipMalloc(&c->set_idx, cap * sizeof(int32_t)));
    launch_fill_u64(st, c->set_keys, 2 * cap, kEmptyKey);
    launch_detset_insert(st, c->dets, n, c->set_keys, c->set_idx, c->set_mask);
    CHK_C(hipGetLastError());
    CHK_C(hipMalloc(&c->diag, (size_t)n * sizeof(double)));
    Ham H = make_ham(sl);
    launch_diag(st, H, c->dets, n, c->diag);
    CHK_C(hipGetLastError());
    // count -> scan -> fill
    const int nsub = hss_nsub(n);
    const int64_t ncnt = n * nsub;
    int32_t *counts = nullptr;
    int64_t *offs = nullptr, *bsum = nullptr, *total = nullptr;
    dnqs_status s;
    if ((s = ws_t(ctx, "hss_counts", (size_t)ncnt, &counts)) != DNQS_OK) return cleanup(s);
    if ((s = ws_t(ctx, "hss_offs", (size_t)ncnt, &offs)) != DNQS_OK) return cleanup(s);
    if ((s = ws_t(ctx, "hss_bsum", (size_t)scan_blocks(ncnt) + 1, &bsum)) != DNQS_OK) return cleanup(s);
    if ((s = ws_t(ctx, "hss_total", 1, &total)) != DNQS_OK) return cleanup(s);
    launch_hss_count(st, H, c->dets, n, nsub, counts);
    CHK_C(hipGetLastError());
    launch_exclusive_scan(st, counts, ncnt, offs, bsum, total);
    CHK_C(hipGetLastError());
    int64_t nnz = 0;
    CHK_C(hipMemcpyAsync(&nnz, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHK_C(hipStreamSynchronize(st));
    c->nnz = nnz;
    CHK_C(hipMalloc(&c->row_ptr, (size_t)(n + 1) * sizeof(int64_t)));
    CHK_C(hipMalloc(&c->col, (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    CHK_C(hipMalloc(&c->val, (size_t)(nnz > 0 ? nnz : 1) * sizeof(float)));
    launch_hss_fill(st, H, c->dets, n, nsub, offs, c->col, c->val);
    CHK_C(hipGetLastError());
    launch_row_ptr(st, offs, n, nsub, nnz, c->row_ptr);
    CHK_C(hipGetLastError());
    tm.stop();
    CHK_C(hipStreamSynchronize(st));
#undef CHK_C
    *out = c;
    return DNQS_OK;
}

dnqs_status dnqs_conn_info(const dnqs_conn *conn, int64_t *n_dets, int64_t *nnz) {
    if (!conn) return DNQS_EINVAL;
    if (n_dets) *n_dets = conn->n;
    if (nnz) *nnz = conn->nnz;
    return DNQS_OK;
}

dnqs_status dnqs_conn_export(dnqs_ctx *ctx, const dnqs_conn *c, int64_t *row_ptr, int32_t *col, float *val,
                             double *diag) {
    if (!ctx) return DNQS_EINVAL;
    if (!c) return fail(ctx, DNQS_EINVAL, "conn is NULL");
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    if (row_ptr)
        HIPCHK(ctx, hipMemcpyAsync(row_ptr, c->row_ptr, (size_t)(c->n + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (col && c->nnz) HIPCHK(ctx, hipMemcpyAsync(col, c->col, (size_t)c->nnz * 4, hipMemcpyDeviceToDevice, st));
    if (val && c->nnz) HIPCHK(ctx, hipMemcpyAsync(val, c->val, (size_t)c->nnz * 4, hipMemcpyDeviceToDevice, st));
    if (diag) HIPCHK(ctx, hipMemcpyAsync(diag, c->diag, (size_t)c->n * 8, hipMemcpyDeviceToDevice, st));
    return DNQS_OK;
}

dnqs_status dnqs_amplitudes(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta, const uint64_t *dets,
                            int64_t n, int precision, double *log_abs, int8_t *sign) {
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    NetView nv;
    TRY(net_view(ctx, net, sl.M, sl.na, sl.nb, &nv));
    if (!theta || !dets || !log_abs || !sign) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (n < 1 || n >= (int64_t)1 << 31) return fail(ctx, DNQS_EINVAL, "n out of range");
    if (orb_lu_group(sl.na + sl.nb) == 0) return fail(ctx, DNQS_EINVAL, "N_e > 32 is not supported");
    if (precision != DNQS_FP32) return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
    TRY(set_device(ctx));
    Timer tm(ctx, "amp");
    return forward(ctx, sl, nv, theta, dets, n, precision, false, log_abs, sign, nullptr);
}

dnqs_status dnqs_energy_and_grad(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta,
                                 const dnqs_conn *conn, int precision, unsigned flags, double *energy,
                                 double *stats, float *grad, double *v_out, double *log_abs, int8_t *sign) {
    (void)flags;
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    NetView nv;
    TRY(net_view(ctx, net, sl.M, sl.na, sl.nb, &nv));
    if (!theta || !conn || !energy || !stats) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (conn->M != sl.M || conn->na != sl.na || conn->nb != sl.nb)
        return fail(ctx, DNQS_EINVAL, "connections were built for another sector");
    if (orb_lu_group(sl.na + sl.nb) == 0) return fail(ctx, DNQS_EINVAL, "N_e > 32 is not supported");
    if (precision != DNQS_FP32) return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t n = conn->n;
    const int M = sl.M, No = 2 * M, Ne = sl.na + sl.nb, L = nv.L;
    const int *w = nv.w;
    Timer tm(ctx, "egrad");
    double *la = log_abs;
    int8_t *sg = sign;
    if (!la) TRY(ws_t(ctx, "logabs", (size_t)n, &la));
    if (!sg) TRY(ws_t(ctx, "sign", (size_t)n, &sg));
    float *Ainv = nullptr;
    const bool want_grad = grad != nullptr;
    TRY(forward(ctx, sl, nv, theta, conn->dets, n, precision, want_grad, la, sg, &Ainv));
    double *psi = nullptr, *v = v_out, *part = nullptr, *part2 = nullptr;
    TRY(ws_t(ctx, "psi", (size_t)n, &psi));
    if (!v) TRY(ws_t(ctx, "v", (size_t)n, &v));
    TRY(ws_t(ctx, "red_part", (size_t)std::max<int64_t>(spmv_blocks(n), reduce_blocks(n)), &part));
    TRY(ws_t(ctx, "red_part2", (size_t)spmv_blocks(n), &part2));
    launch_scale_psi(st, la, sg, n, part, stats + 1, psi);
    CHECK_LAUNCH(ctx);
    launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, v, part, part2, stats, energy);
    CHECK_LAUNCH(ctx);
    if (!want_grad) return DNQS_OK;
    // adjoint: dO, then layer by layer
    float *dO = nullptr;
    TRY(ws_t(ctx, "dO", (size_t)n * w[L], &dO));
    launch_det_bwd(st, conn->dets, n, M, sl.na, sl.nb, psi, v, energy, stats, Ainv, dO);
    CHECK_LAUNCH(ctx);
    int maxw = 0;
    for (int l = 1; l < L; ++l) maxw = std::max(maxw, w[l]);
    float *dbuf[2];
    TRY(ws_t(ctx, "delta0", (size_t)n * maxw, &dbuf[0]));
    TRY(ws_t(ctx, "delta1", (size_t)n * maxw, &dbuf[1]));
    const float *delta = dO;  // delta_l, starting at l = L
    int which = 0;
    for (int l = L; l >= 1; --l) {
        // [h_{l-1}; 1]^T delta_l -> (dW_l, db_l)
        const float *hprev = nullptr;
        void *hp = nullptr;
        if (l == 1) {
            TRY(ws_get(ctx, "U", 1, &hp));
        } else {
            TRY(ws_get(ctx, "h" + std::to_string(l - 1), 1, &hp));
        }
        hprev = (const float *)hp;
        const int din = w[l - 1], dout = w[l];
        GemmArgs g{};
        g.M = din + 1;
        g.N = dout;
        g.K = (int)n;
        g.A = hprev;
        g.lda = din;
        g.B = delta;
        g.ldb = dout;
        g.ldc = dout;
        g.ones_row = din;
        const int splits = splitk_splits(g.M, g.N, n);
        float *partial = nullptr;
        const int64_t cnt = (int64_t)(din + 1) * dout;
        TRY(ws_t(ctx, "splitk", (size_t)cnt * splits, &partial));
        g.C = partial;
        g.c_split_stride = cnt;
        launch_gemm_f32(st, g, false, true, EPI_STORE, splits);
        CHECK_LAUNCH(ctx);
        launch_reduce_splits(st, partial, splits, cnt, grad + nv.offW[l]);
        CHECK_LAUNCH(ctx);
        if (l == 1) break;
        // delta_{l-1} = (delta_l W_l^T) * (1 - h_{l-1}^2)
        float *dnext = dbuf[which];
        which ^= 1;
        GemmArgs d{};
        d.M = (int)n;
        d.N = din;
        d.K = dout;
        d.A = delta;
        d.lda = dout;
        d.B = theta + nv.offW[l];
        d.ldb = dout;
        d.C = dnext;
        d.ldc = din;
        d.act = hprev;
        d.ldact = din;
        d.ones_row = -1;
        launch_gemm_f32(st, d, true, false, EPI_DTANH, 1);
        CHECK_LAUNCH(ctx);
        delta = dnext;
    }
    // dPhi0 equals db_L (Phi0 and b_L enter A(x) the same way)
    launch_copy_f32(st, grad + nv.offb[L], grad + nv.offPhi0, (int64_t)No * Ne);
    CHECK_LAUNCH(ctx);
    return DNQS_OK;
}

dnqs_status dnqs_pt2(dnqs_ctx *ctx, int slot, const dnqs_conn *conn, const double *log_abs, const int8_t *sign,
                     const double *energy, const dnqs_pt2_opts *opts, double *out, int64_t *counts) {
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    if (!conn || !log_abs || !sign || !energy || !out || !counts) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (conn->M != sl.M || conn->na != sl.na || conn->nb != sl.nb)
        return fail(ctx, DNQS_EINVAL, "connections were built for another sector");
    dnqs_pt2_opts o{};
    if (opts) o = *opts;
    if (o.export_cap > 0 && (!o.export_keys || !o.export_w || !o.export_haa || !o.export_count))
        return fail(ctx, DNQS_EINVAL, "export buffers missing");
    if (conn->n > pt2_max_dets())
        return fail(ctx, DNQS_EINVAL, "pt2 supports |S| <= %d (24-bit determinant index in a pair descriptor)",
                    pt2_max_dets());
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t n = conn->n;
    Timer tm(ctx, "pt2");
    Ham H = make_ham(sl);
    // psi (scaled), v = H_SS psi, psi^T psi
    double *psi = nullptr, *v = nullptr, *part = nullptr, *part2 = nullptr, *stats = nullptr, *e_tmp = nullptr;
    TRY(ws_t(ctx, "pt2_psi", (size_t)n, &psi));
    TRY(ws_t(ctx, "pt2_v", (size_t)n, &v));
    TRY(ws_t(ctx, "pt2_part", (size_t)std::max<int64_t>(spmv_blocks(n), 4 * 2048), &part));
    TRY(ws_t(ctx, "pt2_part2", (size_t)spmv_blocks(n), &part2));
    TRY(ws_t(ctx, "pt2_stats", 4, &stats));
    TRY(ws_t(ctx, "pt2_etmp", 1, &e_tmp));
    launch_scale_psi(st, log_abs, sign, n, part, stats + 1, psi);
    launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, v, part, part2, stats, e_tmp);
    CHECK_LAUNCH(ctx);
    double *acc = nullptr;
    TRY(ws_t(ctx, "pt2_acc", 8, &acc));
    launch_pt2_internal(st, psi, v, conn->diag, n, energy, part, acc);
    launch_pt2_init_acc(st, acc + 4);
    CHECK_LAUNCH(ctx);
    int *overflow = nullptr;
    TRY(ws_t(ctx, "pt2_ovf", 1, &overflow));
    DetSet S;
    S.keys = conn->set_keys;
    S.idx = conn->set_idx;
    S.mask = conn->set_mask;
    PT2Export ex;
    ex.cap = o.export_cap;
    ex.keys = o.export_keys;
    ex.w = o.export_w;
    ex.haa = o.export_haa;
    ex.count = o.export_count;
    // external sum: partitioned reduce-by-key (k_pt2_part.hip)
    const int64_t nexc = n_excitations(sl.M, sl.na, sl.nb);
    const int64_t pairs = n * nexc;
    const bool packed = sl.M <= 32 && !(sl.M == 32 && sl.na == 32 && sl.nb == 32);
    // sub-buckets of ~6000 pairs: ~2k unique keys at the measured 3.4 pairs per key,
    // half of the 4096-slot LDS table
    const int64_t nsb_target = std::max<int64_t>(1, pairs / 6000);
    int s1 = 0;
    while (((int64_t)1 << s1) < nsb_target && (1 << s1) < pt2_max_k1()) ++s1;
    int s2 = 0;
    while (((int64_t)1 << (s1 + s2)) < nsb_target && (1 << s2) < pt2_max_k2()) ++s2;
    const int K1 = 1 << s1;
    const int64_t nwg = pt2_l1_groups(n);
    uint32_t *c1 = nullptr;
    int32_t *c1t = nullptr;
    int64_t *offs1 = nullptr, *bsum = nullptr, *tot = nullptr, *bstart_d = nullptr;
    TRY(ws_t(ctx, "pt2_c1", (size_t)nwg * K1, &c1));
    TRY(ws_t(ctx, "pt2_c1t", (size_t)nwg * K1, &c1t));
    TRY(ws_t(ctx, "pt2_offs1", (size_t)nwg * K1, &offs1));
    TRY(ws_t(ctx, "pt2_bsum", (size_t)scan_blocks(nwg * K1) + 1, &bsum));
    TRY(ws_t(ctx, "pt2_tot", 2, &tot));
    TRY(ws_t(ctx, "pt2_bstart", (size_t)K1 + 1, &bstart_d));
    Timer t1(ctx, "pt2_l1");
    launch_pt2_l1(st, H, conn->dets, n, psi, s1, nwg, c1, nullptr, nullptr, false, packed);
    CHECK_LAUNCH(ctx);
    launch_transpose_u32(st, c1, nwg, K1, c1t);
    launch_exclusive_scan(st, c1t, nwg * K1, offs1, bsum, tot);
    CHECK_LAUNCH(ctx);
    int64_t total1 = 0;
    HIPCHK(ctx, hipMemcpyAsync(&total1, tot, sizeof total1, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    uint64_t *desc1 = nullptr;
    TRY(ws_t(ctx, "pt2_desc1", (size_t)std::max<int64_t>(total1, 1), &desc1));
    Timer t1f(ctx, "pt2_l1_fill");
    launch_pt2_l1(st, H, conn->dets, n, psi, s1, nwg, nullptr, offs1, desc1, true, packed);
    CHECK_LAUNCH(ctx);
    t1f.stop();
    t1.stop();
    launch_gather_starts(st, offs1, K1, nwg, tot, bstart_d);
    CHECK_LAUNCH(ctx);
    std::vector<int64_t> bstart(K1 + 1);
    HIPCHK(ctx, hipMemcpyAsync(bstart.data(), bstart_d, sizeof(int64_t) * (K1 + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    int64_t nsb_used = 0;
    for (int attempt = 0;; ++attempt) {
        const int K2 = 1 << s2;
        const uint64_t *desc = desc1;
        const int64_t *sb = bstart_d;
        int64_t nsb = K1;
        if (s2 > 0) {
            const int64_t CH = 65536;
            std::vector<PT2Chunk> chunks;
            std::vector<int64_t> bcb0(K1), bnc(K1);
            for (int b = 0; b < K1; ++b) {
                const int64_t size = bstart[b + 1] - bstart[b];
                const int64_t nc = (size + CH - 1) / CH;
                bcb0[b] = (int64_t)chunks.size();
                bnc[b] = nc;
                for (int64_t c = 0; c < nc; ++c)
                    chunks.push_back({bstart[b] + c * CH, std::min(CH, size - c * CH), bcb0[b], nc});
            }
            const int64_t nchunk = (int64_t)chunks.size();
            PT2Chunk *chunks_d = nullptr;
            int64_t *bcb0_d = nullptr, *bnc_d = nullptr, *offs2 = nullptr, *bsum2 = nullptr, *sb_d = nullptr;
            uint32_t *c2 = nullptr;
            int32_t *c2t = nullptr;
            uint64_t *desc2 = nullptr;
            TRY(ws_t(ctx, "pt2_chunks", (size_t)std::max<int64_t>(nchunk, 1), &chunks_d));
            TRY(ws_t(ctx, "pt2_bcb0", (size_t)K1, &bcb0_d));
            TRY(ws_t(ctx, "pt2_bnc", (size_t)K1, &bnc_d));
            TRY(ws_t(ctx, "pt2_c2", (size_t)std::max<int64_t>(nchunk * K2, 1), &c2));
            TRY(ws_t(ctx, "pt2_c2t", (size_t)std::max<int64_t>(nchunk * K2, 1), &c2t));
            TRY(ws_t(ctx, "pt2_offs2", (size_t)std::max<int64_t>(nchunk * K2, 1), &offs2));
            TRY(ws_t(ctx, "pt2_bsum2", (size_t)scan_blocks(nchunk * K2) + 1, &bsum2));
            TRY(ws_t(ctx, "pt2_sb", (size_t)K1 * K2 + 1, &sb_d));
            TRY(ws_t(ctx, "pt2_desc2", (size_t)std::max<int64_t>(total1, 1), &desc2));
            if (nchunk > 0)
                HIPCHK(ctx, hipMemcpyAsync(chunks_d, chunks.data(), sizeof(PT2Chunk) * nchunk, hipMemcpyHostToDevice, st));
            HIPCHK(ctx, hipMemcpyAsync(bcb0_d, bcb0.data(), sizeof(int64_t) * K1, hipMemcpyHostToDevice, st));
            HIPCHK(ctx, hipMemcpyAsync(bnc_d, bnc.data(), sizeof(int64_t) * K1, hipMemcpyHostToDevice, st));
            Timer t2(ctx, "pt2_l2");
            if (nchunk > 0) {
                launch_pt2_l2(st, desc1, chunks_d, nchunk, s2, c2, nullptr, nullptr, false);
                CHECK_LAUNCH(ctx);
                launch_l2_transpose(st, c2, chunks_d, nchunk, K2, c2t);
                launch_exclusive_scan(st, c2t, nchunk * K2, offs2, bsum2, tot + 1);
                CHECK_LAUNCH(ctx);
                launch_pt2_l2(st, desc1, chunks_d, nchunk, s2, nullptr, offs2, desc2, true);
                CHECK_LAUNCH(ctx);
            }
            launch_sub_starts(st, offs2, bstart_d, bcb0_d, bnc_d, K1, K2, sb_d);
            CHECK_LAUNCH(ctx);
            t2.stop();
            // the host vectors are read by the copies above: wait before they go out of scope
            HIPCHK(ctx, hipStreamSynchronize(st));
            desc = desc2;
            sb = sb_d;
            nsb = (int64_t)K1 * K2;
        }
        double *part_r = nullptr;
        TRY(ws_t(ctx, "pt2_part_r", (size_t)nsb * 4, &part_r));
        launch_pt2_init_acc(st, acc + 4);
        if (o.export_cap > 0) HIPCHK(ctx, hipMemsetAsync(o.export_count, 0, sizeof(int64_t), st));
        HIPCHK(ctx, hipMemsetAsync(overflow, 0, sizeof(int), st));
        Timer tr(ctx, "pt2_reduce");
        launch_pt2_reduce(st, H, conn->dets, psi, desc, sb, nsb, S, energy, o.sample_mask, ex, part_r, overflow,
                          packed);
        CHECK_LAUNCH(ctx);
        tr.stop();
        launch_pt2_accumulate(st, part_r, nsb, acc + 4);
        CHECK_LAUNCH(ctx);
        int ov = 0;
        HIPCHK(ctx, hipMemcpyAsync(&ov, overflow, sizeof ov, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        nsb_used = nsb;
        if (!ov) break;
        if ((1 << s2) >= pt2_max_k2() || attempt > 8)
            return fail(ctx, DNQS_ECAPACITY, "PT2: a sub-bucket holds more than %d unique keys", pt2_red_tab());
        ++s2;
    }
    launch_pt2_final(st, acc, acc + 4, stats, out, counts, pairs, nsb_used);
    CHECK_LAUNCH(ctx);
    tm.stop();
    HIPCHK(ctx, hipStreamSynchronize(st));
    return DNQS_OK;
}

dnqs_status dnqs_timing_enable(dnqs_ctx *ctx, int on) {
    if (!ctx) return DNQS_EINVAL;
    ctx->timing = on != 0;
    return DNQS_OK;
}

dnqs_status dnqs_timing_reset(dnqs_ctx *ctx) {
    if (!ctx) return DNQS_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &kv : ctx->times)
        for (auto &p : kv.second.ev) {
            ctx->event_pool.push_back(p.first);
            ctx->event_pool.push_back(p.second);
        }
    ctx->times.clear();
    return DNQS_OK;
}

dnqs_status dnqs_timing_get(dnqs_ctx *ctx, const char *family, double *total_ms, int64_t *launches) {
    if (!ctx || !family) return DNQS_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    int64_t k = 0;
    auto it = ctx->times.find(family);
    if (it != ctx->times.end()) {
        for (auto &p : it->second.ev) {
            float ms = 0.0f;
            HIPCHK(ctx, hipEventElapsedTime(&ms, p.first, p.second));
            tot += ms;
            ++k;
        }
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = k;
    return DNQS_OK;
}

}  // extern "C"
