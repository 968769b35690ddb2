// C ABI of the library (include/dnqs.h): argument validation, device memory,
// and the order of kernel launches for each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
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
    // 2^wexp bounds every |<a|H|x>| of the sector (a != x): max|h| + 2 N_e max|(pq|rs)|
    int wexp = 0;
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct TimingRec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

// Autotuner entry: a GEMM shape and the configuration chosen for it.
//   engine: 0 FP32 MFMA, 1 split BF16
//   kind: 0 forward, 1 weight gradient, 2 data gradient, 3 weight gradient of a batch
//         (split-K ranges from the batch plan)
struct TuneKey {
    int engine, kind, M, N, K;
    bool operator<(const TuneKey &o) const {
        if (engine != o.engine) return engine < o.engine;
        if (kind != o.kind) return kind < o.kind;
        if (M != o.M) return M < o.M;
        if (N != o.N) return N < o.N;
        return K < o.K;
    }
};
struct GemmCfg {
    int tm = 128;     // tile height (128 or 64)
    int splits = 1;   // split-K count (weight gradients; 0 = the batch plan's table)
};

thread_local std::string g_create_error;

}  // namespace

// Where the library's device memory comes from: the caller's allocator (e.g. torch's
// caching allocator, so that the caller stays the only owner of device memory), or
// hipMalloc / hipFree when the caller brings none.  dev_alloc and dev_free are the only
// places device memory is obtained and returned.
struct DevAlloc {
    void *(*alloc)(size_t bytes, void *user) = nullptr;
    void (*release)(void *p, void *user) = nullptr;
    void *user = nullptr;
};

static hipError_t dev_alloc(const DevAlloc &a, void **p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (!a.alloc) return hipMalloc(p, bytes);
    *p = a.alloc(bytes, a.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

static void dev_free(const DevAlloc &a, void *p) {
    if (!p) return;
    if (!a.alloc)
        (void)hipFree(p);
    else
        a.release(p, a.user);
}

// Scratch region of the allocation-free entry point (dnqs_amplitudes_noalloc): a
// file-scope device array, one copy per device for the life of the process.  Host code
// never passes the array's name to a kernel or a copy: its device address on each
// device is looked up once (hipGetSymbolAddress, at the first dnqs_create on that
// device, with the device current) and only that address is used.
constexpr size_t kNoAllocScratch = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of the scratch region on `device` (the current device), looked up on
// first use.
static hipError_t scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Concatenated layout of a batch of problems (built once per set of conns).
struct BatchPlan {
    bool valid = false;
    std::vector<const dnqs_conn *> conns;
    int G = 0;
    int64_t ntot = 0, nnz = 0;
    std::vector<int64_t> off, nn;
    uint64_t *dets = nullptr;
    int32_t *pid = nullptr;
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    float *val = nullptr;
    double *diag = nullptr;
    int *tile_pid = nullptr;  // per 128-row tile
    int2 *ksplit = nullptr;   // weight-gradient k ranges, problem by problem
    int2 *zrange = nullptr;   // ksplit entries [x, y) of each problem
    std::vector<int64_t> end; // end of each problem's padded span
    // work items of the per-problem reductions: {problem, first row, rows, 0}, largest
    // problem first (one workgroup each); per-item partials
    int4 *items = nullptr;
    int nitems = 0;
    double *ipart = nullptr;
    int nz = 0;
    // per-call pointers (rebuilt when they change, outside any capture)
    std::vector<ProbDev> P_h;
    ProbDev *P_d = nullptr;
    std::vector<const void *> ptr_h;  // [layer][G] weights then [layer][G] biases
    const void **ptr_d = nullptr;
    int ptr_layers = 0;
};

struct dnqs_ctx {
    int device = 0;
    DevAlloc alloc;
    // fixed scratch region: while arena is set, workspaces are carved from it in order
    // (the allocation-free entry point); nothing is allocated
    void *scratch = nullptr;  // this device's scratch region (its device address)
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Slot slots[DNQS_MAX_SLOTS];
    std::map<std::string, Buf> ws;
    bool timing = false;
    std::map<std::string, TimingRec> times;
    std::vector<hipEvent_t> event_pool;
    BatchPlan plan;
    bool capturing = false;
    bool autotune = false;
    std::map<TuneKey, GemmCfg> tuned;
    // auxiliary stream (default priority) for the weight gradients of the backward pass,
    // and its fork / join events (per layer: data ready, weight gradient done)
    hipStream_t aux = nullptr;
    hipEvent_t ev_ready[16] = {}, ev_wdone[16] = {};
    hipEvent_t ev_fwd[2] = {};  // forward output layer: input ready, sparse rows done
};

namespace {
void plan_free(dnqs_ctx *ctx, BatchPlan &b);
}

struct dnqs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

struct dnqs_conn {
    int device = 0;
    DevAlloc alloc;
    int slot = 0;
    int M = 0, na = 0, nb = 0;
    int64_t n = 0, nnz = 0;
    uint64_t *dets = nullptr;
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    float *val = nullptr;
    double *diag = nullptr;
    // target set T = [V; P] (dnqs_build_target): n_v = |V| (0: an ordinary set S)
    int64_t n_v = 0;
    // P = C(S) \ S (DNQS_EMIT_P) and H_PS (DNQS_EMIT_HPS); p_n < 0: not built
    int64_t p_n = -1, ps_nnz = -1;
    uint64_t p_fp[2] = {0, 0};
    uint64_t *p_dets = nullptr;
    double *p_diag = nullptr;
    int64_t *ps_row_ptr = nullptr;
    int32_t *ps_col = nullptr;
    float *ps_val = nullptr;
    // occupied-row plan of the orbital output layer (k_outsplit.hip); os_nd < 0: not used
    int os_nd = -1;
    int64_t os_ne = 0, os_ntiles = 0, os_nitems = 0;
    int *os_dpos = nullptr, *os_dorb = nullptr, *os_ifirst = nullptr, *os_icount = nullptr;
    int32_t *os_ex = nullptr, *os_ej = nullptr, *os_idx = nullptr;
    int4 *os_tiles = nullptr, *os_items = nullptr;
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
    if (ctx->arena) {
        const size_t want = (bytes + 255) & ~(size_t)255;
        if (ctx->arena_used + want > ctx->arena_size)
            return fail(ctx, DNQS_ECAPACITY, "workspace '%s' does not fit the %zu-byte scratch region", name.c_str(),
                        ctx->arena_size);
        *out = ctx->arena + ctx->arena_used;
        ctx->arena_used += want;
        return DNQS_OK;
    }
    Buf &b = ctx->ws[name];
    if (b.bytes < bytes) {
        if (b.p) {
            // queued kernels may still use the old buffer (on either stream)
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->aux) HIPCHK(ctx, hipStreamSynchronize(ctx->aux));
            dev_free(ctx->alloc, b.p);
        }
        b.p = nullptr;
        b.bytes = 0;
        size_t want = bytes + bytes / 8;
        want = (want + 255) & ~(size_t)255;
        hipError_t e = dev_alloc(ctx->alloc, &b.p, want);
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
        if (ctx->timing && !ctx->arena) {
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

int splitk_splits(int M, int N, int64_t K, int tm = 128) {
    int tiles = ((M + tm - 1) / tm) * ((N + 127) / 128);
    int s = (2048 + tiles - 1) / tiles;
    int64_t maxs = K / 256;
    if (maxs < 1) maxs = 1;
    if (s > maxs) s = (int)maxs;
    if (s > 256) s = 256;
    if (s < 1) s = 1;
    return s;
}

// GEMM engine of one layer: FP32 MFMA (0), or split-BF16 MFMA (1) for the hidden layers
// of DNQS_MIXED and for every layer of DNQS_SPLIT_BF16.
int gemm_engine(int precision, bool out_layer) {
    return (precision == DNQS_SPLIT_BF16 || (precision == DNQS_MIXED && !out_layer)) ? 1 : 0;
}

void launch_gemm(int engine, hipStream_t st, const GemmArgs &g, bool a_kcontig, bool b_ncontig, int epi,
                 int splits, int tm) {
    if (engine == 1)
        launch_gemm_x3(st, g, a_kcontig, b_ncontig, epi, splits, tm);
    else
        launch_gemm_f32(st, g, a_kcontig, b_ncontig, epi, splits, tm);
}

// BF16 hi / lo planes of a layer's weights W (din x dout, row-major) for the split-BF16
// engine: [dout][din] for the forward GEMM (transpose), [din][dout] for the data
// gradient; split once per call, in workspace `name`.
dnqs_status weight_planes(dnqs_ctx *ctx, const std::string &name, const float *W, int din, int dout, bool transpose,
                          GemmArgs &g) {
    void *planes = nullptr;
    TRY(ws_get(ctx, name, (size_t)din * dout * 2 * sizeof(uint16_t), &planes));
    launch_split_planes(ctx->stream, W, din, dout, transpose, planes);
    CHECK_LAUNCH(ctx);
    g.bsplit = planes;
    g.ldbs = transpose ? din : dout;
    g.bs_plane = (int64_t)din * dout;
    return DNQS_OK;
}

// Runs launch(cfg) with the configuration of `key`: the tuned one if the table has it;
// else, with tuning on and no capture in progress, every candidate is timed on the
// context stream (one warm-up and three timed runs each, HIP events) and the fastest
// kept; else the first candidate (the default).  launch() must be safe to repeat.
template <typename F>
dnqs_status tuned_launch(dnqs_ctx *ctx, const TuneKey &key, const std::vector<GemmCfg> &cands, F launch,
                         hipStream_t ts = nullptr) {
    if (!ts) ts = ctx->stream;
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return launch(it->second);
    if (!ctx->autotune || ctx->capturing || ctx->arena || cands.size() < 2) return launch(cands[0]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    float best = INFINITY;
    GemmCfg bc = cands[0];
    dnqs_status st = DNQS_OK;
    for (const GemmCfg &c : cands) {
        if ((st = launch(c)) != DNQS_OK) break;
        if (hipEventRecord(e0, ts) != hipSuccess) { st = DNQS_EHIP; break; }
        for (int r = 0; r < 3 && st == DNQS_OK; ++r) st = launch(c);
        if (st != DNQS_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, ts) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = DNQS_EHIP;
            break;
        }
        if (ms < best) {
            best = ms;
            bc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DNQS_OK) return st == DNQS_EHIP ? fail(ctx, st, "autotuner timing failed") : st;
    ctx->tuned[key] = bc;
    return launch(bc);
}

// Candidates: tile heights 128 and 64; for a weight gradient with its own split-K,
// also 1/4, 1/2 and 2 times the default split count (default first).
std::vector<GemmCfg> gemm_candidates(int M, int N, int64_t K, bool wgrad, bool plan_splits);

std::vector<GemmCfg> gemm_candidates(int M, int N, int64_t K, bool wgrad, bool plan_splits) {
    std::vector<GemmCfg> c;
    for (int tm : {128, 64}) {
        if (!wgrad || plan_splits) {
            c.push_back({tm, wgrad ? 0 : 1});
            continue;
        }
        const int s0 = splitk_splits(M, N, K, tm);
        for (int s : {s0, s0 / 4, s0 / 2, 2 * s0}) {
            if (s < 1 || s > 256 || (int64_t)s * 256 > K + 255) continue;
            bool dup = false;
            for (const GemmCfg &q : c) dup |= q.tm == tm && q.splits == s;
            if (!dup) c.push_back({tm, s});
        }
    }
    return c;
}

bool precision_ok(int p) { return p == DNQS_FP32 || p == DNQS_MIXED || p == DNQS_SPLIT_BF16; }

// Split-K of a weight gradient over K rows: chunks of a power of two rows (at least 256),
// so that the ranges of a split count are the same whether the rows are processed at
// once or in blocks of any larger power of two (the activation-recomputing backward
// reproduces the stored one's partial sums exactly).
int wgrad_chunk(int64_t K, int splits) {
    int64_t want = (K + std::max(splits, 1) - 1) / std::max(splits, 1);
    int64_t c = 256;
    while (c < want) c <<= 1;
    return (int)c;
}

// The configuration a weight-gradient GEMM of this shape runs with: the tuned one, else
// the default (first candidate).
GemmCfg wgrad_cfg(dnqs_ctx *ctx, int eng, int M, int N, int64_t K) {
    auto it = ctx->tuned.find(TuneKey{eng, 1, M, N, (int)K});
    if (it != ctx->tuned.end()) return it->second;
    return gemm_candidates(M, N, K, true, false)[0];
}

// Embedding and hidden layers 1 .. upto (<= L-1) for nb configurations (a block of rows):
// U (the occupations, if given), the layers into block workspaces returned in hs[], except
// h_{L-1}, which goes to `last` when that is given.
dnqs_status hidden_block(dnqs_ctx *ctx, const Slot &sl, const NetView &nv, const float *theta, const uint64_t *dets,
                         int64_t nb, int precision, float *U, float *last, float **hs, int upto) {
    hipStream_t st = ctx->stream;
    const int M = sl.M, L = nv.L;
    const int *w = nv.w;
    float *h = nullptr;
    if (L == 2 && last)
        h = last;
    else
        TRY(ws_t(ctx, "rc_h1", (size_t)nb * w[1], &h));
    launch_embed(st, dets, nb, M, w[1], theta + nv.offW[1], theta + nv.offb[1], h, U);
    CHECK_LAUNCH(ctx);
    hs[1] = h;
    for (int l = 2; l <= upto; ++l) {
        float *out = nullptr;
        if (l == L - 1 && last)
            out = last;
        else
            TRY(ws_t(ctx, "rc_h" + std::to_string(l), (size_t)nb * w[l], &out));
        GemmArgs g{};
        g.M = (int)nb;
        g.N = w[l];
        g.K = w[l - 1];
        g.A = hs[l - 1];
        g.lda = w[l - 1];
        g.B = theta + nv.offW[l];
        g.ldb = w[l];
        g.C = out;
        g.ldc = w[l];
        g.bias = theta + nv.offb[l];
        g.ones_row = -1;
        const int eng = gemm_engine(precision, false);
        if (eng == 1) TRY(weight_planes(ctx, "wpT" + std::to_string(l), theta + nv.offW[l], w[l - 1], w[l], true, g));
        TRY(tuned_launch(ctx, TuneKey{eng, 0, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, false, false),
                         [&](const GemmCfg &c) -> dnqs_status {
                             launch_gemm(eng, st, g, true, true, EPI_BIAS_TANH, 1, c.tm);
                             CHECK_LAUNCH(ctx);
                             return DNQS_OK;
                         }));
        hs[l] = out;
    }
    return DNQS_OK;
}

// Forward pass: activations h_1..h_{L-1} kept in workspaces "h1".. (FP32), output layer
// in "O" (FP32), then orbital rows + LU.  With want_grad also U (occupations) and A^-1.
// With a connections object that carries an occupied-row plan, the output layer is
// computed in that form ("O" then holds the dense orbitals' columns, "os_Osp" the entries).
dnqs_status forward(dnqs_ctx *ctx, const Slot &sl, const NetView &nv, const float *theta, const uint64_t *dets,
                    int64_t n, int precision, bool want_grad, double *logabs, int8_t *sign, float **Ainv_out,
                    const dnqs_conn *conn = nullptr, const float *given_last = nullptr) {
    hipStream_t st = ctx->stream;
    const size_t esz = sizeof(float);
    const int M = sl.M, No = 2 * M, Ne = sl.na + sl.nb, L = nv.L;
    const int *w = nv.w;
    void *prev = nullptr;
    int l0 = 2;
    if (given_last) {
        // the hidden layers were formed elsewhere (by blocks of rows): output layer and LU only
        prev = (void *)given_last;
        l0 = L;
    } else {
        void *U = nullptr;
        if (want_grad) TRY(ws_get(ctx, "U", (size_t)n * No * esz, &U));
        void *h = nullptr;
        TRY(ws_get(ctx, "h1", (size_t)n * w[1] * esz, &h));
        launch_embed(st, dets, n, M, w[1], theta + nv.offW[1], theta + nv.offb[1], (float *)h, (float *)U);
        CHECK_LAUNCH(ctx);
        prev = h;
    }
    OutSplit os{};
    const bool split = conn && conn->os_nd >= 0 && L >= 2 && os_fwd_fits(w[L - 1], Ne);
    for (int l = l0; l <= L; ++l) {
        if (l == L && split) {
            const int nd = conn->os_nd, wd = nd * Ne, din = w[L - 1];
            float *WD = nullptr, *OD = nullptr, *Osp = nullptr;
            TRY(ws_t(ctx, "os_WD", (size_t)(din + 1) * std::max(wd, 1), &WD));
            TRY(ws_t(ctx, "O", (size_t)n * std::max(wd, 1), &OD));
            TRY(ws_t(ctx, "os_Osp", (size_t)std::max<int64_t>(conn->os_ne, 1) * Ne, &Osp));
            launch_os_gather_w(st, theta + nv.offW[L], theta + nv.offb[L], din, w[L], Ne, nd, conn->os_dorb, WD);
            CHECK_LAUNCH(ctx);
            // the sparse rows on the auxiliary stream, alongside the dense GEMM (both read
            // only h_{L-1}); joined before the LU.  Not during capture.
            const bool fork = !ctx->capturing;
            hipStream_t ast = st;
            if (fork) {
                if (!ctx->aux) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
                for (hipEvent_t &e : ctx->ev_fwd)
                    if (!e) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
                ast = ctx->aux;
                HIPCHK(ctx, hipEventRecord(ctx->ev_fwd[0], st));
                HIPCHK(ctx, hipStreamWaitEvent(ast, ctx->ev_fwd[0], 0));
            }
            launch_os_fwd(ast, (const float *)prev, din, theta + nv.offW[L], theta + nv.offb[L], w[L], Ne,
                          conn->os_tiles, conn->os_ntiles, conn->os_ex, Osp);
            CHECK_LAUNCH(ctx);
            if (fork) HIPCHK(ctx, hipEventRecord(ctx->ev_fwd[1], ast));
            if (nd > 0) {
                GemmArgs g{};
                g.M = (int)n;
                g.N = wd;
                g.K = din;
                g.A = prev;
                g.lda = din;
                g.B = WD;
                g.ldb = wd;
                g.C = OD;
                g.ldc = wd;
                g.bias = WD + (int64_t)din * wd;
                g.ones_row = -1;
                const int eng = gemm_engine(precision, true);
                if (eng == 1) TRY(weight_planes(ctx, "wpTO", WD, din, wd, true, g));
                TRY(tuned_launch(ctx, TuneKey{eng, 0, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, false, false),
                                 [&](const GemmCfg &c) -> dnqs_status {
                                     launch_gemm(eng, st, g, true, true, EPI_BIAS, 1, c.tm);
                                     CHECK_LAUNCH(ctx);
                                     return DNQS_OK;
                                 }));
            }
            if (fork) HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_fwd[1], 0));
            os.OD = OD;
            os.Osp = Osp;
            os.dpos = conn->os_dpos;
            os.dorb = conn->os_dorb;
            os.idx = conn->os_idx;
            os.nd = nd;
            prev = nullptr;
            break;
        }
        void *out = nullptr;
        if (l < L)
            TRY(ws_get(ctx, "h" + std::to_string(l), (size_t)n * w[l] * esz, &out));
        else
            TRY(ws_get(ctx, "O", (size_t)n * w[l] * sizeof(float), &out));
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
        const int eng = gemm_engine(precision, l == L);
        if (eng == 1) TRY(weight_planes(ctx, "wpT" + std::to_string(l), theta + nv.offW[l], w[l - 1], w[l], true, g));
        const int epi = l < L ? EPI_BIAS_TANH : EPI_BIAS;
        TRY(tuned_launch(ctx, TuneKey{eng, 0, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, false, false),
                         [&](const GemmCfg &c) -> dnqs_status {
                             launch_gemm(eng, st, g, true, true, epi, 1, c.tm);
                             CHECK_LAUNCH(ctx);
                             return DNQS_OK;
                         }));
        prev = out;
    }
    float *Ainv = nullptr;
    if (want_grad) TRY(ws_t(ctx, "Ainv", (size_t)n * Ne * Ne, &Ainv));
    launch_orb_lu(st, dets, n, M, sl.na, sl.nb, (const float *)prev, theta + nv.offPhi0, logabs, sign, Ainv, {}, 0,
                  os);
    CHECK_LAUNCH(ctx);
    if (Ainv_out) *Ainv_out = Ainv;
    return DNQS_OK;
}

// Layers L-1 .. 1 of the backward pass by blocks of RB rows, recomputing U and
// h_1 .. h_{L-2} of each block: delta_{L-1} (all rows) is given.  Each block forms the
// split-K partials of every weight gradient over its own rows (chunk rc_chunk[l], RB a
// multiple of it, so its splits are the stored pass's) and folds them, in split order,
// onto the gradient: the same left-to-right sum as the stored pass's one reduction.
dnqs_status backward_blocks(dnqs_ctx *ctx, const Slot &sl, const NetView &nv, const float *theta,
                            const uint64_t *dets, int64_t n, int precision, int64_t RB, const int *rc_chunk,
                            const GemmCfg *rc_cfg, const float *deltaL1, int maxw, float *grad) {
    hipStream_t st = ctx->stream;
    const int M = sl.M, No = 2 * M, L = nv.L;
    const int *w = nv.w;
    int64_t cnt[DNQS_MAX_LAYERS + 1] = {};
    const int64_t rb = std::min(RB, n);
    size_t part_len = 1;
    for (int l = 1; l <= L - 1; ++l) {
        cnt[l] = (int64_t)(w[l - 1] + 1) * w[l];
        part_len = std::max(part_len, (size_t)cnt[l] * (size_t)((rb + rc_chunk[l] - 1) / rc_chunk[l]));
    }
    float *part = nullptr;  // one block's split partials of one layer
    TRY(ws_t(ctx, "rc_part", part_len, &part));
    float *U = nullptr, *dblk[2] = {};
    TRY(ws_t(ctx, "rc_U", (size_t)rb * No, &U));
    TRY(ws_t(ctx, "rc_d0", (size_t)rb * maxw, &dblk[0]));
    TRY(ws_t(ctx, "rc_d1", (size_t)rb * maxw, &dblk[1]));
    const int eng = gemm_engine(precision, false);
    for (int64_t r0 = 0; r0 < n; r0 += RB) {
        const int64_t nb = std::min(RB, n - r0);
        float *hs[DNQS_MAX_LAYERS + 1] = {};
        TRY(hidden_block(ctx, sl, nv, theta, dets + 2 * r0, nb, precision, U, nullptr, hs, L - 2));
        const float *delta = deltaL1 + r0 * w[L - 1];
        int which = 0;
        for (int l = L - 1; l >= 1; --l) {
            const int din = w[l - 1], dout = w[l];
            const float *hp = l == 1 ? U : hs[l - 1];
            GemmArgs g{};
            g.M = din + 1;
            g.N = dout;
            g.K = (int)nb;
            g.A = hp;
            g.lda = din;
            g.B = delta;
            g.ldb = dout;
            g.ldc = dout;
            g.ones_row = din;
            g.C = part;
            g.c_split_stride = cnt[l];
            g.k_chunk = rc_chunk[l];
            const int sp = (int)((nb + rc_chunk[l] - 1) / rc_chunk[l]);
            launch_gemm(eng, st, g, false, true, EPI_STORE, sp, rc_cfg[l].tm);
            CHECK_LAUNCH(ctx);
            launch_fold_splits(st, part, sp, cnt[l], grad + nv.offW[l], r0 > 0);
            CHECK_LAUNCH(ctx);
            if (l == 1) break;
            float *dnext = dblk[which];
            which ^= 1;
            GemmArgs d{};
            d.M = (int)nb;
            d.N = din;
            d.K = dout;
            d.A = delta;
            d.lda = dout;
            d.B = theta + nv.offW[l];
            d.ldb = dout;
            d.C = dnext;
            d.ldc = din;
            d.act = hs[l - 1];
            d.ldact = din;
            d.ones_row = -1;
            if (eng == 1) TRY(weight_planes(ctx, "wp" + std::to_string(l), theta + nv.offW[l], din, dout, false, d));
            TRY(tuned_launch(ctx, TuneKey{eng, 2, d.M, d.N, d.K}, gemm_candidates(d.M, d.N, d.K, false, false),
                             [&](const GemmCfg &c) -> dnqs_status {
                                 launch_gemm(eng, st, d, true, false, EPI_DTANH, 1, c.tm);
                                 CHECK_LAUNCH(ctx);
                                 return DNQS_OK;
                             }));
            delta = dnext;
        }
    }
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

// Occupied-row plan of the output layer for the configurations of c: the spin-orbitals
// occupied in at least 35% of S take the dense GEMM, the others one entry per occupied
// (configuration, orbital).  Used when it saves at least a fifth of the layer's work
// (a sparse entry costs about three dense rows); else os_nd stays -1.
dnqs_status os_plan(dnqs_ctx *ctx, dnqs_conn *c) {
    hipStream_t st = ctx->stream;
    const int M = c->M, No = 2 * M, Ne = c->na + c->nb;
    const int64_t n = c->n;
    unsigned long long *cnt_d = nullptr;
    TRY(ws_t(ctx, "os_cnt", (size_t)No, &cnt_d));
    HIPCHK(ctx, hipMemsetAsync(cnt_d, 0, sizeof(unsigned long long) * No, st));
    launch_os_count(st, c->dets, n, M, cnt_d);
    CHECK_LAUNCH(ctx);
    std::vector<unsigned long long> cnt(No);
    HIPCHK(ctx, hipMemcpyAsync(cnt.data(), cnt_d, sizeof(unsigned long long) * No, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    std::vector<int> dpos(No, -1), dorb(No, 0), ifirst(No, 0), icount(No, 0);
    std::vector<int64_t> eoff(No + 1, 0);
    int nd = 0;
    for (int p = 0; p < No; ++p)
        if ((double)cnt[p] >= 0.35 * (double)n) {
            dpos[p] = nd;
            dorb[nd++] = p;
        }
    for (int p = 0; p < No; ++p) eoff[p + 1] = eoff[p] + (dpos[p] < 0 ? (int64_t)cnt[p] : 0);
    const int64_t E = eoff[No];
    if (nd == No || (double)nd * n + 3.0 * (double)E > 0.8 * (double)No * n) return DNQS_OK;
    if (E >= ((int64_t)1 << 31) - 1) return DNQS_OK;  // entry ids are int32
    std::vector<int4> tiles, items;
    for (int p = 0; p < No; ++p) {
        if (dpos[p] >= 0) continue;
        for (int64_t e = eoff[p]; e < eoff[p + 1]; e += os_tile())
            tiles.push_back(make_int4(p, (int)e, (int)std::min<int64_t>(os_tile(), eoff[p + 1] - e), 0));
        ifirst[p] = (int)items.size();
        for (int64_t e = eoff[p]; e < eoff[p + 1]; e += os_item())
            items.push_back(make_int4(p, (int)e, (int)std::min<int64_t>(os_item(), eoff[p + 1] - e), 0));
        icount[p] = (int)items.size() - ifirst[p];
    }
    auto dalloc = [&](void **ptr, size_t bytes) -> dnqs_status {
        HIPCHK(ctx, dev_alloc(c->alloc, ptr, bytes > 0 ? bytes : 16));
        return DNQS_OK;
    };
    TRY(dalloc((void **)&c->os_dpos, sizeof(int) * No));
    TRY(dalloc((void **)&c->os_dorb, sizeof(int) * No));
    TRY(dalloc((void **)&c->os_ifirst, sizeof(int) * No));
    TRY(dalloc((void **)&c->os_icount, sizeof(int) * No));
    TRY(dalloc((void **)&c->os_ex, sizeof(int32_t) * E));
    TRY(dalloc((void **)&c->os_ej, sizeof(int32_t) * E));
    TRY(dalloc((void **)&c->os_idx, sizeof(int32_t) * n * Ne));
    TRY(dalloc((void **)&c->os_tiles, sizeof(int4) * tiles.size()));
    TRY(dalloc((void **)&c->os_items, sizeof(int4) * items.size()));
    int64_t *eoff_d = nullptr, *boff = nullptr;
    int *bcnt = nullptr;
    TRY(ws_t(ctx, "os_eoff", (size_t)No + 1, &eoff_d));
    TRY(ws_t(ctx, "os_bcnt", (size_t)os_blocks(n) * No, &bcnt));
    TRY(ws_t(ctx, "os_boff", (size_t)os_blocks(n) * No, &boff));
    HIPCHK(ctx, hipMemcpyAsync(c->os_dpos, dpos.data(), sizeof(int) * No, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(c->os_dorb, dorb.data(), sizeof(int) * No, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(c->os_ifirst, ifirst.data(), sizeof(int) * No, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(c->os_icount, icount.data(), sizeof(int) * No, hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(eoff_d, eoff.data(), sizeof(int64_t) * (No + 1), hipMemcpyHostToDevice, st));
    if (!tiles.empty())
        HIPCHK(ctx, hipMemcpyAsync(c->os_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, st));
    if (!items.empty())
        HIPCHK(ctx, hipMemcpyAsync(c->os_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, st));
    launch_os_build(st, c->dets, n, M, c->na, Ne, c->os_dpos, eoff_d, bcnt, boff, c->os_ex, c->os_ej, c->os_idx);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(st));  // the host vectors are read by the copies above
    c->os_nd = nd;
    c->os_ne = E;
    c->os_ntiles = (int64_t)tiles.size();
    c->os_nitems = (int64_t)items.size();
    return DNQS_OK;
}

// Hash set of S (load <= 1/2) in workspaces, for membership probes of excitations.
dnqs_status s_hash_set(dnqs_ctx *ctx, const uint64_t *dets, int64_t n, DetSet *S) {
    hipStream_t st = ctx->stream;
    uint64_t cap = 1024;
    while (cap < (uint64_t)(2 * n)) cap <<= 1;
    uint64_t *set_keys = nullptr;
    int32_t *set_idx = nullptr;
    TRY(ws_t(ctx, "ps_set_keys", (size_t)cap * 2, &set_keys));
    TRY(ws_t(ctx, "ps_set_idx", (size_t)cap, &set_idx));
    launch_fill_u64(st, set_keys, 2 * cap, kEmptyKey);
    launch_detset_insert(st, dets, n, set_keys, set_idx, cap - 1);
    CHECK_LAUNCH(ctx);
    *S = DetSet{set_keys, set_idx, cap - 1};
    return DNQS_OK;
}

// The determinants a outside S at excitation rank 1 or 2 from some x in S (P of Eq. 1),
// or with psi (scaled) and hb_eps > 0 those with max_x |<a|H|x> psi_x| >= hb_eps
// sqrt(norm2[0]) (Eq. 14), sorted in canonical order and unique, into the workspace
// "ps_p" (*out, *n_out entries).  Every candidate pair is held once: DNQS_ECAPACITY when
// |S| n_exc >= 2^31.  Synchronises the stream.
dnqs_status list_candidates(dnqs_ctx *ctx, const Slot &sl, const uint64_t *dets, int64_t n, const DetSet &S,
                            const double *psi, double hb_eps, const double *norm2, uint64_t **out,
                            int64_t *n_out) {
    hipStream_t st = ctx->stream;
    const int M = sl.M;
    const int64_t nexc = n_excitations(sl.M, sl.na, sl.nb);
    if ((double)n * (double)nexc >= 2147483647.0)
        return fail(ctx, DNQS_ECAPACITY, "candidates are listed only for |S| n_exc < 2^31 (here %.3g)",
                    (double)n * nexc);
    Ham H = make_ham(sl);
    int32_t *cnt = nullptr;
    int64_t *off = nullptr, *bsum = nullptr, *tot = nullptr;
    TRY(ws_t(ctx, "ps_cnt", (size_t)n, &cnt));
    TRY(ws_t(ctx, "ps_off", (size_t)n + 1, &off));
    TRY(ws_t(ctx, "ps_bsum", (size_t)scan_blocks(n) + 1, &bsum));
    TRY(ws_t(ctx, "ps_tot", 2, &tot));
    launch_pc_pass(st, H, dets, n, S, psi, hb_eps, norm2, cnt, nullptr, nullptr, nullptr, false);
    launch_exclusive_scan(st, cnt, n, off, bsum, tot);
    CHECK_LAUNCH(ctx);
    int64_t m = 0;
    HIPCHK(ctx, hipMemcpyAsync(&m, tot, sizeof m, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    const bool two = M > 32;
    uint64_t *ka = nullptr, *kb = nullptr, *key = nullptr;
    int32_t *perm = nullptr;
    TRY(ws_t(ctx, "ps_ka", (size_t)std::max<int64_t>(m, 1), &ka));
    if (two) TRY(ws_t(ctx, "ps_kb", (size_t)std::max<int64_t>(m, 1), &kb));
    TRY(ws_t(ctx, "ps_perm", (size_t)std::max<int64_t>(m, 1), &perm));
    launch_pc_pass(st, H, dets, n, S, psi, hb_eps, norm2, nullptr, off, ka, kb, true);
    CHECK_LAUNCH(ctx);
    // sort the candidates into canonical order
    SortScratch w{};
    const size_t nc = sort_scratch_counts(m);
    TRY(ws_t(ctx, "sort_keys", (size_t)std::max<int64_t>(m, 1), &w.keys));
    TRY(ws_t(ctx, "sort_vals", (size_t)std::max<int64_t>(m, 1), &w.vals));
    TRY(ws_t(ctx, "sort_counts", nc, &w.counts));
    TRY(ws_t(ctx, "sort_offs", nc, &w.offs));
    TRY(ws_t(ctx, "sort_bsum", (size_t)scan_blocks((int64_t)nc) + 1, &w.bsum));
    TRY(ws_t(ctx, "sort_total", 1, &w.total));
    launch_iota_i32(st, perm, m);
    if (!two) {
        launch_radix_sort(st, ka, perm, m, 2 * M, w);
    } else {
        TRY(ws_t(ctx, "ps_key", (size_t)std::max<int64_t>(m, 1), &key));
        HIPCHK(ctx, hipMemcpyAsync(key, kb, (size_t)m * 8, hipMemcpyDeviceToDevice, st));
        launch_radix_sort(st, key, perm, m, M, w);
        launch_gather_u64(st, ka, perm, m, key);
        launch_radix_sort(st, key, perm, m, M, w);
    }
    CHECK_LAUNCH(ctx);
    // drop duplicates
    int32_t *flag = nullptr;
    int64_t *pos = nullptr, *bsum2 = nullptr;
    TRY(ws_t(ctx, "ps_flag", (size_t)std::max<int64_t>(m, 1), &flag));
    TRY(ws_t(ctx, "ps_pos", (size_t)std::max<int64_t>(m, 1), &pos));
    TRY(ws_t(ctx, "ps_bsum2", (size_t)scan_blocks(m) + 1, &bsum2));
    int64_t np = 0;
    if (m > 0) {
        launch_unique(st, ka, kb, perm, m, two, M, flag, pos, bsum2, tot + 1, nullptr, false);
        CHECK_LAUNCH(ctx);
        HIPCHK(ctx, hipMemcpyAsync(&np, tot + 1, sizeof np, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    }
    uint64_t *pd = nullptr;
    TRY(ws_t(ctx, "ps_p", (size_t)std::max<int64_t>(np, 1) * 2, &pd));
    if (m > 0) launch_unique(st, ka, kb, perm, m, two, M, flag, pos, bsum2, tot + 1, pd, true);
    CHECK_LAUNCH(ctx);
    *out = pd;
    *n_out = np;
    return DNQS_OK;
}

// P = C(S) \ S of the connections c, sorted and unique, with H_aa, the fingerprint and
// (hps) the rows H_PS (k_pset.hip).
dnqs_status build_pset(dnqs_ctx *ctx, const Slot &sl, dnqs_conn *c, bool hps) {
    hipStream_t st = ctx->stream;
    const int64_t n = c->n;
    DetSet S{};
    TRY(s_hash_set(ctx, c->dets, n, &S));
    uint64_t *pw = nullptr;
    int64_t np = 0;
    TRY(list_candidates(ctx, sl, c->dets, n, S, nullptr, 0.0, nullptr, &pw, &np));
    c->p_n = np;
    HIPCHK(ctx, dev_alloc(c->alloc, (void **)&c->p_dets, (size_t)std::max<int64_t>(np, 1) * 16));
    HIPCHK(ctx, dev_alloc(c->alloc, (void **)&c->p_diag, (size_t)std::max<int64_t>(np, 1) * 8));
    if (np > 0) HIPCHK(ctx, hipMemcpyAsync(c->p_dets, pw, (size_t)np * 16, hipMemcpyDeviceToDevice, st));
    unsigned long long *fp = nullptr;
    int64_t *tot = nullptr;
    TRY(ws_t(ctx, "ps_fp", 2, &fp));
    TRY(ws_t(ctx, "ps_tot", 2, &tot));
    HIPCHK(ctx, hipMemsetAsync(fp, 0, 16, st));
    launch_fingerprint(st, c->p_dets, np, fp);
    Ham H = make_ham(sl);
    if (np > 0) launch_diag(st, H, c->p_dets, np, c->p_diag);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipMemcpyAsync(c->p_fp, fp, 16, hipMemcpyDeviceToHost, st));
    if (hps) {
        int32_t *rc = nullptr;
        int64_t *roff = nullptr, *rbsum = nullptr;
        TRY(ws_t(ctx, "ps_rcnt", (size_t)std::max<int64_t>(np, 1), &rc));
        TRY(ws_t(ctx, "ps_roff", (size_t)std::max<int64_t>(np, 1), &roff));
        TRY(ws_t(ctx, "ps_rbsum", (size_t)scan_blocks(np) + 1, &rbsum));
        int64_t nnz = 0;
        HIPCHK(ctx, hipMemsetAsync(tot, 0, sizeof(int64_t), st));
        if (np > 0) {
            launch_hps_pass(st, H, c->p_dets, np, S, rc, nullptr, nullptr, nullptr, false);
            launch_exclusive_scan(st, rc, np, roff, rbsum, tot);
            CHECK_LAUNCH(ctx);
            HIPCHK(ctx, hipMemcpyAsync(&nnz, tot, sizeof nnz, hipMemcpyDeviceToHost, st));
            HIPCHK(ctx, hipStreamSynchronize(st));
        }
        c->ps_nnz = nnz;
        HIPCHK(ctx, dev_alloc(c->alloc, (void **)&c->ps_row_ptr, (size_t)(np + 1) * 8));
        HIPCHK(ctx, dev_alloc(c->alloc, (void **)&c->ps_col, (size_t)std::max<int64_t>(nnz, 1) * 4));
        HIPCHK(ctx, dev_alloc(c->alloc, (void **)&c->ps_val, (size_t)std::max<int64_t>(nnz, 1) * 4));
        if (np > 0) launch_hps_pass(st, H, c->p_dets, np, S, rc, roff, c->ps_col, c->ps_val, true);
        launch_rows_finish(st, roff, np, tot, c->ps_row_ptr, c->ps_col, c->ps_val);
        CHECK_LAUNCH(ctx);
    }
    HIPCHK(ctx, hipStreamSynchronize(st));
    return DNQS_OK;
}

// The exported keys of a PT2 call in canonical order (with their w_a and H_aa), when
// all of them fit the caller's buffers; the reduce writes them in workgroup order.
dnqs_status pt2_export_sort(dnqs_ctx *ctx, int M, const dnqs_pt2_opts &o) {
    hipStream_t st = ctx->stream;
    int64_t cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(&cnt, o.export_count, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (cnt > o.export_cap || cnt < 2) return DNQS_OK;
    SortScratch w{};
    const size_t nc = sort_scratch_counts(cnt);
    int32_t *perm = nullptr;
    uint64_t *key = nullptr, *tmp = nullptr;
    TRY(ws_t(ctx, "sort_keys", (size_t)cnt, &w.keys));
    TRY(ws_t(ctx, "sort_vals", (size_t)cnt, &w.vals));
    TRY(ws_t(ctx, "sort_counts", nc, &w.counts));
    TRY(ws_t(ctx, "sort_offs", nc, &w.offs));
    TRY(ws_t(ctx, "sort_bsum", (size_t)scan_blocks((int64_t)nc) + 1, &w.bsum));
    TRY(ws_t(ctx, "sort_total", 1, &w.total));
    TRY(ws_t(ctx, "ex_perm", (size_t)cnt, &perm));
    TRY(ws_t(ctx, "ex_key", (size_t)cnt, &key));
    TRY(ws_t(ctx, "ex_tmp", (size_t)cnt * 2, &tmp));
    launch_sort_dets(st, o.export_keys, cnt, M, perm, key, w);
    launch_permute_words(st, o.export_keys, perm, cnt, 2, tmp);
    HIPCHK(ctx, hipMemcpyAsync(o.export_keys, tmp, (size_t)cnt * 16, hipMemcpyDeviceToDevice, st));
    launch_permute_words(st, (const uint64_t *)o.export_w, perm, cnt, 1, tmp);
    HIPCHK(ctx, hipMemcpyAsync(o.export_w, tmp, (size_t)cnt * 8, hipMemcpyDeviceToDevice, st));
    launch_permute_words(st, (const uint64_t *)o.export_haa, perm, cnt, 1, tmp);
    HIPCHK(ctx, hipMemcpyAsync(o.export_haa, tmp, (size_t)cnt * 8, hipMemcpyDeviceToDevice, st));
    CHECK_LAUNCH(ctx);
    return DNQS_OK;
}

// Lowest eigenvalue of the symmetric tridiagonal matrix (diagonal a, off-diagonal b)
// by bisection on the Sturm count, then its eigenvector by inverse iteration with the
// shift just below it (T - sigma I is then positive definite: elimination without
// pivoting is stable).  Host arithmetic on at most a few hundred entries.
double tri_lowest(const std::vector<double> &a, const std::vector<double> &b, std::vector<double> &y) {
    const int m = (int)a.size();
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto below = [&](double x) {  // eigenvalues < x
        int c = 0;
        double q = a[0] - x;
        if (q < 0) ++c;
        for (int i = 1; i < m; ++i) {
            if (q == 0.0) q = 1e-300;
            q = a[i] - x - b[i - 1] * b[i - 1] / q;
            if (q < 0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 4e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    const double sigma = lo - 1e-12 * std::max(1.0, std::fabs(lam)) - (hi - lo);
    y.assign(m, 1.0);
    std::vector<double> d(m), l(m);
    // LDL^T of T - sigma I
    d[0] = a[0] - sigma;
    for (int i = 1; i < m; ++i) {
        l[i] = b[i - 1] / d[i - 1];
        d[i] = a[i] - sigma - l[i] * b[i - 1];
    }
    for (int it = 0; it < 4; ++it) {
        for (int i = 1; i < m; ++i) y[i] -= l[i] * y[i - 1];
        for (int i = 0; i < m; ++i) y[i] /= d[i];
        for (int i = m - 2; i >= 0; --i) y[i] -= l[i + 1] * y[i + 1];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += y[i] * y[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < m; ++i) y[i] /= nrm;
    }
    return lam;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

dnqs_status dnqs_create(dnqs_ctx **out, int device, void *stream, void *(*alloc)(size_t bytes, void *user),
                        void (*release)(void *p, void *user), void *user) {
    if (!out) {
        g_create_error = "out is NULL";
        return DNQS_EINVAL;
    }
    if ((alloc == nullptr) != (release == nullptr)) {
        g_create_error = "alloc and release must both be given or both be NULL";
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
    void *scr = nullptr;
    if (scratch_address(device, &scr) != hipSuccess) {
        g_create_error = "hipGetSymbolAddress of the scratch region failed";
        return DNQS_EHIP;
    }
    dnqs_ctx *c = new dnqs_ctx();
    c->device = device;
    c->scratch = scr;
    c->stream = (hipStream_t)stream;
    c->alloc.alloc = alloc;
    c->alloc.release = release;
    c->alloc.user = user;
    *out = c;
    return DNQS_OK;
}

void dnqs_destroy(dnqs_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    for (int i = 0; i < 16; ++i) {
        if (ctx->ev_ready[i]) (void)hipEventDestroy(ctx->ev_ready[i]);
        if (ctx->ev_wdone[i]) (void)hipEventDestroy(ctx->ev_wdone[i]);
    }
    for (hipEvent_t e : ctx->ev_fwd)
        if (e) (void)hipEventDestroy(e);
    for (auto &kv : ctx->ws)
        dev_free(ctx->alloc, kv.second.p);
    for (auto &s : ctx->slots) {
        if (!s.set) continue;
        for (void *q : {(void *)s.h64, (void *)s.eri64, (void *)s.eri32, (void *)s.eri_pk, (void *)s.J, (void *)s.K})
            dev_free(ctx->alloc, q);
    }
    for (auto &kv : ctx->times)
        for (auto &p : kv.second.ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    plan_free(ctx, ctx->plan);
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
    {
        const size_t m2 = (size_t)M * M;
        for (size_t i = 0; i < m2; ++i)
            if (!std::isfinite(h[i])) return fail(ctx, DNQS_EINVAL, "h[%zu] is not finite", i);
        for (size_t i = 0; i < m2 * m2; ++i)
            if (!std::isfinite(eri[i])) return fail(ctx, DNQS_EINVAL, "eri[%zu] is not finite", i);
    }
    TRY(set_device(ctx));
    Slot &s = ctx->slots[slot];
    if (s.set) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (void *q : {(void *)s.h64, (void *)s.eri64, (void *)s.eri32, (void *)s.eri_pk, (void *)s.J, (void *)s.K})
            dev_free(ctx->alloc, q);
        s = Slot();
    }
    const size_t m2 = (size_t)M * M, m4 = m2 * m2;
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.h64, m2 * sizeof(double)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.eri64, m4 * sizeof(double)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.eri32, m4 * sizeof(float)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.J, m2 * sizeof(double)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.K, m2 * sizeof(double)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&s.eri_pk, packed_eri_size(M) * sizeof(double)));
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
    {
        double mh = 0.0, me = 0.0;
        for (size_t i = 0; i < m2; ++i) mh = std::max(mh, std::fabs(h[i]));
        for (size_t i = 0; i < m4; ++i) me = std::max(me, std::fabs(eri[i]));
        const double bound = mh + 2.0 * (n_alpha + n_beta) * me;
        int e = 0;
        if (bound > 0.0) (void)std::frexp(bound, &e);  // bound < 2^e
        s.wexp = e + 1;
    }
    s.set = true;
    return DNQS_OK;
}

void dnqs_conn_free(dnqs_conn *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (void *q : {(void *)c->dets, (void *)c->row_ptr, (void *)c->col, (void *)c->val, (void *)c->diag})
        dev_free(c->alloc, q);
    for (void *q : {(void *)c->p_dets, (void *)c->p_diag, (void *)c->ps_row_ptr, (void *)c->ps_col, (void *)c->ps_val})
        dev_free(c->alloc, q);
    for (void *q : {(void *)c->os_dpos, (void *)c->os_dorb, (void *)c->os_ifirst, (void *)c->os_icount,
                    (void *)c->os_ex, (void *)c->os_ej, (void *)c->os_idx, (void *)c->os_tiles, (void *)c->os_items})
        dev_free(c->alloc, q);
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
    if (flags & ~(DNQS_VALIDATE | DNQS_EMIT_P | DNQS_EMIT_HPS))
        return fail(ctx, DNQS_EINVAL, "unknown flags 0x%x", flags);
    TRY(set_device(ctx));
    const Slot &sl = ctx->slots[slot];
    hipStream_t st = ctx->stream;
    if (flags & DNQS_VALIDATE) TRY(validate_dets_dev(ctx, sl, dets, n, true));
    Timer tm(ctx, "hss");
    dnqs_conn *c = new dnqs_conn();
    c->device = ctx->device;
    c->alloc = ctx->alloc;
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
    CHK_C(dev_alloc(c->alloc, (void **)&c->dets, (size_t)n * 16));
    CHK_C(hipMemcpyAsync(c->dets, dets, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
    CHK_C(dev_alloc(c->alloc, (void **)&c->diag, (size_t)n * sizeof(double)));
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
    CHK_C(dev_alloc(c->alloc, (void **)&c->row_ptr, (size_t)(n + 1) * sizeof(int64_t)));
    CHK_C(dev_alloc(c->alloc, (void **)&c->col, (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    CHK_C(dev_alloc(c->alloc, (void **)&c->val, (size_t)(nnz > 0 ? nnz : 1) * sizeof(float)));
    launch_hss_fill(st, H, c->dets, n, nsub, offs, c->col, c->val);
    CHK_C(hipGetLastError());
    launch_row_ptr(st, offs, n, nsub, nnz, c->row_ptr);
    CHK_C(hipGetLastError());
    if (nnz > 0) launch_hss_values(st, H, c->dets, n, c->row_ptr, c->col, c->val);
    CHK_C(hipGetLastError());
    if ((s = os_plan(ctx, c)) != DNQS_OK) return cleanup(s);
    if (flags & (DNQS_EMIT_P | DNQS_EMIT_HPS))
        if ((s = build_pset(ctx, sl, c, (flags & DNQS_EMIT_HPS) != 0)) != DNQS_OK) return cleanup(s);
    tm.stop();
    CHK_C(hipStreamSynchronize(st));
#undef CHK_C
    *out = c;
    return DNQS_OK;
}

dnqs_status dnqs_build_target(dnqs_ctx *ctx, int slot, const dnqs_conn *cv, const uint64_t *p_dets, int64_t n_p,
                              unsigned flags, dnqs_conn **out) {
    if (!ctx) return DNQS_EINVAL;
    if (!out) return fail(ctx, DNQS_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    if (!cv || (n_p > 0 && !p_dets)) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (cv->n_v > 0) return fail(ctx, DNQS_EINVAL, "the connections are already a target set");
    if (cv->M != sl.M || cv->na != sl.na || cv->nb != sl.nb)
        return fail(ctx, DNQS_EINVAL, "connections were built for another sector");
    if (n_p < 0 || cv->n + n_p >= (int64_t)1 << 31) return fail(ctx, DNQS_EINVAL, "n_p out of range");
    if (flags & ~DNQS_VALIDATE) return fail(ctx, DNQS_EINVAL, "unknown flags 0x%x", flags);
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    if ((flags & DNQS_VALIDATE) && n_p > 0) TRY(validate_dets_dev(ctx, sl, p_dets, n_p, true));
    Timer tm(ctx, "target");
    const int64_t nv = cv->n, np = n_p, nt = nv + np;
    DetSet S{};
    TRY(s_hash_set(ctx, cv->dets, nv, &S));
    if (flags & DNQS_VALIDATE) {
        int *cnt_in = nullptr;
        TRY(ws_t(ctx, "tg_in", 1, &cnt_in));
        HIPCHK(ctx, hipMemsetAsync(cnt_in, 0, sizeof(int), st));
        launch_count_in_set(st, p_dets, np, S, cnt_in);
        CHECK_LAUNCH(ctx);
        int h = 0;
        HIPCHK(ctx, hipMemcpyAsync(&h, cnt_in, sizeof h, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (h) return fail(ctx, DNQS_EINVAL, "%d determinants of P are members of V", h);
    }
    Ham H = make_ham(sl);
    // H_PV: rows over P, columns in V (ascending)
    int32_t *rc = nullptr, *pvc = nullptr, *tcnt = nullptr, *vpc = nullptr, *len = nullptr;
    int64_t *pvr = nullptr, *rbsum = nullptr, *tot = nullptr, *vpr = nullptr, *voff = nullptr, *toff = nullptr;
    float *pvv = nullptr, *vpv = nullptr;
    TRY(ws_t(ctx, "tg_rc", (size_t)std::max<int64_t>(np, 1), &rc));
    TRY(ws_t(ctx, "tg_pvr", (size_t)np + 1, &pvr));
    TRY(ws_t(ctx, "tg_bsum", (size_t)scan_blocks(std::max(nt, np)) + 1, &rbsum));
    TRY(ws_t(ctx, "tg_tot", 4, &tot));
    HIPCHK(ctx, hipMemsetAsync(tot, 0, 4 * sizeof(int64_t), st));
    int64_t nnz_pv = 0;
    if (np > 0) {
        launch_hps_pass(st, H, p_dets, np, S, rc, nullptr, nullptr, nullptr, false);
        launch_exclusive_scan(st, rc, np, pvr, rbsum, tot);
        CHECK_LAUNCH(ctx);
        HIPCHK(ctx, hipMemcpyAsync(&nnz_pv, tot, sizeof nnz_pv, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
    }
    TRY(ws_t(ctx, "tg_pvc", (size_t)std::max<int64_t>(nnz_pv, 1), &pvc));
    TRY(ws_t(ctx, "tg_pvv", (size_t)std::max<int64_t>(nnz_pv, 1), &pvv));
    if (np > 0) launch_hps_pass(st, H, p_dets, np, S, rc, pvr, pvc, pvv, true);
    launch_rows_finish(st, pvr, np, tot, pvr, pvc, pvv);
    // H_VP = H_PV^T: rows over V, columns in P (ascending)
    TRY(ws_t(ctx, "tg_tcnt", (size_t)std::max<int64_t>(nv, 1), &tcnt));
    TRY(ws_t(ctx, "tg_voff", (size_t)nv + 1, &voff));
    TRY(ws_t(ctx, "tg_vpr", (size_t)nv + 1, &vpr));
    TRY(ws_t(ctx, "tg_vpc", (size_t)std::max<int64_t>(nnz_pv, 1), &vpc));
    TRY(ws_t(ctx, "tg_vpv", (size_t)std::max<int64_t>(nnz_pv, 1), &vpv));
    HIPCHK(ctx, hipMemsetAsync(tcnt, 0, sizeof(int32_t) * nv, st));
    launch_csr_transpose(st, pvr, pvc, pvv, np, nv, tcnt, voff, rbsum, tot + 1, vpr, vpc, vpv, false);
    HIPCHK(ctx, hipMemsetAsync(tcnt, 0, sizeof(int32_t) * nv, st));
    launch_csr_transpose(st, pvr, pvc, pvv, np, nv, tcnt, voff, rbsum, tot + 1, vpr, vpc, vpv, true);
    CHECK_LAUNCH(ctx);
    // the proxy matrix over T
    dnqs_conn *c = new dnqs_conn();
    c->device = ctx->device;
    c->alloc = ctx->alloc;
    c->slot = slot;
    c->M = sl.M;
    c->na = sl.na;
    c->nb = sl.nb;
    c->n = nt;
    c->n_v = nv;
    auto cleanup = [&](dnqs_status s2) {
        dnqs_conn_free(c);
        return s2;
    };
#define CHK_T(call)                                                                                        \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return cleanup(fail(ctx, e_ == hipErrorOutOfMemory ? DNQS_ENOMEM : DNQS_EHIP, "%s: %s", #call,     \
                                hipGetErrorString(e_)));                                                   \
    } while (0)
    dnqs_status s2;
    if ((s2 = ws_t(ctx, "tg_len", (size_t)nt, &len)) != DNQS_OK) return cleanup(s2);
    if ((s2 = ws_t(ctx, "tg_toff", (size_t)nt + 1, &toff)) != DNQS_OK) return cleanup(s2);
    launch_target_assemble(st, cv->row_ptr, cv->col, cv->val, vpr, vpc, vpv, pvr, pvc, pvv, nv, np, len, toff,
                           rbsum, tot + 2, nullptr, nullptr, false);
    CHK_T(hipGetLastError());
    int64_t nnz = 0;
    CHK_T(hipMemcpyAsync(&nnz, tot + 2, sizeof nnz, hipMemcpyDeviceToHost, st));
    CHK_T(hipStreamSynchronize(st));
    c->nnz = nnz;
    CHK_T(dev_alloc(c->alloc, (void **)&c->dets, (size_t)nt * 16));
    CHK_T(dev_alloc(c->alloc, (void **)&c->diag, (size_t)nt * 8));
    CHK_T(dev_alloc(c->alloc, (void **)&c->row_ptr, (size_t)(nt + 1) * 8));
    CHK_T(dev_alloc(c->alloc, (void **)&c->col, (size_t)std::max<int64_t>(nnz, 1) * 4));
    CHK_T(dev_alloc(c->alloc, (void **)&c->val, (size_t)std::max<int64_t>(nnz, 1) * 4));
    CHK_T(hipMemcpyAsync(c->dets, cv->dets, (size_t)nv * 16, hipMemcpyDeviceToDevice, st));
    if (np > 0) CHK_T(hipMemcpyAsync(c->dets + 2 * nv, p_dets, (size_t)np * 16, hipMemcpyDeviceToDevice, st));
    CHK_T(hipMemcpyAsync(c->diag, cv->diag, (size_t)nv * 8, hipMemcpyDeviceToDevice, st));
    if (np > 0) launch_diag(st, H, p_dets, np, c->diag + nv);
    launch_target_assemble(st, cv->row_ptr, cv->col, cv->val, vpr, vpc, vpv, pvr, pvc, pvv, nv, np, len, toff,
                           rbsum, tot + 2, c->col, c->val, true);
    launch_row_ptr_from_offsets(st, toff, nt, tot + 2, c->row_ptr);
    CHK_T(hipGetLastError());
#undef CHK_T
    if ((s2 = os_plan(ctx, c)) != DNQS_OK) return cleanup(s2);
    tm.stop();
    HIPCHK(ctx, hipStreamSynchronize(st));
    *out = c;
    return DNQS_OK;
}

dnqs_status dnqs_conn_info(const dnqs_conn *conn, int64_t *n_dets, int64_t *nnz) {
    if (!conn) return DNQS_EINVAL;
    if (n_dets) *n_dets = conn->n;
    if (nnz) *nnz = conn->nnz;
    return DNQS_OK;
}

dnqs_status dnqs_conn_output_plan(const dnqs_conn *conn, int *n_dense, int64_t *n_entries) {
    if (!conn) return DNQS_EINVAL;
    if (n_dense) *n_dense = conn->os_nd;
    if (n_entries) *n_entries = conn->os_nd >= 0 ? conn->os_ne : 0;
    return DNQS_OK;
}

dnqs_status dnqs_conn_p_info(const dnqs_conn *conn, int64_t *n_p, int64_t *nnz_ps, uint64_t *fingerprint) {
    if (!conn) return DNQS_EINVAL;
    if (conn->p_n < 0) return DNQS_ESTATE;
    if (n_p) *n_p = conn->p_n;
    if (nnz_ps) *nnz_ps = conn->ps_nnz;
    if (fingerprint) {
        fingerprint[0] = conn->p_fp[0];
        fingerprint[1] = conn->p_fp[1];
    }
    return DNQS_OK;
}

dnqs_status dnqs_conn_export_p(dnqs_ctx *ctx, const dnqs_conn *c, uint64_t *p_dets, double *p_diag, int64_t *row_ptr,
                               int32_t *col, float *val) {
    if (!ctx) return DNQS_EINVAL;
    if (!c) return fail(ctx, DNQS_EINVAL, "conn is NULL");
    if (c->p_n < 0) return fail(ctx, DNQS_ESTATE, "P was not built (DNQS_EMIT_P)");
    if ((row_ptr || col || val) && c->ps_nnz < 0) return fail(ctx, DNQS_ESTATE, "H_PS was not built (DNQS_EMIT_HPS)");
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t np = c->p_n;
    if (p_dets && np) HIPCHK(ctx, hipMemcpyAsync(p_dets, c->p_dets, (size_t)np * 16, hipMemcpyDeviceToDevice, st));
    if (p_diag && np) HIPCHK(ctx, hipMemcpyAsync(p_diag, c->p_diag, (size_t)np * 8, hipMemcpyDeviceToDevice, st));
    if (row_ptr) HIPCHK(ctx, hipMemcpyAsync(row_ptr, c->ps_row_ptr, (size_t)(np + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (col && c->ps_nnz > 0)
        HIPCHK(ctx, hipMemcpyAsync(col, c->ps_col, (size_t)c->ps_nnz * 4, hipMemcpyDeviceToDevice, st));
    if (val && c->ps_nnz > 0)
        HIPCHK(ctx, hipMemcpyAsync(val, c->ps_val, (size_t)c->ps_nnz * 4, hipMemcpyDeviceToDevice, st));
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
    if (!precision_ok(precision))
        return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
    TRY(set_device(ctx));
    Timer tm(ctx, "amp");
    return forward(ctx, sl, nv, theta, dets, n, precision, false, log_abs, sign, nullptr);
}

dnqs_status dnqs_amplitudes_noalloc(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta,
                                    const uint64_t *dets, int64_t n, int precision, double *log_abs, int8_t *sign) {
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    NetView nv;
    TRY(net_view(ctx, net, sl.M, sl.na, sl.nb, &nv));
    if (!theta || !dets || !log_abs || !sign) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (n < 1 || n >= (int64_t)1 << 31) return fail(ctx, DNQS_EINVAL, "n out of range");
    if (orb_lu_group(sl.na + sl.nb) == 0) return fail(ctx, DNQS_EINVAL, "N_e > 32 is not supported");
    if (!precision_ok(precision)) return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
    if (!ctx->scratch) return fail(ctx, DNQS_ESTATE, "no scratch region on this device");
    // the workspaces forward() takes without a gradient: h_1 .. h_{L-1}, the output layer,
    // and the BF16 weight planes of each split-BF16 GEMM, each rounded to 256 bytes
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t per_row = 0, fixed = 0;
    for (int l = 1; l <= nv.L; ++l) per_row += (size_t)nv.w[l] * sizeof(float);
    for (int l = 2; l <= nv.L; ++l)
        if (gemm_engine(precision, l == nv.L) == 1) fixed += al((size_t)nv.w[l - 1] * nv.w[l] * 2 * sizeof(uint16_t));
    size_t need = fixed;
    for (int l = 1; l <= nv.L; ++l) need += al((size_t)n * nv.w[l] * sizeof(float));
    if (need > kNoAllocScratch) {
        const long long maxn = fixed < kNoAllocScratch ? (long long)((kNoAllocScratch - fixed) / per_row) : 0;
        return fail(ctx, DNQS_ECAPACITY,
                    "%lld configurations need %zu bytes of scratch; the region holds %zu (at most about %lld "
                    "configurations of this network per call)",
                    (long long)n, need, kNoAllocScratch, maxn);
    }
    TRY(set_device(ctx));
    ctx->arena = (char *)ctx->scratch;
    ctx->arena_size = kNoAllocScratch;
    ctx->arena_used = 0;
    const dnqs_status st = forward(ctx, sl, nv, theta, dets, n, precision, false, log_abs, sign, nullptr);
    ctx->arena = nullptr;
    return st;
}

dnqs_status dnqs_energy_and_grad(dnqs_ctx *ctx, int slot, const dnqs_net *net, const float *theta,
                                 const dnqs_conn *conn, int precision, unsigned flags, double *energy,
                                 double *stats, float *grad, double *v_out, double *log_abs, int8_t *sign) {
    if (!ctx) return DNQS_EINVAL;
    if (flags & ~(DNQS_FULL_OUTPUT | DNQS_ASYM | DNQS_ASYM_ESTIMATOR | DNQS_RECOMPUTE))
        return fail(ctx, DNQS_EINVAL, "unknown flags 0x%x", flags);
    const bool asym = (flags & (DNQS_ASYM | DNQS_ASYM_ESTIMATOR)) != 0;
    if ((flags & DNQS_ASYM) && (flags & DNQS_ASYM_ESTIMATOR))
        return fail(ctx, DNQS_EINVAL, "DNQS_ASYM and DNQS_ASYM_ESTIMATOR exclude each other");
    if (asym && conn && conn->n_v <= 0)
        return fail(ctx, DNQS_EINVAL, "the Asymmetric objective needs a target set (dnqs_build_target)");
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    NetView nv;
    TRY(net_view(ctx, net, sl.M, sl.na, sl.nb, &nv));
    if (!theta || !conn || !energy || !stats) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (conn->M != sl.M || conn->na != sl.na || conn->nb != sl.nb)
        return fail(ctx, DNQS_EINVAL, "connections were built for another sector");
    if (orb_lu_group(sl.na + sl.nb) == 0) return fail(ctx, DNQS_EINVAL, "N_e > 32 is not supported");
    if (!precision_ok(precision))
        return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
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
    const bool full_out = (flags & DNQS_FULL_OUTPUT) != 0;
    // Activation recomputation: only h_{L-1} (read by the output layer's forward and
    // backward over all rows) is kept; h_1 .. h_{L-2} and U are formed by blocks of RB rows
    // in the forward pass and formed again by block in the backward pass.  RB is a multiple
    // of every hidden layer's weight-gradient split chunk (powers of two), so each block
    // writes whole split partials: the gradient equals the stored path's bit for bit.
    const bool recompute = (flags & DNQS_RECOMPUTE) && L >= 3;
    int64_t RB = n;
    int rc_chunk[DNQS_MAX_LAYERS + 1] = {};
    GemmCfg rc_cfg[DNQS_MAX_LAYERS + 1];
    if (recompute) {
        int64_t maxc = 256;
        for (int l = 1; l <= L - 1; ++l) {
            rc_cfg[l] = wgrad_cfg(ctx, gemm_engine(precision, false), w[l - 1] + 1, w[l], n);
            rc_chunk[l] = wgrad_chunk(n, rc_cfg[l].splits);
            maxc = std::max<int64_t>(maxc, rc_chunk[l]);
        }
        // about eight blocks, 16384 to 65536 rows each (a power of two)
        int64_t want = 16384;
        while (want < 65536 && want * 8 < n) want <<= 1;
        RB = std::max<int64_t>(want, maxc);
        float *hL1 = nullptr;
        TRY(ws_t(ctx, "h" + std::to_string(L - 1), (size_t)n * w[L - 1], &hL1));
        for (int64_t r0 = 0; r0 < n; r0 += RB) {
            float *hs[DNQS_MAX_LAYERS + 1] = {};
            TRY(hidden_block(ctx, sl, nv, theta, conn->dets + 2 * r0, std::min(RB, n - r0), precision, nullptr,
                             hL1 + r0 * w[L - 1], hs, L - 1));
        }
        TRY(forward(ctx, sl, nv, theta, conn->dets, n, precision, want_grad, la, sg, &Ainv,
                    full_out ? nullptr : conn, hL1));
    } else {
        TRY(forward(ctx, sl, nv, theta, conn->dets, n, precision, want_grad, la, sg, &Ainv,
                    full_out ? nullptr : conn));
    }
    double *psi = nullptr, *v = v_out, *part = nullptr, *part2 = nullptr;
    TRY(ws_t(ctx, "psi", (size_t)n, &psi));
    if (!v) TRY(ws_t(ctx, "v", (size_t)n, &v));
    TRY(ws_t(ctx, "red_part", (size_t)std::max<int64_t>(spmv_blocks(n), reduce_blocks(n)), &part));
    TRY(ws_t(ctx, "red_part2", (size_t)spmv_blocks(n), &part2));
    launch_scale_psi(st, la, sg, n, part, stats + 1, psi);
    CHECK_LAUNCH(ctx);
    if (asym) {
        double *u = nullptr, *up = nullptr;
        TRY(ws_t(ctx, "asym_u", (size_t)n, &u));
        TRY(ws_t(ctx, "asym_up", (size_t)n, &up));
        TRY(ws_t(ctx, "red_part3", (size_t)asym_blocks(n), &part2));
        double *part4 = nullptr;
        TRY(ws_t(ctx, "red_part4", (size_t)asym_blocks(n), &part4));
        launch_energy_asym(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, conn->n_v, u, up, part2,
                           part4, stats, energy, (flags & DNQS_ASYM_ESTIMATOR) ? 1 : 0, v);
    } else {
        launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, v, part, part2, stats,
                           energy);
    }
    CHECK_LAUNCH(ctx);
    if (!want_grad) return DNQS_OK;
    // adjoint: dO, then layer by layer
    float *dO = nullptr;
    const bool split = !full_out && conn->os_nd >= 0 && L >= 2 && os_fwd_fits(w[L - 1], Ne);
    const int nd = split ? conn->os_nd : 0, wd = nd * Ne;
    OutSplit og{};
    if (split) {
        // dO in the occupied-row layout only
        float *dOsp = nullptr, *dOD = nullptr;
        TRY(ws_t(ctx, "os_dOD", (size_t)n * std::max(wd, 1), &dOD));
        TRY(ws_t(ctx, "os_dOsp", (size_t)std::max<int64_t>(conn->os_ne, 1) * Ne, &dOsp));
        og.dOD = dOD;
        og.dOsp = dOsp;
        og.dpos = conn->os_dpos;
        og.dorb = conn->os_dorb;
        og.idx = conn->os_idx;
        og.nd = nd;
        launch_det_bwd(st, conn->dets, n, M, sl.na, sl.nb, psi, v, energy, stats, Ainv, nullptr, {}, og);
    } else {
        TRY(ws_t(ctx, "dO", (size_t)n * w[L], &dO));
        launch_det_bwd(st, conn->dets, n, M, sl.na, sl.nb, psi, v, energy, stats, Ainv, dO);
    }
    CHECK_LAUNCH(ctx);
    const size_t esz = sizeof(float);
    int maxw = 0;
    for (int l = 1; l < L; ++l) maxw = std::max(maxw, w[l]);
    void *dbuf[2];
    TRY(ws_get(ctx, "delta0", (size_t)n * maxw * esz, &dbuf[0]));
    TRY(ws_get(ctx, "delta1", recompute ? 1 : (size_t)n * maxw * esz, &dbuf[1]));
    const void *delta = dO;  // delta_l, starting at l = L
    int which = 0;
    // The weight gradient of layer l and the data gradient delta_{l-1} both read only
    // delta_l: the weight gradients run on the auxiliary stream, overlapping the chain of
    // data gradients.  A data gradient that overwrites a delta buffer waits for the weight
    // gradient that read it; the streams join before db_L is copied.  Not during capture.
    const bool fork = !ctx->capturing && L < 16 && !recompute;
    hipStream_t ast = st;
    if (fork) {
        if (!ctx->aux) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        for (int l = 1; l <= L; ++l) {
            if (!ctx->ev_ready[l]) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_ready[l], hipEventDisableTiming));
            if (!ctx->ev_wdone[l]) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_wdone[l], hipEventDisableTiming));
        }
        ast = ctx->aux;
    }
    for (int l = L; l >= 1; --l) {
        void *hp = nullptr;
        TRY(ws_get(ctx, l == 1 ? std::string("U") : "h" + std::to_string(l - 1), 1, &hp));
        const int din = w[l - 1], dout = w[l];
        const bool os_layer = l == L && split;
        const int eng = gemm_engine(precision, l == L);
        // ---- [h_{l-1}; 1]^T delta_l -> (dW_l, db_l), on the auxiliary stream
        if (fork) {
            HIPCHK(ctx, hipEventRecord(ctx->ev_ready[l], st));
            HIPCHK(ctx, hipStreamWaitEvent(ast, ctx->ev_ready[l], 0));
        }
        if (os_layer) {
            // occupied-row output layer: the dense columns by GEMM (scattered into place),
            // the sparse orbitals over their entries
            if (nd > 0) {
                float *GD = nullptr;
                TRY(ws_t(ctx, "os_GD", (size_t)(din + 1) * wd, &GD));
                GemmArgs g{};
                g.M = din + 1;
                g.N = wd;
                g.K = (int)n;
                g.A = hp;
                g.lda = din;
                g.B = og.dOD;
                g.ldb = wd;
                g.ldc = wd;
                g.ones_row = din;
                const int64_t cnt = (int64_t)(din + 1) * wd;
                TRY(tuned_launch(
                    ctx, TuneKey{eng, 1, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, true, false),
                    [&](const GemmCfg &c) -> dnqs_status {
                        const int chunk = wgrad_chunk(g.K, c.splits);
                        const int sp = (int)((g.K + chunk - 1) / chunk);
                        float *partial = nullptr;
                        TRY(ws_t(ctx, "splitk", (size_t)cnt * sp, &partial));
                        GemmArgs gs = g;
                        gs.C = partial;
                        gs.c_split_stride = cnt;
                        gs.k_chunk = chunk;
                        launch_gemm(eng, ast, gs, false, true, EPI_STORE, sp, c.tm);
                        CHECK_LAUNCH(ctx);
                        launch_reduce_splits(ast, partial, sp, cnt, GD);
                        CHECK_LAUNCH(ctx);
                        return DNQS_OK;
                    },
                    ast));
                launch_os_scatter(ast, GD, din, Ne, nd, dout, conn->os_dorb, grad + nv.offW[l]);
                CHECK_LAUNCH(ctx);
            }
            float *part_w = nullptr;
            TRY(ws_t(ctx, "os_wpart", (size_t)std::max<int64_t>(conn->os_nitems, 1) * (din + 1) * Ne, &part_w));
            launch_os_wgrad(ast, (const float *)hp, din, Ne, conn->os_items, conn->os_nitems, conn->os_ex, og.dOsp,
                            part_w, conn->os_dpos, conn->os_ifirst, conn->os_icount, No, grad + nv.offW[l]);
            CHECK_LAUNCH(ctx);
        } else {
            GemmArgs g{};
            g.M = din + 1;
            g.N = dout;
            g.K = (int)n;
            g.A = hp;
            g.lda = din;
            g.B = delta;
            g.ldb = dout;
            g.ldc = dout;
            g.ones_row = din;
            const int64_t cnt = (int64_t)(din + 1) * dout;
            TRY(tuned_launch(
                ctx, TuneKey{eng, 1, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, true, false),
                [&](const GemmCfg &c) -> dnqs_status {
                    const int chunk = wgrad_chunk(g.K, c.splits);
                    const int sp = (int)((g.K + chunk - 1) / chunk);
                    float *partial = nullptr;
                    TRY(ws_t(ctx, "splitk", (size_t)cnt * sp, &partial));
                    GemmArgs gs = g;
                    gs.C = partial;
                    gs.c_split_stride = cnt;
                    gs.k_chunk = chunk;
                    launch_gemm(eng, ast, gs, false, true, EPI_STORE, sp, c.tm);
                    CHECK_LAUNCH(ctx);
                    launch_reduce_splits(ast, partial, sp, cnt, grad + nv.offW[l]);
                    CHECK_LAUNCH(ctx);
                    return DNQS_OK;
                },
                ast));
        }
        if (fork) HIPCHK(ctx, hipEventRecord(ctx->ev_wdone[l], ast));
        if (l == 1) break;
        // ---- delta_{l-1} = (delta_l W_l^T) * (1 - h_{l-1}^2), on the context stream, into
        // the buffer that held delta_{l+1} (read by the weight gradient of layer l + 1)
        void *dnext = dbuf[which];
        which ^= 1;
        if (fork && l < L) HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_wdone[l + 1], 0));
        if (os_layer) {
            // occupied-row output layer: the dense columns by GEMM, the sparse rows by
            // orbital, summed per configuration in row order with tanh'
            float *dD = nullptr;
            if (nd > 0) {
                float *WD = nullptr;  // [W_D; b_D] from this call's forward
                TRY(ws_t(ctx, "os_WD", (size_t)(din + 1) * std::max(wd, 1), &WD));
                TRY(ws_t(ctx, "os_dD", (size_t)n * din, &dD));
                GemmArgs d{};
                d.M = (int)n;
                d.N = din;
                d.K = wd;
                d.A = og.dOD;
                d.lda = wd;
                d.B = WD;
                d.ldb = wd;
                d.C = dD;
                d.ldc = din;
                d.ones_row = -1;
                // K = n_d N_e is small (196 at the benchmark): the split-BF16 kernel's
                // two-step prefetch does not amortise over so few K steps, so this product
                // runs on the FP32 engine in every form (measured 0.22 against 0.36 ms)
                const int deng = wd < 256 ? 0 : eng;
                if (deng == 1) TRY(weight_planes(ctx, "wpO", WD, din, wd, false, d));
                TRY(tuned_launch(ctx, TuneKey{deng, 2, d.M, d.N, d.K}, gemm_candidates(d.M, d.N, d.K, false, false),
                                 [&](const GemmCfg &c) -> dnqs_status {
                                     launch_gemm(deng, st, d, true, false, EPI_STORE, 1, c.tm);
                                     CHECK_LAUNCH(ctx);
                                     return DNQS_OK;
                                 }));
            }
            float *WT = nullptr, *Cr = nullptr;
            TRY(ws_t(ctx, "os_WT", (size_t)din * dout, &WT));
            TRY(ws_t(ctx, "os_C", (size_t)std::max<int64_t>(conn->os_ne, 1) * din, &Cr));
            launch_os_trans_w(st, theta + nv.offW[l], din, dout, WT);
            launch_os_dgrad(st, n, Ne, din, WT, conn->os_tiles, conn->os_ntiles, og.dOsp, Cr, dD, conn->os_idx,
                            (const float *)hp, (float *)dnext);
            CHECK_LAUNCH(ctx);
        } else {
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
            d.act = hp;
            d.ldact = din;
            d.ones_row = -1;
            const int deng = gemm_engine(precision, l == L);
            if (deng == 1) TRY(weight_planes(ctx, "wp" + std::to_string(l), theta + nv.offW[l], din, dout, false, d));
            TRY(tuned_launch(ctx, TuneKey{deng, 2, d.M, d.N, d.K}, gemm_candidates(d.M, d.N, d.K, false, false),
                             [&](const GemmCfg &c) -> dnqs_status {
                                 launch_gemm(deng, st, d, true, false, EPI_DTANH, 1, c.tm);
                                 CHECK_LAUNCH(ctx);
                                 return DNQS_OK;
                             }));
        }
        delta = dnext;
        if (recompute) break;  // layers L-1 .. 1 by blocks of rows, below
    }
    if (recompute) TRY(backward_blocks(ctx, sl, nv, theta, conn->dets, n, precision, RB, rc_chunk, rc_cfg,
                                       (const float *)delta, maxw, grad));
    if (fork) HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_wdone[1], 0));  // join: every weight gradient is done
    // dPhi0 equals db_L (Phi0 and b_L enter A(x) the same way)
    launch_copy_f32(st, grad + nv.offb[L], grad + nv.offPhi0, (int64_t)No * Ne);
    CHECK_LAUNCH(ctx);
    return DNQS_OK;
}

dnqs_status dnqs_lanczos(dnqs_ctx *ctx, const dnqs_conn *conn, int max_iter, double tol, const double *start,
                         double *energy, double *vec, int *iters, double *residual) {
    if (!ctx) return DNQS_EINVAL;
    if (!conn || !energy) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (max_iter < 1 || max_iter > 4096) return fail(ctx, DNQS_EINVAL, "max_iter = %d, need 1..4096", max_iter);
    if (!(tol > 0.0)) return fail(ctx, DNQS_EINVAL, "tol must be positive");
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t n = conn->n;
    const int mmax = (int)std::min<int64_t>(max_iter, n);
    double *V = nullptr, *w = nullptr, *part = nullptr, *part2 = nullptr, *c = nullptr, *sc = nullptr;
    TRY(ws_t(ctx, "lz_V", (size_t)n * (mmax + 1), &V));
    TRY(ws_t(ctx, "lz_w", (size_t)n, &w));
    TRY(ws_t(ctx, "lz_part", (size_t)std::max<int64_t>({spmv_blocks(n), (int64_t)lanczos_dot_blocks() * (mmax + 1),
                                                       (int64_t)lanczos_norm_blocks(n)}), &part));
    TRY(ws_t(ctx, "lz_part2", (size_t)spmv_blocks(n), &part2));
    TRY(ws_t(ctx, "lz_c", 2 * ((size_t)mmax + 1), &c));
    TRY(ws_t(ctx, "lz_sc", 8, &sc));  // [0] norm, [1..3] spmv stats, [4] Rayleigh quotient
    if (start)
        launch_copy_f64(st, start, w, n);
    else
        launch_lz_start(st, conn->diag, n, sc, w);
    launch_lz_norm(st, w, n, part, sc);
    CHECK_LAUNCH(ctx);
    {
        double nrm = 0.0;
        HIPCHK(ctx, hipMemcpyAsync(&nrm, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return fail(ctx, DNQS_EDOMAIN, "lanczos: the start vector has norm %g", nrm);
    }
    launch_lz_scale(st, w, n, sc, V);
    CHECK_LAUNCH(ctx);
    std::vector<double> a, b, y;
    double lam = NAN, res = INFINITY;
    int m = 0;
    for (int j = 0; j < mmax; ++j) {
        double *vj = V + (int64_t)j * n;
        launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, vj, n, w, part, part2, sc + 1,
                           sc + 4);
        // two rounds of classical Gram-Schmidt against v_0 .. v_j (coefficients c, then
        // c2); alpha_j = c[j] + c2[j], beta_j = |w| after the second round
        double *c2 = c + (mmax + 1);
        launch_lz_dots(st, V, n, j + 1, w, n, part, c, false);
        launch_lz_orth(st, V, n, j + 1, c, w, n, part, sc);
        launch_lz_dots(st, V, n, j + 1, w, n, part, c2, false);
        launch_lz_orth(st, V, n, j + 1, c2, w, n, part, sc);
        CHECK_LAUNCH(ctx);
        double hc[3];
        HIPCHK(ctx, hipMemcpyAsync(hc, c + j, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(hc + 1, c2 + j, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipMemcpyAsync(hc + 2, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        hc[0] += hc[1];
        hc[1] = hc[2];
        a.push_back(hc[0]);
        m = j + 1;
        lam = tri_lowest(a, b, y);
        res = hc[1] * std::fabs(y[m - 1]);
        if (res <= tol * std::max(1.0, std::fabs(lam)) || hc[1] == 0.0 || m == mmax) break;
        b.push_back(hc[1]);
        launch_lz_scale(st, w, n, sc, V + (int64_t)(j + 1) * n);
        CHECK_LAUNCH(ctx);
    }
    double *yd = nullptr;
    TRY(ws_t(ctx, "lz_y", (size_t)m, &yd));
    HIPCHK(ctx, hipMemcpyAsync(yd, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    launch_set_f64(st, energy, lam);
    if (vec) launch_lz_combine(st, V, n, m, yd, n, vec);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (iters) *iters = m;
    if (residual) *residual = res;
    return DNQS_OK;
}

dnqs_status dnqs_heatbath_candidates(dnqs_ctx *ctx, int slot, const dnqs_conn *conn, const double *log_abs,
                                     const int8_t *sign, double eps_hb, int64_t cap, uint64_t *out_dets,
                                     int64_t *n_out) {
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    if (!conn || !log_abs || !sign || !n_out || (cap > 0 && !out_dets))
        return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (conn->M != sl.M || conn->na != sl.na || conn->nb != sl.nb)
        return fail(ctx, DNQS_EINVAL, "connections were built for another sector");
    if (!(eps_hb >= 0.0) || !std::isfinite(eps_hb)) return fail(ctx, DNQS_EINVAL, "eps_hb must be finite and >= 0");
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t n = conn->n;
    double *psi = nullptr, *v = nullptr, *part = nullptr, *part2 = nullptr, *stats = nullptr;
    TRY(ws_t(ctx, "hb_psi", (size_t)n, &psi));
    TRY(ws_t(ctx, "hb_v", (size_t)n, &v));
    TRY(ws_t(ctx, "hb_part", (size_t)std::max<int64_t>(spmv_blocks(n), reduce_blocks(n)), &part));
    TRY(ws_t(ctx, "hb_part2", (size_t)spmv_blocks(n), &part2));
    TRY(ws_t(ctx, "hb_stats", 4, &stats));
    launch_scale_psi(st, log_abs, sign, n, part, stats + 1, psi);
    launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, v, part, part2, stats, stats + 3);
    CHECK_LAUNCH(ctx);
    DetSet S{};
    TRY(s_hash_set(ctx, conn->dets, n, &S));
    uint64_t *pw = nullptr;
    int64_t np = 0;
    TRY(list_candidates(ctx, sl, conn->dets, n, S, psi, eps_hb, stats, &pw, &np));
    const int64_t k = std::min<int64_t>(np, std::max<int64_t>(cap, 0));
    if (k > 0) HIPCHK(ctx, hipMemcpyAsync(out_dets, pw, (size_t)k * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    *n_out = np;
    return DNQS_OK;
}

dnqs_status dnqs_select_topk(dnqs_ctx *ctx, int slot, const uint64_t *dets, const double *log_abs,
                             const int8_t *sign, int64_t n, int64_t K, uint64_t *out_dets, int64_t *n_out) {
    if (!ctx) return DNQS_EINVAL;
    TRY(check_slot(ctx, slot));
    const Slot &sl = ctx->slots[slot];
    if (!dets || !log_abs || !out_dets || !n_out) return fail(ctx, DNQS_EINVAL, "NULL pointer argument");
    if (n < 0 || n >= (int64_t)1 << 31 || K < 0) return fail(ctx, DNQS_EINVAL, "n or K out of range");
    TRY(set_device(ctx));
    hipStream_t st = ctx->stream;
    const int64_t k = std::min(n, K);
    *n_out = k;
    if (k == 0) return DNQS_OK;
    SortScratch w{};
    const size_t nc = sort_scratch_counts(n);
    int32_t *perm = nullptr;
    uint64_t *key = nullptr, *tmp = nullptr;
    TRY(ws_t(ctx, "sort_keys", (size_t)n, &w.keys));
    TRY(ws_t(ctx, "sort_vals", (size_t)n, &w.vals));
    TRY(ws_t(ctx, "sort_counts", nc, &w.counts));
    TRY(ws_t(ctx, "sort_offs", nc, &w.offs));
    TRY(ws_t(ctx, "sort_bsum", (size_t)scan_blocks((int64_t)nc) + 1, &w.bsum));
    TRY(ws_t(ctx, "sort_total", 1, &w.total));
    TRY(ws_t(ctx, "tk_perm", (size_t)n, &perm));
    TRY(ws_t(ctx, "tk_key", (size_t)n, &key));
    TRY(ws_t(ctx, "tk_tmp", (size_t)n * 2, &tmp));
    // canonical order first, then a stable sort by descending log|psi|: equal amplitudes
    // keep canonical order (ties go to the lower determinant)
    launch_sort_dets(st, dets, n, sl.M, perm, key, w);
    launch_topk_key(st, log_abs, sign, perm, n, key);
    launch_radix_sort(st, key, perm, n, 64, w);
    launch_permute_words(st, dets, perm, k, 2, tmp);
    // the selected k in canonical order
    launch_sort_dets(st, tmp, k, sl.M, perm, key, w);
    launch_permute_words(st, tmp, perm, k, 2, out_dets);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(st));
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
    if (!(o.eps_hb >= 0.0) || !std::isfinite(o.eps_hb)) return fail(ctx, DNQS_EINVAL, "eps_hb must be finite and >= 0");
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
    TRY(ws_t(ctx, "pt2_part", (size_t)std::max<int64_t>({spmv_blocks(n), 8 * 2048, (int64_t)pt2_accumulate_scratch()}),
             &part));
    TRY(ws_t(ctx, "pt2_part2", (size_t)spmv_blocks(n), &part2));
    TRY(ws_t(ctx, "pt2_stats", 4, &stats));
    TRY(ws_t(ctx, "pt2_etmp", 1, &e_tmp));
    launch_scale_psi(st, log_abs, sign, n, part, stats + 1, psi);
    launch_spmv_energy(st, conn->row_ptr, conn->col, conn->val, conn->diag, psi, n, v, part, part2, stats, e_tmp);
    CHECK_LAUNCH(ctx);
    {
        // the sums are divided by psi^T psi: no finite log_abs (every amplitude zero), or a
        // +inf or NaN one, leaves nothing to normalise
        double pp = 0.0;
        HIPCHK(ctx, hipMemcpyAsync(&pp, stats, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (!(pp > 0.0) || !std::isfinite(pp))
            return fail(ctx, DNQS_EDOMAIN, "pt2: psi^T psi = %g after scaling (log_abs has no finite maximum)", pp);
    }
    double *acc = nullptr;  // 8-double records: [internal | external total | current slice attempt]
    TRY(ws_t(ctx, "pt2_acc", 24, &acc));
    launch_pt2_init_acc(st, acc + 8);
    CHECK_LAUNCH(ctx);
    // internal terms, one per member of S, written by the reduce of the slice it hashes into
    double *int_term = nullptr;
    TRY(ws_t(ctx, "pt2_int_term", (size_t)n, &int_term));
    launch_fill_u64(st, (uint64_t *)int_term, n, 0ull);
    CHECK_LAUNCH(ctx);
    int *overflow = nullptr;
    TRY(ws_t(ctx, "pt2_ovf", 1, &overflow));
    PT2Export ex;
    ex.cap = o.export_cap;
    ex.keys = o.export_keys;
    ex.w = o.export_w;
    ex.haa = o.export_haa;
    ex.count = o.export_count;
    // h_pp and V(p, q) for the diagonal rule in the reduce (M <= 32)
    double *vt = nullptr;
    TRY(ws_t(ctx, "pt2_vt", (size_t)pt2_diag_table_size(sl.M), &vt));
    launch_diag_table(st, H, vt);
    // external sum: partitioned reduce-by-key (k_pt2_part.hip, k_pt2_reduce.hip)
    const int64_t nexc = n_excitations(sl.M, sl.na, sl.nb);
    const int64_t pairs = n * nexc;
    const bool packed = sl.M <= 32 && !(sl.M == 32 && sl.na == 32 && sl.nb == 32);
    uint64_t *rec = nullptr;
    TRY(ws_t(ctx, "pt2_rec", (size_t)4 * std::max<int64_t>(n, 1), &rec));
    launch_pt2_records(st, conn->dets, psi, n, packed, rec);
    CHECK_LAUNCH(ctx);
    // key-space slices: 8-byte descriptors are held twice (L1 and L2 order)
    int64_t budget = o.max_pair_bytes;
    if (budget <= 0) {
        size_t fr = 0, tot_mem = 0;
        HIPCHK(ctx, hipMemGetInfo(&fr, &tot_mem));
        int64_t held = 0;  // descriptor buffers of an earlier call are reused
        for (const char *nm : {"pt2_desc1", "pt2_desc2"}) {
            auto it = ctx->ws.find(nm);
            if (it != ctx->ws.end()) held += (int64_t)it->second.bytes;
        }
        budget = (int64_t)(fr / 2) + held;
    }
    int ss_mem = 0;
    while (ss_mem < 16 && (double)(pairs >> ss_mem) * 16.0 > (double)budget) ++ss_mem;
    int64_t nsb_used = 0;
    // The key space is cut into 2^ss slices when the descriptors of all pairs would not fit
    // the memory budget; a slice whose sub-buckets still overflow at the largest sub-bucket
    // count (few pairs per key: many keys per sub-bucket) restarts the whole sum with twice
    // as many slices, each slice then holding half the keys.
    for (int ss = ss_mem;; ++ss) {
        bool more_slices = false;
        launch_pt2_init_acc(st, acc + 8);
        if (o.export_cap > 0) HIPCHK(ctx, hipMemsetAsync(o.export_count, 0, sizeof(int64_t), st));
        nsb_used = 0;
        const int64_t slice_pairs = std::max<int64_t>(1, pairs >> ss);
        // sub-buckets of ~6000 pairs: ~1.8k unique keys at the 3.4 pairs per key of the
        // benchmark, 0.55 of the 3072-slot LDS table (fewer pairs per key: the overflow
        // retries below)
        const int64_t nsb_target = std::max<int64_t>(1, slice_pairs / 6000);
        int s1 = 0;
        // K1 <= 512: an L1 round of 8192 descriptors then holds ~16 per bucket (one 128-byte
        // line per run), and 2^19 sub-buckets leave K2 <= 1024 for the staged L2 pass
        while (((int64_t)1 << s1) < nsb_target && (1 << s1) < std::min(512, pt2_max_k1())) ++s1;
        int s2 = 0;
        while (((int64_t)1 << (s1 + s2)) < nsb_target && (1 << s2) < pt2_max_k2()) ++s2;
        const int K1 = 1 << s1;
        const int64_t nwg = pt2_l1_groups(n);
        uint32_t *c1 = nullptr;
        int32_t *c1t = nullptr;
        int64_t *offs1 = nullptr, *bsum = nullptr, *tot = nullptr, *bstart_d = nullptr, *ex_save = nullptr;
        TRY(ws_t(ctx, "pt2_c1", (size_t)nwg * K1, &c1));
        TRY(ws_t(ctx, "pt2_c1t", (size_t)nwg * K1, &c1t));
        TRY(ws_t(ctx, "pt2_offs1", (size_t)nwg * K1, &offs1));
        TRY(ws_t(ctx, "pt2_bsum", (size_t)scan_blocks(nwg * K1) + 1, &bsum));
        TRY(ws_t(ctx, "pt2_tot", 2, &tot));
        TRY(ws_t(ctx, "pt2_bstart", (size_t)K1 + 1, &bstart_d));
        TRY(ws_t(ctx, "pt2_exsave", 1, &ex_save));
        // L1 without a count pass when the L2 pass follows (s2 > 0): every bucket gets a region
        // of fixed capacity, the expected share of the slice's pairs plus a margin far above
        // the spread of a hash partition, and the fill appends each round's run at the
        // region's cursor.  The order of descriptors inside a bucket then depends on timing,
        // which no result does (every sum of the reduce is exact).  A region that would
        // overflow sends the slice through the counted pass instead.
        uint64_t *cur1_d = nullptr;
        int *ovf1_d = nullptr;
        TRY(ws_t(ctx, "pt2_cur1", (size_t)K1, &cur1_d));
        TRY(ws_t(ctx, "pt2_ovf1", 1, &ovf1_d));
        for (uint32_t slice = 0; slice < (1u << ss); ++slice) {
            Timer t1(ctx, "pt2_l1");
            uint64_t *desc1 = nullptr;
            int64_t total1 = 0, cap1 = 0;
            std::vector<int64_t> bstart(K1 + 1), bsize(K1);
            bool fused = false;
            if (s2 > 0) {
                cap1 = (int64_t)((double)slice_pairs / K1 * 1.03) + 65536;
                cap1 = (cap1 + 15) / 16 * 16;
                TRY(ws_t(ctx, "pt2_desc1", (size_t)K1 * cap1, &desc1));
                launch_fill_u64(st, cur1_d, (size_t)K1, 0ull);
                HIPCHK(ctx, hipMemsetAsync(ovf1_d, 0, sizeof(int), st));
                Timer t1f(ctx, "pt2_l1_fill");
                launch_pt2_l1(st, H, conn->dets, n, psi, s1, nwg, nullptr, nullptr, desc1, true, packed, ss, slice,
                              cur1_d, cap1, ovf1_d);
                CHECK_LAUNCH(ctx);
                t1f.stop();
                int ovf1 = 0;
                std::vector<uint64_t> cur1(K1);
                HIPCHK(ctx, hipMemcpyAsync(cur1.data(), cur1_d, sizeof(uint64_t) * K1, hipMemcpyDeviceToHost, st));
                HIPCHK(ctx, hipMemcpyAsync(&ovf1, ovf1_d, sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(ctx, hipStreamSynchronize(st));
                if (!ovf1) {
                    fused = true;
                    // bstart: the regions in desc1 (where the L2 chunks read); the device
                    // copy holds the compact starts instead, the bucket offsets in the L2
                    // pass's output, where k_sub_starts reads them
                    std::vector<int64_t> compact(K1 + 1, 0);
                    for (int b = 0; b < K1; ++b) {
                        bstart[b] = (int64_t)b * cap1;
                        bsize[b] = (int64_t)cur1[b];
                        compact[b + 1] = compact[b] + bsize[b];
                    }
                    total1 = compact[K1];
                    bstart[K1] = (int64_t)K1 * cap1;
                    HIPCHK(ctx, hipMemcpyAsync(bstart_d, compact.data(), sizeof(int64_t) * (K1 + 1),
                                               hipMemcpyHostToDevice, st));
                    HIPCHK(ctx, hipStreamSynchronize(st));
                }
            }
            if (!fused) {
                launch_pt2_l1(st, H, conn->dets, n, psi, s1, nwg, c1, nullptr, nullptr, false, packed, ss, slice);
                CHECK_LAUNCH(ctx);
                launch_transpose_u32(st, c1, nwg, K1, c1t);
                launch_exclusive_scan(st, c1t, nwg * K1, offs1, bsum, tot);
                CHECK_LAUNCH(ctx);
                HIPCHK(ctx, hipMemcpyAsync(&total1, tot, sizeof total1, hipMemcpyDeviceToHost, st));
                HIPCHK(ctx, hipStreamSynchronize(st));
                TRY(ws_t(ctx, "pt2_desc1", (size_t)std::max<int64_t>(total1, 1), &desc1));
                Timer t1f(ctx, "pt2_l1_fill");
                launch_pt2_l1(st, H, conn->dets, n, psi, s1, nwg, nullptr, offs1, desc1, true, packed, ss, slice);
                CHECK_LAUNCH(ctx);
                t1f.stop();
                launch_gather_starts(st, offs1, K1, nwg, tot, bstart_d);
                CHECK_LAUNCH(ctx);
                HIPCHK(ctx, hipMemcpyAsync(bstart.data(), bstart_d, sizeof(int64_t) * (K1 + 1), hipMemcpyDeviceToHost,
                                           st));
                HIPCHK(ctx, hipStreamSynchronize(st));
                for (int b = 0; b < K1; ++b) bsize[b] = bstart[b + 1] - bstart[b];
            }
            t1.stop();
            if (o.export_cap > 0)
                HIPCHK(ctx, hipMemcpyAsync(ex_save, o.export_count, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
            HIPCHK(ctx, hipStreamSynchronize(st));
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
                        const int64_t size = bsize[b];
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
                        HIPCHK(ctx, hipMemcpyAsync(chunks_d, chunks.data(), sizeof(PT2Chunk) * nchunk,
                                                   hipMemcpyHostToDevice, st));
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
                // the members of S in this slice, grouped by sub-bucket (same hash bits as the pairs)
                int32_t *scnt = nullptr;
                int64_t *soffs = nullptr, *sbsum = nullptr;
                uint64_t *skeys = nullptr;
                int32_t *sidx = nullptr;
                TRY(ws_t(ctx, "pt2_sidx", (size_t)std::max<int64_t>(n, 1), &sidx));
                TRY(ws_t(ctx, "pt2_scnt", (size_t)nsb, &scnt));
                TRY(ws_t(ctx, "pt2_soffs", (size_t)nsb, &soffs));
                TRY(ws_t(ctx, "pt2_sbsum", (size_t)scan_blocks(nsb) + 1, &sbsum));
                TRY(ws_t(ctx, "pt2_skeys", (size_t)2 * std::max<int64_t>(n, 1), &skeys));
                const int sbits = s1 + (s2 > 0 ? s2 : 0);
                HIPCHK(ctx, hipMemsetAsync(scnt, 0, sizeof(int32_t) * nsb, st));
                launch_s_sub(st, conn->dets, n, sbits, packed, scnt, nullptr, nullptr, nullptr, false, ss, slice);
                CHECK_LAUNCH(ctx);
                launch_exclusive_scan(st, scnt, nsb, soffs, sbsum, tot + 1);
                CHECK_LAUNCH(ctx);
                int64_t n_s = 0;  // members of S in this slice
                HIPCHK(ctx, hipMemcpyAsync(&n_s, tot + 1, sizeof n_s, hipMemcpyDeviceToHost, st));
                HIPCHK(ctx, hipMemsetAsync(scnt, 0, sizeof(int32_t) * nsb, st));
                launch_s_sub(st, conn->dets, n, sbits, packed, scnt, soffs, skeys, sidx, true, ss, slice);
                CHECK_LAUNCH(ctx);
                HIPCHK(ctx, hipStreamSynchronize(st));
                // Few pairs per key leave many keys per sub-bucket: count the keys of 1024
                // sampled sub-buckets first, and cut the key space finer before the reduce
                // if the fullest sample comes near the tables' fill limit: more sub-buckets,
                // or, at the largest sub-bucket count, more key-space slices (the reduce's
                // own overflow retry still covers an unsampled sub-bucket).
                if (s2 > 0) {
                    int *maxk = nullptr;
                    TRY(ws_t(ctx, "pt2_maxk", 1, &maxk));
                    HIPCHK(ctx, hipMemsetAsync(maxk, 0, sizeof(int), st));
                    launch_pt2_keycount(st, rec, desc, sb, nsb, 1024, skeys, soffs, n_s, maxk, packed);
                    CHECK_LAUNCH(ctx);
                    int mk = 0;
                    HIPCHK(ctx, hipMemcpyAsync(&mk, maxk, sizeof(int), hipMemcpyDeviceToHost, st));
                    HIPCHK(ctx, hipStreamSynchronize(st));
                    if (mk > pt2_red_fill_max() / 10 * 9) {
                        if ((1 << s2) < pt2_max_k2()) {
                            ++s2;
                            continue;
                        }
                        more_slices = true;
                        break;
                    }
                }
                double *part_r = nullptr;
                TRY(ws_t(ctx, "pt2_part_r", (size_t)nsb * pt2_red_part(), &part_r));
                launch_pt2_init_acc(st, acc + 16);
                if (o.export_cap > 0)
                    HIPCHK(ctx, hipMemcpyAsync(o.export_count, ex_save, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
                HIPCHK(ctx, hipMemsetAsync(overflow, 0, sizeof(int), st));
                Timer tr(ctx, "pt2_reduce");
                launch_pt2_reduce(st, H, rec, desc, sb, nsb, skeys, sidx, soffs, n_s, vt, energy, o.sample_mask,
                                  sl.wexp, o.eps_hb, stats, ex, part_r, int_term, overflow, packed);
                CHECK_LAUNCH(ctx);
                tr.stop();
                launch_pt2_accumulate(st, part_r, nsb, acc + 16, part);
                CHECK_LAUNCH(ctx);
                int ov = 0;
                HIPCHK(ctx, hipMemcpyAsync(&ov, overflow, sizeof ov, hipMemcpyDeviceToHost, st));
                HIPCHK(ctx, hipStreamSynchronize(st));
                if (!ov) {
                    launch_pt2_merge(st, acc + 8, acc + 16);
                    CHECK_LAUNCH(ctx);
                    nsb_used += nsb;
                    break;
                }
                if ((1 << s2) >= pt2_max_k2() || attempt > 8) {
                    more_slices = true;
                    break;
                }
                ++s2;
            }
            if (more_slices) break;
        }
        if (!more_slices) break;
        if (ss >= 20)
            return fail(ctx, DNQS_ECAPACITY, "PT2: a sub-bucket holds more than %d unique keys", pt2_red_tab());
    }
    launch_pt2_internal(st, int_term, conn->diag, n, energy, part, acc);
    CHECK_LAUNCH(ctx);
    launch_pt2_final(st, acc, acc + 8, stats, out, counts, pairs, nsb_used);
    CHECK_LAUNCH(ctx);
    tm.stop();
    if (o.export_cap > 0) TRY(pt2_export_sort(ctx, sl.M, o));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return DNQS_OK;
}

namespace {

void plan_free(dnqs_ctx *ctx, BatchPlan &b) {
    for (void *q : {(void *)b.dets, (void *)b.pid, (void *)b.row_ptr, (void *)b.col, (void *)b.val, (void *)b.diag,
                    (void *)b.tile_pid, (void *)b.ksplit, (void *)b.zrange, (void *)b.P_d, (void *)b.ptr_d,
                    (void *)b.items, (void *)b.ipart})
        dev_free(ctx->alloc, q);
    b = BatchPlan();
}

// rows of weight-gradient split-K per work item
constexpr int64_t kSplitRows = 4096;

// rows per work item of the per-problem reductions
constexpr int64_t kItemRows = 4096;

dnqs_status plan_build(dnqs_ctx *ctx, int G, const dnqs_problem *pr) {
    BatchPlan &b = ctx->plan;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    plan_free(ctx, b);
    b.G = G;
    // largest problem first in the concatenated layout, so that the work of every launch
    // over all problems (GEMM tiles, split-K ranges, reduction items) is ordered largest-first
    std::vector<int> order(G);
    for (int g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return pr[x].conn->n > pr[y].conn->n; });
    b.off.assign(G, 0);
    b.end.assign(G, 0);
    b.nn.assign(G, 0);
    int64_t off = 0, nnz = 0;
    for (int g = 0; g < G; ++g) {
        b.conns.push_back(pr[g].conn);
        b.nn[g] = pr[g].conn->n;
        nnz += pr[g].conn->nnz;
    }
    for (int g : order) {
        b.off[g] = off;
        off += (pr[g].conn->n + 127) / 128 * 128;
        b.end[g] = off;
    }
    b.ntot = off;
    b.nnz = nnz;
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.dets, (size_t)b.ntot * 16));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.pid, (size_t)b.ntot * 4));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.row_ptr, (size_t)(b.ntot + 1) * 8));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.col, (size_t)std::max<int64_t>(nnz, 1) * 4));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.val, (size_t)std::max<int64_t>(nnz, 1) * 4));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.diag, (size_t)b.ntot * 8));
    int64_t nnz_off = 0;
    for (int g : order) {
        const dnqs_conn *c = pr[g].conn;
        launch_cat_problem(ctx->stream, g, b.off[g], c->n, b.end[g], c->dets, c->row_ptr, c->col, c->val, c->diag,
                           c->nnz, nnz_off, b.dets, b.pid, b.row_ptr, b.col, b.val, b.diag);
        CHECK_LAUNCH(ctx);
        nnz_off += c->nnz;
    }
    launch_set_i64(ctx->stream, b.row_ptr + b.ntot, nnz);
    // tile -> problem, split-K ranges (layout order), reduction items (layout order)
    std::vector<int> tp(b.ntot / 128);
    for (int g = 0; g < G; ++g)
        for (int64_t t = b.off[g] / 128; t < b.end[g] / 128; ++t) tp[t] = g;
    std::vector<int2> ks, zr(G);
    std::vector<int4> it;
    for (int g : order) {
        const int z0 = (int)ks.size();
        for (int64_t r = 0; r < b.nn[g]; r += kSplitRows)
            ks.push_back(make_int2((int)(b.off[g] + r), (int)(b.off[g] + std::min(b.nn[g], r + kSplitRows))));
        zr[g] = make_int2(z0, (int)ks.size());
        for (int64_t r = 0; r < b.nn[g]; r += kItemRows)
            it.push_back(make_int4(g, (int)(b.off[g] + r), (int)std::min(kItemRows, b.nn[g] - r), 0));
    }
    b.nz = (int)ks.size();
    b.nitems = (int)it.size();
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.tile_pid, tp.size() * sizeof(int)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.ksplit, std::max<size_t>(ks.size(), 1) * sizeof(int2)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.zrange, zr.size() * sizeof(int2)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.items, std::max<size_t>(it.size(), 1) * sizeof(int4)));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.ipart, std::max<size_t>(it.size(), 1) * 2 * sizeof(double)));
    HIPCHK(ctx, hipMemcpyAsync(b.tile_pid, tp.data(), tp.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    if (!ks.empty())
        HIPCHK(ctx, hipMemcpyAsync(b.ksplit, ks.data(), ks.size() * sizeof(int2), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(b.zrange, zr.data(), zr.size() * sizeof(int2), hipMemcpyHostToDevice, ctx->stream));
    if (!it.empty())
        HIPCHK(ctx, hipMemcpyAsync(b.items, it.data(), it.size() * sizeof(int4), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.P_d, (size_t)G * sizeof(ProbDev)));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    b.valid = true;
    return DNQS_OK;
}

// refresh the device tables of per-problem pointers if they changed
dnqs_status plan_pointers(dnqs_ctx *ctx, const NetView &nv, int G, const dnqs_problem *pr) {
    BatchPlan &b = ctx->plan;
    std::vector<ProbDev> P(G);
    for (int g = 0; g < G; ++g) P[g] = {pr[g].theta, pr[g].grad, pr[g].energy, pr[g].stats, b.off[g], b.nn[g]};
    std::vector<const void *> ptr;
    for (int l = 0; l <= nv.L; ++l)
        for (int g = 0; g < G; ++g) ptr.push_back(l == 0 ? nullptr : (const void *)(pr[g].theta + nv.offW[l]));
    for (int l = 0; l <= nv.L; ++l)
        for (int g = 0; g < G; ++g) ptr.push_back(l == 0 ? nullptr : (const void *)(pr[g].theta + nv.offb[l]));
    bool same = b.P_h.size() == P.size() && b.ptr_h == ptr && b.ptr_layers == nv.L;
    for (int g = 0; same && g < G; ++g)
        same = !std::memcmp(&b.P_h[g], &P[g], sizeof(ProbDev));
    if (same) return DNQS_OK;
    if (ctx->capturing) return fail(ctx, DNQS_ESTATE, "batched pointers changed during graph capture");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx->alloc, b.ptr_d);
    b.ptr_d = nullptr;
    b.ptr_d = nullptr;
    HIPCHK(ctx, dev_alloc(ctx->alloc, (void **)&b.ptr_d, ptr.size() * sizeof(void *)));
    b.P_h = P;
    b.ptr_h = ptr;
    b.ptr_layers = nv.L;
    HIPCHK(ctx, hipMemcpyAsync(b.P_d, b.P_h.data(), G * sizeof(ProbDev), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(b.ptr_d, b.ptr_h.data(), ptr.size() * sizeof(void *), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return DNQS_OK;
}

}  // namespace

dnqs_status dnqs_energy_and_grad_batched(dnqs_ctx *ctx, const dnqs_net *net, int G, const dnqs_problem *pr,
                                         int precision, unsigned flags) {
    (void)flags;
    if (!ctx) return DNQS_EINVAL;
    if (!pr || G < 1 || G > DNQS_MAX_SLOTS) return fail(ctx, DNQS_EINVAL, "n_problems = %d out of range", G);
    if (!precision_ok(precision))
        return fail(ctx, DNQS_EINVAL, "precision %d not supported", precision);
    TRY(check_slot(ctx, pr[0].slot));
    const Slot &s0 = ctx->slots[pr[0].slot];
    NetView nv;
    TRY(net_view(ctx, net, s0.M, s0.na, s0.nb, &nv));
    const bool want_grad = pr[0].grad != nullptr;
    for (int g = 0; g < G; ++g) {
        TRY(check_slot(ctx, pr[g].slot));
        const Slot &sg = ctx->slots[pr[g].slot];
        if (!pr[g].conn || !pr[g].theta || !pr[g].energy || !pr[g].stats)
            return fail(ctx, DNQS_EINVAL, "problem %d: NULL pointer", g);
        if (sg.M != s0.M || sg.na != s0.na || sg.nb != s0.nb || pr[g].conn->M != s0.M || pr[g].conn->na != s0.na ||
            pr[g].conn->nb != s0.nb)
            return fail(ctx, DNQS_EINVAL, "problem %d: sector differs from problem 0", g);
        if ((pr[g].grad != nullptr) != want_grad) return fail(ctx, DNQS_EINVAL, "grad must be given for all or none");
    }
    if (orb_lu_group(s0.na + s0.nb) == 0) return fail(ctx, DNQS_EINVAL, "N_e > 32 is not supported");
    TRY(set_device(ctx));
    BatchPlan &b = ctx->plan;
    bool same = b.valid && b.G == G;
    for (int g = 0; same && g < G; ++g) same = b.conns[g] == pr[g].conn && b.nn[g] == pr[g].conn->n;
    if (!same) {
        if (ctx->capturing) return fail(ctx, DNQS_ESTATE, "a new batch cannot be planned during graph capture");
        TRY(plan_build(ctx, G, pr));
    }
    TRY(plan_pointers(ctx, nv, G, pr));
    hipStream_t st = ctx->stream;
    Timer tm(ctx, "egrad_batched");
    const size_t esz = sizeof(float);
    const int M = s0.M, No = 2 * M, Ne = s0.na + s0.nb, L = nv.L;
    const int *w = nv.w;
    const int64_t n = b.ntot;
    const RowProblems rp{b.pid, b.P_d};
    auto Wg = [&](int l) { return (const void *const *)(b.ptr_d + (size_t)l * G); };
    auto bg = [&](int l) { return (const float *const *)(b.ptr_d + (size_t)(L + 1 + l) * G); };
    // ---- forward
    void *U = nullptr, *h = nullptr;
    if (want_grad) TRY(ws_get(ctx, "bU", (size_t)n * No * esz, &U));
    TRY(ws_get(ctx, "bh1", (size_t)n * w[1] * esz, &h));
    launch_embed(st, b.dets, n, M, w[1], nullptr, nullptr, (float *)h, (float *)U, rp, nv.offW[1], nv.offb[1]);
    CHECK_LAUNCH(ctx);
    void *prev = h;
    for (int l = 2; l <= L; ++l) {
        void *out = nullptr;
        if (l < L)
            TRY(ws_get(ctx, "bh" + std::to_string(l), (size_t)n * w[l] * esz, &out));
        else
            TRY(ws_get(ctx, "bO", (size_t)n * w[l] * sizeof(float), &out));
        GemmArgs g{};
        g.M = (int)n;
        g.N = w[l];
        g.K = w[l - 1];
        g.A = prev;
        g.lda = w[l - 1];
        g.ldb = w[l];
        g.C = out;
        g.ldc = w[l];
        g.ones_row = -1;
        g.tile_pid = b.tile_pid;
        g.Bg = Wg(l);
        g.biasg = bg(l);
        const int eng = gemm_engine(precision, l == L);
        const int epi = l < L ? EPI_BIAS_TANH : EPI_BIAS;
        TRY(tuned_launch(ctx, TuneKey{eng, 0, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, false, false),
                         [&](const GemmCfg &c) -> dnqs_status {
                             launch_gemm(eng, st, g, true, true, epi, 1, c.tm);
                             CHECK_LAUNCH(ctx);
                             return DNQS_OK;
                         }));
        prev = out;
    }
    double *la = nullptr, *psi = nullptr, *v = nullptr, *pv = nullptr, *pp = nullptr;
    int8_t *sg = nullptr;
    float *Ainv = nullptr;
    TRY(ws_t(ctx, "b_la", (size_t)n, &la));
    TRY(ws_t(ctx, "b_sg", (size_t)n, &sg));
    TRY(ws_t(ctx, "b_psi", (size_t)n, &psi));
    TRY(ws_t(ctx, "b_v", (size_t)n, &v));
    TRY(ws_t(ctx, "b_pv", (size_t)n, &pv));
    TRY(ws_t(ctx, "b_pp", (size_t)n, &pp));
    if (want_grad) TRY(ws_t(ctx, "b_Ainv", (size_t)n * Ne * Ne, &Ainv));
    launch_orb_lu(st, b.dets, n, M, s0.na, s0.nb, (const float *)prev, nullptr, la, sg, Ainv, rp, nv.offPhi0);
    CHECK_LAUNCH(ctx);
    launch_energy_grouped(st, la, sg, n, G, rp, b.row_ptr, b.col, b.val, b.diag, psi, v, pv, pp, b.items, b.nitems,
                          b.ipart);
    CHECK_LAUNCH(ctx);
    if (!want_grad) return DNQS_OK;
    // ---- adjoint
    float *dO = nullptr;
    TRY(ws_t(ctx, "b_dO", (size_t)n * w[L], &dO));
    launch_det_bwd(st, b.dets, n, M, s0.na, s0.nb, psi, v, nullptr, nullptr, Ainv, dO, rp);
    CHECK_LAUNCH(ctx);
    int maxw = 0;
    for (int l = 1; l < L; ++l) maxw = std::max(maxw, w[l]);
    void *dbuf[2];
    TRY(ws_get(ctx, "b_delta0", (size_t)n * maxw * esz, &dbuf[0]));
    TRY(ws_get(ctx, "b_delta1", (size_t)n * maxw * esz, &dbuf[1]));
    const void *delta = dO;
    int which = 0;
    for (int l = L; l >= 1; --l) {
        void *hp = nullptr;
        TRY(ws_get(ctx, l == 1 ? std::string("bU") : "bh" + std::to_string(l - 1), 1, &hp));
        const int din = w[l - 1], dout = w[l];
        GemmArgs g{};
        g.M = din + 1;
        g.N = dout;
        g.K = (int)n;
        g.A = hp;
        g.lda = din;
        g.B = delta;
        g.ldb = dout;
        g.ldc = dout;
        g.ones_row = din;
        g.ksplit = b.ksplit;
        float *partial = nullptr;
        const int64_t cnt = (int64_t)(din + 1) * dout;
        TRY(ws_t(ctx, "b_splitk", (size_t)cnt * b.nz, &partial));
        g.C = partial;
        g.c_split_stride = cnt;
        const int eng = gemm_engine(precision, l == L);
        TRY(tuned_launch(ctx, TuneKey{eng, 3, g.M, g.N, g.K}, gemm_candidates(g.M, g.N, g.K, true, true),
                         [&](const GemmCfg &c) -> dnqs_status {
                             launch_gemm(eng, st, g, false, true, EPI_STORE, b.nz, c.tm);
                             CHECK_LAUNCH(ctx);
                             launch_reduce_splits_grouped(st, partial, b.zrange, cnt, G, b.P_d, nv.offW[l]);
                             CHECK_LAUNCH(ctx);
                             return DNQS_OK;
                         }));
        if (l == 1) break;
        void *dnext = dbuf[which];
        which ^= 1;
        GemmArgs d{};
        d.M = (int)n;
        d.N = din;
        d.K = dout;
        d.A = delta;
        d.lda = dout;
        d.ldb = dout;
        d.C = dnext;
        d.ldc = din;
        d.act = hp;
        d.ldact = din;
        d.ones_row = -1;
        d.tile_pid = b.tile_pid;
        d.Bg = Wg(l);
        const int deng = gemm_engine(precision, l == L);
        TRY(tuned_launch(ctx, TuneKey{deng, 2, d.M, d.N, d.K}, gemm_candidates(d.M, d.N, d.K, false, false),
                         [&](const GemmCfg &c) -> dnqs_status {
                             launch_gemm(deng, st, d, true, false, EPI_DTANH, 1, c.tm);
                             CHECK_LAUNCH(ctx);
                             return DNQS_OK;
                         }));
        delta = dnext;
    }
    launch_copy_grouped(st, b.P_d, G, nv.offb[L], nv.offPhi0, (int64_t)No * Ne);
    CHECK_LAUNCH(ctx);
    return DNQS_OK;
}

dnqs_status dnqs_adamw_batched(dnqs_ctx *ctx, const dnqs_net *net, int G, const dnqs_problem *pr, float *m, float *v,
                               const dnqs_adamw_cfg *cfg, int *step) {
    if (!ctx) return DNQS_EINVAL;
    if (!pr || G < 1 || G > DNQS_MAX_SLOTS || !m || !v || !cfg || !step)
        return fail(ctx, DNQS_EINVAL, "bad argument");
    if (cfg->decay_steps < 1 || !(cfg->eps > 0.0f)) return fail(ctx, DNQS_EINVAL, "bad AdamW configuration");
    TRY(check_slot(ctx, pr[0].slot));
    const Slot &s0 = ctx->slots[pr[0].slot];
    NetView nv;
    TRY(net_view(ctx, net, s0.M, s0.na, s0.nb, &nv));
    BatchPlan &b = ctx->plan;
    bool same = b.valid && b.G == G;
    for (int g = 0; same && g < G; ++g) same = b.conns[g] == pr[g].conn;
    if (!same) return fail(ctx, DNQS_ESTATE, "call dnqs_energy_and_grad_batched with these problems first");
    for (int g = 0; g < G; ++g)
        if (!pr[g].grad || !pr[g].theta) return fail(ctx, DNQS_EINVAL, "problem %d: theta and grad needed", g);
    TRY(set_device(ctx));
    TRY(plan_pointers(ctx, nv, G, pr));
    AdamCfg c{cfg->lr_max, cfg->lr_min, cfg->decay_steps, cfg->beta1, cfg->beta2, cfg->eps, cfg->weight_decay};
    launch_adamw_grouped(ctx->stream, b.P_d, G, m, v, nv.total, c, step);
    CHECK_LAUNCH(ctx);
    return DNQS_OK;
}

dnqs_status dnqs_autotune(dnqs_ctx *ctx, int enable) {
    if (!ctx) return DNQS_EINVAL;
    ctx->autotune = enable != 0;
    return DNQS_OK;
}

int64_t dnqs_tune_export(const dnqs_ctx *ctx, char *buf, int64_t cap) {
    if (!ctx) return -1;
    std::string out;
    char line[128];
    for (const auto &kv : ctx->tuned) {
        const TuneKey &k = kv.first;
        std::snprintf(line, sizeof line, "%d %d %d %d %d %d %d\n", k.engine, k.kind, k.M, k.N, k.K, kv.second.tm,
                      kv.second.splits);
        out += line;
    }
    if (buf && cap > 0) {
        const int64_t m = std::min<int64_t>(cap - 1, (int64_t)out.size());
        std::memcpy(buf, out.data(), (size_t)m);
        buf[m] = 0;
    }
    return (int64_t)out.size();
}

dnqs_status dnqs_tune_import(dnqs_ctx *ctx, const char *text) {
    if (!ctx) return DNQS_EINVAL;
    if (!text) return fail(ctx, DNQS_EINVAL, "text is NULL");
    std::map<TuneKey, GemmCfg> add;
    const char *p = text;
    int lineno = 0;
    while (*p) {
        const char *e = std::strchr(p, '\n');
        const std::string line = e ? std::string(p, e) : std::string(p);
        p = e ? e + 1 : p + line.size();
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k;
        GemmCfg c;
        char extra = 0;
        if (std::sscanf(line.c_str(), "%d %d %d %d %d %d %d %c", &k.engine, &k.kind, &k.M, &k.N, &k.K, &c.tm,
                        &c.splits, &extra) != 7)
            return fail(ctx, DNQS_EINVAL, "tune table line %d: expected 7 integers", lineno);
        const bool ok = (k.engine == 0 || k.engine == 1) && k.kind >= 0 && k.kind <= 3 && k.M > 0 && k.N > 0 &&
                        k.K > 0 && (c.tm == 64 || c.tm == 128) &&
                        (k.kind == 3 ? c.splits == 0 : (k.kind == 1 ? c.splits >= 1 && c.splits <= 256 : c.splits == 1));
        if (!ok) return fail(ctx, DNQS_EINVAL, "tune table line %d: value out of range", lineno);
        add[k] = c;
    }
    for (const auto &kv : add) ctx->tuned[kv.first] = kv.second;
    return DNQS_OK;
}

dnqs_status dnqs_capture_begin(dnqs_ctx *ctx) {
    if (!ctx) return DNQS_EINVAL;
    if (!ctx->stream) return fail(ctx, DNQS_ESTATE, "graph capture needs a non-null stream");
    if (ctx->capturing) return fail(ctx, DNQS_ESTATE, "already capturing");
    TRY(set_device(ctx));
    HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    return DNQS_OK;
}

dnqs_status dnqs_capture_end(dnqs_ctx *ctx, dnqs_graph **out) {
    if (!ctx) return DNQS_EINVAL;
    if (!out) return fail(ctx, DNQS_EINVAL, "out is NULL");
    if (!ctx->capturing) return fail(ctx, DNQS_ESTATE, "not capturing");
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    HIPCHK(ctx, hipStreamEndCapture(ctx->stream, &g));
    dnqs_graph *dg = new dnqs_graph();
    dg->graph = g;
    dg->device = ctx->device;
    hipError_t e = hipGraphInstantiate(&dg->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete dg;
        return fail(ctx, DNQS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = dg;
    return DNQS_OK;
}

dnqs_status dnqs_graph_launch(dnqs_ctx *ctx, dnqs_graph *graph) {
    if (!ctx) return DNQS_EINVAL;
    if (!graph) return fail(ctx, DNQS_EINVAL, "graph is NULL");
    TRY(set_device(ctx));
    HIPCHK(ctx, hipGraphLaunch(graph->exec, ctx->stream));
    return DNQS_OK;
}

void dnqs_graph_free(dnqs_graph *graph) {
    if (!graph) return;
    (void)hipSetDevice(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
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
