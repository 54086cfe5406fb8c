// cm_api.hip -- the C ABI (include/cm.h): argument validation, model weight
// packing, workspace allocation and kernel dispatch.  No device work is
// queued before every argument has been checked.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "cm_internal.h"

struct cm_workspace {
    cm::Workspace w;
};

namespace {
thread_local std::string g_err;
}  // namespace

namespace cm {

cm_status fail(cm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

cm_status check_query_bytes(int64_t q, int64_t S, int64_t N, cm_precision prec, bool table)
{
    if (prec == CM_FP32) return CM_OK;
    const int64_t rows = S * N;  // S, N < 2^31: no overflow
    const int64_t fb = prec == CM_FP8 ? FS : 2 * FS;
    if (!table && rows * fb > MAX_QUERY_BYTES)
        return fail(CM_E2BIG,
                    "query %lld: %lld x %lld rows of schedule features are %lld bytes, above "
                    "the evaluator's %lld per query",
                    (long long)q, (long long)S, (long long)N, (long long)(rows * fb),
                    (long long)MAX_QUERY_BYTES);
    if (rows * C * 4 > MAX_QUERY_BYTES)
        return fail(CM_E2BIG,
                    "query %lld: %lld x %lld rows of cost terms are %lld bytes, above the "
                    "evaluator's %lld per query",
                    (long long)q, (long long)S, (long long)N, (long long)(rows * C * 4),
                    (long long)MAX_QUERY_BYTES);
    return CM_OK;
}

}  // namespace cm

namespace {

using cm::fail;

// Scratch of cm_eval_batch_static: the hoisted rows U[stages][32] of one
// call, in a file-scope device array.  Every device the library runs on
// holds its own copy until the process ends; calls on one device share it.
__device__ __align__(256) float scratch[(size_t)CM_STATIC_MAX_STAGES * cm::H];

// Device address of `scratch` on each device, looked up once per device with
// that device current (in host code the array's name is not a device
// address).
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[SCRATCH_DEVICES] = {};

cm_status static_scratch(int dev, float **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= SCRATCH_DEVICES)
        return fail(CM_EUNSUPPORTED, "device %d is beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(CM_EDEVICE, "address of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CM_OK;
}

uint16_t f32_to_bf16(float f)  // round to nearest even
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// hi + lo bf16 pair of a double value
void split_bf16(double w, uint16_t &hi, uint16_t &lo)
{
    hi = f32_to_bf16((float)w);
    lo = f32_to_bf16((float)(w - (double)bf16_to_f32(hi)));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// OCP e4m3 code of v: round to nearest with ties to the even code, saturate
// at +-448, NaN -> 0x7F.  The quantum of |v| is 2^(floor(log2 |v|) - 3) in the
// normal range and 2^-9 below 2^-6; the rounded multiple n of the quantum
// gives the code directly (n <= 8 below 2^-6: the code is n; above: the
// exponent field is the binade + 7 and the mantissa field n - 8).
uint8_t e4m3_code(double v)
{
    if (std::isnan(v)) return 0x7F;
    const uint8_t sign = std::signbit(v) ? 0x80 : 0x00;
    double a = std::fabs(v);
    if (a >= 448.0) return sign | 0x7E;
    const int binade = a >= 0x1p-6 ? std::ilogb(a) : -6;
    const double quantum = std::ldexp(1.0, binade - 3);
    const double n = std::nearbyint(a / quantum);  // default rounding: to even
    a = std::min(n * quantum, 448.0);
    if (a < 0x1p-6) return sign | (uint8_t)(a * 512.0);
    const int e = std::ilogb(a);
    const int mant = (int)(std::ldexp(a, -e) * 8.0) - 8;
    return sign | (uint8_t)(((e + 7) << 3) | mant);
}

// Largest power of two p with p * amax <= 448 (1 when amax is 0).
double pow2_scale(double amax)
{
    if (!(amax > 0.0)) return 1.0;
    return std::ldexp(1.0, std::ilogb(448.0 / amax));
}

bool is_pow2(float v)
{
    if (!(v > 0.f) || !std::isfinite(v)) return false;
    int e;
    return std::frexp(v, &e) == 0.5f;
}

bool scale_in_range(double v) { return v >= 0x1p-60 && v <= 0x1p60; }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class T>
cm_status dev_alloc(T **p, size_t count, const char *what)
{
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(CM_ENOMEM, "device allocation of %s (%zu bytes) failed", what,
                    count * sizeof(T));
    }
    return CM_OK;
}

void free_model(cm::Model &m)
{
    if (m.d_params) (void)hipFree(m.d_params);
    if (m.d_beta) (void)hipFree(m.d_beta);
    if (m.d_bf16) (void)hipFree(m.d_bf16);
    if (m.d_fp8) (void)hipFree(m.d_fp8);
    delete[] m.h_params;
    m = cm::Model{};
}

void free_ws(cm::Workspace &w)
{
    if (w.d_U) (void)hipFree(w.d_U);
    if (w.d_tpart) (void)hipFree(w.d_tpart);
    if (w.d_tcnt) (void)hipFree(w.d_tcnt);
    w = cm::Workspace{};
}

cm_status check_device(int want)
{
    int dev = -1;
    CM_HIP(hipGetDevice(&dev));
    if (dev != want)
        return fail(CM_EINVAL, "object lives on device %d but device %d is current", want, dev);
    return CM_OK;
}

// Validate a batch's descriptors (no object is read): counts, offsets,
// alignment and, for an evaluation, the per-query byte limit of the
// precision's evaluator (table: features come from a row table).
cm_status check_shape(const cm_batch *b, cm_precision prec, bool eval, bool table = false)
{
    if (!b) return fail(CM_EINVAL, "batch is NULL");
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries > 0 && !b->queries) return fail(CM_EINVAL, "queries is NULL");
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_stages < 1) return fail(CM_EINVAL, "query %d: n_stages %d < 1", q, Q.n_stages);
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        if (Q.pipe_off < 0 || Q.sched_off < 0 || Q.terms_off < 0 || Q.cost_off < 0)
            return fail(CM_EINVAL, "query %d: negative offset", q);
        if (eval && (Q.sched_off % 8) != 0)
            return fail(CM_EINVAL, "query %d: sched_off %lld is not a multiple of 8", q,
                        (long long)Q.sched_off);
        if (eval && (Q.terms_off % 4) != 0)
            return fail(CM_EINVAL, "query %d: terms_off %lld is not a multiple of 4", q,
                        (long long)Q.terms_off);
        if (eval) {
            const cm_status st = cm::check_query_bytes(q, Q.n_stages, Q.n_cands, prec, table);
            if (st != CM_OK) return st;
        }
    }
    return CM_OK;
}

// Validate a batch (already shape-checked) against a workspace's capacities.
cm_status check_batch(const cm_batch *b, const cm::Workspace &w, bool eval)
{
    if (b->n_queries > w.cap.max_queries)
        return fail(CM_E2BIG, "batch has %d queries, workspace holds %d", b->n_queries,
                    w.cap.max_queries);
    int64_t stages = 0, cands = 0, rows = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        stages += Q.n_stages;
        cands += Q.n_cands;
        rows += (int64_t)Q.n_stages * Q.n_cands;
    }
    if (eval) {
        if (stages > w.cap.max_stages)
            return fail(CM_E2BIG, "batch has %lld stages, workspace holds %lld",
                        (long long)stages, (long long)w.cap.max_stages);
        if (rows > w.cap.max_rows)
            return fail(CM_E2BIG, "batch has %lld rows, workspace holds %lld", (long long)rows,
                        (long long)w.cap.max_rows);
    }
    if (cands > w.cap.max_cands)
        return fail(CM_E2BIG, "batch has %lld candidates, workspace holds %lld",
                    (long long)cands, (long long)w.cap.max_cands);
    if (eval && cands > 0) {
        if (!b->pipe || !b->sched || !b->terms)
            return fail(CM_EINVAL, "batch pipe/sched/terms pointer is NULL");
        if (!aligned(b->sched, 16) || !aligned(b->terms, 16) || !aligned(b->pipe, 4))
            return fail(CM_EINVAL, "sched and terms must be 16-byte aligned");
    }
    return CM_OK;
}

}  // namespace

extern "C" {

const char *cm_last_error(void) { return g_err.c_str(); }

int32_t cm_version(void) { return (CM_VERSION_MAJOR << 16) | CM_VERSION_MINOR; }

cm_status cm_model_create(const cm_model_desc *d, const float *params, cm_model **out)
{
    using namespace cm;
    if (!d || !params || !out) return fail(CM_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->n_pipe_features != FP || d->n_sched_features != FS || d->embed != E ||
        d->hidden != H || d->n_coefs != C)
        return fail(CM_EINVAL, "model dimensions must be 56/40/24/32/8");
    for (int i = 0; i < N_PARAMS; ++i)
        if (!std::isfinite(params[i])) return fail(CM_EINVAL, "parameter %d is not finite", i);

    cm_model *M = new (std::nothrow) cm_model;
    if (!M) return fail(CM_ENOMEM, "host allocation failed");
    Model &m = M->m;
    if (hipGetDevice(&m.device) != hipSuccess) {
        delete M;
        return fail(CM_EDEVICE, "no HIP device");
    }

    // W_1[:, 24:] b_s, and the folded schedule layer Wf = W_1[:, 24:] W_s,
    // scaled by ln 2 because the evaluator feeds log2(1 + x).
    const float *Ws = params + OFF_WS, *bs = params + OFF_BS;
    const float *W1 = params + OFF_W1, *W2 = params + OFF_W2;
    float beta[H];
    double Wf[H][FS];
    for (int j = 0; j < H; ++j) {
        double b = 0.0;
        for (int e = 0; e < E; ++e) b += (double)W1[j * 2 * E + E + e] * (double)bs[e];
        beta[j] = (float)b;
        for (int f = 0; f < FS; ++f) {
            double a = 0.0;
            for (int e = 0; e < E; ++e) a += (double)W1[j * 2 * E + E + e] * (double)Ws[e * FS + f];
            Wf[j][f] = a * 0.69314718055994530942;
        }
    }
    Bf16Pack pk;
    std::memset(&pk, 0, sizeof pk);
    // operands of the 16x16x32 bf16 matrix core: lane l holds row l % 16 and
    // k-slots 8g .. 8g+7, g = l / 16
    for (int hh = 0; hh < 2; ++hh)
        for (int lane = 0; lane < 64; ++lane) {
            const int row = 16 * hh + (lane & 15), g = lane >> 4;  // hidden unit
            uint16_t wh[8], wl[8];
            for (int j = 0; j < 8; ++j) split_bf16(Wf[row][8 * g + j], wh[j], wl[j]);
            // last block: features a = 32 + 2g and b = a + 1 against the
            // operand (hi a, hi b, lo a, lo b, hi a, hi b, lo a, lo b)
            uint16_t ha, la, hb, lb;
            split_bf16(Wf[row][32 + 2 * g], ha, la);
            split_bf16(Wf[row][33 + 2 * g], hb, lb);
            const uint16_t wx[8] = {ha, hb, ha, hb, la, lb, 0, 0};
            std::memcpy(&pk.a1[hh][0][lane], wh, 16);
            std::memcpy(&pk.a1[hh][1][lane], wl, 16);
            std::memcpy(&pk.a1[hh][2][lane], wx, 16);
        }
    for (int lane = 0; lane < 64; ++lane) {
        // row m: coefficient m & 7, high weights for m < 8, low ones above;
        // slot j: hidden unit 4g + j (j < 4) or 16 + 4g + j - 4, the order of
        // the first layer's output registers
        const int m = lane & 15, g = lane >> 4;
        uint16_t ws[8], wh[8];
        for (int j = 0; j < 8; ++j) {
            const int p = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
            uint16_t hi, lo;
            split_bf16((double)W2[(m & 7) * H + p], hi, lo);
            ws[j] = m < 8 ? hi : lo;
            wh[j] = m < 8 ? hi : 0;
        }
        std::memcpy(&pk.a2[0][lane], ws, 16);
        std::memcpy(&pk.a2[1][lane], wh, 16);
    }
    for (int mo = 0; mo < C; ++mo) pk.b2[mo] = params[OFF_B2 + mo];

    m.h_params = new (std::nothrow) float[N_PARAMS];
    if (!m.h_params) {
        delete M;
        return fail(CM_ENOMEM, "host allocation failed");
    }
    std::memcpy(m.h_params, params, N_PARAMS * sizeof(float));
    cm_status st;
    if ((st = dev_alloc(&m.d_params, N_PARAMS, "parameters")) != CM_OK ||
        (st = dev_alloc(&m.d_beta, H, "beta")) != CM_OK ||
        (st = dev_alloc(&m.d_bf16, 1, "bf16 operands")) != CM_OK) {
        free_model(m);
        delete M;
        return st;
    }
    if (hipMemcpy(m.d_params, params, N_PARAMS * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(m.d_beta, beta, sizeof beta, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m.d_bf16, &pk, sizeof pk, hipMemcpyHostToDevice) != hipSuccess) {
        free_model(m);
        delete M;
        return fail(CM_EDEVICE, "copy of model parameters failed");
    }
    // the log-transform table of the bf16 evaluator, computed by the device
    if (cm::launch_log_table(m.d_bf16, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
        (void)hipGetLastError();
        free_model(m);
        delete M;
        return fail(CM_EDEVICE, "log table of the bf16 evaluator failed");
    }
    // set-up of cm_eval_batch_static on this device
    float *scr = nullptr;
    if ((st = static_scratch(m.device, &scr)) != CM_OK) {
        free_model(m);
        delete M;
        return st;
    }
    *out = M;
    return CM_OK;
}

cm_status cm_model_destroy(cm_model *M)
{
    if (!M) return fail(CM_EINVAL, "model is NULL");
    free_model(M->m);
    delete M;
    return CM_OK;
}

cm_status cm_workspace_create(const cm_workspace_desc *d, cm_workspace **out)
{
    using namespace cm;
    if (!d || !out) return fail(CM_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->max_queries < 1 || d->max_stages < 1 || d->max_cands < 0 || d->max_rows < 0 ||
        d->max_k < 1 || d->max_k > CM_MAX_K)
        return fail(CM_EINVAL, "bad workspace capacities");
    if (d->max_rows > ((int64_t)1 << 40) || d->max_cands > INT32_MAX ||
        d->max_stages > INT32_MAX / 2)
        return fail(CM_EINVAL, "workspace capacities too large");
    cm_workspace *W = new (std::nothrow) cm_workspace;
    if (!W) return fail(CM_ENOMEM, "host allocation failed");
    Workspace &w = W->w;
    w.cap = *d;
    if (hipGetDevice(&w.device) != hipSuccess) {
        delete W;
        return fail(CM_EDEVICE, "no HIP device");
    }
    w.tpart_cap = (d->max_cands / TOPK_TILE + d->max_queries + 1) * (int64_t)d->max_k;
    cm_status st;
    if ((st = dev_alloc(&w.d_U, (size_t)d->max_stages * H, "hoisted stage vectors")) != CM_OK ||
        (st = dev_alloc(&w.d_tpart, (size_t)w.tpart_cap, "beam lists")) != CM_OK ||
        (st = dev_alloc(&w.d_tcnt, (size_t)QMAX, "beam counters")) != CM_OK) {
        free_ws(w);
        delete W;
        return st;
    }
    if (hipMemset(w.d_tcnt, 0, QMAX * sizeof(int32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_ws(w);
        delete W;
        return fail(CM_EDEVICE, "workspace initialisation failed");
    }
    *out = W;
    return CM_OK;
}

cm_status cm_workspace_destroy(cm_workspace *W)
{
    if (!W) return fail(CM_EINVAL, "workspace is NULL");
    free_ws(W->w);
    delete W;
    return CM_OK;
}

}  // extern "C"

namespace {

// Descriptors of queries [g0, g0 + ng) for one launch.  Hoisted rows of the
// batch are laid out in batch order: query q's rows start at (sum of n_stages
// of the queries before it) * 32 floats.
void fill_eval_launch(cm::EvalLaunch &L, const cm_batch *b, int32_t g0, int32_t ng,
                      int64_t stage_prefix, cm_precision prec)
{
    using namespace cm;
    std::memset(&L, 0, sizeof L);
    L.nq = ng;
    // hoisted rows stay in batch order; workgroups are issued longest stage
    // part first so the longest-running ones start earliest
    int64_t row_of[QMAX];
    int32_t order[QMAX];
    int64_t r = 0;
    for (int32_t j = 0; j < ng; ++j) {
        row_of[j] = r;
        r += b->queries[g0 + j].n_stages;
        order[j] = j;
    }
    if (prec != CM_FP32) {
        auto per_wave = [&](int32_t j) {
            const int S = b->queries[g0 + j].n_stages;
            return (S + stage_parts(S) - 1) / stage_parts(S);
        };
        std::stable_sort(order, order + ng,
                         [&](int32_t x, int32_t y) { return per_wave(x) > per_wave(y); });
    }
    int64_t hrow = 0, task = 0;
    for (int32_t jj = 0; jj < ng; ++jj) {
        const int32_t j = order[jj];
        const cm_query &Q = b->queries[g0 + j];
        EvalQ &e = L.q[jj];
        e.S = Q.n_stages;
        e.N = Q.n_cands;
        e.pipe_off = Q.pipe_off;
        e.sched_off = Q.sched_off;
        e.terms_off = Q.terms_off;
        e.cost_off = Q.cost_off;
        e.u_off = (stage_prefix + row_of[j]) * H;
        e.hrow0 = (int32_t)hrow;
        e.task0 = (int32_t)task;
        e.parts = stage_parts(Q.n_stages);
        e.stage_off = Q.terms_off / C;
        hrow += Q.n_stages;
        if (prec == CM_FP32) {
            task += cdiv(Q.n_cands, 64);
        } else {
            const int64_t tiles = cdiv(Q.n_cands, TILE_ROWS);
            task += cdiv(tiles, EVAL_WAVES / e.parts);
        }
    }
    L.ntasks = (int32_t)task;
    L.nstages = (int32_t)hrow;
}

cm_status check_queries(const cm_batch *b)
{
    if (!b) return fail(CM_EINVAL, "batch is NULL");
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries > 0 && !b->queries) return fail(CM_EINVAL, "queries is NULL");
    int64_t stages = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_stages < 1) return fail(CM_EINVAL, "query %d: n_stages %d < 1", q, Q.n_stages);
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        if (Q.pipe_off < 0) return fail(CM_EINVAL, "query %d: negative offset", q);
        stages += Q.n_stages;
    }
    if (stages > INT32_MAX / 2) return fail(CM_E2BIG, "too many stages");
    if (b->n_queries > 0 && !b->pipe) return fail(CM_EINVAL, "pipe is NULL");
    return CM_OK;
}

cm_status hoist_impl(const cm_model *M, cm_precision prec, const cm_batch *b, float *U,
                     hipStream_t s)
{
    using namespace cm;
    int64_t stage_prefix = 0;
    for (int32_t g0 = 0; g0 < b->n_queries; g0 += QMAX) {
        const int32_t ng = std::min<int32_t>(QMAX, b->n_queries - g0);
        EvalLaunch L;
        fill_eval_launch(L, b, g0, ng, stage_prefix, prec);
        CM_HIP(launch_hoist(L, M->m, prec != CM_FP32, prec == CM_FP8 ? M->m.fp8_uscale : 1.f,
                            b->pipe, U, s));
        stage_prefix += L.nstages;
    }
    return CM_OK;
}

cm_status eval_impl(const cm_model *M, cm_precision prec, const cm_batch *b, const float *U,
                    const cm::Workspace &w, float *cost_out, float *stage_out, hipStream_t s,
                    const int32_t *ridx = nullptr, uint32_t rows = 0)
{
    using namespace cm;
    int64_t stage_prefix = 0;
    for (int32_t g0 = 0; g0 < b->n_queries; g0 += QMAX) {
        const int32_t ng = std::min<int32_t>(QMAX, b->n_queries - g0);
        EvalLaunch L;
        fill_eval_launch(L, b, g0, ng, stage_prefix, prec);
        if (prec == CM_FP32)
            CM_HIP(launch_eval_fp32(L, M->m, (const float *)b->sched, b->terms, U, cost_out,
                                    stage_out, s));
        else if (prec == CM_FP8)
            CM_HIP(launch_eval_fp8(L, M->m, (const uint8_t *)b->sched, b->terms, U, cost_out,
                                   stage_out, s, ridx, rows));
        else
            CM_HIP(launch_eval_bf16(L, M->m, (const uint16_t *)b->sched, b->terms, U, cost_out,
                                    stage_out, s, ridx, rows));
        stage_prefix += L.nstages;
    }
    return CM_OK;
}

cm_status check_eval(const cm_model *M, cm_precision prec, const cm_batch *b,
                     const cm_workspace *W, const float *cost_out, int64_t *cands,
                     bool table = false)
{
    if (!M || !W) return fail(CM_EINVAL, "model or workspace is NULL");
    if (prec != CM_FP32 && prec != CM_BF16 && prec != CM_FP8)
        return fail(CM_EUNSUPPORTED, "precision %d is not supported", prec);
    // the descriptors first: no object is read before they have been checked
    cm_status st = check_shape(b, prec, true, table);
    if (st != CM_OK) return st;
    if (prec == CM_FP8 && !M->m.d_fp8)
        return fail(CM_EINVAL, "model has no FP8 form (cm_model_prepare_fp8)");
    if ((st = check_batch(b, W->w, true)) != CM_OK) return st;
    if ((st = check_device(M->m.device)) != CM_OK) return st;
    if (W->w.device != M->m.device) return fail(CM_EINVAL, "model and workspace devices differ");
    *cands = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) *cands += b->queries[q].n_cands;
    if (*cands > 0 && !cost_out) return fail(CM_EINVAL, "cost_out is NULL");
    return CM_OK;
}

}  // namespace

extern "C" {

cm_status cm_hoist_stages(const cm_model *M, cm_precision prec, const cm_batch *b, float *U_out,
                          cm_stream stream)
{
    if (!M) return fail(CM_EINVAL, "model is NULL");
    if (prec != CM_FP32 && prec != CM_BF16 && prec != CM_FP8)
        return fail(CM_EUNSUPPORTED, "precision %d is not supported", prec);
    if (prec == CM_FP8 && !M->m.d_fp8)
        return fail(CM_EINVAL, "model has no FP8 form (cm_model_prepare_fp8)");
    cm_status st = check_queries(b);
    if (st != CM_OK) return st;
    if (b->n_queries == 0) return CM_OK;
    if (!U_out) return fail(CM_EINVAL, "U_out is NULL");
    if (!aligned(U_out, 16)) return fail(CM_EINVAL, "U_out must be 16-byte aligned");
    if ((st = check_device(M->m.device)) != CM_OK) return st;
    return hoist_impl(M, prec, b, U_out, (hipStream_t)stream);
}

cm_status cm_eval_hoisted(const cm_model *M, cm_precision prec, const cm_batch *b,
                          const float *U, cm_workspace *W, float *cost_out, cm_stream stream)
{
    int64_t cands = 0;
    cm_status st = check_eval(M, prec, b, W, cost_out, &cands);
    if (st != CM_OK) return st;
    if (cands == 0) return CM_OK;
    if (!U || !aligned(U, 16)) return fail(CM_EINVAL, "U is NULL or not 16-byte aligned");
    return eval_impl(M, prec, b, U, W->w, cost_out, nullptr, (hipStream_t)stream);
}

cm_status cm_eval_batch(const cm_model *M, cm_precision prec, const cm_batch *b,
                        cm_workspace *W, float *cost_out, cm_stream stream)
{
    int64_t cands = 0;
    cm_status st = check_eval(M, prec, b, W, cost_out, &cands);
    if (st != CM_OK) return st;
    if (cands == 0) return CM_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = hoist_impl(M, prec, b, W->w.d_U, s)) != CM_OK) return st;
    return eval_impl(M, prec, b, W->w.d_U, W->w, cost_out, nullptr, s);
}

cm_status cm_eval_batch_static(const cm_model *M, cm_precision prec, const cm_batch *b,
                               float *cost_out, cm_stream stream)
{
    using namespace cm;
    if (!M) return fail(CM_EINVAL, "model is NULL");
    if (prec != CM_FP32 && prec != CM_BF16 && prec != CM_FP8)
        return fail(CM_EUNSUPPORTED, "precision %d is not supported", prec);
    // the descriptors first: no object is read before they have been checked
    cm_status st = check_shape(b, prec, true);
    if (st != CM_OK) return st;
    int64_t stages = 0, cands = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        stages += b->queries[q].n_stages;
        cands += b->queries[q].n_cands;
    }
    if (stages > CM_STATIC_MAX_STAGES)
        return fail(CM_E2BIG, "batch has %lld stages, the static scratch holds %d",
                    (long long)stages, CM_STATIC_MAX_STAGES);
    if (prec == CM_FP8 && !M->m.d_fp8)
        return fail(CM_EINVAL, "model has no FP8 form (cm_model_prepare_fp8)");
    if ((st = check_device(M->m.device)) != CM_OK) return st;
    if (cands == 0) return CM_OK;
    if (!cost_out) return fail(CM_EINVAL, "cost_out is NULL");
    if (!b->pipe || !b->sched || !b->terms)
        return fail(CM_EINVAL, "batch pipe/sched/terms pointer is NULL");
    if (!aligned(b->sched, 16) || !aligned(b->terms, 16) || !aligned(b->pipe, 4))
        return fail(CM_EINVAL, "sched and terms must be 16-byte aligned");
    float *U = nullptr;
    if ((st = static_scratch(M->m.device, &U)) != CM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = hoist_impl(M, prec, b, U, s)) != CM_OK) return st;
    return eval_impl(M, prec, b, U, Workspace{}, cost_out, nullptr, s);
}

cm_status cm_eval_stages(const cm_model *M, cm_precision prec, const cm_batch *b,
                         cm_workspace *W, float *cost_out, float *stage_cost_out,
                         cm_stream stream)
{
    int64_t cands = 0;
    cm_status st = check_eval(M, prec, b, W, cost_out, &cands);
    if (st != CM_OK) return st;
    for (int32_t q = 0; q < b->n_queries; ++q)
        if (b->queries[q].terms_off % cm::C != 0)
            return fail(CM_EINVAL, "query %d: terms_off %lld is not a multiple of 8", q,
                        (long long)b->queries[q].terms_off);
    if (cands == 0) return CM_OK;
    if (!stage_cost_out) return fail(CM_EINVAL, "stage_cost_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    if ((st = hoist_impl(M, prec, b, W->w.d_U, s)) != CM_OK) return st;
    return eval_impl(M, prec, b, W->w.d_U, W->w, cost_out, stage_cost_out, s);
}

cm_status cm_eval_indexed(const cm_model *M, cm_precision prec, const cm_batch *b,
                          const int32_t *row_idx, int64_t table_rows, cm_workspace *W,
                          float *cost_out, cm_stream stream)
{
    using namespace cm;
    if (prec == CM_FP32)
        return fail(CM_EUNSUPPORTED, "memoized rows need CM_BF16 or CM_FP8");
    int64_t cands = 0;
    cm_status st = check_eval(M, prec, b, W, cost_out, &cands, true);
    if (st != CM_OK) return st;
    if (cands == 0) return CM_OK;
    const int64_t row_bytes = prec == CM_FP8 ? FS : FS * 2;
    if (table_rows < 1 || table_rows * row_bytes > (int64_t)UINT32_MAX - 256)
        return fail(CM_EINVAL, "table_rows %lld outside [1, %lld]", (long long)table_rows,
                    (long long)(((int64_t)UINT32_MAX - 256) / row_bytes));
    if (!row_idx) return fail(CM_EINVAL, "row_idx is NULL");
    if (!aligned(row_idx, 4)) return fail(CM_EINVAL, "row_idx must be 4-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if ((st = hoist_impl(M, prec, b, W->w.d_U, s)) != CM_OK) return st;
    return eval_impl(M, prec, b, W->w.d_U, W->w, cost_out, nullptr, s, row_idx,
                     (uint32_t)table_rows);
}

cm_status cm_penalize_known_bad(const cm_batch *b, const uint64_t *hashes,
                                const uint64_t *bad_sorted, int64_t n_bad, float penalty,
                                float *cost, cm_stream stream)
{
    using namespace cm;
    if (!b) return fail(CM_EINVAL, "batch is NULL");
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries > 0 && !b->queries) return fail(CM_EINVAL, "queries is NULL");
    if (n_bad < 0) return fail(CM_EINVAL, "n_bad %lld < 0", (long long)n_bad);
    if (n_bad > 0 && !bad_sorted) return fail(CM_EINVAL, "bad_sorted is NULL");
    if (std::isnan(penalty)) return fail(CM_EINVAL, "penalty is NaN");
    int64_t cands = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        if (Q.cost_off < 0) return fail(CM_EINVAL, "query %d: negative cost_off", q);
        cands += Q.n_cands;
    }
    if (cands == 0 || n_bad == 0) return CM_OK;
    if (!hashes || !cost) return fail(CM_EINVAL, "hashes or cost is NULL");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t g0 = 0; g0 < b->n_queries; g0 += QMAX) {
        const int32_t ng = std::min<int32_t>(QMAX, b->n_queries - g0);
        PenaltyLaunch L;
        std::memset(&L, 0, sizeof L);
        L.nq = ng;
        int64_t c0 = 0;
        for (int32_t j = 0; j < ng; ++j) {
            const cm_query &Q = b->queries[g0 + j];
            L.q[j].N = Q.n_cands;
            L.q[j].cost_off = Q.cost_off;
            L.q[j].cand0 = c0;
            c0 += Q.n_cands;
        }
        CM_HIP(launch_penalty(L, hashes, bad_sorted, n_bad, penalty, cost, s));
    }
    return CM_OK;
}

cm_status cm_freeze_stages(const float *stage_cost, const cm_batch *b, const int32_t *cand,
                           int64_t cand_stride, uint8_t *frozen_out, cm_stream stream)
{
    using namespace cm;
    if (!b) return fail(CM_EINVAL, "batch is NULL");
    if (b->n_queries < 0) return fail(CM_EINVAL, "n_queries < 0");
    if (b->n_queries > 0 && !b->queries) return fail(CM_EINVAL, "queries is NULL");
    if (b->n_queries == 0) return CM_OK;
    if (cand_stride < 1) return fail(CM_EINVAL, "cand_stride %lld < 1", (long long)cand_stride);
    if (!cand || !frozen_out) return fail(CM_EINVAL, "cand or frozen_out is NULL");
    int64_t cands = 0, stages = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) {
        const cm_query &Q = b->queries[q];
        if (Q.n_stages < 1) return fail(CM_EINVAL, "query %d: n_stages %d < 1", q, Q.n_stages);
        if (Q.n_cands < 0) return fail(CM_EINVAL, "query %d: n_cands %d < 0", q, Q.n_cands);
        stages += Q.n_stages;
        if (Q.terms_off < 0 || Q.terms_off % C != 0)
            return fail(CM_EINVAL, "query %d: terms_off %lld is not a non-negative multiple of 8",
                        q, (long long)Q.terms_off);
        cands += Q.n_cands;
    }
    if (cands > 0 && !stage_cost) return fail(CM_EINVAL, "stage_cost is NULL");
    if (stages > INT32_MAX) return fail(CM_E2BIG, "too many stages");
    hipStream_t s = (hipStream_t)stream;
    int64_t flag = 0;
    for (int32_t g0 = 0; g0 < b->n_queries; g0 += QMAX) {
        const int32_t ng = std::min<int32_t>(QMAX, b->n_queries - g0);
        FreezeLaunch L;
        std::memset(&L, 0, sizeof L);
        L.nq = ng;
        for (int32_t j = 0; j < ng; ++j) {
            const cm_query &Q = b->queries[g0 + j];
            FreezeQ &f = L.q[j];
            f.S = Q.n_stages;
            f.N = Q.n_cands;
            f.stage_off = Q.terms_off / C;
            f.flag_off = flag;
            f.cand_q = g0 + j;
            flag += Q.n_stages;
        }
        CM_HIP(launch_freeze(L, stage_cost, cand, cand_stride, frozen_out, s));
    }
    return CM_OK;
}

cm_status cm_topk_per_query(const float *cost, const cm_batch *b, int32_t k, cm_workspace *W,
                            int32_t *idx_out, float *val_out, cm_stream stream)
{
    using namespace cm;
    if (!W) return fail(CM_EINVAL, "workspace is NULL");
    if (k < 1 || k > CM_MAX_K || k > W->w.cap.max_k)
        return fail(CM_EINVAL, "k=%d outside [1, %d]", k, std::min(CM_MAX_K, W->w.cap.max_k));
    cm_status st = check_shape(b, CM_FP32, false);
    if (st != CM_OK) return st;
    if ((st = check_batch(b, W->w, false)) != CM_OK) return st;
    if ((st = check_device(W->w.device)) != CM_OK) return st;
    if (b->n_queries == 0) return CM_OK;
    if (!idx_out || !val_out) return fail(CM_EINVAL, "idx_out or val_out is NULL");
    int64_t cands = 0;
    for (int32_t q = 0; q < b->n_queries; ++q) cands += b->queries[q].n_cands;
    if (cands > 0 && !cost) return fail(CM_EINVAL, "cost is NULL");
    hipStream_t s = (hipStream_t)stream;
    const Workspace &w = W->w;

    for (int32_t g0 = 0; g0 < b->n_queries; g0 += QMAX) {
        const int32_t ng = std::min<int32_t>(QMAX, b->n_queries - g0);
        TopkLaunch L;
        std::memset(&L, 0, sizeof L);
        L.nq = ng;
        L.k = k;
        int64_t tile = 0;
        for (int32_t j = 0; j < ng; ++j) {
            const cm_query &Q = b->queries[g0 + j];
            TopkQ &t = L.q[j];
            t.N = Q.n_cands;
            t.out_q = g0 + j;
            t.cost_off = Q.cost_off;
            t.tile0 = (int32_t)tile;
            t.ntiles = (int32_t)std::max<int64_t>(1, cdiv(Q.n_cands, TOPK_TILE));
            tile += t.ntiles;
        }
        if (tile * k > w.tpart_cap) return fail(CM_E2BIG, "batch exceeds workspace beam lists");
        L.ntasks = (int32_t)tile;
        CM_HIP(launch_topk(L, cost, w.d_tpart, w.d_tcnt, idx_out, val_out, s));
    }
    return CM_OK;
}

// ------------------------------------------------------------------ FP8 form

cm_status cm_model_prepare_fp8(cm_model *M, float in_scale, float act_scale)
{
    using namespace cm;
    if (!M) return fail(CM_EINVAL, "model is NULL");
    if (!is_pow2(in_scale) || !is_pow2(act_scale))
        return fail(CM_EINVAL, "in_scale and act_scale must be positive powers of two");
    cm_status st = check_device(M->m.device);
    if (st != CM_OK) return st;
    const float *p = M->m.h_params;
    const float *Ws = p + OFF_WS, *W1 = p + OFF_W1, *W2 = p + OFF_W2;

    // folded first layer over the schedule features: Wf = W_1[:, 24:] W_s
    static_assert(sizeof(Fp8Pack) % 16 == 0, "Fp8Pack size");
    double Wf[H][FS];
    double amax1 = 0.0, amax2 = 0.0;
    for (int j = 0; j < H; ++j)
        for (int f = 0; f < FS; ++f) {
            double a = 0.0;
            for (int e = 0; e < E; ++e) a += (double)W1[j * 2 * E + E + e] * (double)Ws[e * FS + f];
            Wf[j][f] = a;
            amax1 = std::max(amax1, std::fabs(a));
        }
    for (int i = 0; i < C * H; ++i) amax2 = std::max(amax2, std::fabs((double)W2[i]));
    const double sw1 = pow2_scale(amax1), sw2 = pow2_scale(amax2);
    const double su = sw1 * in_scale, r1 = act_scale / su, r2 = 1.0 / (sw2 * act_scale);
    if (!scale_in_range(su) || !scale_in_range(r1) || !scale_in_range(r2))
        return fail(CM_EINVAL, "FP8 scales out of range (s_w1 %g, s_w2 %g, s_in %g, s_h %g)", sw1,
                    sw2, (double)in_scale, (double)act_scale);

    Fp8Pack pk;
    std::memset(&pk, 0, sizeof pk);
    for (int lane = 0; lane < 64; ++lane) {
        const int m = lane & 31, h = lane >> 5;
        uint8_t a1[32] = {}, a2[32] = {};
        // first layer: byte j of lane m + 32h meets schedule feature 20h + j
        for (int j = 0; j < 20; ++j) a1[j] = e4m3_code(Wf[m][20 * h + j] * sw1);
        // coefficient layer: byte j of lane m + 32h meets hidden unit
        // (j / 4) * 8 + 4h + j % 4, the unit the first layer's accumulator
        // register j holds in that lane half
        if (m < C)
            for (int j = 0; j < 16; ++j)
                a2[j] = e4m3_code((double)W2[m * H + (j / 4) * 8 + 4 * h + j % 4] * sw2);
        std::memcpy(pk.a1[lane], a1, 32);
        std::memcpy(pk.a2[lane], a2, 32);
    }
    for (int c = 0; c < C; ++c) pk.b2[c] = p[OFF_B2 + c];
    pk.r1 = (float)r1;
    pk.r2 = (float)r2;
    pk.uh = act_scale;

    Fp8Pack *d = M->m.d_fp8;
    if (!d && (st = dev_alloc(&d, 1, "fp8 operands")) != CM_OK) return st;
    if (hipMemcpy(d, &pk, sizeof pk, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (!M->m.d_fp8) (void)hipFree(d);
        return fail(CM_EDEVICE, "copy of the FP8 operands failed");
    }
    M->m.d_fp8 = d;
    M->m.fp8_uscale = act_scale;
    return CM_OK;
}

cm_status cm_fp8_calibrate(const cm_model *M, int64_t n_rows, const float *pipe_rows,
                           const float *sched_rows, float *in_scale_out, float *act_scale_out)
{
    using namespace cm;
    if (!M || !pipe_rows || !sched_rows || !in_scale_out || !act_scale_out)
        return fail(CM_EINVAL, "NULL argument");
    if (n_rows < 1) return fail(CM_EINVAL, "n_rows %lld < 1", (long long)n_rows);
    const float *p = M->m.h_params;
    const float *Wp = p + OFF_WP, *bp = p + OFF_BP, *Ws = p + OFF_WS, *bs = p + OFF_BS;
    const float *W1 = p + OFF_W1, *b1 = p + OFF_B1;
    double xmax = 0.0, hmax = 0.0;
    for (int64_t r = 0; r < n_rows; ++r) {
        const float *pr = pipe_rows + r * FP, *sr = sched_rows + r * FS;
        double lp[FP], ls[FS], emb[2 * E];
        bool ok = true;
        for (int f = 0; f < FP && ok; ++f) ok = std::isfinite(lp[f] = std::log1p((double)pr[f]));
        for (int f = 0; f < FS && ok; ++f) ok = std::isfinite(ls[f] = std::log1p((double)sr[f]));
        if (!ok) continue;
        for (int f = 0; f < FS; ++f) xmax = std::max(xmax, std::fabs(ls[f]));
        for (int e = 0; e < E; ++e) {
            double a = bp[e], b = bs[e];
            for (int f = 0; f < FP; ++f) a += (double)Wp[e * FP + f] * lp[f];
            for (int f = 0; f < FS; ++f) b += (double)Ws[e * FS + f] * ls[f];
            emb[e] = a;
            emb[E + e] = b;
        }
        for (int j = 0; j < H; ++j) {
            double a = b1[j];
            for (int e = 0; e < 2 * E; ++e) a += (double)W1[j * 2 * E + e] * emb[e];
            hmax = std::max(hmax, a);
        }
    }
    *in_scale_out = (float)pow2_scale(2.0 * xmax);
    *act_scale_out = (float)pow2_scale(2.0 * hmax);
    return CM_OK;
}

cm_status cm_fp8_encode(const float *x, int64_t n, float in_scale, uint8_t *codes,
                        cm_stream stream)
{
    using namespace cm;
    if (n < 0) return fail(CM_EINVAL, "n %lld < 0", (long long)n);
    if (!is_pow2(in_scale)) return fail(CM_EINVAL, "in_scale must be a positive power of two");
    if (n == 0) return CM_OK;
    if (!x || !codes) return fail(CM_EINVAL, "x or codes is NULL");
    if (!aligned(x, 16) || !aligned(codes, 16))
        return fail(CM_EINVAL, "x and codes must be 16-byte aligned");
    const uintptr_t xa = (uintptr_t)x, xb = xa + (uintptr_t)n * 4;
    const uintptr_t ca = (uintptr_t)codes, cb = ca + (uintptr_t)n;
    if (xa < cb && ca < xb) return fail(CM_EINVAL, "x and codes overlap");
    CM_HIP(launch_fp8_encode(x, n, in_scale, codes, (hipStream_t)stream));
    return CM_OK;
}

}  // extern "C"
