// C ABI of the bsi library: contexts, fields, validation, caches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"

namespace bsi {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

namespace {
thread_local int g_untimed = 0;
}

bool untimed() { return g_untimed > 0; }
UntimedScope::UntimedScope() { ++g_untimed; }
UntimedScope::~UntimedScope() { --g_untimed; }

StageTimer::StageTimer(bsi_ctx* ctx, const char* stage, hipStream_t s) : ctx_(ctx), stage_(stage), s_(s) {
    if (!ctx_ || !ctx_->timing || untimed()) return;
    // no timing inside a stream capture (the events would belong to the graph)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s_, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(ctx_->mu);
    if (!ctx_->event_pool.empty()) {
        start_ = ctx_->event_pool.back();
        ctx_->event_pool.pop_back();
    } else if (hipEventCreate(&start_) != hipSuccess) {
        (void)hipGetLastError();
        start_ = nullptr;
        return;
    }
    if (hipEventRecord(start_, s_) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(start_);
        start_ = nullptr;
    }
}

StageTimer::~StageTimer() {
    if (!start_) return;
    std::lock_guard<std::mutex> lk(ctx_->mu);
    hipEvent_t stop = nullptr;
    if (!ctx_->event_pool.empty()) {
        stop = ctx_->event_pool.back();
        ctx_->event_pool.pop_back();
    } else if (hipEventCreate(&stop) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(start_);
        return;
    }
    if (hipEventRecord(stop, s_) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(start_);
        ctx_->event_pool.push_back(stop);
        return;
    }
    ctx_->pending.push_back({std::string(stage_), start_, stop});
}

namespace {
// Resolve recorded event pairs into per-stage totals (caller holds ctx->mu).
bsi_status drain_timing(bsi_ctx* ctx) {
    for (auto& p : ctx->pending) {
        float ms = 0.f;
        BSI_HIP(hipEventSynchronize(p.stop));
        BSI_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
        auto& tot = ctx->stage_totals[p.stage];
        tot.first += double(ms);
        tot.second += 1;
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    ctx->pending.clear();
    return BSI_OK;
}
}  // namespace

hipStream_t pick_stream(bsi_ctx* ctx, void* s) {
    return s ? static_cast<hipStream_t>(s) : ctx->stream;
}

bsi_status get_workspace(std::map<hipStream_t, Workspace>& m, hipStream_t s, size_t bytes, void** out) {
    Workspace& w = m[s];
    if (w.bytes < bytes) {
        if (w.ptr) {
            // the old buffer may still be in use by queued work on this stream
            BSI_HIP(hipStreamSynchronize(s));
            BSI_HIP(hipFree(w.ptr));
            w.ptr = nullptr;
            w.bytes = 0;
        }
        const size_t want = bytes + bytes / 8;
        if (hipMalloc(&w.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            set_error("workspace allocation of " + std::to_string(want) + " bytes failed");
            return BSI_E_NOMEM;
        }
        w.bytes = want;
    }
    *out = w.ptr;
    return BSI_OK;
}

bsi_status get_twiddles(bsi_ctx* ctx, int len, bool dbl, const void** out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_pair(len, dbl ? 1 : 0);
    auto it = ctx->twiddles.find(key);
    if (it != ctx->twiddles.end()) {
        *out = it->second;
        return BSI_OK;
    }
    // exp(+2 pi i m / len) in FP64 on the host; the angle is reduced to the
    // first octant by symmetry so every entry is one correctly rounded call.
    std::vector<double> tab(2 * size_t(len));
    for (int m = 0; m < len; ++m) {
        const double a = 2.0 * M_PI * double(m) / double(len);
        tab[2 * m] = std::cos(a);
        tab[2 * m + 1] = std::sin(a);
        if (4 * m == len) { tab[2 * m] = 0.0; tab[2 * m + 1] = 1.0; }
        if (2 * m == len) { tab[2 * m] = -1.0; tab[2 * m + 1] = 0.0; }
        if (4 * m == 3 * len) { tab[2 * m] = 0.0; tab[2 * m + 1] = -1.0; }
    }
    void* d = nullptr;
    if (dbl) {
        BSI_HIP(hipMalloc(&d, tab.size() * sizeof(double)));
        BSI_HIP(hipMemcpy(d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> tf(tab.size());
        for (size_t i = 0; i < tab.size(); ++i) tf[i] = float(tab[i]);
        BSI_HIP(hipMalloc(&d, tf.size() * sizeof(float)));
        BSI_HIP(hipMemcpy(d, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    ctx->twiddles[key] = d;
    *out = d;
    return BSI_OK;
}

bsi_status get_ctable(bsi_ctx* ctx, int n, int order, int variant, const double** out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_tuple(n, order, variant);
    auto it = ctx->ctabs.find(key);
    if (it != ctx->ctabs.end()) {
        *out = it->second;
        return BSI_OK;
    }
    std::vector<double> tab(n);
    prefilter_table(n, order, variant, tab.data());
    double* d = nullptr;
    BSI_HIP(hipMalloc(&d, n * sizeof(double)));
    BSI_HIP(hipMemcpy(d, tab.data(), n * sizeof(double), hipMemcpyHostToDevice));
    ctx->ctabs[key] = d;
    *out = d;
    return BSI_OK;
}

namespace {

bsi_status check_device_ptr(const void* p, const char* what) {
    if (!p) {
        set_error(std::string(what) + " is NULL");
        return BSI_E_INVAL;
    }
    if (reinterpret_cast<uintptr_t>(p) % 8 != 0) {
        set_error(std::string(what) + " is not 8-byte aligned");
        return BSI_E_INVAL;
    }
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string(what) + " is not a HIP device pointer");
        return BSI_E_INVAL;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) {
        set_error(std::string(what) + " is not device memory");
        return BSI_E_INVAL;
    }
    return BSI_OK;
}

}  // namespace

bsi_status check_device_ptr_ex(const void* p, const char* what) { return check_device_ptr(p, what); }

}  // namespace bsi

using namespace bsi;

extern "C" {

const char* bsi_last_error(void) { return bsi::g_last_error.c_str(); }

const char* bsi_version(void) { return "bsi 0.1 (gfx950)"; }

bsi_status bsi_ctx_create(int device, void* hip_stream, bsi_ctx** out) {
    clear_error();
    BSI_CHECK(out != nullptr, BSI_E_INVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    BSI_HIP(hipGetDeviceCount(&ndev));
    BSI_CHECK(device >= 0 && device < ndev, BSI_E_INVAL, "device index out of range");
    BSI_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    BSI_HIP(hipGetDeviceProperties(&prop, device));
    auto* ctx = new (std::nothrow) bsi_ctx();
    BSI_CHECK(ctx != nullptr, BSI_E_NOMEM, "host allocation failed");
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->num_cus = prop.multiProcessorCount;
    ctx->lds_per_block = prop.sharedMemPerBlock;
    const bsi_status st = static_scratch_init(device);
    if (st != BSI_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return BSI_OK;
}

bsi_status bsi_ctx_set_timing(bsi_ctx* ctx, int32_t enabled) {
    clear_error();
    BSI_CHECK(ctx != nullptr, BSI_E_INVAL, "ctx is NULL");
    ctx->timing = enabled != 0;
    return BSI_OK;
}

bsi_status bsi_ctx_read_timing(bsi_ctx* ctx, const char* stage, double* total_ms, int64_t* launches) {
    clear_error();
    BSI_CHECK(ctx && stage && total_ms && launches, BSI_E_INVAL, "NULL argument");
    BSI_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    BSI_TRY(drain_timing(ctx));
    auto it = ctx->stage_totals.find(stage);
    *total_ms = it == ctx->stage_totals.end() ? 0.0 : it->second.first;
    *launches = it == ctx->stage_totals.end() ? 0 : it->second.second;
    return BSI_OK;
}

bsi_status bsi_ctx_reset_timing(bsi_ctx* ctx) {
    clear_error();
    BSI_CHECK(ctx != nullptr, BSI_E_INVAL, "ctx is NULL");
    BSI_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    BSI_TRY(drain_timing(ctx));
    ctx->stage_totals.clear();
    return BSI_OK;
}

void bsi_ctx_destroy(bsi_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& p : ctx->pending) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    for (auto& kv : ctx->twiddles) (void)hipFree(kv.second);
    for (auto& kv : ctx->ctabs) (void)hipFree(kv.second);
    for (auto& kv : ctx->fft_ws) (void)hipFree(kv.second.ptr);
    for (auto& kv : ctx->eval_ws) (void)hipFree(kv.second.ptr);
    delete ctx;
}

bsi_status bsi_field_create(bsi_ctx* ctx, const bsi_field_desc* desc, bsi_field** out) {
    clear_error();
    BSI_CHECK(ctx && desc && out, BSI_E_INVAL, "NULL argument");
    *out = nullptr;
    BSI_CHECK(desc->basis == BSI_BASIS_BSPLINE || desc->basis == BSI_BASIS_LAGRANGE ||
                  desc->basis == BSI_BASIS_HERMITE,
              BSI_E_INVAL, "unknown basis");
    if (desc->basis == BSI_BASIS_HERMITE)
        BSI_CHECK(desc->order == 4, BSI_E_UNSUPPORTED, "Hermite interpolation is implemented for order 4");
    else
        BSI_CHECK(desc->order == 2 || desc->order == 4 || desc->order == 6, BSI_E_UNSUPPORTED,
                  "only orders 2, 4 and 6 are implemented");
    BSI_CHECK(desc->ncomp == 1 || desc->ncomp == 3, BSI_E_INVAL, "ncomp must be 1 or 3");
    BSI_CHECK(desc->coef == BSI_F64 || desc->coef == BSI_F32 || desc->coef == BSI_BF16, BSI_E_INVAL,
              "unknown coefficient dtype");
    BSI_CHECK(desc->prefilter == BSI_PREFILTER_L2OPT || desc->prefilter == BSI_PREFILTER_INTERP ||
                  desc->prefilter == BSI_PREFILTER_NONE,
              BSI_E_INVAL, "unknown prefilter variant");
    BSI_CHECK(desc->basis == BSI_BASIS_BSPLINE || desc->prefilter == BSI_PREFILTER_NONE, BSI_E_INVAL,
              "Lagrange and Hermite fields hold the field's values: prefilter must be NONE");
    for (int d = 0; d < 3; ++d) {
        const int n = desc->n[d];
        BSI_CHECK(n >= 2 * desc->order && n >= 8 && n <= 1024 && n % 2 == 0, BSI_E_INVAL,
                  "each n must be even with max(2*order, 8) <= n <= 1024");
        BSI_CHECK(is_2a3b(n) && n >= 8, BSI_E_UNSUPPORTED, "each n must be of the form 2^a 3^b");
        const double L = desc->length[d];
        BSI_CHECK(L == 0.0 || (std::isfinite(L) && L > 0.0), BSI_E_INVAL, "lengths must be > 0");
    }
    BSI_HIP(hipSetDevice(ctx->device));
    auto* f = new (std::nothrow) bsi_field();
    BSI_CHECK(f != nullptr, BSI_E_NOMEM, "host allocation failed");
    f->ctx = ctx;
    f->desc = *desc;
    f->N = desc->order;
    f->C = desc->ncomp;
    f->basis = desc->basis;
    const bool herm = desc->basis == BSI_BASIS_HERMITE;
    f->cs = herm ? 2 : 1;
    // B-spline / Lagrange: the stencil of cell c is padded indices [c, c + N);
    // Hermite: doubled indices [2c, 2c + 4) (value and derivative at c, c + 1)
    f->padlo = herm ? 0 : f->N / 2 - 1;
    for (int d = 0; d < 3; ++d) {
        f->n[d] = desc->n[d];
        f->gn[d] = f->cs * desc->n[d];
        f->P[d] = herm ? 2 * desc->n[d] + 2 : desc->n[d] + f->N - 1;
        f->L[d] = desc->length[d] == 0.0 ? 2.0 * 3.141592653589793 : desc->length[d];
        f->inv_h[d] = double(f->n[d]) / f->L[d];
    }
    {
        const int vec = int(16 / dtype_size(desc->coef));
        f->pitch2 = (f->P[2] * f->C + vec - 1) / vec * vec;
    }
    // rows padded to 16 B so tile rows load as 16-byte vectors; 4 KiB of slack
    // after the last row absorbs vector over-reads of partial tiles
    f->grid_bytes = size_t(f->P[0]) * f->P[1] * f->pitch2 * dtype_size(desc->coef) + 4096;
    if (hipMalloc(&f->grid, f->grid_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete f;
        set_error("coefficient grid allocation failed");
        return BSI_E_NOMEM;
    }
    if (hipMalloc(reinterpret_cast<void**>(&f->counters), 64) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(f->grid);
        delete f;
        set_error("counter allocation failed");
        return BSI_E_NOMEM;
    }
    if (hipMemset(f->counters, 0, 64) != hipSuccess || hipMemset(f->grid, 0, f->grid_bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(f->grid);
        (void)hipFree(f->counters);
        delete f;
        set_error("counter init failed");
        return BSI_E_DEVICE;
    }
    ctx->live_fields++;
    *out = f;
    return BSI_OK;
}

void bsi_field_destroy(bsi_field* f) {
    if (!f) return;
    (void)hipSetDevice(f->ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(f->grid);
    (void)hipFree(f->counters);
    f->ctx->live_fields--;
    delete f;
}

size_t bsi_field_bytes(const bsi_field* f) { return f ? f->grid_bytes + 64 : 0; }

bsi_status bsi_field_set_spectrum(bsi_field* f, const void* uhat, int32_t prec, void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(prec == BSI_F64 || prec == BSI_F32, BSI_E_INVAL, "spectrum precision must be F64 or F32");
    BSI_TRY(check_device_ptr(uhat, "uhat"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    return prefilter_run(f, uhat, prec, s);
}

bsi_status bsi_field_set_coefficients(bsi_field* f, const double* grid, void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_TRY(check_device_ptr(grid, "grid"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    return grid_from_dense(f, grid, s);
}

bsi_status bsi_field_get_coefficients(const bsi_field* f, double* grid, void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_TRY(check_device_ptr(grid, "grid"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    return grid_to_dense(f, grid, s);
}

bsi_status bsi_eval_ex(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                       const bsi_eval_config* cfg, void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    if (P == 0) return BSI_OK;
    BSI_TRY(check_device_ptr(pos, "pos"));
    BSI_TRY(check_device_ptr(u, "u"));
    if (grad) BSI_TRY(check_device_ptr(grad, "grad"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    bsi_eval_config c{};
    if (cfg) c = *cfg;
    else BSI_TRY(lookup_config(f->ctx, f, P, &c));
    BSI_CHECK(c.sort_tile >= 0 && c.sort_tile <= 1024, BSI_E_INVAL, "sort_tile out of range");
    return eval_run(f, pos, P, u, grad, c, s);
}

}  // extern "C"

struct bsi_eval_plan {
    bsi_field* f = nullptr;
    bsi_eval_config cfg{};
    int64_t cap = 0;
    int64_t P = -1;              // particles of the last binning (-1: none yet)
    const double* pos = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
};

extern "C" {

bsi_status bsi_eval_plan_create(bsi_field* f, int64_t max_particles, const bsi_eval_config* cfg,
                                bsi_eval_plan** out) {
    clear_error();
    BSI_CHECK(f && out, BSI_E_INVAL, "NULL argument");
    *out = nullptr;
    BSI_CHECK(max_particles >= 0 && max_particles < (int64_t(1) << 31), BSI_E_INVAL,
              "max_particles must be in [0, 2^31)");
    BSI_HIP(hipSetDevice(f->ctx->device));
    bsi_eval_config c{};
    if (cfg) c = *cfg;
    else BSI_TRY(lookup_config(f->ctx, f, std::max<int64_t>(max_particles, 1), &c));
    BSI_TRY(eval_check_config(c));
    auto* pl = new bsi_eval_plan;
    pl->f = f;
    pl->cfg = c;
    pl->cap = max_particles;
    pl->ws_bytes = max_particles > 0 ? eval_ws_bytes(f, max_particles, c) : 0;
    if (pl->ws_bytes && hipMalloc(&pl->ws, pl->ws_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete pl;
        set_error("cannot allocate the plan's workspace");
        return BSI_E_NOMEM;
    }
    *out = pl;
    return BSI_OK;
}

bsi_status bsi_eval_plan_bin(bsi_eval_plan* pl, const double* pos, int64_t P, void* stream) {
    clear_error();
    BSI_CHECK(pl != nullptr, BSI_E_INVAL, "plan is NULL");
    BSI_CHECK(P >= 0 && P <= pl->cap, BSI_E_INVAL, "P exceeds the plan's capacity");
    if (P > 0) BSI_TRY(check_device_ptr(pos, "pos"));
    bsi_field* f = pl->f;
    BSI_CHECK(eval_ws_bytes(f, P, pl->cfg) <= pl->ws_bytes, BSI_E_INVAL,
              "the binning of P particles needs more than the plan's workspace");
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    BSI_TRY(eval_bin_ws(f, pos, P, pl->cfg, s, pl->ws));
    pl->P = P;
    pl->pos = pos;
    return BSI_OK;
}

bsi_status bsi_eval_plan_run(bsi_eval_plan* pl, void* u, void* grad, void* stream) {
    clear_error();
    BSI_CHECK(pl != nullptr, BSI_E_INVAL, "plan is NULL");
    BSI_CHECK(pl->P >= 0, BSI_E_INVAL, "the plan has not binned any positions");
    if (pl->P == 0) return BSI_OK;
    BSI_TRY(check_device_ptr(u, "u"));
    if (grad) BSI_TRY(check_device_ptr(grad, "grad"));
    bsi_field* f = pl->f;
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    return eval_gather_ws(f, pl->pos, pl->P, u, grad, pl->cfg, s, pl->ws);
}

void bsi_eval_plan_destroy(bsi_eval_plan* pl) {
    if (!pl) return;
    if (pl->ws) {
        (void)hipSetDevice(pl->f->ctx->device);
        (void)hipDeviceSynchronize();   // no run may still read the workspace
        (void)hipFree(pl->ws);
    }
    delete pl;
}

bsi_status bsi_eval_hessian(bsi_field* f, const double* pos, int64_t P, void* u, void* grad, void* hess,
                            void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    if (P == 0) return BSI_OK;
    BSI_TRY(check_device_ptr(pos, "pos"));
    BSI_TRY(check_device_ptr(u, "u"));
    BSI_TRY(check_device_ptr(hess, "hess"));
    if (grad) BSI_TRY(check_device_ptr(grad, "grad"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    return hessian_run(f, pos, P, u, grad, hess, s);
}

bsi_status bsi_eval(bsi_field* f, const double* pos, int64_t P, void* u, void* grad, void* stream) {
    return bsi_eval_ex(f, pos, P, u, grad, nullptr, stream);
}

bsi_status bsi_debug_cells(bsi_field* f, const double* pos, int64_t P, int32_t* cell, double* t,
                           void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    if (P == 0) return BSI_OK;
    BSI_TRY(check_device_ptr(pos, "pos"));
    BSI_TRY(check_device_ptr(cell, "cell"));
    BSI_TRY(check_device_ptr(t, "t"));
    BSI_HIP(hipSetDevice(f->ctx->device));
    return debug_cells_run(f, pos, P, cell, t, pick_stream(f->ctx, stream));
}

bsi_status bsi_debug_bins(bsi_field* f, const double* pos, int64_t P, int32_t tile, uint32_t* hist,
                          uint32_t* offs, uint32_t* perm, double* pos_sorted, int64_t* nbuckets, void* stream) {
    clear_error();
    BSI_CHECK(f != nullptr && nbuckets != nullptr, BSI_E_INVAL, "NULL argument");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    const int nmax = std::max(f->n[0], std::max(f->n[1], f->n[2]));
    BSI_CHECK(tile >= 1 && tile >= (nmax + 255) / 256, BSI_E_INVAL,
              "tile must be >= 1 and >= ceil(max(n) / 256)");
    *nbuckets = int64_t(bsi::bin_bucket_count(f, tile) + 1);
    if (hist == nullptr) return BSI_OK;
    BSI_TRY(check_device_ptr(hist, "hist"));
    BSI_TRY(check_device_ptr(offs, "offs"));
    if (P > 0) {
        BSI_TRY(check_device_ptr(pos, "pos"));
        BSI_TRY(check_device_ptr(perm, "perm"));
        BSI_TRY(check_device_ptr(pos_sorted, "pos_sorted"));
    }
    BSI_HIP(hipSetDevice(f->ctx->device));
    return debug_bins_run(f, pos, P, tile, hist, offs, perm, pos_sorted, pick_stream(f->ctx, stream));
}

bsi_status bsi_field_stats(bsi_field* f, int64_t* nonfinite) {
    clear_error();
    BSI_CHECK(f && nonfinite, BSI_E_INVAL, "NULL argument");
    BSI_HIP(hipSetDevice(f->ctx->device));
    if (f->last_stream) BSI_HIP(hipStreamSynchronize(f->last_stream));
    else BSI_HIP(hipDeviceSynchronize());
    unsigned long long v = 0;
    BSI_HIP(hipMemcpy(&v, f->counters, sizeof(v), hipMemcpyDeviceToHost));
    *nonfinite = int64_t(v);
    return BSI_OK;
}

}  // extern "C"
