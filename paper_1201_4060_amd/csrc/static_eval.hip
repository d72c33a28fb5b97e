// Evaluation with a statically allocated device workspace, for callers that
// cannot allocate device memory.  The binning workspace of bsi_eval_ex comes
// from one file-scope device array per GPU instead of the context's
// per-stream workspaces; everything else (kernels, arithmetic, configuration)
// is the evaluation of eval.hip, so results are bitwise those of bsi_eval_ex.
#include <array>
#include <mutex>
#include <string>

#include "common.hpp"

namespace bsi {

constexpr size_t STATIC_SCRATCH_BYTES = size_t(128) << 20;

// The device array.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is looked up per device at context
// creation (static_scratch_init) and only that address is used.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
std::array<void*, MAX_DEVICES> g_scratch_ptr{};

void* scratch_ptr(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

// Once per device, with `device` current: resolve the device address of the
// array.  Called by bsi_ctx_create.
bsi_status static_scratch_init(int device) {
    BSI_CHECK(device >= 0 && device < MAX_DEVICES, BSI_E_UNSUPPORTED, "device index beyond the static table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return BSI_OK;
    void* p = nullptr;
    BSI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BSI_CHECK(p != nullptr && reinterpret_cast<uintptr_t>(p) % 256 == 0, BSI_E_DEVICE,
              "static scratch has no aligned device address");
    g_scratch_ptr[device] = p;
    return BSI_OK;
}

}  // namespace bsi

extern "C" bsi_status bsi_eval_static(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                                      const bsi_eval_config* cfg, void* stream) {
    using namespace bsi;
    clear_error();
    BSI_CHECK(f != nullptr, BSI_E_INVAL, "field is NULL");
    BSI_CHECK(P >= 0 && P < (int64_t(1) << 31), BSI_E_INVAL, "P must be in [0, 2^31)");
    if (P == 0) return BSI_OK;
    BSI_TRY(check_device_ptr_ex(pos, "pos"));
    BSI_TRY(check_device_ptr_ex(u, "u"));
    if (grad) BSI_TRY(check_device_ptr_ex(grad, "grad"));
    bsi_eval_config c{};
    if (cfg) c = *cfg;
    else BSI_TRY(lookup_config(f->ctx, f, P, &c));
    BSI_CHECK(c.sort_tile >= 0 && c.sort_tile <= 1024, BSI_E_INVAL, "sort_tile out of range");
    const size_t need = eval_ws_bytes(f, P, c);
    BSI_CHECK(need <= STATIC_SCRATCH_BYTES, BSI_E_INVAL,
              "bsi_eval_static: this call needs " + std::to_string(need) +
                  " bytes of workspace, more than the static maximum of " +
                  std::to_string(STATIC_SCRATCH_BYTES) + " bytes (use fewer particles or bsi_eval_ex)");
    void* ws = scratch_ptr(f->ctx->device);
    BSI_CHECK(ws != nullptr, BSI_E_DEVICE, "static scratch of this device was not set up");
    BSI_HIP(hipSetDevice(f->ctx->device));
    hipStream_t s = pick_stream(f->ctx, stream);
    f->last_stream = s;
    UntimedScope untimed;  // stage timing would create events
    return eval_run_ws(f, pos, P, u, grad, c, s, need ? ws : nullptr);
}
