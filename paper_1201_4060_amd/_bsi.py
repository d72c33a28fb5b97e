"""ctypes binding of libbsi.so: the C ABI of include/bsi.h, one Python function
per C entry point with the same name.  Argument marshalling only: every step of
the method runs in the HIP library.  Raises BsiError on a non-OK status.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsi.so")

BSI_OK = 0
STATUS_NAMES = {0: "BSI_OK", 1: "BSI_E_INVAL", 2: "BSI_E_NOMEM", 3: "BSI_E_UNSUPPORTED",
                4: "BSI_E_DEVICE", 5: "BSI_E_BUSY", 6: "BSI_E_CANCELLED"}
BSI_F64, BSI_F32, BSI_BF16 = 0, 1, 2
BSI_PREFILTER_L2OPT, BSI_PREFILTER_INTERP, BSI_PREFILTER_NONE = 0, 1, 2
BSI_BASIS_BSPLINE, BSI_BASIS_LAGRANGE, BSI_BASIS_HERMITE = 0, 1, 2


class BsiError(RuntimeError):
    def __init__(self, status, where, msg):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


class FieldDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ncomp", ctypes.c_int32), ("order", ctypes.c_int32),
                ("coef", ctypes.c_int32), ("prefilter", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("length", ctypes.c_double * 3)]


class EvalConfig(ctypes.Structure):
    _fields_ = [("sort_tile", ctypes.c_int32), ("block", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("tiles_per_group", ctypes.c_int32), ("tile_block", ctypes.c_int32),
                ("item_rounds", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class ServerReport(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("p50_ns", ctypes.c_double), ("p99_ns", ctypes.c_double),
                ("device_p50_ns", ctypes.c_double), ("device_p99_ns", ctypes.c_double),
                ("points", ctypes.c_int64), ("points_per_s", ctypes.c_double),
                ("max_inflight", ctypes.c_int64), ("peak_arena_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class EvalItem(ctypes.Structure):
    _fields_ = [("field", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("P", ctypes.c_int64),
                ("u", ctypes.c_void_p), ("grad", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libbsi.so; fail loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1201_4060_amd.build`")
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


VP = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
ST = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "bsi_ctx_create": (ST, [ctypes.c_int, VP, ctypes.POINTER(VP)]),
    "bsi_ctx_destroy": (None, [VP]),
    "bsi_last_error": (ctypes.c_char_p, []),
    "bsi_version": (ctypes.c_char_p, []),
    "bsi_field_create": (ST, [VP, ctypes.POINTER(FieldDesc), ctypes.POINTER(VP)]),
    "bsi_field_destroy": (None, [VP]),
    "bsi_field_bytes": (ctypes.c_size_t, [VP]),
    "bsi_field_set_spectrum": (ST, [VP, VP, I32, VP]),
    "bsi_field_set_coefficients": (ST, [VP, VP, VP]),
    "bsi_field_get_coefficients": (ST, [VP, VP, VP]),
    "bsi_eval": (ST, [VP, VP, I64, VP, VP, VP]),
    "bsi_eval_ex": (ST, [VP, VP, I64, VP, VP, ctypes.POINTER(EvalConfig), VP]),
    "bsi_eval_static": (ST, [VP, VP, I64, VP, VP, ctypes.POINTER(EvalConfig), VP]),
    "bsi_eval_plan_create": (ST, [VP, I64, ctypes.POINTER(EvalConfig), ctypes.POINTER(VP)]),
    "bsi_eval_plan_bin": (ST, [VP, VP, I64, VP]),
    "bsi_eval_plan_run": (ST, [VP, VP, VP, VP]),
    "bsi_eval_plan_destroy": (None, [VP]),
    "bsi_debug_cells": (ST, [VP, VP, I64, VP, VP, VP]),
    "bsi_eval_hessian": (ST, [VP, VP, I64, VP, VP, VP, VP]),
    "bsi_debug_bins": (ST, [VP, VP, I64, I32, VP, VP, VP, VP, ctypes.POINTER(I64), VP]),
    "bsi_field_stats": (ST, [VP, ctypes.POINTER(I64)]),
    "bsi_ctx_set_timing": (ST, [VP, I32]),
    "bsi_ctx_read_timing": (ST, [VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(I64)]),
    "bsi_ctx_reset_timing": (ST, [VP]),
    "bsi_batch_create": (ST, [VP, ctypes.POINTER(EvalItem), I32, ctypes.POINTER(EvalConfig),
                              ctypes.POINTER(VP)]),
    "bsi_batch_run": (ST, [VP, I32, VP]),
    "bsi_batch_item_config": (ST, [VP, I32, ctypes.POINTER(EvalConfig)]),
    "bsi_batch_bytes": (ctypes.c_size_t, [VP]),
    "bsi_batch_destroy": (None, [VP]),
    "bsi_eval_batch": (ST, [VP, ctypes.POINTER(EvalItem), I32, VP]),
    "bsi_tune": (ST, [VP, I64, ctypes.c_uint64, ctypes.c_char_p, ctypes.POINTER(EvalConfig),
                      ctypes.POINTER(ctypes.c_double)]),
    "bsi_ctx_load_tuning": (ST, [VP, ctypes.c_char_p]),
    "bsi_ctx_lookup_config": (ST, [VP, VP, I64, ctypes.POINTER(EvalConfig)]),
    "bsi_server_create": (ST, [VP, ctypes.POINTER(ServerConfig), ctypes.POINTER(VP)]),
    "bsi_server_add_field": (ST, [VP, I32, VP]),
    "bsi_server_submit": (ST, [VP, I32, VP, I64, VP, VP, ctypes.POINTER(ctypes.c_uint64)]),
    "bsi_server_poll": (ST, [VP, ctypes.c_uint64, ctypes.POINTER(I32), ctypes.POINTER(I64)]),
    "bsi_server_wait": (ST, [VP, ctypes.c_uint64, ctypes.POINTER(I64)]),
    "bsi_server_drain": (ST, [VP]),
    "bsi_server_stats": (ST, [VP, ctypes.POINTER(ServerReport)]),
    "bsi_server_reset_stats": (ST, [VP]),
    "bsi_server_destroy": (None, [VP]),
    "bsi_synth_kolmogorov": (ST, [VP, I32, I32, ctypes.c_uint64, I32, I32, VP, VP]),
    "bsi_ctx_trim": (ST, [VP]),
    "bsi_fill_uniform_positions": (ST, [VP, ctypes.c_uint64, I64, ctypes.POINTER(ctypes.c_double), VP, VP]),
}


def _declare(L):
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args


def exported_symbols():
    """Names of SIGNATURES entries the loaded library exports."""
    L = lib()
    return [n for n in SIGNATURES if hasattr(L, n)]


def _check(status, where):
    if status != BSI_OK:
        msg = lib().bsi_last_error()
        raise BsiError(status, where, msg.decode() if msg else "")


def _ptr(x):
    """Raw address of a torch tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


# ---- one function per C entry point ---------------------------------------

def bsi_ctx_create(device=0, stream=None):
    out = VP()
    _check(lib().bsi_ctx_create(device, stream, ctypes.byref(out)), "bsi_ctx_create")
    return out.value


def bsi_ctx_destroy(ctx):
    lib().bsi_ctx_destroy(ctx)


def bsi_last_error():
    v = lib().bsi_last_error()
    return v.decode() if v else ""


def bsi_version():
    return lib().bsi_version().decode()


def make_desc(n, ncomp, order, coef=BSI_F32, prefilter=BSI_PREFILTER_L2OPT, length=(0.0, 0.0, 0.0),
              basis=BSI_BASIS_BSPLINE):
    if isinstance(n, int):
        n = (n, n, n)
    d = FieldDesc()
    d.n = (ctypes.c_int32 * 3)(*n)
    d.ncomp, d.order, d.coef, d.prefilter, d.basis = ncomp, order, coef, prefilter, basis
    d.length = (ctypes.c_double * 3)(*length)
    return d


def bsi_field_create(ctx, desc):
    out = VP()
    _check(lib().bsi_field_create(ctx, ctypes.byref(desc), ctypes.byref(out)), "bsi_field_create")
    return out.value


def bsi_field_destroy(field):
    lib().bsi_field_destroy(field)


def bsi_field_bytes(field):
    return lib().bsi_field_bytes(field)


def bsi_field_set_spectrum(field, uhat, prec, stream=None):
    _check(lib().bsi_field_set_spectrum(field, _ptr(uhat), prec, stream), "bsi_field_set_spectrum")


def bsi_field_set_coefficients(field, grid, stream=None):
    _check(lib().bsi_field_set_coefficients(field, _ptr(grid), stream), "bsi_field_set_coefficients")


def bsi_field_get_coefficients(field, grid, stream=None):
    _check(lib().bsi_field_get_coefficients(field, _ptr(grid), stream), "bsi_field_get_coefficients")


def bsi_eval(field, pos, P, u, grad=None, stream=None):
    _check(lib().bsi_eval(field, _ptr(pos), P, _ptr(u), _ptr(grad), stream), "bsi_eval")


def bsi_eval_ex(field, pos, P, u, grad=None, cfg=None, stream=None):
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(lib().bsi_eval_ex(field, _ptr(pos), P, _ptr(u), _ptr(grad), c, stream), "bsi_eval_ex")


def bsi_eval_static(field, pos, P, u, grad=None, cfg=None, stream=None):
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(lib().bsi_eval_static(field, _ptr(pos), P, _ptr(u), _ptr(grad), c, stream), "bsi_eval_static")


def bsi_eval_plan_create(field, max_particles, cfg=None):
    out = VP()
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(lib().bsi_eval_plan_create(field, max_particles, c, ctypes.byref(out)), "bsi_eval_plan_create")
    return out.value


def bsi_eval_plan_bin(plan, pos, P, stream=None):
    _check(lib().bsi_eval_plan_bin(plan, _ptr(pos), P, stream), "bsi_eval_plan_bin")


def bsi_eval_plan_run(plan, u, grad=None, stream=None):
    _check(lib().bsi_eval_plan_run(plan, _ptr(u), _ptr(grad), stream), "bsi_eval_plan_run")


def bsi_eval_plan_destroy(plan):
    lib().bsi_eval_plan_destroy(plan)


def bsi_eval_hessian(field, pos, P, u, grad, hess, stream=None):
    _check(lib().bsi_eval_hessian(field, _ptr(pos), P, _ptr(u), _ptr(grad), _ptr(hess), stream),
           "bsi_eval_hessian")


def bsi_debug_cells(field, pos, P, cell, t, stream=None):
    _check(lib().bsi_debug_cells(field, _ptr(pos), P, _ptr(cell), _ptr(t), stream), "bsi_debug_cells")


def bsi_debug_bins(field, pos, P, tile, hist, offs, perm, pos_sorted, stream=None):
    """Returns the bucket count; fills the four arrays unless hist is None."""
    n = I64()
    _check(lib().bsi_debug_bins(field, _ptr(pos), P, tile, _ptr(hist), _ptr(offs), _ptr(perm),
                                _ptr(pos_sorted), ctypes.byref(n), stream), "bsi_debug_bins")
    return n.value


def bsi_field_stats(field):
    v = I64()
    _check(lib().bsi_field_stats(field, ctypes.byref(v)), "bsi_field_stats")
    return v.value


def bsi_ctx_set_timing(ctx, enabled):
    _check(lib().bsi_ctx_set_timing(ctx, 1 if enabled else 0), "bsi_ctx_set_timing")


def bsi_ctx_read_timing(ctx, stage):
    ms = ctypes.c_double()
    n = I64()
    _check(lib().bsi_ctx_read_timing(ctx, stage.encode(), ctypes.byref(ms), ctypes.byref(n)),
           "bsi_ctx_read_timing")
    return ms.value, n.value


def bsi_ctx_reset_timing(ctx):
    _check(lib().bsi_ctx_reset_timing(ctx), "bsi_ctx_reset_timing")


def make_items(items):
    """[(field, pos, P, u, grad)] -> ctypes array of EvalItem."""
    arr = (EvalItem * len(items))()
    for i, (field, pos, P, u, grad) in enumerate(items):
        arr[i].field, arr[i].pos, arr[i].P = field, _ptr(pos), P
        arr[i].u, arr[i].grad = _ptr(u), _ptr(grad)
    return arr


def bsi_batch_create(ctx, items, cfgs=None):
    arr = make_items(items)
    c = None
    if cfgs is not None:
        c = (EvalConfig * len(items))(*cfgs)
    out = VP()
    _check(lib().bsi_batch_create(ctx, arr, len(items), c, ctypes.byref(out)), "bsi_batch_create")
    return out.value


def bsi_batch_run(batch, use_graph=False, stream=None):
    _check(lib().bsi_batch_run(batch, 1 if use_graph else 0, stream), "bsi_batch_run")


def bsi_batch_item_config(batch, item):
    c = EvalConfig()
    _check(lib().bsi_batch_item_config(batch, item, ctypes.byref(c)), "bsi_batch_item_config")
    return c


def bsi_batch_bytes(batch):
    return lib().bsi_batch_bytes(batch)


def bsi_batch_destroy(batch):
    lib().bsi_batch_destroy(batch)


def bsi_eval_batch(ctx, items, stream=None):
    arr = make_items(items)
    _check(lib().bsi_eval_batch(ctx, arr, len(items), stream), "bsi_eval_batch")


def bsi_tune(field, P, seed=0, db_path=None):
    c = EvalConfig()
    us = ctypes.c_double()
    _check(lib().bsi_tune(field, P, seed, db_path.encode() if db_path else None, ctypes.byref(c),
                          ctypes.byref(us)), "bsi_tune")
    return c, us.value


def bsi_ctx_load_tuning(ctx, db_path):
    _check(lib().bsi_ctx_load_tuning(ctx, db_path.encode()), "bsi_ctx_load_tuning")


def bsi_ctx_lookup_config(ctx, field, P):
    c = EvalConfig()
    _check(lib().bsi_ctx_lookup_config(ctx, field, P, ctypes.byref(c)), "bsi_ctx_lookup_config")
    return c


def bsi_fill_uniform_positions(ctx, seed, P, length, pos, stream=None):
    L = (ctypes.c_double * 3)(*length)
    _check(lib().bsi_fill_uniform_positions(ctx, seed, P, L, _ptr(pos), stream),
           "bsi_fill_uniform_positions")


def bsi_server_create(ctx, hbm_budget, max_slots, queue_capacity=1 << 20):
    cfg = ServerConfig()
    cfg.hbm_budget, cfg.max_slots, cfg.queue_capacity = hbm_budget, max_slots, queue_capacity
    out = VP()
    _check(lib().bsi_server_create(ctx, ctypes.byref(cfg), ctypes.byref(out)), "bsi_server_create")
    return out.value


def bsi_server_add_field(server, field_id, field):
    _check(lib().bsi_server_add_field(server, field_id, field), "bsi_server_add_field")


def bsi_server_submit(server, field_id, pos_host, P, u_host, grad_host=None):
    t = ctypes.c_uint64()
    _check(lib().bsi_server_submit(server, field_id, _ptr(pos_host), P, _ptr(u_host), _ptr(grad_host),
                                   ctypes.byref(t)), "bsi_server_submit")
    return t.value


def bsi_server_poll(server, ticket):
    """(done, latency_ns); raises the request's own error once it is done."""
    d = I32()
    lat = I64()
    _check(lib().bsi_server_poll(server, ticket, ctypes.byref(d), ctypes.byref(lat)), "bsi_server_poll")
    return bool(d.value), lat.value


def bsi_server_wait(server, ticket):
    lat = I64()
    _check(lib().bsi_server_wait(server, ticket, ctypes.byref(lat)), "bsi_server_wait")
    return lat.value


def bsi_server_drain(server):
    _check(lib().bsi_server_drain(server), "bsi_server_drain")


def bsi_server_stats(server):
    r = ServerReport()
    _check(lib().bsi_server_stats(server, ctypes.byref(r)), "bsi_server_stats")
    return r.as_dict()


def bsi_server_reset_stats(server):
    _check(lib().bsi_server_reset_stats(server), "bsi_server_reset_stats")


def bsi_server_destroy(server):
    lib().bsi_server_destroy(server)


def bsi_synth_kolmogorov(ctx, n, ncomp, seed, out, divergence_free=None, stream=None):
    """out: complex128 or complex64 device tensor [ncomp][n][n][n/2+1]."""
    if divergence_free is None:
        divergence_free = ncomp == 3
    prec = BSI_F64 if str(out.dtype) == "torch.complex128" else BSI_F32
    _check(lib().bsi_synth_kolmogorov(ctx, n, ncomp, seed, 1 if divergence_free else 0, prec, _ptr(out),
                                      stream), "bsi_synth_kolmogorov")


def bsi_ctx_trim(ctx):
    _check(lib().bsi_ctx_trim(ctx), "bsi_ctx_trim")
