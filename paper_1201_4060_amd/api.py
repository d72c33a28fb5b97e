"""Thin object wrappers over the C ABI for torch device tensors.

Only marshalling: tensors are passed as raw device pointers and the current
torch stream as the HIP stream.  Shapes and dtypes are checked here so that a
wrong tensor fails before it reaches the library.
"""
import torch

from . import _bsi


def _stream():
    return torch.cuda.current_stream().cuda_stream


class Context:
    """bsi_ctx on one HIP device."""

    def __init__(self, device=0, stream=None):
        self.device = device
        self.handle = _bsi.bsi_ctx_create(device, stream)

    def close(self):
        if self.handle:
            _bsi.bsi_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Field:
    """bsi_field: a coefficient grid of a scalar or 3-component periodic field."""

    def __init__(self, ctx, n, ncomp, order, coef=_bsi.BSI_F32, prefilter=_bsi.BSI_PREFILTER_L2OPT,
                 length=(0.0, 0.0, 0.0), basis=_bsi.BSI_BASIS_BSPLINE):
        self.ctx = ctx
        self.n = (n, n, n) if isinstance(n, int) else tuple(n)
        self.ncomp, self.order, self.coef, self.basis = ncomp, order, coef, basis
        self.desc = _bsi.make_desc(self.n, ncomp, order, coef, prefilter, length, basis)
        self.handle = _bsi.bsi_field_create(ctx.handle, self.desc)

    @property
    def out_dtype(self):
        return torch.float64 if self.coef == _bsi.BSI_F64 else torch.float32

    def close(self):
        if self.handle:
            _bsi.bsi_field_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def nbytes(self):
        return _bsi.bsi_field_bytes(self.handle)

    def set_spectrum(self, uhat):
        """uhat: complex128/complex64 device tensor [ncomp][n0][n1][n2/2+1]."""
        n0, n1, n2 = self.n
        assert uhat.is_cuda and uhat.is_contiguous()
        assert tuple(uhat.shape) == (self.ncomp, n0, n1, n2 // 2 + 1), uhat.shape
        prec = {torch.complex128: _bsi.BSI_F64, torch.complex64: _bsi.BSI_F32}[uhat.dtype]
        _bsi.bsi_field_set_spectrum(self.handle, uhat, prec, _stream())

    @property
    def grid_shape(self):
        """Shape of the dense coefficient grid: [ncomp][n0][n1][n2], or for a
        Hermite field the interleaved [ncomp][2 n0][2 n1][2 n2]."""
        s = 2 if self.basis == _bsi.BSI_BASIS_HERMITE else 1
        return (self.ncomp,) + tuple(s * v for v in self.n)

    def set_coefficients(self, grid):
        """grid: float64 device tensor of shape grid_shape."""
        assert grid.is_cuda and grid.is_contiguous() and grid.dtype == torch.float64
        assert tuple(grid.shape) == self.grid_shape
        _bsi.bsi_field_set_coefficients(self.handle, grid, _stream())

    def get_coefficients(self):
        out = torch.empty(self.grid_shape, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        _bsi.bsi_field_get_coefficients(self.handle, out, _stream())
        return out

    def eval(self, pos, grad=True, cfg=None, out=None):
        """pos: float64 device tensor [P][3] -> (u [P][C], grad [P][C][3] or None)."""
        assert pos.is_cuda and pos.is_contiguous() and pos.dtype == torch.float64
        assert pos.dim() == 2 and pos.shape[1] == 3
        P = pos.shape[0]
        if out is None:
            u = torch.empty((P, self.ncomp), dtype=self.out_dtype, device=pos.device)
            g = torch.empty((P, self.ncomp, 3), dtype=self.out_dtype, device=pos.device) if grad else None
        else:
            u, g = out
        if P == 0:
            return u, g
        if cfg is None:
            _bsi.bsi_eval(self.handle, pos, P, u, g, _stream())
        else:
            _bsi.bsi_eval_ex(self.handle, pos, P, u, g, cfg, _stream())
        return u, g

    def eval_hessian(self, pos, grad=True, out=None):
        """pos: float64 device tensor [P][3] -> (u [P][C], grad [P][C][3] or None,
        hess [P][C][6]: d2/dx_i dx_j for (i, j) = 00, 01, 02, 11, 12, 22)."""
        assert pos.is_cuda and pos.is_contiguous() and pos.dtype == torch.float64
        assert pos.dim() == 2 and pos.shape[1] == 3
        P = pos.shape[0]
        if out is None:
            u = torch.empty((P, self.ncomp), dtype=self.out_dtype, device=pos.device)
            g = torch.empty((P, self.ncomp, 3), dtype=self.out_dtype, device=pos.device) if grad else None
            h = torch.empty((P, self.ncomp, 6), dtype=self.out_dtype, device=pos.device)
        else:
            u, g, h = out
        if P:
            _bsi.bsi_eval_hessian(self.handle, pos, P, u, g, h, _stream())
        return u, g, h

    def debug_cells(self, pos):
        P = pos.shape[0]
        cell = torch.empty((P, 3), dtype=torch.int32, device=pos.device)
        t = torch.empty((P, 3), dtype=torch.float64, device=pos.device)
        if P:
            _bsi.bsi_debug_cells(self.handle, pos, P, cell, t, _stream())
        return cell, t

    def debug_bins(self, pos, tile):
        """The evaluation's binning of pos by Morton tiles of `tile` cells:
        (hist, offs, perm, pos_sorted) device tensors (bsi_debug_bins)."""
        P = pos.shape[0]
        nb = _bsi.bsi_debug_bins(self.handle, None, P, tile, None, None, None, None, _stream())
        hist = torch.empty(nb, dtype=torch.int32, device=pos.device)
        offs = torch.empty(nb, dtype=torch.int32, device=pos.device)
        perm = torch.empty(P, dtype=torch.int32, device=pos.device)
        ps = torch.empty((P, 3), dtype=torch.float64, device=pos.device)
        _bsi.bsi_debug_bins(self.handle, pos, P, tile, hist, offs, perm, ps, _stream())
        return hist, offs, perm, ps

    def nonfinite_count(self):
        return _bsi.bsi_field_stats(self.handle)


class EvalPlan:
    """bsi_eval_plan: an evaluation of `field` split into a binning of the
    positions (bin, on any stream) and the gather from it (run), for up to
    `max_particles` positions.  The positions passed to bin must stay alive
    and unchanged while runs use them."""

    def __init__(self, field, max_particles, cfg=None):
        self.field = field
        self.handle = _bsi.bsi_eval_plan_create(field.handle, max_particles, cfg)
        self._pos = None

    def bin(self, pos):
        assert pos.is_cuda and pos.is_contiguous() and pos.dtype == torch.float64
        assert pos.dim() == 2 and pos.shape[1] == 3
        _bsi.bsi_eval_plan_bin(self.handle, pos, pos.shape[0], _stream())
        self._pos = pos

    def run(self, grad=True, out=None):
        """-> (u [P][C], grad [P][C][3] or None) at the last binned positions."""
        assert self._pos is not None, "bin positions first"
        P, f = self._pos.shape[0], self.field
        if out is None:
            u = torch.empty((P, f.ncomp), dtype=f.out_dtype, device=self._pos.device)
            g = torch.empty((P, f.ncomp, 3), dtype=f.out_dtype, device=self._pos.device) if grad else None
        else:
            u, g = out
        _bsi.bsi_eval_plan_run(self.handle, u, g, _stream())
        return u, g

    def close(self):
        if self.handle:
            _bsi.bsi_eval_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """bsi_batch: evaluations of several fields run by one persistent gather.

    items: list of (field, pos, u, grad) with device tensors (grad may be None
    for every item).  cfgs: optional list of EvalConfig, one per item.  The
    tensors must stay alive and in place while the batch exists.
    """

    def __init__(self, ctx, items, cfgs=None):
        self.ctx = ctx
        self._keep = items
        raw = []
        for field, pos, u, grad in items:
            assert pos.is_cuda and pos.is_contiguous() and pos.dtype == torch.float64
            assert pos.dim() == 2 and pos.shape[1] == 3
            P = pos.shape[0]
            assert u.shape == (P, field.ncomp) and u.dtype == field.out_dtype and u.is_contiguous()
            if grad is not None:
                assert grad.shape == (P, field.ncomp, 3) and grad.dtype == field.out_dtype
                assert grad.is_contiguous()
            raw.append((field.handle, pos, P, u, grad))
        self.handle = _bsi.bsi_batch_create(ctx.handle, raw, cfgs)

    def run(self, use_graph=False):
        _bsi.bsi_batch_run(self.handle, use_graph, _stream())

    def item_config(self, i):
        return _bsi.bsi_batch_item_config(self.handle, i)

    def nbytes(self):
        return _bsi.bsi_batch_bytes(self.handle)

    def close(self):
        if self.handle:
            _bsi.bsi_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """bsi_server: resident fields served to particle-query requests.

    Host tensors passed to submit() must be CPU tensors (pinned for overlap);
    they are kept referenced here until the request is waited for.
    """

    def __init__(self, ctx, hbm_budget, max_slots, queue_capacity=1 << 20):
        self.ctx = ctx
        self.handle = _bsi.bsi_server_create(ctx.handle, hbm_budget, max_slots, queue_capacity)
        self.fields = {}
        self._keep = {}

    def add_field(self, field_id, field):
        _bsi.bsi_server_add_field(self.handle, field_id, field.handle)
        self.fields[field_id] = field

    def submit(self, field_id, pos, u, grad=None):
        f = self.fields[field_id]
        assert not pos.is_cuda and pos.is_contiguous() and pos.dtype == torch.float64
        P = pos.shape[0]
        assert u.shape == (P, f.ncomp) and u.dtype == f.out_dtype and not u.is_cuda and u.is_contiguous()
        if grad is not None:
            assert grad.shape == (P, f.ncomp, 3) and grad.dtype == f.out_dtype and not grad.is_cuda
            assert grad.is_contiguous()
        t = _bsi.bsi_server_submit(self.handle, field_id, pos, P, u, grad)
        self._keep[t] = (pos, u, grad)
        return t

    def wait(self, ticket):
        try:
            return _bsi.bsi_server_wait(self.handle, ticket)
        finally:
            self._keep.pop(ticket, None)

    def poll(self, ticket):
        done, lat = _bsi.bsi_server_poll(self.handle, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done, lat

    def drain(self):
        _bsi.bsi_server_drain(self.handle)

    def stats(self):
        return _bsi.bsi_server_stats(self.handle)

    def reset_stats(self):
        _bsi.bsi_server_reset_stats(self.handle)

    def close(self):
        if self.handle:
            _bsi.bsi_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
