"""Python binding of libjacobi.so, the gfx950 over-decomposed Jacobi library.

Argument marshalling only: every step of the sweep, halo exchange, residual,
scatter/gather and source scaling runs in the library's HIP kernels.  PyTorch
provides device memory (the workspace and user tensors) and the HIP stream.
There is no CPU fallback: if the library is not built, or no GPU is visible
when a handle is created, an exception is raised.

Module-level functions carry the C names (jacobi_create, jacobi_sweep, ...)
and return Python values, raising JacobiError on a non-zero status.  `Solver`
is a small convenience wrapper that owns a torch workspace.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjacobi.so")

JACOBI_F32 = 0
JACOBI_F64 = 1
JACOBI_FLAG_EXPLICIT_HALO = 1
JACOBI_FLAG_NT_STORES = 2
JACOBI_FLAG_DEEP_PREFETCH = 4
JACOBI_FLAG_OVERLAP = 8

JACOBI_RUNNING = 0
JACOBI_CONVERGED = 1
JACOBI_MAX_SWEEPS = 2
JACOBI_DIVERGED = 3
STATUS_NAMES = {0: "running", 1: "converged", 2: "max_sweeps", 3: "diverged"}

JACOBI_OK = 0
JACOBI_E_INVAL = -1
JACOBI_E_NOMEM = -2
JACOBI_E_HIP = -3
JACOBI_E_STATE = -4
JACOBI_E_UNSUPPORTED = -5

_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double
_PI64 = ctypes.POINTER(ctypes.c_int64)

# name -> argtypes (all return int status unless listed in _RESTYPES)
_SIGNATURES = {
    "jacobi_workspace_bytes": [_I, _PI64, _PI64, _I, ctypes.POINTER(_SZ)],
    "jacobi_create": [_I, _PI64, _PI64, _I, _P, _SZ, _P, ctypes.POINTER(_P)],
    "jacobi_deep_workspace_bytes": [_I, _PI64, _PI64, _I, _I, ctypes.POINTER(_SZ)],
    "jacobi_deep_create": [_I, _PI64, _PI64, _I, _I, _P, _SZ, _P, ctypes.POINTER(_P)],
    "jacobi_get_halo": [_P, ctypes.POINTER(_I)],
    "jacobi_destroy": [_P],
    "jacobi_set_stream": [_P, _P],
    "jacobi_get_layout": [_P, _PI64, _PI64],
    "jacobi_set_state": [_P, _P],
    "jacobi_get_state": [_P, _P],
    "jacobi_set_source": [_P, _P, _D],
    "jacobi_halo_exchange": [_P],
    "jacobi_sweep": [_P, _I64],
    "jacobi_residual_async": [_P, _P],
    "jacobi_residual": [_P, ctypes.POINTER(_D)],
    "jacobi_solve": [_P, _I64, _I64, _P],
    "jacobi_solve_noalloc": [_I, _PI64, _PI64, _I, _P, _P, _D, _I64, _I64, _P, _P, _P],
    "jacobi_set_tuning": [_P, _I, _I, _I],
    "jacobi_get_tuning": [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "jacobi_max_depth": [_I, _I],
    "jacobi_batch_workspace_bytes": [_I, _PI64, _I64, _I, ctypes.POINTER(_SZ)],
    "jacobi_batch_create": [_I, _PI64, _I64, _I, _P, _SZ, _P, ctypes.POINTER(_P)],
    "jacobi_batch_destroy": [_P],
    "jacobi_batch_set_grid": [_P, _I, _P, _P, _D],
    "jacobi_batch_get_grid": [_P, _I, _P],
    "jacobi_batch_set_tuning": [_P, _I, _I, _I],
    "jacobi_batch_get_tuning": [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "jacobi_batch_autotune": [_P, _I64, ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "jacobi_batch_solve": [_P, _D, _I64, _I64, _PI64, ctypes.POINTER(_D), ctypes.POINTER(_I)],
    "jacobi_forward_ckpt": [_P, _I64, _I64, _P],
    "jacobi_adjoint": [_P, _I64, _I64, _P, _D, _P, _P],
    "jacobi_adjoint_begin": [_P, _P, _P],
    "jacobi_adjoint_sweep": [_P, _I64],
    "jacobi_adjoint_end": [_P, _D, _P, _P],
    "jacobi_profile": [_P, _I],
    "jacobi_profile_read": [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(_I64),
                            ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "jacobi_autotune": [_P, _I64, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "jacobi_strerror": [_I],
    "jacobi_last_error": [],
}
_RESTYPES = {"jacobi_strerror": ctypes.c_char_p, "jacobi_last_error": ctypes.c_char_p}


class JacobiError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


def lib():
    """The loaded libjacobi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libjacobi.so is not built (expected at %s); run "
                              "__graft_entry__.build() or python -m paper_2303_02543_amd.build"
                              % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _RESTYPES.get(name, ctypes.c_int)
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(status):
    if status != JACOBI_OK:
        msg = lib().jacobi_last_error().decode(errors="replace")
        raise JacobiError(status, msg or lib().jacobi_strerror(status).decode())
    return status


def _arr64(vals):
    a = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return a


def dtype_code(dtype):
    import torch
    if dtype in (torch.float32, "float32", "f32"):
        return JACOBI_F32
    if dtype in (torch.float64, "float64", "f64"):
        return JACOBI_F64
    raise TypeError("dtype must be float32 or float64, got %r" % (dtype,))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ----------------------------------------------------------- C-name wrappers
def jacobi_workspace_bytes(ndim, grid, blocks, dtype):
    out = _SZ(0)
    _check(lib().jacobi_workspace_bytes(int(ndim), _arr64(grid), _arr64(blocks), int(dtype),
                                        ctypes.byref(out)))
    return out.value


def jacobi_create(ndim, grid, blocks, dtype, workspace_ptr, workspace_bytes, stream_ptr):
    h = _P()
    _check(lib().jacobi_create(int(ndim), _arr64(grid), _arr64(blocks), int(dtype),
                               workspace_ptr, int(workspace_bytes), stream_ptr, ctypes.byref(h)))
    return h


def jacobi_deep_workspace_bytes(ndim, grid, blocks, dtype, halo):
    out = _SZ(0)
    _check(lib().jacobi_deep_workspace_bytes(int(ndim), _arr64(grid), _arr64(blocks), int(dtype),
                                             int(halo), ctypes.byref(out)))
    return out.value


def jacobi_deep_create(ndim, grid, blocks, dtype, halo, workspace_ptr, workspace_bytes,
                       stream_ptr):
    h = _P()
    _check(lib().jacobi_deep_create(int(ndim), _arr64(grid), _arr64(blocks), int(dtype),
                                    int(halo), workspace_ptr, int(workspace_bytes), stream_ptr,
                                    ctypes.byref(h)))
    return h


def jacobi_get_halo(h):
    v = _I()
    _check(lib().jacobi_get_halo(h, ctypes.byref(v)))
    return v.value


def jacobi_destroy(h):
    _check(lib().jacobi_destroy(h))


def jacobi_set_stream(h, stream_ptr):
    _check(lib().jacobi_set_stream(h, stream_ptr))


def jacobi_get_layout(h):
    b = (ctypes.c_int64 * 3)()
    e = (ctypes.c_int64 * 3)()
    _check(lib().jacobi_get_layout(h, b, e))
    return tuple(b), tuple(e)


def jacobi_set_state(h, u_ptr):
    _check(lib().jacobi_set_state(h, u_ptr))


def jacobi_get_state(h, u_ptr):
    _check(lib().jacobi_get_state(h, u_ptr))


def jacobi_set_source(h, f_ptr, h2):
    _check(lib().jacobi_set_source(h, f_ptr, float(h2)))


def jacobi_halo_exchange(h):
    _check(lib().jacobi_halo_exchange(h))


def jacobi_sweep(h, n_iter):
    _check(lib().jacobi_sweep(h, int(n_iter)))


def jacobi_residual_async(h, res_ptr):
    _check(lib().jacobi_residual_async(h, res_ptr))


def jacobi_residual(h):
    out = _D(0.0)
    _check(lib().jacobi_residual(h, ctypes.byref(out)))
    return out.value


def jacobi_solve(h, n_iter, check_every, res_ptr):
    _check(lib().jacobi_solve(h, int(n_iter), int(check_every), res_ptr))


def jacobi_solve_noalloc(ndim, grid, blocks, dtype, u0_ptr, f_ptr, h2, n_iter, check_every,
                         u_out_ptr, res_ptr, stream_ptr):
    _check(lib().jacobi_solve_noalloc(int(ndim), _arr64(grid), _arr64(blocks), int(dtype),
                                      u0_ptr, f_ptr, float(h2), int(n_iter), int(check_every),
                                      u_out_ptr, res_ptr, stream_ptr))


JACOBI_NOALLOC_MAX_BYTES = 64 << 20


def jacobi_set_tuning(h, t_depth=0, rows=0, flags=0):
    _check(lib().jacobi_set_tuning(h, int(t_depth), int(rows), int(flags)))


def jacobi_get_tuning(h):
    t, r, f = _I(), _I(), _I()
    _check(lib().jacobi_get_tuning(h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(f)))
    return t.value, r.value, f.value


def jacobi_max_depth(ndim, dtype):
    v = lib().jacobi_max_depth(int(ndim), int(dtype))
    if v < 0:
        _check(v)
    return v


def jacobi_batch_workspace_bytes(grids, block, dtype):
    flat = [int(v) for g in grids for v in g]
    out = _SZ(0)
    _check(lib().jacobi_batch_workspace_bytes(len(grids), _arr64(flat), int(block), int(dtype),
                                              ctypes.byref(out)))
    return out.value


def jacobi_batch_create(grids, block, dtype, workspace_ptr, workspace_bytes, stream_ptr):
    flat = [int(v) for g in grids for v in g]
    h = _P()
    _check(lib().jacobi_batch_create(len(grids), _arr64(flat), int(block), int(dtype),
                                     workspace_ptr, int(workspace_bytes), stream_ptr,
                                     ctypes.byref(h)))
    return h


def jacobi_batch_destroy(b):
    _check(lib().jacobi_batch_destroy(b))


def jacobi_batch_set_grid(b, i, u_ptr, f_ptr, h2):
    _check(lib().jacobi_batch_set_grid(b, int(i), u_ptr, f_ptr, float(h2)))


def jacobi_batch_get_grid(b, i, u_ptr):
    _check(lib().jacobi_batch_get_grid(b, int(i), u_ptr))


def jacobi_batch_set_tuning(b, t_depth=0, rows=0, use_graph=1):
    _check(lib().jacobi_batch_set_tuning(b, int(t_depth), int(rows), int(use_graph)))


def jacobi_batch_get_tuning(b):
    d, r, g = _I(), _I(), _I()
    _check(lib().jacobi_batch_get_tuning(b, ctypes.byref(d), ctypes.byref(r), ctypes.byref(g)))
    return d.value, r.value, g.value


def jacobi_batch_autotune(b, check_every):
    d, r = _I(), _I()
    _check(lib().jacobi_batch_autotune(b, int(check_every), ctypes.byref(d), ctypes.byref(r)))
    return d.value, r.value


def jacobi_batch_solve(b, count, rel_tol, max_sweeps, check_every):
    sw = (ctypes.c_int64 * count)()
    rl = (ctypes.c_double * count)()
    st = (ctypes.c_int * count)()
    _check(lib().jacobi_batch_solve(b, float(rel_tol), int(max_sweeps), int(check_every), sw, rl,
                                    st))
    return list(sw), list(rl), list(st)


def jacobi_forward_ckpt(h, K, C, ckpt_ptr):
    _check(lib().jacobi_forward_ckpt(h, int(K), int(C), ckpt_ptr))


def jacobi_adjoint(h, K, C, dL_duK_ptr, h2, dL_df_ptr, dL_dU0_ptr):
    _check(lib().jacobi_adjoint(h, int(K), int(C), dL_duK_ptr, float(h2), dL_df_ptr, dL_dU0_ptr))


def jacobi_adjoint_begin(h, lam_ptr, grad_b_ptr):
    _check(lib().jacobi_adjoint_begin(h, lam_ptr, grad_b_ptr))


def jacobi_adjoint_sweep(h, n_iter):
    _check(lib().jacobi_adjoint_sweep(h, int(n_iter)))


def jacobi_adjoint_end(h, h2, grad_f_ptr, grad_ring_ptr):
    _check(lib().jacobi_adjoint_end(h, float(h2), grad_f_ptr, grad_ring_ptr))


def jacobi_profile(h, enable):
    _check(lib().jacobi_profile(h, 1 if enable else 0))


def jacobi_profile_read(h, depth=0):
    """Returns dict(ms, launches, cell_updates, alg_bytes) over the recorded
    launches of passes of `depth` sweeps (0 = all)."""
    ms, n, up, by = _D(), _I64(), _D(), _D()
    _check(lib().jacobi_profile_read(h, int(depth), ctypes.byref(ms), ctypes.byref(n),
                                     ctypes.byref(up), ctypes.byref(by)))
    return dict(ms=ms.value, launches=n.value, cell_updates=up.value, alg_bytes=by.value)


def jacobi_autotune(h, n_sweeps, with_source):
    """Returns the chosen (t_depth, rows, flags); leaves the handle without a state."""
    d, r, f = _I(), _I(), _I()
    _check(lib().jacobi_autotune(h, int(n_sweeps), 1 if with_source else 0, ctypes.byref(d),
                                 ctypes.byref(r), ctypes.byref(f)))
    return d.value, r.value, f.value


def jacobi_strerror(status):
    return lib().jacobi_strerror(int(status)).decode()


def jacobi_last_error():
    return lib().jacobi_last_error().decode(errors="replace")


# ------------------------------------------------------------ convenience
def residual_count(n_iter, check_every):
    """Number of residuals jacobi_solve writes: ceil(n_iter / R) + 1."""
    return -(-int(n_iter) // int(check_every)) + 1


class Solver:
    """A handle plus the torch workspace that backs it.

    grid, blocks: interior nodes and blocks per axis, x first (2 or 3 values).
    dtype: torch.float32 or torch.float64.  Tensors passed in must live on the
    workspace's device, be contiguous and have the solver's dtype; full states
    have shape (n_y+2, n_x+2) / (n_z+2, n_y+2, n_x+2), sources (n_y, n_x) / ...
    """

    def __init__(self, grid, blocks, dtype, device="cuda", stream=None, halo=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the Jacobi library has no CPU path")
        self.grid = tuple(int(g) for g in grid)
        self.blocks = tuple(int(b) for b in blocks)
        self.ndim = len(self.grid)
        self.torch_dtype = dtype
        self.dtype = dtype_code(dtype)
        self.device = torch.device(device)
        if halo:
            # deep-halo block storage: frames of `halo` nodes, exchanged once
            # per pass of up to that many sweeps
            nbytes = jacobi_deep_workspace_bytes(self.ndim, self.grid, self.blocks, self.dtype,
                                                 halo)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.h = jacobi_deep_create(self.ndim, self.grid, self.blocks, self.dtype, halo,
                                        _ptr(self.workspace), nbytes, _stream_handle(stream))
            return
        nbytes = jacobi_workspace_bytes(self.ndim, self.grid, self.blocks, self.dtype)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.h = jacobi_create(self.ndim, self.grid, self.blocks, self.dtype,
                               _ptr(self.workspace), nbytes, _stream_handle(stream))

    # shapes
    @property
    def state_shape(self):
        return tuple(n + 2 for n in reversed(self.grid))

    @property
    def interior_shape(self):
        return tuple(reversed(self.grid))

    def _check_tensor(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.workspace.device:
            raise ValueError("%s must be on %s" % (name, self.workspace.device))
        if t.dtype != self.torch_dtype:
            raise TypeError("%s must have dtype %s" % (name, self.torch_dtype))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    def set_stream(self, stream=None):
        jacobi_set_stream(self.h, _stream_handle(stream))

    def set_state(self, U):
        self._check_tensor(U, self.state_shape, "state")
        jacobi_set_state(self.h, _ptr(U))

    def get_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.state_shape, dtype=self.torch_dtype, device=self.device)
        self._check_tensor(out, self.state_shape, "out")
        jacobi_get_state(self.h, _ptr(out))
        return out

    def set_source(self, f, h2):
        if f is None:
            jacobi_set_source(self.h, None, 1.0)
            return
        self._check_tensor(f, self.interior_shape, "source")
        jacobi_set_source(self.h, _ptr(f), h2)

    def halo_exchange(self):
        jacobi_halo_exchange(self.h)

    def sweep(self, n_iter):
        jacobi_sweep(self.h, n_iter)

    def residual(self):
        return jacobi_residual(self.h)

    def residual_async(self, out):
        import torch
        if out.dtype != torch.float64 or out.numel() < 1 or out.device != self.device:
            raise ValueError("out must be a float64 tensor on the solver's device")
        jacobi_residual_async(self.h, _ptr(out))

    def solve(self, n_iter, check_every, out=None):
        import torch
        cnt = residual_count(n_iter, check_every)
        if out is None:
            out = torch.empty(cnt, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or out.numel() < cnt or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of >= %d values" % cnt)
        jacobi_solve(self.h, n_iter, check_every, _ptr(out))
        return out

    def set_tuning(self, t_depth=0, rows=0, flags=0):
        jacobi_set_tuning(self.h, t_depth, rows, flags)

    def get_tuning(self):
        return jacobi_get_tuning(self.h)

    def forward_ckpt(self, n_iter, chunk, keep=True):
        """n_iter sweeps from the current state; with keep, returns the
        checkpoints (states after 0, C, 2C, ... sweeps, C = chunk) as one
        device tensor of shape (ceil(n_iter / C),) + state_shape, else None."""
        import torch
        n_iter, chunk = int(n_iter), int(chunk)
        ck = None
        if keep and n_iter > 0:
            ck = torch.empty((-(-n_iter // chunk),) + self.state_shape, dtype=self.torch_dtype,
                             device=self.device)
        jacobi_forward_ckpt(self.h, n_iter, chunk, _ptr(ck))
        return ck

    def adjoint(self, dL_duK, n_iter, h2, chunk=None):
        """Reverse sweeps in one library call (jacobi_adjoint): from dL/du_K
        (full state tensor, ring included) return (dL/df FP64 interior,
        dL/dU0 FP64 full array: ring = dL/dg, interior = dL/du_0).  chunk:
        sweeps per adjoint segment (the gradients do not depend on it)."""
        import torch
        self._check_tensor(dL_duK, self.state_shape, "dL_duK")
        gf = torch.empty(self.interior_shape, dtype=torch.float64, device=self.device)
        gU0 = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        chunk = int(n_iter) if not chunk else int(chunk)
        jacobi_adjoint(self.h, n_iter, max(chunk, 1), _ptr(dL_duK), h2, _ptr(gf), _ptr(gU0))
        return gf, gU0

    def adjoint_segments(self, lam_K, n_iter, h2, chunk=None, lam_checkpoints=None):
        """The same reverse sweeps through jacobi_adjoint_begin / _sweep / _end.
        Returns (dL/df, the ring part of dL/dg that flows through the sweeps
        as a full FP64 array, lam_0 as a state tensor); lam_K's ring is read
        as zero.  lam_checkpoints: optional list that receives lam at every
        segment boundary (device tensors)."""
        import torch
        self._check_tensor(lam_K, self.state_shape, "lam_K")
        gb = torch.empty(self.interior_shape, dtype=torch.float64, device=self.device)
        ring = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        jacobi_adjoint_begin(self.h, _ptr(lam_K), _ptr(gb))
        chunk = int(n_iter) if not chunk else int(chunk)
        left = int(n_iter)
        while left > 0:
            step = min(chunk, left)
            jacobi_adjoint_sweep(self.h, step)
            left -= step
            if lam_checkpoints is not None:
                lam_checkpoints.append(self.get_state())
        jacobi_adjoint_end(self.h, h2, _ptr(gb), _ptr(ring))
        return gb, ring, self.get_state()

    def profile(self, enable=True):
        jacobi_profile(self.h, enable)

    def profile_read(self, depth=0):
        return jacobi_profile_read(self.h, depth)

    def autotune(self, n_sweeps, with_source=True):
        """Pick the fastest bit-neutral schedule; the state must be set afterwards."""
        return jacobi_autotune(self.h, n_sweeps, with_source)

    def layout(self):
        return jacobi_get_layout(self.h)

    def halo(self):
        """Stored frame depth of a deep-halo solver (0 for a standard one)."""
        return jacobi_get_halo(self.h)

    def close(self):
        # the library frees the handle even when it reports an error, so
        # forget it first: a second destroy would free it twice
        h = getattr(self, "h", None)
        if h is not None:
            self.h = None
            jacobi_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent 2D Poisson grids of uneven sizes solved together.

    grids: list of (n_x, n_y) interior sizes; dtype torch.float32/float64;
    block: target block side of each grid's decomposition.  The batch runs on
    its own (default-priority) stream so that check intervals can be captured
    as hipGraphs; set_grid / get_grid / solve order it against the caller's
    current stream."""

    def __init__(self, grids, dtype, block=512, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the Jacobi library has no CPU path")
        self.grids = [(int(a), int(b)) for a, b in grids]
        self.count = len(self.grids)
        self.torch_dtype = dtype
        self.dtype = dtype_code(dtype)
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        nbytes = jacobi_batch_workspace_bytes(self.grids, block, self.dtype)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._keep = []
        self.h = jacobi_batch_create(self.grids, block, self.dtype, _ptr(self.workspace), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream))

    def _enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_grid(self, i, U, f, h2):
        nx, ny = self.grids[i]
        for t, shape, name in ((U, (ny + 2, nx + 2), "state"), (f, (ny, nx), "source")):
            if t.dtype != self.torch_dtype or tuple(t.shape) != shape or not t.is_contiguous() \
                    or t.device != self.device:
                raise ValueError("%s of grid %d must be a contiguous %s tensor of shape %s on %s"
                                 % (name, i, self.torch_dtype, shape, self.device))
        self._enter()
        self._keep.extend([U, f])
        jacobi_batch_set_grid(self.h, i, _ptr(U), _ptr(f), h2)

    def get_grid(self, i):
        import torch
        nx, ny = self.grids[i]
        out = torch.empty((ny + 2, nx + 2), dtype=self.torch_dtype, device=self.device)
        self._enter()
        jacobi_batch_get_grid(self.h, i, _ptr(out))
        self._leave()
        return out

    def set_tuning(self, t_depth=0, rows=0, use_graph=True):
        jacobi_batch_set_tuning(self.h, t_depth, rows, 1 if use_graph else 0)

    def get_tuning(self):
        return jacobi_batch_get_tuning(self.h)

    def autotune(self, check_every):
        self._enter()
        out = jacobi_batch_autotune(self.h, check_every)
        self._keep = []
        return out

    def solve(self, rel_tol, max_sweeps, check_every):
        """Returns (sweeps, rel, status) lists, one entry per grid."""
        self._enter()
        out = jacobi_batch_solve(self.h, self.count, rel_tol, max_sweeps, check_every)
        self._keep = []
        self._leave()
        return out

    def close(self):
        h = getattr(self, "h", None)
        if h is not None:
            self.h = None
            jacobi_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
