"""Thin Python binding of libgodec (include/godec.h).

The functions below mirror the C entry points one to one and only marshal
arguments: every step of the decomposition runs in the HIP library.  PyTorch
provides device memory (the workspace and outputs are torch tensors) and the
stream.  If the built library is missing the import of this module still
works, but ``load()`` raises: there is no fallback path.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgodec.so")

GODEC_OK = 0
STATUS = {0: "GODEC_OK", 1: "GODEC_E_INVAL", 2: "GODEC_E_NOMEM",
          3: "GODEC_E_DEVICE", 4: "GODEC_E_NUMERIC", 5: "GODEC_E_STATE",
          6: "GODEC_E_UNSUPPORTED"}
GODEC_F64, GODEC_F32 = 0, 1
GODEC_PREC_NATIVE, GODEC_PREC_BF16_REFINE = 0, 1
GODEC_MAX_RANK = 32


class godec_opts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("prec", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("lstep", ctypes.c_int32),
                ("rank_tol", ctypes.c_double), ("a1_host", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("support_dev", ctypes.c_void_p),
                ("support_nnz", ctypes.c_int64), ("warm_start", ctypes.c_int32),
                ("redraw_a1", ctypes.c_int32)]


class godec_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rank_eff", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rel_err_sq", ctypes.c_double), ("threshold", ctypes.c_double),
                ("sum_r2", ctypes.c_double), ("norm_x2", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class godec_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double),
                ("bytes_per_launch", ctypes.c_double)]


class godec_problem(ctypes.Structure):
    _fields_ = [("X_dev", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("r", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("k", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class godec_grebsmo_info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("inner_iters", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rel_err_sq", ctypes.c_double), ("l1", ctypes.c_double)]


class godec_mse_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rel_err_sq", ctypes.c_double), ("threshold", ctypes.c_double),
                ("sum_r2", ctypes.c_double), ("norm_x2", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GodecError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SIG = {
    "godec_opts_default": (None, [ctypes.POINTER(godec_opts)]),
    "godec_workspace_size": (_I32, [_I64, _I64, _I32, _I64, _I32, _I32,
                                    ctypes.POINTER(godec_opts),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "godec_init": (_I32, [ctypes.POINTER(_P), _P, _I32, _I64, _I64, _I64, _I32,
                          _I64, _I32, ctypes.c_uint64, _P, ctypes.c_size_t,
                          ctypes.POINTER(godec_opts)]),
    "godec_step": (_I32, [_P, _I32, _I32]),
    "godec_set_graphs": (_I32, [_P, _I32]),
    "godec_solve": (_I32, [_P, _I32, _I64, _I64, _I64, _I32, _I64, _I32,
                           ctypes.c_uint64, _I32, _P, ctypes.c_size_t,
                           ctypes.POINTER(godec_opts), _P, _P, _P, _P,
                           ctypes.POINTER(godec_info)]),
    "godec_solve_static": (_I32, [_P, _I32, _I64, _I64, _I64, _I32, _I64, _I32,
                                  ctypes.c_uint64, _I32, ctypes.POINTER(godec_opts),
                                  _P, _P, _P, _P, ctypes.POINTER(godec_info)]),
    "godec_solve_tol": (_I32, [_P, _I32, _I64, _I64, _I64, _I32, _I64, _I32,
                               ctypes.c_uint64, _I32, ctypes.c_double, _P, ctypes.c_size_t,
                               ctypes.POINTER(godec_opts), _P, _P, _P, _P,
                               ctypes.POINTER(godec_info)]),
    "godec_get_factors": (_I32, [_P, _P, _P]),
    "godec_get_L_dense": (_I32, [_P, _P, _I64]),
    "godec_get_S": (_I32, [_P, _P, _P, ctypes.POINTER(_I64)]),
    "godec_get_residual": (_I32, [_P, _P, _I64]),
    "godec_get_A1": (_I32, [_P, _P]),
    "godec_get_info": (_I32, [_P, ctypes.POINTER(godec_info)]),
    "godec_destroy": (_I32, [_P]),
    "godec_last_error": (ctypes.c_char_p, []),
    "godec_draw_a1": (_I32, [ctypes.c_uint64, _I64, _I32, _P]),
    "godec_version": (ctypes.c_char_p, []),
    "godec_profile": (_I32, [_P, _I32]),
    "godec_profile_read": (_I32, [_P, ctypes.POINTER(godec_kernel_stat), _I32,
                                  ctypes.POINTER(_I32)]),
    "godec_batch_workspace_size": (_I32, [ctypes.POINTER(godec_problem), _I32, _I32,
                                          ctypes.POINTER(godec_opts),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "godec_batch_init": (_I32, [ctypes.POINTER(_P), ctypes.POINTER(godec_problem), _I32,
                                _I32, _P, ctypes.c_size_t, ctypes.POINTER(godec_opts)]),
    "godec_batch_step": (_I32, [_P, _I32]),
    "godec_batch_step_eager": (_I32, [_P, _I32]),
    "godec_batch_get_factors": (_I32, [_P, _I32, _P, _P]),
    "godec_batch_get_S": (_I32, [_P, _I32, _P, _P, ctypes.POINTER(_I64)]),
    "godec_batch_get_residual": (_I32, [_P, _I32, _P, _I64]),
    "godec_batch_get_A1": (_I32, [_P, _I32, _P]),
    "godec_batch_get_info": (_I32, [_P, _I32, ctypes.POINTER(godec_info)]),
    "godec_batch_tuning": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "godec_batch_destroy": (_I32, [_P]),
    "godec_layer_workspace_size": (_I32, [_I32, _I64, _I64, _I32, _I64, _I32, _I32, _I32,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "godec_layer_forward": (_I32, [ctypes.POINTER(_P), _P, _I32, _I32, _I64, _I64, _I32, _I64,
                                   _I32, _I32, ctypes.c_uint64, _P, ctypes.c_size_t,
                                   ctypes.POINTER(godec_opts), _P, _P]),
    "godec_layer_backward": (_I32, [_P, _P, _P, _P]),
    "godec_layer_get_mask": (_I32, [_P, _I32, _I32, _P, ctypes.POINTER(_I64)]),
    "godec_layer_get_A1": (_I32, [_P, _I32, _P]),
    "godec_layer_destroy": (_I32, [_P]),
    "godec_grebsmo_workspace_size": (_I32, [_I64, _I64, _I32, _I32,
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "godec_grebsmo_init": (_I32, [ctypes.POINTER(_P), _P, _I32, _I64, _I64, _I64, _I32, _I32,
                                  _I32, ctypes.c_double, ctypes.c_uint64, _P, _P,
                                  ctypes.c_size_t, _P]),
    "godec_grebsmo_stage": (_I32, [_P, _I32]),
    "godec_grebsmo_solve": (_I32, [_P, _I32, ctypes.c_double,
                                   ctypes.POINTER(godec_grebsmo_info)]),
    "godec_grebsmo_get_factors": (_I32, [_P, _P, _P]),
    "godec_grebsmo_get_S": (_I32, [_P, _P, _I64]),
    "godec_grebsmo_get_info": (_I32, [_P, ctypes.POINTER(godec_grebsmo_info)]),
    "godec_grebsmo_destroy": (_I32, [_P]),
    "godec_mse_workspace_size": (_I32, [_I64, _I64, _I32, _P, _P, _I64, _I32,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "godec_mse_init": (_I32, [ctypes.POINTER(ctypes.c_void_p), _P, _I32, _I64, _I64, _I64,
                              _I32, _P, _P, _P, _I64, ctypes.c_uint64, _P, ctypes.c_size_t,
                              _P]),
    "godec_mse_step": (_I32, [_P, _I32]),
    "godec_mse_get_factors": (_I32, [_P, _I32, _P, _P]),
    "godec_mse_get_S": (_I32, [_P, _P, _P, ctypes.POINTER(_I64)]),
    "godec_mse_get_residual": (_I32, [_P, _P, _I64]),
    "godec_mse_get_info": (_I32, [_P, ctypes.POINTER(godec_mse_info)]),
    "godec_mse_destroy": (_I32, [_P]),
}


def load(path: str = LIB_PATH):
    """Load libgodec.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libgodec.so not found at {path}; build it with "
            "`python -m paper_1309_0302_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIG.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != GODEC_OK:
        msg = load().godec_last_error().decode(errors="replace")
        raise GodecError(status, msg)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return GODEC_F64
    if t.dtype == torch.float32:
        return GODEC_F32
    raise ValueError("X must be float32 or float64")


def make_opts(prec=GODEC_PREC_NATIVE, refine_iters=1, rank_tol=0.0, a1=None,
              stream=None, support=None, lstep=0, warm_start=0, redraw_a1=0):
    """support: optional int64 device tensor of strictly ascending linear
    indices (matrix completion: the fixed support of S).  redraw_a1 = 1:
    iteration t draws its own A1 from seed + t."""
    o = godec_opts()
    load().godec_opts_default(ctypes.byref(o))
    o.prec = prec
    o.lstep = lstep
    o.warm_start = warm_start
    o.redraw_a1 = redraw_a1
    o.refine_iters = refine_iters
    o.rank_tol = rank_tol
    keep = None
    if a1 is not None:
        keep = np.ascontiguousarray(a1, dtype=np.float64)
        o.a1_host = keep.ctypes.data
    o.stream = stream
    if support is not None:
        import torch
        if not support.is_cuda or support.dtype != torch.int64 or not support.is_contiguous():
            raise ValueError("support must be a contiguous int64 device tensor")
        o.support_dev = support.data_ptr() if support.numel() else None
        o.support_nnz = support.numel()
    return o, keep


# ---- one-to-one wrappers of the C entry points ----------------------------

def godec_workspace_size(m, n, r, k, q, dtype, opts=None):
    out = ctypes.c_size_t(0)
    _check(load().godec_workspace_size(m, n, r, k, q, dtype,
                                       ctypes.byref(opts) if opts else None,
                                       ctypes.byref(out)))
    return out.value


def godec_init(X_ptr, dtype, m, n, ldx, r, k, q, seed, ws_ptr, ws_bytes,
               opts=None):
    ctx = ctypes.c_void_p()
    _check(load().godec_init(ctypes.byref(ctx), X_ptr, dtype, m, n, ldx, r, k,
                             q, seed, ws_ptr, ws_bytes,
                             ctypes.byref(opts) if opts else None))
    return ctx


def godec_step(ctx, iters, total_iters=0):
    _check(load().godec_step(ctx, iters, total_iters))


def godec_get_factors(ctx, ul_ptr, vl_ptr):
    _check(load().godec_get_factors(ctx, ul_ptr, vl_ptr))


def godec_get_L_dense(ctx, l_ptr, ldl):
    _check(load().godec_get_L_dense(ctx, l_ptr, ldl))


def godec_get_S(ctx, idx_ptr, val_ptr):
    nnz = _I64(0)
    _check(load().godec_get_S(ctx, idx_ptr, val_ptr, ctypes.byref(nnz)))
    return nnz.value


def godec_get_residual(ctx, r_ptr, ldr):
    _check(load().godec_get_residual(ctx, r_ptr, ldr))


def godec_get_A1(ctx, n, r):
    out = np.empty((n, r), dtype=np.float64)
    _check(load().godec_get_A1(ctx, out.ctypes.data))
    return out


def godec_get_info(ctx):
    info = godec_info()
    _check(load().godec_get_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def godec_destroy(ctx):
    _check(load().godec_destroy(ctx))


def godec_draw_a1(seed, n, r):
    out = np.empty((n, r), dtype=np.float64)
    _check(load().godec_draw_a1(seed, n, r, out.ctypes.data))
    return out


def godec_profile(ctx, enable):
    _check(load().godec_profile(ctx, 1 if enable else 0))


def godec_profile_read(ctx):
    arr = (godec_kernel_stat * 16)()
    cnt = _I32(0)
    _check(load().godec_profile_read(ctx, arr, 16, ctypes.byref(cnt)))
    out = []
    for i in range(min(cnt.value, 16)):
        st = arr[i]
        out.append(dict(name=st.name.decode(), launches=st.launches,
                        total_ms=st.total_ms,
                        bytes_per_launch=st.bytes_per_launch))
    return out


def godec_solve(X, r, k, q, seed, iters, opts=None):
    """init + step + results + destroy; returns (UL, VL, S_idx, S_val, info)."""
    import torch
    m, n = X.shape
    dt = _dtype_code(X)
    opts = opts if opts is not None else make_opts()[0]
    ws_bytes = godec_workspace_size(m, n, r, k, q, dt, opts)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=X.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    UL = torch.zeros((m, r), dtype=X.dtype, device=X.device)
    VL = torch.zeros((n, r), dtype=X.dtype, device=X.device)
    sidx = torch.zeros(max(k, 1), dtype=torch.int64, device=X.device)
    sval = torch.zeros(max(k, 1), dtype=X.dtype, device=X.device)
    info = godec_info()
    _check(load().godec_solve(X.data_ptr(), dt, m, n, X.stride(0), r, k, q,
                              seed, iters, base, ws_bytes, ctypes.byref(opts),
                              UL.data_ptr(), VL.data_ptr(), sidx.data_ptr(),
                              sval.data_ptr(), ctypes.byref(info)))
    nnz = info.nnz
    return UL, VL, sidx[:nnz], sval[:nnz], info.as_dict()


GODEC_STATIC_SCRATCH_BYTES = 128 << 20


def godec_solve_static(X, r, k, q, seed, iters, opts=None):
    """godec_solve on the library's own device scratch (no workspace is
    allocated by the library); returns (UL, VL, S_idx, S_val, info)."""
    import torch
    m, n = X.shape
    dt = _dtype_code(X)
    opts = opts if opts is not None else make_opts()[0]
    UL = torch.zeros((m, r), dtype=X.dtype, device=X.device)
    VL = torch.zeros((n, r), dtype=X.dtype, device=X.device)
    sidx = torch.zeros(max(k, 1), dtype=torch.int64, device=X.device)
    sval = torch.zeros(max(k, 1), dtype=X.dtype, device=X.device)
    info = godec_info()
    _check(load().godec_solve_static(X.data_ptr(), dt, m, n, X.stride(0), r, k, q, seed,
                                     iters, ctypes.byref(opts), UL.data_ptr(), VL.data_ptr(),
                                     sidx.data_ptr(), sval.data_ptr(), ctypes.byref(info)))
    nnz = info.nnz
    return UL, VL, sidx[:nnz], sval[:nnz], info.as_dict()


def godec_solve_tol(X, r, k, q, seed, max_iters, eps, opts=None):
    """Iterate until rel_err_sq <= eps (loop test of Algorithm 1) or max_iters;
    returns (UL, VL, S_idx, S_val, info)."""
    import torch
    m, n = X.shape
    dt = _dtype_code(X)
    opts = opts if opts is not None else make_opts()[0]
    ws_bytes = godec_workspace_size(m, n, r, k, q, dt, opts)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=X.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    UL = torch.zeros((m, r), dtype=X.dtype, device=X.device)
    VL = torch.zeros((n, r), dtype=X.dtype, device=X.device)
    sidx = torch.zeros(max(k, 1), dtype=torch.int64, device=X.device)
    sval = torch.zeros(max(k, 1), dtype=X.dtype, device=X.device)
    info = godec_info()
    _check(load().godec_solve_tol(X.data_ptr(), dt, m, n, X.stride(0), r, k, q,
                                  seed, max_iters, eps, base, ws_bytes, ctypes.byref(opts),
                                  UL.data_ptr(), VL.data_ptr(), sidx.data_ptr(),
                                  sval.data_ptr(), ctypes.byref(info)))
    nnz = info.nnz
    return UL, VL, sidx[:nnz], sval[:nnz], info.as_dict()


# ---- convenience object -----------------------------------------------------

class GoDec:
    """One decomposition of a CUDA/HIP tensor X (float32 or float64)."""

    def __init__(self, X, r, k, q, seed=0, prec=GODEC_PREC_NATIVE,
                 refine_iters=1, rank_tol=0.0, a1=None, stream=None, support=None,
                 lstep=0, warm_start=0, redraw_a1=0):
        import torch
        if not X.is_cuda:
            raise ValueError("X must be a device tensor")
        if X.stride(1) != 1:
            raise ValueError("X must be row-major with unit column stride")
        self.X = X
        self.m, self.n = X.shape
        self.r, self.k, self.q = r, k, q
        self.seed, self.a1 = seed, a1
        self.dtype = _dtype_code(X)
        if stream is None:
            stream = torch.cuda.current_stream(X.device).cuda_stream
        self.support = support
        self.opts, self._a1_keep = make_opts(prec, refine_iters, rank_tol, a1,
                                             stream, support, lstep, warm_start,
                                             redraw_a1)
        self.ws_bytes = godec_workspace_size(self.m, self.n, r, k, q,
                                             self.dtype, self.opts)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                              device=X.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        self.ctx = godec_init(X.data_ptr(), self.dtype, self.m, self.n,
                              X.stride(0), r, k, q, seed, base, self.ws_bytes,
                              self.opts)

    def step(self, iters=1, total_iters=0):
        godec_step(self.ctx, iters, total_iters)

    def graphs(self, enable=True):
        """Replay steady iterations from recorded HIP graphs (godec_set_graphs)."""
        _check(load().godec_set_graphs(self.ctx, 1 if enable else 0))

    def factors(self):
        import torch
        UL = torch.empty((self.m, self.r), dtype=self.X.dtype, device=self.X.device)
        VL = torch.empty((self.n, self.r), dtype=self.X.dtype, device=self.X.device)
        godec_get_factors(self.ctx, UL.data_ptr(), VL.data_ptr())
        return UL, VL

    def L_dense(self):
        import torch
        L = torch.empty((self.m, self.n), dtype=self.X.dtype, device=self.X.device)
        godec_get_L_dense(self.ctx, L.data_ptr(), self.n)
        return L

    def residual(self):
        import torch
        R = torch.empty((self.m, self.n), dtype=self.X.dtype, device=self.X.device)
        godec_get_residual(self.ctx, R.data_ptr(), self.n)
        return R

    def S(self):
        import torch
        kk = max(self.k, 1)
        idx = torch.empty(kk, dtype=torch.int64, device=self.X.device)
        val = torch.empty(kk, dtype=self.X.dtype, device=self.X.device)
        nnz = godec_get_S(self.ctx, idx.data_ptr(), val.data_ptr())
        return idx[:nnz], val[:nnz]

    def A1(self):
        return godec_get_A1(self.ctx, self.n, self.r)

    def info(self):
        return godec_get_info(self.ctx)

    def profile(self, enable=True):
        godec_profile(self.ctx, enable)

    def profile_read(self):
        return godec_profile_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            godec_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched form -------------------------------------------------------------

def _problems(specs):
    arr = (godec_problem * len(specs))()
    for i, (X, r, k, seed) in enumerate(specs):
        arr[i].X_dev = X.data_ptr()
        arr[i].m, arr[i].n = X.shape
        arr[i].ldx = X.stride(0)
        arr[i].r = r
        arr[i].reserved = 0
        arr[i].k = k
        arr[i].seed = seed
    return arr


def godec_batch_workspace_size(probs, q, opts=None):
    out = ctypes.c_size_t(0)
    _check(load().godec_batch_workspace_size(probs, len(probs), q,
                                             ctypes.byref(opts) if opts else None,
                                             ctypes.byref(out)))
    return out.value


def godec_batch_init(probs, q, ws_ptr, ws_bytes, opts):
    b = ctypes.c_void_p()
    _check(load().godec_batch_init(ctypes.byref(b), probs, len(probs), q, ws_ptr,
                                   ws_bytes, ctypes.byref(opts)))
    return b


def godec_batch_step(b, iters):
    _check(load().godec_batch_step(b, iters))


def godec_batch_step_eager(b, iters):
    _check(load().godec_batch_step_eager(b, iters))


def godec_batch_get_factors(b, i, ul_ptr, vl_ptr):
    _check(load().godec_batch_get_factors(b, i, ul_ptr, vl_ptr))


def godec_batch_get_S(b, i, idx_ptr, val_ptr):
    nnz = _I64(0)
    _check(load().godec_batch_get_S(b, i, idx_ptr, val_ptr, ctypes.byref(nnz)))
    return nnz.value


def godec_batch_get_residual(b, i, r_ptr, ldr):
    _check(load().godec_batch_get_residual(b, i, r_ptr, ldr))


def godec_batch_get_A1(b, i, n, r):
    out = np.empty((n, r), dtype=np.float64)
    _check(load().godec_batch_get_A1(b, i, out.ctypes.data))
    return out


def godec_batch_get_info(b, i):
    info = godec_info()
    _check(load().godec_batch_get_info(b, i, ctypes.byref(info)))
    return info.as_dict()


def godec_batch_tuning(b):
    rows, items = _I32(0), _I32(0)
    _check(load().godec_batch_tuning(b, ctypes.byref(rows), ctypes.byref(items)))
    return rows.value, items.value


def godec_batch_destroy(b):
    _check(load().godec_batch_destroy(b))


class GoDecBatch:
    """Many independent FP32 decompositions advanced together.

    specs: list of (X, r, k, seed) with X a float32 device tensor.  The batch
    runs on its own stream (a captured graph cannot use the default stream);
    getters synchronise it before returning.
    """

    def __init__(self, specs, q, rank_tol=0.0, stream=None):
        import torch
        self.specs = specs
        self.q = q
        for X, _, _, _ in specs:
            if not X.is_cuda or X.dtype != torch.float32 or X.stride(1) != 1:
                raise ValueError("every X must be a row-major float32 device tensor")
        dev = specs[0][0].device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self.opts, _ = make_opts(rank_tol=rank_tol, stream=self.stream.cuda_stream)
        self.probs = _problems(specs)
        self.ws_bytes = godec_batch_workspace_size(self.probs, q, self.opts)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        torch.cuda.synchronize(dev)
        self.b = godec_batch_init(self.probs, q, base, self.ws_bytes, self.opts)

    def step(self, iters=1, eager=False):
        (godec_batch_step_eager if eager else godec_batch_step)(self.b, iters)

    def synchronize(self):
        self.stream.synchronize()

    def factors(self, i):
        import torch
        X, r = self.specs[i][0], self.specs[i][1]
        m, n = X.shape
        UL = torch.empty((m, r), dtype=torch.float32, device=X.device)
        VL = torch.empty((n, r), dtype=torch.float32, device=X.device)
        self.synchronize()
        godec_batch_get_factors(self.b, i, UL.data_ptr(), VL.data_ptr())
        self.synchronize()
        return UL, VL

    def S(self, i):
        import torch
        X, k = self.specs[i][0], self.specs[i][2]
        kk = max(k, 1)
        idx = torch.empty(kk, dtype=torch.int64, device=X.device)
        val = torch.empty(kk, dtype=torch.float32, device=X.device)
        self.synchronize()
        nnz = godec_batch_get_S(self.b, i, idx.data_ptr(), val.data_ptr())
        return idx[:nnz], val[:nnz]

    def residual(self, i):
        import torch
        X = self.specs[i][0]
        m, n = X.shape
        R = torch.empty((m, n), dtype=torch.float32, device=X.device)
        self.synchronize()
        godec_batch_get_residual(self.b, i, R.data_ptr(), n)
        self.synchronize()
        return R

    def A1(self, i):
        X, r = self.specs[i][0], self.specs[i][1]
        return godec_batch_get_A1(self.b, i, X.shape[1], r)

    def info(self, i):
        return godec_batch_get_info(self.b, i)

    def tuning(self):
        return godec_batch_tuning(self.b)

    def close(self):
        if getattr(self, "b", None) is not None:
            godec_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- differentiable layer -----------------------------------------------------

def godec_layer_workspace_size(batch, m, n, r, k, q, T, dtype):
    out = ctypes.c_size_t(0)
    _check(load().godec_layer_workspace_size(batch, m, n, r, k, q, T, dtype,
                                             ctypes.byref(out)))
    return out.value


def godec_layer_forward(X_ptr, dtype, batch, m, n, r, k, q, T, seed, ws_ptr, ws_bytes,
                        opts, L_ptr, S_ptr):
    h = _P()
    _check(load().godec_layer_forward(ctypes.byref(h), X_ptr, dtype, batch, m, n, r, k, q, T,
                                      seed, ws_ptr, ws_bytes,
                                      ctypes.byref(opts) if opts is not None else None,
                                      L_ptr, S_ptr))
    return h


def godec_layer_backward(h, dL_ptr, dS_ptr, dX_ptr):
    _check(load().godec_layer_backward(h, dL_ptr, dS_ptr, dX_ptr))


def godec_layer_get_mask(h, b, t, k):
    nnz = _I64(0)
    out = np.empty(max(k, 1), dtype=np.int64)
    _check(load().godec_layer_get_mask(h, b, t, out.ctypes.data, ctypes.byref(nnz)))
    return out[:nnz.value].copy()


def godec_layer_get_A1(h, b, n, r):
    out = np.empty((n, r), dtype=np.float64)
    _check(load().godec_layer_get_A1(h, b, out.ctypes.data))
    return out


def godec_layer_destroy(h):
    _check(load().godec_layer_destroy(h))


class GoDecLayer:
    """T unrolled GoDec iterations on a batch of equally shaped problems
    (X: batch x m x n device tensor, float32 or float64) with a backward pass
    through the frozen supports.  forward() runs the iterations and returns
    (L_T, S_T); backward(dL, dS) returns dX."""

    def __init__(self, r, k, q, T, seed=0, rank_tol=0.0, stream=None):
        self.r, self.k, self.q, self.T, self.seed = r, k, q, T, seed
        self.rank_tol = rank_tol
        self.stream = stream
        self.h = None

    def forward(self, X):
        import torch
        if X.dim() == 2:
            X = X.unsqueeze(0)
        if not X.is_cuda or not X.is_contiguous():
            raise ValueError("X must be a contiguous device tensor (batch x m x n)")
        self.close()
        self.X = X
        self.nb, self.m, self.n = X.shape
        self.dtype = _dtype_code(X)
        stream = self.stream
        if stream is None:
            stream = torch.cuda.current_stream(X.device).cuda_stream
        self.opts, _ = make_opts(rank_tol=self.rank_tol, stream=stream)
        self.ws_bytes = godec_layer_workspace_size(self.nb, self.m, self.n, self.r, self.k,
                                                   self.q, self.T, self.dtype)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=X.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        L = torch.empty_like(X)
        S = torch.empty_like(X)
        self.h = godec_layer_forward(X.data_ptr(), self.dtype, self.nb, self.m, self.n,
                                     self.r, self.k, self.q, self.T, self.seed, base,
                                     self.ws_bytes, self.opts, L.data_ptr(), S.data_ptr())
        return L, S

    def backward(self, dL, dS):
        import torch
        dL = dL.reshape(self.X.shape).contiguous()
        dS = dS.reshape(self.X.shape).contiguous()
        if dL.dtype != self.X.dtype or dS.dtype != self.X.dtype:
            raise ValueError("dL and dS must have the dtype of X")
        dX = torch.empty_like(self.X)
        godec_layer_backward(self.h, dL.data_ptr(), dS.data_ptr(), dX.data_ptr())
        return dX

    def mask(self, b, t):
        return godec_layer_get_mask(self.h, b, t, self.k)

    def A1(self, b):
        return godec_layer_get_A1(self.h, b, self.n, self.r)

    def close(self):
        if getattr(self, "h", None) is not None:
            godec_layer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def godec_layer_fn(X, r, k, q, T, seed=0):
    """(L_T, S_T) = GoDec layer of X (batch x m x n) as a torch autograd
    function whose backward calls the library's hand-written adjoints."""
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, Xin):
            layer = GoDecLayer(r, k, q, T, seed)
            L, S = layer.forward(Xin.detach().contiguous())
            ctx.layer = layer
            return L, S

        @staticmethod
        def backward(ctx, dL, dS):
            dL = torch.zeros_like(ctx.layer.X) if dL is None else dL
            dS = torch.zeros_like(ctx.layer.X) if dS is None else dS
            return ctx.layer.backward(dL, dS).reshape(X.shape)

    return _Fn.apply(X)


# ---- GreBsmo ------------------------------------------------------------------

def godec_grebsmo_workspace_size(m, n, r, dtype):
    out = ctypes.c_size_t(0)
    _check(load().godec_grebsmo_workspace_size(m, n, r, dtype, ctypes.byref(out)))
    return out.value


def godec_grebsmo_init(X_ptr, dtype, m, n, ldx, r, dr, power, lam, seed, omega, ws_ptr,
                       ws_bytes, stream):
    h = _P()
    om = None
    if omega is not None:
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        if omega.shape != (n, r):
            raise ValueError("omega must be n x r")
        om = omega.ctypes.data
    _check(load().godec_grebsmo_init(ctypes.byref(h), X_ptr, dtype, m, n, ldx, r, dr, power,
                                     lam, seed, om, ws_ptr, ws_bytes, stream))
    return h


def godec_grebsmo_stage(h, K):
    _check(load().godec_grebsmo_stage(h, K))


def godec_grebsmo_solve(h, K, tau=0.0, want_info=True):
    """Run stages until the rank bound (or tau); with want_info=False and
    tau = 0 the call only enqueues work and returns None."""
    info = godec_grebsmo_info() if want_info else None
    _check(load().godec_grebsmo_solve(h, K, tau, ctypes.byref(info) if want_info else None))
    return info


def godec_grebsmo_get_factors(h, u_ptr, vt_ptr):
    _check(load().godec_grebsmo_get_factors(h, u_ptr, vt_ptr))


def godec_grebsmo_get_S(h, s_ptr, lds):
    _check(load().godec_grebsmo_get_S(h, s_ptr, lds))


def godec_grebsmo_get_info(h):
    info = godec_grebsmo_info()
    _check(load().godec_grebsmo_get_info(h, ctypes.byref(info)))
    return info


def godec_grebsmo_destroy(h):
    _check(load().godec_grebsmo_destroy(h))


class GreBsmo:
    """GreBsmo (greedy bilateral smoothing) of one dense device matrix X
    (m x n, float32 or float64): rank stages of dr appended rows, K inner
    iterations each, soft threshold lam, power steps per greedy direction."""

    def __init__(self, X, r, dr=1, power=2, lam=0.1, seed=0, omega=None, stream=None):
        import torch
        if X.dim() != 2 or not X.is_cuda or X.stride(1) != 1:
            raise ValueError("X must be a 2-D device tensor with unit column stride")
        self.X = X
        self.m, self.n = X.shape
        self.r = r
        self.dtype = _dtype_code(X)
        if stream is None:
            stream = torch.cuda.current_stream(X.device).cuda_stream
        self.stream = stream
        self.ws_bytes = godec_grebsmo_workspace_size(self.m, self.n, r, self.dtype)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=X.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        self.h = None
        self.h = godec_grebsmo_init(X.data_ptr(), self.dtype, self.m, self.n, X.stride(0), r,
                                    dr, power, lam, seed, omega, base, self.ws_bytes, stream)

    def stage(self, K):
        godec_grebsmo_stage(self.h, K)

    def solve(self, K, tau=0.0, want_info=True):
        return godec_grebsmo_solve(self.h, K, tau, want_info)

    def info(self):
        return godec_grebsmo_get_info(self.h)

    def factors(self):
        """(U m x rank, Vt n x rank) device tensors, L = U Vt^T."""
        import torch
        rank = self.info().rank
        U = torch.empty((self.m, rank), dtype=self.X.dtype, device=self.X.device)
        Vt = torch.empty((self.n, rank), dtype=self.X.dtype, device=self.X.device)
        godec_grebsmo_get_factors(self.h, U.data_ptr(), Vt.data_ptr())
        return U, Vt

    def S(self):
        import torch
        S = torch.empty((self.m, self.n), dtype=self.X.dtype, device=self.X.device)
        godec_grebsmo_get_S(self.h, S.data_ptr(), self.n)
        return S

    def close(self):
        if getattr(self, "h", None) is not None:
            godec_grebsmo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- MSE training (Sec. 4.2.1, Algorithm 4) ---------------------------------

def _label_arrays(labels, ranks):
    k = len(labels)
    lptr = np.zeros(k + 1, dtype=np.int64)
    lptr[1:] = np.cumsum([len(r) for r in labels])
    rows = (np.concatenate([np.asarray(r, dtype=np.int64) for r in labels])
            if lptr[-1] > 0 else np.zeros(1, np.int64))
    rk = np.ascontiguousarray(ranks, dtype=np.int32)
    return lptr, np.ascontiguousarray(rows), rk


def godec_mse_workspace_size(n, p, labels, ranks, K, dtype):
    lptr, _, rk = _label_arrays(labels, ranks)
    out = ctypes.c_size_t(0)
    _check(load().godec_mse_workspace_size(n, p, len(labels), rk.ctypes.data,
                                           lptr.ctypes.data, K, dtype, ctypes.byref(out)))
    return out.value


class GoDecMSE:
    """MSE training of a device matrix X (n samples x p features) with label
    row sets `labels` (list of ascending integer arrays), ranks r_i and the
    cardinality K of S."""

    def __init__(self, X, labels, ranks, K, seed=0, stream=None):
        import torch
        if not X.is_cuda or X.stride(1) != 1:
            raise ValueError("X must be a row-major device tensor")
        self.X = X
        self.n, self.p = X.shape
        self.k = len(labels)
        self.labels = [np.asarray(r, dtype=np.int64) for r in labels]
        self.ranks = [int(r) for r in ranks]
        self.K, self.seed = K, seed
        self.dtype = _dtype_code(X)
        if stream is None:
            stream = torch.cuda.current_stream(X.device).cuda_stream
        self.stream = stream
        lptr, rows, rk = _label_arrays(self.labels, self.ranks)
        self.ws_bytes = godec_mse_workspace_size(self.n, self.p, self.labels, self.ranks, K,
                                                 self.dtype)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=X.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        ctx = ctypes.c_void_p()
        _check(load().godec_mse_init(ctypes.byref(ctx), X.data_ptr(), self.dtype, self.n,
                                     self.p, X.stride(0), self.k, rk.ctypes.data,
                                     lptr.ctypes.data, rows.ctypes.data, K, seed, base,
                                     self.ws_bytes, stream))
        self.ctx = ctx

    def step(self, iters=1):
        _check(load().godec_mse_step(self.ctx, iters))

    def factors(self, i):
        """(U, V): L^i on the label's rows is U V^T (U n_i x r_i, V p x r_i)."""
        import torch
        U = torch.empty((len(self.labels[i]), self.ranks[i]), dtype=self.X.dtype,
                        device=self.X.device)
        V = torch.empty((self.p, self.ranks[i]), dtype=self.X.dtype, device=self.X.device)
        _check(load().godec_mse_get_factors(self.ctx, i, U.data_ptr() if U.numel() else
                                            V.data_ptr(), V.data_ptr()))
        return U, V

    def S(self):
        import torch
        kk = max(self.K, 1)
        idx = torch.empty(kk, dtype=torch.int64, device=self.X.device)
        val = torch.empty(kk, dtype=self.X.dtype, device=self.X.device)
        nnz = _I64(0)
        _check(load().godec_mse_get_S(self.ctx, idx.data_ptr(), val.data_ptr(),
                                      ctypes.byref(nnz)))
        return idx[:nnz.value], val[:nnz.value]

    def residual(self):
        import torch
        E = torch.empty((self.n, self.p), dtype=self.X.dtype, device=self.X.device)
        _check(load().godec_mse_get_residual(self.ctx, E.data_ptr(), self.p))
        return E

    def info(self):
        info = godec_mse_info()
        _check(load().godec_mse_get_info(self.ctx, ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if getattr(self, "ctx", None) is not None:
            load().godec_mse_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
