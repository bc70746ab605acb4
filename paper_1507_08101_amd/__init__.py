"""Python binding of libsellcs: SELL-C-sigma sparse matrix times (block) vector on MI355X.

Argument marshalling only. Every computation runs in the HIP kernels of ``libsellcs.so``
(built in-tree by ``__graft_entry__.build()``); there is no fallback: if the library is
missing, importing its functions raises. PyTorch serves as the source of device memory
and of the current HIP stream (``torch.cuda.current_stream().cuda_stream``).

The raw entry points carry the C names (``sell_build``, ``sell_spmmv``, ``sell_spmmv_aug``,
``sell_spmmv_T``, ``sell_bv_create``, ``sell_bv_copy`` ...). The small classes below wrap
the opaque handles: ``SellMatrix`` (a device SELL-C-sigma matrix) and block-vector views of
torch tensors.
"""
from __future__ import annotations

import collections
import ctypes as ct
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsellcs.so")

# ---- constants of include/sellcs.h
SELL_F64, SELL_F32, SELL_BF16 = 0, 1, 2
SELL_ROW_MAJOR, SELL_COL_MAJOR = 0, 1
SELL_OK, SELL_ERR_ARG, SELL_ERR_SHAPE, SELL_ERR_DTYPE = 0, -1, -2, -3
SELL_ERR_UNSUPPORTED, SELL_ERR_OOM, SELL_ERR_HIP, SELL_ERR_STATE = -4, -5, -6, -7
SHIFT, VSHIFT, SCALE, AXPBY = 0x01, 0x02, 0x04, 0x08
DOT_YY, DOT_XY, DOT_XX, CHAIN = 0x10, 0x20, 0x40, 0x80
DOTS = DOT_YY | DOT_XY | DOT_XX

DTYPE_NAMES = {"f64": SELL_F64, "f32": SELL_F32, "bf16": SELL_BF16}


class SellError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})")


class sell_spmv_opts(ct.Structure):
    _fields_ = [("flags", ct.c_uint32), ("alpha", ct.c_double), ("beta", ct.c_double),
                ("gamma", ct.c_double), ("gamma_v", ct.c_void_p), ("delta", ct.c_double),
                ("eta", ct.c_double), ("dot", ct.c_void_p)]


class sell_info_t(ct.Structure):
    _fields_ = [("nrows", ct.c_int64), ("ncols", ct.c_int64), ("nnz", ct.c_int64),
                ("stored", ct.c_int64), ("nchunks", ct.c_int64), ("sigma", ct.c_int64),
                ("C", ct.c_int32), ("vdtype", ct.c_int32), ("on_device", ct.c_int32),
                ("device", ct.c_int32), ("ntiles", ct.c_int32), ("has_perm", ct.c_int32),
                ("matrix_bytes", ct.c_int64), ("batch", ct.c_int32), ("batch_wide", ct.c_int32)]


class sell_tune_result(ct.Structure):
    _fields_ = [("C", ct.c_int32), ("sigma", ct.c_int64), ("vpt", ct.c_int32), ("blocks_per_cu", ct.c_int32),
                ("us", ct.c_double), ("default_us", ct.c_double), ("trials", ct.c_int32), ("slice", ct.c_int32),
                ("waves", ct.c_int32), ("batch", ct.c_int32)]


class sell_cg_stats(ct.Structure):
    _fields_ = [("iterations", ct.c_int64), ("refinements", ct.c_int64), ("relres", ct.c_double),
                ("converged", ct.c_int32)]


_P = ct.c_void_p
_I = ct.c_int
_I32 = ct.c_int32
_I64 = ct.c_int64
_D = ct.c_double
_PP = ct.POINTER(ct.c_void_p)

_SIGNATURES = {
    "sell_strerror": ([_I], ct.c_char_p),
    "sell_version": ([], _I),
    "sell_build": ([_PP, _I64, _I64, _P, _P, _P, _I32, _I64, _I, _P], _I),
    "sell_build_host": ([_PP, _I64, _I64, _P, _P, _P, _I32, _I64, _I], _I),
    "sell_build_device": ([_PP, _I64, _I64, _P, _P, _P, _I32, _I64, _I, _P], _I),
    "sell_update_values": ([_P, _P, _P], _I),
    "sell_update_values_device": ([_P, _P, _P], _I),
    "sell_export_csr": ([_P, _P, _P, _P], _I),
    "sell_export_sell": ([_P, _P, _P, _P, _P, _P], _I),
    "sell_info": ([_P, ct.POINTER(sell_info_t)], _I),
    "sell_destroy": ([_P], _I),
    "sell_bv_create": ([_PP, _I64, _I32, _I, _I, _P, _I64], _I),
    "sell_bv_destroy": ([_P], _I),
    "sell_bv_data": ([_P, _PP, ct.POINTER(_I64), ct.POINTER(_I64), ct.POINTER(_I32), ct.POINTER(_I32),
                      ct.POINTER(_I32)], _I),
    "sell_bv_copy": ([_P, _P, _P], _I),
    "sell_spmmv": ([_P, _P, _P, _P], _I),
    "sell_spmmv_aug": ([_P, _P, _P, _P, ct.POINTER(sell_spmv_opts), _P], _I),
    "sell_spmmv_aug_noalloc": ([_P, _P, _P, _P, ct.POINTER(sell_spmv_opts), _P], _I),
    "sell_spmmv_T": ([_P, _P, _P, _I, _P], _I),
    "sell_kpm": ([_P, _P, _P, _I64, _D, _D, _P, ct.POINTER(_I), _P, _P], _I),
    "sell_cg": ([_P, _P, _P, _D, _I64, ct.POINTER(sell_cg_stats), _P], _I),
    "sell_cg_mixed": ([_P, _P, _P, _P, _D, _I64, _D, _I64, ct.POINTER(sell_cg_stats), _P], _I),
    "sell_probe_bandwidth": ([_I, _P, _P, _I64, _P], _I),
    "sell_probe_stream": ([_I, _I, _I, _I, _I, _P, _P, _I64, _P], _I),
    "sell_debug_fail_alloc": ([_I64], _I),
    "sell_debug_live_allocs": ([ct.POINTER(_I64)], _I),
    "sell_probe_gather": ([_P, _I64, _I32, _P, _I64, _P, _P], _I),
    "sell_kpm_dos": ([_P, _I64, _I32, _I32, _D, _D, _P, _I64, _P, _P], _I),
    "sell_grad_values": ([_P, _P, _P, _D, _I, _P, _P], _I),
    "sell_cheb_forward": ([_P, _P, _P, _I64, _D, _D, _I64, _P, _P], _I),
    "sell_cheb_filter": ([_P, _P, _P, _I64, _P, _D, _D, _P], _I),
    "sell_cheb_backward": ([_P, _P, _I64, _D, _D, _I64, _P, _P, _P, _P], _I),
    "sell_tsmttsm": ([_P, _P, _D, _D, _P, _I64, _I, _P], _I),
    "sell_tsmm": ([_P, _P, _I64, _D, _D, _P, _P], _I),
    "sell_tsmm_inplace": ([_P, _P, _I64, _D, _D, _P], _I),
    "sell_set_launch": ([_P, _I32, _I32], _I),
    "sell_set_slice": ([_P, _I32], _I),
    "sell_set_waves": ([_P, _I32], _I),
    "sell_set_batch": ([_P, _I32], _I),
    "sell_set_stage": ([_P, _I32, _I32], _I),
    "sell_autotune": ([_I64, _I64, _P, _P, _P, _I, _I32, ct.c_uint32, ct.POINTER(sell_tune_result), _P], _I),
    "sell_batch_create": ([_PP, _I32, _PP], _I),
    "sell_batch_destroy": ([_P], _I),
    "sell_batch_info": ([_P, ct.POINTER(_I32), ct.POINTER(_I64), ct.POINTER(_I64)], _I),
    "sell_batch_spmmv_aug": ([_P, _P, _P, _P, ct.POINTER(sell_spmv_opts), _P], _I),
    "sell_batch_set_widths": ([_P, _P], _I),
    "sell_batch_packed_sizes": ([_P, ct.POINTER(_I64), ct.POINTER(_I64), ct.POINTER(_I64)], _I),
    "sell_batch_spmmv_aug_packed": ([_P, _P, _P, _P, ct.POINTER(sell_spmv_opts), _P], _I),
    "sell_batch_cg": ([_P, _P, _P, _P, _D, _I64, _D, _I64, ct.c_uint32, ct.POINTER(sell_cg_stats), _P], _I),
}

_lib = None


def lib():
    """The loaded libsellcs; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsellcs.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().sell_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library itself is absent
        return "error"


def _ok(rc: int, what: str) -> None:
    if rc != SELL_OK:
        raise SellError(rc, what)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _stream(stream=None):
    """HIP stream handle as void*: an explicit int/handle, or torch's current stream."""
    if stream is not None:
        return ct.c_void_p(int(stream))
    import torch

    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(dt) -> int:
    if isinstance(dt, int):
        return dt
    if isinstance(dt, str):
        return DTYPE_NAMES[dt]
    import torch

    return {torch.float64: SELL_F64, torch.float32: SELL_F32, torch.bfloat16: SELL_BF16}[dt]


# ==================================================================== sparse matrices


def _csr_arrays(rowptr, col, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    return rowptr, col, val


def sell_build(nrows, ncols, rowptr, col, val, C, sigma, vdt=SELL_F64, stream=None, host_only=False):
    """Build a SELL-C-sigma matrix from host CSR arrays; returns the opaque handle."""
    rowptr, col, val = _csr_arrays(rowptr, col, val)
    if rowptr.size != nrows + 1:
        raise SellError(SELL_ERR_ARG, "sell_build: rowptr must have nrows + 1 entries")
    nnz = int(rowptr[-1]) if rowptr.size else 0
    if col.size < nnz or val.size < nnz:
        raise SellError(SELL_ERR_ARG, "sell_build: col/val shorter than rowptr[-1]")
    h = ct.c_void_p()
    if host_only:
        rc = lib().sell_build_host(ct.byref(h), nrows, ncols, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val),
                                   int(C), int(sigma), _dtype_code(vdt))
    else:
        rc = lib().sell_build(ct.byref(h), nrows, ncols, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val), int(C),
                              int(sigma), _dtype_code(vdt), _stream(stream))
    _ok(rc, "sell_build")
    return h


def sell_build_device(nrows, ncols, rowptr, col, val, C, sigma, vdt=SELL_F64, stream=None):
    """Build on the GPU from CSR arrays in device memory (torch tensors: int64 rowptr, int32
    col, float64 val, contiguous, on the current device); returns the opaque handle."""
    import torch

    for t, dt in ((rowptr, torch.int64), (col, torch.int32), (val, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise SellError(SELL_ERR_ARG, "sell_build_device: rowptr int64, col int32, val float64 device tensors")
    if rowptr.numel() != nrows + 1:
        raise SellError(SELL_ERR_ARG, "sell_build_device: rowptr must have nrows + 1 entries")
    h = ct.c_void_p()
    _ok(lib().sell_build_device(ct.byref(h), int(nrows), int(ncols), ct.c_void_p(rowptr.data_ptr()),
                                ct.c_void_p(col.data_ptr()) if col.numel() else None,
                                ct.c_void_p(val.data_ptr()) if val.numel() else None, int(C), int(sigma),
                                _dtype_code(vdt), _stream(stream)), "sell_build_device")
    return h


def sell_info(h) -> dict:
    info = sell_info_t()
    _ok(lib().sell_info(h, ct.byref(info)), "sell_info")
    return {k: getattr(info, k) for k, _ in sell_info_t._fields_}


def sell_export_csr(h):
    i = sell_info(h)
    rowptr = np.empty(i["nrows"] + 1, np.int64)
    col = np.empty(i["nnz"], np.int32)
    val = np.empty(i["nnz"], np.float64)
    _ok(lib().sell_export_csr(h, _np_ptr(rowptr), _np_ptr(col), _np_ptr(val)), "sell_export_csr")
    return rowptr, col, val


def sell_export_sell(h):
    i = sell_info(h)
    perm = np.empty(i["nchunks"] * i["C"], np.int32)
    cl = np.empty(i["nchunks"], np.int32)
    cs = np.empty(i["nchunks"] + 1, np.int64)
    col = np.empty(i["stored"], np.int32)
    val = np.empty(i["stored"], np.float64)
    _ok(lib().sell_export_sell(h, _np_ptr(perm), _np_ptr(cl), _np_ptr(cs), _np_ptr(col), _np_ptr(val)),
        "sell_export_sell")
    return perm, cl, cs, col, val


def sell_update_values(h, val, stream=None):
    """New values (CSR order). ``val`` is a host numpy array or a float64 device tensor."""
    if isinstance(val, np.ndarray):
        v = np.ascontiguousarray(val, dtype=np.float64)
        _ok(lib().sell_update_values(h, _np_ptr(v), _stream(stream)), "sell_update_values")
    else:
        import torch

        assert val.dtype == torch.float64 and val.is_cuda and val.is_contiguous()
        _ok(lib().sell_update_values_device(h, ct.c_void_p(val.data_ptr()), _stream(stream)),
            "sell_update_values_device")


def sell_destroy(h) -> None:
    if h:
        lib().sell_destroy(h)


class SellMatrix:
    """Owner of a SELL-C-sigma matrix handle."""

    def __init__(self, handle):
        self.handle = handle
        self.info = sell_info(handle)
        # bumped by every value update: lets a saved computation tell whether the values it
        # used are still the ones on the device
        self.values_version = 0

    @classmethod
    def from_csr(cls, A, C=32, sigma=1, dtype="f64", stream=None, host_only=False):
        """``A`` has nrows, ncols, rowptr, col, val (e.g. a scipy CSR wrapper or synth.CSR)."""
        h = sell_build(A.nrows, A.ncols, A.rowptr, A.col, A.val, C, sigma, _dtype_code(dtype), stream,
                       host_only=host_only)
        return cls(h)

    @property
    def nrows(self):
        return self.info["nrows"]

    @property
    def ncols(self):
        return self.info["ncols"]

    @property
    def vector_dtype(self):
        import torch

        return torch.float64 if self.info["vdtype"] == SELL_F64 else torch.float32

    def set_launch(self, vpt=0, blocks_per_cu=0):
        """Launch parameters of the product kernels for this matrix (0 = defaults)."""
        _ok(lib().sell_set_launch(self.handle, int(vpt), int(blocks_per_cu)), "sell_set_launch")

    def set_waves(self, waves=0):
        """Grid of the product launches in waves of resident workgroups (0 = one wave)."""
        _ok(lib().sell_set_waves(self.handle, int(waves)), "sell_set_waves")

    def set_slice(self, slice_width=0):
        """Process wider blocks in launches over column slices of this width (0 = whole block)."""
        _ok(lib().sell_set_slice(self.handle, int(slice_width)), "sell_set_slice")

    def set_stage(self, stage=0, tile_stride=0):
        """Gather x through the LDS page cache (1) or from global memory (0); tile_stride > 0
        makes each workgroup of a staged launch take every tile_stride-th stage tile."""
        _ok(lib().sell_set_stage(self.handle, int(stage), int(tile_stride)), "sell_set_stage")

    def set_batch(self, batch=0):
        """Index batch length of the products (5, 7 or 8; 0 = the construction's choice)."""
        _ok(lib().sell_set_batch(self.handle, int(batch)), "sell_set_batch")
        self.info = sell_info(self.handle)

    @classmethod
    def from_device_csr(cls, nrows, ncols, rowptr, col, val, C=32, sigma=1, dtype="f64", stream=None):
        """Build on the GPU from CSR arrays that are device tensors."""
        return cls(sell_build_device(nrows, ncols, rowptr, col, val, C, sigma, _dtype_code(dtype), stream))

    @classmethod
    def from_csr_tuned(cls, A, b, dtype="f64", stream=None, cache=True):
        """Build with the format and launch parameters chosen by ``sell_autotune``; the choice
        is kept in ``self.tune``."""
        t = sell_autotune(A, b, dtype, stream=stream, cache=cache)
        M = cls.from_csr(A, C=t["C"], sigma=t["sigma"], dtype=dtype, stream=stream)
        M.set_launch(t["vpt"], t["blocks_per_cu"])
        M.set_slice(t["slice"])
        M.set_waves(t["waves"])
        M.set_batch(t["batch"])
        M.tune = t
        return M

    def export_csr(self):
        return sell_export_csr(self.handle)

    def export_sell(self):
        return sell_export_sell(self.handle)

    def update_values(self, val, stream=None):
        if not self.info["on_device"]:
            stream = 0  # host-only matrix: no stream involved
        sell_update_values(self.handle, val, stream)
        self.values_version += 1

    def close(self):
        if self.handle:
            sell_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - best effort at interpreter exit
        try:
            self.close()
        except Exception:
            pass


# ==================================================================== block vectors


class BlockVector:
    """A libsellcs block vector: a view of a 2-D torch tensor (row- or column-major) or an
    owned allocation. Keeps the tensor alive while the view exists."""

    def __init__(self, handle, tensor=None):
        self.handle = handle
        self.tensor = tensor

    @classmethod
    def view(cls, t):
        if t.dim() == 1:
            t = t.view(-1, 1)
        if t.dim() != 2:
            raise SellError(SELL_ERR_ARG, "block vectors are 2-D")
        n, b = t.shape
        if b == 1 or (t.stride(1) == 1 and t.stride(0) >= b):
            lay, ld = SELL_ROW_MAJOR, max(t.stride(0), b) if n > 1 else b
        elif t.stride(0) == 1 and t.stride(1) >= n:
            lay, ld = SELL_COL_MAJOR, t.stride(1)
        else:
            raise SellError(SELL_ERR_ARG, "tensor is neither row- nor column-major")
        h = ct.c_void_p()
        ptr = ct.c_void_p(t.data_ptr()) if t.numel() else None  # empty: a zero-size owned object
        _ok(lib().sell_bv_create(ct.byref(h), n, b, _dtype_code(t.dtype), lay, ptr, ld), "sell_bv_create")
        return cls(h, t)

    def close(self):
        if self.handle:
            lib().sell_bv_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class _CachedView:
    """A block-vector descriptor from the view cache (owned by the cache, not by this object)."""

    __slots__ = ("handle", "tensor")

    def __init__(self, handle, tensor):
        self.handle = handle
        self.tensor = tensor


# Descriptors of tensor views, keyed by what they describe (address, shape, strides, type): a
# descriptor does not own the memory, so one made for an earlier tensor with the same key
# describes the same memory. One cache per thread (an entry is only evicted by the thread that
# uses it); least recently used entries are destroyed beyond the bound.
_VIEW_TLS = threading.local()
_VIEW_CACHE_MAX = 512


def _bv(x):
    if isinstance(x, (BlockVector, _CachedView)):
        return x
    cache = getattr(_VIEW_TLS, "cache", None)
    if cache is None:
        cache = _VIEW_TLS.cache = collections.OrderedDict()
    key = (x.data_ptr(), tuple(x.shape), tuple(x.stride()), x.dtype)
    h = cache.get(key)
    if h is None:
        v = BlockVector.view(x)
        h, v.handle = v.handle, None  # the cache takes the descriptor over
        cache[key] = h
        if len(cache) > _VIEW_CACHE_MAX:
            _, old = cache.popitem(last=False)
            lib().sell_bv_destroy(old)
    else:
        cache.move_to_end(key)
    return _CachedView(h, x)


def sell_bv_create(nrows, ncols, dtype, layout=SELL_ROW_MAJOR, data=None, ld=0):
    h = ct.c_void_p()
    _ok(lib().sell_bv_create(ct.byref(h), nrows, ncols, _dtype_code(dtype), layout,
                             None if data is None else ct.c_void_p(int(data)), ld), "sell_bv_create")
    return h


def sell_bv_destroy(h):
    lib().sell_bv_destroy(h)


def sell_bv_copy(dst, src, stream=None):
    """dst[:] = src with layout/type conversion (tensors or BlockVector)."""
    d, s = _bv(dst), _bv(src)
    _ok(lib().sell_bv_copy(d.handle, s.handle, _stream(stream)), "sell_bv_copy")


# ==================================================================== products


def _mat(A):
    return A.handle if isinstance(A, SellMatrix) else A


def sell_spmmv(A, X, Y, stream=None):
    """Y = A X (tensors of the matrix's vector type)."""
    x, y = _bv(X), _bv(Y)
    _ok(lib().sell_spmmv(_mat(A), x.handle, y.handle, _stream(stream)), "sell_spmmv")


def make_opts(flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None, delta=0.0, eta=1.0, dot=None):
    o = sell_spmv_opts()
    o.flags = int(flags)
    o.alpha, o.beta, o.gamma, o.delta, o.eta = float(alpha), float(beta), float(gamma), float(delta), float(eta)
    keep = None
    if gamma_v is not None:
        keep = np.ascontiguousarray(gamma_v, dtype=np.float64)
        o.gamma_v = keep.ctypes.data
    if dot is not None:
        o.dot = dot.data_ptr()
    return o, keep


def sell_spmmv_aug(A, X, Y, Z=None, flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None, delta=0.0,
                   eta=1.0, dot=None, stream=None):
    """y = alpha (A - gamma I) x + beta y with optional dots (into the float64 device tensor
    ``dot`` of 3b entries) and chained z = delta z + eta y."""
    x, y = _bv(X), _bv(Y)
    z = _bv(Z) if Z is not None else None
    o, keep = make_opts(flags, alpha, beta, gamma, gamma_v, delta, eta, dot)
    _ok(lib().sell_spmmv_aug(_mat(A), x.handle, y.handle, z.handle if z else None, ct.byref(o), _stream(stream)),
        "sell_spmmv_aug")
    del keep


def sell_spmmv_aug_noalloc(A, X, Y, Z=None, flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None, delta=0.0,
                           eta=1.0, dot=None, stream=None):
    """sell_spmmv_aug without any device allocation: the dot partials live in the library's
    fixed per-device array (calls that overlap on one device race on it)."""
    x, y = _bv(X), _bv(Y)
    z = _bv(Z) if Z is not None else None
    o, keep = make_opts(flags, alpha, beta, gamma, gamma_v, delta, eta, dot)
    _ok(lib().sell_spmmv_aug_noalloc(_mat(A), x.handle, y.handle, z.handle if z else None, ct.byref(o),
                                     _stream(stream)), "sell_spmmv_aug_noalloc")
    del keep


def sell_spmmv_T(A, X, Y, deterministic=True, stream=None):
    """Y = A^T X. deterministic (the default): the forward kernel on a SELL copy of A^T, built
    by the first such call; False: scatter with floating-point atomics (no copy, slower)."""
    x, y = _bv(X), _bv(Y)
    _ok(lib().sell_spmmv_T(_mat(A), x.handle, y.handle, 1 if deterministic else 0, _stream(stream)),
        "sell_spmmv_T")


def sell_kpm(A, V, W, M, s, c, mu, step_ms=None, stream=None):
    """Kernel polynomial method recurrence; returns True if v_M ended in W. ``step_ms``: a
    float32 numpy array of M entries to receive per-product HIP-event durations (the call is
    then synchronous)."""
    v, w = _bv(V), _bv(W)
    last = ct.c_int(0)
    if step_ms is not None:
        assert step_ms.dtype == np.float32 and step_ms.size >= M and step_ms.flags.c_contiguous
    _ok(lib().sell_kpm(_mat(A), v.handle, w.handle, int(M), float(s), float(c), ct.c_void_p(mu.data_ptr()),
                       ct.byref(last), _np_ptr(step_ms), _stream(stream)), "sell_kpm")
    return bool(last.value)


SELL_KPM_NONE, SELL_KPM_JACKSON = 0, 1


def sell_kpm_dos(mu, b, E, s, c=0.0, kernel="jackson", rho=None, stream=None):
    """Density of states at the energies E (float64 device tensor) from block KPM moments mu
    (float64 device tensor of nmom * b entries in sell_kpm's layout); returns rho (a new
    tensor unless given)."""
    import torch

    if mu.dtype != torch.float64 or E.dtype != torch.float64 or not (mu.is_contiguous() and E.is_contiguous()):
        raise SellError(-1, "sell_kpm_dos: mu and E must be contiguous float64")
    if mu.numel() % b:
        raise SellError(-1, "sell_kpm_dos: mu does not hold whole rows of b moments")
    if rho is None:
        rho = torch.empty_like(E)
    kern = {"jackson": SELL_KPM_JACKSON, "none": SELL_KPM_NONE}[kernel]
    _ok(lib().sell_kpm_dos(ct.c_void_p(mu.data_ptr()), int(mu.numel() // b), int(b), kern, float(s), float(c),
                           ct.c_void_p(E.data_ptr()) if E.numel() else None, int(E.numel()),
                           ct.c_void_p(rho.data_ptr()) if rho.numel() else None, _stream(stream)), "sell_kpm_dos")
    return rho


def sell_cg(A, B, X, tol=1e-10, maxit=100000, stream=None):
    """FP64 CG per column of B (A symmetric positive definite); X: initial guess -> solution."""
    st = sell_cg_stats()
    b, x = _bv(B), _bv(X)  # the views must outlive the call
    _ok(lib().sell_cg(_mat(A), b.handle, x.handle, float(tol), int(maxit), ct.byref(st), _stream(stream)),
        "sell_cg")
    return {k: getattr(st, k) for k, _ in sell_cg_stats._fields_}


def sell_cg_mixed(A64, Alo, B, X, tol=1e-10, maxit=100000, inner_tol=0.1, inner_maxit=1000, stream=None):
    """CG with FP64 iterative refinement around an FP32-vector inner solve on Alo."""
    st = sell_cg_stats()
    b, x = _bv(B), _bv(X)
    _ok(lib().sell_cg_mixed(_mat(A64), _mat(Alo), b.handle, x.handle, float(tol), int(maxit), float(inner_tol),
                            int(inner_maxit), ct.byref(st), _stream(stream)), "sell_cg_mixed")
    return {k: getattr(st, k) for k, _ in sell_cg_stats._fields_}


# ==================================================================== parameter choice

SELL_TUNE_NO_CACHE = 0x1


def sell_autotune(A, b, dtype="f64", stream=None, cache=True):
    """Time candidate (C, sigma, columns per lane, workgroups per CU) for products of width
    ``b`` with the CSR matrix ``A``; returns the choice and its timings as a dict."""
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    r = sell_tune_result()
    _ok(lib().sell_autotune(int(A.nrows), int(A.ncols), _np_ptr(rowptr), _np_ptr(col), _np_ptr(val),
                            _dtype_code(dtype), int(b), 0 if cache else SELL_TUNE_NO_CACHE, ct.byref(r),
                            _stream(stream)), "sell_autotune")
    return {k: getattr(r, k) for k, _ in sell_tune_result._fields_}


# ==================================================================== batches

SELL_BATCH_GRAPH = 0x1


class SellBatch:
    """A batch of device matrices processed by single launches. Holds references to the
    matrices (which must stay open while the batch exists)."""

    def __init__(self, mats):
        self.mats = list(mats)
        arr = (ct.c_void_p * len(self.mats))(*[_mat(m).value if isinstance(_mat(m), ct.c_void_p) else _mat(m)
                                                for m in self.mats])
        h = ct.c_void_p()
        _ok(lib().sell_batch_create(arr, len(self.mats), ct.byref(h)), "sell_batch_create")
        self.handle = h
        cnt, rows, cols = _I32(), _I64(), _I64()
        _ok(lib().sell_batch_info(h, ct.byref(cnt), ct.byref(rows), ct.byref(cols)), "sell_batch_info")
        self.count, self.rows, self.cols = cnt.value, rows.value, cols.value

    def set_widths(self, widths=None):
        """Block width of each matrix, for the packed operands of sell_batch_spmmv_aug_packed
        (None clears them)."""
        if widths is None:
            _ok(lib().sell_batch_set_widths(self.handle, None), "sell_batch_set_widths")
            self.widths = None
            return
        w = np.ascontiguousarray(widths, dtype=np.int32)
        if w.shape != (self.count,):
            raise SellError(-1, "sell_batch_set_widths: one width per matrix")
        _ok(lib().sell_batch_set_widths(self.handle, w.ctypes.data_as(ct.c_void_p)), "sell_batch_set_widths")
        self.widths = w.copy()

    def packed_sizes(self):
        """(elements of packed X, elements of packed Y / Z, doubles of packed dots)."""
        x, y, d = _I64(), _I64(), _I64()
        _ok(lib().sell_batch_packed_sizes(self.handle, ct.byref(x), ct.byref(y), ct.byref(d)),
            "sell_batch_packed_sizes")
        return x.value, y.value, d.value

    def close(self):
        if self.handle:
            lib().sell_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def sell_batch_spmmv_aug(Bt, X, Y, Z=None, flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None, delta=0.0,
                         eta=1.0, dot=None, stream=None):
    """The augmented product for every matrix of the batch in one launch; X, Y, Z hold the
    matrices' operands stacked by rows; ``dot`` receives 3b doubles per matrix."""
    x, y = _bv(X), _bv(Y)
    z = _bv(Z) if Z is not None else None
    o, keep = make_opts(flags, alpha, beta, gamma, gamma_v, delta, eta, dot)
    _ok(lib().sell_batch_spmmv_aug(Bt.handle, x.handle, y.handle, z.handle if z else None, ct.byref(o),
                                   _stream(stream)), "sell_batch_spmmv_aug")
    del keep


def sell_batch_spmmv_aug_packed(Bt, X, Y, Z=None, flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None, delta=0.0,
                                eta=1.0, dot=None, stream=None):
    """The batched product over packed operands of per-matrix widths (set with
    ``SellBatch.set_widths``): X, Y, Z are contiguous device tensors holding the matrices'
    blocks one after another, each at its own width; ``dot`` receives the packed dots."""
    import torch

    nx, ny, _ = Bt.packed_sizes()
    want = torch.float64 if Bt.mats[0].info["vdtype"] == SELL_F64 else torch.float32
    for t, need in ((X, nx), (Y, ny), (Z, ny)):
        if t is not None and (not t.is_contiguous() or t.numel() != need):
            raise SellError(-2, "sell_batch_spmmv_aug_packed: operand is not the packed size")
        if t is not None and t.dtype != want:
            raise SellError(-3, "sell_batch_spmmv_aug_packed: operand is not the batch's vector type")
    o, keep = make_opts(flags, alpha, beta, gamma, gamma_v, delta, eta, dot)
    _ok(lib().sell_batch_spmmv_aug_packed(Bt.handle, ct.c_void_p(X.data_ptr()) if X.numel() else None,
                                          ct.c_void_p(Y.data_ptr()) if Y.numel() else None,
                                          ct.c_void_p(Z.data_ptr()) if Z is not None and Z.numel() else None,
                                          ct.byref(o), _stream(stream)), "sell_batch_spmmv_aug_packed")
    del keep


def sell_batch_cg(A64, Alo, B, X, tol=1e-10, maxit=100000, inner_tol=0.1, inner_maxit=1000, graph=True,
                  stream=None):
    """CG for every system of the batch (FP64, or FP32 iterations refined in FP64 when Alo is
    given); returns one stats dict per system."""
    st = (sell_cg_stats * A64.count)()
    b, x = _bv(B), _bv(X)
    _ok(lib().sell_batch_cg(A64.handle, Alo.handle if Alo is not None else None, b.handle, x.handle, float(tol),
                            int(maxit), float(inner_tol), int(inner_maxit), SELL_BATCH_GRAPH if graph else 0, st,
                            _stream(stream)), "sell_batch_cg")
    return [{k: getattr(e, k) for k, _ in sell_cg_stats._fields_} for e in st]


def sell_debug_fail_alloc(k):
    """Test hook: the k-th next allocation of the library fails as out of memory (0 clears)."""
    _ok(lib().sell_debug_fail_alloc(int(k)), "sell_debug_fail_alloc")


def sell_debug_live_allocs():
    """Test hook: device and pinned host allocations the library currently holds."""
    n = _I64()
    _ok(lib().sell_debug_live_allocs(ct.byref(n)), "sell_debug_live_allocs")
    return n.value


def sell_probe_bandwidth(kind, dst, src, nbytes, stream=None):
    _ok(lib().sell_probe_bandwidth(int(kind), ct.c_void_p(dst.data_ptr()),
                                   ct.c_void_p(src.data_ptr()) if src is not None else None, int(nbytes),
                                   _stream(stream)), "sell_probe_bandwidth")


def sell_probe_stream(reads, writes, unroll, nontemporal, grid, dst, src, nbytes, stream=None):
    """Streaming probe: ``reads`` streams of ``nbytes`` each, back to back in ``src``, summed into
    ``dst`` (``writes`` = 1) or reduced to one partial per workgroup in ``dst`` (``writes`` = 0)."""
    _ok(lib().sell_probe_stream(int(reads), int(writes), int(unroll), int(nontemporal), int(grid),
                                ct.c_void_p(dst.data_ptr()), ct.c_void_p(src.data_ptr()) if src is not None else None,
                                int(nbytes), _stream(stream)), "sell_probe_stream")


def sell_probe_gather(x, idx, out, stream=None):
    """Random-gather probe: reads row idx[i] of x (a contiguous device tensor of rows of 8, 16,
    32 or 64 bytes) for every i; idx is a device int32 tensor, out a device float64 tensor."""
    import torch

    if not (x.is_contiguous() and idx.is_contiguous() and idx.dtype == torch.int32):
        raise SellError(-1, "sell_probe_gather: x and idx must be contiguous, idx int32")
    row_bytes = x.element_size() * (x.shape[1] if x.dim() == 2 else 1)
    _ok(lib().sell_probe_gather(ct.c_void_p(x.data_ptr()), int(x.shape[0]), int(row_bytes),
                                ct.c_void_p(idx.data_ptr()), int(idx.numel()), ct.c_void_p(out.data_ptr()),
                                _stream(stream)), "sell_probe_gather")


# ==================================================================== value gradients


def sell_cheb_filter(A, X, coef, s, c=0.0, Z=None, stream=None):
    """Z = sum_m coef[m] T_m((A - cI)/s) X (each recurrence step one augmented product with the
    chained accumulation); returns Z (a new tensor unless given)."""
    import torch

    coef = np.ascontiguousarray(coef, dtype=np.float64)
    if coef.ndim != 1 or coef.size < 1:
        raise SellError(-1, "sell_cheb_filter: coef must hold at least one coefficient")
    if Z is None:
        Z = torch.empty_like(X)
    x, z = _bv(X), _bv(Z)
    _ok(lib().sell_cheb_filter(_mat(A), x.handle, z.handle, int(coef.size - 1), coef.ctypes.data_as(ct.c_void_p),
                               float(s), float(c), _stream(stream)), "sell_cheb_filter")
    return Z


def sell_grad_values(A, G, X, dval, alpha=1.0, accumulate=False, stream=None):
    """dval (float64 device tensor of nnz, CSR order) (+)= alpha * sum_j G[row, j] X[col, j]."""
    g, x = _bv(G), _bv(X)
    _ok(lib().sell_grad_values(_mat(A), g.handle, x.handle, float(alpha), 1 if accumulate else 0,
                               ct.c_void_p(dval.data_ptr()) if dval.numel() else None, _stream(stream)),
        "sell_grad_values")


def cheb_ckpt_elems(n, b, N, K):
    """Elements of the checkpoint buffer of sell_cheb_forward: 2 ceil(N / K) n b."""
    return 2 * ((N + K - 1) // K) * n * b


def sell_cheb_forward(A, X, Y, N, s, c=0.0, K=10, ckpt=None, stream=None):
    x, y = _bv(X), _bv(Y)
    _ok(lib().sell_cheb_forward(_mat(A), x.handle, y.handle, int(N), float(s), float(c), int(K),
                                None if ckpt is None else ct.c_void_p(ckpt.data_ptr()), _stream(stream)),
        "sell_cheb_forward")


def sell_cheb_backward(A, G, N, s, c, K, ckpt, dX, dval, stream=None):
    g, dx = _bv(G), _bv(dX)
    _ok(lib().sell_cheb_backward(_mat(A), g.handle, int(N), float(s), float(c), int(K), ct.c_void_p(ckpt.data_ptr()),
                                 dx.handle, ct.c_void_p(dval.data_ptr()) if dval.numel() else None,
                                 _stream(stream)), "sell_cheb_backward")


# ==================================================================== tall-skinny kernels


def sell_tsmttsm(V, W, X, alpha=1.0, beta=0.0, kahan=False, stream=None):
    """X (m x k float64 device tensor) = alpha V^T W + beta X."""
    v, w = _bv(V), _bv(W)
    _ok(lib().sell_tsmttsm(v.handle, w.handle, float(alpha), float(beta), ct.c_void_p(X.data_ptr()), X.stride(0),
                           1 if kahan else 0, _stream(stream)), "sell_tsmttsm")


def sell_tsmm(V, X, W, alpha=1.0, beta=0.0, stream=None):
    """W = alpha V X + beta W (X: m x k float64 device tensor)."""
    v, w = _bv(V), _bv(W)
    _ok(lib().sell_tsmm(v.handle, ct.c_void_p(X.data_ptr()), X.stride(0), float(alpha), float(beta), w.handle,
                        _stream(stream)), "sell_tsmm")


def sell_tsmm_inplace(V, X, alpha=1.0, beta=0.0, stream=None):
    """V = alpha V X + beta V (X: m x m float64 device tensor)."""
    v = _bv(V)
    _ok(lib().sell_tsmm_inplace(v.handle, ct.c_void_p(X.data_ptr()), X.stride(0), float(alpha), float(beta),
                                _stream(stream)), "sell_tsmm_inplace")
