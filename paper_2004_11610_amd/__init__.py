"""Extra-component fast special-function transforms on MI355X (gfx950).

Thin Python binding of the C ABI in include/spt.h: every step of the
precomputation and of the computation stage runs in the HIP library
(libspt.so); this module only marshals arguments.  PyTorch supplies device
memory and streams.
"""

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

from . import _lib
from ._lib import SptError  # noqa: F401

CHEBYSHEV_T, LEGENDRE, JACOBI, LAGUERRE_FN, HERMITE_FN, SINE, COS_POWER = 1, 2, 3, 4, 5, 6, 7
CEXP, LAGUERRE_SPECTRAL = 8, 9  # complex generators
F64, F32, SPLIT_BF16 = 0, 1, 2
MODE_AUTO, MODE_ROW, MODE_DIRECT = 0, 1, 3
FFT_AUTO, FFT_F32, FFT_F64 = 0, 1, 2
PRODUCT_DEFAULT, PRODUCT_TILE, PRODUCT_WINDOW, PRODUCT_CHUNKED, PRODUCT_WINDOW_2W = 0, 1, 2, 3, 4
TUNE_DEFAULT, TUNE_OFF, TUNE_ON, FFT_EIGHT = 0, 1, 2, 3
TUNING_FIELDS = ("product", "window_rhs", "fft_batch", "fft_half", "inv_four")
EXECUTOR_AUTO, EXECUTOR_STAGED, EXECUTOR_PERSISTENT = 0, 1, 2
FAMILIES = {"chebyshev_t": CHEBYSHEV_T, "legendre": LEGENDRE, "jacobi": JACOBI,
            "laguerre_fn": LAGUERRE_FN, "hermite_fn": HERMITE_FN, "sine": SINE,
            "cos_power": COS_POWER, "cexp": CEXP, "laguerre_spectral": LAGUERRE_SPECTRAL}
PRECISIONS = {"f64": F64, "f32": F32, "split_bf16": SPLIT_BF16}


def _stream_ptr(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def _dtype_for(prec, complex_=False):
    import torch
    if complex_:
        return torch.complex128 if prec == F64 else torch.complex64
    return torch.float64 if prec == F64 else torch.float32


class Plan:
    """A plan for y = A x with the N x N special-function matrix of `family`.

    eps is the threshold eps1 (sec. 2.2); the remaining keywords are the
    fields of spt_params (include/spt.h)."""

    def __init__(self, family, N, eps, alpha=0.0, beta=0.0, eps2=0.0, mode=MODE_AUTO,
                 unweighted=False, precisions=0, min_block=0, exact_fft_len=False,
                 panel_rows=0, nodes=None, executor=EXECUTOR_AUTO, power=0, trig_conv_q=0,
                 reduced_fft=0, eta=0.0, period=0.0):
        self._lib = _lib.load()
        self._h = c_void_p()
        p = _lib.SptParams()
        p.alpha, p.beta, p.eps2 = float(alpha), float(beta), float(eps2)
        p.mode, p.unweighted, p.precisions = int(mode), int(bool(unweighted)), int(precisions)
        p.min_block, p.exact_fft_len, p.panel_rows = int(min_block), int(bool(exact_fft_len)), int(panel_rows)
        p.executor = int(executor)
        p.power = int(power)
        p.trig_conv_q = int(trig_conv_q)
        p.reduced_fft = int(reduced_fft)
        p.eta, p.period = float(eta), float(period)
        self._nodes_buf = None
        if nodes is not None:
            self._nodes_buf = (c_double * N)(*[float(v) for v in nodes])
            p.nodes = ctypes.cast(self._nodes_buf, ctypes.POINTER(c_double))
        fam = FAMILIES.get(family, family)
        _lib.check(self._lib.spt_plan_create(byref(self._h), int(fam), byref(p), int(N),
                                             float(eps)))
        self.family, self.N, self.eps = fam, int(N), float(eps)
        self.is_complex = fam in (CEXP, LAGUERRE_SPECTRAL)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if self._h:
            _lib.check(self._lib.spt_plan_destroy(self._h))
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ queries
    def blocks(self):
        """[(L, m_offset, c_lo, c_hi), ...] of the compressed blocks."""
        n = c_int32()
        cap = 64
        arrs = [(c_int32 * cap)() for _ in range(4)]
        _lib.check(self._lib.spt_plan_blocks(self._h, *arrs, cap, byref(n)))
        return [tuple(a[i] for a in arrs) for i in range(n.value)]

    def info(self):
        inf = _lib.SptPlanInfo()
        _lib.check(self._lib.spt_plan_query(self._h, byref(inf)))
        out = {f: getattr(inf, f) for f, _ in inf._fields_ if f not in ("max_abs", "nnz_blk")}
        out["max_abs"] = list(inf.max_abs)[: max(inf.n_blocks, 0)]
        out["nnz_blk"] = list(inf.nnz_blk)[: max(inf.n_blocks, 0)]
        return out

    def nodes(self):
        import numpy as np
        out = np.empty(self.N)
        _lib.check(self._lib.spt_plan_nodes(self._h, out.ctypes.data_as(ctypes.POINTER(c_double))))
        return out

    def compressed_rows(self, blk, row0, nrows):
        """Stored compressed rows of block `blk` as a complex (nrows, L/2+1) array."""
        import numpy as np
        L = self.blocks()[blk][0]
        out = np.zeros((nrows, L // 2 + 1), dtype=np.complex128)
        _lib.check(self._lib.spt_plan_compressed_rows(
            self._h, int(blk), int(row0), int(nrows),
            out.ctypes.data_as(ctypes.POINTER(c_double))))
        return out

    def set_tuning(self, **choices):
        """Launch choices (spt_tuning fields; the others keep their values)."""
        t = _lib.SptTuning()
        _lib.check(self._lib.spt_plan_get_tuning(self._h, byref(t)))
        for k, v in choices.items():
            if k not in TUNING_FIELDS:
                raise ValueError("unknown tuning field %r" % k)
            setattr(t, k, int(v))
        _lib.check(self._lib.spt_plan_set_tuning(self._h, byref(t)))
        return self

    def tuning(self):
        t = _lib.SptTuning()
        _lib.check(self._lib.spt_plan_get_tuning(self._h, byref(t)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def autotune(self, nrhs, prec=F64, cache_path=None, stream=None):
        """spt_autotune: time the launch choices, keep the fastest; returns
        (choices, microseconds per execute, 0 when read from the cache)."""
        prec = PRECISIONS.get(prec, prec)
        t = _lib.SptTuning()
        us = c_double()
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check(self._lib.spt_autotune(self._h, c_int64(nrhs), c_int32(prec),
                                          _stream_ptr(stream), path, byref(t), byref(us)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}, us.value

    def set_exec_wait(self, ticks):
        """Bound of the persistent executor's dependency waits (100 MHz ticks, 0 = 1 s)."""
        _lib.check(self._lib.spt_plan_set_exec_wait(self._h, c_int64(int(ticks))))

    # ------------------------------------------------------------------ work
    def precompute(self, stream=None):
        _lib.check(self._lib.spt_precompute(self._h, _stream_ptr(stream)))
        return self

    def _check_io(self, X, Y, prec):
        import torch
        dt = _dtype_for(prec, self.is_complex)
        if X.dtype != dt or not X.is_cuda or not X.is_contiguous() or X.shape[-1] != self.N:
            raise ValueError("X must be a contiguous CUDA %s tensor of shape (R, %d)" % (dt, self.N))
        R = X.numel() // self.N
        if Y is None:
            Y = torch.empty((R, self.N), dtype=dt, device=X.device)
        if Y.dtype != dt or not Y.is_contiguous() or Y.numel() != R * self.N:
            raise ValueError("Y must be a contiguous %s tensor with R*N elements" % dt)
        return R, Y

    def execute(self, X, Y=None, prec=F64, stream=None):
        """Y = X A^T (Y[r] = A X[r]) for X of shape (R, N) on the device."""
        prec = PRECISIONS.get(prec, prec)
        R, Y = self._check_io(X, Y, prec)
        _lib.check(self._lib.spt_execute(self._h, c_void_p(X.data_ptr()), c_void_p(Y.data_ptr()),
                                         c_int64(R), c_int32(prec), _stream_ptr(stream)))
        return Y

    def execute_noalloc(self, X, Y, prec=F64, stream=None):
        """execute() through spt_execute_noalloc: the workspace is the library's
        static device array (no allocation); Y must be given."""
        prec = PRECISIONS.get(prec, prec)
        if Y is None:
            raise ValueError("execute_noalloc needs the output tensor Y")
        R, Y = self._check_io(X, Y, prec)
        _lib.check(self._lib.spt_execute_noalloc(
            self._h, c_void_p(X.data_ptr()), c_void_p(Y.data_ptr()), c_int64(R), c_int32(prec),
            _stream_ptr(stream)))
        return Y

    def execute_transposed(self, X, Y=None, prec=F64, stream=None):
        """Y = X A (Y[r] = A^T X[r]) for X of shape (R, N) on the device."""
        prec = PRECISIONS.get(prec, prec)
        R, Y = self._check_io(X, Y, prec)
        _lib.check(self._lib.spt_execute_transposed(
            self._h, c_void_p(X.data_ptr()), c_void_p(Y.data_ptr()), c_int64(R), c_int32(prec),
            _stream_ptr(stream)))
        return Y


def execute_batched(plans, Xs, Ys, prec=F64, stream=None):
    """Y_i = X_i A_i^T for every plan (spt_execute_batched: the plans' FFTs and
    products in shared launches, or one persistent launch)."""
    prec = PRECISIONS.get(prec, prec)
    n = len(plans)
    if len(Xs) != n or len(Ys) != n:
        raise ValueError("plans, Xs and Ys must have the same length")
    for p, x, y in zip(plans, Xs, Ys):
        if y is None:
            raise ValueError("execute_batched needs every output tensor")
        p._check_io(x, y, prec)
    hp = (c_void_p * n)(*[p.handle.value for p in plans])
    xs = (c_void_p * n)(*[x.data_ptr() for x in Xs])
    ys = (c_void_p * n)(*[y.data_ptr() for y in Ys])
    rs = (c_int64 * n)(*[x.numel() // p.N for p, x in zip(plans, Xs)])
    lib = _lib.load()
    _lib.check(lib.spt_execute_batched(hp, xs, ys, rs, c_int32(n), c_int32(prec),
                                       _stream_ptr(stream)))
    return Ys


_hooks = None  # the ctypes callbacks of spt_set_allocator, kept alive while set


def set_allocator(alloc=None, free=None):
    """Route the library's device memory through alloc(bytes, stream) -> int
    pointer (0 when out of memory) and free(ptr, stream) (spt_set_allocator);
    with no arguments, back to hipMalloc / hipFree.  Buffers keep the
    allocator that made them, so the hooks stay referenced here for good."""
    global _hooks
    lib = _lib.load()
    if alloc is None and free is None:
        _lib.check(lib.spt_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None))
        return

    def _a(n, stream, ctx):
        try:
            return int(alloc(int(n), int(stream or 0)) or 0)
        except Exception:
            return 0

    def _f(ptr, stream, ctx):
        free(int(ptr), int(stream or 0))

    hooks = (_lib.ALLOC_FN(_a), _lib.FREE_FN(_f))
    _lib.check(lib.spt_set_allocator(hooks[0], hooks[1], None))
    _kept.append(hooks)
    _hooks = hooks


_kept = []


def use_torch_allocator():
    """Let PyTorch's caching allocator own the library's device memory."""
    import torch

    def alloc(n, stream):
        return torch.cuda.caching_allocator_alloc(n, stream=stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)


STAGES = ("fft", "spmm", "spmm_t", "inv_fft", "tail_t", "exec")


def profile_begin():
    """Start timing every stage of every execute with HIP events."""
    _lib.check(_lib.load().spt_profile_begin())


def profile_end():
    """Stop timing; {stage: (total_ms, launches)}."""
    ms = (c_double * len(STAGES))()
    n = (c_int64 * len(STAGES))()
    _lib.check(_lib.load().spt_profile_end(ms, n))
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


def version():
    return _lib.load().spt_version().decode()
