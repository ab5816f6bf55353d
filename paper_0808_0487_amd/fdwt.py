"""Thin ctypes binding of libfdwt (include/fdwt.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch CUDA tensors (ROCm); the HIP stream is
torch's current stream unless one is passed.  Raises RuntimeError when the
library is not built or a call fails -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdwt.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUDGET, EUNSUPPORTED, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
F32, I32, CF32, F64, CF64 = 1, 2, 3, 4, 5
FAMILY = {"product": 1, "exp": 2, "wangfang": 3, "asian": 4}

# Every function the header declares, with (restype, argtypes).
_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double


class KernelC(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("gamma", ctypes.POINTER(ctypes.c_double)), ("s", ctypes.c_int)]


class EffDimC(ctypes.Structure):
    _fields_ = [("var_trc", ctypes.POINTER(ctypes.c_double)), ("var_sup", ctypes.POINTER(ctypes.c_double)),
                ("var_total", ctypes.c_double), ("var_total_h0", ctypes.c_double),
                ("var_qmc", ctypes.c_double), ("d_trc", ctypes.c_int), ("d_sup", ctypes.c_int)]


class KernelFitC(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("q", ctypes.c_double),
                ("cost", ctypes.c_double), ("evaluations", ctypes.c_int)]


class ServerConfigC(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("lanes", ctypes.c_int), ("max_bypass", ctypes.c_int),
                ("effdim_chunk_bytes", ctypes.c_size_t)]


class RequestC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_int), ("m", ctypes.c_int), ("s", ctypes.c_int),
                ("net_key", ctypes.c_uint64), ("C_host", ctypes.c_void_p), ("family", ctypes.c_int),
                ("a_host", ctypes.c_void_p), ("alpha", ctypes.c_double), ("gamma_host", ctypes.c_void_p),
                ("nq", ctypes.c_int64), ("q_host", ctypes.c_void_p)]


class JobInfoC(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("bytes", ctypes.c_size_t), ("spectrum_hit", ctypes.c_int),
                ("packed_hit", ctypes.c_int)]


class ServerCountersC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ["submitted", "completed", "failed", "rejected", "pending",
                                               "in_flight"]] + \
               [(n, ctypes.c_size_t) for n in ["arena_bytes", "arena_used", "arena_peak"]] + \
               [(n, ctypes.c_int64) for n in ["spectrum_hits", "spectrum_misses", "packed_hits", "packed_misses",
                                               "evictions", "nets_built"]]


SIGNATURES = {
    "fdwt_net_generate": (_i, [_i, _i, _i, _vp, ctypes.POINTER(_vp)]),
    "fdwt_net_info": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i64)]),
    "fdwt_net_digits": (_i, [_vp, _vp, _vp]),
    "fdwt_net_points": (_i, [_vp, _vp, _vp]),
    "fdwt_net_free": (None, [_vp]),
    "fdwt_net_drop_spectrum": (_i, [_vp]),
    "fdwt_sample": (_i, [_vp, _i, _vp, _vp, _vp]),
    "fdwt_dwt_forward": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
    "fdwt_dwt_inverse": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
    "fdwt_dwt_inverse_noalloc": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
    "fdwt_dwt_forward_family": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
    "fdwt_query_depth": (_i, [_i]),
    "fdwt_spline_coef": (_i, [_vp, ctypes.POINTER(KernelC), _i, _vp, _vp, _vp]),
    "fdwt_spline_eval": (_i, [_vp, ctypes.POINTER(KernelC), _vp, _i64, _vp, _vp, _vp]),
    "fdwt_walsh_interp": (_i, [_vp, ctypes.POINTER(KernelC), _vp, _vp, _i64, _vp, _vp, _vp]),
    "fdwt_walsh_interp_depth": (_i, [_vp, ctypes.POINTER(KernelC), _vp, _vp, _i64, _vp, _i, _vp, _vp]),
    "fdwt_eff_dim": (_i, [_vp, ctypes.POINTER(KernelC), _i, _vp, ctypes.POINTER(EffDimC), _vp]),
    "fdwt_eff_dim_data": (_i, [_vp, ctypes.POINTER(KernelC), _vp, ctypes.POINTER(EffDimC), _vp]),
    "fdwt_split_cost": (_i, [_vp, _vp, _d, _d, _d, _vp, ctypes.POINTER(_d)]),
    "fdwt_kernel_tune": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(KernelFitC), _vp]),
    "fdwt_batch_create": (_i, [_i, _vp, _i, ctypes.POINTER(_vp)]),
    "fdwt_batch_run": (_i, [_vp, _vp]),
    "fdwt_batch_check": (_i, [_vp, _vp]),
    "fdwt_batch_autotune": (_i, [_vp, _i, _vp]),
    "fdwt_batch_describe": (_i, [_vp, _i, _vp, _vp, _vp, ctypes.POINTER(_i)]),
    "fdwt_batch_free": (None, [_vp]),
    "fdwt_batch_schedule": (_i, [_i, _vp, _i, _vp, _vp, _vp, _vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "fdwt_server_request_bytes": (_i, [ctypes.POINTER(RequestC), ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "fdwt_server_create": (_i, [ctypes.POINTER(ServerConfigC), ctypes.POINTER(_vp)]),
    "fdwt_server_submit": (_i, [_vp, ctypes.POINTER(RequestC), ctypes.POINTER(_i64)]),
    "fdwt_server_wait": (_i, [_vp, _i64, ctypes.POINTER(JobInfoC), _vp, ctypes.POINTER(EffDimC)]),
    "fdwt_server_stats": (_i, [_vp, ctypes.POINTER(ServerCountersC)]),
    "fdwt_server_free": (None, [_vp]),
    "fdwt_timing_enable": (_i, [_i]),
    "fdwt_timing_query": (_i, [_i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]),
    "fdwt_last_error": (ctypes.c_char_p, []),
}

_LIB = None


def lib():
    """Load libfdwt.so (once).  Raises if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfdwt.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class FdwtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fdwt error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != OK:
        raise FdwtError(rc, lib().fdwt_last_error().decode())


_RAW = None  # (current device, raw current stream of a device) readers, set on first use


def _stream(stream):
    """The HIP stream of a call: the given one (a torch stream or a raw
    handle), else torch's current stream on the current device.  The raw
    readers skip building a torch Stream object per call (a few
    microseconds, which a call's first kernel would wait for)."""
    global _RAW
    if stream is None:
        if _RAW is None:
            import torch
            dev = getattr(torch._C, "_cuda_getDevice", None)
            raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
            _RAW = (dev, raw) if dev and raw else (lambda: 0, lambda d: torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(_RAW[1](_RAW[0]()))
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, numel, dtypes, device=None):
    """Validate a tensor before its pointer crosses the ABI: the kernels
    read or write exactly `numel` contiguous elements of one of `dtypes`
    (torch dtype names) through it, on the net's device, so a shorter,
    differently typed, strided or misplaced tensor is refused here with
    ValueError (a host tensor is refused by _ptr, after every tensor of the
    call has passed these checks)."""
    if t is None:
        raise ValueError("%s is required" % name)
    dt = _dtname(t.dtype)
    if dt not in dtypes:
        raise ValueError("%s must be %s, got %s" % (name, " or ".join(dtypes), dt))
    if t.numel() != numel:
        raise ValueError("%s must hold %d elements, got %d" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if device is not None and t.is_cuda and t.device.index != device:
        raise ValueError("%s is on cuda:%s, the net on cuda:%d" % (name, t.device.index, device))
    return t


def _need_params(a, n, name="a"):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError("%s must have %d values, got shape %s" % (name, n, a.shape))
    return a


# Element types of dwt_inverse: (inputs, input -> outputs), for p odd and p = 2.
_INV_TYPES = {True: (("float32", "int32", "float64"),
                     {"float32": ("float32",), "int32": ("int32",), "float64": ("float64",)}),
              False: (("complex64", "complex128"),
                      {"complex64": ("complex64", "float32"), "complex128": ("complex128", "float64")})}

_DT = None  # torch dtype -> (name, ABI element type), built on first use


def _dtypes():
    global _DT
    if _DT is None:
        import torch
        _DT = {torch.float32: ("float32", F32), torch.int32: ("int32", I32), torch.complex64: ("complex64", CF32),
               torch.float64: ("float64", F64), torch.complex128: ("complex128", CF64)}
    return _DT


def _dtname(dt):
    e = _dtypes().get(dt)
    return e[0] if e else str(dt).replace("torch.", "")


def _type_of(t):
    return _dtypes()[t.dtype][1]


class BatchJobC(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("in_dev", ctypes.c_void_p), ("out_dev", ctypes.c_void_p)]


PREC = {"f32": 0, "bf16x2": 1, "f32_generic": 2, "f32_one_launch": 3}


def batch_schedule(ms):
    """Work items of the one-launch batch for jobs of sizes ms, in ticket
    order (fdwt_batch_schedule, host only): arrays job, pass, tile, need and
    the items per ticket."""
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    n, chunk = ctypes.c_int(), ctypes.c_int()
    _check(lib().fdwt_batch_schedule(len(ms), ms.ctypes.data, 0, None, None, None, None, ctypes.byref(n),
                                     ctypes.byref(chunk)))
    out = [np.zeros(max(n.value, 1), dtype=np.int32) for _ in range(4)]
    _check(lib().fdwt_batch_schedule(len(ms), ms.ctypes.data, n.value, *[o.ctypes.data for o in out],
                                     ctypes.byref(n), ctypes.byref(chunk)))
    return tuple(o[:n.value] for o in out) + (chunk.value,)


class Batch:
    """A ragged batch of p = 2 forward transforms (fdwt_batch_*).
    jobs: list of (m, in_tensor, out_tensor); precision 'f32' (grouped static
    passes), 'f32_generic' or 'bf16x2' (persistent launch per pass level) or
    'f32_one_launch' (every pass of every job in one persistent launch)."""

    def __init__(self, jobs, precision="f32"):
        arr = (BatchJobC * len(jobs))()
        for i, (m, x, y) in enumerate(jobs):
            if x.dtype.itemsize != 4 or x.numel() != 2 ** m or y.numel() != 2 ** m:
                raise ValueError("job %d: float tensors of 2^m elements expected" % i)
            arr[i] = BatchJobC(m, _ptr(x).value, _ptr(y).value)
        self._keep = jobs
        h = ctypes.c_void_p()
        _check(lib().fdwt_batch_create(len(jobs), ctypes.cast(arr, ctypes.c_void_p), PREC[precision], ctypes.byref(h)))
        self.h = h

    def run(self, stream=None):
        _check(lib().fdwt_batch_run(self.h, _stream(stream)))

    def check(self, stream=None):
        _check(lib().fdwt_batch_check(self.h, _stream(stream)))

    def autotune(self, reps=5, stream=None):
        _check(lib().fdwt_batch_autotune(self.h, reps, _stream(stream)))

    def describe(self):
        """[(m, emax, jobs)] of the grouped path."""
        n = ctypes.c_int()
        _check(lib().fdwt_batch_describe(self.h, 0, None, None, None, ctypes.byref(n)))
        m, e, j = (np.zeros(max(n.value, 1), dtype=np.int32) for _ in range(3))
        _check(lib().fdwt_batch_describe(self.h, n.value, m.ctypes.data, e.ctypes.data, j.ctypes.data,
                                         ctypes.byref(n)))
        return [(int(m[i]), int(e[i]), int(j[i])) for i in range(n.value)]

    def close(self):
        if self.h:
            lib().fdwt_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Kernel:
    """Weighted Walsh kernel (alpha, gamma_1..gamma_s) of Section 4."""

    def __init__(self, alpha, gamma):
        self.alpha = float(alpha)
        self.gamma = np.ascontiguousarray(gamma, dtype=np.float64)
        self._c = KernelC(self.alpha, self.gamma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          len(self.gamma))

    @property
    def c(self):
        return ctypes.byref(self._c)


class Net:
    """A digital net handle (fdwt_net_generate)."""

    def __init__(self, p, m, s, C):
        C = np.ascontiguousarray(C, dtype=np.uint8)
        if C.shape != (s, m, m):
            raise ValueError("C must have shape (s, m, m)")
        h = ctypes.c_void_p()
        _check(lib().fdwt_net_generate(p, m, s, C.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.h = h
        self.p, self.m, self.s = p, m, s
        self.N = p ** m
        import torch
        self.device = torch.cuda.current_device()

    # Element types of transform coefficients and of each element type's
    # forward output, per p (fdwt_dwt_forward).
    def _coef_dtype(self):
        return "float32" if self.p == 2 else "complex64"

    def _fwd_out_dtype(self, dt):
        if dt == "int32":
            return "int32"
        if dt in ("float64", "complex128"):
            return "float64" if self.p == 2 else "complex128"
        return "float32" if self.p == 2 else "complex64"

    def _queries(self, q):
        """q: uint32 digits [s][nq] (or int32 holding their bit patterns);
        returns nq."""
        if q is None or q.dim() != 2 or q.shape[0] != self.s:
            raise ValueError("queries must have shape (s, nq) = (%d, nq)" % self.s)
        _need(q, "queries", q.numel(), ("int32", "uint32"), self.device)
        return q.shape[1]

    def close(self):
        if self.h:
            lib().fdwt_net_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        p, m, s, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        _check(lib().fdwt_net_info(self.h, ctypes.byref(p), ctypes.byref(m), ctypes.byref(s), ctypes.byref(n)))
        return p.value, m.value, s.value, n.value

    # --------------------------------------------------------------- net
    def digits(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.s, self.N), dtype=torch.int32, device="cuda")
        _need(out, "out", self.s * self.N, ("int32",), self.device)
        _check(lib().fdwt_net_digits(self.h, _ptr(out), _stream(stream)))
        return out

    def points(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.s, self.N), dtype=torch.float32, device="cuda")
        _need(out, "out", self.s * self.N, ("float32",), self.device)
        _check(lib().fdwt_net_points(self.h, _ptr(out), _stream(stream)))
        return out

    def sample(self, family, a, out=None, stream=None):
        import torch
        a = _need_params(a, 5 if family == "asian" else self.s)
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32, device="cuda")
        _need(out, "out", self.N, ("float32",), self.device)
        _check(lib().fdwt_sample(self.h, FAMILY[family], a.ctypes.data_as(ctypes.c_void_p), _ptr(out),
                                 _stream(stream)))
        return out

    def drop_spectrum(self):
        """Release the cached kernel spectrum (fdwt_net_drop_spectrum)."""
        _check(lib().fdwt_net_drop_spectrum(self.h))

    # --------------------------------------------------------- transforms
    def forward(self, x, out=None, stream=None):
        """dwt_forward: float32 -> float32 (p = 2) or complex64 (p odd);
        int32 -> int32 (p = 2, unnormalised, mod 2^32); float64 -> float64
        (p = 2) or complex128 (p odd)."""
        import torch
        if out is None:
            if x.dtype == torch.int32:
                dt = torch.int32
            elif x.dtype in (torch.float64, torch.complex128):
                dt = torch.float64 if self.p == 2 else torch.complex128
            else:
                dt = torch.float32 if self.p == 2 else torch.complex64
            out = torch.empty(self.N, dtype=dt, device=x.device)
        ins = ("float32", "int32", "float64") if self.p == 2 else ("float32", "complex64", "float64", "complex128")
        _need(x, "x", self.N, ins, self.device)
        _need(out, "out", self.N, (self._fwd_out_dtype(_dtname(x.dtype)),), self.device)
        _check(lib().fdwt_dwt_forward(self.h, _type_of(x), _ptr(x), _type_of(out), _ptr(out), _stream(stream)))
        return out

    def forward_family(self, family, a, out=None, stream=None):
        """dwt_forward of f sampled on the device (fdwt_dwt_forward_family)."""
        import torch
        a = _need_params(a, 5 if family == "asian" else self.s)
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32 if self.p == 2 else torch.complex64, device="cuda")
        _need(out, "out", self.N, (self._coef_dtype(),), self.device)
        _check(lib().fdwt_dwt_forward_family(self.h, FAMILY[family], a.ctypes.data_as(ctypes.c_void_p),
                                             _type_of(out), _ptr(out), _stream(stream)))
        return out

    def inverse(self, x, out=None, real=False, stream=None):
        """dwt_inverse (no normalisation); real=True returns the real part
        (p odd)."""
        import torch
        if out is None:
            dt = x.dtype
            if real and x.dtype == torch.complex64:
                dt = torch.float32
            elif real and x.dtype == torch.complex128:
                dt = torch.float64
            out = torch.empty(self.N, dtype=dt, device=x.device)
        ins, outs = _INV_TYPES[self.p == 2]
        _need(x, "x", self.N, ins, self.device)
        _need(out, "out", self.N, outs[_dtname(x.dtype)], self.device)
        _check(lib().fdwt_dwt_inverse(self.h, _type_of(x), _ptr(x), _type_of(out), _ptr(out), _stream(stream)))
        return out

    # ------------------------------------------------------------ spline
    def spline_coef(self, kern, ft, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32, device=ft.device)
        _need(ft, "ft", self.N, (self._coef_dtype(),), self.device)
        _need(out, "out", self.N, ("float32",), self.device)
        _check(lib().fdwt_spline_coef(self.h, kern.c, _type_of(ft), _ptr(ft), _ptr(out), _stream(stream)))
        return out

    def spline_eval(self, kern, c, q, out=None, stream=None):
        import torch
        nq = self._queries(q)
        if out is None:
            out = torch.empty(nq, dtype=torch.float32, device=c.device)
        _need(c, "c", self.N, ("float32",), self.device)
        _need(out, "out", nq, ("float32",), self.device)
        _check(lib().fdwt_spline_eval(self.h, kern.c, _ptr(c), nq, _ptr(q), _ptr(out), _stream(stream)))
        return out

    def walsh_interp(self, kern, f, q=None, c_out=None, sf_out=None, stream=None, q_depth=None):
        """Spline coefficients of f and Sf at the queries q (uint32/int32
        [s][nq] digit integers of q_depth digits; None: the full depth D)."""
        import torch
        if c_out is None:
            c_out = torch.empty(self.N, dtype=torch.float32, device=f.device)
        nq = 0 if q is None else self._queries(q)
        if nq and sf_out is None:
            sf_out = torch.empty(nq, dtype=torch.float32, device=f.device)
        _need(f, "f", self.N, ("float32",), self.device)
        _need(c_out, "c_out", self.N, ("float32",), self.device)
        if nq:
            _need(sf_out, "sf_out", nq, ("float32",), self.device)
        if q_depth is None:
            _check(lib().fdwt_walsh_interp(self.h, kern.c, _ptr(f), _ptr(c_out), nq, _ptr(q) if nq else None,
                                           _ptr(sf_out) if nq else None, _stream(stream)))
        else:
            _check(lib().fdwt_walsh_interp_depth(self.h, kern.c, _ptr(f), _ptr(c_out), nq,
                                                 _ptr(q) if nq else None, int(q_depth),
                                                 _ptr(sf_out) if nq else None, _stream(stream)))
        return c_out, sf_out

    # ------------------------------------------ kernel-parameter selection
    def split_cost(self, f2, alpha, beta, q, want_sf=False):
        """Section 5.1 cost (and Sf at the second half) for a p = 2 net of
        2N points; f2 float32 [2N] on the device."""
        import torch
        _need(f2, "f2", self.N, ("float32",), self.device)
        sf = torch.empty(self.N // 2, dtype=torch.float32, device=f2.device) if want_sf else None
        c = ctypes.c_double()
        _check(lib().fdwt_split_cost(self.h, _ptr(f2), alpha, beta, q, _ptr(sf) if want_sf else None,
                                     ctypes.byref(c), _stream(None)))
        return (c.value, sf) if want_sf else c.value

    def kernel_tune(self, f2, start=(2.0, 1.0, -2.0), max_evals=200):
        _need(f2, "f2", self.N, ("float32",), self.device)
        st = _need_params(start, 3, "start")
        out = KernelFitC()
        _check(lib().fdwt_kernel_tune(self.h, _ptr(f2), st.ctypes.data, max_evals, ctypes.byref(out), _stream(None)))
        return {"alpha": out.alpha, "beta": out.beta, "q": out.q, "cost": out.cost, "evaluations": out.evaluations}

    def eff_dim(self, kern, ft, stream=None):
        """Effective dimension from the forward transform ft of the data."""
        _need(ft, "ft", self.N, (self._coef_dtype(),), self.device)
        trc = np.zeros(self.s + 1)
        sup = np.zeros(self.s + 1)
        out = EffDimC(trc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      sup.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0, 0)
        _check(lib().fdwt_eff_dim(self.h, kern.c, _type_of(ft), _ptr(ft), ctypes.byref(out), _stream(stream)))
        return self._effdim_dict(trc, sup, out)

    def eff_dim_data(self, kern, f, stream=None):
        """Effective dimension from the data f (float32 [N]) (fdwt_eff_dim_data)."""
        _need(f, "f", self.N, ("float32",), self.device)
        trc = np.zeros(self.s + 1)
        sup = np.zeros(self.s + 1)
        out = EffDimC(trc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      sup.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0, 0)
        _check(lib().fdwt_eff_dim_data(self.h, kern.c, _ptr(f), ctypes.byref(out), _stream(stream)))
        return self._effdim_dict(trc, sup, out)

    @staticmethod
    def _effdim_dict(trc, sup, out):
        return {"var_trc": trc, "var_sup": sup, "var_total": out.var_total, "var_total_h0": out.var_total_h0,
                "var_qmc": out.var_qmc, "d_trc": out.d_trc, "d_sup": out.d_sup}


JOB = {"interp": 1, "eff_dim": 2}


class Request:
    """One serving request (fdwt_request): kind 'interp' or 'eff_dim', the
    net (p, m, s, C, net_key), the test-function family and its parameters a,
    the kernel (alpha, gamma) and, for 'interp', queries uint32 [s][nq]."""

    def __init__(self, kind, p, m, s, C, net_key, family, a, alpha, gamma, queries=None):
        self.kind, self.p, self.m, self.s = kind, p, m, s
        self.C = np.ascontiguousarray(C, dtype=np.uint8)
        self.a = np.ascontiguousarray(a, dtype=np.float64)
        self.gamma = np.ascontiguousarray(gamma, dtype=np.float64)
        self.q = None if queries is None else np.ascontiguousarray(queries, dtype=np.uint32)
        self.net_key, self.family, self.alpha = int(net_key), family, float(alpha)
        na = 5 if family == "asian" else s
        if self.C.shape != (s, m, m) or self.a.shape != (na,) or self.gamma.shape != (s,):
            raise ValueError("C (s, m, m), a (s,) or (5,) for 'asian', and gamma (s,) expected")
        if kind == "interp" and (self.q is None or self.q.ndim != 2 or self.q.shape[0] != s):
            raise ValueError("interp requests need queries of shape (s, nq)")

    @property
    def nq(self):
        return 0 if self.q is None else self.q.shape[1]

    def c(self):
        return RequestC(JOB[self.kind], self.p, self.m, self.s, self.net_key, self.C.ctypes.data,
                        FAMILY[self.family], self.a.ctypes.data, self.alpha, self.gamma.ctypes.data,
                        self.nq, None if self.q is None else self.q.ctypes.data)


def request_bytes(req, effdim_chunk_bytes=0):
    """(job_bytes, cache_bytes) of a request (host-only)."""
    jb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    rc = req.c()
    _check(lib().fdwt_server_request_bytes(ctypes.byref(rc), effdim_chunk_bytes, ctypes.byref(jb), ctypes.byref(cb)))
    return jb.value, cb.value


class Server:
    """The serving loop (fdwt_server_*): submit() returns a job id at once;
    wait(id) blocks and returns (info dict, result) with result = Sf at the
    queries (float32 numpy array) or the eff_dim dict."""

    def __init__(self, hbm_budget, lanes=8, max_bypass=8, effdim_chunk_bytes=0):
        cfg = ServerConfigC(int(hbm_budget), lanes, max_bypass, int(effdim_chunk_bytes))
        h = ctypes.c_void_p()
        _check(lib().fdwt_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._reqs = {}

    def submit(self, req):
        jid = ctypes.c_int64()
        rc = req.c()
        _check(lib().fdwt_server_submit(self.h, ctypes.byref(rc), ctypes.byref(jid)))
        self._reqs[jid.value] = (req.kind, req.s, req.nq)
        return jid.value

    def wait(self, jid):
        kind, s, nq = self._reqs.pop(jid)
        info = JobInfoC()
        if kind == "interp":
            sf = np.empty(nq, dtype=np.float32)
            rc = lib().fdwt_server_wait(self.h, jid, ctypes.byref(info), sf.ctypes.data, None)
            res = sf
        else:
            trc, sup = np.zeros(s + 1), np.zeros(s + 1)
            out = EffDimC(trc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          sup.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0, 0.0, 0.0, 0, 0)
            rc = lib().fdwt_server_wait(self.h, jid, ctypes.byref(info), None, ctypes.byref(out))
            res = {"var_trc": trc, "var_sup": sup, "var_total": out.var_total, "var_total_h0": out.var_total_h0,
                   "var_qmc": out.var_qmc, "d_trc": out.d_trc, "d_sup": out.d_sup}
        _check(rc)
        return ({"t_submit": info.t_submit, "t_admit": info.t_admit, "t_done": info.t_done, "bytes": info.bytes,
                 "spectrum_hit": bool(info.spectrum_hit), "packed_hit": bool(info.packed_hit)}, res)

    def stats(self):
        c = ServerCountersC()
        _check(lib().fdwt_server_stats(self.h, ctypes.byref(c)))
        return {n: getattr(c, n) for n, _ in ServerCountersC._fields_}

    def close(self):
        if self.h:
            lib().fdwt_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_depth(p):
    return lib().fdwt_query_depth(p)


TC = {"pass_f32": 0, "pass_cf32": 1, "pass_f64": 2, "sample": 3, "kcols": 4, "eval": 5, "batch": 6}


def timing_enable(on=True):
    _check(lib().fdwt_timing_enable(1 if on else 0))


def timing_query(cls):
    """(total_ms, launches, work) of a kernel class since timing was enabled."""
    ms, n, w = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().fdwt_timing_query(TC[cls] if isinstance(cls, str) else cls, ctypes.byref(ms), ctypes.byref(n),
                                   ctypes.byref(w)))
    return ms.value, n.value, w.value
