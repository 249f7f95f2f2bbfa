"""ctypes binding of include/nnfft.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device arrays
are torch tensors on the GPU (their data_ptr() is passed); the stream is the
current torch stream unless one is given.  All compute happens in the HIP
library; nothing here falls back to another implementation: if the library
is missing the import-time loader raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnfft.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADERS = [os.path.join(INCLUDE, "nnfft.h"), os.path.join(INCLUDE, "nnfft_serve.h")]

NNFFT_OK = 0
NNFFT_ERR_ARG = 1
NNFFT_ERR_DOMAIN = 2
NNFFT_ERR_NOMEM = 3
NNFFT_ERR_DEVICE = 4
NNFFT_ERR_UNSUPPORTED = 5
NNFFT_ERR_BUSY = 6
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_DOMAIN", 3: "ERR_NOMEM", 4: "ERR_DEVICE",
                5: "ERR_UNSUPPORTED", 6: "ERR_BUSY"}

NNFFT_FP64_PLAIN = 0
NNFFT_FP32_COMP = 1
SINC_QUAD_GAUSS_LEGENDRE = 0
SINC_QUAD_CLENSHAW_CURTIS = 1
NNFFT_WINDOW_SINH, NNFFT_WINDOW_BSPLINE, NNFFT_WINDOW_ALGEBRAIC, NNFFT_WINDOW_KAISER_BESSEL = 0, 1, 2, 3


class NnfftInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("N_star", ctypes.c_int64), ("N1", ctypes.c_int64),
        ("G1", ctypes.c_int64), ("N2", ctypes.c_int64),
        ("M1", ctypes.c_int64), ("M2", ctypes.c_int64),
        ("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("sigma1", ctypes.c_double), ("sigma2", ctypes.c_double),
        ("sigma1_eff", ctypes.c_double), ("sigma2_eff", ctypes.c_double),
        ("a", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
        ("bound_thm41", ctypes.c_double), ("thm41_applies", ctypes.c_int32),
        ("window_degree", ctypes.c_int32), ("window_fit_err", ctypes.c_double),
        ("corr_degree", ctypes.c_int32), ("corr_fit_err", ctypes.c_double),
        ("device_bytes", ctypes.c_int64), ("block_points", ctypes.c_int64),
        ("items_points", ctypes.c_int32), ("spread_workgroups", ctypes.c_int32),
        ("interp_workgroups", ctypes.c_int32), ("fft_n1", ctypes.c_int32),
        ("fft_n2", ctypes.c_int32), ("window", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class NnfftTuning(ctypes.Structure):
    _fields_ = [("items_points", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("block_points", ctypes.c_int64), ("exec_ms", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("tuned", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


NNFFT_REQ_NNFFT = 0
NNFFT_REQ_SINC = 1


class NnfftRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("N", ctypes.c_int64),
                ("M1", ctypes.c_int64), ("M2", ctypes.c_int64),
                ("sigma1", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("quad", ctypes.c_int32),
                ("window", ctypes.c_int32), ("n_quad", ctypes.c_int64),
                ("v", ctypes.c_void_p), ("x", ctypes.c_void_p), ("f", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("plan_key", ctypes.c_uint64)]


class NnfftResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("group_size", ctypes.c_int32),
                ("footprint_bytes", ctypes.c_int64), ("plan_reused", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("submit_ms", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("admit_ms", ctypes.c_double),
                ("launch_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("message", ctypes.c_char * 160)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        d["message"] = self.message.decode(errors="replace")
        return d


class NnfftServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("planner_threads", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class NnfftServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "groups", "admission_waits",
                                             "evictions", "arena_bytes", "arena_in_use", "arena_peak",
                                             "resident_plans")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class NnfftKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("stage", ctypes.c_int), ("avg_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class NnfftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Loads libnnfft.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                          f"python paper_2107_02671_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.nnfft_derive_params.argtypes = [i64, dbl, dbl, ci, ci, ctypes.POINTER(NnfftInfo)]
    L.nnfft_plan.argtypes = [ctypes.POINTER(vp), i64, i64, i64, dbl, dbl, ci, ci, ci, vp, vp, vp]
    L.nnfft_plan_window.argtypes = [ctypes.POINTER(vp), i64, i64, i64, dbl, dbl, ci, ci, ci, ci, vp, vp, vp]
    L.nnfft_exec.argtypes = [vp, vp, vp, vp]
    L.nnfft_exec_noalloc.argtypes = [vp, vp, vp, vp]
    L.nfft_plan.argtypes = [ctypes.POINTER(vp), i64, i64, dbl, ci, ci, vp, vp]
    L.nfft_exec.argtypes = [vp, vp, vp, vp]
    L.nfft_adjoint.argtypes = [vp, vp, vp, vp]
    L.nfft_destroy.argtypes = [vp]
    L.nfft_plan_dry_run.argtypes = [i64, i64, dbl, ci, ci, ctypes.POINTER(dbl), ctypes.POINTER(NnfftInfo)]
    L.nnfft_plan_dry_run.argtypes = [i64, i64, i64, dbl, dbl, ci, ci, ci, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(NnfftInfo)]
    L.nnfft_plan_window_dry_run.argtypes = [i64, i64, i64, dbl, dbl, ci, ci, ci, ci, ctypes.POINTER(dbl),
                                            ctypes.POINTER(dbl), ctypes.POINTER(NnfftInfo)]
    L.nnfft_exec_batch.argtypes = [ci, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.nnfft_plan_digest.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.nnfft_plan_window_dry_run_digest.argtypes = [i64, i64, i64, dbl, dbl, ci, ci, ci, ci, ctypes.POINTER(dbl),
                                                   ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_uint64)]
    L.nnfft_info.argtypes = [vp, ctypes.POINTER(NnfftInfo)]
    L.nnfft_destroy.argtypes = [vp]
    L.sinc_plan.argtypes = [ctypes.POINTER(vp), i64, i64, i64, ci, i64, dbl, dbl, ci, ci, ci, vp, vp, vp]
    L.sinc_exec.argtypes = [vp, vp, vp, vp]
    L.sinc_info.argtypes = [vp, ci, ctypes.POINTER(NnfftInfo)]
    L.sinc_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                             ctypes.POINTER(ci)]
    L.sinc_destroy.argtypes = [vp]
    L.sinc_middle.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.sinc_middle_dry_run.argtypes = [i64, ci, i64, dbl, dbl, ci, ci, ci, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int32), i64, ctypes.POINTER(i64), ctypes.POINTER(ci)]
    dptr = ctypes.POINTER(ctypes.c_double)
    L.nnfft_quadrature.argtypes = [ci, i64, dptr, dptr]
    L.nnfft_profile_start.argtypes = [vp, ci]
    L.nnfft_profile_stop.argtypes = [vp, dptr, ctypes.POINTER(ci)]
    L.nnfft_profile_kernels.argtypes = [vp, ctypes.POINTER(NnfftKernelTime), ci, ctypes.POINTER(ci), dptr, ci,
                                        ctypes.POINTER(ci)]
    tp = ctypes.POINTER(NnfftTuning)
    L.nnfft_autotune.argtypes = [i64, i64, ci, ci, ci, vp, tp]
    L.nnfft_set_tuning.argtypes = [ci, i64, tp]
    L.nnfft_get_tuning.argtypes = [ci, i64, tp]
    L.nnfft_clear_tuning.argtypes = []
    u64 = ctypes.c_uint64
    L.nnfft_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(NnfftServerConfig)]
    L.nnfft_server_submit.argtypes = [vp, ctypes.POINTER(NnfftRequest), ctypes.POINTER(u64)]
    L.nnfft_server_wait.argtypes = [vp, u64, ctypes.POINTER(NnfftResult)]
    L.nnfft_server_poll.argtypes = [vp, u64, ctypes.POINTER(NnfftResult)]
    L.nnfft_server_stats.argtypes = [vp, ctypes.POINTER(NnfftServerStats)]
    L.nnfft_server_evict.argtypes = [vp, u64]
    L.nnfft_server_destroy.argtypes = [vp]
    L.nnfft_last_error.restype = ctypes.c_char_p
    L.nnfft_version.restype = ctypes.c_char_p
    for name in ["nfft_plan", "nfft_exec", "nfft_adjoint", "nfft_destroy", "nfft_plan_dry_run",
                 "nnfft_plan_dry_run", "nnfft_plan_window", "nnfft_plan_digest", "nnfft_plan_window_dry_run_digest", "nnfft_plan_window_dry_run", "nnfft_profile_start", "nnfft_profile_stop", "nnfft_profile_kernels", "nnfft_quadrature", "nnfft_derive_params",
                 "nnfft_plan", "nnfft_exec", "nnfft_exec_noalloc", "nnfft_exec_batch", "nnfft_info", "nnfft_destroy", "sinc_plan",
                 "sinc_exec", "sinc_info", "sinc_sizes", "sinc_destroy", "sinc_middle", "sinc_middle_dry_run", "nnfft_autotune", "nnfft_set_tuning",
                 "nnfft_get_tuning", "nnfft_clear_tuning", "nnfft_server_create", "nnfft_server_submit",
                 "nnfft_server_wait", "nnfft_server_poll", "nnfft_server_stats", "nnfft_server_evict",
                 "nnfft_server_destroy"]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/*.h."""
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(nnfft_\w+|nfft_\w+|sinc_\w+)\s*\(", src))
    return sorted(names)


def _check(status):
    if status != NNFFT_OK:
        raise NnfftError(status, nnfft_last_error())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def nnfft_last_error() -> str:
    return lib().nnfft_last_error().decode()


def nnfft_version() -> str:
    return lib().nnfft_version().decode()


def nnfft_derive_params(N, sigma1, sigma2, m1, m2) -> dict:
    info = NnfftInfo()
    _check(lib().nnfft_derive_params(int(N), float(sigma1), float(sigma2), int(m1), int(m2),
                                     ctypes.byref(info)))
    return info.as_dict()


def nnfft_quadrature(quad, n_quad):
    """Host-side quadrature rule of sinc_plan: (z, w) numpy arrays."""
    import numpy as np
    n = int(n_quad) + (1 if quad == SINC_QUAD_CLENSHAW_CURTIS else 0)
    z = np.zeros(n)
    w = np.zeros(n)
    dptr = ctypes.POINTER(ctypes.c_double)
    _check(lib().nnfft_quadrature(int(quad), int(n_quad), z.ctypes.data_as(dptr), w.ctypes.data_as(dptr)))
    return z, w


def _require(t, dtype, n, name):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of {n} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def nnfft_plan(N, v, x, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP32_COMP, stream=None,
               window=None):
    """v, x: float64 CUDA tensors.  Returns an opaque plan handle (c_void_p).
    window: None (nnfft_plan, sinh windows) or an NNFFT_WINDOW_* family
    (nnfft_plan_window)."""
    import torch
    _require(v, torch.float64, v.numel(), "v")
    _require(x, torch.float64, x.numel(), "x")
    h = ctypes.c_void_p()
    if window is None:
        _check(lib().nnfft_plan(ctypes.byref(h), int(N), v.numel(), x.numel(), float(sigma1), float(sigma2),
                                int(m1), int(m2), int(prec), _ptr(v), _ptr(x), _stream(stream)))
    else:
        _check(lib().nnfft_plan_window(ctypes.byref(h), int(N), v.numel(), x.numel(), float(sigma1),
                                       float(sigma2), int(m1), int(m2), int(prec), int(window), _ptr(v), _ptr(x),
                                       _stream(stream)))
    return h


def nnfft_plan_dry_run(N, v, x, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP32_COMP, window=None) -> dict:
    """Host-only plan construction and layout check on numpy float64 node arrays."""
    import numpy as np
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    info = NnfftInfo()
    dptr = ctypes.POINTER(ctypes.c_double)
    if window is None:
        _check(lib().nnfft_plan_dry_run(int(N), v.size, x.size, float(sigma1), float(sigma2), int(m1), int(m2),
                                        int(prec), v.ctypes.data_as(dptr), x.ctypes.data_as(dptr),
                                        ctypes.byref(info)))
    else:
        _check(lib().nnfft_plan_window_dry_run(int(N), v.size, x.size, float(sigma1), float(sigma2), int(m1),
                                               int(m2), int(prec), int(window), v.ctypes.data_as(dptr),
                                               x.ctypes.data_as(dptr), ctypes.byref(info)))
    return info.as_dict()


def nnfft_plan_digest(plan) -> int:
    """64-bit digest of a plan's layout image on the device."""
    d = ctypes.c_uint64()
    _check(lib().nnfft_plan_digest(plan, ctypes.byref(d)))
    return d.value


def nnfft_plan_dry_run_digest(N, v, x, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP32_COMP,
                              window=NNFFT_WINDOW_SINH) -> int:
    """Digest of the layout the dry run builds on the host from host nodes."""
    import numpy as np
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    dptr = ctypes.POINTER(ctypes.c_double)
    d = ctypes.c_uint64()
    _check(lib().nnfft_plan_window_dry_run_digest(int(N), v.size, x.size, float(sigma1), float(sigma2), int(m1),
                                                  int(m2), int(prec), int(window), v.ctypes.data_as(dptr),
                                                  x.ctypes.data_as(dptr), ctypes.byref(d)))
    return d.value


def nfft_plan(N, x, sigma=2.0, m=6, prec=NNFFT_FP32_COMP, stream=None):
    """NFFT plan for the nodes x (float64 CUDA tensor) and frequencies k in I_N."""
    import torch
    _require(x, torch.float64, x.numel(), "x")
    h = ctypes.c_void_p()
    _check(lib().nfft_plan(ctypes.byref(h), int(N), x.numel(), float(sigma), int(m), int(prec), _ptr(x),
                           _stream(stream)))
    return h


def nfft_exec(plan, f, y, stream=None):
    """y_j = sum_{k in I_N} f_k exp(-2 pi i k x_j)."""
    info = nnfft_info(plan)
    dt = _cdtype(info["precision"])
    _require(f, dt, info["N"], "f")
    _require(y, dt, info["M2"], "y")
    _check(lib().nfft_exec(plan, _ptr(f), _ptr(y), _stream(stream)))


def nfft_adjoint(plan, y, h, stream=None):
    """h_k = sum_j y_j exp(+2 pi i k x_j), k in I_N."""
    info = nnfft_info(plan)
    dt = _cdtype(info["precision"])
    _require(y, dt, info["M2"], "y")
    _require(h, dt, info["N"], "h")
    _check(lib().nfft_adjoint(plan, _ptr(y), _ptr(h), _stream(stream)))


def nfft_destroy(plan):
    _check(lib().nfft_destroy(plan))


def nfft_plan_dry_run(N, x, sigma=2.0, m=6, prec=NNFFT_FP32_COMP) -> dict:
    """Host-only NFFT plan construction and layout check on numpy float64 nodes."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float64)
    info = NnfftInfo()
    dptr = ctypes.POINTER(ctypes.c_double)
    _check(lib().nfft_plan_dry_run(int(N), x.size, float(sigma), int(m), int(prec), x.ctypes.data_as(dptr),
                                   ctypes.byref(info)))
    return info.as_dict()


class NfftPlan:
    """Owning wrapper: NfftPlan(N, x, ...); forward(f) -> y; adjoint(y) -> h."""

    def __init__(self, N, x, sigma=2.0, m=6, prec=NNFFT_FP32_COMP, stream=None):
        self.handle = nfft_plan(N, x, sigma, m, prec, stream)
        self.info = nnfft_info(self.handle)

    def forward(self, f, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.info["M2"], dtype=_cdtype(self.info["precision"]), device=f.device)
        nfft_exec(self.handle, f, y, stream)
        return y

    def adjoint(self, y, h=None, stream=None):
        import torch
        if h is None:
            h = torch.empty(self.info["N"], dtype=_cdtype(self.info["precision"]), device=y.device)
        nfft_adjoint(self.handle, y, h, stream)
        return h

    def close(self):
        if getattr(self, "handle", None) is not None:
            nfft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def nnfft_info(plan) -> dict:
    info = NnfftInfo()
    _check(lib().nnfft_info(plan, ctypes.byref(info)))
    return info.as_dict()


def _cdtype(prec):
    import torch
    return torch.complex64 if prec == NNFFT_FP32_COMP else torch.complex128


def nnfft_exec(plan, f, y, stream=None):
    info = nnfft_info(plan)
    dt = _cdtype(info["precision"])
    _require(f, dt, info["M1"], "f")
    _require(y, dt, info["M2"], "y")
    _check(lib().nnfft_exec(plan, _ptr(f), _ptr(y), _stream(stream)))


def nnfft_exec_noalloc(plan, f, y, stream=None):
    """nnfft_exec with the working memory in the library's static device array."""
    info = nnfft_info(plan)
    dt = _cdtype(info["precision"])
    _require(f, dt, info["M1"], "f")
    _require(y, dt, info["M2"], "y")
    _check(lib().nnfft_exec_noalloc(plan, _ptr(f), _ptr(y), _stream(stream)))


def nnfft_exec_batch(plans, fs, ys, stream=None):
    n = len(plans)
    for p, f, y in zip(plans, fs, ys):
        info = nnfft_info(p)
        dt = _cdtype(info["precision"])
        _require(f, dt, info["M1"], "f")
        _require(y, dt, info["M2"], "y")
    P = (ctypes.c_void_p * n)(*[p.value for p in plans])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    Y = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    _check(lib().nnfft_exec_batch(n, P, F, Y, _stream(stream)))


def nnfft_profile_start(plan, max_execs):
    _check(lib().nnfft_profile_start(plan, int(max_execs)))


def nnfft_profile_stop(plan):
    """Average stage durations (ms) over the profiled execs: (spread, fft, interp), count."""
    ms = (ctypes.c_double * 3)()
    n = ctypes.c_int()
    _check(lib().nnfft_profile_stop(plan, ms, ctypes.byref(n)))
    return (ms[0], ms[1], ms[2]), n.value


def nnfft_profile_kernels(plan, max_execs):
    """Kernel times of the profiled execs: ([{name, stage, avg_ms, min_ms, max_ms}] in launch
    order, [span of each exec in ms])."""
    K = (NnfftKernelTime * 8)()
    E = (ctypes.c_double * max(1, int(max_execs)))()
    nk, ne = ctypes.c_int(), ctypes.c_int()
    _check(lib().nnfft_profile_kernels(plan, K, 8, ctypes.byref(nk), E, int(max_execs), ctypes.byref(ne)))
    kern = [{"name": K[i].name.decode(), "stage": K[i].stage, "avg_ms": K[i].avg_ms, "min_ms": K[i].min_ms,
             "max_ms": K[i].max_ms} for i in range(nk.value)]
    return kern, [E[i] for i in range(min(ne.value, int(max_execs)))]


def nnfft_destroy(plan):
    _check(lib().nnfft_destroy(plan))


def sinc_plan(N, a, b, n_quad, quad=SINC_QUAD_GAUSS_LEGENDRE, sigma1=2.0, sigma2=2.0, m1=6, m2=6,
              prec=NNFFT_FP32_COMP, stream=None):
    import torch
    _require(a, torch.float64, a.numel(), "a")
    _require(b, torch.float64, b.numel(), "b")
    h = ctypes.c_void_p()
    _check(lib().sinc_plan(ctypes.byref(h), int(N), a.numel(), b.numel(), int(quad), int(n_quad),
                           float(sigma1), float(sigma2), int(m1), int(m2), int(prec), _ptr(a), _ptr(b),
                           _stream(stream)))
    return h


def sinc_info(plan, which=0) -> dict:
    info = NnfftInfo()
    _check(lib().sinc_info(plan, int(which), ctypes.byref(info)))
    return info.as_dict()


def sinc_sizes(plan) -> dict:
    """{"L1", "L2", "n_nodes", "nfft_steps"} (nfft_steps bit 0: step 1, bit 1: step 3)."""
    L1, L2, nn, steps = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
    _check(lib().sinc_sizes(plan, ctypes.byref(L1), ctypes.byref(L2), ctypes.byref(nn), ctypes.byref(steps)))
    return {"L1": L1.value, "L2": L2.value, "n_nodes": nn.value, "nfft_steps": steps.value}


def sinc_exec(plan, c, h, stream=None):
    sz = sinc_sizes(plan)
    dt = _cdtype(sinc_info(plan, 0)["precision"])
    _require(c, dt, sz["L1"], "c")
    _require(h, dt, sz["L2"], "h")
    _check(lib().sinc_exec(plan, _ptr(c), _ptr(h), _stream(stream)))


def sinc_destroy(plan):
    _check(lib().sinc_destroy(plan))


def sinc_middle_dry_run(N, quad, n_quad, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP64_PLAIN):
    """Host-only middle operator of a sinc plan: (K [Wb, G1], lo [G1]) numpy arrays."""
    import numpy as np
    G1, Wb = ctypes.c_int64(), ctypes.c_int()
    _check(lib().sinc_middle_dry_run(int(N), int(quad), int(n_quad), float(sigma1), float(sigma2), int(m1), int(m2),
                                     int(prec), None, None, 0, ctypes.byref(G1), ctypes.byref(Wb)))
    K = np.zeros((Wb.value, G1.value))
    lo = np.zeros(G1.value, dtype=np.int32)
    _check(lib().sinc_middle_dry_run(int(N), int(quad), int(n_quad), float(sigma1), float(sigma2), int(m1), int(m2),
                                     int(prec), K.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), K.size,
                                     ctypes.byref(G1), ctypes.byref(Wb)))
    return K, lo


def sinc_middle(plan, on=-1) -> dict:
    """on = 1 / 0: sinc_exec runs the middle operator / the two-kernel form;
    other values leave it.  Returns {"built", "active"}."""
    built, active = ctypes.c_int(), ctypes.c_int()
    _check(lib().sinc_middle(plan, int(on), ctypes.byref(built), ctypes.byref(active)))
    return {"built": built.value, "active": active.value}


class Plan:
    """Owning wrapper: Plan(N, v, x, ...) ; plan(f) -> y ; closed on exit/GC."""

    def __init__(self, N, v, x, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP32_COMP, stream=None,
                 window=None):
        self.handle = nnfft_plan(N, v, x, sigma1, sigma2, m1, m2, prec, stream, window)
        self.info = nnfft_info(self.handle)

    def __call__(self, f, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.info["M2"], dtype=_cdtype(self.info["precision"]), device=f.device)
        nnfft_exec(self.handle, f, y, stream)
        return y

    def close(self):
        if getattr(self, "handle", None) is not None:
            nnfft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class SincPlan:
    def __init__(self, N, a, b, n_quad, quad=SINC_QUAD_GAUSS_LEGENDRE, sigma1=2.0, sigma2=2.0, m1=6,
                 m2=6, prec=NNFFT_FP32_COMP, stream=None):
        self.handle = sinc_plan(N, a, b, n_quad, quad, sigma1, sigma2, m1, m2, prec, stream)
        self.info = [sinc_info(self.handle, 0), sinc_info(self.handle, 1)]
        self.sizes = sinc_sizes(self.handle)

    def __call__(self, c, h=None, stream=None):
        import torch
        if h is None:
            h = torch.empty(self.sizes["L2"], dtype=_cdtype(self.info[0]["precision"]), device=c.device)
        sinc_exec(self.handle, c, h, stream)
        return h

    def close(self):
        if getattr(self, "handle", None) is not None:
            sinc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# layout tuning
# ---------------------------------------------------------------------------
def nnfft_autotune(N, M, m, prec, reps=10, stream=None) -> dict:
    t = NnfftTuning()
    _check(lib().nnfft_autotune(int(N), int(M), int(m), int(prec), int(reps), _stream(stream), ctypes.byref(t)))
    return t.as_dict()


def nnfft_set_tuning(prec, M, items_points, block_points):
    t = NnfftTuning(int(items_points), 0, int(block_points), 0.0, 0, 0)
    _check(lib().nnfft_set_tuning(int(prec), int(M), ctypes.byref(t)))


def nnfft_get_tuning(prec, M) -> dict:
    t = NnfftTuning()
    _check(lib().nnfft_get_tuning(int(prec), int(M), ctypes.byref(t)))
    return t.as_dict()


def nnfft_clear_tuning():
    _check(lib().nnfft_clear_tuning())


# ---------------------------------------------------------------------------
# serving (include/nnfft_serve.h)
# ---------------------------------------------------------------------------
def nnfft_server_create(hbm_budget_bytes=0, planner_threads=0, streams=0, max_batch=0):
    cfg = NnfftServerConfig(int(hbm_budget_bytes), int(planner_threads), int(streams), int(max_batch), 0)
    h = ctypes.c_void_p()
    _check(lib().nnfft_server_create(ctypes.byref(h), ctypes.byref(cfg)))
    return h


def nnfft_server_submit(server, N, v, x, f, y, sigma1=2.0, sigma2=2.0, m1=6, m2=6, prec=NNFFT_FP32_COMP,
                        kind=NNFFT_REQ_NNFFT, quad=SINC_QUAD_GAUSS_LEGENDRE, n_quad=0, plan_key=0,
                        window=0) -> int:
    """v, x: float64 CUDA tensors; f, y: complex CUDA tensors of the plan's
    precision.  The tensors must stay alive until the result is taken."""
    import torch
    _require(v, torch.float64, v.numel(), "v")
    _require(x, torch.float64, x.numel(), "x")
    dt = _cdtype(prec)
    _require(f, dt, v.numel(), "f")
    _require(y, dt, x.numel(), "y")
    r = NnfftRequest(int(kind), int(prec), int(N), v.numel(), x.numel(), float(sigma1), float(sigma2),
                     int(m1), int(m2), int(quad), int(window), int(n_quad), v.data_ptr(), x.data_ptr(), f.data_ptr(),
                     y.data_ptr(), int(plan_key))
    t = ctypes.c_uint64()
    _check(lib().nnfft_server_submit(server, ctypes.byref(r), ctypes.byref(t)))
    return t.value


def nnfft_server_wait(server, ticket) -> dict:
    r = NnfftResult()
    _check(lib().nnfft_server_wait(server, ctypes.c_uint64(ticket), ctypes.byref(r)))
    return r.as_dict()


def nnfft_server_poll(server, ticket):
    """The result dict if finished, else None."""
    r = NnfftResult()
    st = lib().nnfft_server_poll(server, ctypes.c_uint64(ticket), ctypes.byref(r))
    if st == NNFFT_ERR_BUSY:
        return None
    _check(st)
    return r.as_dict()


def nnfft_server_stats(server) -> dict:
    s = NnfftServerStats()
    _check(lib().nnfft_server_stats(server, ctypes.byref(s)))
    return s.as_dict()


def nnfft_server_evict(server, plan_key):
    _check(lib().nnfft_server_evict(server, ctypes.c_uint64(plan_key)))


def nnfft_server_destroy(server):
    _check(lib().nnfft_server_destroy(server))


class Server:
    """Owning wrapper of a server; submit() keeps the request's tensors alive
    until wait()/poll() has returned its result."""

    def __init__(self, hbm_budget_bytes=0, planner_threads=0, streams=0, max_batch=0):
        self.handle = nnfft_server_create(hbm_budget_bytes, planner_threads, streams, max_batch)
        self._keep = {}

    def submit(self, N, v, x, f, y, **kw):
        t = nnfft_server_submit(self.handle, N, v, x, f, y, **kw)
        self._keep[t] = (v, x, f, y)
        return t

    def wait(self, ticket):
        try:
            return nnfft_server_wait(self.handle, ticket)
        finally:
            self._keep.pop(ticket, None)

    def poll(self, ticket):
        r = nnfft_server_poll(self.handle, ticket)
        if r is not None:
            self._keep.pop(ticket, None)
        return r

    def stats(self):
        return nnfft_server_stats(self.handle)

    def evict(self, plan_key):
        nnfft_server_evict(self.handle, plan_key)

    def close(self):
        if getattr(self, "handle", None) is not None:
            nnfft_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
