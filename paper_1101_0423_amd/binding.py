"""ctypes binding of include/dwf.h (same names, argument marshalling only).

Host arrays are numpy float64 in the canonical layouts of dwf.h; device
arrays are torch CUDA (HIP) float64 tensors whose data pointers are passed
straight through together with the current torch stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libdwf.so")

DWF_OK, DWF_PENDING = 0, 1
DWF_EINVAL, DWF_ENOMEM, DWF_EDEVICE, DWF_ENOCONV, DWF_EBUSY, DWF_ENOTFOUND = -1, -2, -3, -4, -5, -6
(OP_DW, OP_HOP_EO, OP_HOP_OE, OP_M5, OP_M5T, OP_C, OP_CDAG, OP_CCDAG, OP_D, OP_DDAG) = range(10)
PREC_FP64, PREC_FP32, PREC_FP16 = 0, 1, 2
# gauge-link storage of dwf_apply, or-ed into prec
LINKS_AUTO, LINKS_18, LINKS_12 = 0x000, 0x100, 0x200
SU3_TOL = 1e-6

# every function declared in include/dwf.h
EXPORTED = [
    "dwf_default_opts", "dwf_default_params", "dwf_create", "dwf_destroy", "dwf_apply", "dwf_apply_dev",
    "dwf_solve", "dwf_solve_dev", "dwf_submit", "dwf_submit_mass", "dwf_poll", "dwf_server_stats_get",
    "dwf_time_kernels", "dwf_last_error", "dwf_version", "dwf_gauge_su3_deviation", "dwf_apply_dev_noalloc",
    "dwf_stream_copy", "dwf_propagator", "dwf_propagator_dev", "dwf_odwf_weights",
]


SYSTEM_D = 0
SYSTEM_CCDAG = 1


class DwfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdwf error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("antiperiodic_t", ctypes.c_int), ("device", ctypes.c_int), ("sites_per_block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_prec", ctypes.c_int), ("reliable", ctypes.c_int),
                ("eps_inner", ctypes.c_double), ("maxiter", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("link_compress", ctypes.c_int), ("use_guess", ctypes.c_int),
                ("debug_stall_after", ctypes.c_int), ("system", ctypes.c_int), ("tile", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("reliable_updates", ctypes.c_int), ("fallback", ctypes.c_int), ("rhs_per_block", ctypes.c_int),
                ("tile", ctypes.c_int), ("sites_per_block", ctypes.c_int), ("block_order", ctypes.c_int),
                ("true_residual", ctypes.c_double), ("schur_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("gflops", ctypes.c_double), ("hbm_gbytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("admitted", ctypes.c_int64), ("peak_batch", ctypes.c_int64),
                ("waits_for_memory", ctypes.c_int64), ("p50_latency", ctypes.c_double),
                ("p99_latency", ctypes.c_double), ("busy_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib_path():
    return _LIB_PATH


def lib():
    """Load libdwf.so; raises if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run paper_1101_0423_amd/build.py "
                          "(or __graft_entry__.build())")
    # One HIP runtime per process.  PyTorch ships its own HIP and HSA
    # runtimes; loaded first, they also serve libdwf.so (same sonames).  Loaded
    # after libdwf.so has pulled in the system ones, a second HSA runtime
    # cannot open the GPU and torch finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    L.dwf_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.dwf_default_params.argtypes = [ctypes.POINTER(SolveParams)]
    L.dwf_create.argtypes = [ctypes.POINTER(vp), _dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double,
                             ctypes.c_double, _dp, _dp, ctypes.POINTER(Opts)]
    L.dwf_destroy.argtypes = [vp]
    L.dwf_destroy.restype = None
    L.dwf_apply.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int]
    L.dwf_apply_dev.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    L.dwf_apply_dev_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    L.dwf_solve.argtypes = [vp, _dp, _dp, ctypes.c_int, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats)]
    L.dwf_solve_dev.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats),
                                vp]
    L.dwf_submit.argtypes = [vp, _dp, ctypes.POINTER(SolveParams), ctypes.POINTER(ctypes.c_uint64)]
    L.dwf_submit_mass.argtypes = [vp, _dp, ctypes.c_double, ctypes.POINTER(SolveParams),
                                  ctypes.POINTER(ctypes.c_uint64)]
    L.dwf_poll.argtypes = [ctypes.c_uint64, _dp, ctypes.POINTER(SolveStats), ctypes.c_int]
    L.dwf_server_stats_get.argtypes = [ctypes.POINTER(ServerStats), ctypes.c_int]
    L.dwf_time_kernels.argtypes = [vp, ctypes.POINTER(SolveParams), ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.dwf_gauge_su3_deviation.argtypes = [_dp, ctypes.POINTER(ctypes.c_int), _dp]
    L.dwf_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp]
    L.dwf_odwf_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
    L.dwf_propagator.argtypes = [vp, _dp, _dp, ctypes.c_int, ctypes.POINTER(SolveParams),
                                 ctypes.POINTER(SolveStats)]
    L.dwf_propagator_dev.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(SolveParams),
                                     ctypes.POINTER(SolveStats), vp]
    L.dwf_last_error.restype = ctypes.c_char_p
    L.dwf_version.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name)
    _lib = L
    return L


def last_error():
    return lib().dwf_last_error().decode()


def _check(rc, ok=(DWF_OK,)):
    if rc not in ok:
        raise DwfError(rc, last_error())
    return rc


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def gauge_shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx, 4, 3, 3, 2)


def spinor_shape(dims, ns, nrhs=None):
    lx, ly, lz, lt = (int(d) for d in dims)
    s = (lt, lz, ly, lx, int(ns), 24)
    return s if nrhs is None else (int(nrhs),) + s


def check_host_spinors(a, dims, ns):
    """A host array of one spinor [Lt][Lz][Ly][Lx][Ns][24] or nrhs of them
    [nrhs][...]; returns it as contiguous float64 and nrhs.  Raises ValueError
    on any other shape (the C side would read or write past its end)."""
    a = _f64(a)
    one = spinor_shape(dims, ns)
    if a.shape == one:
        return a, 1
    if a.ndim == 7 and a.shape[1:] == one and a.shape[0] >= 1:
        return a, a.shape[0]
    raise ValueError(f"spinor array of shape {a.shape}; expected {one} or (nrhs,) + {one}")


def check_device_spinors(t, dims, ns, nrhs, device):
    """A torch tensor handed to a device-pointer entry point: float64, on the
    context's GPU, contiguous and of exactly nrhs spinors.  Raises ValueError
    otherwise (the kernels would read or write out of bounds)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("expected a torch tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"tensor dtype {t.dtype}; expected torch.float64")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"tensor on {t.device}; expected cuda:{device}")
    if not t.is_contiguous():
        raise ValueError("tensor is not contiguous")
    n = int(nrhs) * int(np.prod(spinor_shape(dims, ns)))
    if int(nrhs) < 1 or t.numel() != n:
        raise ValueError(f"tensor of {t.numel()} elements; expected nrhs * V4 * Ns * 24 = {n}")
    return t


def gauge_su3_deviation(gauge, dims):
    """max |U_2b - conj(U_0 x U_1)_b| over the field (dwf_gauge_su3_deviation)."""
    g = _f64(gauge)
    if g.shape != gauge_shape(dims):
        raise ValueError(f"gauge array of shape {g.shape}; expected {gauge_shape(dims)}")
    d = (ctypes.c_int * 4)(*[int(x) for x in dims])
    out = ctypes.c_double()
    _check(lib().dwf_gauge_su3_deviation(g.ctypes.data_as(_dp), d, ctypes.byref(out)))
    return out.value


def _ptr(a):
    return a.ctypes.data_as(_dp)


def default_params(**kw):
    p = SolveParams()
    lib().dwf_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


class Context:
    """One operator: resident gauge field and fifth-dimension tables (dwf_create)."""

    def __init__(self, gauge, dims, ns, m0, mq, sigma, omega, antiperiodic_t=False, device=0,
                 sites_per_block=0, hbm_budget_bytes=0, xcd_remap=0):
        L = lib()
        self._h = ctypes.c_void_p()
        o = Opts()
        L.dwf_default_opts(ctypes.byref(o))
        o.antiperiodic_t = int(antiperiodic_t)
        o.device = device
        o.sites_per_block = sites_per_block
        o.xcd_remap = xcd_remap
        o.hbm_budget_bytes = hbm_budget_bytes
        self.dims = tuple(int(d) for d in dims)
        self.gauge = _f64(gauge)
        if self.gauge.shape != gauge_shape(self.dims):
            raise ValueError(f"gauge array of shape {self.gauge.shape}; expected {gauge_shape(self.dims)}")
        self.device = int(device)
        self.ns, self.m0, self.mq = int(ns), float(m0), float(mq)
        self.sigma, self.omega = _f64(sigma), _f64(omega)
        if self.sigma.shape != (self.ns,) or self.omega.shape != (self.ns,):
            raise ValueError(f"sigma and omega must hold Ns = {self.ns} values")
        d = (ctypes.c_int * 4)(*self.dims)
        _check(L.dwf_create(ctypes.byref(self._h), _ptr(self.gauge), d, self.ns, self.m0, self.mq,
                            _ptr(self.sigma), _ptr(self.omega), ctypes.byref(o)))

    @property
    def handle(self):
        return self._h

    def spinor_shape(self, nrhs=None):
        return spinor_shape(self.dims, self.ns, nrhs)

    def close(self):
        if self._h:
            lib().dwf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- operators -------------------------------------------------------
    def apply(self, op, psi, prec=PREC_FP64):
        """out = op(psi) for host arrays [nrhs?][Lt][Lz][Ly][Lx][Ns][24];
        prec may carry a LINKS_* link storage."""
        psi, nrhs = check_host_spinors(psi, self.dims, self.ns)
        out = np.empty_like(psi)
        _check(lib().dwf_apply(self._h, op, prec, _ptr(psi), _ptr(out), nrhs))
        return out

    def apply_dev(self, op, psi, out, prec=PREC_FP64, nrhs=1, stream=None):
        """Device tensors (torch float64, contiguous, host layout)."""
        check_device_spinors(psi, self.dims, self.ns, nrhs, self.device)
        check_device_spinors(out, self.dims, self.ns, nrhs, self.device)
        _check(lib().dwf_apply_dev(self._h, op, prec, ctypes.c_void_p(psi.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), nrhs, _stream_ptr(stream)))
        return out

    def apply_dev_noalloc(self, op, psi, out, prec=PREC_FP64, nrhs=1, stream=None):
        """apply_dev with the workspace in the library's static device array
        (dwf_apply_dev_noalloc: no device allocation)."""
        check_device_spinors(psi, self.dims, self.ns, nrhs, self.device)
        check_device_spinors(out, self.dims, self.ns, nrhs, self.device)
        _check(lib().dwf_apply_dev_noalloc(self._h, op, prec, ctypes.c_void_p(psi.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), nrhs, _stream_ptr(stream)))
        return out

    # -- solves ----------------------------------------------------------
    def solve(self, b, x0=None, params=None, **kw):
        """Solve D x = b for host arrays; returns (x, [stats dict per rhs], status)."""
        b, nrhs = check_host_spinors(b, self.dims, self.ns)
        p = params if params is not None else default_params(**kw)
        if x0 is not None:
            x = _f64(x0).copy()
            if x.shape != b.shape:
                raise ValueError(f"guess of shape {x.shape}; expected {b.shape}")
            p.use_guess = 1
        else:
            x = np.zeros_like(b)
        st = (SolveStats * nrhs)()
        rc = _check(lib().dwf_solve(self._h, _ptr(b), _ptr(x), nrhs, ctypes.byref(p), st),
                    ok=(DWF_OK, DWF_ENOCONV))
        return x, [s.as_dict() for s in st], rc

    def solve_dev(self, b, x, nrhs=1, params=None, stream=None, **kw):
        p = params if params is not None else default_params(**kw)
        check_device_spinors(b, self.dims, self.ns, nrhs, self.device)
        check_device_spinors(x, self.dims, self.ns, nrhs, self.device)
        st = (SolveStats * nrhs)()
        rc = _check(lib().dwf_solve_dev(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        nrhs, ctypes.byref(p), st, _stream_ptr(stream)),
                    ok=(DWF_OK, DWF_ENOCONV))
        return [s.as_dict() for s in st], rc

    def spinor4_shape(self, nsrc=None):
        lx, ly, lz, lt = self.dims
        s = (lt, lz, ly, lx, 24)
        return s if nsrc is None else (int(nsrc),) + s

    def propagator(self, eta, params=None, **kw):
        """4D propagators R D^-1 W eta for host sources [nsrc?][Lt][Lz][Ly][Lx][24]
        (dwf_propagator); returns (out, [stats dict per source], status)."""
        eta = _f64(eta)
        one = self.spinor4_shape()
        if eta.shape == one:
            nsrc = 1
        elif eta.ndim == 6 and eta.shape[1:] == one and eta.shape[0] >= 1:
            nsrc = eta.shape[0]
        else:
            raise ValueError(f"source array of shape {eta.shape}; expected {one} or (nsrc,) + {one}")
        p = params if params is not None else default_params(**kw)
        out = np.zeros_like(eta)
        st = (SolveStats * nsrc)()
        rc = _check(lib().dwf_propagator(self._h, _ptr(eta), _ptr(out), nsrc, ctypes.byref(p), st),
                    ok=(DWF_OK, DWF_ENOCONV))
        return out, [x.as_dict() for x in st], rc

    def propagator_dev(self, eta, out, nsrc=1, params=None, stream=None, **kw):
        """Device tensors (torch float64, contiguous, nsrc 4D spinors)."""
        import torch
        n = int(nsrc) * int(np.prod(self.spinor4_shape()))
        for t in (eta, out):
            if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and
                    t.device.index == self.device and t.is_contiguous() and t.numel() == n):
                raise ValueError(f"expected contiguous float64 tensors of {n} elements on cuda:{self.device}")
        p = params if params is not None else default_params(**kw)
        st = (SolveStats * nsrc)()
        rc = _check(lib().dwf_propagator_dev(self._h, ctypes.c_void_p(eta.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), nsrc, ctypes.byref(p), st,
                                             _stream_ptr(stream)), ok=(DWF_OK, DWF_ENOCONV))
        return [x.as_dict() for x in st], rc

    def time_kernels(self, params=None, nrhs=1, launches=20, **kw):
        """Average ms and algorithmic bytes of the inner kernels: T (the
        cycle-start t1 = M5^T g5 r) and the iteration's A, B, C, D."""
        p = params if params is not None else default_params(**kw)
        ms = np.zeros(5)
        by = np.zeros(5)
        _check(lib().dwf_time_kernels(self._h, ctypes.byref(p), nrhs, launches, _ptr(ms), _ptr(by)))
        return dict(zip("TABCD", ms)), dict(zip("TABCD", by))

    # -- serving ---------------------------------------------------------
    def submit(self, b, mq=None, params=None, **kw):
        b = _f64(b)
        if b.shape != self.spinor_shape():
            raise ValueError(f"spinor array of shape {b.shape}; expected {self.spinor_shape()}")
        p = params if params is not None else default_params(**kw)
        t = ctypes.c_uint64()
        if mq is None:
            _check(lib().dwf_submit(self._h, _ptr(b), ctypes.byref(p), ctypes.byref(t)))
        else:
            _check(lib().dwf_submit_mass(self._h, _ptr(b), float(mq), ctypes.byref(p), ctypes.byref(t)))
        return t.value


def poll(ticket, shape, timeout_us=0):
    """Returns (status, x or None, stats dict or None)."""
    x = np.empty(shape, dtype=np.float64)
    st = SolveStats()
    rc = lib().dwf_poll(ctypes.c_uint64(ticket), _ptr(x), ctypes.byref(st), int(timeout_us))
    if rc == DWF_PENDING:
        return rc, None, None
    if rc not in (DWF_OK, DWF_ENOCONV):
        raise DwfError(rc, last_error())
    return rc, x, st.as_dict()


def stream_copy(src, dst, nontemporal=False, stream=None):
    """Plain device copy src -> dst (torch tensors of equal byte size, a
    multiple of 16) with cached or non-temporal accesses (dwf_stream_copy):
    the calibration reference of the memory counters.  stream: a HIP stream
    handle other than the legacy null stream (default: torch's current
    stream, which then must not be torch's default one, the null stream).
    Work that wrote src on other streams must be finished first."""
    nb = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("contiguous device tensors expected")
    if dst.numel() * dst.element_size() != nb or nb % 16:
        raise ValueError("equal sizes, a multiple of 16 bytes, expected")
    sp = _stream_ptr(stream)
    if not sp.value:
        raise ValueError("stream_copy needs a stream other than the legacy null stream, "
                         "e.g. torch.cuda.Stream().cuda_stream")
    _check(lib().dwf_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nb,
                                 int(bool(nontemporal)), src.device.index, sp))


def odwf_weights(ns, lambda_min, lambda_max):
    """The optimal domain-wall weights omega_s for |spec(gamma_5 D_w)| in
    [lambda_min, lambda_max] (dwf_odwf_weights); use them as sigma and omega."""
    out = np.zeros(int(ns))
    _check(lib().dwf_odwf_weights(int(ns), float(lambda_min), float(lambda_max), _ptr(out)))
    return out


def server_stats(reset=False):
    s = ServerStats()
    _check(lib().dwf_server_stats_get(ctypes.byref(s), int(reset)))
    return s.as_dict()
