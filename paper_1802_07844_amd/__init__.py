"""MI355X half-space spectral Ewald summation of Stokes Green's functions.

Thin ctypes binding of the C ABI in ``include/ehs.h`` (library ``libehs.so``
in this directory).  Argument marshalling only: every step of the summation
runs in the HIP kernels of the library.  PyTorch provides device memory and
the current stream.

    import torch, paper_1802_07844_amd as ehs
    u = ehs.stokeslet(y, f, y, xi, r_c, tol)        # y, f: (N, 3) float64 on cuda

The library must be built (``python -m paper_1802_07844_amd.build``); a
missing library raises ``RuntimeError`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libehs.so")

STOKESLET, STRESSLET, ROTLET = 0, 1, 2
FAMILIES = {"stokeslet": STOKESLET, "stresslet": STRESSLET, "rotlet": ROTLET}
(OPT_PRECISION, OPT_TIMING, OPT_FORCE_M, OPT_FORCE_P, OPT_FORCE_MT, OPT_MEM_CAP, OPT_ZSLAB, OPT_GATHER_EXTRA,
 OPT_DGRID, OPT_FAIL_PRECOMPUTE, OPT_CELL_REACH, OPT_OVERLAP, OPT_PARTS, OPT_ADMISSION) = range(14)
NOALLOC_SCRATCH_BYTES = 512 << 20
ARENA_MIN_BYTES = 32 << 20
STAGES = ["bbox", "precompute", "binning", "realspace", "spread", "fwd_x", "fwd_y", "z_scale", "inv_y", "inv_x",
          "gather", "total"]
NSTAGES = len(STAGES)

EHS_OK, EHS_EINVAL, EHS_EDOMAIN, EHS_ERANGE, EHS_ENOMEM, EHS_EHIP, EHS_ETIMEDOUT, EHS_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7


class Report(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("P", ctypes.c_int32), ("Mt", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("Q", ctypes.c_int32), ("nf", ctypes.c_int32), ("nf3", ctypes.c_int32), ("warnings", ctypes.c_int32),
        ("ncell", ctypes.c_int32 * 3), ("family", ctypes.c_int32),
        ("L", ctypes.c_double), ("h", ctypes.c_double), ("Lt", ctypes.c_double), ("eta", ctypes.c_double),
        ("xi", ctypes.c_double), ("r_c", ctypes.c_double), ("tol", ctypes.c_double),
        ("est_real", ctypes.c_double), ("est_fourier", ctypes.c_double),
        ("origin", ctypes.c_double * 3),
        ("ms_stage", ctypes.c_double * NSTAGES),
        ("workspace_bytes", ctypes.c_double),
        ("zslab", ctypes.c_int32), ("Pg", ctypes.c_int32),
        ("Ps", ctypes.c_int32), ("dgrid", ctypes.c_int32),
        ("est_fp32", ctypes.c_double),
        ("x3_first", ctypes.c_int32), ("x3_corr_end", ctypes.c_int32),
        ("cell_reach", ctypes.c_int32), ("occupancy", ctypes.c_double),
        ("pairs_direct", ctypes.c_double), ("pairs_image", ctypes.c_double),
        ("free_space", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["ncell"] = list(self.ncell)
        d["origin"] = list(self.origin)
        d["ms_stage"] = dict(zip(STAGES, list(self.ms_stage)))
        return d


class EhsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ehs error {code}: {msg}")
        self.code = code


_lib = None
_lock = threading.Lock()


def lib():
    """Load libehs.so (raises RuntimeError if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_07844_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            vp, dp, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64
            L.ehs_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t]
            L.ehs_create.restype = ctypes.c_int
            L.ehs_destroy.argtypes = [vp]
            L.ehs_destroy.restype = None
            L.ehs_set_option.argtypes = [vp, ctypes.c_int, dp]
            L.ehs_set_option.restype = ctypes.c_int
            for name in ("ewald_halfspace_stokeslet", "ewald_halfspace_stresslet", "ewald_halfspace_rotlet",
                         "ewald_freespace_stokeslet", "ewald_freespace_stresslet", "ewald_freespace_rotlet"):
                fn = getattr(L, name)
                fn.argtypes = [vp, vp, vp, i64, vp, i64, dp, dp, dp, vp, vp, ctypes.POINTER(Report)]
                fn.restype = ctypes.c_int
            L.ewald_halfspace_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, i64, vp, i64, dp, dp, dp, vp, vp,
                                                  ctypes.POINTER(Report)]
            L.ewald_halfspace_noalloc.restype = ctypes.c_int
            L.ehs_context_memory.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int)]
            L.ehs_context_memory.restype = ctypes.c_int
            L.ehs_strerror.argtypes = [ctypes.c_int]
            L.ehs_strerror.restype = ctypes.c_char_p
            L.ehs_xi_for_cutoff.argtypes = [ctypes.c_int, dp, dp, dp]
            L.ehs_xi_for_cutoff.restype = dp
            L.ehs_cutoff_for_estimate.argtypes = [ctypes.c_int, dp, dp, dp]
            L.ehs_cutoff_for_estimate.restype = dp
            L.ehs_tune.argtypes = [vp, ctypes.c_int, vp, vp, i64, vp, i64, dp, dp, dp, ctypes.c_int, vp,
                                   ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int), vp,
                                   ctypes.POINTER(Report)]
            L.ehs_tune.restype = ctypes.c_int
            L.ehs_truncated_kernel_hat.argtypes = [ctypes.c_int, dp, dp]
            L.ehs_truncated_kernel_hat.restype = dp
            L.ehs_plan_query.argtypes = [ctypes.c_int, i64, i64, ctypes.POINTER(dp), ctypes.POINTER(dp), dp, dp, dp,
                                         dp, ctypes.c_int, ctypes.POINTER(Report)]
            L.ehs_plan_query.restype = ctypes.c_int
            L.ehs_debug_line_fft.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, vp]
            L.ehs_debug_line_fft.restype = ctypes.c_int
            L.ehs_debug_grid_taps.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, i64, vp, i64, dp, dp, dp, vp,
                                              vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int32), vp,
                                              ctypes.POINTER(Report)]
            L.ehs_debug_grid_taps.restype = ctypes.c_int
            _bind_serving(L)
            _lib = L
    return _lib


class Request(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("precision", ctypes.c_int32), ("N", ctypes.c_int64),
                ("T", ctypes.c_int64), ("sources", ctypes.c_void_p), ("strengths", ctypes.c_void_p),
                ("targets", ctypes.c_void_p), ("xi", ctypes.c_double), ("r_c", ctypes.c_double),
                ("tol", ctypes.c_double), ("u_out", ctypes.c_void_p)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("slot", ctypes.c_int32), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("footprint_bytes", ctypes.c_double), ("report", Report)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("nslots", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("cache_entries", ctypes.c_int32), ("cache_hits", ctypes.c_int64),
                ("cache_misses", ctypes.c_int64), ("evictions", ctypes.c_int64), ("arena_bytes", ctypes.c_double),
                ("arena_used", ctypes.c_double), ("arena_peak", ctypes.c_double), ("cache_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _bind_serving(L):
    vp = ctypes.c_void_p
    L.ehs_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t, ctypes.c_int]
    L.ehs_server_create.restype = ctypes.c_int
    L.ehs_server_destroy.argtypes = [vp]
    L.ehs_server_destroy.restype = None
    L.ehs_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.ehs_submit.restype = ctypes.c_int
    L.ehs_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(RequestStatus)]
    L.ehs_wait.restype = ctypes.c_int
    L.ehs_server_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.ehs_server_stats.restype = ctypes.c_int
    L.ehs_server_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_double]
    L.ehs_server_set_option.restype = ctypes.c_int


def strerror(code: int) -> str:
    return lib().ehs_strerror(int(code)).decode()


def check(code: int) -> None:
    if code != EHS_OK:
        raise EhsError(code, strerror(code))


def xi_for_cutoff(family, r_c: float, tol: float, L: float = 1.0) -> float:
    """xi for which the real-space truncation estimate equals tol/2 (host arithmetic in the library)."""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    return float(lib().ehs_xi_for_cutoff(fam, float(r_c), float(tol), float(L)))


def cutoff_for_estimate(family, xi: float, est: float, L: float = 1.0) -> float:
    """r_c at which the real-space truncation estimate equals est (host arithmetic in the library)."""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    return float(lib().ehs_cutoff_for_estimate(fam, float(xi), float(est), float(L)))


def plan_query(family, N, T, lo, hi, Q, xi, r_c, tol, precision=0) -> Report:
    """The plan an evaluation would use (host arithmetic only; no GPU needed)."""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    lo3 = (ctypes.c_double * 3)(*[float(v) for v in lo])
    hi3 = (ctypes.c_double * 3)(*[float(v) for v in hi])
    rep = Report()
    check(lib().ehs_plan_query(fam, int(N), int(T), lo3, hi3, float(Q), float(xi), float(r_c), float(tol),
                               int(precision), ctypes.byref(rep)))
    return rep


def truncated_kernel_hat(kind: int, k: float, R: float) -> float:
    return float(lib().ehs_truncated_kernel_hat(int(kind), float(k), float(R)))


def _stream_handle(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _dev_ptr(t, name, cols):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"{name} must have shape (n, {cols})")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """An ehs_ctx on one HIP device (owns workspace and the kernel cache).

    arena_bytes > 0 makes the context allocate one device region now and take
    every later evaluation's tables, octants and workspace from it."""

    def __init__(self, device: int = 0, arena_bytes: int = 0):
        self._h = ctypes.c_void_p()
        check(lib().ehs_create(ctypes.byref(self._h), int(device), int(arena_bytes)))
        self.device = int(device)

    def close(self):
        if self._h:
            lib().ehs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: float) -> None:
        check(lib().ehs_set_option(self._h, int(option), float(value)))

    def memory(self) -> dict:
        """Device memory the context holds (ehs_context_memory)."""
        ws, cb, ne = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        check(lib().ehs_context_memory(self._h, ctypes.byref(ws), ctypes.byref(cb), ctypes.byref(ne)))
        return {"workspace_bytes": ws.value, "cache_bytes": cb.value, "cache_entries": ne.value}

    def evaluate_noalloc(self, family, sources, strengths, targets, xi, r_c, tol, out, stream=None, report=False):
        """ewald_halfspace_noalloc: the evaluation from the library's static
        per-device scratch (no device allocation; `out` must be given)."""
        fam = FAMILIES[family] if isinstance(family, str) else int(family)
        ncol = 6 if fam == STRESSLET else 3
        ys = _dev_ptr(sources, "sources", 3)
        ss = _dev_ptr(strengths, "strengths", ncol)
        if strengths.shape[0] != sources.shape[0]:
            raise ValueError("strengths and sources differ in length")
        xs = _dev_ptr(targets, "targets", 3)
        uo = _dev_ptr(out, "out", 3)
        if out.shape[0] != targets.shape[0]:
            raise ValueError("out and targets differ in length")
        rep = Report()
        check(lib().ewald_halfspace_noalloc(self._h, fam, ys, ss, int(sources.shape[0]), xs, int(targets.shape[0]),
                                            float(xi), float(r_c), float(tol), uo, _stream_handle(stream),
                                            ctypes.byref(rep)))
        return (out, rep) if report else out

    def evaluate(self, family, sources, strengths, targets, xi, r_c, tol, out=None, stream=None, report=False,
                 free_space=False):
        """The half-space sum (or, with free_space, the free-space sum of the
        same kernel: ewald_freespace_*) at the targets."""
        import torch

        fam = FAMILIES[family] if isinstance(family, str) else int(family)
        ncol = 6 if fam == STRESSLET else 3
        ys = _dev_ptr(sources, "sources", 3)
        ss = _dev_ptr(strengths, "strengths", ncol)
        if strengths.shape[0] != sources.shape[0]:
            raise ValueError("strengths and sources differ in length")
        xs = _dev_ptr(targets, "targets", 3)
        T = targets.shape[0]
        if out is None:
            out = torch.empty((T, 3), dtype=torch.float64, device=targets.device)
        uo = _dev_ptr(out, "out", 3)
        rep = Report()
        if free_space:
            fn = {STOKESLET: lib().ewald_freespace_stokeslet, STRESSLET: lib().ewald_freespace_stresslet,
                  ROTLET: lib().ewald_freespace_rotlet}[fam]
        else:
            fn = {STOKESLET: lib().ewald_halfspace_stokeslet, STRESSLET: lib().ewald_halfspace_stresslet,
                  ROTLET: lib().ewald_halfspace_rotlet}[fam]
        rc = fn(self._h, ys, ss, int(sources.shape[0]), xs, int(T), float(xi), float(r_c), float(tol), uo,
                _stream_handle(stream), ctypes.byref(rep))
        check(rc)
        return (out, rep) if report else out

    def tune(self, family, sources, strengths, targets, xi0, r_c0, tol, max_evals=12, out=None, stream=None):
        """Runtime-optimal (xi, r_c) from the starting point (xi0, r_c0) by ehs_tune.

        Returns a dict: u (the result at the chosen parameters), xi, r_c, ms
        (its time), trace (list of (xi, r_c, ms) per timed candidate) and report.
        """
        import torch

        fam = FAMILIES[family] if isinstance(family, str) else int(family)
        ncol = 6 if fam == STRESSLET else 3
        ys = _dev_ptr(sources, "sources", 3)
        ss = _dev_ptr(strengths, "strengths", ncol)
        if strengths.shape[0] != sources.shape[0]:
            raise ValueError("strengths and sources differ in length")
        xs = _dev_ptr(targets, "targets", 3)
        T = targets.shape[0]
        if out is None:
            out = torch.empty((T, 3), dtype=torch.float64, device=targets.device)
        uo = _dev_ptr(out, "out", 3)
        best = (ctypes.c_double * 3)()
        trace = (ctypes.c_double * (3 * int(max_evals)))()
        ntr = ctypes.c_int(0)
        rep = Report()
        check(lib().ehs_tune(self._h, fam, ys, ss, int(sources.shape[0]), xs, int(T), float(xi0), float(r_c0),
                             float(tol), int(max_evals), uo, best, trace, ctypes.byref(ntr), _stream_handle(stream),
                             ctypes.byref(rep)))
        tr = [(trace[3 * i], trace[3 * i + 1], trace[3 * i + 2]) for i in range(ntr.value)]
        return {"u": out, "xi": best[0], "r_c": best[1], "ms": best[2], "trace": tr, "report": rep}

    def stokeslet(self, y, f, x, xi, r_c, tol, **kw):
        return self.evaluate(STOKESLET, y, f, x, xi, r_c, tol, **kw)

    def stresslet(self, y, gq, x, xi, r_c, tol, **kw):
        return self.evaluate(STRESSLET, y, gq, x, xi, r_c, tol, **kw)

    def rotlet(self, y, v, x, xi, r_c, tol, **kw):
        return self.evaluate(ROTLET, y, v, x, xi, r_c, tol, **kw)

    def debug_grid_taps(self, family, sources, strengths, targets, xi, r_c, tol, free_space=False, quad_in=None,
                        stream=None):
        """One evaluation with the stage taps of ehs_debug_grid_taps (unit tests).

        Returns a dict: u (with quad_in: the quadrature of those grids
        alone), spread (the grids as spread, FP64, shape (n, 2 M~, M~, M~)),
        n_spread, n_quad (grid counts) and report.  quad_in: FP64 CUDA tensor
        of shape (n_quad, 2 M~, M~, M~); learn the shape from a call without it.
        """
        import torch

        fam = FAMILIES[family] if isinstance(family, str) else int(family)
        ncol = 6 if fam == STRESSLET else 3
        ys = _dev_ptr(sources, "sources", 3)
        ss = _dev_ptr(strengths, "strengths", ncol)
        if strengths.shape[0] != sources.shape[0]:
            raise ValueError("strengths and sources differ in length")
        xs = _dev_ptr(targets, "targets", 3)
        T = targets.shape[0]
        out = torch.empty((T, 3), dtype=torch.float64, device=targets.device)
        uo = _dev_ptr(out, "out", 3)
        counts = (ctypes.c_int32 * 2)()
        rep = Report()
        args = (self._h, fam, 1 if free_space else 0, ys, ss, int(sources.shape[0]), xs, int(T), float(xi),
                float(r_c), float(tol), uo)
        check(lib().ehs_debug_grid_taps(*args, None, 0, None, 0, counts, _stream_handle(stream), ctypes.byref(rep)))
        Mt = rep.Mt
        spread = torch.empty((counts[0], 2 * Mt, Mt, Mt), dtype=torch.float64, device=targets.device)
        qp, qn = None, 0
        if quad_in is not None:
            if (not quad_in.is_cuda or quad_in.dtype != torch.float64 or not quad_in.is_contiguous()
                    or tuple(quad_in.shape) != (counts[1], 2 * Mt, Mt, Mt)):
                raise ValueError(f"quad_in: contiguous FP64 CUDA tensor of shape {(counts[1], 2 * Mt, Mt, Mt)}")
            qp, qn = ctypes.c_void_p(quad_in.data_ptr()), quad_in.numel()
        check(lib().ehs_debug_grid_taps(*args, ctypes.c_void_p(spread.data_ptr()), spread.numel(), qp, qn, counts,
                                        _stream_handle(stream), ctypes.byref(rep)))
        return {"u": out, "spread": spread, "n_spread": counts[0], "n_quad": counts[1], "report": rep}

    def debug_line_fft(self, x, inverse=False, stream=None):
        """Unnormalised FFT along the last axis of a complex CUDA tensor (unit tests)."""
        import torch

        if not x.is_cuda or x.dtype not in (torch.complex128, torch.complex64):
            raise TypeError("complex CUDA tensor expected")
        x = x.contiguous()
        n = x.shape[-1]
        nl = x.numel() // n
        out = torch.empty_like(x)
        fp32 = 1 if x.dtype == torch.complex64 else 0
        check(lib().ehs_debug_line_fft(self._h, n, nl, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       1 if inverse else 0, fp32, _stream_handle(stream)))
        return out


_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


def stokeslet(y, f, x, xi, r_c, tol, **kw):
    return default_context(y.device.index or 0).stokeslet(y, f, x, xi, r_c, tol, **kw)


def stresslet(y, gq, x, xi, r_c, tol, **kw):
    return default_context(y.device.index or 0).stresslet(y, gq, x, xi, r_c, tol, **kw)


def rotlet(y, v, x, xi, r_c, tol, **kw):
    return default_context(y.device.index or 0).rotlet(y, v, x, xi, r_c, tol, **kw)


class Server:
    """An ehs_server: continuous batching of requests on one device.

    ``submit`` validates, plans and queues a request and returns a ticket;
    ``wait`` returns ``(u, status)`` once it has completed.  The input tensors
    of a request are kept referenced until its ``wait``.  Inputs must be
    complete on the device when submitted (the current stream is synchronised
    first).
    """

    def __init__(self, device: int = 0, arena_bytes: int = 8 << 30, nslots: int = 4):
        self._h = ctypes.c_void_p()
        check(lib().ehs_server_create(ctypes.byref(self._h), int(device), int(arena_bytes), int(nslots)))
        self.device = int(device)
        self._keep = {}

    def submit(self, family, sources, strengths, targets, xi, r_c, tol, precision=0, out=None) -> int:
        import torch

        fam = FAMILIES[family] if isinstance(family, str) else int(family)
        ncol = 6 if fam == STRESSLET else 3
        req = Request()
        req.family = fam
        req.precision = int(precision)
        req.N = int(sources.shape[0])
        req.T = int(targets.shape[0])
        req.sources = _dev_ptr(sources, "sources", 3).value
        req.strengths = _dev_ptr(strengths, "strengths", ncol).value
        if strengths.shape[0] != sources.shape[0]:
            raise ValueError("strengths and sources differ in length")
        req.targets = _dev_ptr(targets, "targets", 3).value
        if out is None:
            out = torch.empty((req.T, 3), dtype=torch.float64, device=targets.device)
        req.u_out = _dev_ptr(out, "out", 3).value
        req.xi, req.r_c, req.tol = float(xi), float(r_c), float(tol)
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        check(lib().ehs_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (sources, strengths, targets, out)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(u, status dict) of a completed request; raises EhsError with its code on failure or timeout."""
        st = RequestStatus()
        rc = lib().ehs_wait(self._h, ctypes.c_uint64(ticket), int(timeout_ms), ctypes.byref(st))
        if rc == EHS_ETIMEDOUT:
            raise EhsError(rc, strerror(rc))
        keep = self._keep.pop(ticket, None)
        check(rc)
        d = {k: getattr(st, k) for k, _ in st._fields_ if k != "report"}
        d["report"] = st.report.as_dict()
        return keep[3], d

    def set_option(self, option: int, value: float) -> None:
        check(lib().ehs_server_set_option(self._h, int(option), float(value)))

    def stats(self) -> dict:
        s = ServeStats()
        check(lib().ehs_server_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h:
            lib().ehs_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
