"""FP64 direct-summation oracle for the half-space Stokes sums (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares nothing with the GPU library:
the C source ``ehs_oracle.c`` is compiled on its own with gcc and loaded here
through ctypes.

The sum evaluated is the half-space representation (paper Sec. 3, eq.
(v_sum_halfspace) with the corrections of eq. (phi)); see the header of
``ehs_oracle.c`` for the normalisation and the one reading that differs from the
printed text (the coefficient of the quadrupole term of phi_T).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ehs_oracle.c")
_LIB = os.path.join(_HERE, "libehs_oracle.so")

KERNELS = {"stokeslet": 0, "stresslet": 1, "rotlet": 2}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable flags: it also runs on other hosts)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("oracle_halfspace", "oracle_freespace"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, dp, dp, ctypes.c_long, dp, ctypes.c_long, dp, ctypes.c_int]
        lib.oracle_correction.restype = None
        lib.oracle_correction.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        lib.oracle_ewald_real.restype = ctypes.c_int
        lib.oracle_ewald_real.argtypes = [ctypes.c_int, dp, dp, ctypes.c_long, dp, ctypes.c_long, ctypes.c_double,
                                          ctypes.c_double, dp, ctypes.c_int]
        lib.oracle_correction_real.restype = None
        lib.oracle_correction_real.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double, dp, dp]
        lib.oracle_set_mutation.argtypes = [ctypes.c_int]
        lib.oracle_set_mutation.restype = None
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def torque_to_pair(v: np.ndarray) -> np.ndarray:
    """Return (g, q) per row with g x q = v (q a unit vector orthogonal to v).

    The rotlet sum depends on (g, q) only through g x q (paper Sec. 2 and
    eq. (phi)), so any such pair represents the torque v.
    """
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    # a helper axis not parallel to v
    a = np.zeros_like(v)
    idx = np.argmin(np.abs(v), axis=1)
    a[np.arange(len(v)), idx] = 1.0
    q = np.cross(v, a)
    nq = np.linalg.norm(q, axis=1, keepdims=True)
    nq[nq == 0] = 1.0
    q = q / nq
    g = np.cross(q, v)  # (q x v) x q = v for unit q orthogonal to v
    return np.concatenate([g, q], axis=1)


def _prep(kernel: str, y, s, x):
    k = KERNELS[kernel]
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    s = np.asarray(s, dtype=np.float64)
    if kernel == "stokeslet":
        s = np.ascontiguousarray(s).reshape(-1, 3)
    elif kernel == "rotlet" and s.reshape(len(y), -1).shape[1] == 3:
        s = np.ascontiguousarray(torque_to_pair(s))
    else:
        s = np.ascontiguousarray(s).reshape(-1, 6)
    if s.shape[0] != y.shape[0]:
        raise ValueError("strengths and sources differ in length")
    return k, y, s, x


def halfspace(kernel: str, y, s, x, nthreads: int = 0) -> np.ndarray:
    """Direct half-space sum u(x_t) over all sources (FP64, O(N*T)).

    kernel: 'stokeslet' (s = f, N x 3), 'stresslet' (s = (g, q), N x 6) or
    'rotlet' (s = (g, q), N x 6, or the torque v = g x q, N x 3).
    """
    lib = _load()
    k, y, s, x = _prep(kernel, y, s, x)
    u = np.zeros((x.shape[0], 3), dtype=np.float64)
    rc = lib.oracle_halfspace(k, _ptr(y), _ptr(s), y.shape[0], _ptr(x), x.shape[0], _ptr(u), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_halfspace failed")
    return u


def freespace(kernel: str, y, s, x, nthreads: int = 0) -> np.ndarray:
    """Direct free-space sum (paper Sec. 2), same conventions as ``halfspace``."""
    lib = _load()
    k, y, s, x = _prep(kernel, y, s, x)
    u = np.zeros((x.shape[0], 3), dtype=np.float64)
    rc = lib.oracle_freespace(k, _ptr(y), _ptr(s), y.shape[0], _ptr(x), x.shape[0], _ptr(u), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_freespace failed")
    return u


def correction(kernel: str, y, s, x):
    """phi and grad phi of one source at one point (eq. (phi))."""
    lib = _load()
    k, y, s, x = _prep(kernel, y, s, x)
    phi = np.zeros(1)
    g = np.zeros(3)
    lib.oracle_correction(k, _ptr(y[0]), _ptr(s[0]), _ptr(x[0]), _ptr(phi), _ptr(g))
    return float(phi[0]), g


def ewald_real(kernel: str, y, s, x, xi: float, rc: float, nthreads: int = 0) -> np.ndarray:
    """The real-space part of the Ewald split of the half-space sum (Sec. 4,
    appendix eq. (kernel_real_parts) and eq. (G_R)): direct pairs within
    r_c, images and corrections within r_c of the image point, and the
    stokeslet's self term; same conventions as ``halfspace``."""
    lib = _load()
    k, y, s, x = _prep(kernel, y, s, x)
    u = np.zeros((x.shape[0], 3), dtype=np.float64)
    rc_ = lib.oracle_ewald_real(k, _ptr(y), _ptr(s), y.shape[0], _ptr(x), x.shape[0], float(xi), float(rc), _ptr(u),
                                int(nthreads))
    if rc_ != 0:
        raise RuntimeError("oracle_ewald_real failed")
    return u


def correction_real(kernel: str, y, s, x, xi: float):
    """phi and grad phi of one source at one point with G_R = erfc(xi r)/r
    in place of 1/r."""
    lib = _load()
    k, y, s, x = _prep(kernel, y, s, x)
    phi = np.zeros(1)
    g = np.zeros(3)
    lib.oracle_correction_real(k, _ptr(y[0]), _ptr(s[0]), _ptr(x[0]), float(xi), _ptr(phi), _ptr(g))
    return float(phi[0]), g


def set_mutation(m: int) -> None:
    """Plant a deliberate mistake in the oracle (tests of the pins only)."""
    _load().oracle_set_mutation(int(m))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def rel_rms(u_ref, u) -> float:
    """Relative RMS error: RMS of the error over RMS of the reference (paper Sec. 5)."""
    u_ref = np.asarray(u_ref, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    return float(np.sqrt(np.sum((u_ref - u) ** 2)) / np.sqrt(np.sum(u_ref**2)))
