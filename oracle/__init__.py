"""ctypes front end of the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  Every function
takes and returns numpy arrays in the link layout (4, Lt, Lz, Ly, Lx, 3, 3)
complex128 (site fields: (Lt, Lz, Ly, Lx, ...)).

Functions that the paper's text does not pin by itself are checked in
``tests/test_oracle.py`` against closed forms, invariants, brute force and
independent library routines.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PLAIN = os.path.join(_HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build, used instead when
# LGF_ORACLE_SANITIZED=1 (the process must preload gcc's libasan.so)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
_SANITIZED = os.environ.get("LGF_ORACLE_SANITIZED") == "1"
_LIB = _LIB_SAN if _SANITIZED else _LIB_PLAIN

BUILD_CMD = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-fcx-limited-range", _SRC, "-o", _LIB_PLAIN, "-lm"]
SAN_BUILD_CMD = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                 "-fcx-limited-range", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                 _SRC, "-o", _LIB_SAN, "-lm"]


def build(sanitize: bool = False) -> str:
    """Compile the oracle with gcc (always recompiles); sanitize: the
    ASan/UBSan build liboracle_san.so."""
    subprocess.run(SAN_BUILD_CMD if sanitize else BUILD_CMD, check=True)
    return _LIB_SAN if sanitize else _LIB_PLAIN


_lib = None
_c = ctypes
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_zp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(sanitize=_SANITIZED)
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_set_threads": (None, [_c.c_int]),
        "orc_get_threads": (_c.c_int, []),
        "orc_functional": (_c.c_double, [_ip, _zp, _c.c_void_p]),
        "orc_F": (_c.c_double, [_ip, _zp]),
        "orc_delta": (None, [_ip, _zp, _zp]),
        "orc_theta_of_delta": (_c.c_double, [_ip, _zp]),
        "orc_theta": (_c.c_double, [_ip, _zp]),
        "orc_fft4d": (_c.c_int, [_ip, _zp, _c.c_int, _c.c_int]),
        "orc_dft4d_naive": (None, [_ip, _zp, _zp, _c.c_int]),
        "orc_p2max": (_c.c_double, [_ip]),
        "orc_fourier_accelerate": (_c.c_int, [_ip, _zp, _zp]),
        "orc_gauge_field": (_c.c_int, [_ip, _zp, _c.c_double, _zp]),
        "orc_gauge_rotate": (None, [_ip, _zp, _zp]),
        "orc_iterate": (_c.c_int, [_ip, _zp, _c.c_double, _c.c_int]),
        "orc_fix": (_c.c_int, [_ip, _zp, _c.c_double, _c.c_double, _c.c_int,
                               _c.POINTER(_c.c_int), _c.POINTER(_c.c_double),
                               _c.POINTER(_c.c_double), _dp, _dp]),
        "orc_fix_ex": (_c.c_int, [_ip, _zp, _c.c_double, _c.c_double, _c.c_int, _c.c_int,
                                  _c.POINTER(_c.c_int), _c.POINTER(_c.c_double),
                                  _c.POINTER(_c.c_double), _dp, _dp]),
        "orc_plaquette": (_c.c_double, [_ip, _zp]),
        "orc_unitarity": (None, [_zp, _c.c_int64, _c.POINTER(_c.c_double),
                                 _c.POINTER(_c.c_double)]),
        "orc_expm_su3": (None, [_dp, _zp]),
        "orc_functional_omega": (_c.c_double, [_ip, _zp, _dp]),
        "orc_functional_omega_grad": (_c.c_double, [_ip, _zp, _dp, _dp]),
        "orc_theta_grad": (_c.c_double, [_ip, _zp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _L_of_links(U: np.ndarray) -> np.ndarray:
    assert U.ndim == 7 and U.shape[0] == 4 and U.shape[-2:] == (3, 3), U.shape
    Lt, Lz, Ly, Lx = U.shape[1:5]
    return np.array([Lx, Ly, Lz, Lt], dtype=np.int32)


def _L_of_sites(a: np.ndarray) -> np.ndarray:
    Lt, Lz, Ly, Lx = a.shape[0:4]
    return np.array([Lx, Ly, Lz, Lt], dtype=np.int32)


def _z(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def functional(U, g=None) -> float:
    """F_U[g] (g=None: the identity)."""
    U = _z(U)
    gp = None if g is None else _z(g)
    ptr = None if gp is None else gp.ctypes.data
    return float(_load().orc_functional(_L_of_links(U), U, ptr))


def F(U) -> float:
    U = _z(U)
    return float(_load().orc_F(_L_of_links(U), U))


def delta(U) -> np.ndarray:
    U = _z(U)
    D = np.empty(U.shape[1:], dtype=np.complex128)
    _load().orc_delta(_L_of_links(U), U, D)
    return D


def theta(U) -> float:
    U = _z(U)
    return float(_load().orc_theta(_L_of_links(U), U))


def theta_of_delta(D) -> float:
    D = _z(D)
    return float(_load().orc_theta_of_delta(_L_of_sites(D), D))


def fft4d(a, sign: int = -1) -> np.ndarray:
    """Unnormalised 4D DFT over the first four axes (t, z, y, x) of ``a``;
    trailing axes are independent components."""
    a = _z(a).copy()
    ncomp = int(np.prod(a.shape[4:])) if a.ndim > 4 else 1
    rc = _load().orc_fft4d(_L_of_sites(a), a, ncomp, int(sign))
    if rc:
        raise ValueError("extent with a prime factor above 64")
    return a


def dft4d_naive(a, sign: int = -1) -> np.ndarray:
    a = _z(a)
    assert a.ndim == 4
    out = np.empty_like(a)
    _load().orc_dft4d_naive(_L_of_sites(a), a, out, int(sign))
    return out


def p2max(L) -> float:
    return float(_load().orc_p2max(np.asarray(L, dtype=np.int32)))


def fourier_accelerate(D) -> np.ndarray:
    D = _z(D)
    out = np.empty_like(D)
    if _load().orc_fourier_accelerate(_L_of_sites(D), D, out):
        raise ValueError("unsupported extent")
    return out


def gauge_field(U, alpha: float) -> np.ndarray:
    """g(x) of one Fourier-accelerated step from the current links."""
    U = _z(U)
    g = np.empty(U.shape[1:], dtype=np.complex128)
    if _load().orc_gauge_field(_L_of_links(U), U, float(alpha), g):
        raise ValueError("unsupported extent")
    return g


def gauge_rotate(U, g) -> np.ndarray:
    U = _z(U).copy()
    _load().orc_gauge_rotate(_L_of_links(U), U, _z(g))
    return U


def iterate(U, alpha: float, n: int) -> np.ndarray:
    U = _z(U).copy()
    if _load().orc_iterate(_L_of_links(U), U, float(alpha), int(n)):
        raise ValueError("unsupported extent")
    return U


def fix(U, alpha: float = 0.08, tol: float = 1e-15, max_iter: int = 10000,
        accelerate: bool = True, exact_exp: bool = False):
    """Gauge fixing to theta < tol.  Returns a dict with the links, the number
    of updates, F and theta of the returned links, their per-iteration
    histories and a status (0 converged, 1 max_iter, 2 non-finite).
    accelerate=False: plain steepest descent (no Fourier acceleration).
    exact_exp=True: g = exp((alpha/2) L Delta) exactly, instead of the first-
    order step followed by reunitarisation."""
    U = _z(U).copy()
    it = ctypes.c_int(0)
    f = ctypes.c_double(0)
    th = ctypes.c_double(0)
    Fh = np.zeros(max_iter + 1)
    Th = np.zeros(max_iter + 1)
    st = _load().orc_fix_ex(_L_of_links(U), U, float(alpha), float(tol), int(max_iter),
                            (1 if accelerate else 0) | (2 if exact_exp else 0), ctypes.byref(it), ctypes.byref(f),
                            ctypes.byref(th), Fh, Th)
    n = it.value
    return {"U": U, "iterations": n, "F": f.value, "theta": th.value,
            "F_hist": Fh[:n + 1], "theta_hist": Th[:n + 1], "status": int(st)}


def plaquette(U) -> float:
    U = _z(U)
    return float(_load().orc_plaquette(_L_of_links(U), U))


def unitarity(M):
    """(max |M M^+ - 1|, max |det M - 1|) over a stack of 3x3 matrices."""
    M = _z(M)
    n = M.size // 9
    a = ctypes.c_double(0)
    b = ctypes.c_double(0)
    _load().orc_unitarity(M, n, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def expm_su3(w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty((3, 3), dtype=np.complex128)
    _load().orc_expm_su3(w, out)
    return out


def functional_omega(U, omega) -> float:
    U = _z(U)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    return float(_load().orc_functional_omega(_L_of_links(U), U, om))


def functional_omega_grad(U, omega):
    """(F, dF/domega) with dF/domega shaped like omega (Lt, Lz, Ly, Lx, 8)."""
    U = _z(U)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    g = np.empty_like(om)
    Fv = _load().orc_functional_omega_grad(_L_of_links(U), U, om, g)
    return float(Fv), g


def theta_grad(U):
    """(theta, dtheta/deps) with dtheta/deps shaped (4, Lt, Lz, Ly, Lx, 8)."""
    U = _z(U)
    out = np.empty(U.shape[:5] + (8,), dtype=np.float64)
    th = _load().orc_theta_grad(_L_of_links(U), U, out)
    return float(th), out
