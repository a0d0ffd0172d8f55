"""Fourier-accelerated Landau gauge fixing of 4D SU(3) lattices on MI355X.

Thin ctypes binding over ``liblgf.so`` (C ABI in ``include/lgf.h``).  Every
step of the solver runs in the library's HIP kernels; this module only checks
tensor shapes, passes device pointers and the current HIP stream, and turns
status codes into exceptions.  PyTorch provides device memory and streams.

Link fields are ``torch.complex128`` CUDA tensors of shape
``(4, Lt, Lz, Ly, Lx, 3, 3)`` (mu = x, y, z, t; x fastest).
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

__all__ = [
    "load", "LgfError", "Context", "Result", "fix", "iterate", "functional", "theta",
    "plaquette", "measure_noalloc", "divergence", "fourier_accelerate", "fft4d", "functional_omega",
    "functional_omega_grad", "theta_grad", "LandauF", "LandauTheta", "EXPORTS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lgf.h")

LGF_OK, LGF_ERR_ARG, LGF_ERR_DEVICE, LGF_ERR_OOM = 0, 1, 2, 3
LGF_NOT_CONVERGED, LGF_ERR_NONFINITE, LGF_DIVERGING = 4, 5, 6
LGF_FP64, LGF_MIXED = 0, 1
STATUS_NAMES = {0: "ok", 1: "bad argument", 2: "device error", 3: "out of memory",
                4: "not converged", 5: "non-finite", 6: "diverging"}


def _declared_exports() -> list[str]:
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(lgf_\w+)\s*\(", text, re.M)))


EXPORTS = _declared_exports() if os.path.exists(HEADER) else []


class LgfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lgf error {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code


class _Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("fp32_iterations", ctypes.c_int),
                ("status", ctypes.c_int), ("F", ctypes.c_double), ("theta", ctypes.c_double),
                ("seconds", ctypes.c_double)]


@dataclass
class Result:
    iterations: int
    fp32_iterations: int
    status: int
    F: float
    theta: float
    seconds: float


_lib = None


def load(path: str | None = None):
    """Load liblgf.so (or the library at ``path`` / $LGF_LIB, e.g. the host-side
    sanitizer build).  torch is imported first so that the library binds to the
    HIP runtime torch already uses (one runtime: shared pointers and streams).
    Raises if the library has not been built -- there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime)

    p = path or os.environ.get("LGF_LIB") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1301_3460_amd.build`")
    lib = ctypes.CDLL(p)
    c = ctypes
    vp, dp, ip = c.c_void_p, c.POINTER(c.c_double), c.POINTER(c.c_int)
    sigs = {
        "lgf_create": (c.c_int, [c.POINTER(vp), c.POINTER(c.c_int * 4), c.c_int, vp]),
        "lgf_create_group": (c.c_int, [c.POINTER(vp), c.POINTER(c.c_int * 4), c.c_int, c.c_int,
                                       vp]),
        "lgf_destroy": (None, [vp]),
        "lgf_set_theta_switch": (c.c_int, [vp, c.c_double]),
        "lgf_set_acceleration": (c.c_int, [vp, c.c_int]),
        "lgf_set_exponential": (c.c_int, [vp, c.c_int]),
        "lgf_set_link_format": (c.c_int, [vp, c.c_int]),
        "lgf_set_field_precision": (c.c_int, [vp, c.c_int]),
        "lgf_iterate": (c.c_int, [vp, vp, c.c_double, c.c_int, c.POINTER(_Result)]),
        "lgf_fix": (c.c_int, [vp, vp, c.c_double, c.c_double, c.c_int, c.POINTER(_Result)]),
        "lgf_functional": (c.c_int, [vp, vp, vp, dp]),
        "lgf_theta": (c.c_int, [vp, vp, dp]),
        "lgf_plaquette": (c.c_int, [vp, vp, dp]),
        "lgf_divergence": (c.c_int, [vp, vp, vp]),
        "lgf_fourier_accelerate": (c.c_int, [vp, vp, vp]),
        "lgf_fft4d": (c.c_int, [vp, vp, c.c_int]),
        "lgf_functional_omega": (c.c_int, [vp, vp, vp, dp]),
        "lgf_functional_omega_grad": (c.c_int, [vp, vp, vp, dp, vp]),
        "lgf_theta_grad": (c.c_int, [vp, vp, vp, dp, vp]),
        "lgf_history": (c.c_int, [vp, vp, vp, c.c_int, ip]),
        "lgf_profile": (c.c_int, [vp, vp, c.c_double, c.c_int, vp]),
        "lgf_measure_noalloc": (c.c_int, [c.POINTER(c.c_int * 4), vp, vp, vp]),
        "lgf_last_error": (c.c_char_p, [vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _lattice_of_links(U) -> tuple:
    if U.dim() != 7 or U.shape[0] != 4 or tuple(U.shape[-2:]) not in ((3, 3), (2, 2)):
        raise ValueError("links must have shape (4, Lt, Lz, Ly, Lx, N, N) with N = 3 or 2, "
                         f"got {tuple(U.shape)}")
    Lt, Lz, Ly, Lx = (int(v) for v in U.shape[1:5])
    return (Lx, Ly, Lz, Lt)


def _check(t, dtype, shape=None, name="tensor"):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context for one lattice shape, gauge group SU(nc), precision,
    device and stream."""

    def __init__(self, L, precision: str = "fp64", stream=None, nc: int = 3):
        import torch

        lib = load()
        self.L = tuple(int(v) for v in L)
        self.nc = int(nc)
        self.precision = precision
        prec = {"fp64": LGF_FP64, "mixed": LGF_MIXED}[precision]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        arr = (ctypes.c_int * 4)(*self.L)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib.lgf_create_group(ctypes.byref(h), ctypes.byref(arr), self.nc, prec,
                                      ctypes.c_void_p(self.stream.cuda_stream))
        if rc != LGF_OK:
            raise LgfError(rc, lib.lgf_last_error(None).decode())
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lgf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        raise LgfError(rc, self._lib.lgf_last_error(self._h).decode())

    def _site_shape(self):
        Lx, Ly, Lz, Lt = self.L
        return (Lt, Lz, Ly, Lx)

    def _links(self, U, name="U"):
        import torch

        return _check(U, torch.complex128, (4,) + self._site_shape() + (self.nc, self.nc), name)

    def set_acceleration(self, on: bool):
        """True: Fourier-accelerated steepest descent; False: plain steepest descent."""
        rc = self._lib.lgf_set_acceleration(self._h, 1 if on else 0)
        if rc:
            self._err(rc)

    def set_exponential(self, exact: bool):
        """True: g = exp((alpha/2) L Delta) exactly; False (default): first-order
        step made unitary by Gram-Schmidt."""
        rc = self._lib.lgf_set_exponential(self._h, 1 if exact else 0)
        if rc:
            self._err(rc)

    def set_link_format(self, nreal: int):
        """12 (default, rows 0,1 stored), 18 (all rows stored) or 8 (the minimal
        SU(3) form) reals per working link in fix/iterate."""
        rc = self._lib.lgf_set_link_format(self._h, int(nreal))
        if rc:
            self._err(rc)

    def set_field_precision(self, bits: int):
        """64 (default) or 32: precision of the Fourier field in FP64 sweeps."""
        rc = self._lib.lgf_set_field_precision(self._h, int(bits))
        if rc:
            self._err(rc)

    def set_theta_switch(self, th: float):
        rc = self._lib.lgf_set_theta_switch(self._h, float(th))
        if rc:
            self._err(rc)

    def fix(self, U, alpha=0.08, theta_tol=1e-15, max_iter=10000, raise_on_status=False) -> Result:
        r = _Result()
        rc = self._lib.lgf_fix(self._h, self._links(U), float(alpha), float(theta_tol),
                               int(max_iter), ctypes.byref(r))
        if rc in (LGF_ERR_ARG, LGF_ERR_DEVICE, LGF_ERR_OOM) or (rc and raise_on_status):
            self._err(rc)
        return Result(r.iterations, r.fp32_iterations, r.status, r.F, r.theta, r.seconds)

    def iterate(self, U, alpha=0.08, n=1) -> Result:
        r = _Result()
        rc = self._lib.lgf_iterate(self._h, self._links(U), float(alpha), int(n), ctypes.byref(r))
        if rc in (LGF_ERR_ARG, LGF_ERR_DEVICE, LGF_ERR_OOM):
            self._err(rc)
        return Result(r.iterations, r.fp32_iterations, r.status, r.F, r.theta, r.seconds)

    def history(self, cap=1 << 16):
        import numpy as np

        F = np.zeros(cap)
        T = np.zeros(cap)
        n = ctypes.c_int(0)
        rc = self._lib.lgf_history(self._h, F.ctypes.data_as(ctypes.c_void_p),
                                   T.ctypes.data_as(ctypes.c_void_p), int(cap), ctypes.byref(n))
        if rc:
            self._err(rc)
        return F[:n.value], T[:n.value]

    KERNELS = ("fft_xy_fwd", "fft_zt", "fft_xy_inv", "update", "finalize")

    def profile(self, U, alpha=0.08, n=20) -> dict:
        """Mean per-kernel duration (ms) over n sweeps, HIP events on the
        context's stream; U is not modified."""
        import numpy as np

        ms = np.zeros(5)
        rc = self._lib.lgf_profile(self._h, self._links(U), float(alpha), int(n),
                                   ms.ctypes.data_as(ctypes.c_void_p))
        if rc:
            self._err(rc)
        return dict(zip(self.KERNELS, (float(v) for v in ms)))

    def functional(self, U, g=None) -> float:
        import torch

        out = ctypes.c_double()
        gp = None if g is None else _check(g, torch.complex128, self._site_shape() + (3, 3), "g")
        rc = self._lib.lgf_functional(self._h, self._links(U), gp, ctypes.byref(out))
        if rc:
            self._err(rc)
        return out.value

    def theta(self, U) -> float:
        out = ctypes.c_double()
        rc = self._lib.lgf_theta(self._h, self._links(U), ctypes.byref(out))
        if rc:
            self._err(rc)
        return out.value

    def plaquette(self, U) -> float:
        out = ctypes.c_double()
        rc = self._lib.lgf_plaquette(self._h, self._links(U), ctypes.byref(out))
        if rc:
            self._err(rc)
        return out.value

    def divergence(self, U):
        import torch

        D = torch.empty(self._site_shape() + (3, 3), dtype=torch.complex128, device=U.device)
        rc = self._lib.lgf_divergence(self._h, self._links(U), ctypes.c_void_p(D.data_ptr()))
        if rc:
            self._err(rc)
        return D

    def fourier_accelerate(self, D):
        import torch

        src = _check(D, torch.complex128, self._site_shape() + (3, 3), "D")
        out = torch.empty_like(D)
        rc = self._lib.lgf_fourier_accelerate(self._h, src, ctypes.c_void_p(out.data_ptr()))
        if rc:
            self._err(rc)
        return out

    def fft4d(self, fields, sign=-1):
        """In-place unnormalised 4D DFT of a (4, Lt, Lz, Ly, Lx) complex128 tensor."""
        import torch

        p = _check(fields, torch.complex128, (4,) + self._site_shape(), "fields")
        rc = self._lib.lgf_fft4d(self._h, p, int(sign))
        if rc:
            self._err(rc)
        return fields

    def functional_omega(self, U, omega) -> float:
        import torch

        out = ctypes.c_double()
        om = _check(omega, torch.float64, self._site_shape() + (8,), "omega")
        rc = self._lib.lgf_functional_omega(self._h, self._links(U), om, ctypes.byref(out))
        if rc:
            self._err(rc)
        return out.value

    def functional_omega_grad(self, U, omega):
        import torch

        out = ctypes.c_double()
        om = _check(omega, torch.float64, self._site_shape() + (8,), "omega")
        grad = torch.empty_like(omega)
        rc = self._lib.lgf_functional_omega_grad(self._h, self._links(U), om, ctypes.byref(out),
                                                 ctypes.c_void_p(grad.data_ptr()))
        if rc:
            self._err(rc)
        return out.value, grad

    def theta_grad(self, U, eps=None, need_grad=True):
        import torch

        out = ctypes.c_double()
        ep = None if eps is None else _check(eps, torch.float64, (4,) + self._site_shape() + (8,),
                                             "eps")
        grad = (torch.empty((4,) + self._site_shape() + (8,), dtype=torch.float64, device=U.device)
                if need_grad else None)
        rc = self._lib.lgf_theta_grad(self._h, self._links(U), ep, ctypes.byref(out),
                                      None if grad is None else ctypes.c_void_p(grad.data_ptr()))
        if rc:
            self._err(rc)
        return out.value, grad


_contexts: dict = {}


def _ctx_for(L, device, precision="fp64", nc=3) -> Context:
    """Cached context for lattice L and SU(nc) on `device`'s current stream."""
    import torch

    stream = torch.cuda.current_stream(device)
    key = (tuple(L), nc, precision, stream.device.index, stream.cuda_stream)
    c = _contexts.get(key)
    if c is None:
        c = Context(L, precision, stream, nc)
        _contexts[key] = c
    return c


def _ctx(U, precision="fp64") -> Context:
    return _ctx_for(_lattice_of_links(U), U.device, precision, int(U.shape[-1]))


def fix(U, alpha=0.08, theta_tol=1e-15, precision="fp64", max_iter=10000, theta_switch=1e-8,
        accelerate=True, exact_exp=False, link_format=12, field_bits=64):
    """Gauge-fix U in place; returns a Result (iterations, F, theta, status).
    accelerate=False runs plain (unaccelerated) steepest descent; exact_exp=True
    exponentiates the step exactly; link_format=18 stores all three rows of
    the working links, link_format=8 the minimal 8-real form."""
    c = _ctx(U, precision)
    if precision == "mixed":
        c.set_theta_switch(theta_switch)
    c.set_acceleration(accelerate)
    c.set_exponential(exact_exp)
    c.set_field_precision(field_bits)
    if c.nc == 3 or link_format != 12:
        c.set_link_format(link_format)
    return c.fix(U, alpha, theta_tol, max_iter)


def iterate(U, alpha=0.08, n=1, precision="fp64", accelerate=True, exact_exp=False,
            link_format=12, field_bits=64):
    c = _ctx(U, precision)
    c.set_acceleration(accelerate)
    c.set_exponential(exact_exp)
    c.set_field_precision(field_bits)
    if c.nc == 3 or link_format != 12:
        c.set_link_format(link_format)
    return c.iterate(U, alpha, n)


def functional(U, g=None):
    return _ctx(U).functional(U, g)


def theta(U):
    return _ctx(U).theta(U)


def plaquette(U):
    return _ctx(U).plaquette(U)


def measure_noalloc(U, out=None, stream=None):
    """{F, theta} of SU(3) links U into the float64 CUDA tensor ``out`` (shape
    (2,)) without a context and without device allocation in the library
    (lgf_measure_noalloc); enqueued on ``stream`` (default: the current one),
    not synchronised.  Returns ``out``."""
    import torch

    lib = load()
    L = _lattice_of_links(U)
    up = _check(U, torch.complex128, None, "U")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=U.device)
    op = _check(out, torch.float64, (2,), "out")
    st = stream if stream is not None else torch.cuda.current_stream(U.device)
    arr = (ctypes.c_int * 4)(*L)
    with torch.cuda.device(U.device):
        rc = lib.lgf_measure_noalloc(ctypes.byref(arr), up, op, ctypes.c_void_p(st.cuda_stream))
    if rc != LGF_OK:
        raise LgfError(rc, lib.lgf_last_error(None).decode())
    return out


def divergence(U):
    return _ctx(U).divergence(U)


def fourier_accelerate(D):
    Lt, Lz, Ly, Lx = (int(v) for v in D.shape[:4])
    return _ctx_for((Lx, Ly, Lz, Lt), D.device).fourier_accelerate(D)


def fft4d(fields, sign=-1):
    Lt, Lz, Ly, Lx = (int(v) for v in fields.shape[1:5])
    return _ctx_for((Lx, Ly, Lz, Lt), fields.device).fft4d(fields, sign)


def functional_omega(U, omega):
    return _ctx(U).functional_omega(U, omega)


def functional_omega_grad(U, omega):
    return _ctx(U).functional_omega_grad(U, omega)


def theta_grad(U, eps=None):
    return _ctx(U).theta_grad(U, eps)


def _autograd_functions():
    import torch

    class LandauF(torch.autograd.Function):
        """F_U[exp(i omega.T)] with a hand-written backward (dF/domega).

        forward evaluates F only (lgf_functional_omega); backward launches
        the gradient kernels (lgf_functional_omega_grad), so a forward under
        torch.no_grad() pays for no gradient."""

        @staticmethod
        def forward(ctx, omega, U):
            om = omega.detach().contiguous()
            F = _ctx(U).functional_omega(U, om)
            ctx.save_for_backward(om, U)
            return torch.tensor(F, dtype=torch.float64, device=omega.device)

        @staticmethod
        def backward(ctx, gout):
            om, U = ctx.saved_tensors
            _, grad = _ctx(U).functional_omega_grad(U, om)
            return gout * grad, None

    class LandauTheta(torch.autograd.Function):
        """theta of the links exp(i eps.T) U with a hand-written backward.

        forward evaluates theta only; backward launches the gradient kernel."""

        @staticmethod
        def forward(ctx, eps, U):
            ep = eps.detach().contiguous()
            th, _ = _ctx(U).theta_grad(U, ep, need_grad=False)
            ctx.save_for_backward(ep, U)
            return torch.tensor(th, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, gout):
            ep, U = ctx.saved_tensors
            _, grad = _ctx(U).theta_grad(U, ep)
            return gout * grad, None

    return LandauF, LandauTheta


def __getattr__(name):
    if name in ("LandauF", "LandauTheta"):
        F, T = _autograd_functions()
        globals()["LandauF"], globals()["LandauTheta"] = F, T
        return globals()[name]
    raise AttributeError(name)
