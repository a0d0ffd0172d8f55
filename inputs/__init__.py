"""Seeded synthetic SU(3) and SU(2) gauge-field inputs.

This module only *makes inputs*: random near-identity link fields, Haar-random
gauge transformations applied to them, tiny Abelian fields and random su(3)
parameter fields.  It holds none of the gauge-fixing arithmetic (no divergence,
no Fourier acceleration, no update step), so both the CPU oracle and the GPU
library can be fed from it without sharing any solver code.

Layout of every link field: complex128, C-contiguous, shape
``(4, Lt, Lz, Ly, Lx, 3, 3)``; direction mu = 0..3 is x, y, z, t and the
site index is ``s = x + Lx*(y + Ly*(z + Lz*t))`` (x fastest).

The paper measures on Wilson-action ensembles at three unstated couplings; they
are not available, so uncorrelated links ``U = exp(i*eps*sum_a h^a lambda_a/2)``
with ``h^a ~ N(0,1)`` stand in for them, the disorder ``eps`` playing the role
of the coupling.  A Haar-random gauge transformation is then applied so that
the gauge-fixing problem is non-trivial.  SU(2) fields (``*_su2``) are made the
same way with the Pauli matrices, shape ``(4, Lt, Lz, Ly, Lx, 2, 2)``.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "GELL_MANN", "site_shape", "random_near_identity_links", "haar_su3",
    "apply_gauge_transformation", "make_config", "unit_config",
    "abelian_config", "random_omega", "CONFIG_SEEDS",
    "PAULI", "haar_su2", "make_config_su2", "unit_config_su2", "abelian_config_su2",
]

# Seeds per (lattice, disorder) workload, so every consumer draws the same field.
CONFIG_SEEDS = {
    ("8^4", 0.5): 1001,
    ("32^4", 0.6): 3206,
    ("32^4", 0.45): 3245,
    ("32^4", 0.35): 3235,
    ("4^4", 0.5): 4005,
    ("16^4", 0.5): 1605,
    ("48^3x96", 0.45): 4845,
    ("36^3x72", 0.45): 3672,
    ("27^4", 0.45): 2745,
    ("su2 8^4", 0.5): 2801,
    ("su2 16^4", 0.5): 2161,
    ("su2 32^4", 0.45): 2324,
}


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


GELL_MANN = _gell_mann()


def site_shape(L) -> tuple:
    """(Lt, Lz, Ly, Lx) for L = (Lx, Ly, Lz, Lt)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return (Lt, Lz, Ly, Lx)


def _nthreads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunked(fn, arr: np.ndarray, out: np.ndarray, chunk: int = 1 << 16) -> None:
    """Apply ``fn`` to leading-axis chunks of ``arr`` on a thread pool (LAPACK
    releases the GIL), writing into ``out``; deterministic per element."""
    n = arr.shape[0]
    starts = list(range(0, n, chunk))

    def work(s):
        out[s:s + chunk] = fn(arr[s:s + chunk])

    if len(starts) <= 1:
        for s in starts:
            work(s)
        return
    with ThreadPoolExecutor(_nthreads()) as ex:
        list(ex.map(work, starts))


def _expi_hermitian(H: np.ndarray) -> np.ndarray:
    """exp(i H) for a stack of hermitian matrices (PyTorch's batched CPU
    matrix exponential, which is multi-threaded)."""
    import torch

    return torch.linalg.matrix_exp(torch.from_numpy(1j * H)).numpy()


def random_near_identity_links(L, eps: float, rng: np.random.Generator) -> np.ndarray:
    """U_mu(x) = exp(i*eps*sum_a h^a lambda_a/2), h^a ~ N(0,1).

    Draw order: h[mu][t][z][y][x][a] (one ``standard_normal`` call)."""
    shp = (4,) + site_shape(L)
    h = rng.standard_normal(shp + (8,))
    hf = h.reshape(-1, 8)
    out = np.empty((hf.shape[0], 3, 3), dtype=np.complex128)
    chunk = 1 << 20  # fixed, so results never depend on the machine
    for a in range(0, hf.shape[0], chunk):
        H = np.tensordot(hf[a:a + chunk], GELL_MANN, axes=([-1], [0])) * (0.5 * eps)
        out[a:a + chunk] = _expi_hermitian(H)
    return out.reshape(shp + (3, 3))


def _haar_from_ginibre(Z: np.ndarray) -> np.ndarray:
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(Q)
    return Q * (det ** (-1.0 / 3.0))[..., None, None]


def haar_su3(n: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(3) matrices: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54 (2007) 592),
    then divided by a cube root of the determinant.  Draw order: real parts of
    all n*9 entries, then imaginary parts."""
    Z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    out = np.empty_like(Z)
    _chunked(_haar_from_ginibre, Z, out)
    return out


def apply_gauge_transformation(U: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Input construction: U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger on every link.

    ``g`` has shape (Lt, Lz, Ly, Lx, 3, 3).  Used only to scramble generated
    inputs along their gauge orbit."""
    out = np.empty_like(U)
    for mu in range(4):
        gp = np.roll(g, -1, axis=3 - mu)  # g(x + mu-hat); array axis of mu is 3-mu
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(gp, -1, -2))
    return out


def make_config(L, eps: float, seed: int, haar: bool = True):
    """Synthetic workload: near-identity links at disorder ``eps`` followed (if
    ``haar``) by a Haar-random gauge transformation.  Returns ``(U, g)``."""
    rng = np.random.default_rng(seed)
    U = random_near_identity_links(L, eps, rng)
    g = None
    if haar:
        g = haar_su3(int(np.prod(site_shape(L))), rng).reshape(site_shape(L) + (3, 3))
        U = apply_gauge_transformation(U, g)
    return np.ascontiguousarray(U), g


def unit_config(L) -> np.ndarray:
    """All links equal to the identity."""
    U = np.zeros((4,) + site_shape(L) + (3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def abelian_config(L, amp: float, seed: int) -> np.ndarray:
    """Tiny field in the Cartan directions (lambda_3, lambda_8):
    U_mu(x) = diag(exp(i*phi)), phi from amp * N(0,1) coefficients."""
    rng = np.random.default_rng(seed)
    c = amp * rng.standard_normal((4,) + site_shape(L) + (2,))
    d3 = np.array([1.0, -1.0, 0.0])
    d8 = np.array([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    phase = 0.5 * (c[..., 0:1] * d3 + c[..., 1:2] * d8)
    U = np.zeros((4,) + site_shape(L) + (3, 3), dtype=np.complex128)
    for i in range(3):
        U[..., i, i] = np.exp(1j * phase[..., i])
    return U


def random_omega(L, sigma: float, seed: int) -> np.ndarray:
    """su(3) parameters omega^a(x) ~ N(0, sigma^2), shape (Lt, Lz, Ly, Lx, 8)."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(site_shape(L) + (8,))


# ----------------------------------------------------------------------- SU(2)

PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
                 dtype=np.complex128)


def _su2_from_quaternion(q: np.ndarray) -> np.ndarray:
    """q0 + i (q1 s1 + q2 s2 + q3 s3) for unit quaternions q (..., 4)."""
    out = np.empty(q.shape[:-1] + (2, 2), dtype=np.complex128)
    out[..., 0, 0] = q[..., 0] + 1j * q[..., 3]
    out[..., 0, 1] = q[..., 2] + 1j * q[..., 1]
    out[..., 1, 0] = -q[..., 2] + 1j * q[..., 1]
    out[..., 1, 1] = q[..., 0] - 1j * q[..., 3]
    return out


def random_near_identity_links_su2(L, eps: float, rng: np.random.Generator) -> np.ndarray:
    """U_mu(x) = exp(i*eps*sum_a h^a sigma_a/2), h^a ~ N(0,1), in the closed form
    cos(w) + i sin(w) (h/|h|).sigma with w = eps |h| / 2.  Draw order h[mu][t][z][y][x][a]."""
    shp = (4,) + site_shape(L)
    h = rng.standard_normal(shp + (3,))
    nh = np.linalg.norm(h, axis=-1, keepdims=True)
    w = 0.5 * eps * nh
    q = np.concatenate([np.cos(w), np.sin(w) * h / np.where(nh > 0, nh, 1.0)], axis=-1)
    return _su2_from_quaternion(q)


def haar_su2(n: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(2) matrices: unit quaternions from normalised
    4-dimensional Gaussian vectors (uniform on the 3-sphere)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    return _su2_from_quaternion(q)


def make_config_su2(L, eps: float, seed: int, haar: bool = True):
    """SU(2) workload: near-identity links at disorder ``eps`` followed (if
    ``haar``) by a Haar-random gauge transformation.  Returns ``(U, g)``."""
    rng = np.random.default_rng(seed)
    U = random_near_identity_links_su2(L, eps, rng)
    g = None
    if haar:
        g = haar_su2(int(np.prod(site_shape(L))), rng).reshape(site_shape(L) + (2, 2))
        U = apply_gauge_transformation(U, g)
    return np.ascontiguousarray(U), g


def unit_config_su2(L) -> np.ndarray:
    U = np.zeros((4,) + site_shape(L) + (2, 2), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = 1.0
    return U


def abelian_config_su2(L, amp: float, seed: int) -> np.ndarray:
    """Tiny field in the sigma_3 direction: U_mu(x) = diag(e^{i phi/2}, e^{-i phi/2})."""
    rng = np.random.default_rng(seed)
    phi = amp * rng.standard_normal((4,) + site_shape(L))
    U = np.zeros((4,) + site_shape(L) + (2, 2), dtype=np.complex128)
    U[..., 0, 0] = np.exp(0.5j * phi)
    U[..., 1, 1] = np.exp(-0.5j * phi)
    return U
