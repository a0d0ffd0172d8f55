"""Plain FP64 numpy oracle for Fourier-accelerated steepest-descent Landau gauge
fixing of 4D SU(2) lattice gauge fields (N_c = 2 in the paper's functional).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU leg, never by the GPU library, with which it shares no code.
Links are full 2x2 complex matrices, shape (4, Lt, Lz, Ly, Lx, 2, 2); sites
s = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 is x, y, z, t and lives on
array axis 3 - mu of a site field.

Every step follows the same readings as the SU(3) oracle, with N_c = 2:
  F_U[g]  = 1/(Nd Nc V) sum_x sum_mu Re Tr[g(x) U_mu(x) g(x+mu)^dagger]
  Delta   = A - Tr(A)/Nc,  A = X - X^dagger,  X = sum_mu [U_mu(x-mu) - U_mu(x)]
  theta   = 1/(Nc V) sum_x Tr[Delta Delta^dagger]
  L Delta = IFFT[K * FFT[Delta]],  K(p) = p2max / p2(p), K(0) = 0
  g       = reunit(1 + (alpha/2) L Delta), or exp((alpha/2) L Delta) exactly
  U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger for every link at once.
reunit normalises row 0 and completes it to SU(2): row 1 = (-conj(r0[1]),
conj(r0[0])).  The transform is numpy's FFT (a library primitive), applied to
every matrix entry; sums are plain numpy FP64 reductions (math.fsum for the
two global scalars).

The pins of this module (tests/test_oracle_su2.py) include an exact
cross-check against the SU(3) oracle: an SU(2) field embedded in the upper
2x2 block of SU(3) links follows the same trajectory there.
"""
from __future__ import annotations

import math

import numpy as np

ND, NC = 4, 2


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _shift(a, mu, d):
    """Site field a(x + d*mu) (d = +1 or -1), periodic."""
    return np.roll(a, -d, axis=3 - mu)


def _volume(U):
    return int(np.prod(U.shape[1:5]))


def functional(U, g=None) -> float:
    """F_U[g] of the display equation (g=None: the identity)."""
    V = _volume(U)
    tot = []
    for mu in range(ND):
        W = U[mu] if g is None else g @ U[mu] @ _dag(_shift(g, mu, +1))
        tot.append(np.real(np.trace(W, axis1=-2, axis2=-1)).ravel())
    return math.fsum(np.concatenate(tot)) / (ND * NC * V)


def F(U) -> float:
    return functional(U)


def delta(U):
    """Delta(x): anti-hermitian, traceless, shape (Lt, Lz, Ly, Lx, 2, 2)."""
    X = np.zeros(U.shape[1:], dtype=np.complex128)
    for mu in range(ND):
        X += _shift(U[mu], mu, -1) - U[mu]
    A = X - _dag(X)
    tr = np.trace(A, axis1=-2, axis2=-1)
    return A - (tr / NC)[..., None, None] * np.eye(NC)


def theta_of_delta(D) -> float:
    V = int(np.prod(D.shape[:4]))
    return math.fsum(np.real(np.sum(D * np.conj(D), axis=(-2, -1))).ravel()) / (NC * V)


def theta(U) -> float:
    return theta_of_delta(delta(U))


def p2_grid(shape):
    """p2(p) = sum_mu 4 sin^2(pi p_mu / L_mu) on the (Lt, Lz, Ly, Lx) grid."""
    axes = [4 * np.sin(np.pi * np.arange(n) / n) ** 2 for n in shape]
    t, z, y, x = np.meshgrid(*axes, indexing="ij")
    return t + z + y + x


def fourier_accelerate(D):
    """IFFT[K * FFT[D]] entry by entry, K = p2max/p2, K(0) = 0."""
    p2 = p2_grid(D.shape[:4])
    K = np.zeros_like(p2)
    nz = p2 > 0
    K[nz] = p2.max() / p2[nz]
    Dh = np.fft.fftn(D, axes=(0, 1, 2, 3))
    return np.fft.ifftn(Dh * K[..., None, None], axes=(0, 1, 2, 3))


def reunit(M):
    """Row 0 normalised, row 1 completing it to SU(2)."""
    r0 = M[..., 0, :] / np.linalg.norm(M[..., 0, :], axis=-1, keepdims=True)
    out = np.empty_like(M)
    out[..., 0, :] = r0
    out[..., 1, 0] = -np.conj(r0[..., 1])
    out[..., 1, 1] = np.conj(r0[..., 0])
    return out


def expm_su2(A):
    """exp(A) for anti-hermitian traceless 2x2 A: A^2 = -|v|^2 1 with
    |v|^2 = -det A, so exp(A) = cos|v| 1 + (sin|v| / |v|) A."""
    v2 = np.real(np.linalg.det(A))  # det(i v.sigma) = |v|^2
    v = np.sqrt(np.maximum(v2, 0.0))
    sinc = np.where(v > 1e-8, np.sin(v) / np.where(v > 0, v, 1.0), 1.0 - v2 / 6.0)
    return np.cos(v)[..., None, None] * np.eye(2) + sinc[..., None, None] * A


def gauge_field(U, alpha, accelerate=True, exact_exp=False):
    D = delta(U)
    LD = fourier_accelerate(D) if accelerate else D
    M = 0.5 * alpha * LD
    if exact_exp:
        return expm_su2(M)
    return reunit(np.eye(2) + M)


def gauge_rotate(U, g):
    out = np.empty_like(U)
    for mu in range(ND):
        out[mu] = g @ U[mu] @ _dag(_shift(g, mu, +1))
    return out


def iterate(U, alpha, n, accelerate=True, exact_exp=False):
    U = np.array(U, dtype=np.complex128)
    for _ in range(n):
        U = gauge_rotate(U, gauge_field(U, alpha, accelerate, exact_exp))
    return U


def fix(U, alpha=0.08, tol=1e-15, max_iter=10000, accelerate=True, exact_exp=False):
    """Iterate until theta < tol (tested before each update) or max_iter updates;
    same return dictionary as the SU(3) oracle's fix."""
    U = np.array(U, dtype=np.complex128)
    Fh, Th = [], []
    n, status = 0, 1
    while True:
        D = delta(U)
        th, f = theta_of_delta(D), F(U)
        Fh.append(f)
        Th.append(th)
        if not np.isfinite(th):
            status = 2
            break
        if th < tol:
            status = 0
            break
        if n >= max_iter:
            break
        LD = fourier_accelerate(D) if accelerate else D
        M = 0.5 * alpha * LD
        g = expm_su2(M) if exact_exp else reunit(np.eye(2) + M)
        U = gauge_rotate(U, g)
        n += 1
    return {"U": U, "iterations": n, "F": Fh[-1], "theta": Th[-1], "F_hist": np.array(Fh),
            "theta_hist": np.array(Th), "status": status}


def plaquette(U) -> float:
    """1/(6 Nc V) sum_x sum_{mu<nu} Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+."""
    V = _volume(U)
    parts = []
    for mu in range(ND):
        for nu in range(mu + 1, ND):
            P = U[mu] @ _shift(U[nu], mu, +1) @ _dag(_shift(U[mu], nu, +1)) @ _dag(U[nu])
            parts.append(np.real(np.trace(P, axis1=-2, axis2=-1)).ravel())
    return math.fsum(np.concatenate(parts)) / (6 * NC * V)


def unitarity(M):
    """(max |M M^+ - 1|, max |det M - 1|) over a stack of 2x2 matrices."""
    M = np.asarray(M).reshape(-1, 2, 2)
    a = np.max(np.abs(M @ _dag(M) - np.eye(2)))
    b = np.max(np.abs(np.linalg.det(M) - 1))
    return float(a), float(b)
