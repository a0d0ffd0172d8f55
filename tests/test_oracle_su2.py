"""Pins of the SU(2) oracle (oracle/su2.py).

The strongest pin is the embedding: an SU(2) field placed in the upper 2x2
block of SU(3) links (1 in the remaining diagonal entry) has a traceless
anti-hermitian A, so the SU(3) divergence equals the SU(2) one in that block;
its first-order step reunit(1 + (alpha/2) L Delta) is the embedded SU(2) step
(row 0 is already orthogonal to row 1, and row 2 is (0, 0, 1)); hence the
pinned SU(3) C oracle must follow the SU(2) trajectory exactly, with
F_3 = (2 F_2 + 1) / 3 and theta_3 = (2/3) theta_2.  The rest are closed forms,
finite differences, invariants and scipy's matrix exponential.
"""
import numpy as np
import pytest
import scipy.linalg

import inputs
import oracle
from oracle import su2

ALPHA = 0.08


def _embed(U2):
    U3 = np.zeros(U2.shape[:-2] + (3, 3), dtype=np.complex128)
    U3[..., :2, :2] = U2
    U3[..., 2, 2] = 1.0
    return U3


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 6, 4, 8)])
def test_embedding_in_su3_follows_the_su3_oracle(L):
    U2, _ = inputs.make_config_su2(L, 0.5, 11 + sum(L))
    U3 = _embed(U2)
    assert oracle.theta(U3) == pytest.approx(2.0 / 3.0 * su2.theta(U2), rel=1e-12)
    assert oracle.F(U3) == pytest.approx((2 * su2.F(U2) + 1) / 3, abs=1e-14)
    r3 = oracle.fix(U3, ALPHA, 0.0, 4)
    r2 = su2.fix(U2, ALPHA, 0.0, 4)
    assert np.max(np.abs(r3["U"][..., :2, :2] - r2["U"])) < 1e-13
    assert np.max(np.abs(r3["U"][..., 2, 2] - 1)) < 1e-13
    assert np.max(np.abs(r3["F_hist"] - (2 * r2["F_hist"] + 1) / 3)) < 1e-14
    assert np.max(np.abs(r3["theta_hist"] / r2["theta_hist"] - 2.0 / 3.0)) < 1e-11


def test_delta_is_the_gradient_of_F():
    """dF/domega^a(x) = -(i/(4 Nd Nc V)) Tr[sigma_a Delta(x)] for g = exp(i omega^a sigma_a/2)
    at one site (central differences)."""
    L = (4, 4, 4, 4)
    U, _ = inputs.make_config_su2(L, 0.6, 21)
    D = su2.delta(U)
    V = 256
    h = 1e-6
    rng = np.random.default_rng(3)
    for _ in range(6):
        x = tuple(rng.integers(0, 4, 4))
        a = int(rng.integers(0, 3))
        grads = []
        for sgn in (+1, -1):
            g = np.broadcast_to(np.eye(2, dtype=np.complex128), inputs.site_shape(L) + (2, 2)).copy()
            g[x] = scipy.linalg.expm(0.5j * sgn * h * inputs.PAULI[a])
            grads.append(su2.functional(U, g))
        fd = (grads[0] - grads[1]) / (2 * h)
        expect = np.real(-1j / (4 * 4 * 2 * V) * np.trace(inputs.PAULI[a] @ D[x]))
        assert abs(fd - expect) < 1e-9 * max(1.0, abs(expect)) + 1e-11


def test_theta_equals_gradient_norm():
    """Delta = i d_a sigma_a: theta = 8 Nd^2 Nc V sum (dF/domega)^2 = 256 V |grad F|^2."""
    U, _ = inputs.make_config_su2((4, 4, 6, 4), 0.5, 22)
    D = su2.delta(U)
    V = 4 * 4 * 6 * 4
    grad = np.stack([np.real(-1j / (4 * 4 * 2 * V) * np.einsum("ij,...ji->...", s, D))
                     for s in inputs.PAULI], axis=-1)
    assert su2.theta(U) == pytest.approx(256 * V * np.sum(grad ** 2), rel=1e-12)


def test_delta_vanishes_on_constant_links_and_unit_F():
    U = inputs.unit_config_su2((4, 4, 4, 4))
    assert su2.F(U) == 1.0 and su2.theta(U) == 0.0
    g = inputs.haar_su2(1, np.random.default_rng(4))[0]
    Uc = np.broadcast_to(g, U.shape).copy()
    assert su2.theta(Uc) < 1e-28


def test_abelian_contraction_factor():
    """A tiny sigma_3 field: theta shrinks by (1 - alpha p2max)^2 = (1 - 16 alpha)^2."""
    U = inputs.abelian_config_su2((8, 8, 8, 8), 1e-6, 23)
    r = su2.fix(U, ALPHA, 0.0, 3)
    ratios = r["theta_hist"][1:] / r["theta_hist"][:-1]
    assert np.all(np.abs(ratios - (1 - 16 * ALPHA) ** 2) < 1e-6)


def test_fourier_acceleration_plane_wave():
    """A plane wave is an eigenfunction of the acceleration operator with
    eigenvalue p2max / p2(p)."""
    shape = (4, 6, 8, 4)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    k = (1, 2, 3, 1)  # (t, z, y, x) wave numbers
    ph = 2 * np.pi * (k[0] * t / 4 + k[1] * z / 6 + k[2] * y / 8 + k[3] * x / 4)
    D = np.zeros(shape + (2, 2), dtype=np.complex128)
    D[..., 0, 1] = np.exp(1j * ph)
    p2 = sum(4 * np.sin(np.pi * kk / n) ** 2 for kk, n in zip(k, shape))
    p2max = 4 * 4.0
    out = su2.fourier_accelerate(D)
    assert np.max(np.abs(out - p2max / p2 * D)) < 1e-13


def test_exact_exponential_matches_scipy():
    rng = np.random.default_rng(5)
    for _ in range(20):
        w = rng.standard_normal(3) * rng.choice([1e-9, 1e-3, 0.3, 2.0])
        A = 1j * np.tensordot(w, inputs.PAULI, axes=(0, 0))
        assert np.max(np.abs(su2.expm_su2(A) - scipy.linalg.expm(A))) < 1e-15


@pytest.mark.parametrize("exact", [False, True])
def test_full_solve_invariants(exact):
    U, _ = inputs.make_config_su2((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("su2 8^4", 0.5)])
    r = su2.fix(U, ALPHA, 1e-13, 500, exact_exp=exact)
    assert r["status"] == 0 and r["theta"] < 1e-13
    assert np.all(np.diff(r["F_hist"]) >= -1e-15)
    assert abs(su2.plaquette(r["U"]) - su2.plaquette(U)) < 1e-12
    mu, md = su2.unitarity(r["U"])
    assert mu < 1e-13 and md < 1e-13


def test_recovers_unit_config_from_random_gauge():
    L = (4, 4, 4, 4)
    g = inputs.haar_su2(256, np.random.default_rng(6)).reshape(inputs.site_shape(L) + (2, 2))
    U = inputs.apply_gauge_transformation(inputs.unit_config_su2(L), g)
    r = su2.fix(U, ALPHA, 1e-15, 500)
    assert r["status"] == 0
    assert r["F"] == pytest.approx(1.0, abs=1e-13)


def test_plain_steepest_descent_needs_more_sweeps():
    U, _ = inputs.make_config_su2((8, 8, 8, 8), 0.5, 24)
    fa = su2.fix(U, ALPHA, 1e-10, 3000)
    sd = su2.fix(U, ALPHA, 1e-10, 3000, accelerate=False)
    assert fa["status"] == 0 and sd["status"] == 0
    assert sd["iterations"] > 2 * fa["iterations"]
