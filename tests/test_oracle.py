"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper fixes F_U[g] (its display equation), the method class (steepest
ascent of F with Fourier acceleration) and the workload parameters
(alpha = 0.08, theta < 1e-15).  Everything else in the oracle is a reading of
the cited method; each piece is pinned here by something other than itself:
a brute-force DFT, an independent library routine (numpy.fft, scipy.linalg),
closed forms (plane waves, the Abelian contraction factor), invariants (gauge
invariance, unitarity, ascent) and finite differences of F.
"""
import numpy as np
import pytest
import scipy.linalg

import inputs
import oracle

ALPHA = 0.08


def _rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --------------------------------------------------------------------- FFT

@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 6, 6, 6), (2, 3, 4, 6), (6, 4, 3, 2)])
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft_matches_bruteforce_dft(L, sign):
    a = _rand_field(inputs.site_shape(L), 1)
    ref = oracle.dft4d_naive(a, sign)
    got = oracle.fft4d(a, sign)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (12, 12, 12, 12), (16, 8, 12, 6), (5, 7, 4, 3)])
def test_fft_matches_numpy(L):
    a = _rand_field(inputs.site_shape(L) + (3,), 2)
    got = oracle.fft4d(a, -1)
    ref = np.fft.fftn(a, axes=(0, 1, 2, 3))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    back = oracle.fft4d(got, +1) / np.prod(L)
    assert np.max(np.abs(back - a)) < 1e-13


def test_fft_parseval_and_plane_wave():
    L = (8, 6, 4, 12)
    a = _rand_field(inputs.site_shape(L), 3)
    A = oracle.fft4d(a, -1)
    V = np.prod(L)
    assert abs(np.sum(np.abs(A) ** 2) / V - np.sum(np.abs(a) ** 2)) < 1e-10
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in inputs.site_shape(L)], indexing="ij")
    n = (3, 2, 1, 5)  # (nx, ny, nz, nt)
    ph = 2 * np.pi * (n[0] * x / L[0] + n[1] * y / L[1] + n[2] * z / L[2] + n[3] * t / L[3])
    W = oracle.fft4d(np.exp(1j * ph), -1)
    expect = np.zeros_like(W)
    expect[n[3], n[2], n[1], n[0]] = V
    assert np.max(np.abs(W - expect)) < 1e-11


# ------------------------------------------------------- Fourier acceleration

def test_p2max():
    assert oracle.p2max((8, 8, 8, 8)) == pytest.approx(16.0, abs=1e-14)
    assert oracle.p2max((4, 6, 8, 12)) == pytest.approx(16.0, abs=1e-14)
    # odd extents never reach the zone corner: max 4 sin^2(pi n/3) = 3
    assert oracle.p2max((3, 3, 3, 3)) == pytest.approx(12.0, abs=1e-13)


def test_fourier_acceleration_plane_wave_eigenvalue():
    L = (8, 4, 6, 12)
    V = np.prod(L)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in inputs.site_shape(L)], indexing="ij")
    A = _rand_field((3, 3), 4)
    for n in [(1, 0, 0, 0), (3, 2, 1, 5), (4, 2, 3, 6), (0, 0, 0, 0)]:
        ph = 2 * np.pi * (n[0] * x / L[0] + n[1] * y / L[1] + n[2] * z / L[2] + n[3] * t / L[3])
        D = np.exp(1j * ph)[..., None, None] * A
        p2 = sum(4 * np.sin(np.pi * n[m] / L[m]) ** 2 for m in range(4))
        K = 0.0 if p2 == 0 else 16.0 / p2
        got = oracle.fourier_accelerate(D)
        assert np.max(np.abs(got - K * D)) < 1e-12 * max(1.0, K), n
    del V


# ------------------------------------------------------------ F, Delta, theta

def test_functional_unit_and_bounds():
    L = (4, 4, 4, 4)
    U1 = inputs.unit_config(L)
    assert oracle.F(U1) == pytest.approx(1.0, abs=1e-15)
    assert oracle.theta(U1) == 0.0
    U, _ = inputs.make_config(L, 0.5, 11)
    assert oracle.F(U) <= 1.0


def test_functional_with_g_matches_transformed_links():
    """F_U[g] evaluated with g equals F of the links transformed (numpy)."""
    L = (4, 6, 4, 4)
    U, _ = inputs.make_config(L, 0.5, 12)
    rng = np.random.default_rng(13)
    g = inputs.haar_su3(int(np.prod(L)), rng).reshape(inputs.site_shape(L) + (3, 3))
    Ug = inputs.apply_gauge_transformation(U, g)
    assert oracle.functional(U, g) == pytest.approx(oracle.F(Ug), abs=1e-14)
    # F is invariant under a global (constant) transformation
    c = inputs.haar_su3(1, rng)[0]
    gc = np.broadcast_to(c, g.shape).copy()
    assert oracle.functional(U, gc) == pytest.approx(oracle.F(U), abs=1e-14)


def test_delta_vanishes_on_constant_links():
    L = (4, 4, 4, 4)
    c = inputs.haar_su3(4, np.random.default_rng(14))
    U = np.empty((4,) + inputs.site_shape(L) + (3, 3), dtype=np.complex128)
    for mu in range(4):
        U[mu] = c[mu]
    assert np.max(np.abs(oracle.delta(U))) < 1e-15
    assert oracle.theta(U) < 1e-30


def test_delta_is_traceless_antihermitian():
    U, _ = inputs.make_config((4, 4, 6, 4), 0.5, 15)
    D = oracle.delta(U)
    assert np.max(np.abs(D + np.conj(np.swapaxes(D, -1, -2)))) < 1e-15
    assert np.max(np.abs(np.trace(D, axis1=-2, axis2=-1))) < 1e-14


def _fd_grad_F(U, omega0, sites, h):
    """Central differences of F_U[exp(i omega T)] at the given (site, a)."""
    out = []
    flat = omega0.reshape(-1, 8)
    for s, a in sites:
        op = flat.copy(); op[s, a] += h
        om = flat.copy(); om[s, a] -= h
        fp = oracle.functional_omega(U, op.reshape(omega0.shape))
        fm = oracle.functional_omega(U, om.reshape(omega0.shape))
        out.append((fp - fm) / (2 * h))
    return np.array(out)


def test_delta_is_the_gradient_of_F():
    """dF/domega^a(x) at omega = 0 equals -(i/(4 Nd Nc V)) Tr[lambda_a Delta(x)]:
    this fixes Delta's sign, its projection and its normalisation against F."""
    L = (4, 4, 4, 4)
    V = np.prod(L)
    U, _ = inputs.make_config(L, 0.5, 16)
    D = oracle.delta(U).reshape(V, 3, 3)
    rng = np.random.default_rng(17)
    sites = [(int(rng.integers(V)), int(rng.integers(8))) for _ in range(24)]
    fd = _fd_grad_F(U, np.zeros(inputs.site_shape(L) + (8,)), sites, 1e-5)
    an = np.array([(-1j / (4 * 4 * 3 * V) * np.trace(inputs.GELL_MANN[a] @ D[s])).real
                   for s, a in sites])
    assert np.max(np.abs(fd - an)) < 1e-9 * np.max(np.abs(an)) + 1e-12


def test_theta_equals_gradient_norm():
    """theta = 384 V sum_{x,a} (dF/domega^a)^2 at omega = 0 (Nd=4, Nc=3)."""
    L = (4, 4, 4, 4)
    V = np.prod(L)
    U, _ = inputs.make_config(L, 0.5, 18)
    _, grad = oracle.functional_omega_grad(U, np.zeros(inputs.site_shape(L) + (8,)))
    assert oracle.theta(U) == pytest.approx(384 * V * np.sum(grad ** 2), rel=1e-13)
    # and the oracle's analytic gradient matches finite differences of F
    rng = np.random.default_rng(19)
    sites = [(int(rng.integers(V)), int(rng.integers(8))) for _ in range(16)]
    fd = _fd_grad_F(U, np.zeros(inputs.site_shape(L) + (8,)), sites, 1e-5)
    an = np.array([grad.reshape(V, 8)[s, a] for s, a in sites])
    assert np.max(np.abs(fd - an)) < 1e-9 * np.max(np.abs(grad))


# ---------------------------------------------------------------- the solve

def test_alpha_normalisation_abelian_contraction():
    """Tiny Abelian field: every momentum mode of the divergence contracts by
    (1 - alpha p2max) per Fourier-accelerated step, so theta shrinks by
    (1 - 16 alpha)^2 = 0.0784 at alpha = 0.08 on an even lattice."""
    L = (8, 8, 8, 8)
    U = inputs.abelian_config(L, 1e-6, 20)
    for alpha in (0.08, 0.04):
        r = oracle.fix(U, alpha, 0.0, 4)
        th = r["theta_hist"]
        ratios = th[1:] / th[:-1]
        assert np.all(np.abs(ratios - (1 - 16 * alpha) ** 2) < 1e-5), ratios


@pytest.mark.parametrize("alpha", [0.01, 0.04, 0.08])
def test_ascent_F_non_decreasing(alpha):
    U, _ = inputs.make_config((4, 4, 4, 4), 0.5, 21)
    r = oracle.fix(U, alpha, 1e-13, 60 if alpha >= 0.04 else 20)
    assert np.all(np.diff(r["F_hist"]) >= -1e-15)


def test_full_solve_invariants_8x4():
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("8^4", 0.5)])
    P0 = oracle.plaquette(U)
    r = oracle.fix(U, ALPHA, 1e-12, 500)
    assert r["status"] == 0 and r["theta"] < 1e-12
    assert 20 <= r["iterations"] <= 60
    assert abs(oracle.plaquette(r["U"]) - P0) < 1e-12
    mu, md = oracle.unitarity(r["U"])
    assert mu < 1e-13 and md < 1e-13
    assert np.all(np.diff(r["F_hist"]) >= -1e-15)
    assert oracle.theta(r["U"]) == pytest.approx(r["theta"], rel=1e-12)


def test_recovers_unit_config_from_random_gauge():
    """A gauge-transformed unit configuration is driven back to F = 1."""
    L = (4, 4, 4, 4)
    g = inputs.haar_su3(int(np.prod(L)), np.random.default_rng(22)).reshape(
        inputs.site_shape(L) + (3, 3))
    U = inputs.apply_gauge_transformation(inputs.unit_config(L), g)
    assert oracle.F(U) < 0.5
    r = oracle.fix(U, ALPHA, 1e-15, 200)
    assert r["status"] == 0
    assert r["F"] == pytest.approx(1.0, abs=1e-13)
    assert abs(oracle.plaquette(r["U"]) - 1.0) < 1e-13


def test_iterate_matches_fix_trajectory():
    U, _ = inputs.make_config((4, 4, 4, 6), 0.5, 23)
    r = oracle.fix(U, ALPHA, 0.0, 5)
    U5 = oracle.iterate(U, ALPHA, 5)
    assert np.max(np.abs(U5 - r["U"])) == 0.0
    g = oracle.gauge_field(U, ALPHA)
    assert np.max(np.abs(oracle.gauge_rotate(U, g) - oracle.iterate(U, ALPHA, 1))) == 0.0
    # the update is the transformation the input generator applies
    assert np.max(np.abs(oracle.gauge_rotate(U, g) - inputs.apply_gauge_transformation(U, g))) < 1e-14


# ------------------------------------------------------------ group checks

def test_plaquette_pins():
    L = (4, 4, 4, 4)
    assert oracle.plaquette(inputs.unit_config(L)) == pytest.approx(1.0, abs=1e-15)
    U, _ = inputs.make_config(L, 0.5, 24, haar=False)
    g = inputs.haar_su3(int(np.prod(L)), np.random.default_rng(25)).reshape(
        inputs.site_shape(L) + (3, 3))
    assert oracle.plaquette(inputs.apply_gauge_transformation(U, g)) == pytest.approx(
        oracle.plaquette(U), abs=1e-14)
    # Abelian field: plaquette is the mean cosine of the lattice curl (closed form)
    A = inputs.abelian_config(L, 0.3, 26)
    ph = np.angle(np.diagonal(A, axis1=-2, axis2=-1))  # (4, t, z, y, x, 3)
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            curl = (ph[mu] + np.roll(ph[nu], -1, axis=3 - mu)
                    - np.roll(ph[mu], -1, axis=3 - nu) - ph[nu])
            tot += np.cos(curl).sum()
    assert oracle.plaquette(A) == pytest.approx(tot / (6 * 3 * np.prod(L)), abs=1e-14)


def test_unitarity_check():
    H = inputs.haar_su3(100, np.random.default_rng(27))
    mu, md = oracle.unitarity(H)
    assert mu < 1e-14 and md < 1e-14
    mu, md = oracle.unitarity(2 * np.eye(3, dtype=np.complex128)[None])
    assert mu == pytest.approx(3.0) and md == pytest.approx(7.0)


# ---------------------------------------------------------- differentiation

def test_expm_matches_scipy():
    rng = np.random.default_rng(28)
    for _ in range(10):
        w = rng.normal(0, 1.5, 8)
        X = 0.5j * np.tensordot(w, inputs.GELL_MANN, axes=(0, 0))
        assert np.max(np.abs(oracle.expm_su3(w) - scipy.linalg.expm(X))) < 1e-14


def test_omega_gradient_matches_finite_differences():
    """Exact-exponential parametrisation at omega != 0: the chain rule through
    the exponential map is needed (a left/right-trivialised gradient alone is
    off by O(omega))."""
    L = (4, 4, 4, 4)
    V = np.prod(L)
    U, _ = inputs.make_config(L, 0.5, 29)
    om = inputs.random_omega(L, 0.5, 30)
    F0, grad = oracle.functional_omega_grad(U, om)
    assert F0 == pytest.approx(oracle.functional_omega(U, om), abs=1e-15)
    rng = np.random.default_rng(31)
    sites = [(int(rng.integers(V)), int(rng.integers(8))) for _ in range(32)]
    fd = _fd_grad_F(U, om, sites, 1e-5)
    an = np.array([grad.reshape(V, 8)[s, a] for s, a in sites])
    assert np.max(np.abs(fd - an)) < 1e-8 * np.max(np.abs(grad))


def test_theta_gradient_matches_finite_differences():
    L = (4, 4, 4, 4)
    V = np.prod(L)
    U, _ = inputs.make_config(L, 0.5, 32)
    th, grad = oracle.theta_grad(U)
    assert th == pytest.approx(oracle.theta(U), rel=1e-14)
    rng = np.random.default_rng(33)
    h = 1e-5
    Uf = U.reshape(4, V, 3, 3)
    errs = []
    for _ in range(16):
        mu, s, a = int(rng.integers(4)), int(rng.integers(V)), int(rng.integers(8))
        w = np.zeros(8); w[a] = h
        Ep = scipy.linalg.expm(0.5j * np.tensordot(w, inputs.GELL_MANN, axes=(0, 0)))
        Up = Uf.copy(); Up[mu, s] = Ep @ Up[mu, s]
        Um = Uf.copy(); Um[mu, s] = np.conj(Ep.T) @ Um[mu, s]
        fd = (oracle.theta(Up.reshape(U.shape)) - oracle.theta(Um.reshape(U.shape))) / (2 * h)
        errs.append(abs(fd - grad.reshape(4, V, 8)[mu, s, a]))
    assert max(errs) < 1e-7 * np.max(np.abs(grad))


# ------------------------------------------------ unaccelerated steepest descent

def test_plain_steepest_descent_mode_contraction():
    """Without Fourier acceleration a single Abelian plane-wave mode of lattice
    momentum p contracts by (1 - alpha p2(p)) per sweep, so theta shrinks by
    (1 - alpha p2)^2: slow for the lowest mode (critical slowing down)."""
    L = (8, 8, 8, 8)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in inputs.site_shape(L)], indexing="ij")
    amp = 1e-6
    phase = amp * np.cos(2 * np.pi * x / L[0])  # longitudinal mode k = (1, 0, 0, 0) in A_x
    U = inputs.unit_config(L)
    d3 = np.array([1.0, -1.0, 0.0])
    for i in range(3):
        U[0, ..., i, i] = np.exp(0.5j * phase * d3[i])
    p2 = 4 * np.sin(np.pi / L[0]) ** 2
    for alpha, acc in ((0.08, False), (0.08, True)):
        r = oracle.fix(U, alpha, 0.0, 3, accelerate=acc)
        ratios = r["theta_hist"][1:] / r["theta_hist"][:-1]
        expect = (1 - alpha * p2) ** 2 if not acc else (1 - 16 * alpha) ** 2
        assert np.all(np.abs(ratios - expect) < 1e-6), (acc, ratios, expect)


def test_plain_steepest_descent_converges_slower():
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, 51)
    fa = oracle.fix(U, ALPHA, 1e-10, 2000)
    sd = oracle.fix(U, ALPHA, 1e-10, 2000, accelerate=False)
    assert fa["status"] == 0 and sd["status"] == 0
    assert sd["iterations"] > 2 * fa["iterations"]
    assert np.all(np.diff(sd["F_hist"]) >= -1e-15)


# ------------------------------------------------------- exact exponential step

def test_exact_exp_step_matches_scipy():
    """One exact-exponential step is the gauge rotation by scipy's expm of
    (alpha/2) L Delta, with L Delta from the pinned transform."""
    U, _ = inputs.make_config((4, 6, 4, 8), 0.5, 52)
    LD = oracle.fourier_accelerate(oracle.delta(U))
    g = np.array([scipy.linalg.expm(0.5 * ALPHA * m) for m in LD.reshape(-1, 3, 3)])
    ref = oracle.gauge_rotate(U, g.reshape(LD.shape))
    got = oracle.fix(U, ALPHA, 0.0, 1, exact_exp=True)["U"]
    assert np.max(np.abs(got - ref)) < 1e-14
    first_order = oracle.fix(U, ALPHA, 0.0, 1)["U"]
    assert np.max(np.abs(first_order - ref)) > 1e-6


def test_exact_exp_abelian_phases():
    """On diagonal (Cartan) links all matrices commute and L Delta is diagonal,
    i*phi_k(x): the exact step adds c (phi_k(x) - phi_k(x+mu)) to the phase of
    each diagonal entry (c = alpha/2).  The first-order step rotates the
    first two by psi_k = atan(c phi_k) instead, and the third by
    -(psi_0 + psi_1), since row 2 is rebuilt from rows 0 and 1."""
    L = (4, 4, 6, 8)
    U = inputs.abelian_config(L, 0.3, 53)
    LD = oracle.fourier_accelerate(oracle.delta(U))
    phi = np.imag(np.diagonal(LD, axis1=-2, axis2=-1))
    c = 0.5 * ALPHA
    got = oracle.fix(U, ALPHA, 0.0, 1, exact_exp=True)["U"]
    fo = oracle.fix(U, ALPHA, 0.0, 1)["U"]
    for mu in range(4):
        phi_p = np.roll(phi, -1, axis=3 - mu)  # phi(x + mu); axes are (t, z, y, x)
        base = np.angle(np.diagonal(U[mu], axis1=-2, axis2=-1))
        expect = np.exp(1j * (base + c * (phi - phi_p)))
        assert np.max(np.abs(np.diagonal(got[mu], axis1=-2, axis2=-1) - expect)) < 1e-14
        off = got[mu] * (1 - np.eye(3))
        assert np.max(np.abs(off)) < 1e-15
        psi = np.arctan(c * phi)
        psi[..., 2] = -(psi[..., 0] + psi[..., 1])
        psi_p = np.roll(psi, -1, axis=3 - mu)
        first = np.exp(1j * (base + psi - psi_p))
        assert np.max(np.abs(np.diagonal(fo[mu], axis1=-2, axis2=-1) - first)) < 1e-14
    assert np.max(np.abs(got - fo)) > 1e-6


def test_exact_exp_reaches_the_same_maximum():
    """The two step rules share their fixed points; from the same start they
    reach the same local maximum of F in about the same number of sweeps."""
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, 54)
    fo = oracle.fix(U, ALPHA, 1e-13, 500)
    ex = oracle.fix(U, ALPHA, 1e-13, 500, exact_exp=True)
    assert fo["status"] == 0 and ex["status"] == 0
    assert abs(fo["iterations"] - ex["iterations"]) <= 2
    assert abs(fo["F"] - ex["F"]) < 1e-12
    assert np.all(np.diff(ex["F_hist"]) >= -1e-15)
    assert abs(oracle.plaquette(ex["U"]) - oracle.plaquette(U)) < 1e-12
    mu, md = oracle.unitarity(ex["U"])
    assert mu < 1e-13 and md < 1e-13
