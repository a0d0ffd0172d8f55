"""Full solves on the GPU against the FP64 oracle, status handling, mixed precision."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

ALPHA = 0.08


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def cpu(t):
    return t.detach().cpu().numpy()


def _check_solution(Uout, Uin, tol, F):
    """The oracle re-measures the returned links."""
    assert oracle.theta(Uout) < tol
    assert oracle.F(Uout) == pytest.approx(F, abs=1e-13)
    assert abs(oracle.plaquette(Uout) - oracle.plaquette(Uin)) < 1e-12
    mu, md = oracle.unitarity(Uout)
    assert mu < 1e-13 and md < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,eps,seed,tol", [
    ((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("8^4", 0.5)], 1e-12),
    ((4, 4, 4, 4), 0.5, inputs.CONFIG_SEEDS[("4^4", 0.5)], 1e-15),
    ((4, 6, 8, 12), 0.45, 77, 1e-15),
    ((6, 6, 6, 6), 0.6, 78, 1e-14),
    # planes where the FP32 sweeps accumulate G inside the inverse (x,y) pass:
    # register columns (32 wide), and the 4-field LDS kernel for wider planes
    # with register spans up to 16 (48 wide) and 32 (Ly = 48 beside Lx = 32)
    ((32, 8, 4, 4), 0.5, 80, 1e-14),
    ((48, 4, 4, 6), 0.5, 79, 1e-14),
    ((32, 48, 2, 2), 0.5, 82, 1e-14),
    # odd extents (p2max below 16) and two-pass / one-axis transform extents
    ((9, 9, 9, 9), 0.5, 83, 1e-14),
    ((27, 4, 6, 9), 0.5, 84, 1e-14),
    ((36, 4, 6, 72), 0.5, 85, 1e-14),
    ((256, 48, 2, 2), 0.5, 86, 1e-14),
])
def test_solve_matches_oracle(lgf_gpu, L, eps, seed, tol, precision):
    U, _ = inputs.make_config(L, eps, seed)
    ref = oracle.fix(U, ALPHA, tol, 1000)
    assert ref["status"] == 0
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, tol, precision=precision, max_iter=1000)
    assert r.status == 0
    Uout = cpu(Ug)
    _check_solution(Uout, U, tol, r.F)
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    else:
        assert r.fp32_iterations > 0 and r.iterations > r.fp32_iterations
        assert r.iterations <= ref["iterations"] + 2


def test_history_monotone_and_consistent(lgf_gpu):
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, 31)
    Ug = gpu(U)
    ctx = lgf_gpu._ctx(Ug)
    r = ctx.fix(Ug, ALPHA, 1e-13, 500)
    F, T = ctx.history()
    assert len(F) == r.iterations + 1
    assert np.all(np.diff(F) >= -1e-15)
    assert T[-1] == r.theta and T[-1] < 1e-13 and np.all(T[:-1] >= 1e-13)
    ref = oracle.fix(U, ALPHA, 1e-13, 500)
    n = min(len(F), len(ref["F_hist"]))
    assert np.max(np.abs(F[:n] - ref["F_hist"][:n])) < 1e-12


def test_converged_input_takes_zero_updates(lgf_gpu):
    U = inputs.unit_config((4, 4, 4, 4))
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-15)
    assert r.status == 0 and r.iterations == 0 and r.theta == 0.0 and r.F == 1.0
    assert np.array_equal(cpu(Ug), U)


def test_max_iter_reached(lgf_gpu):
    U, _ = inputs.make_config((4, 4, 4, 4), 0.5, 32)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-15, max_iter=3)
    assert r.status == lgf_gpu.LGF_NOT_CONVERGED and r.iterations == 3
    assert np.max(np.abs(cpu(Ug) - oracle.iterate(U, ALPHA, 3))) < 1e-13
    assert r.theta == pytest.approx(oracle.theta(cpu(Ug)), rel=1e-12)
    r0 = lgf_gpu.fix(gpu(U), ALPHA, 1e-15, max_iter=0)
    assert r0.status == lgf_gpu.LGF_NOT_CONVERGED and r0.iterations == 0


def test_nonfinite_input(lgf_gpu):
    U, _ = inputs.make_config((4, 4, 4, 4), 0.5, 33)
    U[1, 0, 1, 2, 3, 0, 1] = np.nan
    r = lgf_gpu.fix(gpu(U), ALPHA, 1e-15)
    assert r.status == lgf_gpu.LGF_ERR_NONFINITE and r.iterations == 0


def test_too_large_step_diverges(lgf_gpu):
    """alpha above 2/p2max = 0.125 amplifies the divergence (|1 - 16 alpha| > 1)."""
    U = inputs.abelian_config((8, 8, 8, 8), 1e-4, 34)
    r = lgf_gpu.fix(gpu(U), 0.2, 1e-15, max_iter=100)
    assert r.status == lgf_gpu.LGF_DIVERGING and r.iterations < 100


def test_bad_arguments_raise(lgf_gpu):
    import torch

    U = gpu(inputs.unit_config((4, 4, 4, 4)))
    with pytest.raises(lgf_gpu.LgfError):
        lgf_gpu.fix(U, -0.08, 1e-15)
    with pytest.raises(lgf_gpu.LgfError):
        lgf_gpu.fix(U, 0.08, 0.0)
    with pytest.raises(ValueError):
        lgf_gpu.fix(U.to(torch.complex64), 0.08, 1e-15)
    with pytest.raises(ValueError):
        lgf_gpu.fix(U.cpu(), 0.08, 1e-15)


def _fp32_lockstep_tol(L):
    """1e-4 for axes up to 128 sites.  The acceleration multiplies each mode,
    and with it the FP32 rounding of the field, by p2max/p2; on the lowest
    mode of an axis of n sites that gain grows as 1/sin^2(pi/n), about 4x
    from 128 to 256 sites, and the bar grows with it."""
    gain = lambda n: 1.0 / np.sin(np.pi / n) ** 2
    return 1e-4 * max(1.0, gain(max(L)) / gain(128))


# the FP32 sweeps' kernels by plane shape: register columns with G accumulated
# in the inverse (x,y) pass (8 and 32 wide), the 4-field LDS kernel for wider
# planes with register spans up to 16 (48 wide) and 32 (Ly = 48 beside Lx = 32);
# the update that shares links through LDS (xy-planes of a multiple of 128
# sites, Lt a multiple of 4): x rows inside a block (32, 16 wide), rows that
# straddle blocks (48 wide), one row per block (128 wide), half a row per
# block (256 wide), Lz = 3, a plane of three blocks (384 sites); the
# (x,t)/(y,z) split with G accumulated in the last (x,t) pass (an extent above
# 32 in (z,t)): the lighter and the wider register tier (Lx = 24), a ragged
# last group of x-sites (27 = 6 x 4 + 3); two t groups per XCD range of
# blocks (16 slices of 4 t)
@pytest.mark.parametrize("L,seed", [((8, 8, 8, 8), 35), ((32, 8, 4, 4), 36), ((48, 4, 4, 6), 37),
                                    ((32, 48, 2, 2), 38), ((27, 9, 4, 6), 39),
                                    ((256, 48, 2, 2), 40), ((16, 16, 3, 4), 41),
                                    ((48, 16, 2, 4), 42), ((128, 4, 2, 4), 43),
                                    ((32, 32, 4, 8), 44), ((16, 4, 4, 48), 45),
                                    ((24, 3, 36, 4), 46), ((27, 4, 6, 36), 47),
                                    ((16, 16, 2, 64), 48), ((32, 12, 2, 4), 49),
                                    ((256, 2, 2, 4), 50)])
def test_mixed_iterate_applies_accumulated_transformation(lgf_gpu, L, seed):
    """FP32-phase lockstep: a mixed-precision context runs FP32 sweeps and
    applies the accumulated transformation to the FP64 input, so the result is
    exactly on the gauge orbit and follows the FP64 trajectory of the oracle to
    FP32 accuracy, over a step far larger than that accuracy."""
    U, _ = inputs.make_config(L, 0.5, seed)
    Ug = gpu(U)
    r = lgf_gpu.iterate(Ug, ALPHA, 6, precision="mixed")
    assert r.iterations == 6 and r.fp32_iterations == 6
    out = cpu(Ug)
    assert abs(oracle.plaquette(out) - oracle.plaquette(U)) < 1e-13
    mu, md = oracle.unitarity(out)
    assert mu < 1e-14 and md < 1e-14
    ref = oracle.iterate(U, ALPHA, 6)
    assert np.max(np.abs(ref - U)) > 0.1
    assert np.max(np.abs(out - ref)) < _fp32_lockstep_tol(L)
    assert r.theta == pytest.approx(oracle.theta(out), rel=1e-12)


def test_fixed_count_runs_every_sweep_even_when_theta_rises(lgf_gpu):
    """lgf_iterate has no stopping test: with alpha above 2/p2max theta
    rises every sweep (a solve would stop as diverging), and all n sweeps are
    still applied, in lockstep with the oracle."""
    U = inputs.abelian_config((8, 8, 8, 8), 1e-4, 39)
    Ug = gpu(U)
    r = lgf_gpu.iterate(Ug, 0.2, 12)
    assert r.status == 0 and r.iterations == 12
    ref = oracle.iterate(U, 0.2, 12)
    assert oracle.theta(ref) > 1e4 * oracle.theta(U)
    assert np.max(np.abs(cpu(Ug) - ref)) < 1e-10
    rs = lgf_gpu.fix(gpu(U), 0.2, 1e-15, max_iter=12)
    assert rs.status == lgf_gpu.LGF_DIVERGING and rs.iterations < 12


# ------------------------------------------- plain (unaccelerated) steepest descent

@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 8, 6, 4)])
def test_plain_steepest_descent_lockstep(lgf_gpu, L):
    U, _ = inputs.make_config(L, 0.5, 60 + sum(L))
    for step in range(3):
        Ug = gpu(U)
        lgf_gpu.iterate(Ug, ALPHA, 1, accelerate=False)
        got = cpu(Ug)
        ref = oracle.fix(U, ALPHA, 0.0, 1, accelerate=False)["U"]
        assert np.max(np.abs(got - ref)) < 1e-13, step
        U = got


def test_plain_steepest_descent_mixed(lgf_gpu):
    """Without the transform the FP32 sweeps accumulate G in a kernel of its own."""
    U, _ = inputs.make_config((4, 4, 4, 4), 0.5, 83)
    ref = oracle.fix(U, ALPHA, 1e-12, 3000, accelerate=False)
    assert ref["status"] == 0
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-12, precision="mixed", max_iter=3000, accelerate=False)
    assert r.status == 0 and 0 < r.fp32_iterations < r.iterations
    _check_solution(cpu(Ug), U, 1e-12, r.F)
    assert abs(r.F - ref["F"]) < 1e-12


def test_plain_steepest_descent_solve(lgf_gpu):
    """Converges to the same kind of fixed point but needs many more sweeps
    than the accelerated method (critical slowing down)."""
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, 61)
    ref = oracle.fix(U, ALPHA, 1e-10, 3000, accelerate=False)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-10, max_iter=3000, accelerate=False)
    assert r.status == 0 and ref["status"] == 0
    assert abs(r.iterations - ref["iterations"]) <= 1
    assert abs(r.F - ref["F"]) < 1e-10
    assert oracle.theta(cpu(Ug)) < 1e-10
    fa = lgf_gpu.fix(gpu(U), ALPHA, 1e-10, max_iter=3000)
    assert r.iterations > 2 * fa.iterations


# ------------------------------------------------------------ exact exponential

@pytest.mark.parametrize("L,accelerate", [((4, 4, 4, 4), True), ((4, 6, 8, 12), True),
                                          ((8, 8, 6, 4), False)])
def test_exact_exp_lockstep(lgf_gpu, L, accelerate):
    U, _ = inputs.make_config(L, 0.5, 70 + sum(L))
    for step in range(3):
        Ug = gpu(U)
        lgf_gpu.iterate(Ug, ALPHA, 1, accelerate=accelerate, exact_exp=True)
        got = cpu(Ug)
        ref = oracle.fix(U, ALPHA, 0.0, 1, accelerate=accelerate, exact_exp=True)["U"]
        assert np.max(np.abs(got - ref)) < 1e-13, step
        U = got


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,seed", [((8, 8, 8, 8), inputs.CONFIG_SEEDS[("8^4", 0.5)]),
                                    ((48, 4, 4, 6), 81), ((16, 4, 4, 48), 82)])
def test_exact_exp_solve_matches_oracle(lgf_gpu, precision, L, seed):
    U, _ = inputs.make_config(L, 0.5, seed)
    ref = oracle.fix(U, ALPHA, 1e-14, 1000, exact_exp=True)
    assert ref["status"] == 0
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000, exact_exp=True)
    assert r.status == 0
    _check_solution(cpu(Ug), U, 1e-14, r.F)
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    first_order = oracle.fix(U, ALPHA, 1e-14, 1000)
    assert abs(r.F - first_order["F"]) < 1e-12


# ------------------------------------------------------------ 18-real link storage

@pytest.mark.parametrize("L,exact", [((4, 4, 4, 4), False), ((4, 6, 8, 12), False),
                                     ((6, 6, 6, 6), True)])
def test_link_format_18_lockstep(lgf_gpu, L, exact):
    U, _ = inputs.make_config(L, 0.5, 80 + sum(L))
    for step in range(3):
        Ug = gpu(U)
        lgf_gpu.iterate(Ug, ALPHA, 1, exact_exp=exact, link_format=18)
        got = cpu(Ug)
        ref = oracle.fix(U, ALPHA, 0.0, 1, exact_exp=exact)["U"]
        assert np.max(np.abs(got - ref)) < 1e-13, step
        U = got


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_link_format_18_solve(lgf_gpu, precision):
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("8^4", 0.5)])
    ref = oracle.fix(U, ALPHA, 1e-14, 1000)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000, link_format=18)
    assert r.status == 0
    _check_solution(cpu(Ug), U, 1e-14, r.F)
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    # the context goes back to 12-real links and still agrees
    Ug = gpu(U)
    r12 = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000)
    assert abs(r12.F - r.F) < 1e-13


# ------------------------------------------------------------ 8-real link storage

def _special_links(L, seed):
    """Links on and near the set where the usual 8-parameter form is singular
    (|U00| = 1): diagonal links, diagonal links with their columns and rows
    permuted (signed to stay in SU(3)), the identity, and Haar links."""
    rng = np.random.default_rng(seed)
    U = inputs.abelian_config(L, 2.0, seed)
    n = U[0].size // 9
    flat = U.reshape(4, n, 3, 3)
    perms = [np.eye(3)[list(p)] * (1 if i % 2 == 0 else -1)  # sign keeps det = +1
             for i, p in enumerate([(0, 1, 2), (1, 0, 2), (1, 2, 0), (0, 2, 1),
                                    (2, 0, 1), (2, 1, 0)])]
    pick = rng.integers(0, 6, size=(4, n))
    for mu in range(4):
        for j in range(n):
            flat[mu, j] = perms[pick[mu, j]] @ flat[mu, j]
    flat[0, ::7] = np.eye(3)
    flat[1, ::5] = inputs.haar_su3(flat[1, ::5].shape[0], rng)
    return U


def test_link_format_8_round_trip(lgf_gpu):
    """n = 0 sweeps pack the caller's links to 8 reals and back: every link is
    reproduced to about 1e-15, on generic links and on the singular set of the
    usual 8-real form (no link is lost)."""
    for U in (_config_haar((4, 6, 4, 8), 5), _special_links((4, 4, 6, 4), 6)):
        Ug = gpu(U)
        r = lgf_gpu.iterate(Ug, ALPHA, 0, link_format=8)
        assert r.iterations == 0
        got = cpu(Ug)
        full = U.copy()
        full[..., 2, :] = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
        assert np.max(np.abs(got - full)) < 1e-14
        mu, md = oracle.unitarity(got)
        assert mu < 1e-14 and md < 1e-14


def _config_haar(L, seed):
    return inputs.make_config(L, 0.5, seed)[0]


@pytest.mark.parametrize("L,exact", [((4, 4, 4, 4), False), ((4, 6, 8, 12), False),
                                     ((6, 6, 6, 6), True), ((9, 4, 6, 4), False)])
def test_link_format_8_lockstep(lgf_gpu, L, exact):
    U, _ = inputs.make_config(L, 0.5, 90 + sum(L))
    for step in range(3):
        Ug = gpu(U)
        lgf_gpu.iterate(Ug, ALPHA, 1, exact_exp=exact, link_format=8)
        got = cpu(Ug)
        ref = oracle.fix(U, ALPHA, 0.0, 1, exact_exp=exact)["U"]
        assert np.max(np.abs(got - ref)) < 1e-13, step
        U = got


def test_link_format_8_lockstep_special_links(lgf_gpu):
    """One sweep from links on the singular set of the usual 8-real form."""
    U = _special_links((4, 4, 6, 4), 7)
    Ug = gpu(U)
    lgf_gpu.iterate(Ug, ALPHA, 1, link_format=8)
    ref = oracle.fix(U, ALPHA, 0.0, 1)["U"]
    assert np.max(np.abs(cpu(Ug) - ref)) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_link_format_8_solve(lgf_gpu, precision):
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("8^4", 0.5)])
    ref = oracle.fix(U, ALPHA, 1e-14, 1000)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000, link_format=8)
    assert r.status == 0
    _check_solution(cpu(Ug), U, 1e-14, r.F)
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    else:
        assert 0 < r.fp32_iterations < r.iterations <= ref["iterations"] + 2


@pytest.mark.parametrize("nreal", [8, 18])
def test_link_format_leaves_per_step_entry_points_12_real(lgf_gpu, nreal):
    """The per-step entry points pack 12-real links into the context's link
    buffer whatever the format set for fix/iterate, so the buffers hold at
    least the 12-real form (an 8-real context once overflowed them)."""
    L = (6, 6, 6, 4)
    U, _ = inputs.make_config(L, 0.5, 95)
    c = lgf_gpu.Context(L, "fp64")
    c.set_link_format(nreal)
    Ug = gpu(U)
    r = c.iterate(Ug, ALPHA, 2)
    assert r.iterations == 2
    V = cpu(Ug)
    D = cpu(c.divergence(Ug))
    assert np.max(np.abs(D - oracle.delta(V))) < 1e-13
    assert c.theta(Ug) == pytest.approx(oracle.theta(V), rel=1e-12)
    assert c.functional(Ug) == pytest.approx(oracle.F(V), abs=1e-14)
    assert c.plaquette(Ug) == pytest.approx(oracle.plaquette(V), abs=1e-13)
    c.close()


def test_link_format_rejects_other_sizes(lgf_gpu):
    U = gpu(inputs.unit_config((4, 4, 4, 4)))
    c = lgf_gpu._ctx(U)
    for bad in (7, 9, 0, 24):
        with pytest.raises(lgf_gpu.LgfError):
            c.set_link_format(bad)
    r = c.fix(U, ALPHA, 1e-15, 10)
    assert r.status == 0 and r.iterations == 0


def test_mixed_fp32_phase_hands_over_when_it_stalls(lgf_gpu):
    """A hand-over threshold below the FP32 rounding floor: the FP32 phase ends
    when theta stops reaching new minima and FP64 finishes the solve."""
    U, _ = inputs.make_config((8, 8, 8, 8), 0.5, 36)
    ref = oracle.fix(U, ALPHA, 1e-14, 1000)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision="mixed", max_iter=1000, theta_switch=1e-30)
    assert r.status == 0
    assert 0 < r.fp32_iterations < 200 and r.iterations > r.fp32_iterations
    _check_solution(cpu(Ug), U, 1e-14, r.F)
    assert abs(r.F - ref["F"]) < 1e-12


# ----------------------------------------------- FP32 Fourier field in FP64 sweeps

# register-column transforms (8^4) and the (x,t)/(y,z) split (an extent above
# 32 in (z,t)) of the FP32 field
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,seed", [((8, 8, 8, 8), inputs.CONFIG_SEEDS[("8^4", 0.5)]),
                                    ((16, 4, 4, 48), 83)])
def test_field32_solve_matches_oracle(lgf_gpu, precision, L, seed):
    """The Fourier field in FP32 changes only the step direction (by ~1e-7,
    relative); the fixed point, the stopping test and the sweep count are
    those of the FP64 method."""
    U, _ = inputs.make_config(L, 0.5, seed)
    ref = oracle.fix(U, ALPHA, 1e-14, 1000)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000, field_bits=32)
    assert r.status == 0
    _check_solution(cpu(Ug), U, 1e-14, r.F)
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1


def test_field32_sweep_is_a_gauge_transformation(lgf_gpu):
    U, _ = inputs.make_config((6, 8, 4, 8), 0.5, 37)
    Ug = gpu(U)
    lgf_gpu.iterate(Ug, ALPHA, 1, field_bits=32)
    out = cpu(Ug)
    ref = oracle.iterate(U, ALPHA, 1)
    assert np.max(np.abs(out - ref)) < 1e-5
    assert abs(oracle.plaquette(out) - oracle.plaquette(U)) < 1e-13
    mu, md = oracle.unitarity(out)
    assert mu < 1e-13 and md < 1e-13
    c = lgf_gpu._ctx(Ug)
    for bad in (16, 0, 128):
        with pytest.raises(lgf_gpu.LgfError):
            c.set_field_precision(bad)
