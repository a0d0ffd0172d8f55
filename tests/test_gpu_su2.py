"""SU(2) on the GPU against the numpy SU(2) oracle (through the C ABI).

Lockstep sweeps compare links entry by entry (1e-13); solves compare the
gauge-invariant results: theta < tol re-measured by the oracle, |F - F_oracle|
<= 1e-12, iterations within one, plaquette drift and unitarity.  The 32^4
reference values in tests/golden/oracle_su2324.json are written by
tests/golden/make_oracle_golden.py from the oracle alone.
"""
import json
import os

import numpy as np
import pytest

import inputs
from oracle import su2

pytestmark = pytest.mark.gpu

ALPHA = 0.08
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_su2324.json")


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("L,accelerate,exact", [
    ((4, 4, 4, 4), True, False),
    ((4, 6, 8, 12), True, False),
    ((6, 6, 6, 6), True, True),
    ((8, 8, 6, 4), False, False),
    ((16, 16, 16, 16), True, False),
])
def test_su2_lockstep(lgf_gpu, L, accelerate, exact):
    U, _ = inputs.make_config_su2(L, 0.5, 90 + sum(L))
    for step in range(3):
        Ug = gpu(U)
        r = lgf_gpu.iterate(Ug, ALPHA, 1, accelerate=accelerate, exact_exp=exact)
        got = cpu(Ug)
        ref = su2.iterate(U, ALPHA, 1, accelerate=accelerate, exact_exp=exact)
        assert np.max(np.abs(got - ref)) < 1e-13, step
        assert r.F == pytest.approx(su2.F(ref), abs=1e-14)
        assert r.theta == pytest.approx(su2.theta(ref), rel=1e-11, abs=1e-28)
        U = got


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("L,seed_key,tol,exact", [
    ((8, 8, 8, 8), ("su2 8^4", 0.5), 1e-13, False),
    ((8, 8, 8, 8), ("su2 8^4", 0.5), 1e-13, True),
    ((16, 16, 16, 16), ("su2 16^4", 0.5), 1e-15, False),
])
def test_su2_solve_matches_oracle(lgf_gpu, L, seed_key, tol, exact, precision):
    U, _ = inputs.make_config_su2(L, seed_key[1], inputs.CONFIG_SEEDS[seed_key])
    ref = su2.fix(U, ALPHA, tol, 1000, exact_exp=exact)
    assert ref["status"] == 0
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, tol, precision=precision, max_iter=1000, exact_exp=exact)
    assert r.status == 0
    out = cpu(Ug)
    assert su2.theta(out) < tol
    assert abs(r.F - ref["F"]) < 1e-12
    assert abs(su2.F(out) - r.F) < 1e-13
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    else:
        assert 0 < r.fp32_iterations < r.iterations
    assert abs(su2.plaquette(out) - su2.plaquette(U)) < 1e-12
    mu, md = su2.unitarity(out)
    assert mu < 1e-13 and md < 1e-13


def test_su2_theta_and_functional(lgf_gpu):
    U, _ = inputs.make_config_su2((8, 6, 4, 8), 0.5, 93)
    Ug = gpu(U)
    assert lgf_gpu.theta(Ug) == pytest.approx(su2.theta(U), rel=1e-12)
    assert lgf_gpu.functional(Ug) == pytest.approx(su2.F(U), abs=1e-14)


def test_su2_converged_input_and_errors(lgf_gpu):
    import torch

    U = gpu(inputs.unit_config_su2((4, 4, 4, 4)))
    r = lgf_gpu.fix(U, ALPHA, 1e-15)
    assert r.status == 0 and r.iterations == 0 and r.F == 1.0 and r.theta == 0.0
    with pytest.raises(lgf_gpu.LgfError):
        lgf_gpu.plaquette(U)
    with pytest.raises(lgf_gpu.LgfError):
        lgf_gpu.fix(U, ALPHA, 1e-15, link_format=18)
    with pytest.raises(ValueError):
        lgf_gpu.fix(U.to(torch.complex64), ALPHA, 1e-15)


def test_su2_mixed_iterate_stays_on_the_orbit(lgf_gpu):
    """FP32 sweeps with the accumulated transformation applied to the FP64
    input: exactly on the gauge orbit, close to the FP64 trajectory."""
    U, _ = inputs.make_config_su2((8, 8, 8, 8), 0.5, 95)
    Ug = gpu(U)
    lgf_gpu.iterate(Ug, ALPHA, 6, precision="mixed")
    out = cpu(Ug)
    assert abs(su2.plaquette(out) - su2.plaquette(U)) < 1e-13
    assert su2.unitarity(out)[0] < 1e-14
    assert np.max(np.abs(out - su2.iterate(U, ALPHA, 6))) < 1e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_su2_solve_32x4(lgf_gpu, precision):
    with open(GOLDEN) as f:
        ref = json.load(f)["runs"][0]
    U, _ = inputs.make_config_su2((32, 32, 32, 32), ref["eps"], ref["seed"])
    assert su2.plaquette(U) == pytest.approx(ref["plaquette_in"], abs=1e-13)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-15, precision=precision, max_iter=2000)
    assert r.status == 0
    out = cpu(Ug)
    del Ug
    assert su2.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    assert abs(su2.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = su2.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_su2_field32_solve(lgf_gpu, precision):
    """FP64 sweeps with the Fourier field in FP32: the FP64 method's result."""
    U, _ = inputs.make_config_su2((8, 8, 8, 8), 0.5, inputs.CONFIG_SEEDS[("su2 8^4", 0.5)])
    ref = su2.fix(U, ALPHA, 1e-14, 1000)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, ALPHA, 1e-14, precision=precision, max_iter=1000, field_bits=32)
    assert r.status == 0
    out = cpu(Ug)
    assert su2.theta(out) < 1e-14
    assert abs(r.F - ref["F"]) < 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    assert abs(su2.plaquette(out) - su2.plaquette(U)) < 1e-12
