"""Full-size parity at the paper's 32^4 shape (GPU).

The reference values in tests/golden/oracle_324.json were written by
tests/golden/make_oracle_golden.py, which calls only the CPU oracle and the
input generator (about 100 s per solve on 8 cores).  Here the GPU solves the
same seeded inputs, FP64 and mixed precision, and the oracle re-measures the
returned links: theta < 1e-15, |F - F_oracle| <= 1e-12, plaquette drift
<= 1e-12, unitarity <= 1e-13.  One sweep is also compared link by link.
"""
import json
import os

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

L = (32, 32, 32, 32)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_324.json")


def _golden():
    with open(GOLDEN) as f:
        return {r["eps"]: r for r in json.load(f)["runs"]}


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def configs():
    return {}


def _config(configs, eps):
    if eps not in configs:
        configs.clear()  # keep host memory bounded: one 32^4 field at a time
        configs[eps] = inputs.make_config(L, eps, inputs.CONFIG_SEEDS[("32^4", eps)])[0]
    return configs[eps]


@pytest.mark.parametrize("eps", [0.6, 0.45, 0.35])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_32x4(lgf_gpu, configs, eps, precision):
    ref = _golden()[eps]
    U = _config(configs, eps)
    assert oracle.plaquette(U) == pytest.approx(ref["plaquette_in"], abs=1e-13)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, precision=precision, max_iter=2000)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(oracle.F(out) - ref["F"]) <= 1e-12
    assert abs(oracle.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    else:
        assert 0 < r.fp32_iterations < r.iterations
        assert r.iterations <= ref["iterations"] + 2


def test_lockstep_sweep_32x4(lgf_gpu, configs):
    U = _config(configs, 0.45)
    Ug = gpu(U)
    r = lgf_gpu.iterate(Ug, 0.08, 1)
    got = Ug.cpu().numpy()
    ref = oracle.iterate(U, 0.08, 1)
    assert np.max(np.abs(got - ref)) < 1e-13
    assert r.theta == pytest.approx(_golden()[0.45]["theta_hist"][1], rel=1e-11)
    assert r.F == pytest.approx(_golden()[0.45]["F_hist"][1], abs=1e-14)
    # the FP32 sweep of a mixed solve (G accumulated in the inverse (x,y)
    # pass, links formed from the input copy) follows it to FP32 accuracy
    Ug.copy_(gpu(U))
    r = lgf_gpu.iterate(Ug, 0.08, 1, precision="mixed")
    got = Ug.cpu().numpy()
    del Ug
    assert r.fp32_iterations == 1
    assert np.max(np.abs(got - ref)) < 1e-5
    assert r.theta == pytest.approx(_golden()[0.45]["theta_hist"][1], rel=1e-4)


GOLDEN_EXP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "oracle_324exp.json")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_32x4_exact_exp(lgf_gpu, configs, precision):
    """The exactly exponentiated step at 32^4 (oracle run with the same flag)."""
    with open(GOLDEN_EXP) as f:
        ref = json.load(f)["runs"][0]
    U = _config(configs, ref["eps"])
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, precision=precision, max_iter=2000, exact_exp=True)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(oracle.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1


def test_solve_32x4_link_format_18(lgf_gpu, configs):
    """All three rows stored (no rebuild): the same solve as the 12-real form."""
    ref = _golden()[0.45]
    U = _config(configs, 0.45)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, max_iter=2000, link_format=18)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(r.iterations - ref["iterations"]) <= 1
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13


def test_solve_32x4_link_format_8(lgf_gpu, configs):
    """The minimal 8-real working links: the same solve as the 12-real form."""
    ref = _golden()[0.45]
    U = _config(configs, 0.45)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, max_iter=2000, link_format=8)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(r.iterations - ref["iterations"]) <= 1
    assert abs(oracle.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_32x4_field32(lgf_gpu, configs, precision):
    """FP64 sweeps with the Fourier field in FP32: the FP64 method's result."""
    ref = _golden()[0.45]
    U = _config(configs, 0.45)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, precision=precision, max_iter=2000, field_bits=32)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13


def test_lockstep_sweep_32x4_exact_exp(lgf_gpu, configs):
    with open(GOLDEN_EXP) as f:
        ref = json.load(f)["runs"][0]
    U = _config(configs, ref["eps"])
    Ug = gpu(U)
    r = lgf_gpu.iterate(Ug, 0.08, 2, exact_exp=True)
    del Ug
    assert r.theta == pytest.approx(ref["theta_hist"][2], rel=1e-11)
    assert r.F == pytest.approx(ref["F_hist"][2], abs=1e-14)


GOLDEN48 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_483x96.json")
L48 = (48, 48, 48, 96)


@pytest.fixture(scope="module")
def config48():
    return inputs.make_config(L48, 0.45, inputs.CONFIG_SEEDS[("48^3x96", 0.45)])[0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_48x3x96(lgf_gpu, config48, precision):
    """10.6M sites: radix-3 and two-pass transform extents at scale."""
    with open(GOLDEN48) as f:
        ref = json.load(f)["runs"][0]
    U = config48
    assert oracle.plaquette(U) == pytest.approx(ref["plaquette_in"], abs=1e-13)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, precision=precision, max_iter=2000)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(oracle.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1


# Extents beyond the powers of two and 48/96: 36 = 6x6 and 72 = 8x9 two-pass
# transforms (36^3 x 72, 3.4M sites), and odd extents 27 = 3^3 with p2max
# below 16 (27^4).  Reference values from tests/golden/make_oracle_golden.py.
OTHER = {"27^4": ((27, 27, 27, 27), "oracle_274.json"),
         "36^3x72": ((36, 36, 36, 72), "oracle_363x72.json")}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(OTHER))
def test_solve_other_extents(lgf_gpu, name, precision):
    L, fname = OTHER[name]
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", fname)) as f:
        ref = json.load(f)["runs"][0]
    print(f"solve {name} {precision}", flush=True)
    U = inputs.make_config(L, ref["eps"], inputs.CONFIG_SEEDS[(name, ref["eps"])])[0]
    assert oracle.plaquette(U) == pytest.approx(ref["plaquette_in"], abs=1e-13)
    Ug = gpu(U)
    r = lgf_gpu.fix(Ug, 0.08, 1e-15, precision=precision, max_iter=2000)
    assert r.status == 0
    out = Ug.cpu().numpy()
    del Ug
    assert oracle.theta(out) < 1e-15
    assert abs(r.F - ref["F"]) <= 1e-12
    assert abs(oracle.F(out) - ref["F"]) <= 1e-12
    assert abs(oracle.plaquette(out) - ref["plaquette_in"]) <= 1e-12
    mu, md = oracle.unitarity(out)
    assert mu <= 1e-13 and md <= 1e-13
    if precision == "fp64":
        assert abs(r.iterations - ref["iterations"]) <= 1
    else:
        assert 0 < r.fp32_iterations < r.iterations <= ref["iterations"] + 2
