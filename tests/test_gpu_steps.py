"""Step-by-step parity of the HIP sweep against the FP64 oracle (GPU).

Every check compares the library, called through its C ABI, element by element
with the oracle on the same seeded inputs.  Shapes span several tiles, ragged
tails (xy-planes not a multiple of the (z,t) tile width, volumes not a
multiple of the site block), every extent 2^a 3^b up to 256 (odd ones
included) and each transform scheme: register columns, whole planes in LDS,
one-axis passes, two-pass extents.
Bars: 1e-13 absolute on O(1) quantities (FP64 rounding of a few hundred
operations; the oracle and the kernels order their sums differently).
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

SHAPES = [
    (4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8), (4, 6, 8, 12), (2, 3, 4, 6), (3, 4, 2, 4),
    (12, 12, 12, 12), (48, 4, 4, 6), (4, 48, 6, 4), (4, 4, 48, 8), (4, 6, 4, 96),
    (8, 4, 64, 4), (4, 2, 4, 128), (16, 16, 16, 16),
    # extents of 24 or 32 beside one above 32 (the wider-register FFT instances)
    (32, 48, 2, 2), (2, 2, 32, 64), (2, 4, 96, 24),
    # 32-wide x rows with even and odd Ly
    (32, 6, 4, 2), (32, 24, 2, 2), (32, 2, 3, 4), (32, 3, 2, 4),
    # the other extents 2^a 3^b up to 256 on each axis: register columns (9, 18,
    # 27; odd extents, p2max below 16), whole-plane and one-axis transforms
    # (36 ... 256, two passes N1 x N2 with spans up to 16 and up to 32)
    (9, 4, 3, 2), (4, 9, 2, 6), (18, 18, 3, 4), (27, 2, 9, 4), (2, 3, 27, 27), (3, 2, 9, 18),
    (36, 4, 2, 4), (4, 54, 2, 2), (2, 2, 72, 3), (2, 3, 2, 81), (108, 2, 3, 2),
    (144, 4, 2, 2), (4, 2, 162, 2), (2, 2, 2, 192), (216, 2, 2, 3), (2, 243, 2, 2),
    (256, 2, 2, 2), (2, 2, 4, 256), (27, 27, 3, 2),
    # (x,y) planes beyond one LDS tile: a separate x pass and y pass
    (256, 48, 2, 2), (243, 81, 2, 2),
    # several slices of 4 t per XCD range of site blocks (walked inside z)
    (8, 8, 4, 64), (16, 4, 2, 96),
]


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def cpu(t):
    return t.detach().cpu().numpy()


def _config(L, seed, eps=0.5):
    U, _ = inputs.make_config(L, eps, seed)
    return U


@pytest.mark.parametrize("L", SHAPES)
def test_divergence_theta_F(lgf_gpu, L):
    U = _config(L, 100 + sum(L))
    Ug = gpu(U)
    D = cpu(lgf_gpu.divergence(Ug))
    Dref = oracle.delta(U)
    assert np.max(np.abs(D - Dref)) < 1e-13
    th = lgf_gpu.theta(Ug)
    assert th == pytest.approx(oracle.theta(U), rel=1e-13)
    assert lgf_gpu.functional(Ug) == pytest.approx(oracle.F(U), abs=1e-14)


@pytest.mark.parametrize("L", SHAPES)
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft4d(lgf_gpu, L, sign):
    rng = np.random.default_rng(7 + sum(L))
    shp = (4,) + inputs.site_shape(L)
    a = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    got = cpu(lgf_gpu.fft4d(gpu(a), sign))
    ref = oracle.fft4d(np.moveaxis(a, 0, -1), sign)
    ref = np.moveaxis(ref, -1, 0)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) < 1e-13 * scale
    if sign < 0:  # an independent library as a second reference
        ref2 = np.fft.fftn(a, axes=(1, 2, 3, 4))
        assert np.max(np.abs(got - ref2)) < 1e-13 * scale


# FP64 32 x 32 register-column passes that take two tiles per block (enough
# planes or xy-sites for two blocks per compute unit at half the tile count):
# both (x,y) and (z,t) at 32^4, the (z,t) pass alone (64-wide planes in LDS).
TWO_TILE_SHAPES = [(32, 32, 32, 32), (64, 32, 32, 32)]


# FP64 (x,t) planes and (y,z) tiles of two x-sites (an extent above 32 in
# (z,t), Lx >= 16): t two-pass, z two-pass, both, a ragged last x-group
# (odd Lx), both tile kinds with two-pass extents, the wider register tier
# (162 = 9 x 18), a (y,z) tile beyond 80 KB (one 1024-thread block per
# compute unit), 32 x 32 xy-planes (where the (x,t) planes replace the
# two-tile (x,y) pass)
TILE2_SHAPES = [(16, 4, 4, 48), (18, 3, 36, 4), (27, 4, 6, 36), (16, 6, 48, 96),
                (48, 4, 4, 96), (36, 9, 54, 2), (16, 2, 2, 162), (16, 54, 54, 2),
                (32, 32, 16, 64)]


@pytest.mark.parametrize("L", TILE2_SHAPES)
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft4d_tile2(lgf_gpu, L, sign):
    test_fft4d(lgf_gpu, L, sign)


@pytest.mark.parametrize("L", TILE2_SHAPES)
def test_fourier_accelerate_tile2(lgf_gpu, L):
    test_fourier_accelerate(lgf_gpu, L)


@pytest.mark.parametrize("L", TILE2_SHAPES)
def test_lockstep_sweeps_tile2(lgf_gpu, L):
    test_lockstep_sweeps(lgf_gpu, L)


@pytest.mark.parametrize("L", TWO_TILE_SHAPES)
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft4d_two_tile(lgf_gpu, L, sign):
    test_fft4d(lgf_gpu, L, sign)


@pytest.mark.parametrize("L", TWO_TILE_SHAPES)
def test_fourier_accelerate_two_tile(lgf_gpu, L):
    test_fourier_accelerate(lgf_gpu, L)


@pytest.mark.parametrize("L", SHAPES)
def test_fourier_accelerate(lgf_gpu, L):
    U = _config(L, 200 + sum(L))
    D = oracle.delta(U)
    got = cpu(lgf_gpu.fourier_accelerate(gpu(D)))
    ref = oracle.fourier_accelerate(D)
    assert np.max(np.abs(got - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_link_storage_round_trip(lgf_gpu):
    """n = 0 sweeps: pack to 12 reals and back.  Rows 0,1 are bit-exact; row 2
    is rebuilt as conj(row0 x row1)."""
    U = _config((4, 6, 4, 8), 5)
    Ug = gpu(U)
    r = lgf_gpu.iterate(Ug, 0.08, 0)
    assert r.iterations == 0
    out = cpu(Ug)
    assert np.array_equal(out[..., :2, :], U[..., :2, :])
    rebuilt = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.max(np.abs(out[..., 2, :] - rebuilt)) < 1e-15
    # and within the input's own distance from SU(3) of its stored row 2
    mu, _ = oracle.unitarity(U)
    assert np.max(np.abs(out[..., 2, :] - U[..., 2, :])) < 2 * mu + 1e-15


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 8, 8, 8), (4, 6, 8, 12), (2, 3, 4, 6),
                               (48, 4, 4, 6), (4, 6, 4, 96), (12, 12, 12, 12),
                               (16, 16, 16, 16), (32, 8, 8, 6),
                               (9, 9, 9, 9), (18, 27, 4, 6), (36, 4, 6, 72), (256, 4, 4, 4),
                               (4, 4, 144, 4), (6, 6, 6, 192), (256, 48, 2, 2)])
def test_lockstep_sweeps(lgf_gpu, L):
    """Feed the GPU state to the oracle, take one sweep on each side, compare
    the links; repeat.  Also checks F and theta reported for the new links."""
    U = _config(L, 300 + sum(L))
    for step in range(6):
        Ug = gpu(U)
        r = lgf_gpu.iterate(Ug, 0.08, 1)
        got = cpu(Ug)
        ref = oracle.iterate(U, 0.08, 1)
        assert r.iterations == 1
        assert np.max(np.abs(got - ref)) < 1e-13, step
        assert r.theta == pytest.approx(oracle.theta(got), rel=1e-12, abs=1e-28)
        assert r.F == pytest.approx(oracle.F(got), abs=1e-14)
        U = got


def test_multi_sweep_trajectory(lgf_gpu):
    U = _config((8, 8, 8, 8), 11)
    Ug = gpu(U)
    lgf_gpu.iterate(Ug, 0.08, 10)
    ref = oracle.iterate(U, 0.08, 10)
    assert np.max(np.abs(cpu(Ug) - ref)) < 1e-12


def test_plaquette_and_functional_with_g(lgf_gpu):
    L = (4, 6, 8, 4)
    U = _config(L, 12)
    g = inputs.haar_su3(int(np.prod(L)), np.random.default_rng(13)).reshape(
        inputs.site_shape(L) + (3, 3))
    Ug = gpu(U)
    assert lgf_gpu.plaquette(Ug) == pytest.approx(oracle.plaquette(U), abs=1e-14)
    assert lgf_gpu.functional(Ug, gpu(g)) == pytest.approx(oracle.functional(U, g), abs=1e-14)


def test_sweeps_are_deterministic(lgf_gpu):
    U = _config((8, 8, 8, 8), 14)
    a, b = gpu(U), gpu(U)
    ra = lgf_gpu.iterate(a, 0.08, 5)
    rb = lgf_gpu.iterate(b, 0.08, 5)
    assert np.array_equal(cpu(a), cpu(b))
    assert ra.F == rb.F and ra.theta == rb.theta


def test_resume_is_bitwise(lgf_gpu):
    """k + m sweeps equal k sweeps, a copy to the host and back, then m."""
    U = _config((4, 4, 6, 8), 15)
    a = gpu(U)
    lgf_gpu.iterate(a, 0.08, 7)
    b = gpu(U)
    lgf_gpu.iterate(b, 0.08, 3)
    b = gpu(cpu(b))
    lgf_gpu.iterate(b, 0.08, 4)
    assert np.array_equal(cpu(a), cpu(b))
