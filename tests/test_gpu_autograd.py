"""Differentiation (FP64): dF/domega and dtheta/deps against finite differences
and the oracle; the torch.autograd.Function wrappers."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("L,sigma", [((4, 4, 4, 4), 0.0), ((4, 4, 4, 4), 0.5),
                                     ((16, 16, 16, 16), 0.5), ((4, 6, 8, 4), 1.0)])
def test_omega_gradient_matches_oracle(lgf_gpu, L, sigma):
    U, _ = inputs.make_config(L, 0.5, 40 + sum(L))
    om = inputs.random_omega(L, sigma, 41)
    F, grad = lgf_gpu.functional_omega_grad(gpu(U), gpu(om))
    Fr, gr = oracle.functional_omega_grad(U, om)
    assert F == pytest.approx(Fr, abs=1e-14)
    assert np.max(np.abs(cpu(grad) - gr)) < 1e-12 * max(1e-30, np.max(np.abs(gr))) + 1e-18
    assert lgf_gpu.functional_omega(gpu(U), gpu(om)) == pytest.approx(Fr, abs=1e-14)


def _local_F(U, om, site, L):
    """The terms of F_U[exp(i omega T)] that involve g at `site` (x, y, z, t),
    from the definition, evaluated in numpy with scipy's expm."""
    import scipy.linalg

    Lx, Ly, Lz, Lt = L
    ext = (Lx, Ly, Lz, Lt)

    def g_at(c):
        x, y, z, t = c
        return scipy.linalg.expm(0.5j * np.tensordot(om[t, z, y, x], inputs.GELL_MANN, axes=(0, 0)))

    def link(mu, c):
        x, y, z, t = c
        return U[mu, t, z, y, x]

    def shift(c, mu, d):
        c = list(c)
        c[mu] = (c[mu] + d) % ext[mu]
        return tuple(c)

    acc = 0.0
    g0 = g_at(site)
    for mu in range(4):
        up, dn = shift(site, mu, +1), shift(site, mu, -1)
        acc += np.trace(g0 @ link(mu, site) @ g_at(up).conj().T).real
        acc += np.trace(g_at(dn) @ link(mu, dn) @ g0.conj().T).real
    return acc / (4 * 3 * np.prod(L))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (16, 16, 16, 16)])
def test_omega_gradient_finite_differences(lgf_gpu, L):
    """Central differences (step 1e-6) at 64 random (site, generator) pairs.
    Only the terms of F that touch the perturbed site change, so they are
    differenced alone (the full sum would bury the change in rounding)."""
    V = int(np.prod(L))
    U, _ = inputs.make_config(L, 0.5, 42)
    om = inputs.random_omega(L, 0.5, 43)
    _, grad = lgf_gpu.functional_omega_grad(gpu(U), gpu(om))
    grad = cpu(grad)
    rng = np.random.default_rng(44)
    h = 1e-6
    errs = []
    for _ in range(64):
        site = tuple(int(rng.integers(n)) for n in L)
        a = int(rng.integers(8))
        x, y, z, t = site
        p = om.copy(); p[t, z, y, x, a] += h
        m = om.copy(); m[t, z, y, x, a] -= h
        fd = (_local_F(U, p, site, L) - _local_F(U, m, site, L)) / (2 * h)
        errs.append(abs(fd - grad[t, z, y, x, a]))
    assert max(errs) < 1e-6 * np.max(np.abs(grad))


def test_theta_gradient_matches_oracle(lgf_gpu):
    L = (4, 6, 4, 8)
    U, _ = inputs.make_config(L, 0.5, 45)
    th, grad = lgf_gpu.theta_grad(gpu(U))
    thr, gr = oracle.theta_grad(U)
    assert th == pytest.approx(thr, rel=1e-13)
    assert np.max(np.abs(cpu(grad) - gr)) < 1e-12 * np.max(np.abs(gr))


def test_theta_gradient_at_nonzero_eps(lgf_gpu):
    """theta(exp(i eps T) U): the library's value equals the oracle's theta of the
    links rotated on the host, and its gradient matches central differences."""
    L = (4, 4, 4, 4)
    V = int(np.prod(L))
    U, _ = inputs.make_config(L, 0.5, 46)
    eps = 0.3 * np.random.default_rng(47).standard_normal((4,) + inputs.site_shape(L) + (8,))
    E = np.array([oracle.expm_su3(w) for w in eps.reshape(-1, 8)]).reshape(U.shape)
    Urot = E @ U
    Ug, eg = gpu(U), gpu(eps)
    th, grad = lgf_gpu.theta_grad(Ug, eg)
    assert th == pytest.approx(oracle.theta(Urot), rel=1e-13)
    grad = cpu(grad).reshape(4, V, 8)
    rng = np.random.default_rng(48)
    h = 1e-6
    errs = []
    flat = eps.reshape(4, V, 8)
    for _ in range(32):
        mu, s, a = int(rng.integers(4)), int(rng.integers(V)), int(rng.integers(8))
        p = flat.copy(); p[mu, s, a] += h
        m = flat.copy(); m[mu, s, a] -= h
        fp = lgf_gpu.theta_grad(Ug, gpu(p.reshape(eps.shape)))[0]
        fm = lgf_gpu.theta_grad(Ug, gpu(m.reshape(eps.shape)))[0]
        errs.append(abs((fp - fm) / (2 * h) - grad[mu, s, a]))
    assert max(errs) < 1e-6 * np.max(np.abs(grad))


def test_autograd_functions(lgf_gpu):
    import torch

    L = (4, 4, 4, 4)
    U, _ = inputs.make_config(L, 0.5, 49)
    Ug = gpu(U)
    om = gpu(inputs.random_omega(L, 0.3, 50)).requires_grad_(True)
    F = lgf_gpu.LandauF.apply(om, Ug)
    (2.0 * F).backward()
    _, ref = oracle.functional_omega_grad(U, cpu(om))
    assert np.max(np.abs(cpu(om.grad) - 2.0 * ref)) < 1e-12 * np.max(np.abs(ref))
    eps = torch.zeros((4,) + inputs.site_shape(L) + (8,), dtype=torch.float64,
                      device="cuda", requires_grad=True)
    th = lgf_gpu.LandauTheta.apply(eps, Ug)
    th.backward()
    _, gref = oracle.theta_grad(U)
    assert np.max(np.abs(cpu(eps.grad) - gref)) < 1e-12 * np.max(np.abs(gref))


def test_forward_launches_no_gradient_kernel(lgf_gpu, monkeypatch):
    """The gradient entry points (the only callers of the gradient kernels) run
    in backward, never in forward, with or without grad mode."""
    import torch

    L = (4, 4, 4, 4)
    U, _ = inputs.make_config(L, 0.5, 51)
    Ug = gpu(U)
    om = gpu(inputs.random_omega(L, 0.3, 52)).requires_grad_(True)
    eps = torch.zeros((4,) + inputs.site_shape(L) + (8,), dtype=torch.float64,
                      device="cuda", requires_grad=True)
    calls = []
    Ctx = lgf_gpu.Context
    orig_f, orig_t = Ctx.functional_omega_grad, Ctx.theta_grad

    def spy_f(self, *a, **k):
        calls.append("omega_grad")
        return orig_f(self, *a, **k)

    def spy_t(self, U, eps=None, need_grad=True):
        if need_grad:
            calls.append("theta_grad")
        return orig_t(self, U, eps, need_grad)

    monkeypatch.setattr(Ctx, "functional_omega_grad", spy_f)
    monkeypatch.setattr(Ctx, "theta_grad", spy_t)
    with torch.no_grad():
        F0 = lgf_gpu.LandauF.apply(om, Ug)
        th0 = lgf_gpu.LandauTheta.apply(eps, Ug)
    F = lgf_gpu.LandauF.apply(om, Ug)
    th = lgf_gpu.LandauTheta.apply(eps, Ug)
    assert calls == []
    assert abs(float(F0) - oracle.functional_omega(U, cpu(om))) < 1e-13
    assert float(F) == float(F0) and float(th) == float(th0)
    (F + th).backward()
    assert sorted(calls) == ["omega_grad", "theta_grad"]
    _, ref = oracle.functional_omega_grad(U, cpu(om))
    assert np.max(np.abs(cpu(om.grad) - ref)) < 1e-12 * np.max(np.abs(ref))
