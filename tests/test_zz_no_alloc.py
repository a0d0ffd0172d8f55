"""The allocation-free entry point lgf_measure_noalloc, called through the C
ABI, against the context entry points it mirrors (lgf_functional with
g == NULL, and lgf_theta): F_U[1] of the paper's display equation and the
stopping quantity theta of its comparison runs."""
import ctypes

import numpy as np
import pytest

import inputs


def _call(lib, U, out, stream):
    Lt, Lz, Ly, Lx = (int(v) for v in U.shape[1:5])
    arr = (ctypes.c_int * 4)(Lx, Ly, Lz, Lt)
    return lib.lgf_measure_noalloc(ctypes.byref(arr), ctypes.c_void_p(U.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.gpu
def test_noalloc_matches_context_entry_points_on_two_calls(lgf_gpu):
    import torch

    lib = lgf_gpu.load()
    stream = torch.cuda.Stream()
    # the second call has the smaller lattice: nothing of the first call's
    # partial sums may leak into it
    for L, eps, seed in (((16, 8, 8, 12), 0.5, 9101), ((4, 4, 6, 4), 0.45, 9102)):
        print(f"noalloc: lattice {L} seed {seed}", flush=True)
        U = torch.from_numpy(inputs.make_config(L, eps, seed)[0]).to("cuda")
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        rc = _call(lib, U, out, stream)
        assert rc == 0, lib.lgf_last_error(None)
        stream.synchronize()
        F, th = (float(v) for v in out.cpu())
        ctx = lgf_gpu.Context(L, "fp64")
        F_ref, th_ref = ctx.functional(U), ctx.theta(U)
        ctx.close()
        print(f"noalloc: F {F!r} vs {F_ref!r}; theta {th!r} vs {th_ref!r}", flush=True)
        assert np.isfinite(F) and np.isfinite(th) and th > 0
        assert abs(F - F_ref) <= 1e-15
        assert abs(th - th_ref) <= 1e-14 * th_ref


@pytest.mark.gpu
def test_noalloc_python_wrapper_and_size_limit(lgf_gpu):
    import torch

    U = torch.from_numpy(inputs.make_config((8, 8, 8, 8), 0.5, 9103)[0]).to("cuda")
    out = lgf_gpu.measure_noalloc(U)
    torch.cuda.synchronize()
    ctx = lgf_gpu.Context((8, 8, 8, 8), "fp64")
    assert abs(float(out[0]) - ctx.functional(U)) <= 1e-15
    assert abs(float(out[1]) - ctx.theta(U)) <= 1e-14 * ctx.theta(U)
    ctx.close()
    # beyond the fixed scratch: rejected before anything is enqueued
    lib = lgf_gpu.load()
    arr = (ctypes.c_int * 4)(128, 128, 64, 64)  # 2^26 sites
    rc = lib.lgf_measure_noalloc(ctypes.byref(arr), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), None)
    assert rc == lgf_gpu.LGF_ERR_ARG
