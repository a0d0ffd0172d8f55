"""Benchmark: Fourier-accelerated Landau gauge fixing of a 32^4 SU(3) lattice.

One step = one Fourier-accelerated steepest-descent sweep of the whole
lattice (FFT of the divergence, momentum-space scaling, inverse FFT, gauge
transformation, link update, next divergence, F/theta reductions), FP64.

The headline is the steady-state sweep rate: every lgf_iterate call also packs
the caller's links, computes the first divergence and unpacks the result, so
the bench times iterate(K) and iterate(2K) (medians over repeats, each run
bracketed by device synchronisations) and divides the difference by K; the
per-call costs are reported beside it.

Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--solves R]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "iters/s & time to θ<1e-15, 32^4 SU(3), FP64 vs mixed; % of HBM peak"
HBM_PEAK_GBS = 8000.0
ALPHA = 0.08
TOL = 1e-15
L = (32, 32, 32, 32)
EPS_ALL = (0.6, 0.45, 0.35)
EPS_MAIN = 0.45
REPS = 5  # repeats per timed iterate() length (medians)
BYTES_UPDATE_18 = 4 * 144 * 2 + 128  # update with 18-real links: R+W 4 x 144 B, R+W 64 B
BYTES_UPDATE_8 = 4 * 64 * 2 + 128  # update with 8-real links: R+W 4 x 64 B, R+W 64 B
BYTES_UPDATE_SU2 = 4 * 32 * 2 + 32 * 2  # SU(2) update: R+W 4 links x 32 B, R+W 2 fields
SD_TOL = 1e-10  # plain steepest descent needs thousands of sweeps at 32^4
# algorithmic bytes per site of each sweep kernel: FP64, and the FP32 sweeps
# of a mixed solve, whose last transform pass also does G <- g G (R field 32,
# R+W G 96, the field itself not written back) and whose update forms the
# links from the input copy U0 (R U0 192, R G 48, W field 32).  Where the
# planes of all four fields do not fit one block (fp32_acc_fused), the
# accumulation is a kernel of its own after a plain inverse pass (64 + 32 + 96).
BYTES_PER_SITE = {
    "fp64": {"fft_xy_fwd": 128, "fft_zt": 128, "fft_xy_inv": 128, "update": 896, "finalize": 0},
    "fp32": {"fft_xy_fwd": 64, "fft_zt": 64, "fft_xy_inv": 128, "update": 272, "finalize": 0},
}
BYTES_XY_INV_ACC_SEPARATE = 64 + 32 + 96
# differentiation kernels, algorithmic bytes per site: dF/domega reads the
# divergence of the rotated links (64) and omega (64) and writes the gradient
# (64); dtheta/deps reads the 12-real links (384), Delta (64; neighbours
# reused), eps (4 x 64) and writes the gradient (4 x 64)
BYTES_OMEGA_GRAD = 3 * 64
BYTES_THETA_GRAD = 384 + 64 + 256 + 256

# sources that determine the update kernel's code (for the traffic record)
UPDATE_SOURCES = ("paper_1301_3460_amd/csrc/sweep.hip", "paper_1301_3460_amd/csrc/common.hpp",
                  "paper_1301_3460_amd/csrc/su3.hpp", "paper_1301_3460_amd/csrc/kernels.hpp")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "update_32x4_fp64_traffic.json")


def fp32_acc_fused(L) -> bool:
    """Whether the FP32 sweeps accumulate G inside their last transform pass
    (the library's rule).  With an extent above 32 in (z,t), Lx >= 16 and the
    tiles within LDS, the last pass holds (x,t) planes and fuses when the four
    fields' planes fit 150 KB; otherwise it holds (x,y) planes: a register-
    column plane (both extents up to 32) or four planes within 150 KB."""
    Lx, Ly, Lz, Lt = L
    if Lz > 32 or Lt > 32:
        xt = Lt * (Lx + 1) * 8
        if Lx >= 16 and xt <= 80 * 1024 and Lz * (4 * Ly + 1) * 8 <= 160 * 1024 and Ly * Lz <= 65535:
            return 4 * xt <= 150 * 1024
    if Lx <= 32 and Ly <= 32:
        return 4 * Lx <= 512
    return Ly * (Lx + 1) * 8 <= 160 * 1024 and 4 * Ly * (Lx + 1) * 8 <= 150 * 1024


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha256(paths=UPDATE_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per update launch from the committed rocprofv3 counter record,
    or None when the kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    with open(TRAFFIC_RECORD) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != sources_sha256():
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def cpu_model() -> str:
    """The host CPU's model name (the "Model name" lscpu prints)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed(fn, reps, setup=None):
    """Median wall time of fn() over reps runs, each bracketed by device
    synchronisations (setup(), untimed, runs before each); returns
    (seconds, result of the last run)."""
    import numpy as np
    import torch

    ts, r = [], None
    for _ in range(reps):
        if setup is not None:
            setup()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), r


def steady_sweeps(ctx, U0, work, K, reps=REPS):
    """Steady-state seconds per sweep, (t(2K) - t(K)) / K with t(n) the median
    time of one iterate(n) call, and the per-call cost t(0) (pack, first
    divergence, unpack, status reads).  Every run must apply exactly the n
    sweeps asked for (a fixed count has no stopping test)."""

    def run(n):
        def call():
            r = ctx.iterate(work, ALPHA, n)
            if r.iterations != n:
                raise RuntimeError(f"iterate({n}) applied {r.iterations} sweeps "
                                   f"(status {r.status})")
            return r

        return timed(call, reps, setup=lambda: work.copy_(U0))

    t1, _ = run(K)
    t2, r2 = run(2 * K)
    t0, _ = run(0)
    return {"s_per_sweep": (t2 - t1) / K, "t_K": t1, "t_2K": t2, "t_0": t0, "last": r2}


def solve_timing(ctx, U, work, reps, max_iter=2000):
    t, res = timed(lambda: ctx.fix(work, ALPHA, TOL, max_iter), reps, setup=lambda: work.copy_(U))
    return t, res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--solves", type=int, default=5, help="repeats per time-to-theta solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--no-cpu-solve", action="store_true",
                    help="skip the oracle's full 32^4 solve in the CPU baseline")
    ap.add_argument("--lattice", choices=("32^4", "48^3x96"), default="32^4",
                    help="with --sweeps-only: the lattice whose sweeps are timed and profiled")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 48^3x96 lattice (10.6M sites, beyond the 256 MB cache)")
    ap.add_argument("--sweeps-only", action="store_true",
                    help="only the timed sweeps, the per-kernel timing and one device copy of "
                         "the 32^4 link field (a known-size reference for HBM counters)")
    ap.add_argument("--autograd-only", action="store_true",
                    help="only the forward+backward timing of the differentiable forms")
    ap.add_argument("--link-format", type=int, choices=(8, 12, 18), default=12,
                    help="with --sweeps-only: reals per working link of the timed FP64 sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is not implemented.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import inputs
    import paper_1301_3460_amd as lgf

    torch.cuda.set_device(0)
    lgf.load()

    if args.autograd_only:
        print(json.dumps({"autograd": autograd_variant(lgf, inputs, torch, np)}), flush=True)
        return 0

    Lrun, lat_key = (L, "32^4")
    if args.lattice != "32^4":
        if not args.sweeps_only:
            print("--lattice applies to --sweeps-only runs", file=sys.stderr)
            return 2
        Lrun, lat_key = ((48, 48, 48, 96), "48^3x96")
    V = int(np.prod(Lrun))
    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_324.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            for run in json.load(f)["runs"]:
                golden[run["eps"]] = run
    golden_exp = None
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_324exp.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            golden_exp = json.load(f)["runs"][0]

    golden_su2 = None
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_su2324.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            golden_su2 = json.load(f)["runs"][0]

    def golden_iters_at(tol):
        """Accelerated (oracle) sweeps until theta < tol on the main input."""
        hist = golden.get(EPS_MAIN, {}).get("theta_hist")
        return next((n for n, t in enumerate(hist) if t < tol), None) if hist else None

    # ---- inputs (host generation, not timed)
    configs = {}
    for eps in ((EPS_MAIN,) if args.sweeps_only else EPS_ALL):
        t0 = time.time()
        U, _ = inputs.make_config(Lrun, eps, inputs.CONFIG_SEEDS[(lat_key, eps)])
        configs[eps] = torch.from_numpy(U).to("cuda")
        log(f"generated {lat_key} eps={eps} in {time.time() - t0:.1f} s")
        del U
    U0 = configs[EPS_MAIN]
    work = torch.empty_like(U0)

    ctx64 = lgf.Context(Lrun, "fp64")
    ctx32 = lgf.Context(Lrun, "mixed")
    if args.link_format != 12:
        if not args.sweeps_only:
            print("--link-format applies to --sweeps-only runs", file=sys.stderr)
            return 2
        ctx64.set_link_format(args.link_format)

    # ---- sweep throughput (the headline value), after W warmup sweeps
    work.copy_(U0)
    ctx64.iterate(work, ALPHA, args.warmup)
    ss = steady_sweeps(ctx64, U0, work, args.steps)
    dt_sweep = ss["s_per_sweep"]
    ips = 1.0 / dt_sweep
    overhead = {"per_call_ms": round(1e3 * ss["t_0"], 4),
                "iterate_K_ms": round(1e3 * ss["t_K"], 4),
                "iterate_2K_ms": round(1e3 * ss["t_2K"], 4),
                "single_call_rate": round(args.steps / ss["t_K"], 2)}
    log(f"FP64 sweeps: {1e6 * dt_sweep:.2f} us/sweep -> {ips:.1f} sweeps/s steady state; "
        f"per-call {overhead}")

    # ---- per-kernel durations (HIP events on the library stream)
    prof64 = ctx64.profile(U0, ALPHA, 50)
    prof32 = ctx32.profile(U0, ALPHA, 50)
    per_kernel = {}
    fp32_bytes = dict(BYTES_PER_SITE["fp32"])
    if not fp32_acc_fused(Lrun):
        fp32_bytes["fft_xy_inv"] = BYTES_XY_INV_ACC_SEPARATE
    fp64_bytes = dict(BYTES_PER_SITE["fp64"])
    fp64_bytes["update"] = {12: fp64_bytes["update"], 18: BYTES_UPDATE_18,
                            8: BYTES_UPDATE_8}[args.link_format]
    for name, prof, nbytes in (("fp64", prof64, fp64_bytes), ("fp32", prof32, fp32_bytes)):
        per_kernel[name] = {
            k: {"ms": round(v, 5),
                "GBps": round(nbytes[k] * V / (v * 1e-3) / 1e9, 1) if v > 0 else None}
            for k, v in prof.items()}
    log("per-kernel:", json.dumps(per_kernel))
    upd_ms = prof64["update"]
    achieved = fp64_bytes["update"] * V / (upd_ms * 1e-3) / 1e9

    if args.sweeps_only:
        # reference copy kernel: reads and writes exactly work.numel()*16 bytes
        ref = torch.empty_like(U0)
        torch.cuda.synchronize()
        ref.copy_(U0)
        torch.cuda.synchronize()
        log(f"reference copy: {U0.numel() * 16} bytes read and written")
        print(json.dumps({"value": round(ips, 2), "unit": "iters/s", "per_kernel": per_kernel,
                          "overhead": overhead, "roofline_update_GBps": round(achieved, 1),
                          "sweep_GBps": round(1280 * V * ips / 1e9, 1),
                          "copy_bytes": U0.numel() * 16}), flush=True)
        return 0

    # ---- time to theta < 1e-15, FP64 vs mixed, three disorder levels
    solves = {}
    for eps in EPS_ALL:
        for prec, ctx in (("fp64", ctx64), ("mixed", ctx32)):
            t, res = solve_timing(ctx, configs[eps], work, args.solves)
            entry = {"ms": round(1e3 * t, 3), "iterations": res.iterations,
                     "fp32_iterations": res.fp32_iterations, "status": res.status,
                     "F": res.F, "theta": res.theta}
            if eps in golden:
                entry["dF_vs_oracle"] = abs(res.F - golden[eps]["F"])
                entry["oracle_iterations"] = golden[eps]["iterations"]
            entry["plaquette"] = ctx64.plaquette(work)
            solves[f"eps={eps}/{prec}"] = entry
            log(f"solve eps={eps} {prec}: {entry}")
    t64 = solves[f"eps={EPS_MAIN}/fp64"]["ms"]
    tmx = solves[f"eps={EPS_MAIN}/mixed"]["ms"]

    # ---- variants of the step on the same input: exact exponential; plain
    # steepest descent (no Fourier acceleration) to a looser tolerance
    variants = {}
    for prec, ctx in (("fp64", ctx64), ("mixed", ctx32)):
        ctx.set_exponential(True)
        t, res = solve_timing(ctx, U0, work, args.solves)
        entry = {"ms": round(1e3 * t, 3), "iterations": res.iterations,
                 "fp32_iterations": res.fp32_iterations, "status": res.status, "F": res.F,
                 "theta": res.theta}
        if golden_exp:
            entry["dF_vs_oracle"] = abs(res.F - golden_exp["F"])
            entry["oracle_iterations"] = golden_exp["iterations"]
        if prec == "fp64":
            entry["update_ms"] = round(ctx.profile(U0, ALPHA, 20)["update"], 5)
        ctx.set_exponential(False)
        variants[f"exact_exp/{prec}"] = entry
        log(f"exact exponential {prec}: {entry}")
    # later hand-over points of the mixed solve (FP32 sweeps further down)
    for sw in (1e-9, 1e-10, 1e-11):
        ctx32.set_theta_switch(sw)
        t, res = solve_timing(ctx32, U0, work, args.solves)
        e = {"ms": round(1e3 * t, 3), "iterations": res.iterations,
             "fp32_iterations": res.fp32_iterations, "status": res.status, "F": res.F,
             "theta": res.theta}
        if golden:
            e["dF_vs_oracle"] = abs(res.F - golden[EPS_MAIN]["F"])
        variants[f"mixed_switch_{sw:g}"] = e
        log(f"mixed, switch at {sw:g}: {e}")
    ctx32.set_theta_switch(1e-8)

    # FP64 sweeps with the Fourier field held in FP32
    ctx64.set_field_precision(32)
    ctx32.set_field_precision(32)
    ssf = steady_sweeps(ctx64, U0, work, args.steps)
    proff = ctx64.profile(U0, ALPHA, 20)
    e = {"sweeps_per_s": round(1.0 / ssf["s_per_sweep"], 1),
         "per_kernel_ms": {k: round(v, 5) for k, v in proff.items()}, "bytes_per_site": 1024}
    for prec, ctx in (("fp64", ctx64), ("mixed", ctx32)):
        t, res = solve_timing(ctx, U0, work, args.solves)
        e[f"solve_ms_{prec}"] = round(1e3 * t, 3)
        e[f"iterations_{prec}"] = res.iterations
        if golden:
            e[f"dF_vs_oracle_{prec}"] = abs(res.F - golden[EPS_MAIN]["F"])
    # the fastest combination: mixed, FP32 field, hand-over at 1e-11
    ctx32.set_theta_switch(1e-11)
    t, res = solve_timing(ctx32, U0, work, args.solves)
    ctx32.set_theta_switch(1e-8)
    e["solve_ms_mixed_switch_1e-11"] = round(1e3 * t, 3)
    if golden:
        e["dF_vs_oracle_mixed_switch_1e-11"] = abs(res.F - golden[EPS_MAIN]["F"])
    ctx64.set_field_precision(64)
    ctx32.set_field_precision(64)
    variants["field32"] = e
    log(f"FP32 Fourier field: {e}")

    # 18-real working links (all three rows stored) against the 12-real default
    ctx64.set_link_format(18)
    ss18 = steady_sweeps(ctx64, U0, work, args.steps)
    upd18 = ctx64.profile(U0, ALPHA, 20)["update"]
    t, res = solve_timing(ctx64, U0, work, args.solves)
    ctx64.set_link_format(12)
    variants["link18/fp64"] = {
        "sweeps_per_s": round(1.0 / ss18["s_per_sweep"], 1), "update_ms": round(upd18, 5),
        "update_GBps": round(BYTES_UPDATE_18 * V / (upd18 * 1e-3) / 1e9, 1),
        "update_bytes_per_site": BYTES_UPDATE_18,
        "solve_ms": round(1e3 * t, 3), "iterations": res.iterations,
        "F": res.F, "dF_vs_oracle": abs(res.F - golden[EPS_MAIN]["F"]) if golden else None}
    log(f"18-real links: {variants['link18/fp64']}")
    # the minimal 8-real working links (one third less link traffic, decoding
    # arithmetic instead)
    ctx64.set_link_format(8)
    ss8 = steady_sweeps(ctx64, U0, work, args.steps)
    upd8 = ctx64.profile(U0, ALPHA, 20)["update"]
    t, res = solve_timing(ctx64, U0, work, args.solves)
    ctx64.set_link_format(12)
    variants["link8/fp64"] = {
        "sweeps_per_s": round(1.0 / ss8["s_per_sweep"], 1), "update_ms": round(upd8, 5),
        "update_GBps": round(BYTES_UPDATE_8 * V / (upd8 * 1e-3) / 1e9, 1),
        "update_bytes_per_site": BYTES_UPDATE_8,
        "solve_ms": round(1e3 * t, 3), "iterations": res.iterations,
        "F": res.F, "dF_vs_oracle": abs(res.F - golden[EPS_MAIN]["F"]) if golden else None}
    log(f"8-real links: {variants['link8/fp64']}")
    # SU(2) on the same lattice (N_c = 2; links stored as row 0)
    U2 = inputs.make_config_su2(L, EPS_MAIN, inputs.CONFIG_SEEDS[("su2 32^4", EPS_MAIN)])[0]
    U2 = torch.from_numpy(U2).to("cuda")
    w2 = torch.empty_like(U2)
    c2 = lgf.Context(L, "fp64", nc=2)
    w2.copy_(U2)
    c2.iterate(w2, ALPHA, args.warmup)
    ss2 = steady_sweeps(c2, U2, w2, args.steps)
    prof2 = c2.profile(U2, ALPHA, 20)
    t, res = solve_timing(c2, U2, w2, args.solves)
    entry = {"sweeps_per_s": round(1.0 / ss2["s_per_sweep"], 1),
             "per_kernel_ms": {k: round(v, 5) for k, v in prof2.items()},
             "update_GBps": round(BYTES_UPDATE_SU2 * V / (prof2["update"] * 1e-3) / 1e9, 1),
             "update_bytes_per_site": BYTES_UPDATE_SU2,
             "solve_ms": round(1e3 * t, 3), "iterations": res.iterations,
             "status": res.status, "F": res.F}
    if golden_su2:
        entry["dF_vs_oracle"] = abs(res.F - golden_su2["F"])
        entry["oracle_iterations"] = golden_su2["iterations"]
    variants["su2/fp64"] = entry
    log(f"SU(2): {entry}")
    c2.close()
    c2m = lgf.Context(L, "mixed", nc=2)
    t, res = solve_timing(c2m, U2, w2, args.solves)
    entry = {"solve_ms": round(1e3 * t, 3), "iterations": res.iterations,
             "fp32_iterations": res.fp32_iterations, "status": res.status, "F": res.F}
    if golden_su2:
        entry["dF_vs_oracle"] = abs(res.F - golden_su2["F"])
    variants["su2/mixed"] = entry
    log(f"SU(2) mixed: {entry}")
    c2m.close()
    del U2, w2

    cpu48 = None
    # 48^3 x 96: radix-3 and two-pass transform extents; every working set far
    # beyond the 256 MB Infinity Cache, so HBM rates are not flattered by it
    if not args.no_large:
        L48 = (48, 48, 48, 96)
        V48 = int(np.prod(L48))
        t0 = time.time()
        U48 = torch.from_numpy(
            inputs.make_config(L48, 0.45, inputs.CONFIG_SEEDS[("48^3x96", 0.45)])[0]).to("cuda")
        log(f"generated 48^3x96 in {time.time() - t0:.1f} s")
        w48 = torch.empty_like(U48)
        c48 = lgf.Context(L48, "fp64")
        w48.copy_(U48)
        c48.iterate(w48, ALPHA, 3)
        ss48 = steady_sweeps(c48, U48, w48, 20, reps=3)
        ips48 = 1.0 / ss48["s_per_sweep"]
        prof48 = c48.profile(U48, ALPHA, 5)
        variants["48^3x96/fp64"] = {
            "sweeps_per_s": round(ips48, 2),
            "per_kernel_ms": {k: round(v, 4) for k, v in prof48.items()},
            "update_GBps": round(BYTES_PER_SITE["fp64"]["update"] * V48 /
                                 (prof48["update"] * 1e-3) / 1e9, 1),
            "sweep_GBps": round(1280 * V48 * ips48 / 1e9, 1),
            "per_call_ms": round(1e3 * ss48["t_0"], 3)}
        log(f"48^3x96: {variants['48^3x96/fp64']}")
        g48 = None
        gpath = os.path.join(ROOT, "tests", "golden", "oracle_483x96.json")
        if os.path.exists(gpath):
            with open(gpath) as f:
                g48 = json.load(f)["runs"][0]
        c48m = lgf.Context(L48, "mixed")
        for prec, ctx in (("fp64", c48), ("mixed", c48m)):
            t, res = solve_timing(ctx, U48, w48, 1)
            entry = {"ms": round(1e3 * t, 3),
                     "iterations": res.iterations, "fp32_iterations": res.fp32_iterations,
                     "status": res.status, "F": res.F, "theta": res.theta}
            if g48:
                entry["dF_vs_oracle"] = abs(res.F - g48["F"])
                entry["oracle_iterations"] = g48["iterations"]
            variants[f"48^3x96/solve_{prec}"] = entry
            log(f"48^3x96 solve {prec}: {entry}")
        c48m.close()
        c48.close()
        if not args.no_cpu:
            # the oracle on this host at 48^3 x 96: a bounded sample of sweeps
            import oracle

            oracle.set_threads(len(os.sched_getaffinity(0)))
            Uh48 = U48.cpu().numpy()
            t0 = time.perf_counter()
            oracle.iterate(Uh48, ALPHA, 2)
            c48s = (time.perf_counter() - t0) / 2
            cpu48 = {"sweeps": 2, "s_per_sweep": round(c48s, 3),
                     "gpu_speedup_fp64_sweeps": round(c48s * ips48, 1)}
            log(f"cpu oracle 48^3x96: {cpu48}")
            del Uh48
        del U48, w48
        torch.cuda.empty_cache()

    ctx64.set_acceleration(False)
    t, res = timed(lambda: ctx64.fix(work, ALPHA, SD_TOL, 20000), 1,
                   setup=lambda: work.copy_(U0))
    ctx64.set_acceleration(True)
    variants["plain_sd/fp64"] = {"theta_tol": SD_TOL, "ms": round(1e3 * t, 3),
                                 "iterations": res.iterations, "status": res.status,
                                 "sweeps_per_s": round(res.iterations / t, 1),
                                 "accelerated_iterations_same_tol": golden_iters_at(SD_TOL)}
    log(f"plain steepest descent: {variants['plain_sd/fp64']}")

    # differentiation (forward + backward of the autograd functions)
    variants["autograd"] = autograd_variant(lgf, inputs, torch, np)

    # ---- CPU baseline: the oracle on this host's cores
    cpu = None
    if not args.no_cpu:
        import oracle

        threads = len(os.sched_getaffinity(0))
        oracle.set_threads(threads)
        Uh = configs[EPS_MAIN].cpu().numpy()
        n = args.cpu_sweeps
        t0 = time.perf_counter()
        oracle.iterate(Uh, ALPHA, n)
        cdt = time.perf_counter() - t0
        cpu = {"value": round(n / cdt, 4), "unit": "iters/s", "cores": oracle.get_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{n} FP64 sweeps of the 32^4 eps={EPS_MAIN} configuration "
                         f"({cdt:.1f} s, plain C/OpenMP oracle, "
                         f"{oracle.get_threads()} threads = the process's CPU affinity)"}
        log(f"cpu oracle sweeps: {cpu}")
        if not args.no_cpu_solve:
            t0 = time.perf_counter()
            ref = oracle.fix(Uh, ALPHA, TOL, 2000)
            cs = time.perf_counter() - t0
            cpu["time_to_theta_s"] = round(cs, 3)
            cpu["time_to_theta_iterations"] = ref["iterations"]
            cpu["time_to_theta_F"] = ref["F"]
            cpu["gpu_speedup_time_to_theta_fp64"] = round(1e3 * cs / t64, 1)
            log(f"cpu oracle solve: {cs:.1f} s, {ref['iterations']} sweeps")
        if cpu48 is not None:
            cpu["sample_48x3x96"] = cpu48

    out = {
        "metric": METRIC,
        "value": round(ips, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt_sweep, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "SU(3) 32^4, FP64 Fourier-accelerated steepest descent, "
                               f"alpha={ALPHA}, eps={EPS_MAIN} links + Haar gauge transformation",
                   "lattice": list(L), "sites": V},
        "timing": "steady state: (t(iterate 2K) - t(iterate K)) / K, medians of "
                  f"{REPS} runs each; per-call costs in 'overhead'",
        "overhead": overhead,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "k_update<double> (update + next divergence)",
                     "bytes_per_site": BYTES_PER_SITE["fp64"]["update"]},
        "sweep_roofline_frac": round(1280 * V * ips / 1e9 / HBM_PEAK_GBS, 4),
        "cpu_baseline": cpu,
        "time_to_theta_ms": {"fp64": t64, "mixed": tmx, "speedup_mixed": round(t64 / tmx, 3)},
        "solves": solves,
        "variants": variants,
        "per_kernel": per_kernel,
    }
    print(json.dumps(out), flush=True)
    return 0


def autograd_variant(lgf, inputs, torch, np):
    """Forward and forward+backward rates of LandauF (dF/domega) and
    LandauTheta (dtheta/deps) on the differentiation workloads (4^4 and 16^4,
    eps = 0.5 links + Haar gauge transformation) and on 32^4."""
    out = {}
    for key, L, seed, reps in (("4^4", (4, 4, 4, 4), inputs.CONFIG_SEEDS[("4^4", 0.5)], 50),
                               ("16^4", (16, 16, 16, 16), inputs.CONFIG_SEEDS[("16^4", 0.5)], 20),
                               ("32^4", (32, 32, 32, 32), 3205, 10)):
        V = int(np.prod(L))
        U = torch.from_numpy(inputs.make_config(L, 0.5, seed)[0]).to("cuda")
        om0 = torch.from_numpy(inputs.random_omega(L, 0.3, seed + 1)).to("cuda")
        om = om0.clone().requires_grad_(True)
        eps = torch.zeros((4,) + inputs.site_shape(L) + (8,), dtype=torch.float64,
                          device="cuda", requires_grad=True)

        def fwd_F():
            with torch.no_grad():
                return lgf.LandauF.apply(om, U)

        def fwdbwd_F():
            om.grad = None
            F = lgf.LandauF.apply(om, U)
            F.backward()
            return F

        def fwd_T():
            with torch.no_grad():
                return lgf.LandauTheta.apply(eps, U)

        def fwdbwd_T():
            eps.grad = None
            th = lgf.LandauTheta.apply(eps, U)
            th.backward()
            return th

        fwdbwd_F()
        fwdbwd_T()
        tF, _ = timed(fwd_F, reps)
        tFB, _ = timed(fwdbwd_F, reps)
        tT, _ = timed(fwd_T, reps)
        tTB, _ = timed(fwdbwd_T, reps)
        out[key] = {"sites": V,
                    "F_forward_ms": round(1e3 * tF, 4), "F_fwd_bwd_ms": round(1e3 * tFB, 4),
                    "F_fwd_bwd_per_s": round(1.0 / tFB, 1),
                    "theta_forward_ms": round(1e3 * tT, 4),
                    "theta_fwd_bwd_ms": round(1e3 * tTB, 4),
                    "theta_fwd_bwd_per_s": round(1.0 / tTB, 1),
                    "omega_grad_bytes_per_site": BYTES_OMEGA_GRAD,
                    "theta_grad_bytes_per_site": BYTES_THETA_GRAD}
        log(f"autograd {key}: {out[key]}")
        del U, om, om0, eps
    return out


if __name__ == "__main__":
    sys.exit(main())
