"""Write oracle reference values for the full-size solves.

Calls only ``oracle`` (the plain FP64 CPU implementation) and ``inputs`` (the
seeded generators).  Output: ``tests/golden/oracle_<name>.json`` holding, per
disorder level, the seed, the iteration count, F and theta of the solved
links, the plaquette before and after, and the per-iteration F/theta history.
Nothing here comes from the GPU library.

    python tests/golden/make_oracle_golden.py 32^4
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402
from oracle import su2  # noqa: E402

WORKLOADS = {
    "32^4": {"L": (32, 32, 32, 32), "eps": [0.6, 0.45, 0.35], "alpha": 0.08, "tol": 1e-15},
    "8^4": {"L": (8, 8, 8, 8), "eps": [0.5], "alpha": 0.08, "tol": 1e-12},
    "48^3x96": {"L": (48, 48, 48, 96), "eps": [0.45], "alpha": 0.08, "tol": 1e-15},
    # extents 36 and 72 (two-pass 6x6 and 8x9 transforms) and odd extents
    # (27 = 3^3, p2max below 16)
    "36^3x72": {"L": (36, 36, 36, 72), "eps": [0.45], "alpha": 0.08, "tol": 1e-15},
    "27^4": {"L": (27, 27, 27, 27), "eps": [0.45], "alpha": 0.08, "tol": 1e-15},
    # the same 32^4 input, solved with the exactly exponentiated step
    "32^4-exp": {"L": (32, 32, 32, 32), "eps": [0.45], "alpha": 0.08, "tol": 1e-15,
                 "seeds": "32^4", "exact_exp": True},
    # SU(2) (the numpy SU(2) oracle)
    "su2 32^4": {"L": (32, 32, 32, 32), "eps": [0.45], "alpha": 0.08, "tol": 1e-15,
                 "group": "su2"},
}


def main(name: str) -> None:
    w = WORKLOADS[name]
    exact = w.get("exact_exp", False)
    out = {"workload": name, "L": w["L"], "alpha": w["alpha"], "tol": w["tol"],
           "exact_exp": exact, "threads": oracle.get_threads(), "runs": []}
    for eps in w["eps"]:
        seed = inputs.CONFIG_SEEDS[(w.get("seeds", name), eps)]
        is_su2 = w.get("group") == "su2"
        make = inputs.make_config_su2 if is_su2 else inputs.make_config
        orc = su2 if is_su2 else oracle
        U, _ = make(w["L"], eps, seed)
        P0 = orc.plaquette(U)
        t0 = time.time()
        r = orc.fix(U, w["alpha"], w["tol"], 2000, exact_exp=exact)
        dt = time.time() - t0
        mu, md = orc.unitarity(r["U"])
        run = {"eps": eps, "seed": seed, "status": r["status"], "iterations": r["iterations"],
               "F": r["F"], "theta": r["theta"], "plaquette_in": P0,
               "plaquette_out": orc.plaquette(r["U"]), "unitarity": mu, "det": md,
               "F_hist": list(r["F_hist"]), "theta_hist": list(r["theta_hist"]),
               "seconds": dt}
        print(f"{name} eps={eps}: {r['iterations']} it, F={r['F']:.15f}, theta={r['theta']:.3e}, "
              f"{dt:.1f} s", flush=True)
        out["runs"].append(run)
        del U, r
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"oracle_{name.replace('^', '').replace('-', '').replace(' ', '')}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "32^4")
