"""Long-run energy behaviour of the hot path on one GPU.

Integrates a workload for K steps in FP64 and in FP32C pair arithmetic,
sampling the total energy E and the changeover-weighted energy E_K (the one
the hot path conserves; E also moves when pairs cross the changeover zone
because close encounters are flagged, not resolved) every `every` steps.
The step starts at the workload's dt and is halved until the FP64 run keeps
max |dE_K/E_K| within the bound (at most `halvings` times).  Prints one JSON
line; with --out also writes the sampled curves.

    python -m paper_2601_19654_amd.energy_run --workload c3 --steps 10000
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def run(w, mode, dt, steps, every, nb, resolve=False):
    p = nb.default_params(G=w.G, mode=nb.NB_FP32C if mode == "fp32c" else nb.NB_FP64, drag=int(w.drag),
                          resolve=int(resolve))
    c = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", nbig=w.nbig)
    c.upload(w.m0, w.m, w.x, w.v)
    d0 = c.diagnostics()
    E0, EK0 = d0["E"].copy(), d0["EK"].copy()
    t, dE, dEK, nce, groups = [], [], [], 0, 0
    t0 = time.perf_counter()
    for k in range(0, steps, every):
        st = c.step(dt, min(every, steps - k), allow=(nb.NB_E_CAPACITY, nb.NB_E_KEPLER))
        nce += st["total_nce"]
        groups += st["resolved_groups"]
        d = c.diagnostics()
        t.append((k + min(every, steps - k)) * dt)
        dE.append(float(np.max(np.abs((d["E"] - E0) / E0))))
        dEK.append(float(np.max(np.abs((d["EK"] - EK0) / EK0))))
    wall = time.perf_counter() - t0
    x, v = c.download(nb.NB_DH)
    c.close()
    return {"t": t, "dE": dE, "dEK": dEK, "max_dE": max(dE), "max_dEK": max(dEK),
            "final_dE": dE[-1], "final_dEK": dEK[-1], "flagged_per_step": nce / steps,
            "resolved_groups_per_step": groups / steps,
            "wall_s": round(wall, 3), "x": x, "v": v}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--bound", type=float, default=1e-9)
    ap.add_argument("--halvings", type=int, default=3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--dt", type=float, default=None, help="starting step (default: the workload's)")
    ap.add_argument("--resolve", action="store_true",
                    help="also run the full hybrid method (FP64, encounters resolved on the host)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    from . import nb
    w = workloads.by_name(args.workload)
    dt = args.dt if args.dt else w.dt
    tried = []
    for h in range(args.halvings + 1):
        r64 = run(w, "fp64", dt, args.steps, args.every, nb)
        tried.append({"dt": dt, "max_dEK": r64["max_dEK"], "max_dE": r64["max_dE"]})
        print(f"[energy] fp64 dt={dt}: max|dE_K/E_K| {r64['max_dEK']:.3e}, max|dE/E| {r64['max_dE']:.3e}",
              file=sys.stderr, flush=True)
        if r64["max_dEK"] <= args.bound or h == args.halvings:
            break
        dt *= 0.5
    r32 = run(w, "fp32c", dt, args.steps, args.every, nb)
    pos = float(np.max(np.linalg.norm(r32["x"] - r64["x"], axis=1) / np.linalg.norm(r64["x"], axis=1)))
    out = {"workload": w.name, "steps": args.steps, "dt": dt, "years": args.steps * dt, "bound": args.bound,
           "dt_search": tried,
           "fp64": {k: r64[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK", "flagged_per_step", "wall_s")},
           "fp32c": {k: r32[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK", "flagged_per_step", "wall_s")},
           "fp32c_vs_fp64_max_rel_position_diff_at_end": pos}
    if args.resolve:
        rf = run(w, "fp64", dt, args.steps, args.every, nb, resolve=True)
        print(f"[energy] full method fp64 dt={dt}: max|dE_K/E_K| {rf['max_dEK']:.3e}, max|dE/E| {rf['max_dE']:.3e}",
              file=sys.stderr, flush=True)
        out["fp64_full_method"] = {k: rf[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK",
                                                       "flagged_per_step", "resolved_groups_per_step", "wall_s")}
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": out, "t": r64["t"], "fp64_dE": r64["dE"], "fp64_dEK": r64["dEK"],
                       "fp32c_dE": r32["dE"], "fp32c_dEK": r32["dEK"]}, f)


if __name__ == "__main__":
    main()
