"""Long-run energy behaviour of the hot path on one GPU.

Integrates a workload for K steps in FP64 and in FP32C pair arithmetic,
sampling the total energy E and the changeover-weighted energy E_K (the one
the hot path conserves; E also moves when pairs cross the changeover zone
because close encounters are flagged, not resolved) every `every` steps.
The step starts at the workload's dt and is halved until the FP64 run keeps
max |dE_K/E_K| within the bound (at most `halvings` times).  Prints one JSON
line; with --out also writes the sampled curves, with --log appends a JSON-lines
run log (a header per run, then one record per sample).

    python -m paper_2601_19654_amd.energy_run --workload c3 --steps 10000
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


class RunLog:
    """JSON lines of one run: a header (workload, seed recipe, dt, mode, tiles),
    then one record per sample (time, E, E_K, L, P per system, the interval's
    flagged pairs, largest per-step count, list overflows, failed Kepler solves,
    changeover pair evaluations, resolved groups, wall time per step)."""

    def __init__(self, path):
        self.f = open(path, "a") if path else None

    def write(self, rec):
        if self.f:
            self.f.write(json.dumps(rec) + "\n")
            self.f.flush()

    def close(self):
        if self.f:
            self.f.close()


def run(w, mode, dt, steps, every, nb, resolve=False, log=None):
    p = nb.default_params(G=w.G, mode=nb.NB_FP32C if mode == "fp32c" else nb.NB_FP64, drag=int(w.drag),
                          resolve=int(resolve))
    c = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", nbig=w.nbig)
    c.upload(w.m0, w.m, w.x, w.v)
    d0 = c.diagnostics()
    E0, EK0 = d0["E"].copy(), d0["EK"].copy()
    if log:
        log.write({"kind": "header", "workload": w.name, "seed": "SeedSequence(20260119, spawn_key=(cfg, s))",
                   "n_bodies": int(w.ntot), "n_systems": int(w.nsys), "dt": dt, "steps": steps,
                   "every": every, "mode": mode, "resolve": bool(resolve), "tiles": c.tiles,
                   "params": {k: getattr(c.params, k) for k in ("force_r", "force_g", "force_algo",
                                                                "enc_algo", "step_algo")},
                   "choices": c.choices(), "E0": E0.tolist(), "EK0": EK0.tolist()})
    t, dE, dEK, nce, groups = [], [], [], 0, 0
    t0 = time.perf_counter()
    for k in range(0, steps, every):
        k1 = min(every, steps - k)
        ts = time.perf_counter()
        st = c.step(dt, k1, allow=(nb.NB_E_CAPACITY, nb.NB_E_KEPLER))
        ms = (time.perf_counter() - ts) * 1e3 / k1
        nce += st["total_nce"]
        groups += st["resolved_groups"]
        d = c.diagnostics()
        t.append((k + k1) * dt)
        dE.append(float(np.max(np.abs((d["E"] - E0) / E0))))
        dEK.append(float(np.max(np.abs((d["EK"] - EK0) / EK0))))
        if log:
            log.write({"kind": "sample", "step": k + k1, "t": (k + k1) * dt, "E": d["E"].tolist(),
                       "EK": d["EK"].tolist(), "L": d["L"].tolist(), "P": d["P"].tolist(),
                       "max_rel_dE": dE[-1], "max_rel_dEK": dEK[-1], "nce": st["total_nce"],
                       "max_nce": st["max_nce"], "overflow_steps": st["overflow_steps"],
                       "kepler_fail": st["kepler_fail"], "near_pairs": st["near_pairs"],
                       "resolved_groups": st["resolved_groups"], "max_group": st["max_group"],
                       "wall_ms_per_step": round(ms, 5)})
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
    ap.add_argument("--log", default=None, help="append the runs' JSON lines (header + samples) here")
    args = ap.parse_args()
    log = RunLog(args.log)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    from . import nb
    w = workloads.by_name(args.workload)
    dt = args.dt if args.dt else w.dt
    tried = []
    for h in range(args.halvings + 1):
        r64 = run(w, "fp64", dt, args.steps, args.every, nb, log=log)
        tried.append({"dt": dt, "max_dEK": r64["max_dEK"], "max_dE": r64["max_dE"]})
        print(f"[energy] fp64 dt={dt}: max|dE_K/E_K| {r64['max_dEK']:.3e}, max|dE/E| {r64['max_dE']:.3e}",
              file=sys.stderr, flush=True)
        if r64["max_dEK"] <= args.bound or h == args.halvings:
            break
        dt *= 0.5
    r32 = run(w, "fp32c", dt, args.steps, args.every, nb, log=log)
    pos = float(np.max(np.linalg.norm(r32["x"] - r64["x"], axis=1) / np.linalg.norm(r64["x"], axis=1)))
    out = {"workload": w.name, "steps": args.steps, "dt": dt, "years": args.steps * dt, "bound": args.bound,
           "dt_search": tried,
           "fp64": {k: r64[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK", "flagged_per_step", "wall_s")},
           "fp32c": {k: r32[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK", "flagged_per_step", "wall_s")},
           "fp32c_vs_fp64_max_rel_position_diff_at_end": pos}
    if args.resolve:
        rf = run(w, "fp64", dt, args.steps, args.every, nb, resolve=True, log=log)
        print(f"[energy] full method fp64 dt={dt}: max|dE_K/E_K| {rf['max_dEK']:.3e}, max|dE/E| {rf['max_dE']:.3e}",
              file=sys.stderr, flush=True)
        out["fp64_full_method"] = {k: rf[k] for k in ("max_dE", "max_dEK", "final_dE", "final_dEK",
                                                       "flagged_per_step", "resolved_groups_per_step", "wall_s")}
    print(json.dumps(out), flush=True)
    log.write({"kind": "summary", **out})
    log.close()
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": out, "t": r64["t"], "fp64_dE": r64["dE"], "fp64_dEK": r64["dEK"],
                       "fp32c_dE": r32["dE"], "fp32c_dEK": r32["dEK"]}, f)


if __name__ == "__main__":
    main()
