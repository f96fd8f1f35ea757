#!/usr/bin/env python3
"""Benchmark of the hybrid-step hot path on one MI355X.

Workload: 16384 equal-mass planetesimals (10 Earth masses in total) in a
0.5-5 AU annulus around a solar-mass star, e ~ Rayleigh(0.01),
i ~ Rayleigh(0.005), dt = 0.0021875 yr (0.0175 yr halved until an FP64 run of
1e4 steps keeps the changeover-weighted energy within 1e-9); synthetic, seeded.

A step is one whole hybrid step K S D C S F K (kick, stellar drift, Kepler
drift, encounter check, stellar drift, critical radii + force, kick) of that
system, replayed from captured HIP graphs built before the timed region; the
state stays resident in HBM.  Prints one JSON line: Gpair/s = N(N-1) x steps /
device time of the timed steps (HIP events on the context's stream; FP32C pair
arithmetic as the headline, FP64 alongside), steps/s, the median of 5 further
timed calls, the energy error of each line over 1e4 steps (E_K for the hot
path, E for the full method with encounters resolved on the host), the force
kernel against its roofline, and the CPU oracle (median of 5 steps, serial and
OpenMP).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/sec (Gpair/s) + steps/sec at N=16384, FP32-comp vs FP64"
FLOPS_PER_PAIR = 20          # direct-summation convention (see the design notes)
PEAK_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}   # MI355X vector FP64 / FP32 (published)
KERNEL_SRC = os.path.join(ROOT, "paper_2601_19654_amd", "csrc", "nb_kernels.hip")


def force_kernel_source() -> str:
    """Source text the force kernels are built from: the shared helpers, the
    force section and its launcher (a change elsewhere leaves it alone)."""
    src = open(KERNEL_SRC).read()
    helpers = re.search(r"// small helpers\n.*?(?=\n// -{20,}\n)", src, re.S)
    force = re.search(r"// Interaction force .*?(?=\n// -{20,}\n// Encounter check)", src, re.S)
    launch = re.search(r"hipError_t launch_force\(.*?\n}\n", src, re.S)
    if not (helpers and force and launch):
        raise RuntimeError("force kernel source sections not found")
    return helpers.group(0) + force.group(0) + launch.group(0)


def kernel_hash() -> str:
    return hashlib.sha256(force_kernel_source().encode()).hexdigest()[:16]


def traffic_from_profiles(mode: str, workload: str = "c3"):
    """HBM bytes per force launch from a committed rocprofv3 PMC summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"force_{mode}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]{16})", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def _dev_ms(ctx, torch, fn):
    """Device milliseconds of fn() between two HIP events on the context's stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    out = fn()
    e1.record(ctx.stream)
    e1.synchronize()
    return e0.elapsed_time(e1), out


def run_mode(w, mode: str, steps: int, warmup: int, torch, nb, resolve: bool = False,
             energy_steps: int = 0, overrides=None):
    p = nb.default_params(G=w.G, mode=nb.NB_FP32C if mode == "fp32c" else nb.NB_FP64, drag=int(w.drag),
                          resolve=int(resolve), **(overrides or {}))
    ctx = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", nbig=w.nbig)
    tiles = {"source": ctx.tiles, "force_r": ctx.params.force_r, "force_jchunk": ctx.params.force_jchunk,
             "enc_jchunk": ctx.params.enc_jchunk, **ctx.choices()}
    ctx.upload(w.m0, w.m, w.x, w.v)
    pairs = w.pairs()
    allow = (nb.NB_E_CAPACITY, nb.NB_E_KEPLER)
    # warm-up steps (untimed), then the captured runs the timed call replays
    # are built before the timed region (nb_prepare runs no step)
    if warmup > 0:
        ctx.step_async(w.dt, warmup)
    ctx.prepare(w.dt, steps)
    # timed region: exactly `steps` steps of one nb_step call, device time from
    # HIP events on the context's stream, host wall time beside it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms, stats = _dev_ms(ctx, torch, lambda: ctx.step(w.dt, steps, allow=allow))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # replay protocol: 3 warm-up replays of the same call, then the median of 5
    for _ in range(3):
        ctx.step_async(w.dt, steps)
    reps = sorted(_dev_ms(ctx, torch, lambda: ctx.step_async(w.dt, steps))[0] for _ in range(5))
    # per-kernel timing with HIP events on the context's stream (after the steps:
    # the force at the current state, the check on the last step's drift)
    force_ms = ctx.time_kernel(nb.NB_K_FORCE, reps=100)
    enc_ms = ctx.time_kernel(nb.NB_K_ENCOUNTER, reps=20) if not resolve else None
    a_gpu = ctx.accel()
    x, v = ctx.download(nb.NB_DH)
    ctx.close()
    out = {
        "wall_s": wall, "device_ms": dev_ms, "ms_per_step": dev_ms / steps,
        "wall_ms_per_step": 1e3 * wall / steps,
        "replay_median_ms_per_step": reps[2] / steps,
        "replay_ms_per_step": [round(r / steps, 5) for r in reps],
        "gpair_s": pairs * steps / (dev_ms * 1e-3) / 1e9, "steps_per_s": steps / (dev_ms * 1e-3),
        "force_ms": force_ms, "encounter_ms": enc_ms, "stats": stats,
        "a": a_gpu, "Q": x, "tiles": tiles,
    }
    if energy_steps > 0:
        out["energy"] = energy_run(w, mode, energy_steps, nb, resolve)
    return out


def energy_run(w, mode, steps, nb, resolve, every=100, bound=1e-9):
    """Relative errors of E and E_K over `steps` steps from the upload state,
    sampled every `every` steps (FP64 diagnostics on the device)."""
    p = nb.default_params(G=w.G, mode=nb.NB_FP32C if mode == "fp32c" else nb.NB_FP64, drag=int(w.drag),
                          resolve=int(resolve))
    c = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", nbig=w.nbig)
    c.upload(w.m0, w.m, w.x, w.v)
    d0 = c.diagnostics()
    dE = dEK = 0.0
    for k in range(0, steps, every):
        c.step(w.dt, min(every, steps - k), allow=(nb.NB_E_CAPACITY, nb.NB_E_KEPLER))
        d = c.diagnostics()
        dE = max(dE, float(np.max(np.abs((d["E"] - d0["E"]) / d0["E"]))))
        dEK = max(dEK, float(np.max(np.abs((d["EK"] - d0["EK"]) / d0["EK"]))))
    c.close()
    return {"steps": steps, "dt": w.dt, "max_rel_dE": dE, "max_rel_dEK": dEK, "bound": bound,
            "meets_dE": dE <= bound, "meets_dEK": dEK <= bound,
            "conserved": "E (whole Hamiltonian, encounters resolved)" if resolve
            else "E_K (changeover-weighted; flagged encounters are not resolved on the hot path)"}


KERNEL_SUFFIX = {1: "", 2: "_sym", 3: "_few"}


def roofline(mode, pairs, force_ms, workload="c3", force_algo=1):
    """Algorithmic flops (20 per ordered pair interaction, N_s (N_s - 1) or
    N_s nbig_s per system) over the measured force-kernel duration.  The
    symmetric kernel evaluates each unordered pair once for both bodies, so it
    delivers the same interactions with half the pair evaluations."""
    flops = FLOPS_PER_PAIR * pairs
    achieved = flops / (force_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[mode]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic_from_profiles(mode, workload),
            "kernel": f"k_force{'32c' if mode == 'fp32c' else '64'}{KERNEL_SUFFIX.get(force_algo, '')}",
            "kernel_ms": round(force_ms, 4), "flops_per_launch": flops,
            "flop_convention": f"{FLOPS_PER_PAIR} flops per ordered pair interaction"
                               + (" (each unordered pair evaluated once)" if force_algo == 2 else "")}


def accel_error(w, a_gpu, Q, sample=64, seed=1):
    """Max |a_gpu - a_oracle| / A_i over a sample of targets of the largest
    system (CPU oracle, A_i = sum_j G m_j / r_ij^2)."""
    import oracle
    s = int(np.argmax(np.diff(w.off)))
    lo, hi = int(w.off[s]), int(w.off[s + 1])
    m, Qs = w.m[lo:hi], Q[lo:hi]
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(hi - lo, min(sample, hi - lo), replace=False))
    rc = oracle.rcrit(w.m0[s], m, Qs)
    ref = oracle.force_subset(m, Qs, rc, w.G, idx)
    A = np.empty(len(idx))
    for k, i in enumerate(idx):
        d = Qs - Qs[i]
        r2 = np.einsum("jk,jk->j", d, d)
        r2[i] = np.inf
        A[k] = np.sum(w.G * m / r2)
    return float(np.max(np.max(np.abs(a_gpu[lo:hi][idx] - ref), axis=1) / A))


def cpu_baseline_sampled(w, max_pairs):
    """A single system too large for a full oracle step: time the oracle's force
    sums and encounter scans for a sample of bodies plus every body's drift,
    and scale to one full step."""
    import oracle
    oracle.build(force=False)
    n = w.ntot
    k = max(16, int(max_pairs // n))
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(n, min(k, n), replace=False))
    Q, V = oracle.helio_to_dh(w.m0[0], w.m, w.x, w.v)
    rc = oracle.rcrit(w.m0[0], w.m, Q)
    t0 = time.perf_counter()
    oracle.force_subset(w.m, Q, rc, w.G, idx)
    t_force = (time.perf_counter() - t0) * n / len(idx)
    t0 = time.perf_counter()
    Q1, V1, _ = oracle.drift(w.G * w.m0[0], w.dt, Q, V)
    t_drift = time.perf_counter() - t0
    ks = idx[: max(8, len(idx) // 2)]
    t0 = time.perf_counter()
    for i in ks:
        oracle.pair_scan(w.dt, Q, V, Q1, V1, rc, int(i))
    t_enc = (time.perf_counter() - t0) * n / len(ks) / 2      # each pair once
    step = t_force + t_drift + t_enc
    return {"value": round(w.pairs() / step / 1e9, 5), "unit": "Gpair/s", "cores": 1, "kind": "oracle",
            "sample": f"force sums of {len(idx)} targets, encounter scans of {len(ks)} bodies and the "
                      f"drift of all {n} bodies (FP64, serial), scaled to one full step = {step:.1f} s",
            "steps_per_s": round(1.0 / step, 6)}


def _omp_threads():
    """Threads the OpenMP build of the oracle runs with (its runtime's own count)."""
    import ctypes
    import oracle
    oracle.lib(threads=True)
    try:
        return int(ctypes.CDLL(oracle._LIB_OMP).omp_get_max_threads())
    except (OSError, AttributeError):
        return os.cpu_count() or 1


def cpu_baseline(w, max_pairs=4e8, steps=5):
    """Full hybrid steps of the same workload by the CPU oracle: the median of
    `steps` timed steps on 1 thread, and beside it the median of the same steps
    by the OpenMP build of the oracle (bit-identical results), on as many whole
    systems as fit about max_pairs pair interactions."""
    import oracle
    import workloads as W
    oracle.build(force=False)
    if w.nsys == 1 and w.pairs() > max_pairs:
        return cpu_baseline_sampled(w, max_pairs / 8)
    sizes = np.diff(w.off)
    keep, tot = [], 0
    nbig = sizes if w.nbig is None else np.asarray(w.nbig)
    for s in range(w.nsys):
        p = int(nbig[s]) * (int(sizes[s]) - 1)
        if keep and tot + p > max_pairs:
            break
        keep.append(s)
        tot += p
    lo, hi = int(w.off[keep[0]]), int(w.off[keep[-1] + 1])
    sub = W.Workload(w.name, (w.off[keep[0]:keep[-1] + 2] - lo).astype(np.int32), w.m0[keep],
                     w.m[lo:hi], w.x[lo:hi], w.v[lo:hi], w.dt, 1, G=w.G, drag=w.drag,
                     nbig=None if w.nbig is None else np.asarray(w.nbig)[keep])

    def median_step(threads):
        st = oracle.State.from_workload(sub, threads=threads)   # includes the first force evaluation
        ts = []
        for _ in range(steps):
            t0 = time.perf_counter()
            st.step(w.dt)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), st

    t1, st1 = median_step(False)
    tn, stn = median_step(True)
    same = bool(np.array_equal(st1.Q, stn.Q) and np.array_equal(st1.V, stn.V))
    nthr = _omp_threads()
    what = f"{len(keep)} of {w.nsys} systems" if w.nsys > 1 else f"the N={w.ntot} system"
    return {"value": round(sub.pairs() / t1 / 1e9, 5), "unit": "Gpair/s", "cores": 1, "kind": "oracle",
            "sample": f"median of {steps} full hybrid steps of {what} (FP64, serial): {t1:.3f} s per step",
            "steps_per_s": round(1.0 / t1, 5) if w.nsys == 1 else None,
            "oracle_omp": {"value": round(sub.pairs() / tn / 1e9, 5), "unit": "Gpair/s", "cores": nthr,
                           "kind": "oracle-OMP", "s_per_step": round(tn, 4),
                           "sample": f"median of {steps} steps of the OpenMP build ({nthr} threads; "
                                     f"targets, bodies and encounter rows split over threads)",
                           "bit_identical_to_serial": same}}


def mode_line(w, rr, steps, pairs):
    """The per-mode summary of a run_mode result."""
    out = {"gpair_s": round(rr["gpair_s"], 3), "steps_per_s": round(rr["steps_per_s"], 3),
           "ms_per_step": round(rr["ms_per_step"], 5),
           "wall_ms_per_step": round(rr["wall_ms_per_step"], 5),
           "replay_median_ms_per_step": round(rr["replay_median_ms_per_step"], 5),
           "replay_ms_per_step": rr["replay_ms_per_step"],
           "force_kernel_ms": round(rr["force_ms"], 5),
           "encounter_kernel_ms": None if rr["encounter_ms"] is None else round(rr["encounter_ms"], 5),
           "force_gpair_s": round(pairs / (rr["force_ms"] * 1e-3) / 1e9, 2),
           "tiles": rr["tiles"],
           "nce_per_step": rr["stats"]["total_nce"] / steps,
           "resolved_groups_per_step": rr["stats"]["resolved_groups"] / steps,
           "accel_err_vs_oracle": accel_error(w, rr["a"], rr["Q"])}
    if "energy" in rr:
        out["energy"] = rr["energy"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--modes", default="fp32c,fp64")
    ap.add_argument("--workload", default="c3", help="c1..c5 or bigsmall (the headline is c3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--resolve", action="store_true",
                    help="full hybrid method on the headline lines: resolve close encounters on "
                         "the host every step")
    ap.add_argument("--energy-steps", type=int, default=None,
                    help="steps of the energy-error run of every line (default: 10000 for c3, "
                         "else 0 = none)")
    ap.add_argument("--no-full-method", action="store_true",
                    help="skip the full-method lines (c3 adds them by default)")
    ap.add_argument("--force-g", type=int, default=0,
                    help="super-tile width of the symmetric force (0: tuned or automatic)")
    ap.add_argument("--force-algo", type=int, default=0,
                    help="force algorithm (0: tuned or automatic; 2: symmetric tile pairs; 4: "
                         "symmetric over the radial order, FP32C)")
    ap.add_argument("--force-r", type=int, default=0,
                    help="target tiles of 64 force_r bodies (0: tuned or automatic)")
    ap.add_argument("--enc-algo", type=int, default=0,
                    help="encounter check algorithm (0: tuned or automatic; 4: inside the force pass)")
    ap.add_argument("--log", default=None,
                    help="also append the result line to this JSON-lines run log")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2601_19654_amd import nb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nb.lib()

    w = workloads.by_name(args.workload)
    energy_steps = args.energy_steps if args.energy_steps is not None else (10000 if w.name == "c3" else 0)
    full_lines = w.name == "c3" and not args.resolve and not args.no_full_method
    modes = [m for m in args.modes.split(",") if m]
    res, full = {}, {}
    for mode in modes:
        print(f"[bench] {w.name} mode {mode}: ntot={w.ntot}, warmup {args.warmup}, steps {args.steps}",
              file=sys.stderr, flush=True)
        over = {k: v for k, v in (("force_g", args.force_g), ("enc_algo", args.enc_algo),
                                  ("force_algo", args.force_algo), ("force_r", args.force_r)) if v}
        res[mode] = run_mode(w, mode, args.steps, args.warmup, torch, nb, resolve=args.resolve,
                             energy_steps=energy_steps, overrides=over)
        enc = res[mode]["encounter_ms"]
        print(f"[bench] mode {mode}: {res[mode]['ms_per_step']:.4f} ms/step (replay median "
              f"{res[mode]['replay_median_ms_per_step']:.4f}, wall {res[mode]['wall_ms_per_step']:.4f}), "
              f"force {res[mode]['force_ms']:.4f} ms, encounter {enc if enc is None else round(enc, 4)} ms"
              + (f", energy {res[mode]['energy']}" if "energy" in res[mode] else ""),
              file=sys.stderr, flush=True)
        if full_lines:
            full[mode] = run_mode(w, mode, args.steps, args.warmup, torch, nb, resolve=True,
                                  energy_steps=energy_steps)
            print(f"[bench] full method {mode}: {full[mode]['ms_per_step']:.4f} ms/step"
                  + (f", energy {full[mode]['energy']}" if "energy" in full[mode] else ""),
                  file=sys.stderr, flush=True)
    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    head = "fp32c" if "fp32c" in res else modes[0]
    r = res[head]
    n = w.ntot
    pairs = w.pairs()
    desc = {"c1": "c1: star + 100 planetesimals, m 1e-10..1e-8 log-uniform, a 1-3 AU, dt 0.05 yr",
            "c2": "c2: star + Jupiter at 5.2 AU + 1000 planetesimals of 1e-9, a 2-10 AU, gas drag, dt 0.1 yr",
            "c3": f"c3: star + {n} equal-mass planetesimals (10 Earth masses), "
                  "a 0.5-5 AU, e,i Rayleigh 0.01/0.005, dt 0.0021875 yr (energy-bounded step)",
            "c4": f"c4: {w.nsys} independent systems, N_s uniform 200..4000 (sum {n}), c1 distributions, dt 0.05 yr",
            "c5": f"c5: star + {n} planetesimals of 1e-11 in a 0.9-1.1 AU ring, dt 0.04 yr",
            "bigsmall": f"bigsmall: star + {int(w.nbig[0]) if w.nbig is not None else n} Mars-mass embryos "
                        f"(the only gravity sources) + {n - int(w.nbig[0]) if w.nbig is not None else 0} "
                        "massless planetesimals, a 1-5 AU, dt 0.05 yr"}[args.workload]
    if args.resolve:
        desc += "; full hybrid method (close encounters resolved by Bulirsch-Stoer on the host)"
    out = {
        "metric": METRIC, "value": round(r["gpair_s"], 3), "unit": "Gpair/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_bodies": n, "n_systems": w.nsys, "pairs_per_step": pairs,
                   "mode": head, "tiles": r["tiles"], "parallelism": "single GPU"},
        "steps_per_s": round(r["steps_per_s"], 3),
        "timing": "value and ms_per_step: device time (HIP events on the context's stream) of the "
                  "one timed nb_step call of exactly `steps` steps, its captured runs built "
                  "beforehand; wall_ms_per_step: host time of that call; replay_median_ms_per_step: "
                  "median of 5 further timed calls after 3 warm-up calls",
    }
    for mode, rr in res.items():
        out[mode] = mode_line(w, rr, args.steps, pairs)
    if full:
        out["full_method"] = {mode: mode_line(w, rr, args.steps, pairs) for mode, rr in full.items()}
    out["roofline"] = roofline(head, pairs, r["force_ms"], args.workload, r["tiles"]["force_algo"])
    if "fp64" in res and head != "fp64":
        out["roofline_fp64"] = roofline("fp64", pairs, res["fp64"]["force_ms"], args.workload,
                                        res["fp64"]["tiles"]["force_algo"])
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(w)
    out["kernel_source_sha256_16"] = kernel_hash()
    print(json.dumps(out), flush=True)
    if args.log:
        with open(args.log, "a") as f:
            f.write(json.dumps({"kind": "bench", "time": time.strftime("%Y-%m-%dT%H:%M:%S"), **out}) + "\n")


if __name__ == "__main__":
    main()
