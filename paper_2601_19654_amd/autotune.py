"""Tile-size search for the pair kernels, cached per (GPU arch, mode, size class).

For a given batch of systems it times, with HIP events on the context's stream
(nb_time_kernel), the whole force evaluation (force kernel plus the sum of its
split partials) over targets-per-lane x sources-per-work-item candidates and the encounter kernel over sources-per-work-item candidates, and
stores the fastest choice in ``tuning.json`` (with every candidate's time) under
``<arch>/<mode>/n<max system size, next power of two>/s<systems, next power of two>``,
and the chosen fields in ``tuning.tsv``, the table the library itself reads
(``nb_params.autotune_path``) whenever the caller leaves the tile fields at 0.

    python -m paper_2601_19654_amd.autotune --workloads c1,c2,c3,c4,c5
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(PKG, "tuning.json")

FORCE_R = (1, 2, 4)
FORCE_J = (256, 512, 1024, 2048, 4096)
FORCE_G = (1, 2, 4)          # super-tile widths of the symmetric force
ENC_J = (256, 512, 1024, 2048, 4096)


def _pow2(n: int) -> int:
    p = 1
    while p < n:
        p <<= 1
    return p


def arch() -> str:
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def key(mode: str, off, arch_name: str | None = None, nbig=None) -> str:
    """Size class: largest system and number of systems (next powers of two),
    plus the largest big-body count when some bodies are small."""
    sizes = np.diff(np.asarray(off))
    k = f"{arch_name or arch()}/{mode}/n{_pow2(int(sizes.max()))}/s{_pow2(len(sizes))}"
    if nbig is not None and np.any(np.asarray(nbig) < sizes):
        k += f"/b{_pow2(int(np.max(nbig)))}"
    return k


TABLE = os.path.join(PKG, "tuning.tsv")
TABLE_FIELDS = ("force_algo", "force_r", "force_jchunk", "enc_algo", "enc_jchunk", "step_algo", "force_g")


def write_table(cache: dict, path: str = TABLE) -> None:
    """The table the library reads (nb_params.autotune_path): one line per size
    class, the key then the seven chosen fields (force_g 0: the automatic width)."""
    lines = ["# key " + " ".join(TABLE_FIELDS) + "  (written by autotune.py from tuning.json)"]
    for k in sorted(cache):
        e = cache[k]
        lines.append(k + " " + " ".join(str(int(e.get(f, 0))) for f in TABLE_FIELDS))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def _mode_id(mode):
    return 1 if mode == "fp32c" else 0


def tune(w, mode: str, reps: int = 10, verbose: bool = True) -> dict:
    """Time every candidate on workload w; returns the best entry (not saved)."""
    from . import nb
    res_force, res_enc = {}, {}
    all_big = w.nbig is None or np.all(np.asarray(w.nbig) == np.diff(w.off))
    # 4: the symmetric force over the radial order (FP32C only)
    for fa in (((1, 2, 4) if mode == "fp32c" else (1, 2)) if all_big else (1,)):
        for r in FORCE_R:
            # the symmetric tile pairs have no source-chunk parameter, but a
            # super-tile width (tiles per workgroup)
            for j, g in ([(j, 0) for j in FORCE_J] if fa == 1 else [(1024, g) for g in FORCE_G]):
                if j > max(256, _pow2(int(np.diff(w.off).max()))) * 2:
                    continue
                p = nb.default_params(G=w.G, mode=_mode_id(mode), drag=int(w.drag), force_r=r, force_jchunk=j,
                                      force_algo=fa, force_g=g)
                c = nb.Context(w.off, p, enc_cap=1 << 16, device="cuda:0", tuned=False, nbig=w.nbig)
                c.upload(w.m0, w.m, w.x, w.v)
                # ranked by the whole force evaluation: more source chunks or
                # narrower super-tiles mean more split partials for the finalize
                ms = c.time_kernel(nb.NB_K_FORCE_EVAL, reps=reps)
                res_force[(fa, r, j, g)] = ms
                if verbose:
                    print(f"[autotune] {mode} force evaluation algo={fa} r={r} j={j} g={g}: {ms:.4f} ms",
                          file=sys.stderr, flush=True)
                c.close()
    # encounter candidates: (1, j) direct with source chunks of j, (2, 0) sorted
    # tiles, (3, 0) every body against its system's big bodies (some small
    # bodies, at most 256 big bodies per system)
    sizes = np.diff(w.off)
    nbig = sizes if w.nbig is None else np.asarray(w.nbig)
    enc_cands = [(1, j) for j in ENC_J if j <= max(256, _pow2(int(sizes.max()))) * 2] + [(2, 0)]
    if np.any(nbig < sizes) and int(nbig.max()) <= 256:
        enc_cands.append((3, 0))
    for ea, j in enc_cands:
        p = nb.default_params(G=w.G, mode=_mode_id(mode), drag=int(w.drag), enc_jchunk=j or 1024,
                              enc_algo=ea)
        c = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", tuned=False, nbig=w.nbig)
        c.upload(w.m0, w.m, w.x, w.v)
        c.drift(w.dt, allow_fail=True)
        ms = c.time_kernel(nb.NB_K_ENCOUNTER, reps=reps)
        res_enc[(ea, j)] = ms
        if verbose:
            print(f"[autotune] {mode} encounter algo={ea} j={j}: {ms:.4f} ms", file=sys.stderr, flush=True)
        c.close()
    (fa, r, j, g), fms = min(res_force.items(), key=lambda kv: kv[1])
    (ea, ej), ems = min(res_enc.items(), key=lambda kv: kv[1])

    def step_ms(fa_, r_, j_, g_, sa):
        p = nb.default_params(G=w.G, mode=_mode_id(mode), drag=int(w.drag), force_r=r_, force_jchunk=j_,
                              force_algo=fa_, force_g=g_, enc_jchunk=ej or 1024, enc_algo=ea, step_algo=sa)
        c = nb.Context(w.off, p, enc_cap=1 << 18, device="cuda:0", tuned=False, nbig=w.nbig)
        c.upload(w.m0, w.m, w.x, w.v)
        c.step(w.dt, 3, allow=(nb.NB_E_CAPACITY, nb.NB_E_KEPLER))
        ms = c.time_kernel(nb.NB_K_STEP, reps=max(2, reps // 2), dt=w.dt)
        c.close()
        return ms

    # force evaluations within 10 % of the fastest are told apart by the whole
    # step, where the force pass shares the GPU with the encounter check (the
    # super-tile width trades force-kernel time for partial traffic there)
    near = [k for k, v in res_force.items() if v <= 1.10 * fms]
    res_near = {}
    if len(near) > 1:
        for k in near:
            res_near[k] = step_ms(*k, 1)
            if verbose:
                print(f"[autotune] {mode} step with force algo={k[0]} r={k[1]} j={k[2]} g={k[3]}: "
                      f"{res_near[k]:.4f} ms", file=sys.stderr, flush=True)
        fa, r, j, g = min(res_near.items(), key=lambda kv: kv[1])[0]
        fms = res_force[(fa, r, j, g)]
    # the encounter test inside the force pass (FP32C, every body big, symmetric
    # force): only a whole step compares it with the separate check
    if mode == "fp32c" and all_big and fa == 2 and ea == 2:
        base = res_near.get((fa, r, j, g)) or step_ms(fa, r, j, g, 1)
        p4 = nb.default_params(G=w.G, mode=_mode_id(mode), drag=int(w.drag), force_r=r, force_jchunk=j,
                               force_algo=fa, force_g=g, enc_jchunk=ej or 1024, enc_algo=4, step_algo=1)
        c = nb.Context(w.off, p4, enc_cap=1 << 18, device="cuda:0", tuned=False, nbig=w.nbig)
        c.upload(w.m0, w.m, w.x, w.v)
        c.step(w.dt, 3, allow=(nb.NB_E_CAPACITY, nb.NB_E_KEPLER))
        fused = c.time_kernel(nb.NB_K_STEP, reps=max(2, reps // 2), dt=w.dt)
        c.close()
        res_enc[(4, 0)] = fused
        if verbose:
            print(f"[autotune] {mode} step with the check in the force pass: {fused:.4f} ms "
                  f"(separate: {base:.4f} ms)", file=sys.stderr, flush=True)
        # the step time of the chosen check (the per-phase launch's entry below)
        res_near[(fa, r, j, g)] = min(base, fused)
        if fused < base:
            ea = 4
    # whole-step launch: per-phase launches (tuned tiles) vs the persistent launch
    res_step = {}
    for sa in ((1, 2) if mode == "fp64" and int(np.diff(w.off).max()) <= 8192 else (1,)):
        res_step[sa] = (res_near[(fa, r, j, g)] if sa == 1 and (fa, r, j, g) in res_near
                        else step_ms(fa, r, j, g, sa))
        if verbose:
            print(f"[autotune] {mode} step launch {sa}: {res_step[sa]:.4f} ms", file=sys.stderr, flush=True)
    sa, sms = min(res_step.items(), key=lambda kv: kv[1])
    return {"force_algo": fa, "force_r": r, "force_jchunk": j, "force_g": g, "enc_jchunk": ej or 1024,
            "enc_algo": ea,
            "step_algo": sa, "step_ms": round(sms, 5), "step_candidates": {str(k): round(v, 5) for k, v in res_step.items()},
            "force_ms": round(fms, 5),
            "encounter_ms": round(ems, 5), "workload": w.name, "tuned_at": time.strftime("%Y-%m-%d"),
            "force_candidates": {f"a{f}_r{a}_j{b}_g{h}": round(v, 5) for (f, a, b, h), v in res_force.items()},
            "near_tie_steps": {f"a{f}_r{a}_j{b}_g{h}": round(v, 5) for (f, a, b, h), v in res_near.items()},
            "encounter_candidates": {f"a{a}_j{b}": round(v, 5) for (a, b), v in res_enc.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="c1,c2,c3,c4,c5,bigsmall")
    ap.add_argument("--modes", default="fp64,fp32c")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(PKG))
    import workloads
    cache = load_cache()
    a = arch()
    for name in args.workloads.split(","):
        w = workloads.by_name(name)
        for mode in args.modes.split(","):
            best = tune(w, mode, reps=args.reps)
            k = key(mode, w.off, a, w.nbig)
            cache[k] = best
            print(f"[autotune] {k} -> force_algo={best['force_algo']} r={best['force_r']} j={best['force_jchunk']} "
                  f"enc_algo={best['enc_algo']} enc_j={best['enc_jchunk']} step_algo={best['step_algo']} "
                  f"({best['force_ms']:.4f} / {best['encounter_ms']:.4f} ms)",
                  file=sys.stderr, flush=True)
            with open(args.out, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            write_table(cache, os.path.join(os.path.dirname(os.path.abspath(args.out)), "tuning.tsv"))


if __name__ == "__main__":
    main()
