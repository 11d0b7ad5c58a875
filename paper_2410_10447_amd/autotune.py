"""Per-size-bucket choice of the launch options of the local search.

Ligands are bucketed by atom count (width 32) and torsion count (width 8).
For each bucket a representative synthetic ligand is timed, at a population
that fills the GPU several times over in whole rounds (12,288 individuals:
4, 8 and 16 rounds of the 3072, 1536 and 768 individuals resident at once
with one, two and four waves each, 2 rounds of 6144 with two per wave), so
that a choice that takes more waves per individual pays for the waves it
takes from other individuals and no candidate gains from a partial last
round, with every
candidate (reduction variant x threads per individual (64, 128, 256) x
individuals per wave x grid layout) through the C ABI, and the fastest
candidate is stored in a JSON table keyed by GPU architecture and bucket. `choose()` reads the table; a persistent launch over ligands of mixed
sizes then passes each item its bucket's variant and threads per individual
(items with different thread counts run in separate launches side by side).
Within a kernel family the buckets share one variant and layout when that
costs at most 6 % in every bucket (`unify_families`).

Usage: python -m paper_2410_10447_amd.autotune [--out table.json]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_gfx950.json")
ATOM_BUCKET = 32
TORSION_BUCKET = 8
DEFAULT = {"variant": 0, "threads_per_ind": 64, "plain_maps": False}


def bucket(n_atoms: int, n_torsions: int) -> str:
    return f"a{min(n_atoms - 1, 127) // ATOM_BUCKET}_t{min(n_torsions, 31) // TORSION_BUCKET}"


def bucket_centre(key: str):
    a, t = key.split("_")
    ia, it = int(a[1:]), int(t[1:])
    return ia * ATOM_BUCKET + ATOM_BUCKET // 2, it * TORSION_BUCKET + TORSION_BUCKET // 2


def all_buckets():
    return [f"a{a}_t{t}" for a in range(128 // ATOM_BUCKET) for t in range(32 // TORSION_BUCKET)]


_cache = {}


def load(path: str = TABLE_PATH) -> dict:
    if path not in _cache:
        if os.path.exists(path):
            with open(path) as f:
                _cache[path] = json.load(f)
        else:
            _cache[path] = {"arch": "gfx950", "buckets": {}}
    return _cache[path]


def two_per_wave_ok(n_atoms: int, n_torsions: int) -> bool:
    """Two individuals fit one wave: <= 32 atoms and <= 32 genes."""
    return n_atoms <= 32 and 7 + n_torsions <= 32


def choose(n_atoms: int, n_torsions: int, path: str = TABLE_PATH) -> dict:
    c = dict(load(path)["buckets"].get(bucket(n_atoms, n_torsions), DEFAULT))
    if c.get("two_per_wave") and not two_per_wave_ok(n_atoms, n_torsions):
        c["two_per_wave"] = False          # the bucket's other ligands may take it; this one cannot
    return c


def candidates(n_atoms: int = 64, n_torsions: int = 0):
    """Reduction variant x threads per individual (one wave, or two or four
    waves splitting the pair batches and, past 64 atoms, the atoms) x grid
    layout (the corner-expanded copy, or the planar maps); for ligands that
    fit, also two individuals per wave (shuffle reduction, either layout)."""
    from . import dock
    out = [{"variant": v, "threads_per_ind": b, "plain_maps": p} for p in (False, True)
           for b in (64, 128, 256) for v in (dock.REDUCE_SHUFFLE, dock.REDUCE_MFMA_F32)]
    if two_per_wave_ok(n_atoms, n_torsions):
        out += [{"variant": dock.REDUCE_SHUFFLE, "threads_per_ind": 64, "plain_maps": p, "two_per_wave": True}
                for p in (False, True)]
    return out


def cand_key(c) -> str:
    return (f"v{c['variant']}_b{c['threads_per_ind']}" + ("_plain" if c.get("plain_maps") else "")
            + ("_x2" if c.get("two_per_wave") else ""))


def time_candidate(G, L, gen, cand, iterations=20, reps=3):
    import torch
    from . import dock
    st0 = dock.LSState.start(gen)
    ws = torch.empty(dock.workspace_bytes(1), dtype=torch.uint8, device=gen.device)
    times = []
    for r in range(reps + 1):
        st = st0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dock.local_search([dock.LsJob(G, L, st, cand["variant"], threads_per_ind=cand.get("threads_per_ind", 64),
                                      plain_maps=cand.get("plain_maps", False),
                                      two_per_wave=cand.get("two_per_wave", False))],
                          iterations, workspace=ws)
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    return gen.shape[0] * (iterations + 1) / dt


def tune(out: str = TABLE_PATH, n_individuals: int = 12288, iterations: int = 20, seed: int = 77):
    import torch
    from . import dock, synth
    grd = synth.grids(64, 10, seed)
    G = dock.Grids.from_synth(grd)
    ff = synth.force_field()
    table = {"arch": "gfx950", "n_individuals": n_individuals, "iterations": iterations,
             "buckets": {}}
    for key in all_buckets():
        n, t = bucket_centre(key)
        lig = synth.ligand(n, t, seed + n * 100 + t)
        L = dock.Ligand(lig, ff)
        gen = torch.from_numpy(synth.genotypes(lig, grd, n_individuals, seed)).cuda()
        best, rates = None, {}
        for c in candidates(n, lig.n_torsions):
            rate = time_candidate(G, L, gen, c, iterations)
            rates[cand_key(c)] = rate
            if best is None or rate > best[1]:
                best = (c, rate)
        entry = dict(best[0])
        entry["evals_per_s"] = best[1]
        entry["measured"] = rates
        entry["atoms"], entry["torsions"] = n, lig.n_torsions
        table["buckets"][key] = entry
        print(key, entry, flush=True)
    unify_families(table)
    unify_shared_launch(table)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    _cache.pop(out, None)
    return table


def family(entry) -> str:
    """Kernel family a bucket's items run in: two individuals per wave, four
    or two waves per individual, or one wave with one atom per lane (<= 64
    atoms) or two (larger ligands)."""
    if entry.get("two_per_wave"):
        return "two-per-wave"
    if entry["threads_per_ind"] == 256:
        return "four-wave"
    if entry["threads_per_ind"] == 128:
        return "two-wave"
    return "one-slot" if entry["atoms"] <= 64 else "two-slot"


def unify_families(table, tol: float = 0.06):
    """One reduction variant and grid layout per kernel family where it
    costs little.

    A launch whose items use different variants (or layouts) runs the kernel
    that dispatches per item, which holds every variant's registers (the
    two-wave one spills 72 bytes per lane; on the uneven 64-ligand batch its
    launch was about 4 % slower than the specialised one); one choice per
    family keeps the specialised kernels. Per family, the
    (variant, layout) whose worst relative loss over the family's buckets
    (against each bucket's best candidate, at the bucket's thread count) is
    smallest is given to every bucket of the family, if that loss is at most
    `tol`.
    """
    fams = {}
    for key, e in table["buckets"].items():
        fams.setdefault(family(e), []).append(key)
    for fam, keys in fams.items():
        opts = sorted({(int(k.split("_")[0][1:]), "_plain" in k)
                       for e in (table["buckets"][k] for k in keys) for k in e["measured"]})
        best_o, best_loss = None, None
        for v, plain in opts:
            loss = 0.0
            for key in keys:
                e = table["buckets"][key]
                r = e["measured"].get(cand_key({"variant": v, "threads_per_ind": e["threads_per_ind"],
                                                "plain_maps": plain,
                                                "two_per_wave": e.get("two_per_wave", False)}))
                loss = max(loss, 1.0 if r is None else 1.0 - r / e["evals_per_s"])
            if best_loss is None or loss < best_loss:
                best_o, best_loss = (v, plain), loss
        if best_loss is not None and best_loss <= tol:
            for key in keys:
                e = table["buckets"][key]
                e["variant"], e["plain_maps"] = best_o[0], best_o[1]
                e["evals_per_s"] = e["measured"][cand_key(e)]
        table.setdefault("families", {})[fam] = {
            "variant": None if best_o is None else best_o[0],
            "plain_maps": None if best_o is None else best_o[1],
            "worst_loss": best_loss, "unified": best_loss is not None and best_loss <= tol}
    return table


SHARED_FAMILIES = ("two-wave", "one-slot", "two-per-wave")


def unify_shared_launch(table, tol: float = 0.06):
    """One reduction variant, on the corner-expanded maps, for the kernel
    families that can share one persistent launch (two waves per individual,
    one wave for ligands of <= 64 atoms, two individuals per wave), where it
    costs at most `tol` in every bucket against the bucket's best candidate
    at its threads per individual and individuals per wave: a batch mixing
    those families then runs as one launch. Two per wave has the shuffle
    reduction only, so with such buckets the shuffle is the one choice."""
    keys = [k for k, e in table["buckets"].items() if family(e) in SHARED_FAMILIES]
    if not keys:
        return table
    fams = {family(table["buckets"][k]) for k in keys}
    variants = [0] if "two-per-wave" in fams else sorted(
        {int(m.split("_")[0][1:]) for k in keys for m in table["buckets"][k]["measured"]})
    best_v, best_loss = None, None
    for v in variants:
        loss = 0.0
        for key in keys:
            e = table["buckets"][key]
            best = max(r for m, r in e["measured"].items()
                       if m.startswith("v") and m.split("_")[1] == f"b{e['threads_per_ind']}"
                       and m.endswith("_x2") == bool(e.get("two_per_wave")))
            r = e["measured"].get(cand_key({"variant": v, "threads_per_ind": e["threads_per_ind"],
                                            "plain_maps": False, "two_per_wave": e.get("two_per_wave", False)}))
            loss = max(loss, 1.0 if r is None else 1.0 - r / best)
        if best_loss is None or loss < best_loss:
            best_v, best_loss = v, loss
    shared = best_loss is not None and best_loss <= tol
    if shared:
        for key in keys:
            e = table["buckets"][key]
            e["variant"], e["plain_maps"] = best_v, False
            e["evals_per_s"] = e["measured"][cand_key(e)]
    table["shared_launch"] = {"families": sorted(fams), "variant": best_v, "worst_loss": best_loss,
                              "unified": shared}
    return table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--n", type=int, default=12288)
    ap.add_argument("--iters", type=int, default=20)
    a = ap.parse_args()
    tune(a.out, a.n, a.iters)
