"""Autotuner for the stage-kernel tile (elements per workgroup) per degree.

    python -m paper_2312_07725_amd.tune [--ne 16,32] [--reps 200] [--out PATH]
    python -m paper_2312_07725_amd.tune --ensemble [--reps 50] [--out PATH]

For every p in 2..5 it times the full right-hand side (nsfr_rhs: volume and
surface fluxes, weight-adjusted inverse with c = c_HU) of the warped TGV on an
ne^3 mesh for every tile the library accepts, and writes the fastest tile per
degree to tiles_gfx950.json next to this file. NSFR(tile=0) and Ensemble read
that table. Timing uses HIP events on the current stream, median of 5 batches.

With --ensemble it tunes the tiles the ensemble kernels use instead, on the
ensemble itself (64 TGV flows, seed 0, mixed degrees and mesh sizes): for each
degree in turn, every tile is timed with the other degrees' tiles held, and
the fastest is kept (one coordinate sweep). The result is stored as
"ensemble_tiles" next to the single-flow "tiles" of the same file; Ensemble
reads it (falling back to "tiles").
"""
import argparse
import json
import os
import statistics
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
TILES_PATH = os.path.join(HERE, "tiles_gfx950.json")


def load_tiles(path=TILES_PATH):
    """{p: epb} from the tuned table, or {} if there is none."""
    try:
        with open(path) as fh:
            d = json.load(fh)
        return {int(k): int(v["epb"]) for k, v in d.get("tiles", {}).items()}
    except (OSError, ValueError, KeyError):
        return {}


def load_ensemble_tiles(path=TILES_PATH):
    """{p: epb} tuned on the ensemble, else the single-flow table."""
    try:
        with open(path) as fh:
            d = json.load(fh)
        t = d.get("ensemble_tiles")
        if t:
            return {int(k): int(v["epb"]) for k, v in t.items()}
    except (OSError, ValueError, KeyError):
        pass
    return load_tiles(path)


def tune_ensemble(reps=50, out=TILES_PATH, base=TILES_PATH, verbose=True):
    from . import inputs
    from .nsfr import Ensemble, NSFR, NSFRError, c_hu, make_config
    draws = inputs.ensemble_draws(64, seed=0)
    ens = Ensemble([make_config(p, ne, beta=0.2, c=c_hu(p)) for (ne, p, m) in draws])
    U = ens.empty()
    for i, (ne, p, mach) in enumerate(draws):
        g = NSFR(p, ne, beta=0.2, c=c_hu(p))
        ens.flow_view(U, i).copy_(inputs.tgv_state(g.node_coords().cpu(), 1.4, mach))
        del g
    out_t = ens.empty()
    table = {}
    for p in sorted({p for (_, p, _) in draws}):
        res = {}
        for epb in range(1, 33):
            try:
                ens.set_tile(p, epb)
            except NSFRError:
                continue
            res[epb] = time_rhs(ens, U, out_t, reps)
            if verbose:
                print(f"ensemble p={p} epb={epb}: {res[epb]:.2f} us", flush=True)
        best = min(res, key=res.get)
        ens.set_tile(p, best)
        table[str(p)] = {"epb": best, "rhs_us": res[best], "all_us": {str(k): v for k, v in res.items()}}
    try:
        with open(base) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        doc = {}
    doc["ensemble_tiles"] = table
    doc["ensemble"] = "64 TGV flows (inputs.ensemble_draws(64, seed=0)), c=c_HU; time of one ensemble rhs (us)"
    if out:
        with open(out, "w") as fh:
            json.dump(doc, fh, indent=1)
    return doc


def time_rhs(g, U, out, reps):
    st = torch.cuda.current_stream()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(10):
        g.rhs(U, out)
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        s.record(st)
        for _ in range(reps):
            g.rhs(U, out)
        e.record(st)
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e) * 1e3 / reps)
    return statistics.median(times)


def select_tile(per_mesh):
    """per_mesh: {mesh: {tile: time}}. Returns (tile, worst slowdown): among
    the tiles timed on every mesh, the one whose largest ratio to the fastest
    time of a mesh is smallest (ties to the smaller tile)."""
    common = set.intersection(*(set(r) for r in per_mesh.values()))
    if not common:
        raise ValueError("no tile was timed on every mesh")
    worst = {t: max(r[t] / min(r.values()) for r in per_mesh.values()) for t in common}
    best = min(sorted(common), key=worst.get)
    return best, worst[best]


def tune(nes=(16, 32), reps=200, ps=(2, 3, 4, 5), out=TILES_PATH, verbose=True):
    """Time nsfr_rhs of the warped TGV (c = c_HU) for every valid tile on each
    mesh in nes; per degree keep the tile whose worst slowdown against the
    fastest tile of each mesh is smallest. The ensemble section of an
    existing table is kept."""
    from . import inputs
    from .nsfr import NSFR, NSFRError, c_hu
    table = {}
    for p in ps:
        per_ne = {}
        for ne in nes:
            res = {}
            U = None
            for epb in range(1, 33):
                try:
                    g = NSFR(p, ne, beta=0.2, c=c_hu(p), tile=epb)
                except NSFRError:
                    continue
                if U is None:
                    U = inputs.tgv_state(g.node_coords().cpu()).cuda().contiguous()
                o = g.empty()
                res[epb] = time_rhs(g, U, o, reps)
                if verbose:
                    print(f"p={p} ne={ne} epb={epb}: {res[epb]:.2f} us", flush=True)
                del g, o
            per_ne[ne] = res
        best, worst = select_tile(per_ne)
        entry = {"epb": best, "worst_slowdown": worst}
        for ne in nes:
            entry[f"rhs_us_{ne}"] = per_ne[ne][best]
            entry[f"all_us_{ne}"] = {str(k): v for k, v in sorted(per_ne[ne].items())}
        table[str(p)] = entry
    try:
        with open(out) as fh:
            old = json.load(fh)
    except (OSError, ValueError, TypeError):
        old = {}
    doc = {"device": torch.cuda.get_device_name(0),
           "mesh": " and ".join(f"{ne}^3" for ne in nes) + " warped TGV (beta=0.2), c=c_HU",
           "metric": "median time of one nsfr_rhs (us)",
           "rule": "per degree the tile with the smallest worst slowdown against the fastest tile of each mesh",
           "tiles": table}
    for k in ("ensemble_tiles", "ensemble"):
        if k in old:
            doc[k] = old[k]
    if out:
        with open(out, "w") as fh:
            json.dump(doc, fh, indent=1)
    return doc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ne", default="16,32", help="comma-separated mesh sizes")
    ap.add_argument("--reps", type=int, default=200)
    ap.add_argument("--out", default=TILES_PATH)
    ap.add_argument("--ensemble", action="store_true", help="tune the ensemble kernels' tiles on the ensemble")
    a = ap.parse_args()
    if a.ensemble:
        doc = tune_ensemble(a.reps, out=a.out)
        json.dump({k: v["epb"] for k, v in doc["ensemble_tiles"].items()}, sys.stdout)
    else:
        doc = tune(tuple(int(v) for v in str(a.ne).split(",")), a.reps, out=a.out)
        json.dump({k: v["epb"] for k, v in doc["tiles"].items()}, sys.stdout)
    print()


if __name__ == "__main__":
    main()
