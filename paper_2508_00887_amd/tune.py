"""Autotuner for the tile edge of a solve's SDSN passes and GEMMs, per size bucket.

The streaming SDSN pass (Algorithm 2, one launch per pass) is what a solve
spends its time on, and its speed depends on the square tile edge (64, 128 or
256) through the grid size, the number of FP64 partial sums each workgroup
combines and the occupancy.  For every probe size n the tuner times the pass
at each edge on a synthetic nonnegative matrix of that size (HIP events, no
host waits between launches), keeps the fastest, and turns the winners into a
bucket table for fram_set_tile_table: the boundary between two neighbouring
probe sizes is their geometric mean, neighbouring buckets with the same edge
merge, and sizes above the last probe keep the library's built-in rule.

The table is a small JSON file.  When the environment variable
FRAM_TUNE_CACHE names one, the binding applies it as it loads the library.

    python -m paper_2508_00887_amd.tune --out tune.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from .fram import Context, fram_set_tile_table

TILES = (64, 128, 256)
DEFAULT_SIZES = (64, 128, 256, 512, 1000, 1500, 2000, 3000, 4000, 6000, 8000)


def measure(ctx: Context, n: int, tile: int, passes: int = 200, seed: int = 0) -> float:
    """Microseconds per streaming SDSN pass at size n and tile edge `tile`."""
    rng = np.random.default_rng(seed + n)
    K = (rng.random((n, n)) ** 2).astype(np.float32)
    _, st = ctx.sdsn_project(K, 2.0, tile=tile, sdsn_mode="stream", profile=2,
                             sdsn_max=passes, gamma_tol=0.0)
    return 1e3 * st["ms_sdsn"] / max(1, st["sdsn_passes"])


def buckets_from(probes: list[dict]) -> list[dict]:
    """Bucket table from probe results sorted by n (each {"n", "tile"})."""
    probes = sorted(probes, key=lambda p: p["n"])
    out: list[dict] = []
    for k, p in enumerate(probes):
        if k + 1 < len(probes):
            n_max = int(math.isqrt(p["n"] * probes[k + 1]["n"]))
            n_max = max(n_max, p["n"])
        else:
            n_max = p["n"]
        if out and out[-1]["tile"] == p["tile"]:
            out[-1]["n_max"] = n_max
        else:
            out.append({"n_max": n_max, "tile": int(p["tile"])})
    return out


def tune(ctx: Context, sizes=DEFAULT_SIZES, tiles=TILES, passes: int = 200, reps: int = 2,
         log=None) -> dict:
    """Time every (size, tile) pair and return the table (not yet applied)."""
    probes = []
    for n in sorted(set(int(s) for s in sizes)):
        times = {}
        for t in tiles:
            times[t] = min(measure(ctx, n, t, passes) for _ in range(reps))
        best = min(times, key=lambda t: (times[t], t))
        probes.append({"n": n, "tile": best, "us_per_pass": {str(t): times[t] for t in tiles}})
        if log:
            log(f"n={n}: " + ", ".join(f"{t}: {times[t]:.2f} us" for t in tiles) + f" -> {best}")
    return {"version": 1, "created": time.strftime("%Y-%m-%d %H:%M:%S"), "passes": passes,
            "probes": probes, "buckets": buckets_from(probes)}


def validate(table: dict) -> list[dict]:
    b = table.get("buckets")
    if table.get("version") != 1 or not isinstance(b, list):
        raise ValueError("not a version-1 tile table")
    prev = 0
    for e in b:
        if not (isinstance(e.get("n_max"), int) and e["n_max"] > prev and e.get("tile") in TILES):
            raise ValueError(f"bad bucket {e!r}")
        prev = e["n_max"]
    return b


def apply(table: dict) -> None:
    """Install the table in the library (process-wide)."""
    b = validate(table)
    fram_set_tile_table([e["n_max"] for e in b], [e["tile"] for e in b])


def clear() -> None:
    fram_set_tile_table([], [])


def save(table: dict, path: str) -> None:
    validate(table)
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)


def load(path: str) -> dict:
    with open(path) as fh:
        table = json.load(fh)
    validate(table)
    return table


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", type=int, nargs="*", default=list(DEFAULT_SIZES))
    ap.add_argument("--passes", type=int, default=200)
    ap.add_argument("--device", type=int, default=0)
    args = ap.parse_args(argv)
    ctx = Context(args.device)
    try:
        table = tune(ctx, args.sizes, passes=args.passes, log=lambda m: print(m, flush=True))
    finally:
        ctx.close()
    save(table, args.out)
    print(json.dumps(table["buckets"]), flush=True)


if __name__ == "__main__":
    main()
