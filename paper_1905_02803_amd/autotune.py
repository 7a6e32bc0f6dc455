"""Autotuner for the batched transforms: per transform, a radix order and a
tile width per axis (pf_tune), chosen by timing on the device.

For each transform of the batch, the three axes are tuned one after the
other (x, then y, then z), each by timing a one-transform batch
(forward + backward) for every candidate of that axis with the other axes at
their best so far.  Two searches per transform:

* radix orders 0..3 (16-first, 8-first, 4-first, odd-first) with the default
  tiles -- the plans of the fused mode, whose launches group transforms by
  block size: a tile width of its own would put a transform in a group of
  smaller blocks and split the launch, which one-transform timings cannot
  see;
* from there, radix orders times tile widths {default, 1, 2, 4, 8, 16, 32}
  line pairs for x and {default, 1, 2, 4, 8} columns for y and z -- the
  plans of the serial mode.

The result is cached as JSON keyed by "nx,ny,nz".

Usage (on a GPU):  python -m paper_1905_02803_amd.autotune --count 64 --seed 4 --out FILE
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned", "batch_gfx950.json")

TILES = {0: (0, 1, 2, 4, 8, 16, 32), 1: (0, 1, 2, 4, 8), 2: (0, 1, 2, 4, 8)}
ORDERS = (0, 1, 2, 3)


def key(d) -> str:
    return ",".join(str(int(v)) for v in d)


def load(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tune_for(dims, path: str = DEFAULT_CACHE, mode: str = "serial"):
    """pf_tune entries for dims from the cache (mode "serial": radix orders and
    tiles; "fused": radix orders, default tiles), or None if any transform is missing."""
    cache = load(path).get("entries", {})
    out = []
    for d in dims:
        e = cache.get(key(d))
        if e is None or (mode == "fused" and "fused_radix_order" not in e):
            return None
        if mode == "fused":
            out.append((tuple(e["fused_radix_order"]), (0, 0, 0)))
        else:
            out.append((tuple(e["radix_order"]), tuple(e["tile"])))
    return out


def _time_one(pf, torch, d, tune, reps: int, warm: int) -> float:
    with pf.Batch([d], tune=[tune]) as b:
        R = b.empty(0).zero_()
        C = b.empty(1).zero_()
        R2 = b.empty(0)
        for _ in range(warm):
            b.ftran(R, C)
            b.btran(C, R2)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for i in range(reps):
            b.ftran(R, C)
            b.btran(C, R2)
            ev[i + 1].record()
        torch.cuda.synchronize()
        return statistics.median(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))


def tune_batch(dims, reps: int = 7, warm: int = 2, log=print) -> dict:
    import torch

    import paper_1905_02803_amd as pf

    entries = {}
    for n, d in enumerate(dims):
        k = key(d)
        if k in entries:
            continue
        best = [[0, 0, 0], [0, 0, 0]]  # radix orders, tiles
        base = _time_one(pf, torch, d, (tuple(best[0]), tuple(best[1])), reps, warm)
        cur = base

        def search(tiles):
            nonlocal cur, best
            for axis in range(3):
                for order in ORDERS:
                    for tile in tiles[axis]:
                        cand = [list(best[0]), list(best[1])]
                        cand[0][axis], cand[1][axis] = order, tile
                        if cand == best:
                            continue
                        t = _time_one(pf, torch, d, (tuple(cand[0]), tuple(cand[1])), reps, warm)
                        if t < cur:
                            cur, best = t, cand

        search({0: (0,), 1: (0,), 2: (0,)})  # radix orders only
        orders, ms_orders = list(best[0]), cur
        search(TILES)
        entries[k] = {"radix_order": best[0], "tile": best[1], "fused_radix_order": orders,
                      "ms_default": base, "ms_orders": ms_orders, "ms_tuned": cur}
        log(f"[{n + 1}/{len(dims)}] {k}: default {base:.4f} ms -> orders {orders} {ms_orders:.4f} ms -> "
            f"{cur:.4f} ms with {best}", flush=True)
    return entries


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    import synth

    dims = synth.batch_sizes(args.seed, args.count)
    entries = tune_batch(dims, reps=args.reps)
    rec = {"device": torch.cuda.get_device_name(0), "generator": f"synth.batch_sizes({args.seed}, {args.count})",
           "command": "python -m paper_1905_02803_amd.autotune " + " ".join(argv or sys.argv[1:]),
           "entries": entries}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    tot_d = sum(e["ms_default"] for e in entries.values())
    tot_t = sum(e["ms_tuned"] for e in entries.values())
    print(f"sum over transforms: default {tot_d:.3f} ms, tuned {tot_t:.3f} ms", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
