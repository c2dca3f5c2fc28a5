"""Autotuner of the launch shapes (tile_config) of the PPM library.

For each workload class (one big periodic grid; a batch of uneven AMR
patches) and each precision, every candidate tile_config is timed over a few
steps from the same seeded initial state on the GPU, and the fastest is
written to data/tiles.json, which bench.py reads.  Results do not depend on
the launch shapes (the GPU tests check every layout against the oracle), so
the choice is purely a matter of speed.

    python -m paper_1307_2265_amd.autotune [--n 512] [--npatch 4096] [--steps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import harness as H
from . import ppm

HERE = os.path.dirname(os.path.abspath(__file__))
TILES_JSON = os.path.join(HERE, "data", "tiles.json")

CANDIDATES = {
    "single": [
        "lanes=1 block=256 lanes_block=256",
        "lanes=1 block=256 lanes_block=128",
        "lanes=1 block=256 lanes_block=64",
        "lanes=1 block=128 lanes_block=256",
        "lanes=1 block=128 lanes_block=64",
        "lanes=1 block=256 lanes_block=128 tail=0",
        "lanes=0 block=256",
        "lanes=3 block=256 lanes_block=256",
        "lanes=5 block=256 lanes_block=256",
        "lanes=7 lanes_block=256",
        "lanes=7 lanes_block=64",
    ],
    "batch": [
        "persistent=1 lanes=1 batch_block=256",
        "persistent=1 lanes=1 batch_block=128",
        "persistent=0 lanes=1 block=64 lanes_block=64",
        "persistent=0 lanes=1 block=64 lanes_block=128",
        "persistent=0 lanes=1 block=128 lanes_block=64",
        "persistent=0 lanes=1 block=128 lanes_block=128",
        "persistent=0 lanes=1 block=256 lanes_block=64",
        "persistent=0 lanes=1 block=64 lanes_block=64 group=0",
        "persistent=0 lanes=0 block=64",
        "persistent=0 lanes=1 block=256 lanes_block=128",
        "persistent=0 lanes=1 block=256 lanes_block=256",
        "persistent=0 lanes=3 block=256 lanes_block=64",
        "persistent=0 lanes=5 block=256 lanes_block=64",
        "persistent=0 lanes=7 lanes_block=64",
        "persistent=0 lanes=7 lanes_block=128",
        "persistent=0 lanes=7 lanes_block=256",
        "persistent=1 lanes=7 batch_block=256",
    ],
}


def log(msg):
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


def tune(run: H.Run, kind: str, steps: int, graphs: bool) -> dict:
    res = {}
    for tiles in CANDIDATES[kind]:
        run.replan(tiles)
        run.reset()
        run.step(0)  # warm-up (first launch of each kernel)
        run.reset()
        t, _ = run.timed(steps, graphs=graphs)
        res[tiles] = t / steps * 1e3
        log(f"{kind} {tiles!r}: {res[tiles]:.3f} ms/step")
    best = min(res, key=res.get)
    return {"tiles": best, "ms_per_step": res[best], "candidates_ms_per_step": res,
            "steps_timed": steps, "graphs": graphs}


def load() -> dict:
    if os.path.exists(TILES_JSON):
        with open(TILES_JSON) as f:
            return json.load(f)
    return {}


def best_tiles(key: str) -> str | None:
    return load().get(key, {}).get("tiles")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--npatch", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--out", default=TILES_JSON)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the autotuner times kernels on a GPU"
    out = {"device": torch.cuda.get_device_name(0), "when": time.strftime("%Y-%m-%d %H:%M"),
           "workloads": {"single": f"{args.n}^3 periodic grid, strongly shocked (seed 1002)",
                         "batch": f"{args.npatch} uneven patches, levels 0-6 (seed 1003)"}}
    d = H.single_grid_input(args.n)
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        run = H.Run.single(d, args.n, prec)
        out[f"single/{name}"] = tune(run, "single", args.steps, graphs=False)
        run.close()
    del d
    specs, fields = H.batch_input(args.npatch)
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        run = H.Run.batch(specs, fields, prec)
        out[f"batch/{name}"] = tune(run, "batch", args.steps, graphs=True)
        run.close()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
