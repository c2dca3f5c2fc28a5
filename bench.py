"""Benchmark of the PPM hot path on one MI355X.

Workload (default): the strongly shocked 512^3 periodic grid (density
lognormal sigma_ln = 2, Gaussian velocities of rms Mach 5, lognormal pressure
sigma_ln = 1, gamma = 5/3, seed 1002), advanced for K steps in FP64 and in
mixed precision side by side.  One step = periodic ghost fill + device CFL
reduction + the three sweeps (xyz on even steps, zyx on odd ones).  Inputs are
synthetic and already resident in HBM when the timed region starts.

Prints ONE JSON line: cell-updates/s of the FP64 path as `value` (one
cell-update = one active cell advanced through the x, y and z sweeps of a
step), the mixed-precision rate with its per-field L1 difference from the
FP64 path, the roofline of the dominant kernel (the sweep kernel) measured
with HIP events on its stream, and the CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0         # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TF = 78.6    # MI355X FP64 vector, TFLOP/s
FP32_VECTOR_PEAK_TF = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="active cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-sample-planes", type=int, default=64,
                    help="z-planes of the grid the CPU oracle advances (its sample)")
    ap.add_argument("--tiles", default=None, help="tile_config passed to ppm_plan_create")
    return ap.parse_args()


def make_input(n):
    import numpy as np
    from paper_1307_2265_amd import workloads as W
    cfg = W.CONFIGS[2]
    t0 = time.time()
    d = W.random_grid(n, n, n, cfg["seed"], cfg["recipe"])
    # both paths start from the same stored values: rho and v representable in FP32
    for f in ("rho", "vx", "vy", "vz"):
        d[f] = d[f].astype(np.float32).astype(np.float64)
    log(f"generated {n}^3 input in {time.time() - t0:.1f}s")
    return d


class Run:
    """One precision's patch, plan and dt on the device."""

    def __init__(self, d, prec, n, tiles=None):
        import torch
        from paper_1307_2265_amd import ppm
        low = torch.float32 if prec == ppm.PPM_MIXED else torch.float64
        self.t = {}
        for f, a in d.items():
            dt = torch.float64 if f in ("etot", "eint") else low
            self.t[f] = torch.from_numpy(a).to("cuda", dtype=dt)
        self.init = {f: v.clone() for f, v in self.t.items()}
        self.patch = ppm.Patch(**self.t, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
        self.plan = ppm.Plan([self.patch], 1, prec, ppm.params(), tile_config=tiles)
        self.tiles = tiles
        self.dt = torch.zeros(1, dtype=torch.float64, device="cuda")

    def reset(self):
        for f, v in self.t.items():
            v.copy_(self.init[f])

    def step(self, s):
        self.plan.ppm_fill_periodic()
        self.plan.ppm_cfl_dt(self.dt)
        self.plan.ppm_step(self.dt, s % 2)

    ORDERS = ((0, 1, 2), (2, 1, 0))  # xyz on even steps, zyx on odd ones

    def timed(self, steps):
        """Time `steps` steps.  Each step is the ghost fill, the CFL reduction
        and the three sweeps of ppm_step, issued here as three ppm_sweep calls
        (the same kernels with the same extents) so that HIP events on the
        launch stream bracket every sweep kernel.  Returns (total seconds,
        {kernel kind: mean seconds per launch})."""
        import torch
        lanes_mask = 1
        if self.tiles and "lanes=" in self.tiles:
            lanes_mask = int(self.tiles.split("lanes=")[1].split()[0])
        E = lambda: torch.cuda.Event(enable_timing=True)
        ev = [[(E(), E()) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0, t1 = E(), E()
        t0.record()
        for s in range(steps):
            self.plan.ppm_fill_periodic()
            self.plan.ppm_cfl_dt(self.dt)
            mask = 0
            for k, axis in enumerate(self.ORDERS[s % 2]):
                ev[s][k][0].record()
                self.plan.ppm_sweep(self.dt, axis, mask)
                ev[s][k][1].record()
                mask |= 1 << axis
        t1.record()
        torch.cuda.synchronize()
        total = t0.elapsed_time(t1) / 1e3
        per = {}
        for s in range(steps):
            for k, axis in enumerate(self.ORDERS[s % 2]):
                kind = "lanes" if (lanes_mask >> axis) & 1 else "march"
                per.setdefault(kind, []).append(ev[s][k][0].elapsed_time(ev[s][k][1]) / 1e3)
        return total, {k: sum(v) / len(v) for k, v in per.items()}

    def close(self):
        self.plan.close()


def cpu_baseline(d, n, planes):
    """The oracle (all host threads) on a slab of the same grid: `planes`
    z-planes treated as a periodic box of their own, one step."""
    import numpy as np
    import oracle as O
    g = 3
    sub = {f: np.ascontiguousarray(a[:planes + 2 * g]) for f, a in d.items()}
    G = O.Grid(**sub, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
    O.fill_periodic(G)
    prm = O.params()
    dt = O.cfl_dt(G, prm)
    t0 = time.perf_counter()
    O.step(G, prm, dt, 0)
    el = time.perf_counter() - t0
    cells = n * n * planes
    return dict(value=cells / el, unit="cell-updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"one step of a {n}x{n}x{planes} slab of the same seeded grid "
                       f"(periodic), FP64, {el:.1f}s wall")


def l1_per_field(a, b, g=3):
    """sum |a - b| / sum |b| over active cells, per field (a, b: dicts of tensors)."""
    out = {}
    for f in b:
        x = a[f][g:-g, g:-g, g:-g].double()
        y = b[f][g:-g, g:-g, g:-g].double()
        out[f] = float((x - y).abs().sum() / y.abs().sum())
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ppm.lib()
    n, K, Wm = args.n, args.steps, args.warmup
    d = make_input(n)
    cells = n ** 3

    ops_file = os.path.join(ROOT, "paper_1307_2265_amd", "data", "algorithmic_ops.json")
    with open(ops_file) as f:
        ops = json.load(f)["shocked"]["per_cell_sweep"]

    results = {}
    runs = {}
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        if name == "mixed" and args.no_mixed:
            continue
        r = Run(d, prec, n, args.tiles)
        for s in range(Wm):
            r.step(s)
        torch.cuda.synchronize()
        r.reset()
        log(f"{name}: warmup done, timing {K} steps")
        total, kern = r.timed(K)
        fb, fl = r.plan.ppm_event_counts()
        results[name] = dict(seconds=total, kern=kern, rate=cells * K / total,
                             fallback_faces=fb, floored_cells=fl)
        log(f"{name}: {K} steps in {total:.3f}s -> {cells * K / total / 1e9:.3f} G cell-updates/s, "
            + ", ".join(f"{k} sweep {v * 1e3:.3f} ms" for k, v in kern.items()))
        runs[name] = r

    # one-step and K-step L1 difference of the mixed path from the FP64 path
    l1 = None
    if "mixed" in runs:
        l1 = {"after_%d_steps" % K: l1_per_field(runs["mixed"].t, runs["fp64"].t)}
        for r in runs.values():
            r.reset()
            r.step(0)
        torch.cuda.synchronize()
        l1["after_1_step"] = l1_per_field(runs["mixed"].t, runs["fp64"].t)
    for r in runs.values():
        r.close()
    del runs

    # Roofline of the dominant kernel: the pencil-marching sweep kernel of the
    # FP64 run (it does the y sweep of every step and the z sweep, first or
    # last, so its launches average the first and last extents with the
    # second).  Algorithmic work of one launch: every pencil reads its n+6
    # cells and writes its n active cells (6 fields of 8 B), and performs the
    # oracle-counted FP64 operations for each of its n updated cells.
    g = 3
    nf = n + 2 * g
    kern = results["fp64"]["kern"]
    dom = "march" if "march" in kern else "lanes"
    pencils = [nf * nf, n * nf, n * n]  # first, second, third sweep of a step
    mean_pencils = sum(pencils) / 3.0
    if dom == "march" and "lanes" in kern:   # x sweeps go to the lane kernel
        mean_pencils = (n * nf + (nf * nf + n * n) / 2.0) / 2.0
    bytes_launch = mean_pencils * (nf + n) * 48.0
    cell_sweeps_launch = mean_pencils * n
    flops_launch = cell_sweeps_launch * ops["flops"]
    sw = kern[dom]
    hbm = dict(bound="hbm", achieved=bytes_launch / sw / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    alu = dict(bound="alu", achieved=flops_launch / sw / 1e12, peak=FP64_VECTOR_PEAK_TF,
               unit="TFLOP/s")
    alu["frac"] = alu["achieved"] / alu["peak"]
    for r_ in (hbm, alu):
        r_["traffic"] = None
        r_["kernel"] = f"sweep_kernel<PrecF64> ({dom})"
    roofline = alu if alu["frac"] >= hbm["frac"] else hbm
    other = hbm if roofline is alu else alu

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(d, n, min(args.cpu_sample_planes, n))
        log(f"cpu baseline: {cpu['value'] / 1e6:.2f} M cell-updates/s on {cpu['cores']} threads")

    fp = results["fp64"]
    line = {
        "metric": "cell-updates/sec (x+y+z sweeps) FP64 vs mixed-precision at stated L1 error, "
                  "1 MI355X",
        "value": fp["rate"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": fp["seconds"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single {n}^3 periodic grid, strongly shocked (rho lognormal "
                               "sigma 2, rms Mach 5, p lognormal sigma 1), gamma 5/3, "
                               "ghost 3, CFL 0.4, fill+cfl+xyz/zyx sweeps per step",
                   "cells": cells, "precision_of_value": "fp64"},
        "roofline": roofline,
        "roofline_other": other,
        "sweep_kernel_ms": {k: v * 1e3 for k, v in kern.items()},
        "events": {"fallback_faces": fp["fallback_faces"], "floored_cells": fp["floored_cells"]},
    }
    if "mixed" in results:
        mx = results["mixed"]
        line["mixed"] = {"value": mx["rate"], "unit": "cell-updates/s",
                         "ms_per_step": mx["seconds"] / K * 1e3, "dtype": "f32+f64",
                         "sweep_kernel_ms": {k: v * 1e3 for k, v in mx["kern"].items()},
                         "l1_rel_vs_fp64": l1,
                         "speedup_vs_fp64": mx["rate"] / fp["rate"]}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
