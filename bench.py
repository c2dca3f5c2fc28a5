"""Benchmark of the PPM hot path on one MI355X.

Headline workload: the strongly shocked 512^3 periodic grid (density
lognormal sigma_ln = 2, Gaussian velocities of rms Mach 5, lognormal pressure
sigma_ln = 1, gamma = 5/3, 3 ghost layers, CFL 0.4, seed 1002), advanced K
steps in FP64 and in mixed precision side by side from the same stored input.
One step = periodic ghost fill + the three sweeps (xyz on even steps, zyx on
odd ones), the last of which also yields the next step's CFL timestep; the
first step's timestep is reduced before the timed region.  Inputs are
synthetic and resident in HBM when the timed region starts; launch shapes
come from the autotuner's table (data/tiles.json) when it exists.

Also measured: the same grid and steps with the HLLC solver in place of
two-shock (FP64 and mixed), and with the optional diffusive flux; the same grid with a seeded acceleration field
and comoving expansion factors (gravity sources in every sweep, a pass of the
expansion terms per step, FP64 and mixed); the AMR W-cycle (ppm_amr_step:
subcycled levels, flux correction, projection) on a nested hierarchy; the AMR
patch ghost fill (parent interpolation and
sibling copies) on a nested hierarchy; the batched form -- 4096 uneven AMR patches (dims from
{8,12,16,24,32}, levels 0-6 with their own dt, seeded ghosts, flux registers
on) advanced by replaying one captured HIP graph per step (the three sweeps
and the next timestep) -- and its rate relative to the single grid.

Prints ONE JSON line: FP64 cell-updates/s of the single grid as `value` (one
cell-update = one active cell through the x, y and z sweeps of one step), the
mixed rate and its per-field L1 difference from the FP64 path after 1 and K
steps, the batch rates, the roofline of the dominant kernel measured with HIP
events on its launch stream, and the CPU oracle timed on a bounded sample of
the same workload.
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
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 39.3 T
# operations/s; the published 78.6 TFLOP/s counts a fused multiply-add as two.
# The sweep's operations are separate adds, multiplies, divides and square
# roots (the FP64 path is built without contraction so that it reproduces the
# oracle bit for bit), so 39.3 T op/s is the ceiling of its arithmetic.
FP64_OP_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="active cells per axis")
    ap.add_argument("--npatch", type=int, default=4096, help="patches of the batch (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-sample-planes", type=int, default=0,
                    help="z-planes of the grid the CPU oracle advances (0: all)")
    ap.add_argument("--cpu-sample-steps", type=int, default=2,
                    help="steps the CPU oracle advances")
    ap.add_argument("--tiles", default=None, help="tile_config of the single-grid plans")
    ap.add_argument("--batch-tiles", default=None, help="tile_config of the batch plans")
    ap.add_argument("--no-hllc", action="store_true", help="skip the HLLC-solver runs")
    ap.add_argument("--no-amr-fill", action="store_true", help="skip the AMR ghost-fill timing")
    ap.add_argument("--no-amr-step", action="store_true", help="skip the AMR W-cycle timing")
    ap.add_argument("--no-diffusion", action="store_true",
                    help="skip the runs with the diffusive flux")
    ap.add_argument("--amr-step-only", action="store_true",
                    help="time only the AMR W-cycle and print its JSON (for profiling it)")
    ap.add_argument("--no-sources", action="store_true",
                    help="skip the runs with gravity and comoving expansion")
    return ap.parse_args()


def cpu_baseline(d, n, planes, steps):
    """The oracle (all host threads) on the same grid, or on a slab of its
    first `planes` z-planes treated as a periodic box of its own: `steps`
    steps (fill + CFL + xyz/zyx sweeps), only the sweeps timed."""
    import numpy as np
    import oracle as O
    g = 3
    sub = {f: np.array(a[:planes + 2 * g], dtype=np.float64, copy=True) for f, a in d.items()}
    G = O.Grid(**sub, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
    prm = O.params()
    el = 0.0
    for s in range(steps):
        O.fill_periodic(G)
        dt = O.cfl_dt(G, prm)
        t0 = time.perf_counter()
        O.step(G, prm, dt, s % 2)
        el += time.perf_counter() - t0
    cells = n * n * planes * steps
    what = f"the full {n}^3 grid" if planes == n else f"a {n}x{n}x{planes} periodic slab of the grid"
    cores = O.num_threads()
    # one host thread, on a 16-plane periodic slab of the same grid, one step
    # (its ghost planes add 3/8 to the z-extent of the x and y sweeps)
    O.set_num_threads(1)
    sub1 = {f: np.array(a[:16 + 2 * g], dtype=np.float64, copy=True) for f, a in d.items()}
    G1 = O.Grid(**sub1, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
    O.fill_periodic(G1)
    dt1 = O.cfl_dt(G1, prm)
    t0 = time.perf_counter()
    O.step(G1, prm, dt1, 0)
    el1 = time.perf_counter() - t0
    O.set_num_threads(cores)
    single = dict(value=n * n * 16 / el1, unit="cell-updates/s", cores=1,
                  sample=f"1 step of a {n}x{n}x16 periodic slab of the grid, FP64, {el1:.1f}s wall")
    return dict(value=cells / el, unit="cell-updates/s", cores=cores, kind="oracle",
                sample=f"{steps} steps of {what} (same seeded input), FP64, sweeps {el:.1f}s wall",
                single_thread=single)


def amr_ghost_fill(reps: int = 5) -> dict:
    """Time ppm_fill_ghosts (parent interpolation + sibling copies) level by
    level on a nested FP64 hierarchy: a 128^3 root, 64 level-1 blocks of 32^3
    tiling its centre, 512 level-2 blocks of 24^3 (8 in each level-1 block)."""
    import numpy as np
    import torch
    from paper_1307_2265_amd import ppm, workloads as W
    from paper_1307_2265_amd import harness as H
    hier = W.nested_hierarchy(128, (32, 24), (4, 2))
    fields = [W.random_grid(*h.dims, 4000 + i, W.SHOCKED) for i, h in enumerate(hier)]
    run = H.Run(fields, [(*h.dims, h.level, 0.5 ** h.level / 128) for h in hier], ppm.PPM_FP64,
                3, False)
    run.plan.ppm_set_hierarchy([(h.parent, 2, h.start) for h in hier])
    run.plan.ppm_fill_boundary(0, [ppm.PPM_FACE_PERIODIC] * 6)
    g = W.GHOST
    out = {"workload": "nested FP64 hierarchy: 128^3 root, 64 level-1 blocks of 32^3, 512 "
                       "level-2 blocks of 24^3 (refinement 2, siblings abutting)",
           "levels": {}}
    for level in (1, 2):
        run.plan.ppm_fill_ghosts(level)   # warm-up
    torch.cuda.synchronize()
    for level in (1, 2):
        cells = sum((h.dims[0] + 2 * g) ** 3 - h.dims[0] ** 3 for h in hier if h.level == level)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run.plan.ppm_fill_ghosts(level)
        b.record()
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) / 1e3 / reps
        # algorithmic bytes: 48 B written per ghost cell, plus the parent cell
        # that covers it read once per r^3 = 8 fine cells
        byt = cells * (48.0 + 48.0 / 8)
        out["levels"][str(level)] = {"ghost_cells": cells, "ms": sec * 1e3,
                                     "ghost_cells_per_s": cells / sec,
                                     "algorithmic_GBps": byt / sec / 1e9,
                                     "hbm_frac": byt / sec / 1e9 / HBM_PEAK_GBS}
    run.close()
    return out


def amr_w_cycle(steps: int = 3, warmup: int = 1) -> dict:
    """Time ppm_amr_step (the W-cycle with subcycling, flux correction and
    projection) on the nested hierarchy of amr_ghost_fill with gentle fields
    (rms Mach 0.5) and a periodic root, in FP64 and mixed precision.  A
    cell-update is one active cell through one level step."""
    import time as _time
    import torch
    from paper_1307_2265_amd import ppm, workloads as W
    from paper_1307_2265_amd import harness as H
    hier = W.nested_hierarchy(128, (32, 24), (4, 2))
    fields = [W.random_grid(*h.dims, 5000 + i, W.GENTLE) for i, h in enumerate(hier)]
    cells = [h.dims[0] * h.dims[1] * h.dims[2] for h in hier]
    per_level = [sum(c for c, h in zip(cells, hier) if h.level == l) for l in range(3)]
    out = {"workload": "nested hierarchy: 128^3 periodic root, 64 level-1 blocks of 32^3, 512 "
                       "level-2 blocks of 24^3 (refinement 2, abutting siblings), gentle fields",
           "active_cells_per_level": per_level}
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        run = H.Run(fields, [(*h.dims, h.level, 0.5 ** h.level / 128) for h in hier], prec, 3,
                    True, with_reg=True)
        run.plan.close()
        amr = ppm.Amr(run.patches, [(h.parent, 2, h.start) for h in hier], 3, prec)
        for _ in range(warmup):
            amr.ppm_amr_step()
        _, n0 = amr.ppm_amr_times()
        torch.cuda.synchronize()
        t0 = _time.perf_counter()
        for _ in range(steps):
            amr.ppm_amr_step()
        torch.cuda.synchronize()
        sec = _time.perf_counter() - t0
        _, n1 = amr.ppm_amr_times()
        nsteps = [b - a for a, b in zip(n0, n1)]
        upd = sum(n * c for n, c in zip(nsteps, per_level))
        fb, fl = amr.ppm_amr_event_counts()
        out[name] = {"root_steps": steps, "level_steps": nsteps,
                     "ms_per_root_step": sec / steps * 1e3, "cell_updates_per_s": upd / sec,
                     "events": {"fallback_faces": fb, "floored_cells": fl}}
        amr.close()
        del run
        torch.cuda.empty_cache()
    return out


def copy_bandwidth(nbytes: int = 1 << 31, reps: int = 10) -> dict:
    """Achievable HBM bandwidth beside the published peak: a device-to-device
    copy of nbytes (read and write counted), timed with events on the current
    stream."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    gbs = 2 * nbytes / sec / 1e9
    return {"bytes_moved": 2 * nbytes, "ms": sec * 1e3, "GB_per_s": gbs,
            "frac_of_published_peak": gbs / HBM_PEAK_GBS}


def measured_traffic(kernel: str):
    """Calibrated HBM bytes per dispatch of `kernel` from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if the kernel sources changed
    since those counters were taken."""
    from paper_1307_2265_amd import profsummary
    path = os.path.join(ROOT, "paper_1307_2265_amd", "data", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_digest") != profsummary.kernel_source_digest() or kernel not in t["kernels"]:
        return None
    return t["kernels"][kernel]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import torch
    from paper_1307_2265_amd import autotune, ppm
    from paper_1307_2265_amd import harness as H
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ppm.lib()
    if args.amr_step_only:
        print(json.dumps({"amr_w_cycle": amr_w_cycle()}))
        return
    n, K, Wm = args.n, args.steps, args.warmup
    cells = n ** 3
    t0 = time.time()
    d = H.single_grid_input(n)
    log(f"generated {n}^3 input in {time.time() - t0:.1f}s")
    with open(os.path.join(ROOT, "paper_1307_2265_amd", "data", "algorithmic_ops.json")) as f:
        all_ops = json.load(f)
    ops = all_ops["shocked"]["per_cell_sweep"]

    # ---- single grid, FP64 and mixed
    results, runs = {}, {}
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        if name == "mixed" and args.no_mixed:
            continue
        tiles = args.tiles or autotune.best_tiles(f"single/{name}")
        r = H.Run.single(d, n, prec, tiles)
        for s in range(Wm):
            r.step(s)
        torch.cuda.synchronize()
        r.reset()
        r.plan.ppm_event_counts(reset=True)
        log(f"{name}: timing {K} steps (tiles {tiles})")
        total, kern = r.timed(K, per_sweep=True)
        fb, fl = r.plan.ppm_event_counts()
        results[name] = dict(seconds=total, kern=kern, rate=cells * K / total, tiles=tiles,
                             fallback_faces=fb, floored_cells=fl)
        log(f"{name}: {K} steps in {total:.3f}s -> {cells * K / total / 1e9:.3f} G cell-updates/s, "
            + ", ".join(f"{k} sweep {v * 1e3:.3f} ms" for k, v in kern.items()))
        runs[name] = r
    l1 = None
    if "mixed" in runs:
        l1 = {f"after_{K}_steps": H.l1_per_field(runs["mixed"], runs["fp64"])}
        for r in runs.values():
            r.reset()
            r.step(0)
        torch.cuda.synchronize()
        l1["after_1_step"] = H.l1_per_field(runs["mixed"], runs["fp64"])
    for r in runs.values():
        r.close()
    del runs
    torch.cuda.empty_cache()

    # ---- the same grid and steps with the HLLC solver in place of two-shock
    hllc = None
    if not args.no_hllc:
        hllc = {"flags": "PPM_ALL_FLAGS | PPM_HLLC"}
        for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
            if name == "mixed" and args.no_mixed:
                continue
            tiles = args.tiles or autotune.best_tiles(f"single/{name}")
            r = H.Run.single(d, n, prec, tiles, flags=ppm.PPM_ALL_FLAGS | ppm.PPM_HLLC)
            for s in range(Wm):
                r.step(s)
            torch.cuda.synchronize()
            r.reset()
            r.plan.ppm_event_counts(reset=True)
            total, hk = r.timed(K, per_sweep=True)
            fb, fl = r.plan.ppm_event_counts()
            hllc[name] = {"value": cells * K / total, "unit": "cell-updates/s",
                          "ms_per_step": total / K * 1e3, "tiles": tiles,
                          "sweep_kernel_ms": {k: v * 1e3 for k, v in hk.items()},
                          "speedup_vs_two_shock": results[name]["seconds"] / total,
                          "events": {"fallback_faces": fb, "floored_cells": fl}}
            log(f"hllc {name}: {cells * K / total / 1e9:.3f} G cell-updates/s")
            r.close()
        torch.cuda.empty_cache()

    # ---- the same grid and steps with the optional diffusive flux
    diffusion = None
    if not args.no_diffusion:
        diffusion = {"flags": "PPM_ALL_FLAGS | PPM_DIFFUSION"}
        for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
            if name == "mixed" and args.no_mixed:
                continue
            tiles = args.tiles or autotune.best_tiles(f"single/{name}")
            r = H.Run.single(d, n, prec, tiles, flags=ppm.PPM_ALL_FLAGS | ppm.PPM_DIFFUSION)
            for s in range(Wm):
                r.step(s)
            torch.cuda.synchronize()
            r.reset()
            r.plan.ppm_event_counts(reset=True)
            total, dk = r.timed(K, per_sweep=True)
            fb, fl = r.plan.ppm_event_counts()
            diffusion[name] = {"value": cells * K / total, "unit": "cell-updates/s",
                               "ms_per_step": total / K * 1e3, "tiles": tiles,
                               "sweep_kernel_ms": {k: v * 1e3 for k, v in dk.items()},
                               "slowdown_vs_plain": total / results[name]["seconds"],
                               "events": {"fallback_faces": fb, "floored_cells": fl}}
            log(f"diffusion {name}: {cells * K / total / 1e9:.3f} G cell-updates/s")
            r.close()
        torch.cuda.empty_cache()

    # ---- the same grid with an acceleration field and comoving expansion:
    # every sweep adds the gravity sources and divides by a, and a pass of
    # the expansion terms precedes the sweeps
    sources = None
    if not args.no_sources:
        src = dict(seed=4242, amp=3.0, a=1.7, adot=0.6)
        sources = {"recipe": "acceleration: 4 random plane waves per component over the "
                             "ghosted box, amplitude 3; a = 1.7, adot = 0.6", "kernels": {}}
        for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
            if name == "mixed" and args.no_mixed:
                continue
            tiles = args.tiles or autotune.best_tiles(f"single/{name}")
            r = H.Run.single(d, n, prec, tiles, sources=src)
            for s in range(Wm):
                r.step(s)
            torch.cuda.synchronize()
            r.reset()
            r.plan.ppm_event_counts(reset=True)
            total, sk = r.timed(K, per_sweep=True)
            fb, fl = r.plan.ppm_event_counts()
            ex_ms = sk["expansion"] * 1e3
            # algorithmic bytes of the expansion pass: read and write the three
            # velocities (storage type) and the two energies (double) per cell
            ex_bytes = cells * 2 * (3 * (8 if name == "fp64" else 4) + 2 * 8)
            sources[name] = {"value": cells * K / total, "unit": "cell-updates/s",
                             "ms_per_step": total / K * 1e3, "tiles": tiles,
                             "sweep_kernel_ms": {k: v * 1e3 for k, v in sk.items()},
                             "slowdown_vs_static": total / results[name]["seconds"],
                             "expansion": {"ms": ex_ms, "bytes": ex_bytes,
                                           "GB_per_s": ex_bytes / (ex_ms / 1e3) / 1e9,
                                           "frac_of_hbm_peak":
                                               ex_bytes / (ex_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
                             "events": {"fallback_faces": fb, "floored_cells": fl}}
            log(f"sources {name}: {cells * K / total / 1e9:.3f} G cell-updates/s, "
                f"expansion {ex_ms:.3f} ms ({ex_bytes / (ex_ms / 1e3) / 1e9:.0f} GB/s)")
            r.close()
        sources["kernels"] = {
            "march": "sweep_kernel<Prec, cfl, false, true, true>",
            "lanes": "sweep_lanes_kernel<Prec, cfl, true, true>",
            "expansion": "expansion_kernel<Prec>"}
        torch.cuda.empty_cache()

    amr = None
    if not args.no_amr_fill:
        amr = amr_ghost_fill()
        log("amr ghost fill: " + ", ".join(
            f"level {k} {v['ms']:.3f} ms ({v['ghost_cells_per_s'] / 1e9:.2f} G cells/s)"
            for k, v in amr["levels"].items()))
        torch.cuda.empty_cache()
    wcyc = None
    if not args.no_amr_step:
        wcyc = amr_w_cycle()
        for name in ("fp64", "mixed"):
            v = wcyc[name]
            log(f"amr W-cycle {name}: {v['ms_per_root_step']:.2f} ms per root step, level steps "
                f"{v['level_steps']}, {v['cell_updates_per_s'] / 1e9:.3f} G cell-updates/s")

    # ---- batch of uneven patches, one captured graph per step
    batch = None
    if args.npatch > 0:
        t0 = time.time()
        specs, fields = H.batch_input(args.npatch)
        log(f"generated {args.npatch} patches in {time.time() - t0:.1f}s")
        batch = {"workload": f"{args.npatch} patches, dims iid from {{8,12,16,24,32}}, levels "
                             "0-6 (dx = 2^-level, own dt per level), strongly shocked fields "
                             "with seeded ghosts, flux registers on, one HIP graph per step "
                             "(three sweeps + next dt)"}
        bruns = {}
        for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
            if name == "mixed" and args.no_mixed:
                continue
            tiles = args.batch_tiles or autotune.best_tiles(f"batch/{name}")
            r = H.Run.batch(specs, fields, prec, tiles)
            r.make_graphs()
            r.ensure_dt()
            for s in range(Wm):
                r.graphs[s % 2].ppm_graph_launch()
            torch.cuda.synchronize()
            r.reset()
            total, _ = r.timed(K, graphs=True)
            batch[name] = {"value": r.cells * K / total, "unit": "cell-updates/s",
                           "ms_per_step": total / K * 1e3, "tiles": tiles,
                           "active_cells": r.cells}
            log(f"batch {name}: {r.cells * K / total / 1e9:.3f} G cell-updates/s")
            bruns[name] = r
        if "mixed" in bruns:
            batch["mixed"]["l1_rel_vs_fp64"] = H.l1_per_field(bruns["mixed"], bruns["fp64"])
        for name in bruns:
            batch[name]["single_over_batch"] = results[name]["rate"] / batch[name]["value"]
            bruns[name].close()
        del bruns
        torch.cuda.empty_cache()

    # ---- roofline of the dominant kernel: the pencil-marching sweep kernel of
    # the FP64 single-grid run, in its plain form (the y sweeps, and the z
    # sweeps that open a zyx step; the z sweeps that close an xyz step run the
    # variant that also takes the next timestep).  Such a sweep is one
    # marching launch over whole rounds of resident threads plus, when
    # pencils are left over, a tail launch (sweep_tail_kernel) that streams
    # them; the unit measured is the sweep, both launches.
    # Algorithmic work of one sweep: every pencil reads its n+6 cells and
    # writes its n active cells (6 fields of 8 B), and performs the
    # oracle-counted FP64 operations (add, mul, div, sqrt) for each of its n
    # updated cells.  The bound is the roof the kernel's arithmetic intensity
    # meets first: ops per byte above FP64_OP_PEAK / HBM peak -> "alu".
    g = 3
    nf = n + 2 * g
    kern = results["fp64"]["kern"]
    dom = "march" if "march" in kern else "lanes"
    if dom == "march" and "lanes" in kern:  # x sweeps go to the lane kernel
        mean_pencils = (n * nf + nf * nf + n * nf) / 3.0
    else:
        mean_pencils = (nf * nf + n * nf) / 2.0
    bytes_launch = mean_pencils * (nf + n) * 48.0
    flops_launch = mean_pencils * n * ops["flops"]
    sw = kern[dom]
    # kernel names as the profiler reports them (template arguments: precision,
    # takes the next dt, spans patches, HLLC solver, gravity sources)
    kname = ("sweep_kernel<PrecF64, false, false, false, false>" if dom == "march"
             else "sweep_lanes_kernel<PrecF64, false, false, false>")
    tr = measured_traffic(kname)
    traffic = None if tr is None else tr["bytes"]
    if dom == "march" and traffic is not None:
        tt = measured_traffic("sweep_tail_kernel<PrecF64, false, false, false>")
        if tt is not None:  # mean bytes of the tail launches of the same sweeps
            traffic += tt["bytes"]
            kname += " + sweep_tail_kernel<PrecF64, false, false, false>"

    hbm = dict(bound="hbm", achieved=bytes_launch / sw / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
               frac=0.0, traffic=traffic, kernel=kname, algorithmic_bytes=bytes_launch,
               launch_ms=sw * 1e3)
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    copy_bw = copy_bandwidth()
    log(f"device-to-device copy: {copy_bw['GB_per_s']:.0f} GB/s")
    hbm["frac_of_copy"] = hbm["achieved"] / copy_bw["GB_per_s"]
    alu = dict(bound="alu", achieved=flops_launch / sw / 1e12, peak=FP64_OP_PEAK_T,
               unit="TFLOP/s", frac=0.0, traffic=traffic, kernel=kname,
               algorithmic_flops=flops_launch, launch_ms=sw * 1e3,
               peak_note="FP64 add/mul/div/sqrt issue rate, 256 CU x 64 lanes x 2.4 GHz")
    alu["frac"] = alu["achieved"] / alu["peak"]
    intensity = flops_launch / bytes_launch
    ridge = FP64_OP_PEAK_T * 1e12 / (HBM_PEAK_GBS * 1e9)
    roofline, other = (alu, hbm) if intensity > ridge else (hbm, alu)
    if hllc is not None and "march" in hllc["fp64"]["sweep_kernel_ms"]:
        # the same marching sweeps with the HLLC flux: their own operation count
        hops = all_ops["shocked_hllc"]["per_cell_sweep"]["flops"]
        sw_h = hllc["fp64"]["sweep_kernel_ms"]["march"] / 1e3
        fl_h = mean_pencils * n * hops
        hllc["fp64"]["roofline"] = dict(
            bound="alu", achieved=fl_h / sw_h / 1e12, peak=FP64_OP_PEAK_T, unit="TFLOP/s",
            frac=fl_h / sw_h / 1e12 / FP64_OP_PEAK_T,
            kernel=("sweep_kernel<PrecF64, false, false, true, false> + "
                    "sweep_tail_kernel<PrecF64, false, true, false>"),
            algorithmic_flops=fl_h, launch_ms=sw_h * 1e3, ops_per_cell_sweep=hops)
    if (diffusion is not None and "fp64" in diffusion
            and "march" in diffusion["fp64"]["sweep_kernel_ms"]):
        # the same marching sweeps in the general build with the diffusive flux
        dops = all_ops["shocked_diffusion"]["per_cell_sweep"]["flops"]
        sw_d = diffusion["fp64"]["sweep_kernel_ms"]["march"] / 1e3
        fl_d = mean_pencils * n * dops
        diffusion["fp64"]["roofline"] = dict(
            bound="alu", achieved=fl_d / sw_d / 1e12, peak=FP64_OP_PEAK_T, unit="TFLOP/s",
            frac=fl_d / sw_d / 1e12 / FP64_OP_PEAK_T,
            kernel=("sweep_kernel<PrecF64, false, false, true, true> + "
                    "sweep_tail_kernel<PrecF64, false, true, true>"),
            algorithmic_flops=fl_d, launch_ms=sw_d * 1e3, ops_per_cell_sweep=dops)
    if (sources is not None and "fp64" in sources
            and "march" in sources["fp64"]["sweep_kernel_ms"]):
        # the same marching sweeps in the general build with the gravity source
        # terms and the expansion factor (the expansion pass is priced on HBM)
        gops = all_ops["shocked_gravity_comoving"]["per_cell_sweep"]["flops"]
        sw_g = sources["fp64"]["sweep_kernel_ms"]["march"] / 1e3
        fl_g = mean_pencils * n * gops
        sources["fp64"]["roofline"] = dict(
            bound="alu", achieved=fl_g / sw_g / 1e12, peak=FP64_OP_PEAK_T, unit="TFLOP/s",
            frac=fl_g / sw_g / 1e12 / FP64_OP_PEAK_T,
            kernel=("sweep_kernel<PrecF64, false, false, true, true> + "
                    "sweep_tail_kernel<PrecF64, false, true, true>"),
            algorithmic_flops=fl_g, launch_ms=sw_g * 1e3, ops_per_cell_sweep=gops)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        planes = n if args.cpu_sample_planes <= 0 else min(args.cpu_sample_planes, n)
        cpu = cpu_baseline(d, n, planes, args.cpu_sample_steps)
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
                               "sigma 2, rms Mach 5, p lognormal sigma 1), gamma 5/3, ghost 3, "
                               "CFL 0.4, fill + xyz/zyx sweeps per step, the last sweep also yielding "
                               "the next CFL dt",
                   "cells": cells, "precision_of_value": "fp64", "tiles": fp["tiles"]},
        "roofline": roofline,
        "roofline_other": other,
        "sweep_kernel_ms": {k: v * 1e3 for k, v in kern.items()},
        "events": {"fallback_faces": fp["fallback_faces"], "floored_cells": fp["floored_cells"]},
        "hbm_copy": copy_bw,
    }
    if "mixed" in results:
        mx = results["mixed"]
        line["mixed"] = {"value": mx["rate"], "unit": "cell-updates/s",
                         "ms_per_step": mx["seconds"] / K * 1e3, "dtype": "f32+f64",
                         "sweep_kernel_ms": {k: v * 1e3 for k, v in mx["kern"].items()},
                         "l1_rel_vs_fp64": l1, "speedup_vs_fp64": mx["rate"] / fp["rate"],
                         "tiles": mx["tiles"]}
    if hllc is not None:
        line["hllc"] = hllc
    if diffusion is not None:
        line["diffusion"] = diffusion
    if sources is not None:
        line["gravity_comoving"] = sources
    if amr is not None:
        line["amr_ghost_fill"] = amr
    if wcyc is not None:
        line["amr_w_cycle"] = wcyc
    if batch is not None:
        line["batch"] = batch
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
