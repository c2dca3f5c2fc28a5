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

Also measured on the GPU: the gentle 256^3 grid for 10 steps (rate and
algorithmic HBM bandwidth); the 512^3 grid with the HLLC solver, with the
optional diffusive flux, and with gravity and comoving terms; the AMR patch
ghost fill and the W-cycle on a nested hierarchy; the batched form (4096
uneven AMR patches, one captured HIP graph per step) and its rate relative to
the single grid; the cosmology-shaped hierarchy (1024^3 root + 20000 patches
on levels 1-8, one captured graph per step: fill, CFL, step); the roofline
of the dominant kernels (FP64 and mixed marching sweeps) from HIP events on
their launch stream.

Then on the host, the oracle (plain FP64 C++, all host threads): the 512^3
grid for all K steps from the same input -- its own CFL timestep each step --
against which the FP64 path (same timesteps, which it must reproduce) and the
mixed path (driven by the same timestep sequence) are compared after 1 and K
steps; and the oracle's rates on the other workloads (one thread on 32^3 and
on one step of 256^3, all threads on 256^3, the batch and a sample of the
hierarchy).

Prints ONE JSON line: FP64 cell-updates/s of the single grid as `value` (one
cell-update = one active cell through the x, y and z sweeps of one step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0         # MI355X HBM3E, GB/s (published)
FP64_PEAK_T = 78.6            # MI355X FP64 vector, TFLOP/s (published; an FMA counts two)
FP32_PEAK_T = 157.3           # MI355X FP32 vector, TFLOP/s (published)
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 39.3 T
# instructions/s.  The FP64 path is built without contraction (it reproduces
# the oracle bit for bit), so its adds, multiplies, divisions and square roots
# each take at least one issue: a secondary ceiling, stated beside the
# published one.
FP64_ISSUE_T = 256 * 4 * 16 * 2.4e9 / 1e12
FIELDS = ("rho", "vx", "vy", "vz", "etot", "eint")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="active cells per axis")
    ap.add_argument("--npatch", type=int, default=4096, help="patches of the batch (0: skip)")
    ap.add_argument("--quick", action="store_true",
                    help="the single grid and the batch only (no oracle, no other legs)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--tiles", default=None, help="tile_config of the single-grid plans")
    ap.add_argument("--batch-tiles", default=None, help="tile_config of the batch plans")
    ap.add_argument("--no-hllc", action="store_true", help="skip the HLLC-solver runs")
    ap.add_argument("--no-amr-fill", action="store_true", help="skip the AMR ghost-fill timing")
    ap.add_argument("--no-amr-step", action="store_true", help="skip the AMR W-cycle timing")
    ap.add_argument("--no-diffusion", action="store_true",
                    help="skip the runs with the diffusive flux")
    ap.add_argument("--amr-step-only", action="store_true",
                    help="only the AMR W-cycle timing (for profiling it)")
    ap.add_argument("--no-sources", action="store_true",
                    help="skip the runs with gravity and comoving terms")
    ap.add_argument("--no-gentle256", action="store_true", help="skip the 256^3 leg")
    ap.add_argument("--no-cosmology", action="store_true",
                    help="skip the 1024^3 + 20000-patch hierarchy")
    a = ap.parse_args()
    if a.quick:
        a.no_cpu_baseline = a.no_hllc = a.no_amr_fill = a.no_amr_step = True
        a.no_diffusion = a.no_sources = a.no_gentle256 = a.no_cosmology = True
    return a


def timed_single(d, n, prec, K, Wm, tiles, flags=None, sources=None):
    """K timed steps of the single grid (after Wm warm-up steps from the same
    input), sweeps bracketed by HIP events; returns (result dict, Run)."""
    import torch
    from paper_1307_2265_amd import harness as H
    r = H.Run.single(d, n, prec, tiles, flags=flags, sources=sources)
    for s in range(Wm):
        r.step(s)
    torch.cuda.synchronize()
    r.reset()
    r.plan.ppm_event_counts(reset=True)
    total, kern = r.timed(K, per_sweep=True)
    fb, fl = r.plan.ppm_event_counts()
    cells = n ** 3
    return dict(seconds=total, kern=kern, rate=cells * K / total, tiles=tiles,
                fallback_faces=fb, floored_cells=fl), r


def sweep_work(n: int, lanes_x: bool = True):
    """Mean pencils of one marching sweep of the n^3 grid (the y sweeps and the
    z sweeps; x sweeps go to the lane kernel) and its algorithmic cells."""
    g = 3
    nf = n + 2 * g
    if lanes_x:
        mean_pencils = (n * nf + nf * nf + n * nf) / 3.0
    else:
        mean_pencils = (nf * nf + n * nf) / 2.0
    return mean_pencils, nf


def gentle256(K: int = 10, Wm: int = 2) -> dict:
    """The gentle 256^3 grid (seed 1001), FP64, K steps with the CFL timestep
    from the device each step: rate and algorithmic HBM bandwidth."""
    import torch
    from paper_1307_2265_amd import autotune, ppm
    from paper_1307_2265_amd import harness as H
    n = 256
    d = H.single_grid_input(n, "gentle256")
    tiles = autotune.best_tiles("single/fp64")
    r = H.Run.single(d, n, ppm.PPM_FP64, tiles)
    for s in range(Wm):
        r.step(s)
    torch.cuda.synchronize()
    r.reset()
    total, _ = r.timed(K)
    r.close()
    torch.cuda.empty_cache()
    byt = H.step_bytes([(n, n, n)], 48.0, 48.0) * K
    gbs = byt / total / 1e9
    return {"workload": "single 256^3 periodic grid, rho lognormal sigma 0.5, rms velocity 0.5 "
                        "c_s per component, p = 1 +- 10 %, seed 1001, FP64, CFL timestep reduced on "
                        "the device each step (folded into the last sweep)",
            "steps": K, "value": n ** 3 * K / total, "unit": "cell-updates/s",
            "ms_per_step": total / K * 1e3, "tiles": tiles,
            "hbm": {"algorithmic_bytes_per_step": byt / K, "achieved_GBps": gbs,
                    "peak_GBps": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
                    "bytes_note": "per sweep, 48 B read for each of a pencil's n+6 cells and "
                                  "48 B written for each of its n active cells, over the sweep "
                                  "extents (mean of the xyz and zyx orders)"}}


def cosmology(prec_name: str, steps: int = 3, warmup: int = 1, want_sample: bool = False):
    """The cosmology-shaped hierarchy: 1024^3 periodic root and 20000 patches
    of 16^3-48^3 on levels 1-8, advanced by one captured graph per step (the
    root's periodic fill, the per-level CFL reduction and the step)."""
    import torch
    from paper_1307_2265_amd import ppm
    from paper_1307_2265_amd import harness as H
    prec = ppm.PPM_FP64 if prec_name == "fp64" else ppm.PPM_MIXED
    t0 = time.time()
    h = H.Hierarchy(prec, log=log)
    log(f"cosmology {prec_name}: hierarchy built in {time.time() - t0:.1f}s, "
        f"{h.cells / 1e9:.3f} G active cells")
    plan = ppm.Plan(h.patches, h.NLEV, prec, ppm.params())
    dt = torch.zeros(h.NLEV, dtype=torch.float64, device="cuda")
    parts = ppm.PPM_GRAPH_FILL | ppm.PPM_GRAPH_CFL | ppm.PPM_GRAPH_STEP
    graphs = [ppm.Graph(plan, dt, o, parts) for o in (0, 1)]
    for s in range(warmup):
        graphs[s % 2].ppm_graph_launch()
    torch.cuda.synchronize()
    plan.ppm_event_counts(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(steps):
        graphs[(warmup + s) % 2].ppm_graph_launch()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    fb, fl = plan.ppm_event_counts()
    sb = 4.0 if prec_name == "mixed" else 8.0
    cell_b = 4 * sb + 16.0
    byt = (H.step_bytes(h.dims, cell_b, cell_b) + h.cells * cell_b) * steps  # + CFL read
    gbs = byt / sec / 1e9
    for g in graphs:
        g.close()
    plan.close()
    sample = None
    if want_sample:  # host copies for the oracle's rate: a 16-plane root slab, 200 patches
        G3 = h.ghost
        grids = [({f: h.root[f][:16 + 2 * G3].double().cpu().numpy() for f in FIELDS},
                  1.0 / h.n_root, True)]
        for i in range(200):
            s = h.specs[i]
            shape = (s.nz + 2 * G3, s.ny + 2 * G3, s.nx + 2 * G3)
            grids.append(({f: h.flat[f][h.offs[i]:h.offs[i + 1]].view(shape).double().cpu().numpy()
                           for f in FIELDS}, s.dx, False))
        sample = {"grids": grids, "what": "1 step of a 1024x1024x16 slab of the root (periodic "
                                          "in itself) and of 200 patches, after the timed steps"}
    out = {"workload": "1024^3 periodic root (log-normal Gaussian random field density, "
                       "sigma 1.5, P(k) ~ k^-2; cold bulk flows, kinetic/thermal up to 1e6) + "
                       "20000 patches of 16^3-48^3 on levels 1-8, ghosts injected from the root; "
                       "one captured graph per step (fill, CFL, step)",
           "precision": prec_name, "active_cells": h.cells, "steps": steps,
           "value": h.cells * steps / sec, "unit": "cell-updates/s",
           "ms_per_step": sec / steps * 1e3,
           "hbm": {"algorithmic_bytes_per_step": byt / steps, "achieved_GBps": gbs,
                   "peak_GBps": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS},
           "events": {"fallback_faces": fb, "floored_cells": fl}}
    del h
    torch.cuda.empty_cache()
    return out, sample


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




def parity_runs(d, n: int, K: int) -> dict:
    """Untimed GPU runs of the headline grid for the comparison with the
    oracle: FP64 with its own CFL timestep each step (recorded), and mixed
    precision driven by the same timestep sequence, so that both are compared
    at the oracle's times.  Host copies of the active fields after step 1
    and step K."""
    import torch
    from paper_1307_2265_amd import ppm
    from paper_1307_2265_amd import harness as H
    out = {"dts": [], "fp64": {}, "mixed": {}}
    shape = d["rho"].shape
    keep = {1, K}

    def snap(r):
        return {f: H.active(r.flat[f].view(shape)).cpu().numpy() for f in FIELDS}

    r = H.Run.single(d, n, ppm.PPM_FP64)
    r.ensure_dt()
    for s in range(K):
        out["dts"].append(float(r.dt.item()))
        r.step(s)
        if s + 1 in keep:
            torch.cuda.synchronize()
            out["fp64"][s + 1] = snap(r)
    r.close()
    del r
    torch.cuda.empty_cache()
    rm = H.Run.single(d, n, ppm.PPM_MIXED)
    for s in range(K):
        rm.dt.fill_(out["dts"][s])
        rm.plan.ppm_fill_periodic()
        rm.plan.ppm_step(rm.dt, s % 2)
        if s + 1 in keep:
            torch.cuda.synchronize()
            out["mixed"][s + 1] = snap(rm)
    rm.close()
    del rm
    torch.cuda.empty_cache()
    return out


def _fp64_worst(g: dict, o: dict) -> dict:
    """Worst |g - o| / max(|o|, mean |o| of the field) and the cells not equal
    bit for bit, over the six fields."""
    import numpy as np
    worst, differ = 0.0, 0
    for f in FIELDS:
        a, b = g[f], o[f]
        scale = max(float(np.abs(b).mean()), 1e-300)
        err = np.abs(a - b) / np.maximum(np.abs(b), scale)
        worst = max(worst, float(err.max()))
        differ += int(np.count_nonzero(a != b))
    return {"worst_rel": worst, "cells_not_bitwise_equal": differ}


def _l1(g: dict, o: dict) -> dict:
    import numpy as np
    return {f: float(np.abs(g[f].astype(np.float64) - o[f]).sum() / np.abs(o[f]).sum())
            for f in FIELDS}


def oracle_headline(d, n: int, K: int, par: dict) -> dict:
    """The oracle on all host threads, K steps of the headline grid from the
    same stored input, its own CFL timestep each step (fill, CFL and sweeps
    timed); the FP64 path's timesteps and states and the mixed path's states
    compared with it after step 1 and step K."""
    import numpy as np
    import oracle as O
    from paper_1307_2265_amd import harness as H
    G = O.Grid(**{f: np.array(d[f], dtype=np.float64, copy=True) for f in FIELDS},
               dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
    prm = O.params()
    el, dts = 0.0, []
    comp = {}
    for s in range(K):
        t0 = time.perf_counter()
        O.fill_periodic(G)
        dt = O.cfl_dt(G, prm)
        O.step(G, prm, dt, s % 2)
        el += time.perf_counter() - t0
        dts.append(dt)
        log(f"oracle {n}^3 step {s + 1}/{K}: {time.perf_counter() - t0:.1f}s")
        if s + 1 in par["fp64"]:
            o = {f: H.active(getattr(G, f)) for f in FIELDS}
            comp[f"after_{s + 1}_steps"] = {"fp64": _fp64_worst(par["fp64"][s + 1], o),
                                            "mixed_l1_rel": _l1(par["mixed"][s + 1], o)}
    same = [a == b for a, b in zip(dts, par["dts"])]
    cores = O.num_threads()
    return {"value": n ** 3 * K / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"all {K} steps of the full {n}^3 headline grid (same stored input, its "
                      f"own CFL timestep each step; fill, CFL and sweeps timed), FP64, "
                      f"{el:.1f}s wall",
            "comparison": {"timesteps_equal_fp64_path": f"{sum(same)}/{K}", **comp}}


def oracle_rate(grids: list, steps: int, threads: int | None = None) -> tuple:
    """(active cell-updates/s, seconds) of the oracle over `steps` steps of
    every grid (a list of (field dict, dx, periodic)), patch by patch."""
    import numpy as np
    import oracle as O
    prm = O.params()
    keep = O.num_threads()
    if threads:
        O.set_num_threads(threads)
    el, cells = 0.0, 0
    for d, dx, periodic in grids:
        G = O.Grid(**{f: np.array(d[f], dtype=np.float64, copy=True) for f in FIELDS},
                   dx=dx, dy=dx, dz=dx)
        nz, ny, nx = (s - 6 for s in d["rho"].shape)
        for s in range(steps):
            t0 = time.perf_counter()
            if periodic:
                O.fill_periodic(G)
            dt = O.cfl_dt(G, prm)
            O.step(G, prm, dt, s % 2)
            el += time.perf_counter() - t0
            cells += nx * ny * nz
    O.set_num_threads(keep)
    return cells / el, el


def oracle_other(cosmo_sample) -> dict:
    """The oracle's rate on the other workloads: one host thread on the 32^3
    grid and on one step of the 256^3 grid; all threads on 10 steps of the
    256^3 grid, one step of the 4096-patch batch (patch by patch) and one step
    of a sample of the cosmology-shaped hierarchy."""
    from paper_1307_2265_amd import harness as H
    out = {}
    d32 = H.single_grid_input(32, "gentle32")
    v, el = oracle_rate([(d32, 1.0 / 32, True)], 1, threads=1)
    out["gentle32_single_thread"] = {"value": v, "cores": 1, "sample": f"1 step, {el:.2f}s"}
    d256 = H.single_grid_input(256, "gentle256")
    v, el = oracle_rate([(d256, 1.0 / 256, True)], 1, threads=1)
    out["gentle256_single_thread"] = {"value": v, "cores": 1, "sample": f"1 step, {el:.1f}s"}
    log(f"oracle 256^3 one thread: {v / 1e6:.2f} M cell-updates/s")
    v, el = oracle_rate([(d256, 1.0 / 256, True)], 10)
    out["gentle256"] = {"value": v, "sample": f"10 steps, {el:.1f}s"}
    log(f"oracle 256^3 all threads: {v / 1e6:.2f} M cell-updates/s")
    specs, fields = H.batch_input(4096)
    v, el = oracle_rate([(f, sp.dx, False) for f, sp in zip(fields, specs)], 1)
    out["batch4096"] = {"value": v, "sample": f"1 step of all 4096 patches, patch by patch, "
                                              f"{el:.1f}s"}
    log(f"oracle batch: {v / 1e6:.2f} M cell-updates/s")
    if cosmo_sample is not None:
        v, el = oracle_rate(cosmo_sample["grids"], 1)
        out["cosmology_sample"] = {"value": v, "sample": cosmo_sample["what"] + f", {el:.1f}s"}
        log(f"oracle hierarchy sample: {v / 1e6:.2f} M cell-updates/s")
    for k in out:
        out[k]["unit"] = "cell-updates/s"
    return out


def roofline_of(kern_ms: float, n: int, sb: float, flops: float, kname: str, traffic) -> dict:
    """Roofline of one plain marching sweep of the n^3 grid (the unit is the
    sweep: its marching launch plus, when pencils are left over, its tail
    launch).  Algorithmic bytes: every pencil reads its n+6 cells and writes
    its n active ones (sb = bytes per cell: 48 FP64, 32 mixed); algorithmic
    operations: the oracle's count per cell-sweep times the cells written."""
    mean_pencils, nf = sweep_work(n)
    byt = mean_pencils * (nf + n) * sb
    ops = mean_pencils * n * flops
    sec = kern_ms / 1e3
    gbs = byt / sec / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
            "algorithmic_bytes": byt, "launch_ms": kern_ms,
            "ops": {"algorithmic_ops": ops, "T_op_per_s": ops / sec / 1e12,
                    "ops_per_cell_sweep": flops,
                    "note": "the oracle's adds, multiplies, divisions and square roots"}}


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

    # ---- headline: the single grid, FP64 and mixed
    results = {}
    for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
        if name == "mixed" and args.no_mixed:
            continue
        tiles = args.tiles or autotune.best_tiles(f"single/{name}")
        log(f"{name}: timing {K} steps (tiles {tiles})")
        res, r = timed_single(d, n, prec, K, Wm, tiles)
        r.close()
        results[name] = res
        log(f"{name}: {K} steps in {res['seconds']:.3f}s -> {res['rate'] / 1e9:.3f} G "
            "cell-updates/s, " + ", ".join(f"{k} sweep {v * 1e3:.3f} ms"
                                           for k, v in res["kern"].items()))
    torch.cuda.empty_cache()

    # ---- the same grid with the HLLC solver, the diffusive flux, gravity
    def variant(tag, **kw):
        out = {}
        for name, prec in (("fp64", ppm.PPM_FP64), ("mixed", ppm.PPM_MIXED)):
            if name == "mixed" and args.no_mixed:
                continue
            tiles = args.tiles or autotune.best_tiles(f"single/{name}")
            res, r = timed_single(d, n, prec, K, Wm, tiles, **kw)
            r.close()
            out[name] = {"value": res["rate"], "unit": "cell-updates/s",
                         "ms_per_step": res["seconds"] / K * 1e3, "tiles": tiles,
                         "sweep_kernel_ms": {k: v * 1e3 for k, v in res["kern"].items()},
                         "relative_to_plain": results[name]["seconds"] / res["seconds"],
                         "events": {"fallback_faces": res["fallback_faces"],
                                    "floored_cells": res["floored_cells"]}}
            log(f"{tag} {name}: {res['rate'] / 1e9:.3f} G cell-updates/s")
        torch.cuda.empty_cache()
        return out

    hllc = diffusion = sources = None
    if not args.no_hllc:
        hllc = {"flags": "PPM_ALL_FLAGS | PPM_HLLC",
                **variant("hllc", flags=ppm.PPM_ALL_FLAGS | ppm.PPM_HLLC)}
    if not args.no_diffusion:
        diffusion = {"flags": "PPM_ALL_FLAGS | PPM_DIFFUSION",
                     **variant("diffusion", flags=ppm.PPM_ALL_FLAGS | ppm.PPM_DIFFUSION)}
    if not args.no_sources:
        src = dict(seed=4242, amp=3.0, a=1.7, adot=0.6)
        sources = {"recipe": "acceleration: 4 random plane waves per component over the "
                             "ghosted box, amplitude 3; a = 1.7, adot = 0.6",
                   **variant("sources", sources=src)}
        for name in ("fp64", "mixed"):
            if name in sources and "expansion" in sources[name]["sweep_kernel_ms"]:
                ex_ms = sources[name]["sweep_kernel_ms"]["expansion"]
                ex_b = cells * 2 * (3 * (8 if name == "fp64" else 4) + 2 * 8)
                sources[name]["expansion"] = {"ms": ex_ms, "bytes": ex_b,
                                              "GB_per_s": ex_b / (ex_ms / 1e3) / 1e9,
                                              "frac_of_hbm_peak":
                                                  ex_b / (ex_ms / 1e3) / 1e9 / HBM_PEAK_GBS}

    g256 = None
    if not args.no_gentle256:
        g256 = gentle256()
        log(f"gentle 256^3: {g256['value'] / 1e9:.3f} G cell-updates/s, "
            f"{g256['hbm']['achieved_GBps']:.0f} GB/s algorithmic")
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
                           "active_cells": r.cells,
                           "single_over_batch": results[name]["rate"] / (r.cells * K / total)}
            log(f"batch {name}: {r.cells * K / total / 1e9:.3f} G cell-updates/s, single/batch "
                f"{batch[name]['single_over_batch']:.3f}")
            bruns[name] = r
        if "mixed" in bruns:
            batch["mixed"]["l1_rel_vs_fp64"] = H.l1_per_field(bruns["mixed"], bruns["fp64"])
        for r in bruns.values():
            r.close()
        del bruns
        torch.cuda.empty_cache()

    # ---- the cosmology-shaped hierarchy, one captured graph per step
    cosmo, cosmo_sample = None, None
    if not args.no_cosmology:
        cosmo = {}
        for name in ("mixed", "fp64"):
            cosmo[name], smp = cosmology(name, want_sample=(name == "mixed"
                                                            and not args.no_cpu_baseline))
            cosmo_sample = cosmo_sample or smp
            log(f"cosmology {name}: {cosmo[name]['value'] / 1e9:.3f} G cell-updates/s, "
                f"{cosmo[name]['hbm']['achieved_GBps']:.0f} GB/s algorithmic")

    # ---- rooflines of the dominant kernels (the plain marching sweep)
    def tr_of(prec_name):
        base = f"sweep_kernel<Prec{'F64' if prec_name == 'fp64' else 'Mixed'}, false, false, false, false>"
        tail = f"sweep_tail_kernel<Prec{'F64' if prec_name == 'fp64' else 'Mixed'}, false, false, false>"
        a, b = measured_traffic(base), measured_traffic(tail)
        if a is None:
            return None, base + " + " + tail
        return a["bytes"] + (b["bytes"] if b else 0.0), base + " + " + tail

    traffic, kname = tr_of("fp64")
    roofline = roofline_of(results["fp64"]["kern"]["march"] * 1e3, n, 48.0, ops["flops"], kname,
                           traffic)
    roofline["fp64_vector"] = {"achieved": roofline["ops"]["T_op_per_s"], "peak": FP64_PEAK_T,
                               "unit": "TFLOP/s",
                               "frac": roofline["ops"]["T_op_per_s"] / FP64_PEAK_T,
                               "note": "algorithmic operations against the published FP64 "
                                       "vector peak (which counts an FMA as two)"}
    roofline["fp64_issue"] = {"achieved": roofline["ops"]["T_op_per_s"], "peak": FP64_ISSUE_T,
                              "unit": "T op/s",
                              "frac": roofline["ops"]["T_op_per_s"] / FP64_ISSUE_T,
                              "note": "secondary: 256 CU x 4 SIMD x 16 FP64 lanes x 2.4 GHz, one "
                                      "issue per add, multiply, division or square root (the "
                                      "FP64 path is built without contraction)"}
    copy_bw = copy_bandwidth()
    log(f"device-to-device copy: {copy_bw['GB_per_s']:.0f} GB/s")
    roofline["frac_of_copy"] = roofline["achieved"] / copy_bw["GB_per_s"]
    mixed = None
    if "mixed" in results:
        mx = results["mixed"]
        mtr, mkname = tr_of("mixed")
        mroof = roofline_of(mx["kern"]["march"] * 1e3, n, 32.0, ops["flops"], mkname, mtr)
        mroof["frac_of_copy"] = mroof["achieved"] / copy_bw["GB_per_s"]
        mixed = {"value": mx["rate"], "unit": "cell-updates/s",
                 "ms_per_step": mx["seconds"] / K * 1e3, "dtype": "f32+f64",
                 "sweep_kernel_ms": {k: v * 1e3 for k, v in mx["kern"].items()},
                 "speedup_vs_fp64": mx["rate"] / results["fp64"]["rate"],
                 "tiles": mx["tiles"], "roofline": mroof,
                 "events": {"fallback_faces": mx["fallback_faces"],
                            "floored_cells": mx["floored_cells"]}}

    # ---- the oracle on the host
    cpu, oracle_other_rates = None, None
    if not args.no_cpu_baseline:
        log(f"untimed FP64 and mixed runs of {K} steps for the comparison with the oracle")
        par = parity_runs(d, n, K)
        log(f"oracle: {K} steps of the {n}^3 grid on the host")
        cpu = oracle_headline(d, n, K, par)
        del par
        log(f"oracle: {cpu['value'] / 1e6:.2f} M cell-updates/s on {cpu['cores']} threads; "
            f"comparison {json.dumps(cpu['comparison'])}")
        oracle_other_rates = oracle_other(cosmo_sample)
        cpu["other_workloads"] = oracle_other_rates
        if mixed is not None:
            mixed["l1_rel_vs_oracle"] = {k: v["mixed_l1_rel"] for k, v in
                                         cpu["comparison"].items() if k.startswith("after_")}

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
        "sweep_kernel_ms": {k: v * 1e3 for k, v in fp["kern"].items()},
        "events": {"fallback_faces": fp["fallback_faces"], "floored_cells": fp["floored_cells"]},
        "hbm_copy": copy_bw,
    }
    for key, val in (("mixed", mixed), ("gentle256", g256), ("hllc", hllc),
                     ("diffusion", diffusion), ("gravity_comoving", sources),
                     ("amr_ghost_fill", amr), ("amr_w_cycle", wcyc), ("batch", batch),
                     ("cosmology", cosmo), ("cpu_baseline", cpu)):
        if val is not None:
            line[key] = val
    print(json.dumps(line))


if __name__ == "__main__":
    main()
