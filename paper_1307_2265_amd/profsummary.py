"""Short text summaries of rocprofv3 runs of bench.py, for profiles/.

kernels  -- from a `rocprofv3 --kernel-trace --stats --output-format csv`
            run: per kernel (and per launch grid of the sweep kernels) the
            number of dispatches and their mean / total duration.
sq       -- from one `rocprofv3 --pmc` run of SQ counters: issue and wait
            fractions and VALU instructions per wave of the sweep kernels.
valu     -- from two `rocprofv3 --pmc` runs: the VALU instruction mix by type
            (FP64 / FP32 add, mul, fma, transcendental) with the FLOP rate it
            gives, and LDS instructions with their bank-conflict cycles.
traffic  -- from two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs:
            HBM bytes per dispatch of every kernel, each counter scaled by
            what it reads for a device-to-device copy of known size that the
            same run performs (bench.py copies every (n+2g)^3 double field of
            the grid when it resets it).  Also writes data/traffic.json, which
            bench.py reports beside its roofline as long as the kernel sources
            hash to the digest stored there.

Usage:
  python -m paper_1307_2265_amd.profsummary kernels DIR/run_kernel_stats.csv \
      DIR/run_kernel_trace.csv --cmd "..." --out profiles/x.md
  python -m paper_1307_2265_amd.profsummary traffic FETCH.csv WRITE.csv --n 512 \
      --cmd-fetch "..." --cmd-write "..." --out profiles/y.md [--json data/traffic.json]
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def kernel_source_digest() -> str:
    """sha256 over the device code (.hip, .hpp) and the build script."""
    h = hashlib.sha256()
    names = sorted(n for n in os.listdir(CSRC) if n.endswith((".hip", ".hpp"))) + ["../build.py"]
    for name in names:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short(name: str) -> str:
    base = name.split("(")[0]
    return base.replace("void ", "").replace("ppm::", "")


def kernels(stats_csv: str, trace_csv: str, cmd: str, out: str):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel durations: {os.path.basename(out)[:-3]}", "",
             "Command (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", cmd, "```", "",
             "## rocprofv3 --stats summary", "",
             "| kernel | calls | mean ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        if "sweep" not in r["Kernel_Name"] and "batch" not in r["Kernel_Name"]:  # incl. tails
            continue
        key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]),
               int(r["VGPR_Count"]), int(r["Scratch_Size"]), int(r["LDS_Block_Size"]))
        agg[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    lines += ["", "## Sweep kernels by launch grid (from the kernel trace)", "",
              "| kernel | grid threads | block | VGPRs | scratch B | LDS B | calls | mean ms |",
              "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k, d in sorted(agg.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        lines.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {k[3]} | {k[4]} | {k[5]} | {len(d)} | "
                     f"{sum(d) / len(d):.3f} |")
    # the single-grid and the batch launches of one kernel differ in block size
    byblock = collections.defaultdict(list)
    for k, d in agg.items():
        byblock[(k[0], k[2])] += d
    lines += ["", "## Mean duration per kernel and block size", "",
              "| kernel | block | calls | mean ms |", "|---|---:|---:|---:|"]
    for k, d in sorted(byblock.items()):
        lines.append(f"| `{k[0]}` | {k[1]} | {len(d)} | {sum(d) / len(d):.3f} |")
    # a marching sweep of the big grid is its marching launch plus, when
    # pencils are left over after whole rounds, a tail launch; the big grid's
    # marching launches are the largest of their kernel (other workloads, such
    # as the AMR root grid, launch the same kernel on fewer pencils), and only
    # the big grid needs tail launches
    def big_grid_mean(name):
        grids = [kk[1] for kk in agg if kk[0] == name]
        if "tail" not in name:
            grids = [max(grids)]
        d = [x for kk, dd in agg.items() if kk[0] == name and kk[1] in grids for x in dd]
        return sum(d) / len(d)
    means = {name: big_grid_mean(name) for name in {kk[0] for kk in agg}}
    sweeps = []
    for prec in ("PrecF64", "PrecMixed"):
        for cfl in ("false", "true"):
            for hllc in ("false", "true"):
                m = f"sweep_kernel<{prec}, {cfl}, false, {hllc}, false>"
                t = f"sweep_tail_kernel<{prec}, {cfl}, {hllc}, false>"
                if m not in means or t not in means:
                    continue
                sweeps.append(f"| `{m}` + `{t}` | {means[m]:.3f} | {means[t]:.3f} | "
                              f"{means[m] + means[t]:.3f} |")
    if sweeps:
        lines += ["", "## Marching sweeps of the single grid (marching launch + tail launch)", "",
                  "| launches | marching ms | tail ms | sweep ms |", "|---|---:|---:|---:|"]
        lines += sweeps
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(path: str, counter: str):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        out.append((r["Kernel_Name"], int(r["Grid_Size"]),
                    float(r["Counter_Value"]) * 1024.0))  # KiB -> bytes
    return out


def traffic(fetch_csv: str, write_csv: str, n: int, ghost: int, cmd_fetch: str, cmd_write: str,
            out: str, json_out: str | None, copy_bytes: float = float(1 << 31)):
    """copy_bytes: size of the largest device-to-device copies of the run
    (bench.py's achievable-bandwidth copy, 2 GiB), whose counter readings
    calibrate each counter."""
    F = _per_dispatch(fetch_csv, "FETCH_SIZE")
    Wr = _per_dispatch(write_csv, "WRITE_SIZE")

    def calib(rows):
        # the device-to-device copies of one whole field: the largest copies
        big = [v for name, g, v in rows if "copyBuffer" in name]
        top = max(big)
        sel = [v for v in big if v > 0.9 * top]
        return copy_bytes / (sum(sel) / len(sel)), len(sel)

    cf, nf = calib(F)
    cw, nw = calib(Wr)

    def table(rows, scale):
        agg = collections.defaultdict(list)
        for name, g, v in rows:
            if "ppm::" in name:
                agg[(short(name), g)].append(v * scale)
        return agg

    TF, TW = table(F, cf), table(Wr, cw)
    lines = [f"# HBM bytes per dispatch: {os.path.basename(out)[:-3]}", "",
             "Commands (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", cmd_fetch, cmd_write, "```", "",
             f"Calibration: the largest device-to-device copies of the run move "
             f"{copy_bytes / 1e9:.4f} GB each (the benchmark's achievable-bandwidth copy); "
             f"FETCH_SIZE reads "
             f"{copy_bytes / cf / 1e9:.4f} GB for such a copy ({nf} copies), WRITE_SIZE "
             f"{copy_bytes / cw / 1e9:.4f} GB ({nw} copies).  Scale factors: fetch x{cf:.4f}, "
             f"write x{cw:.4f}.", "",
             "| kernel | grid threads | dispatches | fetch GB | write GB | total GB |",
             "|---|---:|---:|---:|---:|---:|"]
    summary = {}
    for key in sorted(TF, key=lambda k: (k[0], -k[1])):
        f = sum(TF[key]) / len(TF[key])
        w = sum(TW.get(key, [0.0])) / max(1, len(TW.get(key, [])))
        lines.append(f"| `{key[0]}` | {key[1]} | {len(TF[key])} | {f / 1e9:.3f} | {w / 1e9:.3f} | "
                     f"{(f + w) / 1e9:.3f} |")
        s = summary.setdefault(key[0], {"fetch": [], "write": []})
        s["fetch"] += TF[key]
        s["write"] += TW.get(key, [])
    lines += ["", "Mean over all dispatches of a kernel:", "",
              "| kernel | fetch GB | write GB | total GB |", "|---|---:|---:|---:|"]
    per_kernel = {}
    for k, s in sorted(summary.items()):
        f = sum(s["fetch"]) / len(s["fetch"])
        w = sum(s["write"]) / max(1, len(s["write"]))
        per_kernel[k] = {"fetch_bytes": f, "write_bytes": w, "bytes": f + w,
                         "dispatches": len(s["fetch"])}
        lines.append(f"| `{k}` | {f / 1e9:.3f} | {w / 1e9:.3f} | {(f + w) / 1e9:.3f} |")
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    if json_out:
        with open(json_out, "w") as fo:
            json.dump({"source_digest": kernel_source_digest(), "workload_n": n, "ghost": ghost,
                   "calibration_copy_bytes": copy_bytes,
                       "fetch_scale": cf, "write_scale": cw, "profile": os.path.basename(out),
                       "kernels": per_kernel}, fo, indent=1)


def sq(counters_csv: str, cmd: str, out: str):
    """Per dispatch group (kernel, grid): per-wave fractions of SQ_WAVE_CYCLES
    issuing VALU / anything, waiting on memory counters, ready but not issued,
    and VALU instructions per wave."""
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    n = collections.Counter()
    for r in csv.DictReader(open(counters_csv)):
        k = (short(r["Kernel_Name"]), int(r["Grid_Size"]), int(r["Workgroup_Size"]))
        agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
        if r["Counter_Name"] == "SQ_WAVES":
            n[k] += 1
    lines = [f"# SQ counters: {os.path.basename(out)[:-3]}", "",
             "Command (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", cmd, "```", "",
             "Per dispatch group (kernel, grid threads): per-wave fractions of SQ_WAVE_CYCLES spent "
             "issuing VALU (SQ_ACTIVE_INST_VALU), issuing anything (SQ_ACTIVE_INST_ANY), waiting on "
             "a memory counter (SQ_WAIT_ANY) and ready but not issued (SQ_WAIT_INST_ANY); VALU "
             "instructions per wave.  With w waves per SIMD sharing one VALU, w x the VALU fraction "
             "is the SIMD's VALU occupancy (the marching kernels hold 2 waves per SIMD, the lane "
             "kernels 4; values slightly above 1 come from the counters' cycle granularity).", "",
             "| kernel | grid threads | block | dispatches | waves | VALU | any | wait mem | "
             "wait issue | VALU instr / wave |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k, c in sorted(agg.items()):
        if "sweep" not in k[0]:
            continue
        wc = c["SQ_WAVE_CYCLES"]
        lines.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {n[k]} | {c['SQ_WAVES'] / n[k]:.0f} | "
                     f"{c['SQ_ACTIVE_INST_VALU'] / wc:.2f} | {c['SQ_ACTIVE_INST_ANY'] / wc:.2f} | "
                     f"{c['SQ_WAIT_ANY'] / wc:.2f} | {c['SQ_WAIT_INST_ANY'] / wc:.2f} | "
                     f"{c['SQ_INSTS_VALU'] / c['SQ_WAVES']:.0f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def valu(flops_csv: str, lds_csv: str, cmd_flops: str, cmd_lds: str, out: str):
    """Per dispatch group of the sweep kernels: FP64 and FP32 VALU
    instructions by type (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F{64,32}) and the
    FLOP rate they give, 64 lanes x (ADD + MUL + 2 FMA + TRANS) per
    instruction over the dispatch's own duration (an upper bound on the
    lane-level rate: the counters do not see the execution mask), against the
    published vector peaks; LDS instructions and bank-conflict cycles."""
    def load(path):
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(dict)
        for r in csv.DictReader(open(path)):
            k = (short(r["Kernel_Name"]), int(r["Grid_Size"]), int(r["Workgroup_Size"]))
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        return agg, disp
    fa, fd = load(flops_csv)
    la, ld = load(lds_csv)
    lines = [f"# VALU mix, FLOP rate and LDS conflicts: {os.path.basename(out)[:-3]}", "",
             "Commands (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```", cmd_flops, cmd_lds, "```", "",
             "FP64 (FP32) FLOP per dispatch = 64 x (ADD + MUL + 2 FMA + TRANS) over the "
             "SQ_INSTS_VALU_*_F64 (_F32) counters, an upper bound on the lane-level count (the "
             "counters count wave instructions whatever the execution mask); rate over the mean "
             "duration of the same dispatches in the counter run; peaks: FP64 vector 78.6 TFLOP/s, "
             "FP32 vector 157.3 TFLOP/s (an FMA counted as two).  The hot path compiles with "
             "-ffp-contract=off, so it issues separate adds and multiplies, and its FMAs are the "
             "Newton and remainder steps of divisions and square roots.", "",
             "| kernel | grid threads | dispatches | mean ms | F64 add / mul / fma / trans (M instr) "
             "| FP64 TFLOP/s (frac) | F32 add / mul / fma / trans (M instr) | FP32 TFLOP/s (frac) |",
             "|---|---:|---:|---:|---|---:|---|---:|"]
    for k, c in sorted(fa.items()):
        if "sweep" not in k[0] and "persistent" not in k[0]:
            continue
        nd = len(fd[k])
        ms = sum(fd[k].values()) / nd / 1e6
        def mix(t):
            v = [c[f"SQ_INSTS_VALU_{op}_{t}"] / nd / 1e6 for op in ("ADD", "MUL", "FMA", "TRANS")]
            flop = 64e6 * (v[0] + v[1] + 2 * v[2] + v[3])
            return v, flop / (ms / 1e3) / 1e12
        v64, r64 = mix("F64")
        v32, r32 = mix("F32")
        lines.append(f"| `{k[0]}` | {k[1]} | {nd} | {ms:.3f} | "
                     + " / ".join(f"{x:.1f}" for x in v64) + f" | {r64:.2f} ({r64 / 78.6:.3f}) | "
                     + " / ".join(f"{x:.1f}" for x in v32) + f" | {r32:.2f} ({r32 / 157.3:.3f}) |")
    lines += ["", "LDS: instructions per dispatch, cycles issuing LDS and bank-conflict cycles "
              "(SQ_INSTS_LDS, SQ_ACTIVE_INST_LDS, SQ_LDS_BANK_CONFLICT), and the conflict cycles "
              "as a fraction of the LDS issue cycles.", "",
              "| kernel | grid threads | dispatches | LDS instr (M) | LDS issue cycles (M) | "
              "bank-conflict cycles (M) | conflict / issue |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for k, c in sorted(la.items()):
        if "sweep" not in k[0] and "persistent" not in k[0]:
            continue
        nd = len(ld[k])
        act = c["SQ_ACTIVE_INST_LDS"] / nd / 1e6
        bc = c["SQ_LDS_BANK_CONFLICT"] / nd / 1e6
        lines.append(f"| `{k[0]}` | {k[1]} | {nd} | {c['SQ_INSTS_LDS'] / nd / 1e6:.2f} | "
                     f"{act:.2f} | {bc:.3f} | {bc / act if act else 0.0:.3f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    q = sub.add_parser("sq")
    q.add_argument("counters")
    q.add_argument("--cmd", required=True)
    q.add_argument("--out", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("stats")
    k.add_argument("trace")
    k.add_argument("--cmd", required=True)
    k.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--n", type=int, default=512)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 31))
    t.add_argument("--ghost", type=int, default=3)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--json", default=None)
    v = sub.add_parser("valu")
    v.add_argument("flops")
    v.add_argument("lds")
    v.add_argument("--cmd-flops", required=True)
    v.add_argument("--cmd-lds", required=True)
    v.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.mode == "sq":
        sq(a.counters, a.cmd, a.out)
    elif a.mode == "kernels":
        kernels(a.stats, a.trace, a.cmd, a.out)
    elif a.mode == "valu":
        valu(a.flops, a.lds, a.cmd_flops, a.cmd_lds, a.out)
    else:
        traffic(a.fetch, a.write, a.n, a.ghost, a.cmd_fetch, a.cmd_write, a.out, a.json,
                a.copy_bytes)


if __name__ == "__main__":
    main()
