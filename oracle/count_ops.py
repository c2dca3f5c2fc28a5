"""Write the algorithmic operation counts of one PPM step per cell-sweep.

TEST/MEASUREMENT INFRASTRUCTURE: runs the oracle instantiated with its
operation-counting scalar on seeded grids of each workload recipe and stores
the mean FP64 operation counts per cell-sweep (one cell advanced by one 1-D
sweep) in paper_1307_2265_amd/data/algorithmic_ops.json, which the benchmark
reads to turn kernel time into an algorithmic FLOP rate.  A division or a
square root counts as one operation; comparisons are listed separately and
not counted as FLOPs.

    python oracle/count_ops.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1307_2265_amd import workloads as W  # noqa: E402

OUT = os.path.join(ROOT, "paper_1307_2265_amd", "data", "algorithmic_ops.json")


def count(recipe, n, seed, flags=O.ALL_FLAGS, sources=None):
    d = W.random_grid(n, n, n, seed, recipe)
    G = O.Grid(**d, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n)
    O.fill_periodic(G)
    if sources is None:
        prm = O.params(flags=flags)
    else:
        G.accel = W.acceleration_field(G.rho.shape, sources["seed"], sources["amp"])
        prm = O.params(flags=flags, a=sources["a"], adot=sources["adot"])
    dt = O.cfl_dt(G, prm)
    ops = O.count_ops(G, prm, dt, 0)
    cs = ops["cell_sweeps"]
    per = {k: ops[k] / cs for k in ("add", "mul", "div", "sqrt", "cmp")}
    per["flops"] = per["add"] + per["mul"] + per["div"] + per["sqrt"]
    return dict(grid=f"{n}^3", seed=seed, cell_sweeps=cs, per_cell_sweep=per)


def main():
    res = {
        "note": "FP64 operations per cell-sweep of one step, from the oracle's counting "
                "scalar; flops = add + mul + div + sqrt; shocked_hllc: the HLLC solver in "
                "place of two-shock; shocked_diffusion: with the diffusive flux; "
                "shocked_gravity_comoving: the sweeps with an acceleration field and "
                "a = 1.7 (the expansion step itself not included)",
        "gentle": count(W.GENTLE, 48, 1000),
        "shocked": count(W.SHOCKED, 48, 1002),
        "shocked_hllc": count(W.SHOCKED, 48, 1002, O.ALL_FLAGS | O.HLLC),
        "shocked_diffusion": count(W.SHOCKED, 48, 1002, O.ALL_FLAGS | O.DIFFUSION),
        "shocked_gravity_comoving": count(W.SHOCKED, 48, 1002, O.ALL_FLAGS,
                                          dict(seed=4242, amp=3.0, a=1.7, adot=0.6)),
    }
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
