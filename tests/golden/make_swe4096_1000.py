"""Writes swe4096_1000steps.json: the CPU FP64 oracle's state after 1000
steps of the 4096 x 4096 reflective-wall Gaussian-bump workload (8 bumps,
seed 2, g 9.8, dx 1, CFL 0.5), for the paper's scheme and the transverse
scheme, each started from the FP64 initial state and from its FP32 rounding
(what an FP32 run starts from).  Stored per run: the time reached, per-field
sums, 2-norms and max-norms over the interior, and the values at a 16 x 16
lattice of cells (corners and edges included).

Calls only oracle/ (and the seeded initial-state generator).  Four runs of
about 10 minutes each, in parallel processes:

    python tests/golden/make_swe4096_1000.py
"""
from __future__ import annotations

import json
import math
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "swe4096_1000steps.json")

N, STEPS, SEED = 4096, 1000, 2
LATTICE = [int(round(x)) for x in np.linspace(0, N - 1, 16)]


def run(args):
    scheme, start = args
    import oracle
    from paper_1107_2157_amd import ics
    h, hu, hv = (a.numpy() for a in ics.bumps_state(N, N, seed=SEED, periodic=False, count=8))
    if start == "f32":
        h, hu, hv = (a.astype(np.float32).astype(np.float64) for a in (h, hu, hv))
    H, U, V, t = oracle.run(h, hu, hv, STEPS, scheme=scheme, raise_unstable=False)
    fields = {}
    for name, a in (("h", H), ("hu", U), ("hv", V)):
        x = a[1:-1, 1:-1]
        fields[name] = {"sum": math.fsum(x.ravel()), "l2": float(np.sqrt(np.sum(x * x))),
                        "max_abs": float(np.max(np.abs(x))),
                        "lattice": [[float(x[j, i]) for i in LATTICE] for j in LATTICE]}
    return {"scheme": "paper" if scheme == 0 else "transverse", "start": start, "t": t,
            "finite": bool(np.all(np.isfinite(H)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))),
            "fields": fields}


def main():
    jobs = [(s, st) for s in (0, 1) for st in ("f64", "f32")]
    with mp.Pool(len(jobs)) as pool:
        runs = pool.map(run, jobs)
    doc = {"workload": "4096x4096, reflective walls, 8 Gaussian bumps (seed 2), g 9.8, dx = dy = 1, CFL 0.5",
           "steps": STEPS, "lattice": LATTICE, "source": "oracle/ (CPU FP64), tests/golden/make_swe4096_1000.py",
           "runs": runs}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
