"""Prints the oracle's FP64 operation census of one step of a workload, per
sweep and per cell -- measurement infrastructure (the algorithmic flop count
per cell update that prices the arithmetic roof of the sweeps).

    python -m oracle.census [n]     (default: the 4096 x 4096 roofline grid)
"""
import json
import sys

import numpy as np

import oracle
from paper_1803_01450_amd import inputs


def census(n=4096):
    c = inputs.roofline_grid(n=n, L=409.6e3 * n / 4096)
    dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
    r = oracle.count_ops(c["B"], c["q"], c["dx"], c["dx"], dt, r=c["r"])
    out = {}
    for k in ("x", "y"):
        d = r[k]
        out[k] = {key: d[key] / d["cells"] for key in ("add", "mul", "div", "sqrt", "neg", "fma", "flops")}
        out[k]["cells"] = d["cells"]
    return out


if __name__ == "__main__":
    print(json.dumps(census(int(sys.argv[1]) if len(sys.argv) > 1 else 4096), indent=1))
