"""Write h3_pairs.json: the number of ordered pairs of the 100k-point
hyperbolic-3-space catalogue (inputs.c11_h3_4pcf) whose geodesic distance lies in the
catalogue's bins, counted by the FP64 oracle over every primary (the bins are
e_b <= theta < e_{b+1}, decided on the FP64 Minkowski product).

Run from the repository root: python tests/golden/make_h3_pairs.py
(a few minutes on 8 cores)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2106_10278_amd import inputs  # noqa: E402


def main():
    wl = inputs.c11_h3_4pcf()
    n = wl.pos.shape[1]
    total = 0
    for p0 in range(0, n, 10_000):
        _, pairs = oracle.npcf(3, 3, 0, wl.edges, wl.box, wl.pos, wl.w, prims=np.arange(p0, min(n, p0 + 10_000)),
                               hyperbolic=True)
        total += int(pairs)
        print(f"primaries [{p0}, {min(n, p0 + 10_000)}): {total} pairs so far", flush=True)
    out = {"workload": wl.name, "n": n, "edges": [float(e) for e in wl.edges], "pairs": total,
           "source": "oracle.npcf (FP64), lmax 0, every primary"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "h3_pairs.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(total)


if __name__ == "__main__":
    main()
