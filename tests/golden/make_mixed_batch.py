"""Writes mixed_batch.json: the 64 mixed-size grids of the batched benchmark.

Sizes are log-uniform in [500, 20000] (seed 4); grid g starts from seed
1000 + g and, if the oracle's Newton-Raphson does not converge from flat
start in 20 iterations (tolerance 1e-8), takes seed + 10**6 until it does.
Runs the generator and the CPU oracle only.  Usage:
    python tests/golden/make_mixed_batch.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gridgen  # noqa: E402
from oracle import oracle  # noqa: E402

COUNT, SIZE_SEED, LOAD_SCALE = 64, 4, gridgen.DEFAULT_LOAD_SCALE


def main():
    sizes = gridgen.mixed_sizes(COUNT, SIZE_SEED)
    grids = []
    for g, n in enumerate(sizes):
        seed, tries = 1000 + g, 0
        while True:
            res = oracle.solve_grid(gridgen.make_grid(int(n), seed, load_scale=LOAD_SCALE))
            if res.status == 0:
                break
            seed += 10 ** 6
            tries += 1
        grids.append({"n": int(n), "seed": seed, "reseeds": tries, "iters": res.iters})
        print(g, n, seed, tries, res.iters, flush=True)
    out = {"load_scale": LOAD_SCALE, "size_seed": SIZE_SEED,
           "rule": "seed 1000+g, plus 10**6 until the oracle converges", "grids": grids}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed_batch.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
