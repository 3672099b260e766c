"""Write the oracle's results for the large workloads to ``tests/golden/oracle_runs.json``.

Calls only the CPU oracle (``oracle/``) on the inputs stated in ``workloads.py``; the
GPU tests compare the library's outputs with these stored values.  Each entry holds
the SHA-256 of the final grid (N bytes, C order), the counts, the terminal status and
the per-step series |F_t|, |New_t|, the solid count at the start of each step and the
step's work (draws, high-half Philox blocks) and the sizes of the one-voxel bands
around F_t and around F_t u New_t (the occupancy a step reads).  The group ``lit`` runs
cases with the literal Algorithm 3 front rule (entries named ``<case>_literal``,
``literal_front`` true).

    python tests/golden/make_goldens.py [--jobs 8] [--only c2,c3,lit,c4,c4s,c5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")


def run_case(job: tuple) -> dict:
    case_dict, literal = job
    c = workloads.Case(**{**case_dict, "dims": tuple(case_dict["dims"]),
                          "g_ref": tuple(case_dict["g_ref"])})
    t0 = time.time()
    r = oracle.generate(c.dims, c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key,
                        max_steps=c.max_steps, log_cap=100000, literal_front=literal,
                        bands=True)
    return {
        "name": c.name + ("_literal" if literal else ""), "literal_front": literal,
        "case": c.as_dict(),
        "grid_sha256": hashlib.sha256(r.grid.tobytes()).hexdigest(),
        "n_candidates": r.n_candidates, "n_seeds": r.n_seeds, "solid_count": r.solid_count,
        "target_count": r.target_count, "front_size": r.front_size, "steps": r.steps,
        "status": r.status,
        "log_front": [int(x) for x in r.log_front], "log_new": [int(x) for x in r.log_new],
        "log_count": [int(x) for x in r.log_count],
        "log_draws": [int(x) for x in r.log_draws], "log_blocks": [int(x) for x in r.log_blocks],
        "log_band": [int(x) for x in r.log_band],
        "log_band_union": [int(x) for x in r.log_band_union],
        "oracle_seconds": round(time.time() - t0, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--only", default="c1,c2,c3")
    args = ap.parse_args()
    oracle.build()
    groups = {"c1": workloads.config1, "c2": workloads.config2, "c3": workloads.config3,
              "c4": workloads.config4, "c4s": workloads.config4_singletons,
              "c5": workloads.config5_parity,
              "lit": lambda: workloads.config1() + workloads.config2()[:1] +
              workloads.config3()[1:2]}
    cases = []
    for g in args.only.split(","):
        cases += [(c, g == "lit") for c in groups[g]()]
    existing = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            existing = json.load(f)
    # largest first so the pool stays busy
    cases.sort(key=lambda cl: -cl[0].n)
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for res in ex.map(run_case, [(c.as_dict(), lit) for c, lit in cases]):
            existing[res["name"]] = res
            print(res["name"], res["steps"], res["solid_count"], res["oracle_seconds"],
                  flush=True)
            with open(OUT, "w") as f:
                json.dump(existing, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
