"""Write block_max_rows.json: for the full-size plans that the GPU tests check
row by row against the oracle's compressed method, the row of every block where
max |A_e W F| (the threshold's reference, Alg. 1 step 1.3, taken per block) is
attained, with that maximum.  Computed by the oracle alone, over every row.

    python tests/golden/make_block_max_rows.py [--only NAME]

Plans: the 48-plan batch's members listed in workloads.BATCH_ORACLE_C and the
Laguerre-function workload (N = 65536), all at workloads.shared_nodes, row
mode, eps2 = 1e-2."""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import compressed, matrix  # noqa: E402

OUT = os.path.join(HERE, "block_max_rows.json")


def cases():
    ws = workloads.batch_plans()
    out = [ws[i] for i in workloads.BATCH_ORACLE_C]
    out.append(workloads.LAGUERRE_65536)
    return out


def oracle_plan(w):
    fam = matrix.MatrixFamily(w["family"], w["N"], alpha=w.get("alpha", 0.0),
                              beta=w.get("beta", 0.0),
                              given_nodes=workloads.shared_nodes(w["family"], w["N"]))
    return compressed.Plan(fam, w["eps"], 1e-2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for w in cases():
        if args.only and w["name"] != args.only:
            continue
        t0 = time.time()
        plan = oracle_plan(w)
        rows = compressed.block_max_rows(plan, panel=512)
        data[w["name"]] = {"family": w["family"], "N": w["N"], "alpha": w.get("alpha", 0.0),
                           "beta": w.get("beta", 0.0), "eps1": w["eps"], "eps2": 1e-2,
                           "blocks": [[r, m] for r, m in rows]}
        print(w["name"], w["N"], "%.0f s" % (time.time() - t0), rows, flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
