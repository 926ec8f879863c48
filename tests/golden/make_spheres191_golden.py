"""Write spheres191_oracle.json: oracle C* columns of the 191^3 sphere-pack
workload (all six loads, Jacobi-PCG to rtol 1e-11; resumes from the file).

Calls only the CPU oracle and the input generator.  About half an hour of CPU
per column:
    OMP_NUM_THREADS=6 python tests/golden/make_spheres191_golden.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres191_oracle.json")


def main(loads=(0, 3, 1, 2, 4, 5), rtol=1e-11):
    m = synth.workload_spheres191()
    K, G = m.fields()
    digest = hashlib.sha256(m.phase.tobytes()).hexdigest()
    res = {"workload": "191^3 sphere pack, 10% fluid pores (synth.workload_spheres191)", "phase_sha256": digest,
           "info": m.info, "rtol": rtol, "columns": {}}
    if os.path.exists(OUT):
        old = json.load(open(OUT))
        if old.get("phase_sha256") == digest:
            res["columns"] = old.get("columns", {})
    for J in loads:
        if str(J) in res["columns"]:
            continue
        t = time.time()
        u, it, rel = oracle.solve_load(K, G, J, rtol=rtol)
        col = oracle.average_stress(K, G, oracle.unit_strain(J), u)
        res["columns"][str(J)] = {"C_column": col.tolist(), "iterations": it, "relres": rel,
                                  "seconds": time.time() - t}
        json.dump(res, open(OUT, "w"), indent=1)
        print(f"load {J}: {it} iterations, relres {rel:.2e}, {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
