"""Wall time of the oracle's solve to C* on the 32^3 single-sphere workload (all
six loads, Jacobi-PCG to rtol 1e-11) -- TEST INFRASTRUCTURE, used only by the
CPU-baseline leg of bench.py, which runs it as a child process so that the
OpenMP thread count (OMP_NUM_THREADS) can differ between runs.

Prints one JSON line: seconds, threads, iterations per load.
"""
import json
import os
import sys
import time


def main():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import oracle
    import synth
    m = synth.workload_sphere32()
    K, G = m.fields()
    oracle.lib()  # load (and first touch) outside the timed region
    t = time.perf_counter()
    C, info = oracle.ceff(K, G, rtol=1e-11)
    dt = time.perf_counter() - t
    print(json.dumps({"seconds": dt, "threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0),
                      "iterations": [int(info[J][0]) for J in range(6)], "C11": float(C[0, 0])}))


if __name__ == "__main__":
    main()
