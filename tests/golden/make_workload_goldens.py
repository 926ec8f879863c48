"""Write oracle goldens of three workload families (calls only the CPU oracle
and the input generators; resumes from the files it has written):

  cracks128  -> cracks128_oracle.json: all six C* columns of the cracked-solid
               recipe (penny cracks, a ~ U[10, 30], aspect 0.05, fluid filled)
               at its crack number density, 2000 cracks per 479^3, in a 128^3
               box (38 cracks).
  batch      -> batch_oracle.json: all six C* columns of three samples of the
               48-sample three-phase batch: the smallest (n = 51), the first
               (n = 57) and the largest (n = 128).
  grad128    -> grad128_oracle.json: C* of the 128^3 15%-pore pack and the
               oracle's gradients of C11, C44 and trace(C) with respect to K(x)
               and G(x) at 4096 seeded voxels.

Jacobi-PCG to rtol 1e-11 per column.  With 5 OpenMP threads on the build
container: about 20 minutes per column at 128^3.
    OMP_NUM_THREADS=5 python tests/golden/make_workload_goldens.py grad128 batch cracks128
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

HERE = os.path.dirname(os.path.abspath(__file__))
RTOL = 1e-11
BATCH_SAMPLES = (30, 0, 35)       # indices into synth.workload_batch(): n = 51, 57, 128
GRAD_SAMPLE_SEED = 0x6A4D
GRAD_NSAMPLE = 4096


def cracks128():
    n = 128
    return synth.penny_cracks(n, round(2000 * (n / 479) ** 3), 0xC3)


def grad_sample_indices(N):
    """4096 distinct flat voxel indices, drawn with the project's generator."""
    rng = synth.SplitMix64(GRAD_SAMPLE_SEED)
    seen, out = set(), []
    while len(out) < GRAD_NSAMPLE:
        i = rng.randint(0, N - 1)
        if i not in seen:
            seen.add(i)
            out.append(i)
    return np.array(sorted(out), np.int64)


def _digest(m):
    return hashlib.sha256(np.ascontiguousarray(m.phase).tobytes()).hexdigest()


def _load(path, digest_key):
    if os.path.exists(path):
        old = json.load(open(path))
        if old.get("digest") == digest_key:
            return old
    return None


def _columns(m, res, path, fields=None, root=None):
    """Solve the columns `res` lacks; after each, write `root` (the whole file; `res` itself when
    it is the file's top level) so that an interrupted run resumes."""
    K, G = m.fields()
    for J in range(6):
        if str(J) in res["columns"] and fields is None:
            continue
        t = time.time()
        u, it, rel = oracle.solve_load(K, G, J, rtol=RTOL)
        col = oracle.average_stress(K, G, oracle.unit_strain(J), u)
        res["columns"][str(J)] = {"C_column": col.tolist(), "iterations": it, "relres": rel,
                                  "seconds": time.time() - t}
        if fields is not None:
            fields[J] = u
        json.dump(res if root is None else root, open(path, "w"), indent=1)
        print(f"{os.path.basename(path)} load {J}: {it} iterations, relres {rel:.2e}, {time.time() - t:.0f} s",
              flush=True)


def make_cracks128():
    path = os.path.join(HERE, "cracks128_oracle.json")
    m = cracks128()
    d = _digest(m)
    res = _load(path, d) or {"workload": "cracked-solid recipe at 2000 cracks per 479^3, 128^3 box "
                                         "(synth.penny_cracks(128, 38, 0xC3))", "digest": d, "info": m.info,
                             "rtol": RTOL, "columns": {}}
    _columns(m, res, path)


def make_batch():
    path = os.path.join(HERE, "batch_oracle.json")
    ms = synth.workload_batch()
    d = hashlib.sha256("".join(_digest(ms[s]) for s in BATCH_SAMPLES).encode()).hexdigest()
    res = _load(path, d) or {"workload": "three samples of synth.workload_batch() (48 three-phase GRF cubes)",
                             "digest": d, "rtol": RTOL, "samples": {}}
    for s in BATCH_SAMPLES:
        sub = res["samples"].setdefault(str(s), {"n": int(ms[s].phase.shape[0]), "info": ms[s].info,
                                                 "columns": {}})
        _columns(ms[s], sub, path, root=res)
        json.dump(res, open(path, "w"), indent=1)


def make_grad128():
    path = os.path.join(HERE, "grad128_oracle.json")
    m = synth.workload_grad128()
    K, G = m.fields()
    d = _digest(m)
    res = _load(path, d)
    if res is not None and "gradients" in res:
        return
    res = {"workload": "128^3 sphere pack, 15% fluid pores (synth.workload_grad128)", "digest": d, "info": m.info,
           "rtol": RTOL, "columns": {}}
    fields = {}
    _columns(m, res, path, fields=fields)
    idx = grad_sample_indices(K.size)
    Ws = {"C11": np.diag([1.0, 0, 0, 0, 0, 0]), "C44": np.diag([0, 0, 0, 1.0, 0, 0]), "trace": np.eye(6)}
    res["sample"] = {"seed": GRAD_SAMPLE_SEED, "flat_indices": idx.tolist()}
    res["gradients"] = {}
    for name, W in Ws.items():
        dK, dG = oracle.gradient(K, G, fields, W)
        res["gradients"][name] = {"dK": [float("%.13g" % v) for v in dK.ravel()[idx]],
                                  "dG": [float("%.13g" % v) for v in dG.ravel()[idx]],
                                  "max_abs_dK": float(np.abs(dK).max()), "max_abs_dG": float(np.abs(dG).max()),
                                  "euler_sum": float(np.sum(K * dK + G * dG))}
    json.dump(res, open(path, "w"), indent=1)
    print("grad128 gradients written", flush=True)


if __name__ == "__main__":
    jobs = {"cracks128": make_cracks128, "batch": make_batch, "grad128": make_grad128}
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
