"""Benchmark: effective stiffness of a 191^3 fluid-filled sphere pack on one MI355X.

One step = one complete solve of the hot path: six unit macroscopic-strain
loads (fused in one launch per iteration, or one after another when a single
load's working set fits in the Infinity Cache; the library's automatic
choice unless --fuse says otherwise), FP32 sweeps with FP64 residuals and
defect-correction folds, FP64 volume averages, giving the 6x6 C* on the host.
The material (a phase image) is resident in HBM before timing starts.

Prints one JSON line.  value = voxel-updates per second over the timed steps
(N x iterations summed over loads / wall time).  The roofline object covers
the iteration kernel: algorithmic bytes of its launches over their device time
(HIP events recorded by the library on the stream the kernel runs on).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the iteration kernel measured with rocprofv3 FETCH_SIZE /
# WRITE_SIZE (scaled against a 1 GiB copy kernel; profiles/step_kernel_spheres191_trace_and_counters.md and
# profiles/step_kernel_spheres480_trace_and_counters.md), valid only for the kernel source they were taken on.
MEASURED_TRAFFIC = {"ceff_kernels_sha256_prefix": "75b988406fdf0a49", "bytes_per_launch": 3.201660e+08,
                    # (loads per block, kernel variant, loads fused, moduli from the phase image, high occupancy,
                    # block x, block y, z-chunk)
                    "launch_signature": (1, 9, 0, 1, 1, 32, 8, 12),
                    # mean algorithmic bytes per launch of the profiled solve: fixes its mix of
                    # macroscopic-strain and body-force launches
                    "algorithmic_bytes_per_launch": 3.009393e+08,
                    "launch": "step_kernel_x<float,1,PAL,high occupancy>, mean over all launches of a full solve"}
# the same for the HBM-resident measurement (480^3, one load, 200 iterations without body force; the mean over
# its launches after the first, which reads no u^{n-1})
MEASURED_TRAFFIC_HBM = {"ceff_kernels_sha256_prefix": "75b988406fdf0a49", "n": 480, "bytes_per_launch": 4.373917e+09,
                        "algorithmic_bytes_per_launch": 4.091904e+09, "launch_shape": "64x8x32 variant 9"}


# iteration-kernel variant (ceff_stats.tile_variant) -> kernel name
VARIANT_KERNEL = {0: "step_kernel", 1: "step_kernel", 2: "step_kernel_u2", 3: "step_kernel_b", 4: "step_kernel_p3",
                  5: "step_kernel_c", 6: "step_kernel_t", 9: "step_kernel_x"}


# Swept Strouhal numbers per workload family (six loads, mixed precision, rtol 1e-8):
#   spheres191 (now run with the automatic St 3.48): St 3.0 / 3.25 / 3.5 / 3.75 -> 32400 / 30000 / 28200 / 28000, 32400 / 30200 / 29800 / 30800 and
#               32400 / 30200 / 29600 / 31800 load-iterations for three seeds (checks every 200); 3.5 is the
#               lowest on average and below 3.25 for each seed; St 4.0 gave 34600 for the third
#   (the sweeps below ran with checks every 200 iterations)
#   cracks479:  St 2.0 / 2.5 / 3.0 / 4.0 / 5.0 / 6.5 / 8.0 -> 152 / 125 / 103 / 76 / 61 / 58 / 78 s (5.0: even
#               counts over the six loads)
#   batch48:    St 2.0 / 2.5 / 3.0 / 3.5 -> 15.4 / 13.1 / 12.6 / 13.7 s
#   spheres703: St 5.0 / 6.5 / 8.0 / 11.5 -> 12000 / 9200 / 7400 / 9200 iterations of load 0
# The 191^3 benchmark runs with the library's automatic choice (strouhal = 0: St 3.48 at 191^3, next to the
# swept 3.5); the other workloads keep their swept values.
STROUHAL_BY_WORKLOAD = {"cracks479": 5.0, "batch48": 3.0, "spheres703": 8.0}


def kernel_source_hash():
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "paper_2410_20441_amd", "csrc", "ceff_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stream_ceiling(torch, dev, mib=1024):
    """Bandwidth of plain torch copy (1 read, 1 write) and add (2 reads, 1 write)
    kernels on mib-MiB buffers: the practical streaming ceiling of the device."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device=dev)
    b = torch.ones(n, device=dev)
    c = torch.empty(n, device=dev)
    out = {}
    for name, f, nbytes in (("copy_GB_s", lambda: c.copy_(a), 8 * n), ("add_GB_s", lambda: torch.add(a, b, out=c),
                                                                        12 * n)):
        for _ in range(3):
            f()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            f()
        e1.record()
        torch.cuda.synchronize(dev)
        out[name] = nbytes / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return out


def calibrate_copy(torch, dev, mib):
    """Copy a buffer of `mib` MiB three times: a plain copy kernel of known size against which
    rocprofv3's HBM byte counters are scaled."""
    nb = mib * (1 << 20)
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize(dev)
    print(f"# copy calibration: {nb} bytes read and {nb} bytes written per copy kernel", file=sys.stderr, flush=True)
    del src, dst
    torch.cuda.empty_cache()


def hbm_roofline(a, torch, synth, ceff, dev):
    """The iteration kernel where its working set far exceeds the 256 MiB Infinity Cache: one load of
    an n^3 sphere pack (10% fluid pores, the benchmark's recipe; 480^3 by default, 4.1 GB of
    displacements, body-force slot and phase image), a fixed number of iterations timed by the
    library's HIP events on its stream.  Same kernel family as the headline roofline, at the launch
    shape the library picks for grids beyond the cache."""
    t0 = time.perf_counter()
    m = synth.random_spheres(a.hbm_n, 0.10, 0xC2)
    N = m.phase.size
    print(f"# hbm roofline: {a.hbm_n}^3 sphere pack generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    ctx = ceff.Context(0)
    ctx.set_phases(m.phase, m.K_tab, m.G_tab)
    opts = dict(loads=[0], precision="mixed", rtol=1e-8, strouhal=a.strouhal, check_every=100,
                max_iter=a.hbm_iters, allow_unconverged=True)
    ctx.solve(**dict(opts, max_iter=20, check_every=10))  # warm-up (allocation, graph, code objects)
    C, info = ctx.solve(**opts)
    st = info["stats"]
    ctx.close()
    achieved = st["step_bytes"] / (st["step_time_ms"] * 1e-3) / 1e9
    shape = f"{st['tile_bx']}x{st['tile_by']}x{st['tile_kc']} variant {st['tile_variant']}"
    mt = MEASURED_TRAFFIC_HBM
    traffic = mt["bytes_per_launch"] if (kernel_source_hash() == mt["ceff_kernels_sha256_prefix"] and
                                         a.hbm_n == mt["n"] and shape == mt["launch_shape"] and
                                         st["tile_occ"] == 1) else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_note": "HBM bytes per launch after the first (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, rocprofv3, "
                            "scaled against a 1 GiB copy), taken on this kernel source" if traffic else None,
            "kernel": "%s<float,%s>%s (heavy-ball APT iteration, loads per block = %s)" % (
                VARIANT_KERNEL[st["tile_variant"]], st["tile_group"], ", high occupancy" if st["tile_occ"] else "",
                st["tile_group"]),
            "workload": f"{a.hbm_n}^3 sphere pack (10% fluid pores), load 0, {st['step_launches']} iterations",
            "launch_shape": shape,
            "avg_launch_ms": st["step_time_ms"] / max(st["step_launches"], 1),
            "launches": st["step_launches"],
            "bytes_per_launch": st["step_bytes"] / max(st["step_launches"], 1),
            "working_set_bytes": float(N) * 37.0, "infinity_cache_bytes": 256 * 2 ** 20}


def oracle_time_to_ceff(threads):
    """Oracle time to C* on the 32^3 single sphere (six loads), in a child process with
    `threads` OpenMP threads."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, "-m", "oracle.timing"], cwd=here, capture_output=True, text=True,
                       env=dict(os.environ, OMP_NUM_THREADS=str(threads)), timeout=900, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=191, help="grid size of the sphere pack")
    ap.add_argument("--rtol", type=float, default=1e-8)
    # St is a numerical parameter of the APT iteration; its best value depends on the microstructure
    # and the box size (the library picks it from the box when it is 0).  The workload families of
    # STROUHAL_BY_WORKLOAD run at the value a sweep found best for them.
    ap.add_argument("--strouhal", type=float, default=None,
                    help="APT Strouhal number (default: the swept value of the workload, else the library's "
                         "automatic choice)")
    ap.add_argument("--check-every", type=int, default=100, help="iterations between residual checks (library default)")
    ap.add_argument("--no-fp64-baseline", action="store_true", help="skip the FP64 one-load-at-a-time solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-roofline", action="store_true",
                    help="skip the second roofline measurement on a grid beyond the Infinity Cache")
    ap.add_argument("--hbm-n", type=int, default=480, help="grid of the HBM-resident roofline measurement")
    ap.add_argument("--hbm-iters", type=int, default=200, help="iterations of that measurement")
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle APT iterations timed for the CPU baseline")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--fuse", default="auto", choices=["auto", "on", "off"],
                    help="load fusion: library choice (auto), one launch for all loads (on), one load at a time (off)")
    ap.add_argument("--max-iter", type=int, default=400000)
    ap.add_argument("--loads", default="012345", help="other single-image workloads: the loads to solve")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"],
                    help="batch48, cracks479, spheres703: precision of the solve (the benchmark line is mixed)")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for counter collection: allow stopping at --max-iter")
    ap.add_argument("--workload", default="spheres191",
                    choices=["spheres191", "batch48", "cracks479", "spheres703", "walls191", "hsweep", "grad128",
                             "hbm480"],
                    help="spheres191 (default bench line); batch48: 48 uneven three-phase samples in one solve; "
                         "cracks479: 479^3 cracked solid; spheres703: 703^3 sphere pack (the largest grid; --fuse off solves the loads one after another and reports each); "
                         "walls191: the paper's layered model at 191^3 under the direct tests' walls, with the triaxial "
                         "off-diagonals; "
                         "hsweep: contribution tensors of single spheroids, aspect ratio x contrast, one batch; "
                         "hbm480: only the HBM-resident roofline measurement (for profiling)")
    ap.add_argument("--hsweep-r", type=int, default=12, help="hsweep: largest semi-axis of the coarse spheroids")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB three times (a plain copy kernel of known size "
                         "against which HBM byte counters are scaled)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the solve would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2410_20441_amd as ceff

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if a.strouhal is None:
        a.strouhal = STROUHAL_BY_WORKLOAD.get(a.workload, 0.0)
    if a.workload != "spheres191":
        return other_workload(a, torch, synth, ceff, dev)
    m = synth.workload_spheres191(n=a.n)
    N = m.phase.size
    print(f"# workload {m.info}", file=sys.stderr, flush=True)

    if a.calibrate_copy:
        calibrate_copy(torch, dev, a.calibrate_copy)

    ctx = ceff.Context(0)
    ctx.set_phases(m.phase, m.K_tab, m.G_tab)
    fuse = {"auto": "auto", "on": True, "off": False}[a.fuse]
    opts = dict(precision="mixed", rtol=a.rtol, strouhal=a.strouhal, check_every=a.check_every, fuse_loads=fuse,
                use_graph=True, autotune=a.autotune, max_iter=a.max_iter, allow_unconverged=a.profile_run)

    for w in range(a.warmup):
        C, info = ctx.solve(**opts)
        print(f"# warmup {w}: status {info['status']} iters {info['iters'].tolist()} "
              f"{info['stats']['solve_ms']:.1f} ms", file=sys.stderr, flush=True)

    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    tot = {"vu": 0.0, "iters": 0, "step_ms": 0.0, "step_bytes": 0.0, "launches": 0}
    groups = set()
    Cs = []
    for k in range(a.steps):
        C, info = ctx.solve(**opts)
        st = info["stats"]
        tot["vu"] += N * float(info["iters"].sum())
        tot["iters"] += int(info["iters"].sum())
        tot["step_ms"] += st["step_time_ms"]
        tot["step_bytes"] += st["step_bytes"]
        tot["launches"] += st["step_launches"]
        groups.add((st["tile_group"], st["tile_variant"], st["fused_loads"], st["phase_moduli"], st["tile_occ"],
                    st["tile_bx"], st["tile_by"], st["tile_kc"]))
        Cs.append(C)
        print(f"# step {k}: status {info['status']} iters {info['iters'].tolist()} solve {st['solve_ms']:.1f} ms, "
              f"kernel {st['step_time_ms'] / max(st['step_launches'], 1):.4f} ms/launch, tile {st['tile_bx']}x"
              f"{st['tile_by']}x{st['tile_kc']} group {st['tile_group']} variant {st['tile_variant']} "
              f"fused {st['fused_loads']} phase moduli {st['phase_moduli']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    C = Cs[-1]
    achieved = tot["step_bytes"] / (tot["step_ms"] * 1e-3) / 1e9
    traffic = None
    bpl = tot["step_bytes"] / max(tot["launches"], 1)
    if kernel_source_hash() == MEASURED_TRAFFIC["ceff_kernels_sha256_prefix"] and \
            groups == {MEASURED_TRAFFIC["launch_signature"]} and \
            abs(bpl / MEASURED_TRAFFIC["algorithmic_bytes_per_launch"] - 1.0) < 0.01:
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]

    out = {
        "metric": "GVoxel-updates/s (six-load effective stiffness solve, 191^3)",
        "value": tot["vu"] / wall / 1e9,
        "unit": "GVoxel-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.n}^3 periodic sphere pack, 10% fluid-filled pores (K=2.2, G=1e-3 GPa) "
                               f"in a K=70, G=32 GPa matrix; six unit loads "
                               f"{'fused' if st['fused_loads'] else 'one after another'}; FP32 sweeps with FP64 "
                               f"residuals, folds and averages; rtol {a.rtol:g}",
                   "n": a.n, "voxels": N, "loads": 6, "rtol": a.rtol, "precision": "mixed",
                   "fused_loads": bool(st["fused_loads"]), "moduli": "phase image" if st["phase_moduli"] else "fields",
                   "strouhal": a.strouhal if a.strouhal > 0 else ceff.ceff_auto_strouhal(a.n, a.n, a.n),
                   "strouhal_choice": "explicit" if a.strouhal > 0 else "automatic",
                   "porosity": m.info["porosity"]},
        "time_to_ceff_s": wall / a.steps,
        "iterations_per_solve": tot["iters"] / a.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "%s<float,%s>%s (heavy-ball APT iteration, loads per block = %s)" % (
                         VARIANT_KERNEL[st["tile_variant"]], st["tile_group"],
                         ", high occupancy" if st["tile_occ"] else "", st["tile_group"]),
                     "avg_launch_ms": tot["step_ms"] / max(tot["launches"], 1),
                     "bytes_per_launch": tot["step_bytes"] / max(tot["launches"], 1),
                     # the launch's distinct data: per voxel and load the two FP32 displacement
                     # buffers (u^n, and the one u^{n-1} is read from and u^{n+1} written to) and the
                     # body force, 12 B each, plus the 1-byte phase image; when it fits in the 256 MiB
                     # Infinity Cache, part of the traffic is served there rather than by HBM
                     "working_set_bytes": float(N) * (36.0 * (6 if st["fused_loads"] else 1) + 1.0),
                     "infinity_cache_bytes": 256 * 2 ** 20},
        "C_eff_GPa": np.round(C, 6).tolist(),
    }

    out["stream_ceiling"] = stream_ceiling(torch, dev)

    # time to C* including the upload of the material from host memory (a new context: the phase
    # image and table go host -> device, the FP64 K and G fields are expanded on the device)
    torch.cuda.synchronize(dev)
    t3 = time.perf_counter()
    ctx_u = ceff.Context(0)
    ctx_u.set_phases(m.phase, m.K_tab, m.G_tab)
    Cu, info_u = ctx_u.solve(**opts)
    torch.cuda.synchronize(dev)
    out["time_to_ceff_with_upload_s"] = time.perf_counter() - t3
    ctx_u.close()
    if not np.array_equal(Cu, C):
        print("# warning: the solve after a fresh upload differs from the timed ones", file=sys.stderr, flush=True)

    if not a.no_hbm_roofline:
        out["roofline_hbm"] = hbm_roofline(a, torch, synth, ceff, dev)

    if not a.no_fp64_baseline:
        t1 = time.perf_counter()
        C64, info64 = ctx.solve(**dict(opts, precision="fp64", fuse_loads=False))
        if info64["status"] != 0:
            print(f"# fp64 single-load status {info64['status']}", file=sys.stderr, flush=True)
        t64 = time.perf_counter() - t1
        st64 = info64["stats"]
        out["fp64_single_load"] = {
            "time_to_ceff_s": t64, "iterations": info64["iters"].tolist(),
            "gvu_s": N * float(info64["iters"].sum()) / t64 / 1e9,
            "kernel_GB_s": st64["step_bytes"] / (st64["step_time_ms"] * 1e-3) / 1e9,
            "avg_launch_ms": st64["step_time_ms"] / max(st64["step_launches"], 1)}
        out["speedup_vs_fp64_single_load"] = t64 / (wall / a.steps)
        out["ceff_max_rel_diff_mixed_vs_fp64"] = float(np.max(np.abs(C - C64)) / np.max(np.abs(C64)))
        print(f"# fp64 single-load: {t64:.2f} s iters {info64['iters'].tolist()}", file=sys.stderr, flush=True)
    ctx.close()

    if not a.no_cpu_baseline:
        import oracle
        K, G = m.fields()
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        oracle.apt_steps(K, G, 0, 1, courant=0.95, strouhal=a.strouhal)  # load + first touch
        t2 = time.perf_counter()
        oracle.apt_steps(K, G, 0, a.cpu_steps, courant=0.95, strouhal=a.strouhal)
        tc = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": N * a.cpu_steps / tc / 1e9, "unit": "GVoxel-updates/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{a.cpu_steps} APT iterations of one load on the same {a.n}^3 grid "
                                         f"(oracle, paper-form variables), {tc:.1f} s"}
        # the oracle's own solve (Jacobi-PCG to rtol 1e-11) to C* on the 32^3 single sphere, all cores and
        # one thread; the 191^3 figure is the recorded run that wrote the stored oracle columns
        ttc = {"workload": "32^3 single sphere (r = 8, fluid), six loads, Jacobi-PCG to rtol 1e-11"}
        for t in (threads, 1):
            r = oracle_time_to_ceff(t)
            ttc[f"seconds_{t}_threads"] = r["seconds"]
            ttc["iterations"] = r["iterations"]
        out["cpu_baseline"]["time_to_ceff_32"] = ttc
        gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "spheres191_oracle.json")
        if os.path.exists(gold):
            g = json.load(open(gold))
            out["cpu_baseline"]["time_to_ceff_191_recorded"] = {
                "seconds": sum(c["seconds"] for c in g["columns"].values()), "threads": 6,
                "host": "8-core build container (not this host); the run that wrote tests/golden/spheres191_oracle.json",
                "iterations": [g["columns"][str(J)]["iterations"] for J in range(6)]}
    print(json.dumps(out), flush=True)


def hsweep(a, torch, synth, ceff, dev):
    """Compliance contribution tensors of single spheroids (aspect ratio x inclusion contrast,
    each at two resolutions r and 2r in a box of 8r) from one batch solve, with the error
    against Eshelby's tensor before and after first-order extrapolation in r."""
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    import closed_forms as cf
    host = (36.0, 44.0)
    incs = {"soft": (7.2, 8.8), "stiff": (180.0, 220.0), "pore": (1e-3, 2e-3)}
    alphas = (0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0)
    r0 = a.hsweep_r
    cases, ms = [], []
    for al in alphas:
        shape = (1.0, 1.0, al) if al <= 1 else (1.0 / al, 1.0 / al, 1.0)
        for name, inc in incs.items():
            for r in (r0, 2 * r0):
                cases.append((al, name, r, shape))
                ms.append(synth.centred_spheroid(8 * r, tuple(r * f for f in shape), matrix=host, inclusion=inc))
    # one table for the whole batch: the host, then the three inclusions; each image's
    # inclusion voxels (phase 1) take the id of its own inclusion
    names = list(incs)
    Ktab = np.array([host[0]] + [incs[q][0] for q in names])
    Gtab = np.array([host[1]] + [incs[q][1] for q in names])
    phases = [np.where(m.phase == 1, 1 + names.index(cs[1]), 0).astype(np.uint8) for m, cs in zip(ms, cases)]
    N = sum(m.phase.size for m in ms)
    print(f"# hsweep: {len(ms)} samples, {N} voxels", file=sys.stderr, flush=True)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    C, it, info = ceff.solve_batch_phases(phases, Ktab, Gtab, precision="mixed", rtol=a.rtol,
                                          check_every=a.check_every, max_iter=a.max_iter)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t1
    K1, G1 = host
    nu = (3 * K1 - 2 * G1) / (2 * (3 * K1 + G1))
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    C1 = cf.c_iso(*host)
    rows = []
    for q in range(0, len(cases), 2):
        al, name, r, shape = cases[q]
        He = cf.compliance_contribution(C1, cf.c_iso(*incs[name]), cf.eshelby_tensor(np.array(shape), nu))
        He = He * np.outer(w, w)
        H1, _ = ceff.contribution_tensors(C[q], C1, ms[q].info["phi"])
        H2, _ = ceff.contribution_tensors(C[q + 1], C1, ms[q + 1].info["phi"])
        err = lambda H: float(np.abs(H - He).max() / np.abs(He).max())
        rows.append({"aspect": al, "inclusion": name, "r": [r, 2 * r],
                     "phi": [ms[q].info["phi"], ms[q + 1].info["phi"]],
                     "H_2r_voigt_11_33_44_12_13": [float(H2[0, 0]), float(H2[2, 2]), float(H2[3, 3]), float(H2[0, 1]),
                                                  float(H2[0, 2])],
                     "err_r": err(H1), "err_2r": err(H2), "err_extrapolated": err(2 * H2 - H1)})
    vu = float(sum(ms[s].phase.size * it[s].sum() for s in range(len(ms))))
    st = info["stats"]
    res = {"workload": "hsweep", "samples": len(ms), "voxels": N, "status": info["status"], "time_s": wall,
           "gvu_s": vu / wall / 1e9, "kernel_GB_s": st["step_bytes"] / (st["step_time_ms"] * 1e-3) / 1e9,
           "rows": rows}
    print(json.dumps(res), flush=True)


def grad128(a, torch, synth, ceff, dev):
    """Adjoint gradients of C11, C44 and trace(C) with respect to K(x) and G(x) on the
    128^3 15%-pore pack: one solve keeping the FP64 fields, then each gradient sweep
    timed (device outputs, FP32)."""
    m = synth.workload_grad128()
    K, G = m.fields()
    N = K.size
    ctx = ceff.Context(0)
    ctx.set_material(K, G)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    C, info = ctx.solve(precision="mixed", rtol=a.rtol, strouhal=a.strouhal, check_every=a.check_every,
                        keep_fields=True)
    torch.cuda.synchronize(dev)
    solve_s = time.perf_counter() - t0
    print(f"# grad128: solve {solve_s:.3f} s, iterations {info['iters'].tolist()}", file=sys.stderr, flush=True)
    Ws = {"C11": (np.diag([1.0, 0, 0, 0, 0, 0]), 1), "C44": (np.diag([0, 0, 0, 1.0, 0, 0]), 1),
          "trace": (np.eye(6), 6)}
    out = {}
    for name, (W, nl) in Ws.items():
        ctx.gradient(W, device=dev)
        torch.cuda.synchronize(dev)
        reps = 20
        t1 = time.perf_counter()
        for _ in range(reps):
            ctx.gradient(W, device=dev)
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t1) / reps * 1e3
        # FP64 displacements of the loads W touches, K and G (FP64), two FP32 outputs
        nbytes = N * (24.0 * nl + 16.0 + 8.0)
        out[name] = {"ms": ms, "loads_read": nl, "bytes": nbytes, "GB_s": nbytes / (ms * 1e-3) / 1e9,
                     "share_of_solve": ms * 1e-3 / solve_s}
    ctx.close()
    res = {"workload": "grad128", "voxels": N, "info": m.info, "solve_s": solve_s,
           "iterations": info["iters"].tolist(), "gradients": out}
    print(json.dumps(res), flush=True)


def other_workload(a, torch, synth, ceff, dev):
    """Measurement runs of the other workloads (one solve each, not the bench line)."""
    if a.workload == "hsweep":
        return hsweep(a, torch, synth, ceff, dev)
    if a.workload == "grad128":
        return grad128(a, torch, synth, ceff, dev)
    if a.calibrate_copy:
        calibrate_copy(torch, dev, a.calibrate_copy)
    if a.workload == "hbm480":
        print(json.dumps(hbm_roofline(a, torch, synth, ceff, dev)), flush=True)
        return
    opts = dict(precision=a.precision, rtol=a.rtol, strouhal=a.strouhal, check_every=a.check_every, max_iter=a.max_iter,
                allow_unconverged=a.profile_run, autotune=a.autotune,
                fuse_loads={"auto": "auto", "on": True, "off": False}[a.fuse])
    t0 = time.perf_counter()
    if a.workload == "batch48":
        ms = synth.workload_batch()
        # the samples share one phase table: the batch runs on the phase images
        assert all(np.array_equal(m.K_tab, ms[0].K_tab) and np.array_equal(m.G_tab, ms[0].G_tab) for m in ms)
        N = sum(m.phase.size for m in ms)
        print(f"# batch of {len(ms)}: sizes {[m.phase.shape[0] for m in ms]}, {N} voxels, generated in "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        C, it, info = ceff.solve_batch_phases([m.phase for m in ms], ms[0].K_tab, ms[0].G_tab, **opts)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t1
        vu = float(sum(ms[s].phase.size * it[s].sum() for s in range(len(ms))))
        st = info["stats"]
        res = {"workload": "batch48", "precision": a.precision, "voxels": N, "samples": len(ms), "status": info["status"],
               "time_s": wall, "gvu_s": vu / wall / 1e9, "max_iterations": int(it.max()),
               "kernel_GB_s": st["step_bytes"] / (st["step_time_ms"] * 1e-3) / 1e9,
               "avg_launch_ms": st["step_time_ms"] / max(st["step_launches"], 1), "launches": st["step_launches"]}
    else:
        if a.workload == "cracks479":
            m = synth.workload_cracks()
        elif a.workload == "walls191":
            m = synth.laminate_z(191, 191, 191, 6, 15)  # six stiff layers 15 cells thick in a soft host
        else:
            m = synth.random_spheres(703, 0.10, 0xC2)
        N = m.phase.size
        print(f"# {a.workload}: {m.info}, generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
        ctx = ceff.Context(0)
        ctx.set_phases(m.phase, m.K_tab, m.G_tab)
        if a.workload == "walls191":
            ctx.set_boundary("walls")
        loads = [int(q) for q in a.loads]
        # one load at a time (--fuse off): one solve call per load, each reported as it ends
        groups = [[J] for J in loads] if a.fuse == "off" else [loads]
        C = np.full((6, 6), np.nan)
        iters = np.zeros(6, np.int64)
        relres = {}
        status, step_bytes, step_ms, launches = 0, 0.0, 0.0, 0
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        for grp in groups:
            tg = time.perf_counter()
            Cg, info = ctx.solve(loads=grp, **opts)
            for J in grp:
                C[:, J] = Cg[:, J]
                iters[J] = info["iters"][J]
                h = info["hist"]
                hj = h[h[:, 1] == J]
                relres[J] = float(hj[-1, 2]) if len(hj) else 0.0
            status = status or info["status"]
            st = info["stats"]
            step_bytes += st["step_bytes"]; step_ms += st["step_time_ms"]; launches += st["step_launches"]
            print(f"# loads {grp}: status {info['status']}, iterations {[int(iters[J]) for J in grp]}, "
                  f"final relative residual {[relres[J] for J in grp]}, {time.perf_counter() - tg:.1f} s",
                  file=sys.stderr, flush=True)
        wall = time.perf_counter() - t1
        ctx.close()
        res = {"workload": a.workload, "precision": a.precision, "voxels": N, "info": m.info, "status": status,
               "time_s": wall,
               "loads": loads, "iterations": iters.tolist(), "final_relres": relres, "strouhal": a.strouhal,
               "gvu_s": N * float(iters.sum()) / wall / 1e9,
               "kernel_GB_s": step_bytes / (step_ms * 1e-3) / 1e9 if step_ms > 0 else None,
               "avg_launch_ms": step_ms / max(launches, 1),
               "C_eff_GPa": np.round(C, 5).tolist()}
        if a.workload == "walls191":
            res["boundary"] = "walls"
            if not np.isnan(C[:3, :3]).any():
                res["triaxial_offdiagonals_GPa"] = [round(float(v), 5) for v in ceff.triaxial_offdiagonals(C)]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
