"""CPU baseline of the hydro cycle (TEST INFRASTRUCTURE): the oracle, as it
stands, compiled -O3 -march=native -fopenmp on the host it runs on, timed on
the 256^3 periodic turbulent box in 512 blocks of 32^3 (the GPU bench's
workload) on all of the process's cores and on one core; median of several
repetitions. Prints one JSON line.

    python -m oracle.timing [--threads N] [--cycles-all 4] [--cycles-one 1] [--reps 3]
"""
import argparse
import ctypes
import json
import os
import platform
import statistics
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0, help="all-core thread count (0: OMP_NUM_THREADS "
                    "or the process's CPU affinity)")
    ap.add_argument("--cycles-all", type=int, default=4)
    ap.add_argument("--cycles-one", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--block", type=int, default=32)
    args = ap.parse_args()
    affinity = len(os.sched_getaffinity(0))
    nthr = args.threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or affinity

    from oracle import build as obuild
    from oracle import oracle as orc
    from paper_2202_12309_amd import inputs
    tmpdir = tempfile.mkdtemp(prefix="pkh_oracle_timing_")
    path = obuild.build_timing(os.path.join(tmpdir, "liboracle_timing.so"))
    orc.use(path)
    gomp = ctypes.CDLL("libgomp.so.1")

    N, blk = args.n, args.block
    n = (blk,) * 3
    nrb = (N // blk,) * 3
    lv = inputs.uniform_leaves(nrb)
    om = orc.OracleMesh(n, nrb, lv)
    U0 = inputs.turbulent_box(om.leaves(), n, nrb, seed=2)

    def timed(threads, cycles):
        gomp.omp_set_num_threads(int(threads))
        runs = []
        for _ in range(args.reps):
            om.set_state(U0)
            om.set_time(0.0, 0)
            t0 = time.perf_counter()
            om.step(cycles)
            runs.append(time.perf_counter() - t0)
        med = statistics.median(runs)
        return {"threads": threads, "cycles": cycles, "seconds": [round(r, 3) for r in runs],
                "median_s": round(med, 3), "zone_cycles_per_s": N ** 3 * cycles / med}

    all_core = timed(nthr, args.cycles_all)
    one_core = timed(1, args.cycles_one)
    print(json.dumps({"workload": f"{N}^3 periodic turbulent box, {len(lv)} blocks of {blk}^3 (seed 2)",
                      "build": "gcc -O3 -march=native -fopenmp (OpenMP over blocks)",
                      "cpu_model": cpu_model(), "affinity_cpus": affinity,
                      "all_core": all_core, "one_core": one_core}))
    os.remove(path)
    os.rmdir(tmpdir)


if __name__ == "__main__":
    main()
