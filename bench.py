#!/usr/bin/env python3
"""Throughput of the hydro hot path on one MI355X.

One step = one full VL2 cycle (predictor, ghost fill, corrector with the
fused CFL reduction, ghost fill, device clock) over every block of the
256^3 FP64 periodic mesh cut into 512 blocks of 32^3 (log-normal density,
rms Mach 0.5; seeded, synthetic). Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--block 32]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-cycles/s & %HBM peak (256^3 FP64 hydro); adjoint/forward cost ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, a fused multiply-add counted as two
# Algorithmic FP64 operations (add, multiply, divide, square root) per zone of
# each stage and of the CFL signal speed, as the method's formulas are written
# (no contraction, no ghost-cell recomputation): counted by the
# operation-counting mirror of the oracle's formulas, which a test keeps equal
# to these numbers.
ALG_FLOPS = {"predictor": 461, "corrector": 731, "cfl": 21}
N = 256
STAGE_END_MARK = "// ---- end of the stage kernels (the persistent batch kernel follows) ----"
DEVICE_STRUCTS = ("BlockInfo", "DevTime", "LevelMaps", "Geom", "FineFace", "StageLaunch", "GroupItem")


def stage_device_source():
    """The source text that defines the stage kernels' device code: the
    stage kernels of pkh_stage.hip (up to the persistent batch kernel and the
    host-side launchers that follow them), the device helpers and pointwise
    physics they include, and the layouts of the structures they read from
    pkh_internal.h. Host-side changes (launch shapes, tables, entry points)
    leave it unchanged."""
    import re
    csrc = os.path.join(ROOT, "paper_2202_12309_amd", "csrc")
    st = open(os.path.join(csrc, "pkh_stage.hip")).read()
    parts = [st[:st.index(STAGE_END_MARK)] if STAGE_END_MARK in st else st]
    for f in ("pkh_device.h", "pkh_physics.h"):
        parts.append(open(os.path.join(csrc, f)).read())
    inter = open(os.path.join(csrc, "pkh_internal.h")).read()
    for name in DEVICE_STRUCTS:
        m = re.search(r"struct %s \{.*?\n\};" % name, inter, re.S)
        parts.append(m.group(0) if m else name)
    parts += re.findall(r"^constexpr int [A-Z]+ = \d+;|^enum : int \{[^}]*\};", inter, re.M)
    return "\n".join(parts)


def stage_source_sha():
    """SHA-256 of the stage kernels' device source (stage_device_source): the
    committed rocprofv3 counters are used only while it is unchanged."""
    return hashlib.sha256(stage_device_source().encode()).hexdigest()


def algorithmic_bytes(n):
    """Bytes per zone for the corrector kernel and for the whole cycle, FP64,
    5 variables (40 B per cell and state), counting the face halo each stage
    reads (x, y and z neighbours of the block's faces; no edges or corners):
    h = 1 + 12/n cells per zone for the two-cell halo of the piecewise-linear
    corrector, h1 = 1 + 6/n for the one-cell halo of the donor-cell
    predictor; no ghost zones are written.

    Corrector: read U* (h * 40 B), read U^n (40 B), write U^(n+1) (40 B).
    Predictor: h1 * 40 + 40. Cycle: 40 h + 40 h1 + 120 (222.5 B at n = 32)."""
    h = 1.0 + 12.0 / n
    h1 = 1.0 + 6.0 / n
    return h * 40.0 + 80.0, 40.0 * h + 40.0 * h1 + 120.0


def stage_floor_bytes():
    """The stage-wise floor of the method, FP64, 5 variables: each stage reads
    its input state and writes its output once, the corrector also reads U^n
    (no halo re-reads): corrector 40 + 40 + 40 = 120 B per zone, the cycle
    (40 + 40) + 120 = 200 B per zone-cycle."""
    return 120.0, 200.0


def ghost_materialised_bytes(n):
    """Bytes per zone-cycle of a design that writes and reads 26-region
    ghost zones after every stage, 240 r_g - 40 with r_g = (n+4)^3 / n^3
    (302 B at n = 32): the reference figure the HBM target is quoted at."""
    rg = (n + 4) ** 3 / n ** 3
    return 240.0 * rg - 40.0


def traffic_from_profile(kernel_sha):
    """Measured HBM bytes per corrector launch from the committed rocprofv3
    counter summary, when it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "corrector_256cube_32blocks_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_sha256") != kernel_sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def valu_from_profile(kernel_sha):
    """VALU instructions and issue floor per stage launch from the committed
    SQ_INSTS_VALU summary, when it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernels_256cube_32blocks_valu.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_sha256") != kernel_sha:
        return None
    return rec


def cpu_baseline(blk):
    """The oracle, as it stands, compiled -O3 -march=native -fopenmp on this
    host and timed on the same 256^3 workload in a child process: all cores
    of the process (OMP_NUM_THREADS, else its CPU affinity) over 4 cycles and
    one core over 1 cycle, median of 3 runs each."""
    import subprocess
    r = subprocess.run([sys.executable, "-m", "oracle.timing", "--block", str(blk)], cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError("oracle timing failed: " + r.stderr[-2000:])
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    a, o = rec["all_core"], rec["one_core"]
    return {"value": a["zone_cycles_per_s"], "unit": "zone-cycles/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": f"{a['cycles']} full cycles of the same 256^3 mesh per run "
                      f"({N ** 3 * a['cycles']} zone-cycles), median of {len(a['seconds'])} runs "
                      f"({a['median_s']} s); one core: {o['cycles']} cycle per run, median "
                      f"{o['median_s']} s",
            "build": rec["build"], "cpu_model": rec["cpu_model"], "affinity_cpus": rec["affinity_cpus"],
            "single_core": {"value": o["zone_cycles_per_s"], "cores": 1},
            "runs_s": {"all_core": a["seconds"], "one_core": o["seconds"]}}


def adjoint_ratio(cycles=50, ckpt=10):
    """Reverse mode on 128^3 FP64 as 64 blocks of 32^3: 50 cycles from a
    smooth seeded density perturbation (amplitude 1e-3, |k|_inf <= 4),
    checkpoint every 10 cycles; loss = L2 misfit of the final density to a
    seeded target. Returns the per-cycle cost of the reverse sweep (the
    adjoint stage kernels only) and of the whole gradient (recomputation
    included) relative to one plain forward cycle (pkh_step, no tape) of the
    same mesh."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    Nn, blk = 128, 32
    n = (blk,) * 3
    nrb = (Nn // blk,) * 3
    mesh = Mesh((Nn,) * 3, n, inputs.uniform_leaves(nrb))
    lv = mesh.leaves()
    U0 = inputs.smooth_density(lv, n, nrb, seed=5)
    tgt = torch.tensor(inputs.smooth_density(lv, n, nrb, seed=6)[:, 0], device="cuda")
    tape = mesh.tape(ckpt)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for rep in range(2):  # the second repetition is timed
        mesh.upload(U0)
        mesh.sync()
        ev[0].record(mesh.stream)
        tape.forward(cycles)
        ev[1].record(mesh.stream)
        UN = mesh.download(device=True)
        lam = torch.zeros_like(UN)
        lam[:, 0] = (UN[:, 0] - tgt) / Nn ** 3
        torch.cuda.synchronize()
        mesh.kernel_timing(Mesh.KT_ADJOINT)
        ev[2].record(mesh.stream)
        tape.adjoint(lam)
        ev[3].record(mesh.stream)
        ev[3].synchronize()
        kt = mesh.kernel_times()
        mesh.kernel_timing(0)
    t_taped = ev[0].elapsed_time(ev[1]) / cycles
    t_adj = ev[2].elapsed_time(ev[3]) / cycles
    t_rev = kt["adjoint"][0] / cycles
    # the denominator: plain forward cycles (no tape) of the same mesh and state
    tape.close()
    mesh.upload(U0)
    mesh.step(5)
    mesh.sync()
    ev[0].record(mesh.stream)
    mesh.step(cycles)
    ev[1].record(mesh.stream)
    ev[1].synchronize()
    t_fwd = ev[0].elapsed_time(ev[1]) / cycles
    mesh.close()
    return {"workload": "128^3 FP64, 64 blocks of 32^3, 50 cycles, checkpoint every 10",
            "forward_ms_per_cycle": round(t_fwd, 4), "taped_forward_ms_per_cycle": round(t_taped, 4),
            "reverse_sweep_ms_per_cycle": round(t_rev, 4),
            "gradient_ms_per_cycle": round(t_adj, 4),
            "reverse_sweep_over_forward": round(t_rev / t_fwd, 3),
            "gradient_over_forward": round(t_adj / t_fwd, 3)}


def batch_leg(cycles=50):
    """64 independent FP64 periodic instances (edges 32..128, blocks 16^3 or
    32^3, sound-wave or blast initial conditions; seed 4): aggregate
    zone-cycles/s of the plain per-instance launches, the grouped launches,
    the captured-graph replays, the persistent launch, and the graph and the
    persistent launch after autotuning (tile rows of the grouped launches,
    waves per SIMD of the persistent kernel)."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Batch, Mesh
    specs = inputs.batch_mix(n=64, seed=4)
    stream = torch.cuda.Stream()
    meshes = []
    cells = 0
    for sp in specs:
        n = (sp["blk"],) * 3
        nrb = (sp["N"] // sp["blk"],) * 3
        m = Mesh((sp["N"],) * 3, n, inputs.uniform_leaves(nrb), stream=stream)
        m.upload(inputs.batch_state(sp, m.leaves()))
        meshes.append(m)
        cells += sp["N"] ** 3
    b = Batch(meshes)
    out = {"workload": "64 instances, edges 32..128, blocks 16^3/32^3, wave or blast, seed 4",
           "cells": cells, "cycles_timed": cycles}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for label, mode, tune in (("plain", "plain", False), ("fused", "fused", False),
                              ("graph", "graph", False), ("persistent", "persistent", False),
                              ("graph_autotuned", "graph", True), ("persistent_autotuned", "persistent", False)):
        if tune:
            out["autotuned_tile_rows"] = sorted(set(b.autotune(3)))
            out["autotuned_persistent_waves_per_simd"] = b.tuning()["waves_per_simd"]
        b.step(cycles, mode)  # warm-up (and graph capture)
        torch.cuda.synchronize()
        ev0.record(stream)
        b.step(cycles, mode)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1)
        out[label] = cells * cycles / (ms / 1e3)
    out["speedup_graph_vs_plain"] = out["graph_autotuned"] / out["plain"]
    out["speedup_persistent_vs_plain"] = out["persistent_autotuned"] / out["plain"]
    out["speedup_persistent_vs_fused"] = out["persistent_autotuned"] / out["fused"]
    b.close()
    return out


def amr_leg(cycles=200, regrid_every=10):
    """Two-level blast: 128^3 root in blocks of 16^3, the root blocks meeting
    the open ball r < 0.25 refined once (960 leaves), P = 100 inside r < 0.1
    and 0.1 outside, rho = 1 at rest. Every 10 cycles the device
    pressure-jump indicator sets the flags (refine above 0.1, derefine below
    0.02) and the mesh is regridded. Zone-cycles count the leaf cells of
    every cycle; the time includes the indicator and the regrids."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    blk, nrb = 16, (8, 8, 8)
    n = (blk,) * 3
    lv = inputs.sphere_refined_leaves(nrb, radius=0.25)
    # warm-up on a throwaway mesh of the same layout (cycles, indicator,
    # regrid), so the first launch of each kernel stays out of the timed
    # region as in the other legs
    w = Mesh((128,) * 3, n, lv, max_level=1)
    w.upload(inputs.blast(w.leaves(), n, nrb))
    w.step(2)
    w.flag_pressure_jump(0.1, 0.02)
    w.regrid()
    w.step(1)
    w.sync()
    w.close()
    mesh = Mesh((128,) * 3, n, lv, max_level=1)
    mesh.upload(inputs.blast(mesh.leaves(), n, nrb))
    mesh.sync()
    leaves0 = mesh.nleaves
    counts = []
    zc = 0
    t_regrid = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(cycles // regrid_every):
        zc += mesh.nleaves * blk ** 3 * regrid_every
        mesh.step(regrid_every)
        t1 = time.perf_counter()
        mesh.flag_pressure_jump(0.1, 0.02)  # waits for the cycles
        t2 = time.perf_counter()
        mesh.regrid()
        t_regrid += time.perf_counter() - t2
        counts.append(mesh.nleaves)
    mesh.sync()
    el = time.perf_counter() - t0
    t, dt, cyc = mesh.time()
    return {"workload": "two-level blast, 128^3 root in 16^3 blocks, sphere r=0.25 refined once, "
                        "regrid every 10 cycles (pressure-jump flags 0.1 / 0.02)",
            "cycles": cyc, "zone_cycles": zc, "seconds": round(el, 4),
            "zone_cycles_per_s": zc / el, "regrid_seconds": round(t_regrid, 4),
            "leaves_start": leaves0, "leaves_after_each_regrid": counts, "sim_time": t}


def kh_leg(cycles=3000, regrid_every=10):
    """Kelvin-Helmholtz shear layers with dynamic refinement: 64^3 root in
    blocks of 16^3, up to level 2 (256^3 at the finest), seed amplitude 0.1.
    The mesh is first adapted twice to the initial state by the device
    density-jump indicator (refine above 0.02, derefine below 0.005); then
    every 10 cycles the indicator sets the flags and the mesh is regridded.
    Zone-cycles count the leaf cells of every cycle; the time includes the
    indicator and the regrids."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    blk, nrb = 16, (4, 4, 4)
    n = (blk,) * 3
    mesh = Mesh((64,) * 3, n, inputs.uniform_leaves(nrb), max_level=2)
    for _ in range(2):
        mesh.upload(inputs.kelvin_helmholtz(mesh.leaves(), n, nrb, amp=0.1))
        mesh.flag_density_jump(0.02, 0.005)
        mesh.regrid()
    mesh.upload(inputs.kelvin_helmholtz(mesh.leaves(), n, nrb, amp=0.1))
    mesh.sync()
    leaves0 = mesh.nleaves
    counts = []
    zc = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(cycles // regrid_every):
        zc += mesh.nleaves * blk ** 3 * regrid_every
        mesh.step(regrid_every)
        mesh.flag_density_jump(0.02, 0.005)  # waits for the cycles
        mesh.regrid()
        counts.append(mesh.nleaves)
    mesh.sync()
    el = time.perf_counter() - t0
    t, dt, cyc = mesh.time()
    mesh.close()
    return {"workload": "Kelvin-Helmholtz, 64^3 root in 16^3 blocks, max level 2, seed 0.1, "
                        "regrid every 10 cycles (density-jump flags 0.02 / 0.005)",
            "cycles": cyc, "zone_cycles": zc, "seconds": round(el, 4),
            "zone_cycles_per_s": zc / el, "leaves_start": leaves0,
            "leaves_min": min(counts), "leaves_max": max(counts), "leaves_end": counts[-1],
            "sim_time": t}


def packs_leg(cycles=20, warmup=3):
    """The paper's MeshBlockPack knob on the 256^3 turbulent box: each stage
    launched once per pack of contiguous leaves (packs = 1 is one launch
    over all leaves), for blocks of 32^3 (512 leaves) and 16^3 (4096
    leaves). Zone-cycles/s per pack count, HIP events on the mesh stream."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    out = {"workload": "256^3 turbulent box (seed 2), 20 cycles per point"}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for blk, packs in ((32, (1, 2, 4, 8, 16, 64, 512)), (16, (1, 4, 16, 64, 256, 1024, 4096))):
        n = (blk,) * 3
        nrb = (N // blk,) * 3
        mesh = Mesh((N,) * 3, n, inputs.uniform_leaves(nrb))
        mesh.upload(inputs.turbulent_box(mesh.leaves(), n, nrb, seed=2))
        res = {}
        for P in packs:
            mesh.set_tuning(0, P)
            mesh.step(warmup)
            torch.cuda.synchronize()
            ev0.record(mesh.stream)
            mesh.step(cycles)
            ev1.record(mesh.stream)
            ev1.synchronize()
            res[str(P)] = N ** 3 * cycles / (ev0.elapsed_time(ev1) / 1e3)
        out[f"block_{blk}"] = res
        mesh.close()
    return out


def block_sweep_leg(cycles=20, warmup=5):
    """The 256^3 turbulent box (seed 2) cut into blocks of 16^3 (4096), 32^3
    (512) and 64^3 (64), one pack, default tiles: zone-cycles/s and the
    stage-kernel times for each block size."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    out = {"workload": f"256^3 turbulent box (seed 2), {cycles} cycles per point"}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fields = inputs.turbulent_box_global((N, N, N), seed=2)
    for blk in (16, 32, 64):
        n = (blk,) * 3
        nrb = (N // blk,) * 3
        mesh = Mesh((N,) * 3, n, inputs.uniform_leaves(nrb))
        mesh.upload(inputs.scatter_global(fields, mesh.leaves(), n))
        mesh.step(warmup)
        mesh.sync()
        mesh.kernel_timing(Mesh.KT_PREDICTOR | Mesh.KT_CORRECTOR)
        torch.cuda.synchronize()
        ev0.record(mesh.stream)
        mesh.step(cycles)
        ev1.record(mesh.stream)
        ev1.synchronize()
        kt = mesh.kernel_times()
        ms = ev0.elapsed_time(ev1) / cycles
        out[f"block_{blk}"] = {"blocks": len(mesh.leaves()), "tile_rows": mesh.tuning()["tile_rows"],
                               "ms_per_cycle": round(ms, 4), "zone_cycles_per_s": N ** 3 / (ms / 1e3),
                               "predictor_ms": round(kt["predictor"][0] / kt["predictor"][1], 4),
                               "corrector_ms": round(kt["corrector"][0] / kt["corrector"][1], 4)}
        mesh.close()
        torch.cuda.empty_cache()
    return out


def remote_leg(cycles=20, warmup=3):
    """The multi-GPU data path on one GPU: the 256^3 turbulent box in 512
    blocks of 32^3 cut into P contiguous Morton parts; same-level faces
    between parts are packed, moved as one device copy per (sender,
    receiver) pair and unpacked after each stage. Zone-cycles/s, the
    exchange time per cycle and the bytes one exchange moves per cycle."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    blk = 32
    n = (blk,) * 3
    nrb = (N // blk,) * 3
    mesh = Mesh((N,) * 3, n, inputs.uniform_leaves(nrb))
    mesh.upload(inputs.turbulent_box(mesh.leaves(), n, nrb, seed=2))
    out = {"workload": "256^3 turbulent box (seed 2), 512 blocks of 32^3, 20 cycles per point"}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for P in (1, 2, 8, 64, 512):
        mesh.set_partition(P)
        info = mesh.partition()
        mesh.step(warmup)
        torch.cuda.synchronize()
        ev0.record(mesh.stream)
        mesh.step(cycles)
        ev1.record(mesh.stream)
        ev1.synchronize()
        zcs = N ** 3 * cycles / (ev0.elapsed_time(ev1) / 1e3)
        mesh.kernel_timing(Mesh.KT_REMOTE)
        mesh.step(cycles)
        kt = mesh.kernel_times()["remote"]
        mesh.kernel_timing(0)
        # two stages per cycle, 2 layers x 32^2 cells x 40 B per remote face
        mbytes = 2 * info["remote_faces"] * 2 * blk * blk * 40
        out[str(P)] = {"zone_cycles_per_s": zcs, "remote_faces": info["remote_faces"],
                       "messages_per_stage": info["messages"],
                       "exchange_ms_per_cycle": round(kt[0] / cycles, 4),
                       "message_bytes_per_cycle": mbytes}
    mesh.close()
    return out


def fp32_leg(steps=100, warmup=10, blk=32):
    """The 256^3 cycle with the state stored in FP32 (FP64 arithmetic, each
    stage rounding its output once): zone-cycles/s, stage-kernel times, the
    algorithmic bytes (20 B per cell and state: corrector h*20 + 40, cycle
    40 h + 60) and the distance from the FP64-stored run after the same
    cycles."""
    import numpy as np
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _helpers import rel_err  # per-variable error scales (no method arithmetic)
    n = (blk,) * 3
    nrb = (N // blk,) * 3
    lv = inputs.uniform_leaves(nrb)
    U0 = inputs.turbulent_box(lv, n, nrb, seed=2).astype(np.float32).astype(np.float64)
    res = {}
    for fp32 in (True, False):
        mesh = Mesh((N,) * 3, n, lv, fp32_state=fp32)
        mesh.upload(U0)
        mesh.step(warmup)
        mesh.sync()
        mesh.kernel_timing(Mesh.KT_PREDICTOR | Mesh.KT_CORRECTOR)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(mesh.stream)
        mesh.step(steps)
        ev1.record(mesh.stream)
        ev1.synchronize()
        kt = mesh.kernel_times()
        res[fp32] = (ev0.elapsed_time(ev1) / steps, kt, mesh.download())
        mesh.close()
    ms, kt, U32 = res[True]
    h = 1.0 + 12.0 / blk
    b_corr, b_cycle = h * 20.0 + 40.0, 40.0 * h + 60.0
    corr_ms = kt["corrector"][0] / max(kt["corrector"][1], 1)
    zcs = N ** 3 / (ms / 1e3)
    return {"workload": f"hydro 256^3, 512 blocks of 32^3, FP32 state storage, FP64 arithmetic, "
                        f"{warmup} + {steps} cycles",
            "zone_cycles_per_s": zcs, "ms_per_step": round(ms, 4),
            "kernel_avg_ms": {"predictor": round(kt["predictor"][0] / max(kt["predictor"][1], 1), 4),
                              "corrector": round(corr_ms, 4)},
            "bytes_per_zone_cycle": b_cycle,
            "hbm_frac_cycle": round(zcs * b_cycle / (HBM_PEAK_GBS * 1e9), 4),
            "corrector_hbm_frac": round(b_corr * N ** 3 / (corr_ms / 1e3) / (HBM_PEAK_GBS * 1e9), 4),
            "fp64_ms_per_step": round(res[False][0], 4),
            "speedup_vs_fp64_storage": round(res[False][0] / ms, 3),
            "rel_err_vs_fp64_storage": [float(x) for x in rel_err(U32, res[False][2], 5.0 / 3.0)]}


def deep_amr_leg(cycles=10):
    """The paper's multilevel mesh: 256^3 root grid in blocks of 32^3, a
    centred cube of side 0.4 refined to level 3 (296, 1216, 1352 and 21952
    leaves on levels 0-3: 24,816 blocks, 813M zones), a spherical blast
    inside the refined cube, static mesh. Zone-cycles/s over the timed
    cycles and the per-kernel split (stage kernels, level-jump face fill,
    flux correction)."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh
    n, nrb = (32, 32, 32), (8, 8, 8)
    lv = inputs.cube_refined_leaves(nrb)
    mesh = Mesh((256,) * 3, n, lv, max_level=3)
    U0 = inputs.blast(mesh.leaves(), n, nrb)
    mesh.upload(U0)
    del U0
    mesh.step(2)  # warm-up
    mesh.sync()
    mesh.kernel_timing(Mesh.KT_PREDICTOR | Mesh.KT_CORRECTOR | Mesh.KT_FILL | Mesh.KT_FLUXCORR)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(mesh.stream)
    mesh.step(cycles)
    ev1.record(mesh.stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    kt = mesh.kernel_times()
    mesh.sync()
    cells = len(lv) * n[0] * n[1] * n[2]
    counts = [int((lv[:, 0] == L).sum()) for L in range(4)]
    out = {"workload": "paper multilevel mesh: 256^3 root, 32^3 blocks, 0.4 cube to level 3, blast",
           "leaves_per_level": counts, "cells": cells, "cycles_timed": cycles,
           "ms_per_cycle": round(ms / cycles, 4), "zone_cycles_per_s": cells * cycles / (ms / 1e3),
           "kernel_ms_per_cycle": {k: round(v[0] / cycles, 4) for k, v in kt.items() if v[1]}}
    mesh.close()
    return out


def main_leg(args):
    """The 256^3 hydro cycle: zone-cycles/s, stage-kernel times and the
    corrector's roofline."""
    import torch
    from paper_2202_12309_amd import inputs
    from paper_2202_12309_amd.binding import Mesh

    blk = args.block
    n = (blk,) * 3
    nrb = (N // blk,) * 3
    lv = inputs.uniform_leaves(nrb)
    mesh = Mesh((N, N, N), n, lv, graph=args.graph)
    mesh.set_tuning(args.tile_rows)
    U0 = inputs.turbulent_box(mesh.leaves(), n, nrb, seed=2)
    mesh.upload(U0)
    mesh.step(args.warmup)
    mesh.sync()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(mesh.stream)
    mesh.step(args.steps)
    ev1.record(mesh.stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    mesh.sync()
    t, dt, cyc = mesh.time()
    # per-kernel launch times from a second run with events around each
    # launch (after the timed region, so its markers do not enter `value`)
    kinds = Mesh.KT_PREDICTOR | Mesh.KT_CORRECTOR | Mesh.KT_FILL
    mesh.kernel_timing(kinds)
    mesh.step(min(args.steps, 50))
    mesh.sync()
    kt = mesh.kernel_times()
    mesh.kernel_timing(0)
    # Host buffers through the boundary, after the timed region: upload from
    # host memory (pageable numpy), the same cycles, download to host memory.
    mesh.sync()
    h0 = time.perf_counter()
    mesh.upload(U0)
    mesh.sync()
    h1 = time.perf_counter()
    mesh.step(args.steps)
    mesh.sync()
    h2 = time.perf_counter()
    mesh.download()
    h3 = time.perf_counter()
    pcie = {"what": f"upload of the state from host memory, {args.steps} cycles, download to host memory",
            "upload_s": round(h1 - h0, 4), "cycles_s": round(h2 - h1, 4), "download_s": round(h3 - h2, 4),
            "state_bytes": int(U0.nbytes),
            "zone_cycles_per_s": N ** 3 * args.steps / (h3 - h0)}

    zc = N ** 3 * args.steps / (ms / 1e3)
    b_corr, b_cycle = algorithmic_bytes(blk)
    cells = N ** 3
    avg = {k: (v[0] / v[1] if v[1] else None) for k, v in kt.items()}
    corr_ms = avg["corrector"]
    roof = None
    if corr_ms:
        b_floor = stage_floor_bytes()[0]
        ach = b_floor * cells / (corr_ms / 1e3) / 1e9
        ach_halo = b_corr * cells / (corr_ms / 1e3) / 1e9
        sha = stage_source_sha()
        roof = {"bound": "hbm", "kernel": "stage_kernel<PLM> (corrector)",
                "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profile(sha),
                "algorithmic_bytes_per_zone": b_floor,
                "algorithmic_bytes_per_launch": int(b_floor * cells),
                "avg_launch_ms": round(corr_ms, 4),
                "halo_model": {"bytes_per_zone": round(b_corr, 3), "achieved": round(ach_halo, 1),
                               "frac": round(ach_halo / HBM_PEAK_GBS, 4)}}
        # the second ceiling: FP64 VALU issue (one wave64 instruction holds a
        # SIMD for 4 cycles) for the instructions the counters saw per launch
        vr = valu_from_profile(sha)
        if vr and blk == 32 and args.tile_rows == 0:
            c = vr["corrector"]
            roof["valu"] = {"instructions_per_cell": round(c["valu_instructions_per_cell"], 1),
                            "floor_ms": round(c["valu_floor_ms"], 4),
                            "frac": round(c["valu_floor_ms"] / corr_ms, 4)}
        # the same launch against the FP64 vector peak, counting the
        # method's own operations (corrector and the fused CFL reduction)
        fl = (ALG_FLOPS["corrector"] + ALG_FLOPS["cfl"]) * cells / (corr_ms / 1e3) / 1e12
        roof["alu"] = {"flops_per_zone": ALG_FLOPS["corrector"] + ALG_FLOPS["cfl"],
                       "achieved": round(fl, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(fl / FP64_PEAK_TFLOPS, 4)}
    out = {
        "metric": METRIC,
        "value": zc,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hydro 256^3 FP64 periodic, {len(lv)} blocks of {blk}^3, one pack; "
                               "log-normal density (sigma 0.5), P=1, rms Mach 0.5, seed 2; VL2 "
                               "PLM-MC + HLLE, CFL 0.3",
                   "cells": cells, "block": blk, "blocks": len(lv), "graph": bool(args.graph),
                   "tile_rows": mesh.tuning()["tile_rows"]},
        "hbm_frac_cycle": round(zc * b_cycle / (HBM_PEAK_GBS * 1e9), 4),
        "hbm_frac_cycle_at_stage_floor": round(zc * stage_floor_bytes()[1] / (HBM_PEAK_GBS * 1e9), 4),
        "bytes_per_zone_cycle": round(b_cycle, 2),
        "flops_per_zone_cycle": sum(ALG_FLOPS.values()),
        "fp64_tflops_cycle": round(zc * sum(ALG_FLOPS.values()) / 1e12, 3),
        "hbm_frac_at_ghost_materialised_bytes": round(zc * ghost_materialised_bytes(blk) / (HBM_PEAK_GBS * 1e9),
                                                      4),
        "kernel_avg_ms": {k: (round(v, 4) if v else None) for k, v in avg.items()},
        "sim_time": t,
        "roofline": roof,
        "pcie_inclusive": pcie,
    }
    del mesh
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--block", type=int, default=32, choices=[16, 32, 64])
    ap.add_argument("--graph", action="store_true", help="replay captured cycles")
    ap.add_argument("--tile-rows", type=int, default=0, help="stage-kernel tile rows (0: default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-kh", action="store_true")
    ap.add_argument("--no-block-sweep", action="store_true",
                    help="skip the 256^3 cycle in blocks of 16^3 and 64^3 beside 32^3")
    ap.add_argument("--fp32-storage", action="store_true",
                    help="also run the 256^3 cycle with the state stored in FP32")
    ap.add_argument("--remote-split", action="store_true",
                    help="also time the pack / transfer / unpack path of a virtual partition")
    ap.add_argument("--packs-sweep", action="store_true",
                    help="also sweep the number of stage launches per stage (MeshBlockPacks)")
    ap.add_argument("--no-deep-amr", action="store_true",
                    help="skip the paper's four-level mesh (813M zones, ~130 GB of HBM)")
    ap.add_argument("--no-main", action="store_true",
                    help="skip the 256^3 leg (for profiling the other legs alone)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (the HBM-counter calibration kernel)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding across GPUs is "
              "not built (its data path runs on one GPU through pkh_set_partition).", file=sys.stderr)
        sys.exit(2)

    import torch

    blk = args.block
    if args.no_main:
        out = {"metric": METRIC, "value": None, "unit": "zone-cycles/s", "n_gpus": 1, "steps": 0,
               "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "main 256^3 leg skipped"}, "roofline": None}
    else:
        out = main_leg(args)
    out.update({"adjoint_forward_ratio": None, "adjoint": None, "batch": None, "amr": None, "packs_sweep": None,
                "kh_amr": None, "deep_amr": None, "block_sweep": None})
    if not args.no_adjoint:
        adj = adjoint_ratio()
        out["adjoint"] = adj
        # both readings of the cost ratio against plain forward cycles: the
        # reverse sweep of a cycle with its intermediates at hand, and the
        # whole gradient with the checkpoint recomputation
        out["adjoint_forward_ratio"] = {"reverse_sweep": adj["reverse_sweep_over_forward"],
                                        "gradient_with_recompute": adj["gradient_over_forward"]}
    if not args.no_block_sweep:
        torch.cuda.empty_cache()
        out["block_sweep"] = block_sweep_leg()
    if not args.no_amr:
        out["amr"] = amr_leg()
    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batch"] = batch_leg()
    if args.fp32_storage:
        torch.cuda.empty_cache()
        out["fp32_storage"] = fp32_leg()
    if args.remote_split:
        torch.cuda.empty_cache()
        out["remote_split"] = remote_leg()
    if args.packs_sweep:
        torch.cuda.empty_cache()
        out["packs_sweep"] = packs_leg()
    if not args.no_kh:
        torch.cuda.empty_cache()
        out["kh_amr"] = kh_leg()
    if not args.no_deep_amr:
        torch.cuda.empty_cache()
        out["deep_amr"] = deep_amr_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(blk)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
