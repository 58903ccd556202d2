#!/usr/bin/env python3
"""Benchmark of the coupled D3Q19 lattice-Boltzmann / DEM step on one MI355X.

Workload (the FCC wave-propagation case): a 4 x 4 x 16 FCC packing of 1024 spheres (cell
edge 24 lu, touching radius plus a seed-jittered 1e-3 overlap) in a 96 x 96 x 384
lattice, periodic in x and y, density inlet at z = 0 driven by a single-period cosine
(amplitude 1e-3, period 200 steps), constant density at z = 383, probes every 16 lu,
tau = 1, Hertz-Mindlin spheres with E* = 10.37, nu = 0.2, mu = 0, rho_p* = 2.466.

One step = one pass of the whole coupled path (fluid, link, motion and re-projection
kernels, replayed from a HIP graph).  ``value`` is fluid-node updates per second
(millions) over K timed steps with all data resident in HBM; ``roofline`` prices the
fluid kernel's algorithmic bytes (19 populations read and written per fluid node)
against 8 TB/s, using its average duration from HIP events recorded around each launch
on the library's stream in eager steps of the same set.  ``traffic`` is the HBM bytes
per launch of that kernel from the committed rocprofv3 counter summary (FETCH_SIZE and
WRITE_SIZE scaled by a calibration copy), reported only while the kernel source is the
one the counters were taken on.
The FP16 / BF16 deviation-storage variants and their errors against the FP64 path are
reported beside it, and the FP64 CPU oracle is timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_VALUE = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _case(seed=0):
    from paper_1808_08921_amd import inputs

    params, pk = inputs.wave_fcc_case(seed=seed)
    params["max_particles"] = len(pk["x"])
    return params, pk


def _make(params, pk, precision, graph_steps=8, probe_ring=4096):
    from paper_1808_08921_amd.lbdem import LatticeSet

    gs = LatticeSet([params], precision=precision, graph_steps=graph_steps, probe_ring=probe_ring)
    gs.particles_set(0, pk["x"], pk["radius"], fixed=pk["fixed"])
    return gs


def _fluid_nodes(gs):
    return int((gs.owner(0) < 0).sum())


def time_steps(gs, steps, warmup):
    import torch

    gs.step(warmup)
    gs.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs.step(steps)
    gs.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_times(gs, steps):
    """Average duration of each kernel over `steps` eager steps, from HIP events recorded
    on the library's stream around every launch."""
    gs.timing_enable(True)
    gs.step(steps)
    ms, cnt = gs.timing_read()
    gs.timing_enable(False)
    return ms / np.maximum(cnt, 1)


def arrival_velocity(probes, zs, tmax):
    """P-wave speed from the arrival time of the peak cross-section momentum
    sum(rho u_z)/sum(rho) at each probe plane (3-point parabolic refinement of the
    argmax), fitted by least squares over the planes."""
    mom = probes[:tmax, :, 2] / probes[:tmax, :, 3]
    times = []
    for k in range(mom.shape[1]):
        s = mom[:, k]
        i = int(np.argmax(s))
        if 0 < i < len(s) - 1:
            a, b, c = s[i - 1], s[i], s[i + 1]
            den = a - 2 * b + c
            i = i + (0.5 * (a - c) / den if den != 0 else 0.0)
        times.append(i + 1.0)
    slope = np.polyfit(np.asarray(times), np.asarray(zs, float), 1)[0]
    return float(slope), times


def front_velocity(probes, zs, tmax):
    """Front speed of a step source: the first step at which the cross-section averaged
    density rho' reaches half of its largest value at each probe plane (the pulse weakens
    along the packing), fitted by least squares over the planes."""
    rho = probes[:tmax, :, 1] / probes[:tmax, :, 0]
    times = [float(np.argmax(rho[:, k] >= 0.5 * rho[:, k].max()) + 1) for k in range(rho.shape[1])]
    return float(np.polyfit(np.asarray(times), np.asarray(zs, float), 1)[0])


def precision_errors(params, pk, steps=20000, arrival_steps=900, planes=12, every=100):
    """Error of each storage precision against the FP64 GPU path (itself checked against
    the FP64 CPU oracle to 1e-10 by the test-suite) over the workload's full length: the
    P-wave arrival speed (planes 1-12, from the first `arrival_steps` steps, before the
    outlet's reflection comes back), particle velocities sampled every `every` steps and
    the cross-section averaged density of every probe plane at every step."""
    out = {}
    ref = None
    zs = list(params["probe_z"])[1:planes + 1]
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        gs = _make(params, pk, prec, graph_steps=8, probe_ring=steps)
        vs = []
        for _ in range(steps // every):
            gs.step(every)
            vs.append(gs.particles_get(0)["v"])
        probes = gs.probes(0, 0, steps)
        status = gs.status()
        vel, _ = arrival_velocity(probes[:, 1:planes + 1, :], zs, arrival_steps)
        vs = np.stack(vs)
        gs.close()
        rho = probes[..., 1] / np.maximum(probes[..., 0], 1.0)
        if prec == "fp64":
            ref = (vel, vs, rho)
            out[prec] = {"p_wave_velocity": vel, "steps": steps, "status": status,
                         "max_particle_speed": float(np.abs(vs).max())}
            continue
        out[prec] = {
            "p_wave_velocity": vel,
            "p_wave_velocity_rel_err": abs(vel - ref[0]) / abs(ref[0]),
            "particle_velocity_rel_err": float(np.linalg.norm(vs - ref[1]) / np.linalg.norm(ref[1])),
            "probe_rho_prime_rel_err": float(np.abs(rho - ref[2]).max() / np.abs(ref[2]).max()),
            "steps": steps, "status": status,
        }
    return out


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo and the process's
    CPU affinity)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail, os.cpu_count()


def _oracle_steps(params, pk, budget_s, max_steps, ready=None):
    """Steps of the oracle on the full FCC case until about `budget_s` seconds have passed
    (at most `max_steps`); `ready` is called after the set-up, before the timed loop.
    Returns (fluid nodes, steps, seconds)."""
    import oracle

    p = params
    s = oracle.Sim(p["nx"], p["ny"], p["nz"], tau=p["tau"], bc=p["bc"], wave=p["wave"], amp=p["amp"],
                   omega=p["omega"], t_n=p["t_n"], E=p["E"], nu=p["nu"], mu=p["mu"], rho_p=p["rho_p"],
                   probe_z=p["probe_z"])
    s.set_particles(pk["x"], pk["radius"], fixed=pk["fixed"])
    nfl = int((s.owner() < 0).sum())
    if ready is not None:
        ready()
    t0 = time.perf_counter()
    n = 0
    while True:
        s.step(1)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= max_steps:
            break
    dt = time.perf_counter() - t0
    s.close()
    return nfl, n, dt


def cpu_worker(budget_s):
    """One process of the all-core baseline: set up, report, wait for the start line on
    stdin, run the timed steps and print (fluid nodes, steps, seconds) as JSON."""
    params, pk = _case(seed=0)

    def ready():
        print("ready", flush=True)
        sys.stdin.readline()

    nfl, n, dt = _oracle_steps(params, pk, budget_s, 1 << 30, ready)
    print(json.dumps({"fluid_nodes": nfl, "steps": n, "seconds": dt}), flush=True)


def cpu_baseline(params, pk, budget_s=15.0, all_core_s=15.0, max_procs=16):
    """The FP64 oracle on the host on the same workload, timed two ways: one thread (steps of
    the full 96 x 96 x 384 lattice until about `budget_s` seconds have passed), and every
    available core, as one independent oracle process per core stepping its own copy of the
    case (the oracle itself is single-threaded and is not changed for this); the processes
    start their timed loops together and the whole host's rate is the sum of theirs."""
    import subprocess

    import oracle

    oracle.build()
    nfl, n, dt = _oracle_steps(params, pk, budget_s, 50)
    model, avail, total = host_cpu()
    single = {"value": nfl * n / dt / 1e6, "unit": "MLUPS (fluid nodes)", "cores": 1,
              "sample": f"{n} full steps of the 96x96x384 FCC case (oracle, FP64, one host thread)"}
    k = max(1, min(avail or 1, max_procs))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(all_core_s)],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
             for _ in range(k)]
    try:
        for pr in procs:
            if pr.stdout.readline().strip() != "ready":
                raise RuntimeError("an oracle worker failed during set-up")
        for pr in procs:
            pr.stdin.write("go\n")
            pr.stdin.flush()
        res = []
        for pr in procs:
            res.append(json.loads(pr.stdout.readline()))
            pr.wait(timeout=600)
    finally:
        for pr in procs:
            if pr.poll() is None:
                pr.kill()
    rate = sum(r["fluid_nodes"] * r["steps"] / r["seconds"] for r in res) / 1e6
    return {"value": rate, "unit": "MLUPS (fluid nodes)", "cores": k, "kind": "oracle",
            "sample": f"{k} concurrent oracle processes (one per available core), "
                      f"{min(r['steps'] for r in res)}-{max(r['steps'] for r in res)} full steps each of "
                      f"the 96x96x384 FCC case (FP64, about {all_core_s:g} s)",
            "single_thread": single, "host_cpu": model, "host_cpus_available": avail, "host_cpus_total": total}


KERNEL_SRC = os.path.join(ROOT, "paper_1808_08921_amd", "csrc", "lbdem_kernels.hip")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_fluid_fcc96x96x384_fp32_counters.txt")


def counters_file(precision):
    """Path of the committed counter summary of the FCC case at one storage precision."""
    return os.path.join(ROOT, "profiles", f"k_fluid_fcc96x96x384_{precision}_counters.txt")
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read and 1 GiB written


def kernel_source_hash():
    import hashlib

    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def counters_workload(steps, precision="fp32"):
    """Workload for the rocprofv3 counter passes: `steps` eager steps of the FCC case at the
    given storage precision, then a plain device-to-device copy of COPY_BYTES that
    calibrates the counters."""
    import torch

    params, pk = _case(seed=0)
    gs = _make(params, pk, precision, graph_steps=0)
    gs.step(steps)
    gs.synchronize()
    gs.close()
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    _log("counter workload done")


def summarize_counters(fetch_csv, write_csv, out_path, command, precision="fp32"):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of each kernel from two rocprofv3 --pmc
    passes, scaled by the same counters' reading for the calibration copy (COPY_BYTES read
    and written), written as a text summary with the kernel source hash."""
    import csv

    def load(path, counter):
        rows = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return rows

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    copy_name = max((k for k in fetch if "copy" in k.lower()), key=lambda k: max(fetch[k]))
    f_scale = COPY_BYTES / (max(fetch[copy_name]) * 1024.0)
    w_scale = COPY_BYTES / (max(write[copy_name]) * 1024.0)
    label = {"fp32": "FP32", "fp16": "FP16 deviations", "bf16": "BF16 deviations"}[precision]
    lines = [f"# rocprofv3 counters, FCC 96x96x384 {label} (1024 spheres), per dispatch",
             f"# command: {command}",
             f"# kernel source sha256[:16]: {kernel_source_hash()}",
             f"# calibration: {copy_name} copying {COPY_BYTES} B reads FETCH_SIZE {max(fetch[copy_name]):.0f} KiB, "
             f"WRITE_SIZE {max(write[copy_name]):.0f} KiB -> scale fetch {f_scale:.4f}, write {w_scale:.4f}",
             "kernel | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) | HBM bytes per dispatch (scaled)"]
    for k in sorted(fetch):
        if k == copy_name or k not in write:
            continue
        fm, wm = float(np.mean(fetch[k])), float(np.mean(write[k]))
        lines.append(f"{k} | {len(fetch[k])} | {fm:.1f} | {wm:.1f} | {(fm * f_scale + wm * w_scale) * 1024.0:.0f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def measured_traffic(kernel_name="lbdem::k_fluid<1, true, false>("):
    """HBM bytes per dispatch of the FP32 fluid kernel from the committed counter summary,
    or None when it is missing or was taken on another version of the kernel source."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    txt = open(COUNTERS_FILE).read()
    if f"sha256[:16]: {kernel_source_hash()}" not in txt:
        return None
    for line in txt.splitlines():
        if kernel_name in line.split("|")[0]:
            return float(line.split("|")[-1])
    return None


def ensemble_bench(n_members, steps, warmup, kernel_steps, precision="fp32", emit=True):
    """The batched-ensemble workload: n_members uneven FCC samples (2x2x8 to 4x4x16 cubic
    cells, overlaps 1e-4..1e-2 R0, inlet periods 50..400 steps) advanced together, one
    launch per kernel per step, graph-replayed; fluid tiles chosen by the autotuner."""
    import torch
    from paper_1808_08921_amd import inputs
    from paper_1808_08921_amd.autotune import autotune
    from paper_1808_08921_amd.lbdem import LatticeSet

    members = inputs.ensemble_members(n_members)
    lats, parts = [], []
    for params, pk in members:
        lats.append(dict(params, max_particles=len(pk["x"])))
        parts.append(pk)
    _log(f"ensemble: {n_members} lattices, {sum(d['nx'] * d['ny'] * d['nz'] for d in lats)} cells")
    tuned, nzt, lists, report = autotune(lats, parts, precision=precision)
    _log(f"autotune: node lists {lists}, z_per_thread {nzt}, tiles " +
         str(sorted({(d['nx'], d['tile_x']) for d in tuned})))
    out = {}
    for label, lset, z, nl in (("autotuned", tuned, nzt, lists), ("default_tiles", lats, 0, 0)):
        gs = LatticeSet(lset, precision=precision, z_per_thread=z, graph_steps=8, probe_ring=64, node_lists=nl)
        for k, pk in enumerate(parts):
            gs.particles_set(k, pk["x"], pk["radius"], fixed=pk["fixed"])
        nfl = sum(int((gs.owner(k) < 0).sum()) for k in range(len(lset)))
        dt = time_steps(gs, steps, warmup)
        kt = kernel_times(gs, kernel_steps)
        status = gs.status()
        gs.close()
        torch.cuda.empty_cache()
        alg = 2 * 19 * BYTES_PER_VALUE[precision] * nfl
        out[label] = {"ms_per_step": 1e3 * dt / steps, "mlups": nfl * steps / dt / 1e6, "fluid_nodes": nfl,
                      "kernel_ms": {"refresh": kt[4], "fluid": kt[2], "links": kt[0], "motion": kt[1], "remap": kt[3]},
                      "fluid_roofline_frac": alg / (kt[2] * 1e-3) / 1e9 / HBM_PEAK_GBS, "status": status}
        _log(f"{label}: {out[label]}")
    cells = sum(d["nx"] * d["ny"] * d["nz"] for d in lats)
    line = {"metric": "batched ensemble, fluid-node MLUPS", "value": out["autotuned"]["mlups"],
            "unit": "MLUPS (fluid-node updates/s, millions)", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": out["autotuned"]["ms_per_step"], "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{n_members} uneven FCC samples (seeds 1000..{999 + n_members}), one launch "
                                   "per kernel per step", "cells": cells, "precision": precision,
                       "node_lists": lists, "z_per_thread": nzt, "tile_x_by_nx": {str(k): v for k, v in sorted(
                           {d["nx"]: d["tile_x"] for d in tuned}.items())}},
            "results": out, "autotune_report": report}
    if emit:
        print(json.dumps(line), flush=True)
    return line


def adjoint_bench(nsteps=2000, ckpt=100, emit=True):
    """The adjoint workload: 64x64x256 lattice, frozen touching FCC packing of 275 spheres of
    radius 8 (walls in x and y, density faces in z), a 2000-step window with checkpoints
    every 100 steps.  Loss: L2 misfit of the probe signals against a twin target made by
    the FP64 window at (tau + 0.01, 1.1 A); gradients w.r.t. tau, A and the velocities of
    the first 256 spheres, FP32 and FP64 windows, checked against central differences of
    the FP64 forward (relative step 1e-4 for tau and A, 1e-6 lu/step for a velocity)."""
    import torch
    from paper_1808_08921_amd import inputs
    from paper_1808_08921_amd.lbdem import AdjointWindow, LatticeSet

    params, pk = inputs.adjoint_fcc_case()
    params = dict(params, max_particles=len(pk["x"]))
    n = len(pk["x"])
    tau0, amp0 = params["tau"], params["amp"]
    v0 = np.zeros((n, 3))
    out = {}
    wins = {}
    for prec in ("fp64", "fp32"):
        gs = LatticeSet([params], precision=prec, graph_steps=0, probe_ring=64)
        gs.particles_set(0, pk["x"], pk["radius"], fixed=pk["fixed"])
        win = AdjointWindow(gs, 0, nsteps=nsteps, ckpt_every=ckpt)
        wins[prec] = (gs, win)
    win64 = wins["fp64"][1]
    target = win64.forward(tau0 + 0.01, 1.1 * amp0, v0)

    def loss(win, tau=tau0, amp=amp0, v=v0):
        P = win.forward(tau, amp, v)
        return float(((P - target) ** 2).sum()), P

    for prec in ("fp64", "fp32"):
        win = wins[prec][1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, P = loss(win)
        t1 = time.perf_counter()
        gt, ga, gv = win.backward(2.0 * (P - target))
        t2 = time.perf_counter()
        out[prec] = {"loss": L, "forward_s": t1 - t0, "backward_s": t2 - t1, "dL_dtau": gt, "dL_damp": ga,
                     "dL_dv_first256_norm": float(np.linalg.norm(gv[:256])), "gv": gv}
        _log(f"adjoint {prec}: L={L:.6e} fwd {t1 - t0:.2f}s bwd {t2 - t1:.2f}s dtau {gt:.6e} damp {ga:.6e}")
    # central differences on the FP64 forward
    h = 1e-4
    fd = {"dL_dtau": (loss(win64, tau=tau0 * (1 + h))[0] - loss(win64, tau=tau0 * (1 - h))[0]) / (2 * h * tau0),
          "dL_damp": (loss(win64, amp=amp0 * (1 + h))[0] - loss(win64, amp=amp0 * (1 - h))[0]) / (2 * h * amp0)}
    g64 = out["fp64"]["gv"]
    comps = [tuple(int(c) for c in np.unravel_index(np.argmax(np.abs(g64[:256])), (256, 3)))]
    hv = 1e-6  # velocities enter the collision's u^2 terms: a step far below the flow speed
    for (q, a) in comps:
        vp, vm = v0.copy(), v0.copy()
        vp[q, a] += hv
        vm[q, a] -= hv
        fd[f"dL_dv[{q},{a}]"] = (loss(win64, v=vp)[0] - loss(win64, v=vm)[0]) / (2 * hv)
    checks = {}
    for prec in ("fp64", "fp32"):
        r = out[prec]
        checks[prec] = {"dL_dtau_rel_err_vs_fd": abs(r["dL_dtau"] - fd["dL_dtau"]) / abs(fd["dL_dtau"]),
                        "dL_damp_rel_err_vs_fd": abs(r["dL_damp"] - fd["dL_damp"]) / abs(fd["dL_damp"])}
        for (q, a) in comps:
            key = f"dL_dv[{q},{a}]"
            checks[prec][key + "_rel_err_vs_fd"] = abs(r["gv"][q, a] - fd[key]) / abs(fd[key])
    checks["fp32_vs_fp64_dL_dv_rel"] = float(np.linalg.norm(out["fp32"]["gv"][:256] - g64[:256]) / np.linalg.norm(g64[:256]))
    for prec in out:
        out[prec].pop("gv")
    for gs, win in wins.values():
        win.close()
        gs.close()
    torch.cuda.empty_cache()
    line = {"metric": "adjoint window: forward + backward seconds, gradient errors vs central differences",
            "config": {"workload": f"64x64x256 frozen FCC, {n} spheres R=8, {nsteps} steps, checkpoint every {ckpt}",
                       "loss": "L2 probe misfit vs twin target (tau+0.01, 1.1 A)"},
            "results": out, "finite_differences_fp64": fd, "checks": checks}
    if emit:
        print(json.dumps(line), flush=True)
    return line


def sweep_bench(steps, warmup, kernel_steps, precision="fp32"):
    """The source sweep of Table tab:source as a batched ensemble: the FCC wave case
    (96 x 96 x 384, 1024 spheres) driven by each of the six sources (single-period step,
    cosine and sine at 6.50 MHz; cosine at 1.30, 3.25 and 13.0 MHz; rho' = 2e-4), advanced
    together, one launch per kernel per step.  Reports the ensemble's fluid-node MLUPS and
    each member's P-wave arrival speed from its momentum probes."""
    import torch
    from paper_1808_08921_amd import inputs
    from paper_1808_08921_amd.lbdem import LatticeSet

    members = inputs.source_sweep_fcc()
    rows = inputs.source_table_rows()
    lats = [dict(p, max_particles=len(pk["x"])) for p, pk in members]
    gs = LatticeSet(lats, precision=precision, graph_steps=8, probe_ring=4096)
    for k, (_, pk) in enumerate(members):
        gs.particles_set(k, pk["x"], pk["radius"], fixed=pk["fixed"])
    nfl = sum(int((gs.owner(k) < 0).sum()) for k in range(len(lats)))
    dt = time_steps(gs, steps, warmup)
    tmax = min(steps + warmup, 1200)
    speeds = []
    for k, r in enumerate(rows):
        pr = gs.probes(k, 0, tmax)
        zs = lats[k]["probe_z"]
        # planes beyond the inlet that the pulse reaches within the record; a step source
        # has no momentum peak, its front is timed where rho' first reaches half its peak
        if r["wave"] == inputs.WAVE_STEP:
            c = front_velocity(pr[:, 2:12, :], zs[2:12], tmax)
        else:
            c, _ = arrival_velocity(pr[:, 2:12, :], zs[2:12], tmax)
        speeds.append({"f_mhz": r["f_mhz"], "wave": {1: "sine", 2: "cosine", 3: "step"}[r["wave"]],
                       "p_wave_velocity": c})
    kt = kernel_times(gs, kernel_steps)
    status = gs.status()
    gs.close()
    torch.cuda.empty_cache()
    cells = sum(d["nx"] * d["ny"] * d["nz"] for d in lats)
    alg = 2 * 19 * BYTES_PER_VALUE[precision] * nfl
    line = {"metric": "source sweep ensemble (Table tab:source), fluid-node MLUPS", "value": nfl * steps / dt / 1e6,
            "unit": "MLUPS (fluid-node updates/s, millions)", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * dt / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp32": "f32", "fp64": "f64"}.get(precision, precision), "data": "synthetic",
            "config": {"workload": "six FCC wave cases (4x4x16 cells, 96x96x384, 1024 spheres) driven by the six "
                                   "sources of Table tab:source, one launch per kernel per step",
                       "cells": cells, "fluid_nodes": nfl, "status": status,
                       "kernel_ms": {"refresh": kt[4], "fluid": kt[2], "links": kt[0], "motion": kt[1], "remap": kt[3]},
                       "fluid_roofline_frac": alg / (kt[2] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "p_wave_velocity_by_source": speeds}}
    print(json.dumps(line), flush=True)


def drag_force(v_rel, radius, tau, rho_f=1.0):
    """Eq. (termVel): drag of a sphere at relative speed v_rel, with C_d = 24/Re + 3.6/Re^0.313,
    Re = 2 v_rel R / nu and nu = (tau - 1/2) / 3."""
    nu = (tau - 0.5) / 3.0
    re = 2.0 * v_rel * radius / nu
    cd = 24.0 / re + 3.6 / re ** 0.313
    return 0.5 * cd * math.pi * radius ** 2 * rho_f * v_rel ** 2


def settling_bench(steps=40000, taus=(0.6, 0.8, 1.0, 1.4, 1.8, 2.0), precision="fp32", every=100,
                   kernel_steps=200, emit=True):
    """The settling sweep of Sec. 3.1 at the paper's size: a 160^3 fully periodic cube, one
    sphere of radius 5.005 released at rest at the centre under F_g = 0.1 (net of buoyancy),
    tau from 0.6 to 2.0.  The terminal speed is the relative speed |V_p - u_bar| averaged
    over the second half of the run (sampled every `every` steps: the sphere's speed
    ripples as it crosses lattice planes), with u_bar, the fluid velocity averaged over the
    lattice, from the momentum balance of the periodic box (F_g t = m_p V_p + rho_f N u_bar)
    and checked against the populations at the end; its drag by Eq. (termVel) is compared
    with F_g.  The all-fluid 4.1 M-cell lattice is also a second roofline case of the fluid
    kernel."""
    import torch
    from paper_1808_08921_amd import inputs
    from paper_1808_08921_amd.lbdem import LatticeSet

    # lattice vectors in the order of Eq. (3d19q), the order of the populations the library returns
    c = np.array([[1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0],
                  [0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0],
                  [0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0]], dtype=np.float64)
    rows = []
    roof = None
    for tau in taus:
        params, pk = inputs.settling_periodic_case(tau)
        radius = float(pk["radius"][0])
        m_p = params["rho_p"] * 4.0 / 3.0 * math.pi * radius ** 3
        fg = float(pk["fg"][0, 2])
        gs = LatticeSet([params], precision=precision, graph_steps=8, probe_ring=16)
        gs.particles_set(0, pk["x"], pk["radius"], fg=pk["fg"], fixed=pk["fixed"])
        nfl = int((gs.owner(0) < 0).sum())
        t0 = time.perf_counter()
        samples = []
        for _ in range(steps // every):
            gs.step(every)
            v = gs.particles_get(0)["v"][0]
            u_bar = -m_p * v / (params["rho_f"] * nfl)
            u_bar[2] += fg * gs.t / (params["rho_f"] * nfl)
            samples.append((gs.t, float(np.linalg.norm(v - u_bar)), float(v[2]), float(u_bar[2])))
        wall = time.perf_counter() - t0
        f = gs.populations(0)
        fluid = gs.owner(0) < 0
        u_pop = (c @ f[:, fluid]).sum(1) / f[:, fluid].sum()
        if tau == 1.0:
            kt = kernel_times(gs, kernel_steps)
            alg = 2 * 19 * BYTES_PER_VALUE[precision] * nfl
            roof = {"fluid_kernel_ms": kt[2], "fluid_nodes": nfl,
                    "achieved_GBs": alg / (kt[2] * 1e-3) / 1e9, "frac": alg / (kt[2] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "kernel_ms": {"refresh": kt[4], "fluid": kt[2], "links": kt[0], "motion": kt[1], "remap": kt[3]}}
        status = gs.status()
        gs.close()
        del f
        torch.cuda.empty_cache()
        vr = np.array([x[1] for x in samples[len(samples) // 2:]])
        v_t = float(vr.mean())
        fd = drag_force(v_t, radius, tau)
        q = len(samples) // 4
        rows.append({"tau": tau, "v_t": v_t, "v_t_ripple": float(vr.std() / v_t),
                     "v_t_quarters": [float(np.mean([x[1] for x in samples[k * q:(k + 1) * q]])) for k in range(4)],
                     "re": 2 * v_t * radius / ((tau - 0.5) / 3.0), "drag_eq_termVel": fd,
                     "rel_err_vs_Fg": (fd - fg) / fg, "u_bar_end_balance": samples[-1][3],
                     "u_bar_end_populations": float(u_pop[2]), "status": status, "wall_s": wall})
        _log(f"settling tau {tau}: V_t {v_t:.5e} drag {fd:.5f} err {(fd - fg) / fg:+.4f} "
             f"u_bar {samples[-1][3]:.4e} / {u_pop[2]:.4e} ({wall:.1f} s)")
    line = {"metric": "settling sweep (Sec. 3.1): drag error of Eq. (termVel) vs F_g", "value": None,
            "unit": "relative error", "n_gpus": 1, "steps": steps, "warmup": 0, "higher_is_better": False,
            "dtype": {"fp32": "f32", "fp64": "f64"}.get(precision, precision), "data": "synthetic",
            "config": {"workload": "160^3 fully periodic cube, one sphere R = 5.005, F_g = 0.1, tau 0.6..2.0",
                       "precision": precision},
            "results": rows, "fluid_roofline_160cube": roof}
    if emit:
        print(json.dumps(line), flush=True)
    return line


def pure_fluid_bench(steps=2000, warmup=200, kernel_steps=200):
    """The pure-fluid roofline reference: the FCC case's lattice (96 x 96 x 384) fully periodic
    without particles, started from f = w_d (1 + 1e-3 sin(2 pi z / 384)) (a small acoustic
    wave), in every storage precision; the fluid kernel runs on dense tiles (the automatic
    mapping without particles).  Also the bandwidth of a plain 1 GiB device copy, the
    achievable figure beside the 8 TB/s peak."""
    import torch
    from paper_1808_08921_amd.lbdem import LatticeSet

    nx, ny, nz = 96, 96, 384
    w = np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3])      # order of Eq. (3d19q): rest last
    prof = 1.0 + 1e-3 * np.sin(2.0 * math.pi * np.arange(nz) / nz)
    f = w[:, None, None, None] * prof[None, :, None, None] * np.ones((1, 1, ny, nx))
    out = {}
    for prec in ("fp32", "fp16", "bf16", "fp64"):
        params = dict(nx=nx, ny=ny, nz=nz, tau=1.0, bc=(0,) * 6, probe_z=tuple(range(0, nz, 16)), max_particles=0)
        gs = LatticeSet([params], precision=prec, graph_steps=8, probe_ring=64)
        gs.set_populations(0, f)
        dt = time_steps(gs, steps, warmup)
        kt = kernel_times(gs, kernel_steps)
        status = gs.status()
        gs.close()
        torch.cuda.empty_cache()
        alg = 2 * 19 * BYTES_PER_VALUE[prec] * nx * ny * nz
        out[prec] = {"ms_per_step": 1e3 * dt / steps, "fluid_kernel_ms": float(kt[2]),
                     "achieved_GBs": alg / (kt[2] * 1e-3) / 1e9, "frac": alg / (kt[2] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": alg, "status": status}
        _log(f"pure fluid {prec}: {out[prec]}")
    # achievable copy bandwidth: 1 GiB read and 1 GiB written per copy
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 20 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"workload": "96x96x384 fully periodic pure fluid, small sine wave in z, dense tiles",
            "steps": steps, "by_precision": out, "device_copy_GBs": copy_gbs,
            "device_copy_frac_of_peak": copy_gbs / HBM_PEAK_GBS}


def dispersion_bench(calls=50, warmup=5):
    """The dispersion-analysis workload (Sec. 3.2): a probe record of 20000 steps x 24 planes
    (the FCC wave case's probes every 16 lu) through the space-time DFT on a 1024 x 1024
    (omega, kappa) grid with its ridge, and the Eq. (1Dwave) fit at the inserted frequency.
    The record is a seeded synthetic damped wave with noise (inputs.probe_signal)."""
    import torch
    from paper_1808_08921_amd import inputs, lbdem

    nt, nz, nw, nk = 20000, 24, 1024, 1024
    zpos = 16.0 * np.arange(nz)
    om = 2 * math.pi / 200
    x = inputs.probe_signal(nt, zpos, om, -0.6 - 0.1j, 6e-3, om / 0.7, offset=1e-3, harmonic=0.1, noise=0.02, seed=3)
    w0, dw = 0.0, 0.2 / nw
    k0, dk = -math.pi / 16, (2 * math.pi / 16) / nk
    xd = torch.from_numpy(x).cuda()
    nb = ctypes.c_size_t()
    L = lbdem.lib()
    lbdem._check(L.lbdem_dft_workspace_size(nt, nz, nw, nk, ctypes.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        F, r = lbdem.st_dft(xd, zpos, 0.0, w0, dw, nw, k0, dk, nk, work=work)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(calls):
        F, r = lbdem.st_dft(xd, zpos, 0.0, w0, dw, nw, k0, dk, nk, work=work)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    fit = lbdem.wave_fit(xd, zpos, 0.0, om)
    e0.record()
    for _ in range(calls):
        lbdem.wave_fit(xd, zpos, 0.0, om)
    e1.record()
    torch.cuda.synchronize()
    ms_fit = e0.elapsed_time(e1) / calls
    # algorithmic flops: time stage 2 FMAs per (omega, t, z), space stage 4 FMAs per (omega, z, kappa)
    flops = 4.0 * nw * nt * nz + 8.0 * nw * nz * nk
    achieved = flops / (ms * 1e-3) / 1e12
    kidx = int(r.cpu()[int(round(om / dw))])
    out = {"metric": "space-time DFT of a probe record (Sec. 3.2)", "value": flops / (ms * 1e-3) / 1e9,
           "unit": "GFLOP/s (algorithmic, FP64)", "n_gpus": 1, "steps": calls, "warmup": warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"probe record {nt} steps x {nz} planes, spectrum {nw} x {nk}, ridge; "
                                  "Eq. (1Dwave) fit at omega = 2 pi / 200",
                      "fit_ms": ms_fit, "fit": {"alpha": fit["alpha"], "c": fit["c"], "A": [fit["A"].real, fit["A"].imag]},
                      "ridge_speed_at_omega": (round(om / dw) * dw) / (k0 + kidx * dk)},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6,
                        "traffic": None, "kernel": "st_dft (time stage, chunk sums, phase table, space stage, ridge)",
                        "algorithmic_flops_per_call": flops}}
    try:
        from threadpoolctl import threadpool_limits

        import oracle.analysis as an

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            an.space_time_dft(x, 0.0, zpos, w0 + np.arange(nw) * dw, k0 + np.arange(nk) * dk)
            dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": flops / dt / 1e9, "unit": "GFLOP/s (algorithmic, FP64)", "cores": 1,
                               "kind": "oracle", "sample": "the full workload, one call, one host thread"}
    except Exception as exc:  # the baseline is a reported figure only
        out["cpu_baseline"] = {"error": str(exc)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--kernel-steps", type=int, default=200, help="eager steps timed per kernel with HIP events")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip FP16/BF16 timing and the error study")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the ensemble, adjoint-window and settling-sweep summaries of the main line")
    ap.add_argument("--counters", type=int, default=0, metavar="STEPS",
                    help="only run the workload of the rocprofv3 counter passes (STEPS eager steps + a copy)")
    ap.add_argument("--counters-precision", choices=("fp32", "fp16", "bf16"), default="fp32",
                    help="storage precision of the counter workload and of its summary's file")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write the counter summary from two rocprofv3 --pmc CSV files")
    ap.add_argument("--ensemble", type=int, default=0, metavar="N",
                    help="run the batched-ensemble workload with N lattices instead of the main line")
    ap.add_argument("--settling", type=int, default=0, metavar="STEPS",
                    help="run the 160^3 periodic settling sweep over tau with STEPS steps per tau instead")
    ap.add_argument("--taus", type=float, nargs="+", default=[0.6, 0.8, 1.0, 1.4, 1.8, 2.0],
                    help="relaxation times of the settling sweep")
    ap.add_argument("--sweep", action="store_true",
                    help="run the Table tab:source sweep (six FCC cases, one per source) as a batched ensemble")
    ap.add_argument("--dispersion", action="store_true",
                    help="run the dispersion-analysis workload (space-time DFT of a probe record) instead")
    ap.add_argument("--adjoint", action="store_true", help="run the adjoint-window workload instead of the main line")
    ap.add_argument("--cpu-worker", type=float, default=0.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker)
        return
    if args.dispersion:
        dispersion_bench()
        return
    if args.settling:
        settling_bench(steps=args.settling, taus=tuple(args.taus))
        return
    if args.sweep:
        sweep_bench(args.steps, args.warmup, args.kernel_steps)
        return
    if args.adjoint:
        adjoint_bench()
        return
    if args.ensemble:
        ensemble_bench(args.ensemble, args.steps, args.warmup, args.kernel_steps)
        return
    if args.summarize_counters:
        fetch_csv, write_csv, command = args.summarize_counters
        summarize_counters(fetch_csv, write_csv, counters_file(args.counters_precision), command,
                           args.counters_precision)
        return
    if args.counters:
        counters_workload(args.counters, args.counters_precision)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a slab decomposition over several "
              "GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    params, pk = _case(seed=0)
    results = {}
    kt = None
    nfl = None
    for prec in (("fp32",) if args.no_variants else ("fp32", "fp16", "bf16")):
        gs = _make(params, pk, prec)
        if nfl is None:
            nfl = _fluid_nodes(gs)
        dt = time_steps(gs, args.steps, args.warmup)
        k = kernel_times(gs, args.kernel_steps)
        status = gs.status()
        gs.close()
        torch.cuda.empty_cache()
        results[prec] = {"ms_per_step": 1e3 * dt / args.steps, "mlups": nfl * args.steps / dt / 1e6,
                         "kernel_ms": [float(x) for x in k], "status": status}
        _log(f"{prec}: {results[prec]}")
        if prec == "fp32":
            kt = k
    ncell = params["nx"] * params["ny"] * params["nz"]
    r32 = results["fp32"]
    alg_bytes = 2 * 19 * BYTES_PER_VALUE["fp32"] * nfl
    achieved = alg_bytes / (kt[2] * 1e-3) / 1e9
    line = {
        "metric": "coupled D3Q19 MLUPS + % HBM roofline; FP16-stored vs FP32 at stated error",
        "value": r32["mlups"],
        "unit": "MLUPS (fluid-node updates/s, millions)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FCC wave propagation, 4x4x16 FCC cells, 1024 spheres, 96x96x384 D3Q19, FP32 "
                               "populations, cosine inlet 1e-3 / 200 steps, probes every 16 lu",
                   "cells": ncell, "fluid_nodes": nfl, "solid_fraction": 1 - nfl / ncell,
                   "fluid_mapping": "per-plane node lists, compact population storage",
                   "mlups_all_cells": ncell * args.steps / (r32["ms_per_step"] * 1e-3 * args.steps) / 1e6,
                   "kernel_ms": {"refresh": kt[4], "fluid": kt[2], "links": kt[0], "motion": kt[1], "remap": kt[3]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_fluid<FP32, compact>", "algorithmic_bytes_per_launch": alg_bytes,
                     "step_frac": alg_bytes / (r32["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_variants:
        line["variants"] = {}
        for prec in ("fp16", "bf16"):
            r = results[prec]
            ab = 2 * 19 * BYTES_PER_VALUE[prec] * nfl
            line["variants"][prec] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"],
                                      "speedup_vs_fp32": r32["ms_per_step"] / r["ms_per_step"],
                                      "fluid_kernel_ms": r["kernel_ms"][2],
                                      "fluid_kernel_speedup_vs_fp32": kt[2] / r["kernel_ms"][2],
                                      "roofline_frac": ab / (r["kernel_ms"][2] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        _log("error study against the FP64 path")
        line["errors_vs_fp64"] = precision_errors(params, pk)
    if not args.no_extra:
        # the batched ensemble and the adjoint window, summarised beside the main line
        _log("64-lattice ensemble")
        ens = ensemble_bench(64, 400, 50, 100, emit=False)
        _log("adjoint window")
        adj = adjoint_bench(emit=False)
        _log("pure fluid reference")
        pf = pure_fluid_bench()
        _log("settling sweep")
        st = settling_bench(emit=False)
        line["other_workloads"] = {
            "ensemble_64": {"workload": ens["config"]["workload"], "cells": ens["config"]["cells"],
                            "mlups": ens["value"], "ms_per_step": ens["ms_per_step"],
                            "results": ens["results"]},
            "adjoint_window": {"workload": adj["config"]["workload"], "results": adj["results"],
                               "checks": adj["checks"]},
            "pure_fluid_reference": pf,
            "settling_sweep": {"workload": st["config"]["workload"], "steps_per_tau": st["steps"],
                               "drag_rel_err_vs_Fg": {str(r["tau"]): r["rel_err_vs_Fg"] for r in st["results"]},
                               "v_t": {str(r["tau"]): r["v_t"] for r in st["results"]},
                               "fluid_roofline_160cube": st["fluid_roofline_160cube"]}}
    if not args.no_cpu:
        _log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(params, pk)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
