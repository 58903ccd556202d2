"""Tile autotuner for batched ensembles of uneven lattices.

The fluid kernel maps a 256-thread workgroup to a tile of tile_x * (256 / tile_x) nodes
of one lattice, nzt planes deep.  Which tile is fastest depends on the lattice's x extent
(partial tiles waste lanes) and on its solid fraction.  The tuner times the fluid kernel
with HIP events for every candidate on one representative lattice per distinct shape
(its particles included), keeps the fastest tile_x per shape, then picks the planes per
thread for the whole set.  Everything it times runs through the library's kernels.
"""
from __future__ import annotations

import numpy as np

from .lbdem import LatticeSet

TILE_X = (8, 16, 32, 64)
Z_PER_THREAD = (1, 2, 4)


def _time_fluid(lattices, particles, precision, tile_x=0, nzt=0, steps=20, warmup=5, node_lists=0):
    """Average fluid-kernel milliseconds of one set (HIP events, eager steps)."""
    import torch

    gs = LatticeSet(lattices, precision=precision, tile_x=tile_x, z_per_thread=nzt, graph_steps=0, probe_ring=64,
                    node_lists=node_lists)
    try:
        for k, pk in enumerate(particles):
            if pk is not None:
                gs.particles_set(k, pk["x"], pk["radius"], fixed=pk.get("fixed"), fg=pk.get("fg"))
        gs.step(warmup)
        gs.timing_enable(True)
        gs.step(steps)
        ms, cnt = gs.timing_read()
        return float(ms[2] / max(cnt[2], 1))
    finally:
        gs.close()
        torch.cuda.empty_cache()


def autotune(lattices, particles, precision="fp32", tile_x=TILE_X, z_per_thread=Z_PER_THREAD, steps=20):
    """Choose the fluid-kernel mapping of a set: dense tiles (a tile width per lattice shape
    and the planes per thread of the set), per-plane node lists, or node lists with compact
    storage, whichever is fastest.

    lattices: parameter dicts (as for LatticeSet); particles: matching list of particle
    dicts (x, radius, fixed) or None.  Returns (tuned lattices with a ``tile_x`` key,
    z_per_thread, node_lists, report) where report lists every timing taken.
    """
    shapes = {}
    for k, d in enumerate(lattices):
        shapes.setdefault((d["nx"], d["ny"], d["nz"]), k)
    report = []
    best_tx = {}
    for shape, k in sorted(shapes.items()):
        cands = [tx for tx in tile_x if tx <= max(8, 1 << int(np.ceil(np.log2(shape[0]))))]
        times = {}
        for tx in cands:
            times[tx] = _time_fluid([lattices[k]], [particles[k]], precision, tile_x=tx, nzt=2, steps=steps)
            report.append({"shape": shape, "tile_x": tx, "z_per_thread": 2, "fluid_ms": times[tx]})
        best_tx[shape] = min(times, key=times.get)
    tuned = [dict(d, tile_x=best_tx[(d["nx"], d["ny"], d["nz"])]) for d in lattices]
    # planes per thread, on a sample of the set (one lattice per shape)
    ks = sorted(shapes.values())
    sample = [tuned[k] for k in ks]
    sample_p = [particles[k] for k in ks]
    zt = {}
    for nzt in z_per_thread:
        zt[nzt] = _time_fluid(sample, sample_p, precision, nzt=nzt, steps=steps)
        report.append({"shape": "sample", "tile_x": "tuned", "z_per_thread": nzt, "fluid_ms": zt[nzt]})
    best_nzt = min(zt, key=zt.get)
    modes = {0: zt[best_nzt]}
    for nl in (1, 2):
        modes[nl] = _time_fluid(sample, sample_p, precision, steps=steps, node_lists=nl)
        report.append({"shape": "sample", "node_lists": nl, "fluid_ms": modes[nl]})
    return tuned, best_nzt, min(modes, key=modes.get), report
