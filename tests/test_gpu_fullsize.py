"""Parity at the benchmark's full size and launch configuration, and the settling-sphere
workload over a long window.

The FCC wave case is run at 96 x 96 x 384 (1024 spheres) exactly as bench.py launches it
(HIP graphs of 8 steps, automatic tiles) for a few steps, which the oracle can afford:
FP64 to the 1e-10 bar with bit-exact node maps; FP32 against the same FP64 oracle state.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1808_08921_amd import inputs

pytestmark = pytest.mark.gpu


def _oracle(params, pk):
    p = params
    s = oracle.Sim(p["nx"], p["ny"], p["nz"], tau=p["tau"], rho_f=p["rho_f"], bc=p["bc"], wave=p["wave"],
                   amp=p["amp"], omega=p["omega"], t_n=p["t_n"], E=p["E"], nu=p["nu"], mu=p["mu"], rho_p=p["rho_p"],
                   probe_z=p["probe_z"])
    s.set_particles(pk["x"], pk["radius"], v=pk.get("v"), w=pk.get("w"), fg=pk.get("fg"), fixed=pk.get("fixed"))
    return s


@pytest.fixture(scope="module")
def fcc_oracle():
    params, pk = inputs.wave_fcc_case(seed=0)
    params["max_particles"] = len(pk["x"])
    s = _oracle(params, pk)
    s.step(8)
    yield params, pk, s
    s.close()


@pytest.mark.parametrize("seed", [1, 2])
def test_full_size_fcc_other_seeds_fp64(seed):
    """The full-size FCC case with the packings of seeds 1 and 2 (other overlap jitter), FP64,
    8 steps as the benchmark launches them: node maps bit-exact, populations 1e-10,
    particles within the force-rounding floor of the seed-0 test."""
    from paper_1808_08921_amd.lbdem import LatticeSet

    params, pk = inputs.wave_fcc_case(seed=seed)
    params["max_particles"] = len(pk["x"])
    s = _oracle(params, pk)
    s.step(8)
    with LatticeSet([params], precision="fp64", graph_steps=8, probe_ring=64) as gs:
        gs.particles_set(0, pk["x"], pk["radius"], fixed=pk["fixed"])
        gs.step(8)
        assert np.array_equal(gs.owner(0), s.owner())
        fl = s.owner() < 0
        assert np.abs(gs.populations(0)[:, fl] - s.populations()[:, fl]).max() <= 1e-10
        g, o = gs.particles_get(0), s.particles()
        assert np.abs(g["x"] - o["x"]).max() <= 1e-10 * 384
        m_min = params["rho_p"] * 4.0 / 3.0 * np.pi * float(np.min(pk["radius"])) ** 3
        floor = np.abs(o["force"]).max() * 2.0 ** -52 * math.sqrt(4.8e3) * 8 / m_min
        assert np.abs(g["v"] - o["v"]).max() <= 1e-10 * np.abs(o["v"]).max() + floor
        assert gs.status() == 0
    s.close()


# FP32: populations up to 1/3 are stored with a unit in the last place of 2^-25 = 3.0e-8;
# the bound allows four of them after 8 steps of FP32 arithmetic
@pytest.mark.parametrize("precision,tol_f,tol_probe,tol_v", [("fp64", 1e-10, 1e-10, 1e-10),
                                                             ("fp32", 4 * 2.0 ** -25, 1e-4, 1e-4)])
def test_full_size_fcc_bench_configuration(fcc_oracle, precision, tol_f, tol_probe, tol_v):
    from paper_1808_08921_amd.lbdem import LatticeSet

    params, pk, s = fcc_oracle
    with LatticeSet([params], precision=precision, graph_steps=8, probe_ring=4096) as gs:
        gs.particles_set(0, pk["x"], pk["radius"], fixed=pk["fixed"])
        gs.step(8)
        own_g, own_o = gs.owner(0), s.owner()
        diff = own_g != own_o
        if precision == "fp64":
            assert not diff.any(), f"{int(diff.sum())} nodes differ"
        else:
            # FP32 particle forces differ from FP64 at ~1e-7 relative, so a node within
            # that distance of a surface may change owner a step apart: count them
            assert int(diff.sum()) <= 16, f"{int(diff.sum())} nodes differ"
        near = diff.copy()
        for ax in range(3):
            near |= np.roll(diff, 1, axis=ax) | np.roll(diff, -1, axis=ax)
        fl = (own_o < 0) & (own_g < 0) & ~near
        df = np.abs(gs.populations(0)[:, fl] - s.populations()[:, fl]).max()
        assert df <= tol_f, f"populations differ by {df:.3e}"
        pg, po = gs.probes(0, 0, 8), s.probes(0, 8)
        if precision == "fp64":
            assert np.array_equal(pg[..., 0], po[..., 0])       # fluid-node counts per plane
        # plane averages of rho - rho_f; the oracle forms rho - rho_f from the full
        # populations, so its values carry an absolute rounding floor of ~1e-16
        rg, ro = pg[..., 1] / pg[..., 0], po[..., 1] / po[..., 0]
        assert np.abs(rg - ro).max() <= tol_probe * np.abs(ro).max() + 1e-15
        g, o = gs.particles_get(0), s.particles()
        assert np.abs(g["x"] - o["x"]).max() <= 1e-10 * 384
        # the hydrodynamic force is a sum over ~4.8k links whose partial sums reach |F|
        # (up to ~40 on spheres whose surface a neighbour's lens cuts); two summation
        # orders of it differ by ~|F| 2^-52 sqrt(4.8k) per step in FP64 (4.8k x 4e-9 ~ 2e-5
        # with FP32 populations), which bounds how well two codes can agree on velocities
        # this early (|v| ~ 1e-6): 8 steps of that over the lightest sphere's mass
        m_min = params["rho_p"] * 4.0 / 3.0 * np.pi * float(np.min(pk["radius"])) ** 3
        f_step = np.abs(o["force"]).max() * 2.0 ** -52 * math.sqrt(4.8e3) if precision == "fp64" else 2e-5
        floor = f_step * 8 / m_min
        assert np.abs(g["v"] - o["v"]).max() <= tol_v * np.abs(o["v"]).max() + floor
        assert gs.status() == 0


def _brenner(h, radius, nmax=60):
    """Drag of a sphere of this radius moving normal to a plane wall at centre distance h,
    relative to Stokes drag (Brenner's exact series, 1961)."""
    a = math.acosh(h / radius)
    tot = 0.0
    for n in range(1, nmax):
        num = 2.0 * math.sinh((2 * n + 1) * a) + (2 * n + 1) * math.sinh(2.0 * a)
        den = 4.0 * math.sinh((n + 0.5) * a) ** 2 - (2 * n + 1) ** 2 * math.sinh(a) ** 2
        tot += n * (n + 1) / ((2 * n - 1) * (2 * n + 3)) * (num / den - 1.0)
    return 4.0 / 3.0 * math.sinh(a) * tot


def test_settling_sphere_near_top_wall_1000_steps_fp64():
    """The settling-sphere workload: 32^3 box with half-way walls, a sphere of radius 6 at the top
    centre (centre 2 lu below the top wall's gap, (15.5, 15.5, 23.5)), density ratio 2,
    g = 1e-5, tau = 0.8, 1000 FP64 steps: trajectory parity with the oracle every 100
    steps, node maps exact; then the settling speed against Stokes drag with the walls'
    correction.  The top wall is 8 lu from the centre (h / R = 1.33) and dominates:
    Brenner's exact drag factor for a sphere moving normal to a plane wall is 4.0 - 4.3
    there, the side walls alone (Haberman-Sayre, the duct bracketed by cylinders of radius
    16 and 32 / sqrt(pi)) give 2.7 - 3.2.  The measured factor must be at least the nearer
    wall's alone and at most the sum of the two excess drags."""
    from paper_1808_08921_amd.lbdem import LatticeSet

    params, pk = inputs.settling_case()
    params["max_particles"] = 1
    assert tuple(pk["x"][0]) == (15.5, 15.5, 23.5)
    s = _oracle(params, pk)
    with LatticeSet([params], precision="fp64", graph_steps=8) as gs:
        gs.particles_set(0, pk["x"], pk["radius"], fg=pk["fg"], fixed=pk["fixed"])
        for _ in range(10):
            gs.step(100)
            s.step(100)
            g, o = gs.particles_get(0), s.particles()
            assert np.abs(g["x"] - o["x"]).max() <= 1e-10 * 32
            assert np.abs(g["v"] - o["v"]).max() <= 1e-10 * np.abs(o["v"]).max()
            assert np.array_equal(gs.owner(0), s.owner())
        assert gs.t == 1000 and gs.status() == 0
    s.close()
    nu = (params["tau"] - 0.5) / 3.0
    radius = float(pk["radius"][0])
    v_stokes = -pk["fg"][0, 2] / (6.0 * math.pi * nu * radius)
    vz = g["v"][0, 2]
    assert vz < 0.0
    ratio = v_stokes / -vz
    top = params["nz"] - 0.5                      # half-way wall above the last node
    h_start, h_end = top - pk["x"][0, 2], top - g["x"][0, 2]
    assert _brenner(h_end, radius) <= ratio <= 3.2 + _brenner(h_start, radius) - 1.0, ratio


def test_full_size_fcc_moving_spheres_fp64():
    """The full 96 x 96 x 384 FCC case in FP64 with the mobile spheres given seeded
    velocities of up to 0.02 lu per step: 25 steps with nodes covered and uncovered every
    step and the compact node lists rebuilt as the spheres cross the list skin; node maps
    bit-exact and particles within 1e-10 of the oracle every 5 steps."""
    from paper_1808_08921_amd.lbdem import LatticeSet

    params, pk = inputs.wave_fcc_case(seed=0)
    params["max_particles"] = len(pk["x"])
    rng = np.random.default_rng(31)
    v = rng.uniform(-0.02, 0.02, (len(pk["x"]), 3))
    v[pk["fixed"] == 1] = 0.0
    s = _oracle(params, dict(pk, v=v))
    with LatticeSet([params], precision="fp64", graph_steps=8) as gs:
        gs.particles_set(0, pk["x"], pk["radius"], v=v, fixed=pk["fixed"])
        own0 = gs.owner(0)
        for _ in range(5):
            gs.step(5)
            s.step(5)
            own_g, own_o = gs.owner(0), s.owner()
            assert np.array_equal(own_g, own_o), f"{int((own_g != own_o).sum())} nodes differ"
            g, o = gs.particles_get(0), s.particles()
            assert np.abs(g["x"] - o["x"]).max() <= 1e-10 * 384
            assert np.abs(g["v"] - o["v"]).max() <= 1e-10 * np.abs(o["v"]).max()
            assert np.abs(g["force"] - o["force"]).max() <= 1e-10 * np.abs(o["force"]).max()
        assert int((own_g != own0).sum()) > 10000   # conversions all over the packing
        assert gs.status() & 0x1da == 0
    s.close()
