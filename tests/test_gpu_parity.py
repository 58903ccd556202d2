"""GPU parity: the HIP path (through the C interface) against the FP64 CPU oracle on the
same seeded inputs.

Bar (FP64 storage): node maps bit-exact; populations, probes, particle positions,
velocities, forces and torques within 1e-10 relative (or absolute where the quantity
is near zero).  FP32 / FP16 / BF16 storage: errors against the FP64 oracle are measured
and bounded loosely here; the stated values are recorded by the benchmark.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1808_08921_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu_set(params_list, precision="fp64", **kw):
    import torch

    from paper_1808_08921_amd.lbdem import LatticeSet

    assert torch.cuda.is_available()
    return LatticeSet(params_list, precision=precision, **kw)


def _oracle(params, pk=None):
    p = params
    s = oracle.Sim(p["nx"], p["ny"], p["nz"], tau=p["tau"], rho_f=p.get("rho_f", 1.0), bc=p["bc"],
                   wave=p.get("wave", 0), amp=p.get("amp", 0.0), omega=p.get("omega", 0.0), t_n=p.get("t_n", 0),
                   E=p.get("E", 10.0), nu=p.get("nu", 0.2), mu=p.get("mu", 0.0), rho_p=p.get("rho_p", 1.0),
                   probe_z=p.get("probe_z", ()))
    if pk is not None:
        s.set_particles(pk["x"], pk["radius"], v=pk.get("v"), w=pk.get("w"), fg=pk.get("fg"), fixed=pk.get("fixed"))
    return s


def _set_particles(gs, k, pk):
    gs.particles_set(k, pk["x"], pk["radius"], v=pk.get("v"), w=pk.get("w"), fg=pk.get("fg"), fixed=pk.get("fixed"))


def _rel(a, b, floor):
    return np.abs(a - b).max() / (np.abs(b).max() + floor)


def _compare_state(gs, k, s, pk=None, tol=TOL):
    own_g, own_o = gs.owner(k), s.owner()
    assert np.array_equal(own_g, own_o), f"node maps differ at {int((own_g != own_o).sum())} nodes"
    fl = own_o < 0
    fg, fo = gs.populations(k)[:, fl], s.populations()[:, fl]
    assert np.abs(fg - fo).max() <= tol, f"populations differ by {np.abs(fg - fo).max():.3e}"
    if pk is not None and s.np:
        g, o = gs.particles_get(k), s.particles()
        # Scales for the 1e-10 relative bar.  Net angular quantities come from sums that
        # cancel (zero by symmetry for a centred sphere), so they are measured against the
        # magnitude they would have without cancellation: |V|/R for Omega, |F| R for torque.
        rmax = float(np.max(pk["radius"]))
        box = float(max(gs.shapes[k]))
        vs = np.abs(o["v"]).max() + 1e-300
        fs = np.abs(o["force"]).max() + 1e-300
        scales = {"x": box, "v": vs, "w": max(np.abs(o["w"]).max(), vs / rmax),
                  "force": fs, "torque": max(np.abs(o["torque"]).max(), fs * rmax)}
        for key, sc in scales.items():
            err = np.abs(g[key] - o[key]).max()
            assert err <= tol * sc, f"{key}: {err:.3e} > {tol:.0e} x {sc:.3e}"


# ---------------------------------------------------------------------------
# fluid only
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,bc", [
    ((20, 18, 22), (0, 0, 0, 0, 0, 0)),
    ((33, 17, 9), (1, 1, 0, 0, 1, 1)),     # ragged tiles, walls on x and z
    ((12, 12, 40), (0, 0, 0, 0, 2, 2)),     # density faces on z
    ((7, 70, 13), (1, 1, 1, 1, 2, 2)),      # walls and density faces meet at edges
])
def test_fluid_parity_fp64(shape, bc):
    nx, ny, nz = shape
    params = dict(nx=nx, ny=ny, nz=nz, tau=0.83, bc=bc, wave=inputs.WAVE_COSINE, amp=1e-3,
                  omega=2 * math.pi / 30, t_n=30, probe_z=(0, nz // 2, nz - 1))
    f0 = inputs.random_populations(shape, amp=2e-3, seed=nx + ny + nz)
    s = _oracle(params)
    s.set_populations(f0)
    with _gpu_set([params], graph_steps=0) as gs:
        gs.set_populations(0, f0)
        gs.step(37)
        s.step(37)
        _compare_state(gs, 0, s)
        po = s.probes()
        assert np.abs(gs.probes(0, 0, 37) - po).max() <= 1e-12 * np.abs(po).max()


def test_graph_replay_equals_eager_launches():
    params = dict(nx=32, ny=16, nz=24, tau=0.9, bc=(0, 0, 0, 0, 2, 2), wave=inputs.WAVE_SINE, amp=1e-3, omega=0.1,
                  t_n=1000, probe_z=(3, 11), max_particles=4)
    pk = {"x": np.array([[10.3, 8.1, 12.2], [22.0, 7.6, 11.9]]), "radius": np.array([3.3, 2.9]),
          "v": np.array([[1e-3, 0, 2e-3], [0, -1e-3, 0]])}
    res = []
    for gsteps in (0, 8):
        with _gpu_set([params], graph_steps=gsteps) as gs:
            _set_particles(gs, 0, pk)
            gs.step(29)
            res.append((gs.populations(0), gs.owner(0), gs.particles_get(0), gs.probes(0, 0, 29)))
    a, b = res
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k])


# ---------------------------------------------------------------------------
# projection of spheres (integer, bit-exact)
# ---------------------------------------------------------------------------
def test_projection_bitexact_with_ties():
    X = np.array([(4.0, 4.0, 4.0), (7.0, 4.0, 4.0), (0.25, 8.5, 3.75), (10.0, 10.0, 8.0)])
    R = np.array([2.0, 2.0, 2.5, 1.75])
    params = dict(nx=12, ny=13, nz=11, tau=1.0, bc=(0, 0, 0, 0, 1, 1), max_particles=8)
    s = _oracle(params, {"x": X, "radius": R})
    with _gpu_set([params]) as gs:
        gs.particles_set(0, X, R)
        assert np.array_equal(gs.owner(0), s.owner())


@pytest.mark.parametrize("seed", [0, 1])
def test_projection_bitexact_fcc(seed):
    params, pk = inputs.wave_fcc_case(seed=seed, ncx=2, ncy=2, ncz=3, a=24.0, overlap_rel=1e-2)
    params["max_particles"] = len(pk["x"])
    s = _oracle(params, pk)
    with _gpu_set([params]) as gs:
        _set_particles(gs, 0, pk)
        assert np.array_equal(gs.owner(0), s.owner())


# ---------------------------------------------------------------------------
# coupled steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("node_lists", [0, 1, 2])
def test_coupled_moving_sphere_with_conversions_fp64(node_lists):
    """A fast sphere in a periodic box: links, cover/uncover conversions every step; with
    node lists, the lists are rebuilt every few steps as the sphere moves (with compact
    storage the populations move with them, and every comparison reads them back through
    the node layout)."""
    params = dict(nx=16, ny=15, nz=17, tau=0.8, bc=(0,) * 6, rho_p=1.2, max_particles=2)
    pk = {"x": np.array([[7.3, 6.9, 8.6]]), "radius": np.array([3.2]), "v": np.array([[0.03, -0.02, 0.025]]),
          "w": np.array([[0.0, 0.01, -0.02]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=0, node_lists=node_lists) as gs:
        _set_particles(gs, 0, pk)
        for _ in range(4):
            gs.step(15)
            s.step(15)
            _compare_state(gs, 0, s, pk)
        ph_o, lh_o = s.pending()
        assert gs.status() & 0x192 == 0


def test_compact_planes_beyond_the_grid_estimate_fp64():
    """Three heavily overlapping large spheres: the fluid grid's estimate (sphere
    cross-sections summed, overlaps counted twice) leaves one workgroup per plane, so
    every plane's second chunk of listed nodes is done by a further pass of the same
    workgroup; the state and the probe sums still match the oracle."""
    params = dict(nx=32, ny=32, nz=12, tau=0.9, bc=(0, 0, 0, 0, 1, 1), rho_p=1.5, E=1e-9, max_particles=3,
                  max_radius=14.0, probe_z=[2, 6, 9])
    pk = {"x": np.array([[15.6, 16.2, 5.5], [16.4, 15.7, 5.9], [16.0, 16.5, 5.2]]),
          "radius": np.array([13.5, 13.2, 13.4]),
          "v": np.array([[0.01, -0.004, 0.002], [-0.006, 0.008, -0.003], [0.002, 0.003, 0.004]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=4, node_lists=2) as gs:
        _set_particles(gs, 0, pk)
        gs.step(24)
        s.step(24)
        _compare_state(gs, 0, s, pk)
        pg, po = gs.probes(0, 0, 24), s.probes()
        assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
        assert gs.status() & 0x1da == 0


def test_large_moving_sphere_fp64():
    """One sphere of radius 20 moving through a periodic 48^3 box: a chunk of its shell list
    holds more link entries than a rebuild keeps in LDS (its link-set sums read the entries
    back from memory), and past a tenth of a node of motion the re-projection takes its
    candidates from the whole shell list, in many batches; the state matches the oracle."""
    params = dict(nx=48, ny=48, nz=48, tau=0.8, bc=(0,) * 6, rho_p=2.0, max_particles=1, max_radius=20.0,
                  probe_z=[10, 24])
    pk = {"x": np.array([[23.6, 24.3, 24.1]]), "radius": np.array([20.0]),
          "v": np.array([[0.02, -0.015, 0.01]]), "w": np.array([[0.0, 0.001, -0.0005]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=4) as gs:
        _set_particles(gs, 0, pk)
        for n in (8, 12):
            gs.step(n)
            s.step(n)
            _compare_state(gs, 0, s, pk)
        assert gs.status() & 0x1da == 0


@pytest.mark.parametrize("margin", [0, 2])
def test_moving_sphere_parked_refills_fp64(margin):
    """Compact storage with the list rebuild trigger's look-ahead switched off: nodes turn
    fluid outside the lists, their refills wait for the next step's rebuild (status bit
    0x200), and the state still matches the oracle step for step."""
    params = dict(nx=18, ny=16, nz=17, tau=0.8, bc=(0,) * 6, rho_p=3.0, max_particles=2)
    pk = {"x": np.array([[7.3, 6.9, 8.6]]), "radius": np.array([3.2]), "v": np.array([[0.09, -0.06, 0.07]]),
          "w": np.array([[0.0, 0.01, -0.02]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=0, node_lists=2, list_margin=margin) as gs:
        _set_particles(gs, 0, pk)
        gs.step(23)
        s.step(23)
        _compare_state(gs, 0, s, pk)
        gs.step(37)
        s.step(37)
        _compare_state(gs, 0, s, pk)
        st = gs.status()
        assert st & 0x1da == 0
        if margin == 0:
            assert st & 0x200, "no refill was parked"


@pytest.mark.parametrize("node_lists", [0, 2])
def test_head_on_collision_fp64(node_lists):
    """Two spheres driven into each other: the overlap grows to ~0.75 lu (lens nodes change
    owner, shell lists are rebuilt) and the Hertz contact reverses the motion, so the
    displacement from a shell list's reference shrinks again while nodes keep changing."""
    params = dict(nx=40, ny=20, nz=20, tau=0.8, bc=(0,) * 6, E=10.0, nu=0.2, mu=0.3, rho_p=1.5, max_particles=2)
    pk = {"x": np.array([[12.0, 10.0, 10.2], [22.4, 9.8, 9.9]]), "radius": np.array([5.0, 5.0]),
          "v": np.array([[0.04, 0.0, 0.01], [-0.04, 0.005, 0.0]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=0, node_lists=node_lists) as gs:
        _set_particles(gs, 0, pk)
        for _ in range(6):
            gs.step(10)
            s.step(10)
            _compare_state(gs, 0, s, pk)
        assert gs.status() & 0x1da == 0


@pytest.mark.parametrize("node_lists", [0, 1, 2])
def test_coupled_fcc_wave_fp64(node_lists):
    params, pk = inputs.wave_fcc_case(seed=2, ncx=2, ncy=2, ncz=3, a=24.0, overlap_rel=1e-2, period=40.0, amp=5e-3)
    params["max_particles"] = len(pk["x"])
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=4, node_lists=node_lists) as gs:
        _set_particles(gs, 0, pk)
        gs.step(60)
        s.step(60)
        _compare_state(gs, 0, s, pk)
        pg, po = gs.probes(0, 0, 60), s.probes()
        assert np.abs(pg - po).max() <= 1e-12 * np.abs(po).max()
        assert gs.status() & 0x180 == 0


def test_settling_sphere_walls_fp64():
    params, pk = inputs.settling_case()
    params["max_particles"] = 1
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=8) as gs:
        _set_particles(gs, 0, pk)
        gs.step(120)
        s.step(120)
        _compare_state(gs, 0, s, pk)


@pytest.mark.parametrize("tau,centre,node_lists", [(0.8, (16.0, 16.0, 16.0), None), (0.6, (16.0, 16.0, 16.0), None),
                                                   (1.4, (1.3, 30.6, 31.85), None), (1.4, (1.3, 30.6, 31.85), 2)])
def test_settling_sphere_periodic_fp64(tau, centre, node_lists):
    """The settling set-up of Sec. 3.1 (fully periodic cube, R = 5.005, F_g = 0.1 net of
    buoyancy) in a 32^3 box; the last cases start next to the box corner, so the sphere
    straddles three periodic faces and crosses the top face while it falls upwards (with
    the automatic mapping, dense tiles here, and with compact node lists)."""
    params, pk = inputs.settling_periodic_case(tau, n=32)
    pk = dict(pk, x=np.array([centre]))
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=8, node_lists=node_lists) as gs:
        _set_particles(gs, 0, pk)
        gs.step(150)
        s.step(150)
        _compare_state(gs, 0, s, pk)
        assert gs.status() == 0


def test_friction_contacts_fp64():
    """Two spheres pressed together and sheared: Hertz + Mindlin with a Coulomb cap."""
    params = dict(nx=40, ny=24, nz=24, tau=1.0, bc=(0,) * 6, E=10.0, nu=0.2, mu=0.3, rho_p=2.0, max_particles=3)
    pk = {"x": np.array([[14.0, 12.0, 11.7], [21.95, 12.2, 11.9]]), "radius": np.array([4.0, 4.0]),
          "v": np.array([[0.0, 2e-3, 0.0], [0.0, -2e-3, 1e-3]]), "w": np.array([[0, 0, 1e-3], [0, 0, 0]])}
    s = _oracle(params, pk)
    with _gpu_set([params], graph_steps=0) as gs:
        _set_particles(gs, 0, pk)
        gs.step(40)
        s.step(40)
        _compare_state(gs, 0, s, pk)
        assert gs.status() == 0


def test_ensemble_members_match_independent_oracles():
    members = []
    for k, (ncx, ncz, ov, per) in enumerate([(2, 2, 1e-3, 50), (2, 3, 1e-2, 80), (2, 2, 1e-4, 120)]):
        params, pk = inputs.wave_fcc_case(seed=10 + k, ncx=ncx, ncy=ncx, ncz=ncz, a=24.0, overlap_rel=ov,
                                          period=per, amp=3e-3)
        params["max_particles"] = len(pk["x"]) + 3
        members.append((params, pk))
    sims = [_oracle(p, pk) for p, pk in members]
    with _gpu_set([p for p, _ in members], graph_steps=4) as gs:
        for k, (_, pk) in enumerate(members):
            _set_particles(gs, k, pk)
        gs.step(24)
        for k, (p, pk) in enumerate(members):
            sims[k].step(24)
            _compare_state(gs, k, sims[k], pk)
            po = sims[k].probes()
            assert np.abs(gs.probes(k, 0, 24) - po).max() <= 1e-12 * np.abs(po).max()


def test_runs_are_bit_reproducible():
    params, pk = inputs.wave_fcc_case(seed=4, ncx=2, ncy=2, ncz=2, a=24.0, overlap_rel=1e-2, period=30.0, amp=5e-3)
    params["max_particles"] = len(pk["x"])
    outs = []
    for _ in range(2):
        with _gpu_set([params], precision="fp32", graph_steps=8) as gs:
            _set_particles(gs, 0, pk)
            gs.step(48)
            outs.append((gs.populations(0), gs.particles_get(0)))
    assert np.array_equal(outs[0][0], outs[1][0])
    for k in outs[0][1]:
        assert np.array_equal(outs[0][1][k], outs[1][1][k])


@pytest.mark.parametrize("precision,tol_f,tol_probe", [("fp32", 2e-6, 1e-6), ("fp16", 1e-3, 3e-4), ("bf16", 1e-2, 3e-3)])
def test_reduced_precision_error_bounds(precision, tol_f, tol_probe):
    """Stored precision changes only rounding: errors against the FP64 oracle stay within
    the storage resolution (relative to the deviation scale 1e-3 of the wave)."""
    params, pk = inputs.wave_fcc_case(seed=5, ncx=2, ncy=2, ncz=2, a=24.0, overlap_rel=1e-2, period=40.0, amp=1e-3)
    params["max_particles"] = len(pk["x"])
    s = _oracle(params, pk)
    with _gpu_set([params], precision=precision, graph_steps=8) as gs:
        _set_particles(gs, 0, pk)
        gs.step(40)
        s.step(40)
        own = s.owner()
        fl = own < 0
        df = np.abs(gs.populations(0)[:, fl] - s.populations()[:, fl]).max()
        pg, po = gs.probes(0, 0, 40), s.probes()
        rp = np.abs(pg[..., 1] / pg[..., 0] - po[..., 1] / po[..., 0]).max()
        assert df <= tol_f, df
        assert rp <= tol_probe, rp


def test_settling_full_size_momentum_balance():
    """The 160^3 settling set-up (Sec. 3.1) at full size, FP32 storage as benchmarked: the
    periodic box has no other external force than F_g, so the fluid momentum summed from
    the populations equals F_g t - m_p V_p (up to the MEM's refill and emptying exchange)."""
    params, pk = inputs.settling_periodic_case(1.0)
    c = _printed_matrix_local()
    with _gpu_set([params], precision="fp32", graph_steps=8) as gs:
        _set_particles(gs, 0, pk)
        gs.step(2000)
        f = gs.populations(0)
        fluid = gs.owner(0) < 0
        p = gs.particles_get(0)
        assert gs.status() == 0
    mom = (c.T @ f[:, fluid]).sum(1)
    m_p = params["rho_p"] * 4.0 / 3.0 * math.pi * pk["radius"][0] ** 3
    want = 0.1 * 2000 - m_p * p["v"][0, 2]
    assert mom[2] == pytest.approx(want, rel=2e-3)
    assert abs(mom[0]) < 1e-3 * want and abs(mom[1]) < 1e-3 * want
    # the sphere falls along +z at about the terminal speed of Eq. (termVel) reached later
    assert 4e-3 < p["v"][0, 2] < 8e-3


def _printed_matrix_local():
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "d3q19_velocity_matrix.txt")
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    return np.array(rows, dtype=float).T  # (19, 3)
