"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module only builds input arrays (particle packings, per-sample parameters).  It
holds none of the method's arithmetic: no lattice-Boltzmann, contact or coupling
formula lives here, so both sides of every parity check consume identical inputs
without sharing any of the code under test.

Packings follow the setups of the paper (arXiv 1808.08921):
  * FCC packing of equal spheres with end layers fixed and periodic sides
    (Sec. "Face-centered cubic packing of frictionless spheres"), radius
    R = R0 + |u_n|/2 where R0 leaves zero overlap and |u_n| is the overlap;
  * a single sphere settling under a body force (Sec. "Terminal velocity");
  * a chain of spheres along the propagation axis (Sec. "Pressure wave ...").
"""
from __future__ import annotations

import math

import numpy as np

# face codes shared with the C interfaces (-x,+x,-y,+y,-z,+z order)
PERIODIC, WALL, PRESSURE = 0, 1, 2
WAVE_NONE, WAVE_SINE, WAVE_COSINE, WAVE_STEP = 0, 1, 2, 3

# FCC basis in units of the cubic cell edge
_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_packing(ncx: int, ncy: int, ncz: int, a: float = 24.0, overlap_rel: float = 1e-3,
                jitter: float = 0.05, seed: int = 0, z_shift: float | None = None,
                fix_end_layers: bool = True, touching: bool = True, radius: float | None = None):
    """FCC packing of ncx*ncy*ncz cubic cells (4 spheres each), cell edge ``a``.

    R0 = a / (2 sqrt 2) is the touching radius (zero overlap).  Each sphere gets an
    overlap u_p = overlap_rel * R0 * (1 + jitter * (2 U_p - 1)), U_p ~ U(0,1) from
    ``numpy.random.default_rng(seed)``, and radius R0 + u_p / 2.  With
    ``touching=False`` every sphere has the literal ``radius`` instead.
    Centres sit on the FCC sites shifted by ``z_shift`` (default a/4) along z so that
    both z ends cut the packing alike.  Spheres of the lowest and highest z layer are
    flagged fixed.  Returns dict(x (n,3), radius (n,), fixed (n,) uint8, shape (nx,ny,nz)).
    """
    if z_shift is None:
        z_shift = a / 4.0
    sites = []
    for k in range(ncz):
        for j in range(ncy):
            for i in range(ncx):
                for b in _FCC_BASIS:
                    sites.append(((i + b[0]) * a, (j + b[1]) * a, (k + b[2]) * a + z_shift))
    x = np.array(sites, dtype=np.float64)
    # order spheres by (z, y, x) so that indices grow along the propagation axis
    order = np.lexsort((x[:, 0], x[:, 1], x[:, 2]))
    x = x[order]
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    r0 = a / (2.0 * math.sqrt(2.0))
    if touching:
        overlap = overlap_rel * r0 * (1.0 + jitter * (2.0 * u - 1.0))
        rad = r0 + 0.5 * overlap
    else:
        rad = np.full(n, float(radius if radius is not None else r0))
    fixed = np.zeros(n, dtype=np.uint8)
    if fix_end_layers and n:
        zmin, zmax = x[:, 2].min(), x[:, 2].max()
        fixed[np.isclose(x[:, 2], zmin)] = 1
        fixed[np.isclose(x[:, 2], zmax)] = 1
    shape = (int(round(ncx * a)), int(round(ncy * a)), int(round(ncz * a)))
    return {"x": x, "radius": rad, "fixed": fixed, "shape": shape}


def wave_fcc_case(seed: int = 0, ncx: int = 4, ncy: int = 4, ncz: int = 16, a: float = 24.0,
                  overlap_rel: float = 1e-3, period: float = 200.0, amp: float = 1e-3):
    """FCC wave-propagation workload: periodic x,y, density inlet at z = 0 driven by a
    single-period cosine pulse, constant density at the top face, probes every 16 lu.
    Material constants follow the paper's parameter table in lattice units
    (rho_p* = 2.466, E* = 10.37, nu_p = 0.2, mu = 0, tau* = 1)."""
    pk = fcc_packing(ncx, ncy, ncz, a=a, overlap_rel=overlap_rel, seed=seed)
    nx, ny, nz = pk["shape"]
    params = dict(nx=nx, ny=ny, nz=nz, tau=1.0, rho_f=1.0,
                  bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC, PRESSURE, PRESSURE),
                  wave=WAVE_COSINE, amp=amp, omega=2.0 * math.pi / period, t_n=int(round(period)),
                  E=10.37, nu=0.2, mu=0.0, rho_p=2.466,
                  probe_z=tuple(range(0, nz, 16)), max_radius=float(np.ceil(pk["radius"].max())))
    return params, pk


def fcc_layers(x, a: float = 24.0, z_shift: float | None = None):
    """Layer index of each sphere of an FCC packing made by fcc_packing: its planes normal to
    z are a / 2 apart, starting at z_shift (default a / 4)."""
    if z_shift is None:
        z_shift = a / 4.0
    return np.rint((np.asarray(x)[:, 2] - z_shift) / (0.5 * a)).astype(np.int32)


def settling_case(n: int = 32, radius: float = 6.0, density_ratio: float = 2.0, g: float = 1e-5,
                  tau: float = 0.8, centre=None):
    """Single sphere settling in a closed box with half-way walls on every face.  The
    fluid carries no body force; the sphere gets its weight net of buoyancy,
    F_g = (rho_p - rho_f) (4/3) pi R^3 g, pointing to -z."""
    if centre is None:
        centre = (n / 2 - 0.5, n / 2 - 0.5, n - 8.5)
    vol = 4.0 / 3.0 * math.pi * radius ** 3
    fg = np.array([[0.0, 0.0, -(density_ratio - 1.0) * vol * g]])
    params = dict(nx=n, ny=n, nz=n, tau=tau, rho_f=1.0, bc=(WALL,) * 6, wave=WAVE_NONE, amp=0.0,
                  omega=0.0, t_n=0, E=10.0, nu=0.2, mu=0.0, rho_p=density_ratio, probe_z=(),
                  max_radius=float(radius))
    pk = {"x": np.array([centre], dtype=np.float64), "radius": np.array([radius]),
          "fixed": np.zeros(1, np.uint8), "fg": fg, "shape": (n, n, n)}
    return params, pk


def chain_case(n_spheres: int = 60, r0: float = 5.0, overlap: float = 0.01, side: int = 12,
               length: int = 620, fixed: bool = False):
    """Granular chain along z (Sec. "Pressure wave in fluids ..."): spheres of radius
    R0 + overlap/2 at z = i (2R - overlap), i = 1..n, centred at x = y = side/2."""
    rad = r0 + 0.5 * overlap
    z = np.array([i * (2.0 * rad - overlap) for i in range(1, n_spheres + 1)])
    x = np.stack([np.full(n_spheres, side / 2.0), np.full(n_spheres, side / 2.0), z], axis=1)
    return {"x": x, "radius": np.full(n_spheres, rad),
            "fixed": np.full(n_spheres, 1 if fixed else 0, np.uint8), "shape": (side, side, length)}


def adjoint_fcc_case(n_xy: int = 64, nz: int = 256, radius: float = 8.0, offset: float = 8.0,
                     period: float = 200.0, amp: float = 1e-3):
    """Frozen packing of the adjoint workload: touching FCC spheres of radius R (cubic cell
    a = 2 sqrt(2) R) in an n_xy x n_xy x nz lattice with walls on the x and y faces and
    density faces in z; FCC sites shifted by `offset` on every axis, keeping the spheres
    whose centres lie at least R inside the lattice on every axis (275 spheres for the
    defaults).  Returns (params, packing) like wave_fcc_case."""
    a = 2.0 * math.sqrt(2.0) * radius
    hi = (n_xy - 1 - radius, n_xy - 1 - radius, nz - 1 - radius)
    sites = []
    for k in range(int(nz / a) + 2):
        for j in range(int(n_xy / a) + 2):
            for i in range(int(n_xy / a) + 2):
                for b in _FCC_BASIS:
                    p = ((i + b[0]) * a + offset, (j + b[1]) * a + offset, (k + b[2]) * a + offset)
                    if all(radius <= p[ax] <= hi[ax] for ax in range(3)):
                        sites.append(p)
    x = np.array(sites, dtype=np.float64)
    x = x[np.lexsort((x[:, 0], x[:, 1], x[:, 2]))]
    n = x.shape[0]
    params = dict(nx=n_xy, ny=n_xy, nz=nz, tau=1.0, rho_f=1.0, bc=(WALL, WALL, WALL, WALL, PRESSURE, PRESSURE),
                  wave=WAVE_COSINE, amp=amp, omega=2.0 * math.pi / period, t_n=int(round(period)),
                  E=10.37, nu=0.2, mu=0.0, rho_p=2.466, probe_z=tuple(range(16, nz, 16)), max_radius=radius + 1.0)
    pk = {"x": x, "radius": np.full(n, radius), "fixed": np.ones(n, np.uint8), "shape": (n_xy, n_xy, nz)}
    return params, pk


def ensemble_members(n: int = 64, base_seed: int = 1000, a: float = 24.0):
    """Uneven FCC samples for the batched ensemble: sample s draws, from
    default_rng(base_seed + s), n_xy in {2,3,4}, n_z in {8..16}, overlap
    10**U(-4,-2) of R0 and an inlet period in {50..400} steps."""
    out = []
    for s in range(n):
        rng = np.random.default_rng(base_seed + s)
        nxy = int(rng.integers(2, 5))
        ncz = int(rng.integers(8, 17))
        ov = float(10.0 ** rng.uniform(-4.0, -2.0))
        period = int(rng.integers(50, 401))
        params, pk = wave_fcc_case(seed=base_seed + s, ncx=nxy, ncy=nxy, ncz=ncz, a=a, overlap_rel=ov,
                                   period=period)
        out.append((params, pk))
    return out


def random_populations(shape, rho_f: float = 1.0, amp: float = 1e-3, seed: int = 0):
    """Seeded near-equilibrium populations [19][nz][ny][nx]: rest weights times
    (rho_f + noise).  The weights are the D3Q19 lattice weights listed in the paper
    (1/3 rest, 1/18 axis, 1/36 diagonal), indexed as in its velocity matrix."""
    w = np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3])
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    noise = amp * (2.0 * rng.random((19, nz, ny, nx)) - 1.0)
    return w[:, None, None, None] * (rho_f + noise)


def probe_signal(n_t: int, zpos, omega: float, amp: complex, alpha: float, k: float, t0: float = 0.0,
                 offset: float = 0.0, harmonic: float = 0.0, noise: float = 0.0, seed: int = 0):
    """Synthetic probe record x[t, z] (float64, [n_t, len(zpos)]) for the dispersion analysis:
    a damped harmonic wave Re[amp exp(-alpha z) exp(j (omega (t0 + t) - k z))] travelling
    towards +z, plus a constant offset, a second harmonic of relative size `harmonic` and
    seeded Gaussian noise of standard deviation `noise`."""
    z = np.asarray(zpos, dtype=np.float64)[None, :]
    t = (t0 + np.arange(n_t, dtype=np.float64))[:, None]
    base = np.real(amp * np.exp(-alpha * z) * np.exp(1j * (omega * t - k * z)))
    sec = harmonic * np.real(amp * np.exp(-2 * alpha * z) * np.exp(2j * (omega * t - k * z)))
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(base + sec + offset + noise * rng.standard_normal((n_t, z.shape[1])))


# Table tab:source of the paper: (input frequency in MHz, waveform) of the oscillating
# density boundary; the density amplitude is 0.2 kg/m^3 against rho_f = 1e3 kg/m^3, and
# the waveform acts for a single period.  Table 1 fixes the time unit, 1.54e-6 ms.
SOURCE_TABLE = ((6.50, WAVE_STEP), (6.50, WAVE_COSINE), (6.50, WAVE_SINE),
                (1.30, WAVE_COSINE), (3.25, WAVE_COSINE), (13.0, WAVE_COSINE))
TIME_UNIT_S = 1.54e-9
SOURCE_AMP = 0.2 / 1.0e3


def source_omega(f_mhz: float) -> float:
    """Angular frequency in lattice units (rad per step) of an input frequency in MHz."""
    return 2.0 * math.pi * f_mhz * 1.0e6 * TIME_UNIT_S


def source_table_rows():
    """The six sources of Table tab:source as lattice parameters (wave, amp, omega, t_n),
    each acting for one period (t_n = the period rounded to whole steps)."""
    rows = []
    for f, wave in SOURCE_TABLE:
        om = source_omega(f)
        rows.append(dict(wave=wave, amp=SOURCE_AMP, omega=om, t_n=int(round(2.0 * math.pi / om)), f_mhz=f))
    return rows


def source_sweep_fcc(seed: int = 0, **kw):
    """The Table tab:source sweep as a batched ensemble: the FCC wave case (same packing
    for every member) driven by each of the six sources."""
    out = []
    for row in source_table_rows():
        params, pk = wave_fcc_case(seed=seed, **kw)
        params.update({k: row[k] for k in ("wave", "amp", "omega", "t_n")})
        out.append((params, pk))
    return out


def impulse_fcc_case(seed: int = 0, ncx: int = 2, ncy: int = 2, ncz: int = 6, a: float = 12.0,
                     overlap_rel: float = 1e-3, push: float = 5.0):
    """Mechanically agitated impulse (Sec. 4.2): the FCC case without an acoustic source
    (both density faces held at rho_f), the first mobile layer of spheres moved towards the
    fixed layer at z = 0 by `push` times the mean overlap, so that its contacts with the
    fixed layer start with overlaps larger than elsewhere."""
    params, pk = wave_fcc_case(seed=seed, ncx=ncx, ncy=ncy, ncz=ncz, a=a, overlap_rel=overlap_rel)
    params.update(wave=WAVE_NONE, amp=0.0, omega=0.0, t_n=0)
    z = pk["x"][:, 2]
    zl = np.unique(np.round(z, 6))
    first_free = np.isclose(z, zl[1], atol=1e-5)
    r0 = a / (2.0 * math.sqrt(2.0))
    mean_overlap = float(np.mean(2.0 * (pk["radius"] - r0)))
    x = pk["x"].copy()
    x[first_free, 2] -= push * mean_overlap
    pk = dict(pk, x=x)
    return params, pk


def settling_periodic_case(tau: float, n: int = 160, r0: float = 5.0, overlap: float = 0.01, fg: float = 0.1,
                           rho_p: float = 2.466):
    """Single sphere settling in a fully periodic cube (Sec. 3.1): radius R0 + |u_n|/2
    (5.005 for the paper's values), released at rest at the centre, driven by the constant
    force F_g = (0, 0, fg) net of buoyancy; the fluid carries no body force."""
    radius = r0 + 0.5 * overlap
    params = dict(nx=n, ny=n, nz=n, tau=tau, rho_f=1.0, bc=(PERIODIC,) * 6, wave=WAVE_NONE, amp=0.0, omega=0.0,
                  t_n=0, E=10.0, nu=0.2, mu=0.0, rho_p=rho_p, probe_z=(), max_radius=float(math.ceil(radius)),
                  max_particles=1)
    pk = {"x": np.array([[n / 2.0, n / 2.0, n / 2.0]]), "radius": np.array([radius]),
          "fixed": np.zeros(1, np.uint8), "fg": np.array([[0.0, 0.0, fg]]), "shape": (n, n, n)}
    return params, pk


def dry_chain_case(side: int = 12, length: int = 620, rho_p: float = 2.466):
    """The dry granular chain of Sec. 3.2 (second benchmark, hydrodynamics switched off):
    60 spheres of radius 5.005 at z = i (2R - 0.01) on the axis x = y = side / 2, the first
    one moved to z = 10.001, E_p = 10, nu_p = 0.2, in the paper's 12 x 12 cross-section.
    Without fluid the lattice only hosts the node map."""
    pk = chain_case(side=side, length=length)
    x = pk["x"].copy()
    x[0, 2] = 10.001
    pk = dict(pk, x=x)
    params = dict(nx=side, ny=side, nz=length, tau=1.0, rho_f=1.0,
                  bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC, PRESSURE, PRESSURE), wave=WAVE_NONE, amp=0.0,
                  omega=0.0, t_n=0, E=10.0, nu=0.2, mu=0.0, rho_p=rho_p, probe_z=(),
                  max_particles=len(x), max_radius=6.0)
    return params, pk
