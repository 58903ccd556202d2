"""Test infrastructure only: a ctypes wrapper around the plain FP64 CPU oracle.

The oracle (``lbdem_oracle.c``) is a slow, obviously correct reference of the coupled
lattice-Boltzmann / DEM step of Cheng et al. (arXiv 1808.08921).  Only the tests, the
package smoke check and the CPU-baseline leg of ``bench.py`` may import this module.
The GPU library never imports, links or calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbdem_oracle.c")
_LIB = os.path.join(_HERE, "liblbdem_oracle.so")

BC_PERIODIC, BC_WALL, BC_PRESSURE = 0, 1, 2
WAVE_NONE, WAVE_SINE, WAVE_COSINE, WAVE_STEP = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        D, I, L64, P = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_ubyte)
        L.orc_create.restype = P
        L.orc_create.argtypes = [I, I, I, D, D, ip, I, D, D, L64, D, D, D, D, I, ip]
        L.orc_destroy.argtypes = [P]
        L.orc_set_particles.argtypes = [P, I, dp, dp, dp, dp, dp, up]
        L.orc_step.argtypes = [P, L64]
        L.orc_time.restype = L64
        L.orc_time.argtypes = [P]
        L.orc_ncell.restype = L64
        L.orc_ncell.argtypes = [P]
        for fn in (L.orc_get_populations, L.orc_set_populations):
            fn.argtypes = [P, dp]
        L.orc_get_owner.argtypes = [P, ip]
        L.orc_classify.argtypes = [P, ip]
        L.orc_get_particles.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_get_pending.argtypes = [P, dp, dp]
        L.orc_get_probes.restype = I
        L.orc_get_probes.argtypes = [P, L64, L64, dp]
        L.orc_velocity_set.argtypes = [ip, dp, ip]
        L.orc_equilibrium.argtypes = [D, dp, dp]
        L.orc_collide_node.argtypes = [dp, D, dp]
        L.orc_zou_he.argtypes = [dp, D, I]
        L.orc_rho_in_value.restype = D
        L.orc_rho_in_value.argtypes = [I, D, D, D, L64, L64]
        L.orc_set_frozen.argtypes = [P, I]
        L.orc_set_fluid_off.argtypes = [P, I]
        L.orc_set_rest_free.argtypes = [P, I]
        L.orc_set_velocities.argtypes = [P, dp, dp]
        L.orc_adjoint.restype = I
        L.orc_adjoint.argtypes = [P, L64, D, D, dp, dp, dp, dp, dp]
        L.orc_contact.restype = I
        L.orc_contact.argtypes = [dp, dp, D, D, dp, dp, dp, dp, D, D, D, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------------------
# node-level functions
# ---------------------------------------------------------------------------
def velocity_set():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().orc_velocity_set(_ip(c), _dp(w), _ip(opp))
    return c, w, opp


def equilibrium(rho, u):
    u = _f64(u, (3,))
    out = np.zeros(19)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def collide_node(f, tau):
    f = _f64(f, (19,))
    out = np.zeros(19)
    lib().orc_collide_node(_dp(f), float(tau), _dp(out))
    return out


def zou_he(f, rho, outlet=False):
    f = _f64(f, (19,)).copy()
    lib().orc_zou_he(_dp(f), float(rho), 1 if outlet else 0)
    return f


def rho_in(wave, rho_f, amp, omega, t_n, t):
    return lib().orc_rho_in_value(int(wave), float(rho_f), float(amp), float(omega), int(t_n), int(t))


def contact(Xi, Xj, Ri, Rj, Vi=(0, 0, 0), Vj=(0, 0, 0), Wi=(0, 0, 0), Wj=(0, 0, 0), E=10.0, nu=0.2,
            mu=0.0, box=(0, 0, 0), ft_old=(0, 0, 0)):
    """Force/torque on particle i from j; returns (in_contact, F, T, ft_new)."""
    args = [_f64(a, (3,)) for a in (Xi, Xj)]
    vel = [_f64(a, (3,)) for a in (Vi, Vj, Wi, Wj)]
    bx, fo = _f64(box, (3,)), _f64(ft_old, (3,))
    F, T, fn = np.zeros(3), np.zeros(3), np.zeros(3)
    c = lib().orc_contact(_dp(args[0]), _dp(args[1]), float(Ri), float(Rj), _dp(vel[0]), _dp(vel[1]),
                          _dp(vel[2]), _dp(vel[3]), float(E), float(nu), float(mu), _dp(bx), _dp(fo),
                          _dp(F), _dp(T), _dp(fn))
    return bool(c), F, T, fn


# ---------------------------------------------------------------------------
# whole simulation
# ---------------------------------------------------------------------------
class Sim:
    """One lattice with its particles, stepped by the oracle."""

    def __init__(self, nx, ny, nz, tau=1.0, rho_f=1.0, bc=(0, 0, 0, 0, 0, 0), wave=WAVE_NONE, amp=0.0,
                 omega=0.0, t_n=0, E=10.0, nu=0.2, mu=0.0, rho_p=1.0, probe_z=(), rest_free=False):
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        self.rho_f = rho_f
        bc6 = np.ascontiguousarray(np.asarray(bc, dtype=np.int32))
        pz = np.ascontiguousarray(np.asarray(list(probe_z) or [0], dtype=np.int32))
        self.n_probe = len(probe_z)
        self._h = lib().orc_create(nx, ny, nz, float(tau), float(rho_f), _ip(bc6), int(wave), float(amp),
                                   float(omega), int(t_n), float(E), float(nu), float(mu), float(rho_p),
                                   len(probe_z), _ip(pz))
        if not self._h:
            raise ValueError("oracle: invalid lattice parameters")
        self.np = 0
        if rest_free:
            self.set_rest_free(True)

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_frozen(self, frozen=True):
        """Frozen geometry: particles keep X, V, Omega; no DEM and no re-projection."""
        lib().orc_set_frozen(self._h, 1 if frozen else 0)

    def set_fluid_off(self, off=True):
        """Hydrodynamics switched off (the dry granular chain of Sec. 3.2): steps move the
        particles under contacts and their own forces only."""
        lib().orc_set_fluid_off(self._h, 1 if off else 0)

    def set_rest_free(self, on=True):
        """Link forces of Eq. (fFS) without the rest state's part w_d rho_f (a reading for
        touching particles; for separated ones the part sums to zero)."""
        lib().orc_set_rest_free(self._h, 1 if on else 0)

    def set_velocities(self, v=None, w=None):
        v = None if v is None else _f64(v).reshape(self.np, 3)
        w = None if w is None else _f64(w).reshape(self.np, 3)
        lib().orc_set_velocities(self._h, _dp(v), _dp(w))

    def adjoint(self, nsteps, tau, amp, dLdP):
        """Forward nsteps over frozen geometry from the current state (probe signals P,
        plane averages of rho - rho_f), then the discrete adjoint for the loss gradient
        dLdP [nsteps][n_probe]: returns (P, dL/dtau, dL/damp, dL/dV [np][3])."""
        dLdP = _f64(dLdP).reshape(nsteps, self.n_probe)
        P = np.zeros((nsteps, max(self.n_probe, 1)))
        gt, ga = ctypes.c_double(), ctypes.c_double()
        gv = np.zeros((max(self.np, 1), 3))
        rc = lib().orc_adjoint(self._h, int(nsteps), float(tau), float(amp), _dp(dLdP), _dp(P), ctypes.byref(gt),
                               ctypes.byref(ga), _dp(gv))
        if rc != 0:
            raise MemoryError("oracle adjoint: out of memory")
        return P[:, : self.n_probe], gt.value, ga.value, gv[: self.np]

    def set_particles(self, x, radius, v=None, w=None, fg=None, fixed=None):
        x = _f64(x).reshape(-1, 3)
        n = x.shape[0]
        r = _f64(radius).reshape(n)
        v = _f64(np.zeros((n, 3)) if v is None else v).reshape(n, 3)
        w = _f64(np.zeros((n, 3)) if w is None else w).reshape(n, 3)
        fg = _f64(np.zeros((n, 3)) if fg is None else fg).reshape(n, 3)
        fx = np.ascontiguousarray(np.zeros(n, np.uint8) if fixed is None else np.asarray(fixed, np.uint8))
        lib().orc_set_particles(self._h, n, _dp(x), _dp(v), _dp(w), _dp(r), _dp(fg),
                                fx.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        self.np = n

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def t(self):
        return lib().orc_time(self._h)

    def populations(self):
        f = np.zeros((19,) + self.shape)
        lib().orc_get_populations(self._h, _dp(f))
        return f

    def set_populations(self, f):
        f = _f64(f).reshape((19,) + self.shape)
        lib().orc_set_populations(self._h, _dp(f))

    def owner(self):
        o = np.zeros(self.shape, dtype=np.int32)
        lib().orc_get_owner(self._h, _ip(o))
        return o

    def classify(self):
        o = np.zeros(self.shape, dtype=np.int32)
        lib().orc_classify(self._h, _ip(o))
        return o

    def particles(self):
        n = max(self.np, 1)
        out = [np.zeros((n, 3)) for _ in range(5)]
        lib().orc_get_particles(self._h, *[_dp(a) for a in out])
        return {k: a[: self.np] for k, a in zip(("x", "v", "w", "force", "torque"), out)}

    def pending(self):
        n = max(self.np, 1)
        ph, lh = np.zeros((n, 3)), np.zeros((n, 3))
        lib().orc_get_pending(self._h, _dp(ph), _dp(lh))
        return ph[: self.np], lh[: self.np]

    def probes(self, first=0, n=None):
        if n is None:
            n = self.t - first
        out = np.zeros((n, max(self.n_probe, 1), 4))
        if lib().orc_get_probes(self._h, int(first), int(n), _dp(out)) != 0:
            raise IndexError("oracle: probe range not recorded")
        return out[:, : self.n_probe, :]
