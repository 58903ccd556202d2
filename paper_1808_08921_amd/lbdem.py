"""ctypes binding of the C interface in ``include/lbdem.h``.

Argument marshalling only: every step of the coupled lattice-Boltzmann / DEM method runs
in the HIP kernels of ``liblbdem.so``.  PyTorch supplies the device workspace (one
``torch.uint8`` allocation) and the HIP stream (torch's current stream).  The library
must have been built (``paper_1808_08921_amd.build``); a missing library raises, there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbdem.so")

OK, EINVAL, EDEVICE, ECAPACITY, ENOMEM, ESTATE, ERANGE, ENUMERIC = 0, -1, -2, -3, -4, -5, -6, -7
PERIODIC, WALL, PRESSURE = 0, 1, 2
WAVE_NONE, WAVE_SINE, WAVE_COSINE, WAVE_STEP = 0, 1, 2, 3
FP64, FP32, FP16DEV, BF16DEV = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16DEV, "fp16dev": FP16DEV, "bf16": BF16DEV, "bf16dev": BF16DEV}
MAX_PROBES = 64

STATUS_NEAR_OVERFLOW = 0x2
STATUS_CHANGE_OVERFLOW = 0x4
STATUS_HISTORY_OVERFLOW = 0x8
STATUS_TOO_FAST = 0x10
STATUS_SHELL_OVERFLOW = 0x40
STATUS_LINK_OVERFLOW = 0x80
STATUS_LIST_MISS = 0x100
STATUS_LIST_PARKED = 0x200
STATUS_NONFINITE = 0x400


class LbdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbdem error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("face_bc", ctypes.c_int32 * 6),
        ("tau", ctypes.c_double), ("rho_f", ctypes.c_double),
        ("wave", ctypes.c_int32), ("rho_amp", ctypes.c_double), ("omega", ctypes.c_double),
        ("t_n", ctypes.c_int64),
        ("young_E", ctypes.c_double), ("poisson_nu", ctypes.c_double), ("friction_mu", ctypes.c_double),
        ("rho_p", ctypes.c_double),
        ("n_probe", ctypes.c_int32), ("probe_z", ctypes.c_int32 * MAX_PROBES),
        ("max_particles", ctypes.c_int32),
        ("max_radius", ctypes.c_double),
        ("tile_x", ctypes.c_int32),
        ("rest_free", ctypes.c_int32),
    ]


class Config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("probe_ring", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("z_per_thread", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("node_lists", ctypes.c_int32),
                ("list_margin", ctypes.c_int32), ("fluid_off", ctypes.c_int32), ("particle_ring", ctypes.c_int32)]


_lib = None


def lib():
    """Load liblbdem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1808_08921_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, VP, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbdem_last_error.restype = ctypes.c_char_p
        L.lbdem_default_config.argtypes = [ctypes.POINTER(Config)]
        L.lbdem_workspace_size.argtypes = [I32, ctypes.POINTER(Params), ctypes.POINTER(Config), ctypes.POINTER(SZ)]
        L.lbdem_create.argtypes = [I32, ctypes.POINTER(Params), ctypes.POINTER(Config), VP, SZ, VP, ctypes.POINTER(P)]
        L.lbdem_destroy.argtypes = [P]
        L.lbdem_set_stream.argtypes = [P, VP]
        L.lbdem_particles_set.argtypes = [P, I32, I32, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.lbdem_particles_get.argtypes = [P, I32, I32, dp, dp, dp, dp, dp]
        L.lbdem_step.argtypes = [P, I64]
        L.lbdem_time.argtypes = [P, ctypes.POINTER(I64)]
        L.lbdem_synchronize.argtypes = [P]
        L.lbdem_status.argtypes = [P, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int]
        L.lbdem_probe_read.argtypes = [P, I32, I64, I64, dp]
        L.lbdem_populations_get.argtypes = [P, I32, dp]
        L.lbdem_populations_set.argtypes = [P, I32, dp]
        L.lbdem_owner_get.argtypes = [P, I32, ctypes.POINTER(ctypes.c_int32)]
        L.lbdem_fields_get.argtypes = [P, I32, dp, dp, ctypes.POINTER(ctypes.c_int32)]
        L.lbdem_state_size.argtypes = [P, ctypes.POINTER(SZ)]
        L.lbdem_state_save.argtypes = [P, VP, SZ, ctypes.POINTER(SZ)]
        L.lbdem_state_load.argtypes = [P, VP, SZ]
        L.lbdem_timing_enable.argtypes = [P, ctypes.c_int]
        L.lbdem_timing_read.argtypes = [P, dp, ctypes.POINTER(I64)]
        L.lbdem_tile_info.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.lbdem_adj_workspace_size.argtypes = [P, I32, I64, I32, ctypes.POINTER(SZ)]
        L.lbdem_adj_create.argtypes = [P, I32, I64, I32, VP, SZ, ctypes.POINTER(P)]
        L.lbdem_adj_forward.argtypes = [P, ctypes.c_double, ctypes.c_double, dp, dp]
        L.lbdem_adj_backward.argtypes = [P, dp, dp, dp, dp]
        L.lbdem_adj_destroy.argtypes = [P]
        D = ctypes.c_double
        L.lbdem_probe_signal.argtypes = [P, I32, I64, I64, I32, VP]
        L.lbdem_particle_signal.argtypes = [P, I32, I64, I64, ctypes.POINTER(I32), I32, I32, VP]
        L.lbdem_biot_velocities.argtypes = [D, D, D, D, D, D, D, D, dp]
        L.lbdem_dft_workspace_size.argtypes = [I64, I32, I32, I32, ctypes.POINTER(SZ)]
        L.lbdem_st_dft.argtypes = [VP, I64, I32, VP, D, D, D, I32, D, D, I32, VP, VP, VP, SZ, VP]
        L.lbdem_wave_fit.argtypes = [VP, I64, I32, VP, D, D, VP, VP, SZ, VP]
        L.lbdem_wave_fit_noalloc.argtypes = [VP, I64, I32, VP, D, D, VP, VP]
        for name in ("lbdem_default_config", "lbdem_workspace_size", "lbdem_create", "lbdem_destroy",
                     "lbdem_set_stream", "lbdem_particles_set", "lbdem_particles_get", "lbdem_step", "lbdem_time",
                     "lbdem_synchronize", "lbdem_status", "lbdem_probe_read", "lbdem_populations_get",
                     "lbdem_populations_set", "lbdem_owner_get", "lbdem_fields_get", "lbdem_state_size",
                     "lbdem_state_save", "lbdem_state_load", "lbdem_timing_enable", "lbdem_timing_read",
                     "lbdem_tile_info", "lbdem_adj_workspace_size", "lbdem_adj_create", "lbdem_adj_forward",
                     "lbdem_adj_backward", "lbdem_adj_destroy", "lbdem_probe_signal", "lbdem_dft_workspace_size",
                     "lbdem_st_dft", "lbdem_wave_fit", "lbdem_wave_fit_noalloc", "lbdem_particle_signal",
                     "lbdem_biot_velocities"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise LbdemError(rc, lib().lbdem_last_error().decode())


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def make_params(nx, ny, nz, tau=1.0, rho_f=1.0, bc=(0, 0, 0, 0, 0, 0), wave=WAVE_NONE, amp=0.0, omega=0.0,
                t_n=0, E=10.0, nu=0.2, mu=0.0, rho_p=1.0, probe_z=(), max_particles=0, max_radius=12.0, tile_x=0,
                rest_free=False, **_ignored):
    p = Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for k in range(6):
        p.face_bc[k] = int(bc[k])
    p.tau, p.rho_f = float(tau), float(rho_f)
    p.wave, p.rho_amp, p.omega, p.t_n = int(wave), float(amp), float(omega), int(t_n)
    p.young_E, p.poisson_nu, p.friction_mu, p.rho_p = float(E), float(nu), float(mu), float(rho_p)
    pz = list(probe_z)
    if len(pz) > MAX_PROBES:
        raise ValueError("too many probe planes")
    p.n_probe = len(pz)
    for k, z in enumerate(pz):
        p.probe_z[k] = int(z)
    p.max_particles = int(max_particles)
    p.max_radius = float(max_radius)
    p.tile_x = int(tile_x)
    p.rest_free = 1 if rest_free else 0
    return p


class LatticeSet:
    """A set of lattices advanced together on one GPU (one lattice, or a batched ensemble).

    ``lattices``: list of dicts with the keys of :func:`make_params`.
    """

    def __init__(self, lattices, precision="fp32", probe_ring=4096, tile_x=0, z_per_thread=0, graph_steps=8,
                 device="cuda", node_lists=None, list_margin=None, fluid_off=False, particle_ring=0):
        import torch

        self._torch = torch
        L = lib()
        n = len(lattices)
        arr = (Params * n)()
        for k, d in enumerate(lattices):
            arr[k] = make_params(**d)
        self.shapes = [(d["nz"], d["ny"], d["nx"]) for d in lattices]
        self.n_probe = [len(d.get("probe_z", ())) for d in lattices]
        self.n_particles = [0] * n
        cfg = Config()
        _check(L.lbdem_default_config(ctypes.byref(cfg)))
        cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cfg.probe_ring, cfg.tile_x, cfg.z_per_thread, cfg.graph_steps = probe_ring, tile_x, z_per_thread, graph_steps
        if node_lists is not None:
            # 0 dense tiles, 1 node lists, 2 node lists with compact storage
            cfg.node_lists = int(node_lists)
        if list_margin is not None:
            cfg.list_margin = int(list_margin)
        # hydrodynamics switched off (the dry granular chain of Sec. 3.2)
        cfg.fluid_off = 1 if fluid_off else 0
        # steps of particle velocities kept for particle_signal
        cfg.particle_ring = int(particle_ring)
        nbytes = ctypes.c_size_t()
        _check(L.lbdem_workspace_size(n, arr, ctypes.byref(cfg), ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.device = torch.device(device)
        self._ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(L.lbdem_create(n, arr, ctypes.byref(cfg), ctypes.c_void_p(self._ws.data_ptr()), nbytes.value,
                              ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._arr = arr

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbdem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def particles_set(self, lattice, x, radius, v=None, w=None, fg=None, fixed=None):
        x = _f64(x, (-1, 3))
        n = x.shape[0]
        r = _f64(radius, (n,))
        v = None if v is None else _f64(v, (n, 3))
        w = None if w is None else _f64(w, (n, 3))
        fg = None if fg is None else _f64(fg, (n, 3))
        fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.uint8).reshape(n))
        fxp = None if fx is None else fx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        _check(lib().lbdem_particles_set(self._h, lattice, n, _dp(x), _dp(v), _dp(w), _dp(r), _dp(fg), fxp))
        self.n_particles[lattice] = n

    def particles_get(self, lattice):
        n = self.n_particles[lattice]
        out = {k: np.zeros((n, 3)) for k in ("x", "v", "w", "force", "torque")}
        _check(lib().lbdem_particles_get(self._h, lattice, n, *[_dp(out[k]) for k in ("x", "v", "w", "force", "torque")]))
        return out

    def step(self, n=1):
        _check(lib().lbdem_step(self._h, int(n)))

    def synchronize(self):
        _check(lib().lbdem_synchronize(self._h))

    @property
    def t(self):
        t = ctypes.c_int64()
        _check(lib().lbdem_time(self._h, ctypes.byref(t)))
        return t.value

    def status(self, clear=False):
        b = ctypes.c_uint32()
        rc = lib().lbdem_status(self._h, ctypes.byref(b), 1 if clear else 0)
        if rc not in (OK, ECAPACITY, ENUMERIC):
            _check(rc)
        return b.value

    def check(self):
        """Raise LbdemError when a device error bit is set (ENUMERIC for the density watchdog)."""
        b = ctypes.c_uint32()
        _check(lib().lbdem_status(self._h, ctypes.byref(b), 0))

    def probes(self, lattice, first=0, n=None):
        if n is None:
            n = self.t - first
        out = np.zeros((n, max(self.n_probe[lattice], 1), 4))
        _check(lib().lbdem_probe_read(self._h, lattice, int(first), int(n), _dp(out)))
        return out[:, : self.n_probe[lattice], :]

    def probe_signal(self, lattice, first=0, n=None, quantity="density"):
        """Cross-section averages of every probe plane for steps [first, first + n) as a device
        tensor [n][n_probe] (float64), gathered from the probe ring on the set's stream:
        quantity "density" gives rho', "momentum" gives sum(rho u_z) / sum(rho)."""
        torch = self._torch
        if n is None:
            n = self.t - first
        q = {"density": 0, "momentum": 1}[quantity]
        x = torch.zeros((n, self.n_probe[lattice]), dtype=torch.float64, device=self.device)
        _check(lib().lbdem_probe_signal(self._h, lattice, int(first), int(n), q, ctypes.c_void_p(x.data_ptr())))
        return x

    def particle_signal(self, lattice, layer, n_layers, first=0, n=None, component=2):
        """Layer-averaged particle velocities for steps [first, first + n) as a device tensor
        [n][n_layers] (float64), gathered from the particle-velocity ring: ``layer[q]`` is the
        layer of particle q (-1: left out), ``component`` the velocity component (0, 1, 2)."""
        torch = self._torch
        if n is None:
            n = self.t - first
        lay = np.ascontiguousarray(np.asarray(layer, dtype=np.int32))
        if lay.shape != (self.n_particles[lattice],):
            raise ValueError(f"need one layer per particle ({self.n_particles[lattice]}), got {lay.shape}")
        x = torch.zeros((n, n_layers), dtype=torch.float64, device=self.device)
        _check(lib().lbdem_particle_signal(self._h, lattice, int(first), int(n),
                                           lay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(n_layers),
                                           int(component), ctypes.c_void_p(x.data_ptr())))
        return x

    def populations(self, lattice):
        f = np.zeros((19,) + self.shapes[lattice])
        _check(lib().lbdem_populations_get(self._h, lattice, _dp(f)))
        return f

    def set_populations(self, lattice, f):
        f = _f64(f, (19,) + self.shapes[lattice])
        _check(lib().lbdem_populations_set(self._h, lattice, _dp(f)))

    def owner(self, lattice):
        o = np.zeros(self.shapes[lattice], dtype=np.int32)
        _check(lib().lbdem_owner_get(self._h, lattice, o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return o

    def fields(self, lattice):
        """rho [nz][ny][nx], u [3][nz][ny][nx] (0 at solid nodes) and the node map, computed on
        the device from the current populations."""
        shp = self.shapes[lattice]
        rho, u = np.zeros(shp), np.zeros((3,) + shp)
        o = np.zeros(shp, dtype=np.int32)
        _check(lib().lbdem_fields_get(self._h, lattice, _dp(rho), _dp(u),
                                      o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return rho, u, o

    def state_save(self):
        """Checkpoint of the whole set as a bytes object."""
        n = ctypes.c_size_t()
        _check(lib().lbdem_state_size(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        used = ctypes.c_size_t()
        _check(lib().lbdem_state_save(self._h, buf, n.value, ctypes.byref(used)))
        return buf.raw[: used.value]

    def state_load(self, data, n_particles=None):
        """Restore the set from a checkpoint made by state_save on a set with the same
        parameters; n_particles (per lattice) restores the binding's particle counts."""
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check(lib().lbdem_state_load(self._h, buf, len(data)))
        if n_particles is not None:
            self.n_particles = list(n_particles)

    def timing_enable(self, on=True):
        _check(lib().lbdem_timing_enable(self._h, 1 if on else 0))

    def timing_read(self):
        """Summed milliseconds and launch counts of the kernels: links, motion, fluid, remap,
        refresh."""
        ms = np.zeros(5)
        cnt = np.zeros(5, dtype=np.int64)
        _check(lib().lbdem_timing_read(self._h, _dp(ms), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return ms, cnt

    def tile_info(self, lattice=0):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbdem_tile_info(self._h, lattice, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value


class AdjointWindow:
    """Adjoint of ``nsteps`` fluid steps of one lattice of a set over its current (frozen)
    particle geometry, with checkpoints every ``ckpt_every`` steps (C ABI lbdem_adj_*).

    forward(tau, amp, v) returns the probe signals [nsteps][n_probe] (plane averages of
    rho - rho_f); backward(dL_dP) returns (dL/dtau, dL/dA, dL/dV [n][3]) for the last
    forward.  The set must not be stepped while the window is in use."""

    def __init__(self, lset, lattice=0, nsteps=2000, ckpt_every=100):
        import torch

        self._set = lset
        self.nsteps = int(nsteps)
        self.n_probe = lset.n_probe[lattice]
        self.n_particles = lset.n_particles[lattice]
        nbytes = ctypes.c_size_t()
        _check(lib().lbdem_adj_workspace_size(lset._h, lattice, self.nsteps, int(ckpt_every), ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=lset.device)
        h = ctypes.c_void_p()
        _check(lib().lbdem_adj_create(lset._h, lattice, self.nsteps, int(ckpt_every), ctypes.c_void_p(self._ws.data_ptr()),
                                      nbytes.value, ctypes.byref(h)))
        self._h = h
        self.generation = 0

    def forward(self, tau, amp, v=None):
        out = np.zeros((self.nsteps, max(self.n_probe, 1)))
        vv = None if v is None else _f64(v, (self.n_particles, 3))
        _check(lib().lbdem_adj_forward(self._h, float(tau), float(amp), _dp(vv), _dp(out)))
        self.generation += 1
        return out[:, : self.n_probe]

    def backward(self, dL_dP):
        g = _f64(dL_dP, (self.nsteps, self.n_probe))
        gt, ga = ctypes.c_double(), ctypes.c_double()
        gv = np.zeros((max(self.n_particles, 1), 3))
        _check(lib().lbdem_adj_backward(self._h, _dp(g), ctypes.byref(gt), ctypes.byref(ga), _dp(gv)))
        return gt.value, ga.value, gv[: self.n_particles]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lbdem_adj_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def biot_velocities(k_dry, g_dry, phi, k_p, k_f, rho_p, rho_f, r=0.5):
    """Biot's fast and slow P-wave and S-wave speeds of a saturated packing (Eqs. vp, vs)."""
    out = np.zeros(3)
    _check(lib().lbdem_biot_velocities(float(k_dry), float(g_dry), float(phi), float(k_p), float(k_f),
                                       float(rho_p), float(rho_f), float(r), _dp(out)))
    return float(out[0]), float(out[1]), float(out[2])


def _probe_function():
    import torch

    class ProbeSignals(torch.autograd.Function):
        """Probe signals of an AdjointWindow as a differentiable function of (tau, A, V);
        the backward pass is the window's discrete adjoint (checkpointed)."""

        @staticmethod
        def forward(ctx, tau, amp, v, window):
            P = window.forward(float(tau), float(amp), v.detach().cpu().numpy())
            ctx.window = window
            ctx.generation = window.generation
            return torch.from_numpy(P).to(torch.float64)

        @staticmethod
        def backward(ctx, grad_P):
            w = ctx.window
            if w.generation != ctx.generation:
                raise RuntimeError("the adjoint window ran another forward since this one")
            gt, ga, gv = w.backward(grad_P.detach().cpu().numpy())
            return (torch.tensor(gt, dtype=torch.float64), torch.tensor(ga, dtype=torch.float64),
                    torch.from_numpy(gv).to(torch.float64), None)

    return ProbeSignals


def probe_signals(window, tau, amp, v):
    """Differentiable probe signals [nsteps][n_probe] for float64 tensors tau, amp (scalars)
    and v [n][3]."""
    return _probe_function().apply(tau, amp, v, window)


# ---------------------------------------------------------------------------
# dispersion analysis of probe records (Sec. 3.2)
# ---------------------------------------------------------------------------
def _analysis_args(x, zpos):
    import torch

    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.dim() == 2):
        raise TypeError("x must be a 2-D float64 CUDA tensor [nt, nz]")
    x = x.contiguous()
    zpos = torch.as_tensor(zpos, dtype=torch.float64, device=x.device).contiguous()
    if zpos.numel() != x.shape[1]:
        raise ValueError("zpos must hold one position per column of x")
    return torch, x, zpos


def _workspace(torch, nt, nz, nw, nk, device):
    nb = ctypes.c_size_t()
    _check(lib().lbdem_dft_workspace_size(int(nt), int(nz), int(nw), int(nk), ctypes.byref(nb)))
    return torch.empty(max(nb.value, 256), dtype=torch.uint8, device=device), nb.value


def st_dft(x, zpos, t0, w0, dw, nw, k0, dk, nk, ridge=True, work=None):
    """Space-time DFT of the record x[t][z] (float64 CUDA tensor), row t at time t0 + t:
    F[m][n] = sum_t sum_z x[t][z] exp(-j (omega_m (t0 + t) - kappa_n zpos[z])) with
    omega_m = w0 + m dw and kappa_n = k0 + n dk.  Returns the complex128 tensor F [nw][nk]
    and, with ridge=True, the int32 tensor of the wavenumber index of each row's maximum."""
    torch, x, zpos = _analysis_args(x, zpos)
    nt, nz = x.shape
    if work is None:
        work, nb = _workspace(torch, nt, nz, nw, nk, x.device)
    else:
        nb = work.numel() * work.element_size()
    F = torch.empty((nw, nk, 2), dtype=torch.float64, device=x.device)
    r = torch.empty(nw, dtype=torch.int32, device=x.device) if ridge else None
    st = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib().lbdem_st_dft(ctypes.c_void_p(x.data_ptr()), int(nt), int(nz), ctypes.c_void_p(zpos.data_ptr()),
                              float(t0), float(w0), float(dw), int(nw), float(k0), float(dk), int(nk),
                              ctypes.c_void_p(F.data_ptr()), None if r is None else ctypes.c_void_p(r.data_ptr()),
                              ctypes.c_void_p(work.data_ptr()), nb, ctypes.c_void_p(st)))
    F = torch.view_as_complex(F)
    return (F, r) if ridge else F


def wave_fit(x, zpos, t0, omega):
    """Fit of Eq. (1Dwave) to the stationary record x[t][z] at the inserted frequency omega.
    Returns dict(A=complex, alpha=alpha_s, k=k, c=omega / k, n_used=columns used)."""
    torch, x, zpos = _analysis_args(x, zpos)
    nt, nz = x.shape
    work, nb = _workspace(torch, nt, nz, 1, 1, x.device)
    out = torch.empty(6, dtype=torch.float64, device=x.device)
    st = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib().lbdem_wave_fit(ctypes.c_void_p(x.data_ptr()), int(nt), int(nz), ctypes.c_void_p(zpos.data_ptr()),
                                float(t0), float(omega), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(work.data_ptr()), nb, ctypes.c_void_p(st)))
    o = out.cpu().numpy()
    return {"A": complex(o[0], o[1]), "alpha": float(o[2]), "k": float(o[3]), "c": float(o[4]), "n_used": int(o[5])}


def wave_fit_noalloc(x, zpos, t0, omega, out=None):
    """wave_fit through the allocation-free entry point (static device scratch).  ``out``:
    an optional float64 CUDA tensor of 6 values to write into; returns it."""
    torch, x, zpos = _analysis_args(x, zpos)
    nt, nz = x.shape
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=x.device)
    st = torch.cuda.current_stream(x.device).cuda_stream
    _check(lib().lbdem_wave_fit_noalloc(ctypes.c_void_p(x.data_ptr()), int(nt), int(nz),
                                        ctypes.c_void_p(zpos.data_ptr()), float(t0), float(omega),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st)))
    return out
