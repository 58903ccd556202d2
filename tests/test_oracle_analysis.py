"""Pins of the oracle's dispersion analysis (Sec. 3.2: Eq. (1Dwave) fit and the space-time DFT).

The transform is checked against numpy's FFT on its own bins and against a brute-force
double loop; the fit against signals built from known parameters, where a whole number of
periods makes the harmonic amplitude exact; and the whole chain against the paper's
printed pure-fluid values on an oracle run of the first benchmark.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1808_08921_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def an():
    from oracle import analysis
    return analysis


def test_dft_on_fft_bins_equals_numpy_fft(an):
    rng = np.random.default_rng(3)
    nt, nz = 48, 20
    x = rng.standard_normal((nt, nz))
    om = 2 * np.pi * np.arange(nt) / nt
    ka = 2 * np.pi * np.arange(nz) / nz
    F = an.space_time_dft(x, 0, np.arange(nz), om, ka)
    # exp(-j w t) over t is the forward FFT; exp(+j k z) over z is nz times the inverse FFT
    want = np.fft.fft(np.fft.ifft(x, axis=1) * nz, axis=0)
    assert np.abs(F - want).max() < 1e-11 * np.abs(x).sum()


def test_dft_brute_force_on_a_tiny_grid(an):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 2))
    zpos = [0.5, 2.25]
    om = [0.1, -0.7, 1.3]
    ka = [0.0, 0.4]
    t0 = 17.0
    F = an.space_time_dft(x, t0, zpos, om, ka)
    for m in range(3):
        for n in range(2):
            acc = 0j
            for t in range(3):
                for z in range(2):
                    ang = om[m] * (t0 + t) - ka[n] * zpos[z]
                    acc += x[t, z] * complex(math.cos(ang), -math.sin(ang))
            assert F[m, n] == pytest.approx(acc, abs=1e-14)


@pytest.mark.parametrize("k", [0.05, 1.1])
def test_fit_recovers_a_known_wave(an, k):
    """Four whole periods: the harmonic amplitude is exact, also with an offset and a
    second harmonic; k = 1.1 turns the phase by more than pi between probes (unwrap)."""
    om = 2 * np.pi / 50
    zpos = np.array([0.0, 1.5, 3.0, 4.0, 6.5, 8.0, 9.0, 11.5])
    A = 0.3 - 0.8j
    x = inputs.probe_signal(200, zpos, om, A, 0.04, k, t0=11.0, offset=0.2, harmonic=0.3)
    A_f, al, k_f, c = an.wave_fit(x, 11.0, zpos, om)
    assert A_f == pytest.approx(A, abs=1e-12)
    assert al == pytest.approx(0.04, abs=1e-12)
    assert k_f == pytest.approx(k, abs=1e-12)
    assert c == pytest.approx(om / k, rel=1e-12)


def test_ridge_peaks_at_the_wavenumber(an):
    """|sum_z exp(-(alpha + j (k - kappa)) z)| is largest at kappa = k (all terms in phase),
    so on a fine grid the ridge sits at the grid point next to k."""
    om = 2 * np.pi / 40
    zpos = np.arange(0, 64, 2.0)
    k = 0.0937
    x = inputs.probe_signal(160, zpos, om, 1.0, 0.01, k)
    ka = np.linspace(0.0, 0.3, 3001)
    F = an.space_time_dft(x, 0, zpos, [om], ka)
    assert abs(ka[an.ridge(F)[0]] - k) <= 0.5001e-4
    assert an.branch_speed([om], ka, F)[0] == pytest.approx(om / k, rel=2e-3)


def test_ridge_takes_the_first_of_equal_values(an):
    F = np.array([[1.0, 2.0, -2.0, 2j], [0.0, 0.0, 0.0, 0.0]])
    assert list(an.ridge(F)) == [1, 0]


def test_absorption_closed_form_matches_printed_value(an):
    g = _golden()["pure_fluid_wave"]
    a = an.lossy_alpha(g["omega"], _golden()["sound_speed"]["value"], g["tau"])
    assert a == pytest.approx(g["alpha_s"], rel=1e-3)


def test_pure_fluid_fit_matches_paper(orc, an):
    """First benchmark of Sec. 3.2 (tau = 1, omega = 0.03, rho' = 1e-4), 64 probe planes at
    x3 = 1 + 7 i of a 1 x 1 x 1200 column (a uniform cross-section, so the same flow as
    12 x 12), five periods once the wave is stationary and before the outlet's echo."""
    g = _golden()["pure_fluid_wave"]
    cs = _golden()["sound_speed"]["value"]
    fit = _golden()["pure_fluid_fit"]
    zs = tuple(1 + 7 * i for i in range(64))
    s = orc.Sim(1, 1, 1200, tau=g["tau"], bc=(0, 0, 0, 0, 2, 2), wave=orc.WAVE_SINE, amp=g["rho_amp"],
                omega=g["omega"], t_n=10 ** 9, probe_z=zs)
    s.step(2300)
    pr = s.probes()
    n = int(round(5 * 2 * math.pi / g["omega"]))
    first = 1200
    x = pr[first:first + n, :, 1] / pr[first:first + n, :, 0] / g["rho_amp"]
    # the record of step i holds time level i + 1
    A, al, k, c = an.wave_fit(x, first + 1, np.array(zs, float), g["omega"])
    assert al == pytest.approx(g["alpha_s"], rel=0.01)
    assert c == pytest.approx(cs, rel=2e-3)
    assert abs(A - complex(fit["A_re"], fit["A_im"])) < 0.03
    ka = np.linspace(0.0, 0.2, 2001)
    F = an.space_time_dft(x, first + 1, np.array(zs, float), [g["omega"]], ka)
    assert an.branch_speed([g["omega"]], ka, F)[0] == pytest.approx(cs, rel=3e-3)


@pytest.mark.parametrize("f_mhz,rel_alpha,rel_c", [(1.30, 0.005, 0.002), (3.25, 0.005, 0.002),
                                                   (6.50, 0.01, 0.004), (13.0, 0.02, 0.01)])
def test_frequency_sweep_follows_the_lossy_wave(orc, an, f_mhz, rel_alpha, rel_c):
    """The input frequencies of Table tab:source (continuous sine source, rho' = 2e-4) in the
    pure fluid: the fitted absorption and speed follow the closed form of Eq. (1Dwave) with
    tau_s = tau = 1 and c_s = 1/sqrt(3); the lattice's own dispersion grows with frequency
    (1.3 % in alpha_s and 0.85 % in c_s at 13 MHz, a wavelength of 29 nodes)."""
    cs = _golden()["sound_speed"]["value"]
    om = inputs.source_omega(f_mhz)
    zs = tuple(1 + 7 * i for i in range(64))
    s = orc.Sim(1, 1, 1400, tau=1.0, bc=(0, 0, 0, 0, 2, 2), wave=orc.WAVE_SINE, amp=inputs.SOURCE_AMP, omega=om,
                t_n=100000, probe_z=zs)
    s.step(3200)
    pr = s.probes()
    first, n = 1200, 1998
    x = pr[first:first + n, :, 1] / pr[first:first + n, :, 0] / inputs.SOURCE_AMP
    A, al, k, c = an.wave_fit(x, first + 1, np.array(zs, float), om)
    assert al == pytest.approx(an.lossy_alpha(om, cs, 1.0), rel=rel_alpha)
    assert c == pytest.approx(cs, rel=rel_c)
    assert abs(A - (-1j)) < 0.01


# ---------------------------------------------------------------------------
# Biot's wave velocities (Sec. "Biot's equations ...", Eqs. vp, vs)
# ---------------------------------------------------------------------------
_BIOT_CASES = [
    # k_dry, g_dry, phi, k_p, k_f, rho_p, rho_f (lattice units: the FCC packing's porosity,
    # E* = 10.37 and nu = 0.2 give k_p = E / (3 (1 - 2 nu)), k_f = rho_f c_s^2 = 1/3)
    (0.05, 0.04, 0.266, 10.37 / 1.8, 1.0 / 3.0, 2.466, 1.0),
    (0.5, 0.35, 0.266, 10.37 / 1.8, 1.0 / 3.0, 2.466, 1.0),
    (2.0, 1.5, 0.40, 12.0, 2.25, 2.65, 1.0),
]


@pytest.mark.parametrize("case", _BIOT_CASES)
def test_biot_velocities_solve_the_characteristic_equation(an, case):
    """The fast and slow P-wave speeds of Eq. (vp) are the two roots of
    det(rho v^2 - E) = 0 with E = [[P, Q], [Q, R]] and the mass matrix [[rho11, rho12],
    [rho12, rho22]]: generalized eigenvalues computed by numpy (this fixes the printed
    denominator's reading, rho11 rho22 - rho12^2).  The S-wave speed of Eq. (vs) is the
    nonzero root of the shear problem det(rho v^2 - diag(G_dry, 0)) = 0, G_dry / (rho11 -
    rho12^2 / rho22)."""
    k_dry, g_dry, phi, k_p, k_f, rho_p, rho_f = case
    vf, vsl, vs = an.biot_velocities(*case)
    P, Q, R = an.biot_moduli(k_dry, g_dry, phi, k_p, k_f)
    alpha = 1.0 - 0.5 * (1.0 - 1.0 / phi)
    rho12 = (1.0 - alpha) * phi * rho_f
    rho11 = (1.0 - phi) * rho_p - rho12
    rho22 = alpha * phi * rho_f
    M = np.array([[rho11, rho12], [rho12, rho22]])
    E = np.array([[P, Q], [Q, R]])
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(M, E)).real)
    assert vsl ** 2 == pytest.approx(ev[0], rel=1e-12)
    assert vf ** 2 == pytest.approx(ev[1], rel=1e-12)
    assert vs ** 2 == pytest.approx(g_dry / (rho11 - rho12 ** 2 / rho22), rel=1e-12)
    assert vf > vsl > 0.0 and vs > 0.0


@pytest.mark.parametrize("case", _BIOT_CASES)
def test_biot_moduli_give_gassmanns_undrained_modulus(an, case):
    """P + 2Q + R - (4/3) G_dry is the undrained bulk modulus of the saturated packing,
    which Gassmann's relation gives independently: K_dry + (1 - K_dry/K_p)^2 /
    (phi/K_f + (1 - phi)/K_p - K_dry/K_p^2)."""
    k_dry, g_dry, phi, k_p, k_f, rho_p, rho_f = case
    P, Q, R = an.biot_moduli(k_dry, g_dry, phi, k_p, k_f)
    k_sat = k_dry + (1.0 - k_dry / k_p) ** 2 / (phi / k_f + (1.0 - phi) / k_p - k_dry / k_p ** 2)
    assert P + 2.0 * Q + R - 4.0 / 3.0 * g_dry == pytest.approx(k_sat, rel=1e-12)
