"""Test infrastructure only: plain FP64 reference of the dispersion analysis of probe records.

Cheng et al. (arXiv 1808.08921), Sec. 3.2: the cross-section averaged density signal
rho'(t, x3) is described by the stationary solution of the one-dimensional lossy wave
equation, Eq. (1Dwave), rho' = A exp(-alpha_s x) exp(j (omega t - k x)), and the
dispersion relation is read from the discrete Fourier transform of the space-time data:
the wavenumber at which the spectrum peaks for the inserted frequency gives the sound
speed c_s = omega / k.  Only the tests, the package smoke check and the CPU-baseline leg
of the benchmark may import this module; the GPU library never uses it.

Readings (the paper does not spell these out):
- the space-time transform uses the sign pair of Eq. (1Dwave), exp(-j (omega t - kappa x)),
  so a wave running towards +x3 peaks at positive omega and positive kappa;
- the Eq. (1Dwave) fit takes, at every probe plane, the complex amplitude of the signal at
  the inserted frequency over a window of whole periods, P(x) = (2 / n_t) sum_t rho'(t, x)
  exp(-j omega t) (= A exp(-(alpha_s + j k) x) for a stationary wave), and fits a straight
  line by least squares to log |P| and to the unwrapped phase of P against x: the slopes
  are -alpha_s and -k, the intercepts log |A| and arg A.
"""
from __future__ import annotations

import numpy as np


def space_time_dft(x, t0, zpos, omegas, kappas):
    """F[m, n] = sum_t sum_z x[t, z] exp(-j (omega_m (t0 + t) - kappa_n zpos[z])).

    x: real [n_t, n_z] signal, row t taken at time t0 + t; zpos: [n_z] positions along x3;
    omegas [n_w], kappas [n_k]: the frequencies and wavenumbers to evaluate (any grid).
    The double sum is written as two products with the time and space phase matrices.
    """
    x = np.asarray(x, dtype=np.float64)
    t = t0 + np.arange(x.shape[0], dtype=np.float64)
    e_t = np.exp(-1j * np.outer(np.asarray(omegas, np.float64), t))              # [n_w, n_t]
    e_z = np.exp(1j * np.outer(np.asarray(zpos, np.float64), np.asarray(kappas, np.float64)))  # [n_z, n_k]
    return (e_t @ x) @ e_z


def ridge(F):
    """For every frequency row, the index of the wavenumber with the largest
    |F|^2 = re^2 + im^2 (the first one among equal values)."""
    F = np.asarray(F)
    a = F.real ** 2 + F.imag ** 2
    return np.argmax(a, axis=1)


def branch_speed(omegas, kappas, F):
    """Sound speed of the branch through each frequency row: omega_m / kappa at the ridge."""
    r = ridge(F)
    return np.asarray(omegas, np.float64) / np.asarray(kappas, np.float64)[r]


def harmonic_amplitudes(x, t0, omega):
    """P[z] = (2 / n_t) sum_t x[t, z] exp(-j omega (t0 + t)): the complex amplitude at omega."""
    x = np.asarray(x, dtype=np.float64)
    n_t = x.shape[0]
    t = t0 + np.arange(n_t, dtype=np.float64)
    return (2.0 / n_t) * (np.exp(-1j * omega * t) @ x)


def wave_fit(x, t0, zpos, omega):
    """Fit of Eq. (1Dwave) to the stationary signal x[t, z] at the inserted frequency omega.

    Returns (A, alpha_s, k, c_s) with c_s = omega / k.  Columns whose amplitude is exactly
    zero (a probe plane without fluid nodes records 0) carry no phase and are left out.
    """
    P = harmonic_amplitudes(x, t0, omega)
    z = np.asarray(zpos, np.float64)
    keep = P != 0
    P, z = P[keep], z[keep]
    mag = np.log(np.abs(P))
    ph = np.unwrap(np.angle(P))
    s_mag, i_mag = np.polyfit(z, mag, 1)
    s_ph, i_ph = np.polyfit(z, ph, 1)
    alpha = -s_mag
    k = -s_ph
    A = np.exp(i_mag + 1j * i_ph)
    return A, alpha, k, omega / k


def lossy_alpha(omega, c_s, tau_s):
    """Spatial absorption coefficient of Eq. (1Dwave) for sound speed c_s and relaxation time tau_s."""
    q = np.sqrt(1.0 + (omega * tau_s) ** 2)
    return omega / (c_s * np.sqrt(2.0)) * np.sqrt((q - 1.0) / q)


def biot_velocities(k_dry, g_dry, phi, k_p, k_f, rho_p, rho_f, r=0.5):
    """Wave velocities of a saturated poroelastic packing from Biot's theory (Sec. "Biot's
    equations of wave velocities in saturated poroelastic media", Eqs. vp and vs): the fast
    and slow P-waves and the S-wave, from the dry packing's moduli k_dry, g_dry, the
    porosity phi, the particles' and the fluid's bulk moduli k_p, k_f and densities rho_p,
    rho_f, with the tortuosity alpha = 1 - r (1 - 1/phi).

    Reading: the denominator of Eq. (vp) is 2 (rho_11 rho_22 - rho_12^2), the discriminant
    of the quadratic det(rho v^2 - E) = 0 that Eq. (vp) solves (the printed rho_12 rho_22 is
    taken as a typo).  Returns (v_fast, v_slow, v_s)."""
    alpha = 1.0 - r * (1.0 - 1.0 / phi)
    rho11 = (1.0 - phi) * rho_p - (1.0 - alpha) * phi * rho_f
    rho22 = alpha * phi * rho_f
    rho12 = (1.0 - alpha) * phi * rho_f
    rho_hat = (1.0 - phi) * rho_p + phi * rho_f
    den = 1.0 - phi - k_dry / k_p + phi * k_p / k_f
    P = ((1.0 - phi) * (1.0 - phi - k_dry / k_p) * k_p + phi * k_p * k_dry / k_f) / den + 4.0 / 3.0 * g_dry
    Q = (1.0 - phi - k_dry / k_p) * phi * k_p / den
    R = phi * phi * k_p / den
    delta = P * rho22 + R * rho11 - 2.0 * Q * rho12
    disc = np.sqrt(delta * delta - 4.0 * (rho11 * rho22 - rho12 * rho12) * (P * R - Q * Q))
    two_d = 2.0 * (rho11 * rho22 - rho12 * rho12)
    v_fast = np.sqrt((delta + disc) / two_d)
    v_slow = np.sqrt((delta - disc) / two_d)
    v_s = np.sqrt(g_dry / (rho_hat - phi * rho_f / alpha))
    return float(v_fast), float(v_slow), float(v_s)


def biot_moduli(k_dry, g_dry, phi, k_p, k_f):
    """Biot's elastic moduli P, Q, R of the same section (for checks)."""
    den = 1.0 - phi - k_dry / k_p + phi * k_p / k_f
    P = ((1.0 - phi) * (1.0 - phi - k_dry / k_p) * k_p + phi * k_p * k_dry / k_f) / den + 4.0 / 3.0 * g_dry
    Q = (1.0 - phi - k_dry / k_p) * phi * k_p / den
    R = phi * phi * k_p / den
    return P, Q, R
