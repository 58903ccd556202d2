"""Pins of the oracle's adjoint of the frozen-geometry fluid step.

The oracle's reverse sweep (collision Jacobian, density-face transpose, streaming
transpose, moving-wall term) is checked against central finite differences of the
oracle's own forward map, an independent computation: only forward steps are taken.
The loss is the L2 misfit of the plane-averaged density probes against a seeded target.
"""
import numpy as np
import pytest

import oracle

N_STEPS = 30


def _sim(tau=1.0, amp=1e-3, v=None, w=None):
    s = oracle.Sim(8, 9, 20, tau=tau, bc=(1, 1, 0, 0, 2, 2), wave=oracle.WAVE_COSINE, amp=amp,
                   omega=2 * np.pi / 16, t_n=16, probe_z=(3, 9, 14))
    x = np.array([[3.4, 4.6, 8.2], [4.5, 4.1, 13.4]])
    s.set_particles(x, np.array([2.4, 2.1]))
    s.set_frozen(True)
    s.set_velocities(v, w)
    return s


V0 = np.array([[1e-3, -2e-3, 5e-4], [-1e-3, 1.5e-3, 2e-3]])
W0 = np.array([[0.0, 2e-4, -1e-4], [3e-4, 0.0, 1e-4]])
TARGET = np.random.default_rng(7).normal(0.0, 1e-4, (N_STEPS, 3))


def _loss(tau=1.0, amp=1e-3, v=V0):
    s = _sim(tau, amp, v, W0)
    P, *_ = s.adjoint(N_STEPS, tau, amp, np.zeros((N_STEPS, 3)))
    s.close()
    return float(((P - TARGET) ** 2).sum()), P


@pytest.fixture(scope="module")
def adjoint_result():
    _, P = _loss()
    s = _sim(1.0, 1e-3, V0, W0)
    out = s.adjoint(N_STEPS, 1.0, 1e-3, 2.0 * (P - TARGET))
    s.close()
    return out


def test_forward_of_adjoint_matches_frozen_steps():
    # the probes recorded by the adjoint's forward are those of ordinary frozen steps
    s = _sim(1.0, 1e-3, V0, W0)
    s.step(N_STEPS)
    pr = s.probes(0, N_STEPS)
    s.close()
    _, P = _loss()
    assert np.allclose(P, pr[:, :, 1] / pr[:, :, 0], rtol=0, atol=1e-15)


def test_adjoint_tau_and_amplitude_vs_central_differences(adjoint_result):
    _, g_tau, g_amp, _ = adjoint_result
    h = 1e-5
    fd_tau = (_loss(tau=1.0 + h)[0] - _loss(tau=1.0 - h)[0]) / (2 * h)
    ha = 1e-8
    fd_amp = (_loss(amp=1e-3 + ha)[0] - _loss(amp=1e-3 - ha)[0]) / (2 * ha)
    assert abs(g_tau - fd_tau) <= 1e-6 * abs(fd_tau)
    assert abs(g_amp - fd_amp) <= 1e-6 * abs(fd_amp)


@pytest.mark.parametrize("q,a", [(0, 0), (0, 2), (1, 1), (1, 2)])
def test_adjoint_particle_velocity_vs_central_differences(adjoint_result, q, a):
    g_v = adjoint_result[3]
    h = 1e-6
    vp, vm = V0.copy(), V0.copy()
    vp[q, a] += h
    vm[q, a] -= h
    fd = (_loss(v=vp)[0] - _loss(v=vm)[0]) / (2 * h)
    assert abs(g_v[q, a] - fd) <= 1e-6 * abs(fd)
