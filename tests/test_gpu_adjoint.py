"""GPU adjoint window (C ABI lbdem_adj_*) against the FP64 oracle's adjoint and against
central finite differences of the GPU forward map.

Bar: forward probes of the frozen-geometry window within 1e-10 (relative to the signal
scale) of the oracle's frozen steps; FP64 gradients within 1e-9 of the oracle adjoint and
within 1e-6 of central differences (h = 1e-4 relative); FP32 gradients within 2 % of the
FP64 ones; the torch autograd Function returns the window's vector-Jacobian product.
"""
import numpy as np
import pytest

import oracle
from paper_1808_08921_amd import inputs

pytestmark = pytest.mark.gpu

N_STEPS = 30
PARAMS = dict(nx=8, ny=9, nz=20, tau=1.0, rho_f=1.0, bc=(1, 1, 0, 0, 2, 2), wave=inputs.WAVE_COSINE, amp=1e-3,
              omega=2 * np.pi / 16, t_n=16, probe_z=(3, 9, 14), max_particles=2, max_radius=3.0)
X = np.array([[3.4, 4.6, 8.2], [4.5, 4.1, 13.4]])
RAD = np.array([2.4, 2.1])
V0 = np.array([[1e-3, -2e-3, 5e-4], [-1e-3, 1.5e-3, 2e-3]])
W0 = np.array([[0.0, 2e-4, -1e-4], [3e-4, 0.0, 1e-4]])
TARGET = np.random.default_rng(7).normal(0.0, 1e-4, (N_STEPS, 3))


def _window(precision, ckpt=7):
    from paper_1808_08921_amd.lbdem import AdjointWindow, LatticeSet

    gs = LatticeSet([PARAMS], precision=precision, graph_steps=0)
    gs.particles_set(0, X, RAD, v=V0, w=W0)
    return gs, AdjointWindow(gs, 0, nsteps=N_STEPS, ckpt_every=ckpt)


@pytest.fixture(scope="module")
def oracle_result():
    p = PARAMS
    s = oracle.Sim(p["nx"], p["ny"], p["nz"], tau=p["tau"], bc=p["bc"], wave=p["wave"], amp=p["amp"],
                   omega=p["omega"], t_n=p["t_n"], probe_z=p["probe_z"])
    s.set_particles(X, RAD, v=V0, w=W0)
    s.set_frozen(True)
    P, *_ = s.adjoint(N_STEPS, 1.0, 1e-3, np.zeros((N_STEPS, 3)))
    s.close()
    s = oracle.Sim(p["nx"], p["ny"], p["nz"], tau=p["tau"], bc=p["bc"], wave=p["wave"], amp=p["amp"],
                   omega=p["omega"], t_n=p["t_n"], probe_z=p["probe_z"])
    s.set_particles(X, RAD, v=V0, w=W0)
    s.set_frozen(True)
    out = s.adjoint(N_STEPS, 1.0, 1e-3, 2.0 * (P - TARGET))
    s.close()
    return out


@pytest.fixture(scope="module")
def fp64_window():
    gs, win = _window("fp64")
    yield win
    win.close()
    gs.close()


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_forward_matches_oracle(fp64_window, oracle_result):
    P = fp64_window.forward(1.0, 1e-3, V0)
    assert _rel(P, oracle_result[0]) <= 1e-10


def test_gradients_match_oracle(fp64_window, oracle_result):
    P = fp64_window.forward(1.0, 1e-3, V0)
    gt, ga, gv = fp64_window.backward(2.0 * (P - TARGET))
    _, ot, oa, ov = oracle_result
    assert abs(gt - ot) <= 1e-9 * abs(ot)
    assert abs(ga - oa) <= 1e-9 * abs(oa)
    assert _rel(gv, ov) <= 1e-9


def _loss(win, tau=1.0, amp=1e-3, v=V0):
    P = win.forward(tau, amp, v)
    return float(((P - TARGET) ** 2).sum())


def test_gradients_match_central_differences(fp64_window):
    P = fp64_window.forward(1.0, 1e-3, V0)
    gt, ga, gv = fp64_window.backward(2.0 * (P - TARGET))
    h = 1e-4
    fd_t = (_loss(fp64_window, tau=1.0 + h) - _loss(fp64_window, tau=1.0 - h)) / (2 * h)
    fd_a = (_loss(fp64_window, amp=1e-3 * (1 + h)) - _loss(fp64_window, amp=1e-3 * (1 - h))) / (2e-3 * h)
    assert abs(gt - fd_t) <= 1e-6 * abs(fd_t)
    assert abs(ga - fd_a) <= 1e-6 * abs(fd_a)
    for q, a in [(0, 2), (1, 1)]:
        vp, vm = V0.copy(), V0.copy()
        vp[q, a] += 1e-4 * abs(V0[q, a])
        vm[q, a] -= 1e-4 * abs(V0[q, a])
        fd = (_loss(fp64_window, v=vp) - _loss(fp64_window, v=vm)) / (2e-4 * abs(V0[q, a]))
        assert abs(gv[q, a] - fd) <= 1e-6 * abs(fd)


def test_checkpoint_interval_does_not_change_gradients(fp64_window):
    P = fp64_window.forward(1.0, 1e-3, V0)
    ref = fp64_window.backward(2.0 * (P - TARGET))
    for ck in (1, 30):
        gs, win = _window("fp64", ckpt=ck)
        P2 = win.forward(1.0, 1e-3, V0)
        out = win.backward(2.0 * (P2 - TARGET))
        win.close()
        gs.close()
        assert np.array_equal(P, P2)
        assert out[0] == ref[0] and out[1] == ref[1] and np.array_equal(out[2], ref[2])


def test_fp32_gradients_track_fp64(fp64_window):
    P = fp64_window.forward(1.0, 1e-3, V0)
    gt, ga, gv = fp64_window.backward(2.0 * (P - TARGET))
    gs, win = _window("fp32")
    P32 = win.forward(1.0, 1e-3, V0)
    g32 = win.backward(2.0 * (P32 - TARGET))
    win.close()
    gs.close()
    assert _rel(P32, P) <= 1e-4
    assert abs(g32[0] - gt) <= 2e-2 * abs(gt)
    assert abs(g32[1] - ga) <= 2e-2 * abs(ga)
    assert _rel(g32[2], gv) <= 2e-2


def test_autograd_function(fp64_window):
    import torch
    from paper_1808_08921_amd.lbdem import probe_signals

    tau = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    amp = torch.tensor(1e-3, dtype=torch.float64, requires_grad=True)
    v = torch.tensor(V0, dtype=torch.float64, requires_grad=True)
    P = probe_signals(fp64_window, tau, amp, v)
    loss = ((P - torch.from_numpy(TARGET)) ** 2).sum()
    loss.backward()
    gt, ga, gv = fp64_window.backward(2.0 * (P.detach().numpy() - TARGET))
    assert tau.grad.item() == gt and amp.grad.item() == ga
    assert np.array_equal(v.grad.numpy(), gv)
