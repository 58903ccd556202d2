"""GPU parity of the dispersion analysis (Sec. 3.2): space-time DFT, ridge and the fit of
Eq. (1Dwave), through the C interface, against the FP64 oracle on the same seeded records.

Bar: spectra within 1e-12 of the record's absolute sum (different summation orders of
the same FP64 terms); ridge indices equal wherever the oracle's largest value leads the
next by more than that error, else the GPU's pick is one of the tied values; fitted
parameters within 1e-9 relative; probe signals bit-exact against the probe records.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analysis as an
from paper_1808_08921_amd import inputs

pytestmark = pytest.mark.gpu


def _lb():
    import torch

    from paper_1808_08921_amd import lbdem

    assert torch.cuda.is_available()
    return torch, lbdem


def _grid(a0, da, n):
    return a0 + np.arange(n, dtype=np.float64) * da


def _check_ridge(Fo, r_gpu, tol):
    p = Fo.real ** 2 + Fo.imag ** 2
    r_o = an.ridge(Fo)
    for m in range(p.shape[0]):
        top = p[m, r_o[m]]
        near = np.nonzero(p[m] >= top - tol * max(top, 1e-300))[0]
        if len(near) == 1:
            assert r_gpu[m] == r_o[m], f"row {m}: ridge {r_gpu[m]} vs {r_o[m]}"
        else:
            assert r_gpu[m] in near, f"row {m}: ridge {r_gpu[m]} not among the tied {near}"


@pytest.mark.parametrize("nt,nz,nw,nk", [(1000, 13, 100, 300), (4099, 40, 64, 64), (20000, 24, 70, 33),
                                         (1, 1, 1, 1), (37, 7, 3, 257)])
def test_st_dft_matches_oracle(nt, nz, nw, nk):
    torch, lb = _lb()
    rng = np.random.default_rng(nt + nz)
    zpos = np.sort(rng.uniform(0.0, 300.0, nz))
    x = inputs.probe_signal(nt, zpos, 2 * math.pi / 97, 0.4 - 0.3j, 2e-3, 0.071, t0=5.0, offset=0.1,
                            harmonic=0.2, noise=0.05, seed=nt)
    t0, w0, dw, k0, dk = 5.0, -0.05, 0.0021, -0.02, 0.0009
    xd = torch.from_numpy(x).cuda()
    F, r = lb.st_dft(xd, zpos, t0, w0, dw, nw, k0, dk, nk)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    Fo = an.space_time_dft(x, t0, zpos, _grid(w0, dw, nw), _grid(k0, dk, nk))
    scale = np.abs(x).sum()
    err = np.abs(Fg - Fo).max() / scale
    assert err < 1e-12, f"spectrum differs by {err:.3e} of the record's sum"
    # |F|^2 error relative to the row maximum: twice the spectrum's relative error
    _check_ridge(Fo, r.cpu().numpy(), 4 * err * scale / max(np.abs(Fo).max(), 1e-300) + 1e-13)


def test_st_dft_on_fft_bins_peaks_at_the_wave():
    """Uniform probes and FFT bins: a travelling wave on bin (3, 5) gives the ridge 5 in row 3."""
    torch, lb = _lb()
    nt, nz = 256, 32
    zpos = np.arange(nz, dtype=np.float64)
    om, ka = 2 * math.pi * 3 / nt, 2 * math.pi * 5 / nz
    x = inputs.probe_signal(nt, zpos, om, 1.0, 0.0, ka)
    F, r = lb.st_dft(torch.from_numpy(x).cuda(), zpos, 0.0, 0.0, 2 * math.pi / nt, 8, 0.0, 2 * math.pi / nz, nz)
    Fg = F.cpu().numpy()
    assert int(r.cpu()[3]) == 5
    assert abs(Fg[3, 5]) == pytest.approx(nt * nz / 2, rel=1e-12)


@pytest.mark.parametrize("k,zero_col", [(0.05, None), (1.1, None), (0.3, 2)])
def test_wave_fit_matches_oracle(k, zero_col):
    torch, lb = _lb()
    om = 2 * math.pi / 50
    zpos = np.array([0.0, 1.5, 3.0, 4.0, 6.5, 8.0, 9.0, 11.5, 13.0, 14.25])
    x = inputs.probe_signal(1003, zpos, om, 0.3 - 0.8j, 0.04, k, t0=11.0, offset=0.2, harmonic=0.3, noise=0.01,
                            seed=7)
    if zero_col is not None:
        x[:, zero_col] = 0.0
    g = lb.wave_fit(torch.from_numpy(x).cuda(), zpos, 11.0, om)
    A, al, kk, c = an.wave_fit(x, 11.0, zpos, om)
    assert g["n_used"] == len(zpos) - (zero_col is not None)
    assert g["A"] == pytest.approx(A, rel=1e-9)
    assert g["alpha"] == pytest.approx(al, rel=1e-9)
    assert g["k"] == pytest.approx(kk, rel=1e-9)
    assert g["c"] == pytest.approx(c, rel=1e-9)


def test_wave_fit_with_too_few_columns_gives_nan():
    torch, lb = _lb()
    x = np.zeros((64, 3))
    x[:, 1] = np.cos(0.3 * np.arange(64))
    g = lb.wave_fit(torch.from_numpy(x).cuda(), [0.0, 1.0, 2.0], 0.0, 0.3)
    assert g["n_used"] == 1 and math.isnan(g["alpha"]) and math.isnan(g["c"])


def test_analysis_argument_errors():
    torch, lb = _lb()
    x = torch.zeros((10, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(lb.LbdemError):
        lb.st_dft(x, [0.0, 1.0, 2.0, 3.0], 0.0, 0.0, 0.1, 0, 0.0, 0.1, 4)
    with pytest.raises(lb.LbdemError):
        lb.wave_fit(x, [0.0, 1.0, 2.0, 3.0], 0.0, 0.0)
    with pytest.raises(lb.LbdemError):
        lb.st_dft(x, [0.0, 1.0, 2.0, 3.0], 0.0, 0.0, 0.1, 4, 0.0, 0.1, 4,
                  work=torch.empty(256, dtype=torch.uint8, device="cuda"))


def test_pure_fluid_wave_end_to_end():
    """First benchmark of Sec. 3.2 on the GPU path (FP64): a 12 x 12 x 1200 column with periodic
    sides, 64 probe planes at x3 = 1 + 7 i; probe signals gathered on the device, then the
    fit and the space-time DFT.  Parity with the oracle's run of the same flow (a 1 x 1
    column: the cross-section is uniform), and the paper's printed values."""
    import json
    import os

    torch, lb = _lb()
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as fh:
        gold = json.load(fh)
    g = gold["pure_fluid_wave"]
    cs = gold["sound_speed"]["value"]
    zs = tuple(1 + 7 * i for i in range(64))
    params = dict(nx=12, ny=12, nz=1200, tau=g["tau"], bc=(0, 0, 0, 0, 2, 2), wave=inputs.WAVE_SINE,
                  amp=g["rho_amp"], omega=g["omega"], t_n=100000, probe_z=zs)
    n = int(round(5 * 2 * math.pi / g["omega"]))
    first = 1200
    with lb.LatticeSet([params], precision="fp64", probe_ring=4096) as gs:
        gs.step(2300)
        sig = gs.probe_signal(0, first, n)
        torch.cuda.synchronize()
        pr = gs.probes(0, first, n)
    assert np.array_equal(sig.cpu().numpy(), pr[:, :, 1] / pr[:, :, 0])
    zpos = np.array(zs, dtype=np.float64)
    x = sig / g["rho_amp"]
    fit = lb.wave_fit(x, zpos, first + 1, g["omega"])
    ka0, dka, nk = 0.0, 1e-4, 2001
    F, r = lb.st_dft(x, zpos, first + 1, g["omega"], 0.0, 1, ka0, dka, nk)
    c_ridge = g["omega"] / (ka0 + int(r.cpu()[0]) * dka)

    s = oracle.Sim(1, 1, 1200, tau=g["tau"], bc=(0, 0, 0, 0, 2, 2), wave=oracle.WAVE_SINE, amp=g["rho_amp"],
                   omega=g["omega"], t_n=100000, probe_z=zs)
    s.step(2300)
    po = s.probes()
    xo = po[first:first + n, :, 1] / po[first:first + n, :, 0] / g["rho_amp"]
    A, al, k, c = an.wave_fit(xo, first + 1, zpos, g["omega"])
    assert fit["alpha"] == pytest.approx(al, rel=1e-8)
    assert fit["c"] == pytest.approx(c, rel=1e-8)
    assert fit["A"] == pytest.approx(A, rel=1e-8)
    # the paper's values
    assert fit["alpha"] == pytest.approx(g["alpha_s"], rel=0.01)
    assert fit["c"] == pytest.approx(cs, rel=2e-3)
    assert abs(fit["A"] - complex(gold["pure_fluid_fit"]["A_re"], gold["pure_fluid_fit"]["A_im"])) < 0.03
    assert c_ridge == pytest.approx(cs, rel=3e-3)


def test_st_dft_full_size_sampled_against_oracle():
    """The benchmark's launch: a 20000 x 24 record on a 1024 x 1024 grid.  Sampled spectrum
    values (rows and columns spread over the grid, ragged ends included) and the ridge of
    sampled rows against the oracle's transform of those rows."""
    torch, lb = _lb()
    nt, nz, nw, nk = 20000, 24, 1024, 1024
    zpos = 16.0 * np.arange(nz)
    om = 2 * math.pi / 200
    x = inputs.probe_signal(nt, zpos, om, -0.6 - 0.1j, 6e-3, om / 0.7, offset=1e-3, harmonic=0.1, noise=0.02, seed=3)
    w0, dw = 0.0, 0.2 / nw
    k0, dk = -math.pi / 16, (2 * math.pi / 16) / nk
    F, r = lb.st_dft(torch.from_numpy(x).cuda(), zpos, 0.0, w0, dw, nw, k0, dk, nk)
    Fg, rg = F.cpu().numpy(), r.cpu().numpy()
    rows = np.array([0, 1, 63, 64, 255, 511, int(round(om / dw)), 1000, 1023])
    ka = _grid(k0, dk, nk)
    Fo = an.space_time_dft(x, 0.0, zpos, _grid(w0, dw, nw)[rows], ka)
    scale = np.abs(x).sum()
    err = np.abs(Fg[rows] - Fo).max() / scale
    assert err < 1e-12, err
    _check_ridge(Fo, rg[rows], 4 * err * scale / np.abs(Fo).max() + 1e-13)
