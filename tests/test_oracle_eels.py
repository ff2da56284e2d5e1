"""Pins of the 2D EELS oracle (Eq. (17)): the resolution function has unit
area and the stated full width at half maximum, the spectrum integrates to
the total cross section, each peak sits at its energy loss, closed
channels contribute nothing, and the per-final shares reproduce the pinned
cross sections of the final states."""
import numpy as np

from oracle import eels, observables
from paper_2307_13483_amd import inputs


def test_resolution_area_and_fwhm():
    w = 0.010
    x = np.linspace(-0.2, 0.2, 400001)
    r = eels.resolution(x, w)
    assert abs(np.trapezoid(r, x) - 1.0) < 1e-10
    peak = eels.resolution(0.0, w)
    assert abs(eels.resolution(w / 2, w) - peak / 2) < 1e-12 * peak
    assert abs(eels.resolution(-w / 2, w) - peak / 2) < 1e-12 * peak


def test_spectrum_integrates_to_the_total_and_peaks_at_the_losses():
    shares = np.array([0.7, 0.2, 0.05])
    losses = np.array([0.0, 0.15, 0.30])
    grid = np.linspace(-0.1, 0.45, 55001)
    S = eels.spectrum(shares, losses, grid)
    assert abs(np.trapezoid(S, grid) - shares.sum()) < 1e-9
    for d in losses:
        k = np.argmin(np.abs(grid - d))
        assert S[k] >= S[k - 5] and S[k] >= S[k + 5]


def test_shares_match_cross_sections_and_closed_channels_vanish():
    p = inputs.draw_params(5)
    Ng, Nu, eps = 7, 6, 0.42
    sig = {}
    for mu in (0, 1):
        s, loss = eels.final_shares(p, Ng, Nu, eps, (0, 0), mu)
        sig[mu] = s
        assert np.all(s[loss > eps] == 0.0)           # eps_f <= 0: closed
    finals = [(0, 0), (1, 0), (2, 0), (0, 1)]
    ref = observables.cross_sections(p, Ng, Nu, eps, (0, 0), finals)
    got = np.array([sig[0][g, u] + sig[1][g, u] for g, u in finals])
    assert np.allclose(got, ref, rtol=1e-12, atol=0)
