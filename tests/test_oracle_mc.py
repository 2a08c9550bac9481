"""Pins of the oracle's photon-transport Monte Carlo of the response table
(Sec 2.1.1, Eq.1: the table the paper obtains by simulation), against facts
fixed outside it: the published known-answer vectors of its random-number
generator, the analytic first-interaction table it must reproduce in
expectation, the Thomson limit and the tabulated Klein-Nishina cross section
of its scatter physics, and the symmetries of the geometry.

The scatter mode's cross-section model (photoelectric fraction, its energy
scaling, the 350 keV threshold, centroid positioning) is a reading that no
published number here fixes; only its sampler, its cross section and its
symmetries are pinned.
"""
import math

import numpy as np
import pytest

from paper_1607_06170_amd import synth as S

CFG = S.CFG_2D
CFG3 = S.CFG_3D
MU, L = 0.087, 15.0


def test_philox_known_answers(oracle):
    """Philox4x32-10 (Salmon et al., SC 2011) against the known-answer vectors
    published with its reference implementation."""
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert oracle.philox4x32_10(ctr, key).tolist() == want


@pytest.mark.parametrize("row", [0, 20, 45, 60])
def test_first_interaction_mc_is_the_analytic_table_2d(oracle, row):
    """Mode 0 samples the first interaction of the analytic table (reading:
    the table is the first-interaction probability): every entry within 5
    binomial sigma of the closed-form table, for every sub-position."""
    n = 200_000
    c = oracle.table_mc_counts(CFG, False, n, 11, False, (row * 4, row * 4 + 4))
    est = c[:, :, 2] / n
    ref = oracle.table_2d(CFG).data[row]
    sig = np.sqrt(np.maximum(ref * (1 - ref), 1e-12) / n)
    assert np.all(np.abs(est - ref) <= 5 * sig + 1e-12), (row, est, ref)
    assert np.all(c[:, :, [0, 1, 3, 4]] == 0)


@pytest.mark.parametrize("rt,rz", [(0, 0), (17, 44), (60, 5)])
def test_first_interaction_mc_is_the_analytic_table_3d(oracle, rt, rz):
    n = 100_000
    cell0 = (rt * 61 + rz) * 16
    c = oracle.table_mc_counts(CFG3, True, n, 12, False, (cell0, cell0 + 16)).reshape(4, 4, 5, 5)
    ref = oracle.table3_rows(CFG3, [rt], [rz])[0]
    sig = np.sqrt(np.maximum(ref * (1 - ref), 1e-12) / n)
    assert np.all(np.abs(c / n - ref) <= 5 * sig + 1e-12)


def test_kn_cross_section_thomson_limit_and_511(oracle):
    """The Klein-Nishina total cross section tends to the Thomson value (4/3
    in units of 2 pi r_e^2) at low energy, and at 511 keV it is 0.2867 barn
    against the Thomson 0.6652 barn (ratio 0.4310)."""
    assert abs(oracle.kn_sigma(1e-4) - 4.0 / 3.0) < 1e-3
    assert abs(oracle.kn_sigma(1.0) / (4.0 / 3.0) - 0.4310) < 1e-3
    # it falls with energy
    s = [oracle.kn_sigma(k) for k in (0.1, 0.3, 1.0, 3.0)]
    assert all(a > b for a, b in zip(s, s[1:]))


def test_kn_sampler(oracle):
    """The scattering-angle sampler: in the Thomson limit cos(theta) has mean
    0 and mean square 2/5 (the (1 + cos^2) law); at 511 keV forward scatter
    dominates; the histogram at 511 keV follows the Klein-Nishina shape
    (normalised by quadrature) within 5 sigma per bin."""
    n = 400_000
    c = oracle.kn_cos_samples(1e-6, n, 5)
    assert abs(c.mean()) < 5 * math.sqrt(0.4 / n)
    assert abs((c * c).mean() - 0.4) < 5 * math.sqrt(0.1 / n)
    c = oracle.kn_cos_samples(1.0, n, 6)
    assert c.mean() > 0.2
    edges = np.linspace(-1, 1, 21)
    x = np.linspace(-1, 1, 200_001)
    eps = 1 / (1 + 1.0 * (1 - x))
    f = eps * eps * (eps + 1 / eps - (1 - x * x))
    cdf = np.concatenate([[0], np.cumsum((f[1:] + f[:-1]) / 2 * np.diff(x))])
    cdf /= cdf[-1]
    p = np.diff(np.interp(edges, x, cdf))
    h = np.histogram(c, edges)[0] / n
    assert np.all(np.abs(h - p) <= 5 * np.sqrt(p * (1 - p) / n))


def test_scatter_mode_properties(oracle):
    """With Compton scatter: at normal incidence the response of sub-position
    p at offset a equals that of sub-position P - 1 - p at offset -a (the
    geometry's mirror), within 5 sigma; scatter spreads counts into
    neighbours the first interaction never reaches at normal incidence; no
    more photons are detected than interact, 1 - exp(-mu L)."""
    n = 200_000
    c = oracle.table_mc_counts(CFG, False, n, 13, True, (0, 4))[:, :, 2] / n
    sig = np.sqrt(np.maximum(c * (1 - c), 1e-12) / n)
    for p in range(4):
        m = c[3 - p, ::-1]
        assert np.all(np.abs(c[p] - m) <= 5 * np.hypot(sig[p], sig[3 - p][::-1]) + 1e-12)
    assert np.all(c[:, [1, 3]] > 0)
    assert np.all(c.sum(axis=1) <= 1 - math.exp(-MU * L) + 5 * np.sqrt(0.25 / n))


def test_3d_mc_reduces_to_2d(oracle):
    """No axial tilt: the 3D first-interaction response stays in axial offset
    0 and its transaxial profile is the 2D one (independent photons; 5 sigma)."""
    n = 100_000
    rt = 33
    c3 = oracle.table_mc_counts(CFG3, True, n, 14, False, ((rt * 61) * 16, (rt * 61) * 16 + 16)).reshape(4, 4, 5, 5)
    c2 = oracle.table_mc_counts(CFG, False, n, 15, False, (rt * 4, rt * 4 + 4))[:, :, 2]
    assert np.all(c3[..., [0, 1, 3, 4]] == 0)
    for pz in range(4):
        a, b = c3[:, pz, :, 2] / n, c2 / n
        sig = np.sqrt(np.maximum(a * (1 - a), 1e-12) / n + np.maximum(b * (1 - b), 1e-12) / n)
        assert np.all(np.abs(a - b) <= 5 * sig + 1e-12)
