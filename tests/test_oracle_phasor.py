"""Pins of the oracle's frequency-space film (Sec. 4.3, Eq. 14): the zero
frequency is the steady image, a single-bounce plane gives the closed form
value * exp(-2 pi i f tof) per pixel, and the phasor equals the discrete
Fourier sum of a fine time histogram of the same paths within the bound
set by the bin width."""
import math

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.test_oracle_analytic import _pixel_dirs

FREQS = [0.5, 5.0, 7.5, 16.6]  # cycles per metre (wavelengths 2 m .. 6 cm)


def test_zero_frequency_is_the_steady_image(oracle_mod):
    sc = scenes.box_scene(width=16, height=12)
    O = oracle_mod.Oracle(sc)
    ph, st = O.render_phasor([0.0] + FREQS, spp=8)
    _, st2, _ = O.render(spp=8)
    assert (ph[:, 0].real == st).all() and (ph[:, 0].imag == 0).all()
    assert (st == st2).all()
    assert (np.abs(ph) <= st[:, None] * (1 + 1e-12)).all()


@pytest.mark.parametrize("unwarp", [False, True])
def test_single_bounce_plane_closed_form(oracle_mod, unwarp):
    """Every pixel sees one path: phasor = rho I cos / (pi r^2) times
    exp(-2 pi i f tof) with tof = |c - x| + |x - l| (camera time) or |x - l|
    (unwarped)."""
    sc = scenes.plane_scene(h=1.0, albedo=0.6, unwarp=unwarp)
    O = oracle_mod.Oracle(sc)
    ph, _ = O.render_phasor(FREQS, spp=1, max_depth=2, pixel_centre=True)
    d = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    t = -o[1] / d[:, 1]
    x = o[None] + t[:, None] * d
    r = np.linalg.norm(x - light[None], axis=1)
    value = 0.6 * 1.0 * (light[1] / r) / (math.pi * r**2)
    tof = r + (0.0 if unwarp else t)
    f = np.asarray(FREQS)[None]
    want = value[:, None] * np.exp(-2j * math.pi * f * tof[:, None])
    # FP32 geometry: value to 1e-5, tof to a few 1e-7 relative
    tol = value[:, None] * (1e-5 + 2 * math.pi * f * tof[:, None] * 1e-6)
    assert (np.abs(ph - want) <= tol).all()


def test_phasor_matches_fine_histogram_dft(oracle_mod):
    """Box room, depth 4: the phasor against sum_b film[b] exp(-2 pi i f
    (start + (b + 1/2) w)); each contribution's tof lies in its bin, so
    |difference| <= steady * pi f w."""
    w = 2e-4
    sc = scenes.box_scene(width=8, height=6, n_bins=50000, bin_width=w, bin_start=0.0)
    O = oracle_mod.Oracle(sc)
    film, steady, oow = O.render(spp=16)
    assert oow.max() == 0.0
    ph, st = O.render_phasor(FREQS, spp=16)
    np.testing.assert_array_equal(st, steady)
    centres = sc.bin_start + (np.arange(sc.n_bins) + 0.5) * w
    for j, f in enumerate(FREQS):
        dft = film @ np.exp(-2j * math.pi * f * centres)
        bound = steady * math.pi * f * w * (1 + 1e-3) + 1e-12
        assert (np.abs(ph[:, j] - dft) <= bound).all()
        # the bound is tight enough to see a conjugated or mis-scaled phase
        assert np.abs(ph[:, j].imag).max() > 20 * bound.max()
