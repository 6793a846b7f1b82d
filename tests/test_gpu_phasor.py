"""GPU frequency-space film (trhip_render_phasor) against the oracle's on
the same seeded paths.  Tolerance per pixel and frequency: 1e-4 of the
pixel's steady value (the sum of |c| over its contributions): the FP32
phase f * tof carries a relative error of 2^-24, i.e. at most
2 pi * 100 cycles * 6e-8 = 4e-5 rad for the optical paths and frequencies
used here, plus FP32 accumulation."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_vec

pytestmark = pytest.mark.gpu

FREQS = [0.0, 0.5, 5.0, 7.5, 10.0, 16.6]


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    return tr


def _check(tr, oracle_mod, sc, pixels=None, freqs=FREQS, **kw):
    import torch
    with tr.upload(sc) as dev:
        st, ph = tr.render_phasor(dev, freqs, **kw)
        torch.cuda.synchronize()
        g = ph.cpu().numpy().reshape(sc.n_pixels, len(freqs)).astype(np.complex128)
        gst = st.cpu().numpy().ravel().astype(np.float64)
    ora_kw = {k: v for k, v in kw.items() if k in ("spp", "seed", "max_depth", "sample_offset", "pixel_centre")}
    o, ost = oracle_mod.Oracle(sc).render_phasor(np.float32(freqs).astype(np.float64), pixels=pixels, **ora_kw)
    if pixels is not None:
        g, gst = g[pixels], gst[pixels]
    assert ost.sum() > 0
    compare_vec(gst, ost, what="steady")
    err = np.abs(g - o)
    tol = 1e-4 * ost[:, None] + 1e-7 * ost.max()
    assert (err <= tol).all(), float((err / np.maximum(tol, 1e-30)).max())
    return g, o


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_box_phasor(tr, oracle_mod, kernel):
    """Box room 64x64, 16 spp, depth 4, the paper's modulation frequencies."""
    _announce(f"phasor box {kernel}")
    _check(tr, oracle_mod, scenes.box_scene(), kernel=kernel)


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_confocal_phasor_reduced(tr, oracle_mod, kernel):
    _announce(f"phasor confocal 16x16 {kernel}")
    _check(tr, oracle_mod, scenes.confocal_nlos(grid=16, spp=256), kernel=kernel)


def test_confocal_phasor_full_size_sampled(tr, oracle_mod):
    """Full confocal workload (4096 spp, automatic form with sample chunks),
    the oracle recomputes 16 sampled scan points."""
    sc = scenes.confocal_nlos()
    pix = np.sort(np.random.default_rng(9).choice(sc.n_pixels, 16, replace=False)).astype(np.int32)
    _announce("phasor confocal full sampled")
    _check(tr, oracle_mod, sc, pixels=pix)


def test_phasor_fog_ggx_unwarp(tr, oracle_mod):
    """GGX and Lambertian surfaces in fog, camera unwarping, 32 frequencies."""
    sc = scenes.large_scene(cells=24, sphere_freq=4, grid=3, width=40, height=30, n_bins=256, bin_width=0.02,
                            spp=4)
    sc.camera_unwarp = True
    _announce("phasor fog ggx unwarp")
    _check(tr, oracle_mod, sc, freqs=list(np.linspace(0.0, 20.0, 32)))


def test_phasor_accumulate_and_dc(tr):
    """Split sample ranges accumulate to the full render; f = 0 is the steady
    image."""
    import torch
    sc = scenes.confocal_nlos(grid=8, spp=8192)
    _announce("phasor accumulate")
    with tr.upload(sc) as dev:
        st, ph = tr.render_phasor(dev, FREQS)
        st2, ph2 = tr.render_phasor(dev, FREQS, spp=4096, norm_spp=8192)
        tr.render_phasor(dev, FREQS, spp=4096, sample_offset=4096, norm_spp=8192, accumulate=True,
                         phasor=torch.view_as_real(ph2), steady=st2)
        torch.cuda.synchronize()
        a, b = ph.cpu().numpy(), ph2.cpu().numpy()
        s = st.cpu().numpy()
    scale = s.max()
    assert np.abs(a - b).max() <= 1e-5 * scale
    np.testing.assert_allclose(a[..., 0].real, s, rtol=2e-6, atol=1e-9 * scale)
    assert np.abs(a[..., 0].imag).max() == 0.0


def test_phasor_rejects(tr):
    from paper_2510_25660_amd._binding import TrhipError
    sc = scenes.box_scene(width=8, height=8)
    with tr.upload(sc) as dev:
        with pytest.raises(TrhipError):
            tr.render_phasor(dev, FREQS, kernel="wavefront")
        with pytest.raises(TrhipError):
            tr.render_phasor(dev, list(range(33)))
        with pytest.raises(TrhipError):
            tr.render_phasor(dev, [1.0, float("nan")])
