"""Degenerate renders on the GPU against the oracle: paths with no vertex
(max_depth 1 pinhole, 3 confocal), scenes where every ray misses, a film
window that no contribution reaches (all mass out of window), the last
representable sample indices (sample_offset + spp = 2^32), one sample per
pixel, and a one-pixel film."""
import copy
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films, compare_vec

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    return tr


def _render(tr, sc, **kw):
    import torch
    with tr.upload(sc) as dev:
        st, film, oow = tr.render_transient(dev, return_oow=True, **kw)
        torch.cuda.synchronize()
        return (film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins), st.cpu().numpy().ravel(),
                oow.cpu().numpy().ravel())


@pytest.mark.parametrize("kernel", ["path", "deferred", "wavefront"])
def test_no_vertex(tr, kernel):
    _announce(f"no vertex {kernel}")
    film, st, oow = _render(tr, scenes.box_scene(width=16, height=16), max_depth=1, kernel=kernel)
    assert not film.any() and not st.any() and not oow.any()
    film, st, oow = _render(tr, scenes.confocal_nlos(grid=4, n_tris=500, spp=64), max_depth=3, kernel=kernel)
    assert not film.any() and not st.any() and not oow.any()


@pytest.mark.parametrize("kernel", ["path", "deferred", "wavefront"])
def test_everything_misses(tr, kernel):
    """The blob moved behind the relay wall: no first ray reaches it."""
    sc = scenes.confocal_nlos(grid=8, n_tris=2000, spp=256)
    v = sc.vertices.copy()
    blob = np.unique(sc.indices[2:])
    v[blob, 2] -= 3.0
    sc.vertices = v
    _announce(f"everything misses {kernel}")
    film, st, oow = _render(tr, sc, kernel=kernel)
    assert not film.any() and not st.any() and not oow.any()


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_window_misses_everything(tr, oracle_mod, kernel):
    """A window after every arrival: the film is zero and the mass sits out
    of window, equal to the steady image."""
    sc = scenes.box_scene(width=24, height=24, bin_start=50.0)
    _announce(f"window misses {kernel}")
    film, st, oow = _render(tr, sc, kernel=kernel)
    assert not film.any()
    assert st.sum() > 0
    np.testing.assert_allclose(oow, st, rtol=1e-6)
    o, ost, ooow = oracle_mod.Oracle(sc).render()
    compare_vec(st, ost, what="steady")
    compare_vec(oow, ooow, what="oow")


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_last_sample_indices(tr, oracle_mod, kernel):
    """Samples [2^32 - 7, 2^32): the counter's sample word at its end."""
    sc = scenes.confocal_nlos(grid=6, n_tris=2000, spp=7)
    off = (1 << 32) - 7
    _announce(f"last sample indices {kernel}")
    film, st, _ = _render(tr, sc, sample_offset=off, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(sample_offset=off)
    compare_films(film, o)


@pytest.mark.parametrize("kernel", ["path", "deferred", "wavefront"])
def test_one_sample_one_pixel(tr, oracle_mod, kernel):
    sc = scenes.box_scene(width=1, height=1, spp=1)
    sc.tan_x = sc.tan_y = 0.2
    _announce(f"one sample one pixel {kernel}")
    film, st, _ = _render(tr, sc, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render()
    assert ost.sum() > 0
    compare_films(film, o)
    sc2 = scenes.box_scene(width=40, height=30, spp=1)
    film, st, _ = _render(tr, sc2, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc2).render()
    compare_films(film, o)
