"""The counting build of the forward kernels (trhip_render_transient_counted),
whose counts give the algorithmic work of the roofline: it renders the same
film as the plain build (and as the oracle); the per-path work counts do not
depend on which kernel form scheduled the paths; the counts the workload
fixes hold (one closest-hit ray per confocal path sample, one shadow ray per
vertex); and each wave count lies between 1/64 of its lane count and the
lane count."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films

pytestmark = pytest.mark.gpu

# per-path work: the same rays, traversals and vertices in every form
WORK = ("nodes", "tris", "rays", "shadow_rays", "vertices", "contributions")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    return tr


def _wave_counts_consistent(c):
    for lanes, waves in (("nodes", "wave_nodes"), ("tris", "wave_tris"), ("vertices", "wave_vertices")):
        assert (c[lanes] == 0) == (c[waves] == 0), (lanes, c)
        assert c[waves] <= c[lanes] <= 64 * c[waves], (lanes, c)


def _counted(tr, sc, **kw):
    import torch
    with tr.upload(sc) as dev:
        st, film, c = tr.render_transient_counted(dev, **kw)
        _, ref = tr.render_transient(dev, **kw)
        torch.cuda.synchronize()
        g = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        r = ref.cpu().numpy().reshape(sc.n_pixels, sc.n_bins).astype(np.float64)
    compare_films(g, r, what="counted film vs plain film")
    _wave_counts_consistent(c)
    return g, c


def test_counted_confocal_forms(tr, oracle_mod):
    """Confocal scan 16 x 16, 2,000-triangle blob, 256 spp: every form counts
    the same work, one closest-hit ray per path sample and one shadow ray per
    vertex, and renders the oracle's film."""
    sc = scenes.confocal_nlos(grid=16, n_tris=2000, spp=256)
    counts = {}
    for form in ("path", "deferred", "wavefront"):
        _announce(f"counted confocal {form}")
        g, counts[form] = _counted(tr, sc, kernel=form)
        if form == "path":
            o, _, _ = oracle_mod.Oracle(sc).render()
            compare_films(g, o, what="counted film vs oracle")
    c = counts["path"]
    assert c["rays"] == sc.n_pixels * sc.spp
    assert 0 < c["vertices"] < c["rays"]
    assert c["shadow_rays"] == c["vertices"]
    assert 0 < c["contributions"] <= c["vertices"]
    for form in ("deferred", "wavefront"):
        assert {k: counts[form][k] for k in WORK} == {k: c[k] for k in WORK}, (form, counts[form], c)


def test_counted_box_room(tr):
    """Pinhole box room, depth 4: the three forms count the same work; every
    path sample casts its camera ray."""
    sc = scenes.box_scene(width=32, height=32, spp=8)
    counts = {}
    for form in ("path", "deferred", "wavefront"):
        _announce(f"counted box room {form}")
        _, counts[form] = _counted(tr, sc, kernel=form)
    cp = counts["path"]
    for form in ("deferred", "wavefront"):
        assert {k: counts[form][k] for k in WORK} == {k: cp[k] for k in WORK}, (form, counts[form], cp)
    assert cp["rays"] >= sc.n_pixels * sc.spp
    assert 0 < cp["vertices"] <= cp["rays"]


def test_counted_nlos_area(tr):
    """NLOS area sampling: no closest-hit ray at all; one vertex per path
    sample, each joined to its scan point by a shadow ray."""
    sc = scenes.confocal_nlos(grid=16, n_tris=2000, spp=256)
    for form in ("path", "deferred"):
        _announce(f"counted NLOS area {form}")
        _, c = _counted(tr, sc, kernel=form, nlos_area=True)
        assert c["rays"] == 0
        assert c["vertices"] == sc.n_pixels * sc.spp
        assert 0 < c["shadow_rays"] <= c["vertices"]
        assert c["contributions"] <= c["shadow_rays"]
