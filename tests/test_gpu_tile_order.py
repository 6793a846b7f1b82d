"""Tile order of camera images in scenes larger than an XCD's L2 (more than
32,768 triangles): one-pixel tiles walk the image in 16 x 16 pixel blocks
(8 x 8 when its sides are multiples of 8 but not of 16).  Images of a box
cluttered with 40,000 triangles at 64 spp (16 x 16 and 48 x 32: one and six
16 x 16 blocks; 24 x 16: 8 x 8 blocks) take that order in every per-pixel
kernel; each result must still land on its own pixel: the film
(path-per-lane and wavefront forms), the forward-mode derivative and the
adjoint, against the oracle."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[(16, 16), (24, 16), (48, 32)], ids=["16x16", "24x16", "48x32"])
def setup(oracle_mod, request):
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    w, h = request.param
    sc = scenes.cluttered_box(40000, width=w, height=h, spp=64)
    return tr, sc, oracle_mod.Oracle(sc)


@pytest.mark.parametrize("kernel", ["path", "wavefront"])
def test_block_order_film(setup, kernel):
    import torch
    tr, sc, O = setup
    _announce(f"block tile order film {kernel}")
    with tr.upload(sc) as dev:
        _, film = tr.render_transient(dev, kernel=kernel)
        torch.cuda.synchronize()
        g = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
    o, _, _ = O.render()
    assert o.sum() > 0
    compare_films(g, o)


def test_block_order_tangent(setup):
    import torch
    tr, sc, O = setup
    va = np.random.default_rng(8).uniform(-1.0, 1.0, sc.n_tris).astype(np.float32)
    _announce("block tile order tangent")
    with tr.upload(sc) as dev:
        _, film, dfilm = tr.render_transient_tangent(dev, torch.from_numpy(va).cuda(), None)
        torch.cuda.synchronize()
        g = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        gd = dfilm.cpu().numpy().reshape(sc.n_pixels, sc.n_bins).astype(np.float64)
    o, od, _ = O.render_tangent(va, None)
    compare_films(g, o, what="primal film")
    scale = np.abs(od).max()
    assert scale > 0
    assert np.abs(gd - od).max() <= 1e-4 * scale


@pytest.mark.parametrize("kernel", ["auto", "path"])
def test_block_order_adjoint(setup, kernel):
    import torch
    tr, sc, O = setup
    ta, trough = scenes.perturbed_params(sc, seed=9)
    _announce(f"block tile order adjoint {kernel}")
    target, _, _ = O.render(stream_id=1, albedo=ta, roughness=trough)
    film_o, _, _ = O.render()
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr = tr.render_transient_backward(dev, d, kernel=kernel)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
    assert np.abs(ga - ga_o).max() <= 1e-4 * np.abs(ga_o).max()
    assert np.abs(gr - gr_o).max() <= 1e-4 * np.abs(gr_o).max()
