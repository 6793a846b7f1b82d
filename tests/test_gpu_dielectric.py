"""GPU refractive indices, dielectric interfaces and scattering delays
(Eqs. 3 and 10) against the oracle on the same seeded paths: film (bin
indices exact, 1e-4 relative on bins >= 1e-3 of the peak) through a glass
tank, a glass slab and the box room with a glass box (every kernel form),
with scattering delays, in fog with an index around the meshes, with NLOS
area sampling of a delayed hidden object; the adjoint (|dg| <= 1e-4
max|g|), the forward-mode derivative, the phasor film and the batch with
such scenes."""
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


def _check(tr, oracle_mod, sc, pixels=None, **kw):
    import torch
    with tr.upload(sc) as dev:
        st, film = tr.render_transient(dev, **kw)
        torch.cuda.synchronize()
        g = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        gst = st.cpu().numpy().ravel()
    ora_kw = {k: v for k, v in kw.items()
              if k in ("spp", "seed", "max_depth", "sample_offset", "stream_id", "pixel_centre", "nlos_area")}
    o, ost, _ = oracle_mod.Oracle(sc).render(pixels=pixels, **ora_kw)
    if pixels is not None:
        g, gst = g[pixels], gst[pixels]
    assert ost.sum() > 0
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")


@pytest.mark.parametrize("centre", [True, False])
def test_glass_tank(tr, oracle_mod, centre):
    _announce(f"glass tank centre={centre}")
    _check(tr, oracle_mod, scenes.glass_tank_scene(ior=1.33), pixel_centre=centre)


def test_glass_slab(tr, oracle_mod):
    _announce("glass slab")
    _check(tr, oracle_mod, scenes.glass_slab_scene(ior=1.5))


@pytest.mark.parametrize("kernel", ["path", "deferred", "wavefront"])
def test_glass_box_room(tr, oracle_mod, kernel):
    """Box room with a glass box, 64 x 64, 16 spp, depth 8 (internal
    reflections and total internal reflection inside the box)."""
    _announce(f"glass box room {kernel}")
    _check(tr, oracle_mod, scenes.glass_box_scene(), kernel=kernel)


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_scattering_delays(tr, oracle_mod, kernel):
    _announce(f"scattering delays {kernel}")
    _check(tr, oracle_mod, scenes.glass_box_scene(delay_mean=0.05), kernel=kernel)


def test_fog_index_around_glass(tr, oracle_mod):
    """Fog (free flight only around the meshes) with index 1.2 around them,
    the glass box and delays, depth 6."""
    sc = scenes.glass_box_scene(delay_mean=0.02, width=48, height=48, spp=16, max_depth=6)
    sc.sigma_t, sc.medium_albedo, sc.medium_ior = 0.6, 0.8, 1.2
    _announce("fog + index + glass + delays")
    _check(tr, oracle_mod, sc)


@pytest.mark.parametrize("area", [False, True])
def test_confocal_delayed_hidden_object(tr, oracle_mod, area):
    """A fluorescent hidden blob (delay mean 2 cm), cosine and NLOS area
    sampling."""
    sc = scenes.confocal_nlos(grid=16, spp=256)
    sc.delay = np.where(np.arange(sc.n_tris) >= 2, 0.02, 0.0).astype(np.float32)
    _announce(f"confocal delayed blob area={area}")
    _check(tr, oracle_mod, sc, nlos_area=area)


@pytest.mark.parametrize("kernel", ["auto", "path"])
def test_adjoint_with_glass(tr, oracle_mod, kernel):
    """Albedo and roughness gradients with a glass box and delays in the
    room, register-stash and path-replay adjoints."""
    import torch
    sc = scenes.glass_box_scene(delay_mean=0.03, width=24, height=24, spp=64, max_depth=5)
    sc.mat_type = sc.mat_type.copy()
    sc.mat_type[22:34] = scenes.MAT_GGX      # the tall box as a rough conductor
    ta = np.clip(sc.albedo + np.random.default_rng(3).uniform(-0.1, 0.1, sc.n_tris), 0.05, 0.95)
    ta = ta.astype(np.float32)
    _announce(f"adjoint with glass {kernel}")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(stream_id=1, albedo=ta)
    film_o, _, _ = O.render()
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr, primal = tr.render_transient_backward(dev, d, primal=True, kernel=kernel)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
        primal = primal.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
    compare_films(primal, film_o, what="primal film")
    for g, go in ((ga, ga_o), (gr, gr_o)):
        scale = np.abs(go).max()
        assert scale > 0
        assert np.abs(g - go).max() <= 1e-4 * scale, np.abs(g - go).max() / scale
    assert (ga[sc.mat_type == scenes.MAT_DIELECTRIC] == 0).all()


def test_tangent_with_glass(tr, oracle_mod):
    import torch
    sc = scenes.glass_box_scene(delay_mean=0.03, width=24, height=24, spp=64, max_depth=5)
    va = np.random.default_rng(4).uniform(-1.0, 1.0, sc.n_tris).astype(np.float32)
    _announce("tangent with glass")
    with tr.upload(sc) as dev:
        _, film, dfilm = tr.render_transient_tangent(dev, torch.from_numpy(va).cuda(), None)
        torch.cuda.synchronize()
        g_film = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        g_d = dfilm.cpu().numpy().reshape(sc.n_pixels, sc.n_bins).astype(np.float64)
    o_film, o_d, _ = oracle_mod.Oracle(sc).render_tangent(va, None)
    compare_films(g_film, o_film, what="primal film")
    scale = np.abs(o_d).max()
    assert np.abs(g_d - o_d).max() <= 1e-4 * scale, np.abs(g_d - o_d).max() / scale


def test_phasor_with_delays_and_glass(tr, oracle_mod):
    import torch
    sc = scenes.glass_box_scene(delay_mean=0.05, width=32, height=32, spp=16, max_depth=6)
    freqs = [0.0, 0.7, 3.1, 12.5]
    _announce("phasor with delays and glass")
    with tr.upload(sc) as dev:
        st, ph = tr.render_phasor(dev, freqs)
        torch.cuda.synchronize()
        g = ph.cpu().numpy().reshape(sc.n_pixels, len(freqs)).astype(np.complex128)
        gst = st.cpu().numpy().ravel()
    o, ost = oracle_mod.Oracle(sc).render_phasor(np.float32(freqs).astype(np.float64))
    compare_vec(gst, ost, what="steady")
    err = np.abs(g - o)
    tol = 1e-4 * ost[:, None] + 1e-7 * ost.max()
    assert (err <= tol).all(), float((err / np.maximum(tol, 1e-30)).max())


def test_batch_with_glass_and_delays(tr):
    """The persistent batch renders a glass room, a delayed confocal scene
    and a plain one exactly as single renders do."""
    import torch
    scs = [scenes.glass_box_scene(width=32, height=32, spp=8, max_depth=6),
           scenes.glass_box_scene(delay_mean=0.04, width=16, height=24, spp=8),
           scenes.confocal_nlos(grid=12, n_tris=1000, spp=64)]
    scs[2].delay = np.full(scs[2].n_tris, 0.01, np.float32)
    _announce("batch with glass and delays")
    devs = [tr.upload(sc) for sc in scs]
    try:
        with tr.Batch(devs, autotune=False) as b:
            films = [f.clone() for f in b.render()]
            torch.cuda.synchronize()
        for dev, f in zip(devs, films):
            _, ref = tr.render_transient(dev)
            torch.cuda.synchronize()
            compare_films(f.cpu().numpy().reshape(dev.scene.n_pixels, -1),
                          ref.cpu().numpy().reshape(dev.scene.n_pixels, -1).astype(np.float64), what="batch film")
    finally:
        for d in devs:
            d.destroy()
