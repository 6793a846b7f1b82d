"""GPU NLOS area sampling (TRHIP_FLAG_NLOS_AREA_SAMPLING) against the
oracle's on the same seeded paths: film (bin indices exact, 1e-4 relative
on bins >= 1e-3 of the peak), phasor film, forward-mode derivative and
adjoint (|dg| <= 1e-4 max|g|), at a reduced scan grid and at full size on
sampled scan points; the unbiasedness check against cosine sampling on the
GPU; and the requests the flag rejects."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films, compare_vec

pytestmark = pytest.mark.gpu

STATUS_UNSUPPORTED = 4


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    return tr


def _film(tr, sc, **kw):
    import torch
    with tr.upload(sc) as dev:
        st, film = tr.render_transient(dev, nlos_area=True, **kw)
        torch.cuda.synchronize()
        return st.cpu().numpy().ravel(), film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)


@pytest.mark.parametrize("kernel", ["deferred", "path"])
def test_area_sampling_reduced(tr, oracle_mod, kernel):
    """16 x 16 scan grid, 256 spp, every scan point."""
    sc = scenes.confocal_nlos(grid=16, spp=256)
    _announce(f"nlos area confocal 16x16 {kernel}")
    gst, g = _film(tr, sc, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True)
    assert ost.min() > 0
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")


def test_area_sampling_full_size_sampled(tr, oracle_mod):
    """The full confocal workload (64 x 64 scan points, 4096 spp, 10k
    triangles); the oracle recomputes 16 sampled scan points."""
    sc = scenes.confocal_nlos()
    pix = np.sort(np.random.default_rng(31).choice(sc.n_pixels, 16, replace=False)).astype(np.int32)
    _announce("nlos area confocal full sampled")
    gst, g = _film(tr, sc)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True, pixels=pix)
    compare_films(g[pix], o)
    compare_vec(gst[pix], ost, what="steady")


@pytest.mark.parametrize("kernel", ["deferred", "path"])
def test_area_sampling_ragged_offsets(tr, oracle_mod, kernel):
    """A 7 x 7 grid in tiles of 4 scan points (the last tile holds one), a
    sample offset and a second Philox stream."""
    sc = scenes.confocal_nlos(grid=7, spp=99)
    _announce(f"nlos area ragged offsets {kernel}")
    gst, g = _film(tr, sc, sample_offset=12345, stream_id=3, tile_pixels=4, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True, sample_offset=12345, stream_id=3)
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")


@pytest.mark.parametrize("kernel", ["deferred", "path"])
def test_area_sampling_two_triangle_plane(tr, oracle_mod, kernel):
    """Smallest sampling set (the two triangles of a plane facing the wall;
    a four-cell guide table): against the oracle."""
    sc = scenes.parallel_plane_confocal(d=0.4, half=0.5, grid=4, n_bins=512, bin_width=0.0024, bin_start=0.7,
                                        spp=2048)
    _announce(f"nlos area two-triangle plane {kernel}")
    gst, g = _film(tr, sc, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True)
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")


@pytest.mark.parametrize("kernel", ["deferred", "path"])
def test_area_sampling_deeper_paths(tr, oracle_mod, kernel):
    """Five bounces on the blob (16 x 16, 256 spp) and four behind an
    occluder: paths continue from the drawn vertex only when its first
    segment is unoccluded."""
    _announce(f"nlos area deeper {kernel}")
    sc = scenes.confocal_nlos(grid=16, n_tris=4000, spp=256, bounces=5)
    gst, g = _film(tr, sc, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True)
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")
    sc = scenes.occluded_nlos_scene(grid=4, spp=1024, bounces=4)
    gst, g = _film(tr, sc, kernel=kernel)
    o, ost, _ = oracle_mod.Oracle(sc).render(nlos_area=True)
    compare_films(g, o)
    compare_vec(gst, ost, what="steady")


def test_area_sampling_adjoint_deeper(tr, oracle_mod):
    """Albedo gradients with two hidden vertices (path replay and stash)."""
    import torch
    sc = scenes.confocal_nlos(grid=8, n_tris=2000, spp=128, bounces=4)
    ta = np.clip(sc.albedo * np.random.default_rng(9).uniform(0.7, 1.3, sc.n_tris), 0.05, 1.0).astype(np.float32)
    _announce("nlos area adjoint deeper")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(stream_id=1, albedo=ta, nlos_area=True)
    film_o, _, _ = O.render(nlos_area=True)
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, _ = O.backward(delta, nlos_area=True)
    scale = np.abs(ga_o).max()
    assert scale > 0
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        for kernel in ("auto", "path"):
            ga, _ = tr.render_transient_backward(dev, d, kernel=kernel, nlos_area=True)
            torch.cuda.synchronize()
            ga = ga.cpu().numpy().astype(np.float64)
            assert np.abs(ga - ga_o).max() <= 1e-4 * scale, (kernel, np.abs(ga - ga_o).max() / scale)


@pytest.mark.parametrize("autotune", [False, True])
def test_area_sampling_batch(tr, autotune):
    """A batch mixing area-sampled and cosine-sampled confocal scans of
    different sizes: every film equals its single render."""
    import torch
    scs = [scenes.confocal_nlos(grid=12, n_tris=3000, spp=256), scenes.confocal_nlos(grid=8, n_tris=1000, spp=128),
           scenes.confocal_nlos(grid=10, n_tris=2000, spp=64, bounces=4)]
    renders = [{"nlos_area": True}, {}, {"nlos_area": True}]
    _announce(f"nlos area batch autotune={autotune}")
    devs = [tr.upload(sc) for sc in scs]
    try:
        with tr.Batch(devs, renders=renders, autotune=autotune) as b:
            films = [f.clone() for f in b.render()]
            torch.cuda.synchronize()
        for dev, kw, f in zip(devs, renders, films):
            _, ref = tr.render_transient(dev, **kw)
            torch.cuda.synchronize()
            compare_films(f.cpu().numpy().reshape(dev.scene.n_pixels, -1),
                          ref.cpu().numpy().reshape(dev.scene.n_pixels, -1).astype(np.float64), what="batch film")
    finally:
        for d in devs:
            d.destroy()


def test_area_sampling_unbiased_on_gpu(tr):
    """Same expectation as cosine sampling: 4-seed steady images of both
    estimators agree within 5 pooled standard errors; area sampling has
    the lower spread."""
    sc = scenes.confocal_nlos(grid=8, spp=2048)
    _announce("nlos area vs cosine on the GPU")
    import torch
    a, c = [], []
    with tr.upload(sc) as dev:
        for i in range(4):
            a.append(tr.render_transient(dev, seed=200 + i, nlos_area=True)[0].cpu().numpy().ravel())
            c.append(tr.render_transient(dev, seed=300 + i)[0].cpu().numpy().ravel())
        torch.cuda.synchronize()
    a, c = np.array(a, np.float64), np.array(c, np.float64)
    se = np.sqrt(a.var(0, ddof=1) / len(a) + c.var(0, ddof=1) / len(c))
    z = np.abs(a.mean(0) - c.mean(0)) / (se + 1e-3 * c.mean(0))
    assert (z < 5).all(), z.max()
    assert a.std(0).mean() < c.std(0).mean()


def test_area_sampling_phasor(tr, oracle_mod):
    import torch
    sc = scenes.confocal_nlos(grid=8, spp=256)
    freqs = [0.0, 2.5, 10.0, 16.6]
    _announce("nlos area phasor")
    with tr.upload(sc) as dev:
        st, ph = tr.render_phasor(dev, freqs, nlos_area=True)
        torch.cuda.synchronize()
        g = ph.cpu().numpy().reshape(sc.n_pixels, len(freqs)).astype(np.complex128)
        gst = st.cpu().numpy().ravel()
    o, ost = oracle_mod.Oracle(sc).render_phasor(np.float32(freqs).astype(np.float64), nlos_area=True)
    compare_vec(gst, ost, what="steady")
    err = np.abs(g - o)
    tol = 1e-4 * ost[:, None] + 1e-7 * ost.max()
    assert (err <= tol).all(), float((err / np.maximum(tol, 1e-30)).max())


def test_area_sampling_tangent(tr, oracle_mod):
    import torch
    sc = scenes.confocal_nlos(grid=8, n_tris=2000, spp=256)
    va = np.random.default_rng(4).uniform(-1.0, 1.0, sc.n_tris).astype(np.float32)
    _announce("nlos area tangent")
    with tr.upload(sc) as dev:
        st, film, dfilm = tr.render_transient_tangent(dev, torch.from_numpy(va).cuda(), None, nlos_area=True)
        torch.cuda.synchronize()
        g_film = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        g_d = dfilm.cpu().numpy().reshape(sc.n_pixels, sc.n_bins).astype(np.float64)
    o_film, o_d, _ = oracle_mod.Oracle(sc).render_tangent(va, None, nlos_area=True)
    compare_films(g_film, o_film, what="primal film")
    scale = np.abs(o_d).max()
    assert scale > 0
    assert np.abs(g_d - o_d).max() <= 1e-4 * scale, np.abs(g_d - o_d).max() / scale


@pytest.mark.parametrize("kernel", ["auto", "path"])
def test_area_sampling_adjoint(tr, oracle_mod, kernel):
    """Albedo gradient of L = sum (I - I*)^2 (target rendered with other
    albedos), register-stash and path-replay adjoints."""
    import torch
    sc = scenes.confocal_nlos(grid=8, n_tris=2000, spp=256)
    ta = np.clip(sc.albedo * np.random.default_rng(8).uniform(0.7, 1.3, sc.n_tris), 0.05, 1.0).astype(np.float32)
    _announce(f"nlos area adjoint {kernel}")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(stream_id=1, albedo=ta, nlos_area=True)
    film_o, _, _ = O.render(nlos_area=True)
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, _ = O.backward(delta, nlos_area=True)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr, primal = tr.render_transient_backward(dev, d, primal=True, kernel=kernel, nlos_area=True)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy()
        primal = primal.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
    compare_films(primal, film_o, what="primal film")
    scale = np.abs(ga_o).max()
    assert scale > 0
    assert np.abs(ga - ga_o).max() <= 1e-4 * scale, np.abs(ga - ga_o).max() / scale
    assert (gr == 0).all()


def test_area_sampling_rejections(tr):
    """Other sensors, shallow depths, media, the wavefront form and a scene
    with nothing off the relay wall are refused (no launch)."""
    _announce("nlos area rejections")
    box = scenes.box_scene(width=8, height=8, spp=2)
    with tr.upload(box) as dev:
        with pytest.raises(tr.TrhipError) as e:
            tr.render_transient(dev, nlos_area=True)
        assert e.value.status == STATUS_UNSUPPORTED
    sc = scenes.confocal_nlos(grid=4, n_tris=500, spp=4)
    with tr.upload(sc) as dev:
        for kw in ({"max_depth": 3}, {"kernel": "wavefront"}):
            with pytest.raises(tr.TrhipError) as e:
                tr.render_transient(dev, nlos_area=True, **kw)
            assert e.value.status == STATUS_UNSUPPORTED, kw
    fog = scenes.confocal_nlos(grid=4, n_tris=500, spp=4)
    fog.sigma_t, fog.medium_albedo = 0.5, 0.8
    with tr.upload(fog) as dev:
        with pytest.raises(tr.TrhipError) as e:
            tr.render_transient(dev, nlos_area=True)
        assert e.value.status == STATUS_UNSUPPORTED
    wall_only = scenes.confocal_nlos(grid=4, n_tris=500, spp=4)
    wall_only.indices = wall_only.indices[:2]
    for f in ("mat_type", "albedo", "roughness"):
        setattr(wall_only, f, getattr(wall_only, f)[:2])
    with tr.upload(wall_only) as dev:
        with pytest.raises(tr.TrhipError) as e:
            tr.render_transient(dev, nlos_area=True)
        assert e.value.status == STATUS_UNSUPPORTED
