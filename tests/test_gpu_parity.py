"""GPU (HIP, through the C ABI) against the CPU oracle on the same seeded
inputs: per pixel-bin values within 1e-4 relative on bins >= 1e-3 of the
peak, identical sets of non-zero bins, steady and out-of-window images."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films, compare_vec

pytestmark = pytest.mark.gpu

KERNELS = ["path", "deferred", "wavefront"]


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tr():
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    return tr


def _gpu_render(tr, sc, **kw):
    import torch
    with tr.upload(sc) as dev:
        steady, film, oow = tr.render_transient(dev, return_oow=True, **kw)
        torch.cuda.synchronize()
        return (film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins), steady.cpu().numpy().ravel(),
                oow.cpu().numpy().ravel(), dev.info())


def _check(tr, oracle_mod, sc, pixels=None, **kw):
    g_film, g_st, g_oow, info = _gpu_render(tr, sc, **kw)
    O = oracle_mod.Oracle(sc)
    ora_kw = {k: v for k, v in kw.items() if k in ("spp", "seed", "max_depth", "sample_offset", "stream_id",
                                                    "pixel_centre", "frozen")}
    o_film, o_st, o_oow = O.render(pixels=pixels, **ora_kw)
    if pixels is not None:
        g_film, g_st, g_oow = g_film[pixels], g_st[pixels], g_oow[pixels]
    err = compare_films(g_film, o_film)
    compare_vec(g_st, o_st, what="steady")
    if np.abs(o_oow).max() > 0:
        compare_vec(g_oow, o_oow, what="oow")
    assert o_film.sum() > 0
    return err, info


@pytest.mark.parametrize("kernel", KERNELS)
def test_box_scene_full(tr, oracle_mod, kernel):
    """The 34-triangle box room at its full size: 64x64, 256 bins, 16 spp, depth 4."""
    sc = scenes.box_scene()
    _announce(f"box 64x64x256 spp16 d4 {kernel}")
    err, info = _check(tr, oracle_mod, sc, kernel=kernel)
    assert info["n_triangles"] == 34


@pytest.mark.parametrize("kernel", KERNELS)
def test_box_scene_ragged_unwarp(tr, oracle_mod, kernel):
    """Odd film size (ragged last tile), camera unwarping, 5 spp, depth 6."""
    sc = scenes.box_scene(width=37, height=23, n_bins=300, bin_width=0.007, bin_start=0.3)
    sc.camera_unwarp = True
    _announce("box 37x23 unwarp")
    _check(tr, oracle_mod, sc, spp=5, max_depth=6, seed=99, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("tile,block", [(1, 64), (3, 128), (7, 256)])
def test_launch_shapes(tr, oracle_mod, tile, block, kernel):
    sc = scenes.box_scene(width=20, height=13)
    _announce(f"box launch shape tile={tile} block={block} {kernel}")
    _check(tr, oracle_mod, sc, spp=11, tile_pixels=tile, block_size=block, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_pixel_centre_plane(tr, oracle_mod, kernel):
    sc = scenes.plane_scene()
    _announce("plane pixel centre")
    _check(tr, oracle_mod, sc, spp=1, max_depth=2, pixel_centre=True, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_confocal_reduced(tr, oracle_mod, kernel):
    """Confocal NLOS, 9,682 triangles, 16x16 scan grid, 256 spp."""
    sc = scenes.confocal_nlos(grid=16, spp=256)
    _announce("confocal 16x16 spp256")
    err, info = _check(tr, oracle_mod, sc, kernel=kernel)
    assert info["n_triangles"] == 9682


@pytest.mark.parametrize("kernel", KERNELS)
def test_confocal_full_size_sampled(tr, oracle_mod, kernel):
    """Confocal NLOS at its full size (64x64 scan points, 4096 spp, 512 bins),
    the launch the benchmark times; the oracle recomputes 24 sampled rows."""
    sc = scenes.confocal_nlos()
    rng = np.random.default_rng(4)
    pix = np.sort(rng.choice(sc.n_pixels, 24, replace=False)).astype(np.int32)
    _announce(f"confocal 64x64 spp4096 sampled {kernel}")
    _check(tr, oracle_mod, sc, pixels=pix, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_ggx_fog_scene(tr, oracle_mod, kernel):
    """Terrain + spheres with GGX and Lambertian triangles in fog, depth 8."""
    sc = scenes.large_scene(cells=24, sphere_freq=4, grid=3, width=40, height=30, n_bins=256, bin_width=0.02,
                            spp=4)
    _announce(f"terrain+spheres fog ggx nt={sc.n_tris}")
    _check(tr, oracle_mod, sc, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_large_scene_full_size_sampled(tr, oracle_mod, kernel):
    """~1M triangles, 512x512 pixels, 1024 bins, 64 spp, depth 8, fog: the
    oracle recomputes 12 sampled pixels."""
    sc = scenes.large_scene()
    rng = np.random.default_rng(5)
    pix = np.sort(rng.choice(sc.n_pixels, 12, replace=False)).astype(np.int32)
    _announce(f"large nt={sc.n_tris} 512x512x1024 spp64 sampled {kernel}")
    err, info = _check(tr, oracle_mod, sc, pixels=pix, kernel=kernel)
    assert info["n_triangles"] == sc.n_tris


@pytest.mark.parametrize("kernel", KERNELS)
def test_sphere_furnace(tr, oracle_mod, kernel):
    sc = scenes.sphere_furnace(radius=1.003, freq=40, width=16, height=16)
    _announce("sphere furnace")
    _check(tr, oracle_mod, sc, spp=16, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n_tris", [1, 2, 3])
def test_tiny_bvh(tr, oracle_mod, n_tris, kernel):
    """Root-is-a-leaf and one/two internal-node BVHs."""
    sc = scenes.plane_scene(half=2.0)
    if n_tris == 1:
        sc.indices = sc.indices[:1].copy()
    elif n_tris == 3:
        extra = np.array([[0.0, 0.5, 0.0], [0.3, 0.5, 0.0], [0.0, 0.5, 0.3]], np.float32)
        sc.vertices = np.concatenate([sc.vertices, extra])
        sc.indices = np.concatenate([sc.indices, np.array([[4, 5, 6]], np.uint32)])
    nt = len(sc.indices)
    sc.mat_type = sc.mat_type[:1].repeat(nt)
    sc.albedo = sc.albedo[:1].repeat(nt)
    sc.roughness = sc.roughness[:1].repeat(nt)
    _announce(f"tiny bvh nt={nt}")
    _check(tr, oracle_mod, sc, spp=8, max_depth=3, kernel=kernel)


@pytest.mark.parametrize("kernel", KERNELS)
def test_time_sum_equals_steady_gpu(tr, kernel):
    sc = scenes.box_scene()
    _announce(f"sum over time {kernel}")
    film, st, oow, _ = _gpu_render(tr, sc, kernel=kernel)
    np.testing.assert_allclose(film.sum(1, dtype=np.float64) + oow, st, rtol=1e-5)


def test_accumulate_split_ranges(tr):
    """Samples [0,8) then [8,16) accumulated with norm_spp=16 equal one 16-spp render."""
    import torch
    sc = scenes.box_scene()
    _announce("accumulate")
    with tr.upload(sc) as dev:
        st, film = tr.render_transient(dev, spp=16)
        st2, film2 = tr.render_transient(dev, spp=8, norm_spp=16)
        tr.render_transient(dev, spp=8, sample_offset=8, norm_spp=16, accumulate=True, film=film2, steady=st2)
        torch.cuda.synchronize()
        np.testing.assert_allclose(film2.cpu().numpy(), film.cpu().numpy(), rtol=2e-6, atol=1e-9)
        np.testing.assert_allclose(st2.cpu().numpy(), st.cpu().numpy(), rtol=2e-6)


def test_kernel_forms_agree(tr):
    """Path-per-lane, deferred and wavefront forms give the same film (same
    paths, FP32 sums in a different order) with identical non-zero bins."""
    sc = scenes.large_scene(cells=32, sphere_freq=5, grid=3, width=48, height=40, n_bins=512, bin_width=0.01,
                            spp=8)
    _announce("path vs deferred vs wavefront")
    a = _gpu_render(tr, sc, kernel="path")[0]
    for form in ("deferred", "wavefront"):
        b = _gpu_render(tr, sc, kernel=form)[0]
        assert ((a != 0) == (b != 0)).all()
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=0)


def test_repeatable(tr):
    """Two renders with the same seed agree to FP32 summation order."""
    import torch
    sc = scenes.confocal_nlos(grid=8, spp=512)
    _announce("repeatable")
    with tr.upload(sc) as dev:
        a = tr.render_transient(dev)[1].cpu().numpy()
        b = tr.render_transient(dev)[1].cpu().numpy()
        torch.cuda.synchronize()
    assert ((a != 0) == (b != 0)).all()
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=0)


@pytest.mark.parametrize("make", ["confocal", "large_small", "furnace"])
def test_bvh_builders_agree(tr, make):
    """LBVH and PLOC trees give the same film: the closest hit is a function
    of the triangle set alone."""
    import torch
    if make == "confocal":
        sc = scenes.confocal_nlos(grid=16, spp=256)
    elif make == "large_small":
        sc = scenes.large_scene(cells=64, sphere_freq=8, grid=3, width=48, height=40, n_bins=256, spp=4)
    else:
        sc = scenes.sphere_furnace(radius=1.003, freq=40, width=16, height=16)
    _announce(f"builders {make}")
    out = {}
    for b in ("lbvh", "ploc"):
        with tr.upload(sc, builder=b) as dev:
            info = dev.info()
            assert info["bvh_internal_nodes"] == sc.n_tris - 1
            out[b] = tr.render_transient(dev)[1].cpu().numpy()
            torch.cuda.synchronize()
    a, c = out["lbvh"], out["ploc"]
    assert ((a != 0) == (c != 0)).all()
    np.testing.assert_allclose(a, c, rtol=1e-5, atol=0)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n_tris", [32768, 32769])
def test_stack_link_widths(tr, oracle_mod, n_tris, kernel):
    """Either side of the largest scene whose traversal stacks hold 16-bit
    links (32,768 triangles): both stack widths against the oracle."""
    sc = scenes.cluttered_box(n_tris)
    _announce(f"cluttered box nt={n_tris} {kernel}")
    err, info = _check(tr, oracle_mod, sc, kernel=kernel)
    assert info["n_triangles"] == n_tris


def test_deferred_sample_chunks(tr, oracle_mod):
    """More samples per pixel than one sort batch: the deferred form splits
    each pixel's samples over several workgroups that add their partial
    films atomically (fresh film, then accumulated onto an existing one)."""
    import torch
    sc = scenes.confocal_nlos(grid=8, spp=8192)
    _announce("deferred sample chunks 8x8 spp 8192")
    _check(tr, oracle_mod, sc, kernel="deferred")
    with tr.upload(sc) as dev:
        st, film = tr.render_transient(dev, kernel="deferred")
        st2, film2 = tr.render_transient(dev, kernel="deferred", spp=4096, norm_spp=8192)
        tr.render_transient(dev, kernel="deferred", spp=4096, sample_offset=4096, norm_spp=8192, accumulate=True,
                            film=film2, steady=st2)
        torch.cuda.synchronize()
        a, b = film.cpu().numpy(), film2.cpu().numpy()
    assert ((a != 0) == (b != 0)).all()
    np.testing.assert_allclose(b, a, rtol=1e-5, atol=0)
    np.testing.assert_allclose(st2.cpu().numpy(), st.cpu().numpy(), rtol=1e-5)


def test_hbm_film_accumulate_and_oracle(tr, oracle_mod):
    """A scene above the 16-bit link limit with a long film takes the path
    form with the film in HBM (float atomics, no LDS film): two accumulated
    sample ranges equal one render, and sampled pixels equal the oracle's
    film, steady image and out-of-window mass."""
    import torch
    sc = scenes.large_scene(cells=128, sphere_freq=8, grid=3, width=48, height=40, n_bins=512, bin_width=0.01,
                            spp=8)
    assert sc.n_tris > 32768
    _announce(f"hbm film nt={sc.n_tris} 48x40x512")
    with tr.upload(sc) as dev:
        st, film, oow = tr.render_transient(dev, return_oow=True)
        st2, film2, oow2 = tr.render_transient(dev, spp=4, norm_spp=8, return_oow=True)
        tr.render_transient(dev, spp=4, sample_offset=4, norm_spp=8, accumulate=True, film=film2, steady=st2,
                            oow=oow2)
        torch.cuda.synchronize()
        a, b = film.cpu().numpy(), film2.cpu().numpy()
        assert ((a != 0) == (b != 0)).all()
        np.testing.assert_allclose(b, a, rtol=2e-6, atol=1e-9)
        np.testing.assert_allclose(st2.cpu().numpy(), st.cpu().numpy(), rtol=2e-6)
        g_film = a.reshape(sc.n_pixels, sc.n_bins)
        g_st, g_oow = st.cpu().numpy().ravel(), oow.cpu().numpy().ravel()
    pix = np.sort(np.random.default_rng(9).choice(sc.n_pixels, 48, replace=False)).astype(np.int32)
    o_film, o_st, o_oow = oracle_mod.Oracle(sc).render(pixels=pix)
    compare_films(g_film[pix], o_film)
    compare_vec(g_st[pix], o_st, what="steady")
    if np.abs(o_oow).max() > 0:
        compare_vec(g_oow[pix], o_oow, what="oow")
