"""Contribution-by-contribution parity (Sec. 3, "Path reuse and
histogramming": each next-event contribution c of a path of time of flight
tof lands in bin floor((tof - b_start) / b_width)).

The recording build of each kernel form lists every contribution of a set
of pixels (pixel, sample, vertex, bin, value, tof, triangle) while it
renders; the oracle lists the same from its own paths.  The two lists must
hold the same (pixel, sample, vertex) keys, the same bin and triangle for
each, the same time of flight bit for bit, and the same value bit for bit
(within a few ulp where a transmittance exp() enters: the device and host
exponentials are different implementations).  A contribution moved by one
bin, or a contribution present on one side only, fails here even where the
summed film would hide it.  Full-size workloads, sampled pixels, all three
kernel forms.
"""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes

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


_SCENES = {}
_ORACLES = {}


def _scene(name):
    """Scenes built once per module (their oracles too, in _run)."""
    if name not in _SCENES:
        sc = {
            "box": lambda: scenes.box_scene(),
            "confocal": lambda: scenes.confocal_nlos(),
            "large": lambda: scenes.large_scene(),
            "layers": lambda: scenes.layered_scene(),
            "confocal_big": lambda: scenes.confocal_nlos(grid=16, n_tris=40000, spp=512),
            "glass": lambda: scenes.glass_box_scene(delay_mean=0.05, width=24, height=24),
            "fog_small": lambda: scenes.large_scene(cells=24, sphere_freq=4, grid=3, width=40, height=30,
                                                    n_bins=256, bin_width=0.02, spp=8),
        }[name]()
        _SCENES[name] = sc
    return _SCENES[name]


def _ulps(a, b):
    """Distance in units in the last place between float32 arrays of equal sign."""
    ia = a.astype(np.float32).view(np.int32).astype(np.int64)
    ib = b.astype(np.float32).view(np.int32).astype(np.int64)
    same_sign = np.sign(a) == np.sign(b)
    d = np.abs(ia - ib)
    return np.where(same_sign, d, np.iinfo(np.int64).max)


def _sorted(r):
    return r[np.lexsort((r["vertex"], r["sample"], r["pixel"]))]


def compare_records(g, o, value_ulps=0, what="records"):
    g = _sorted(g)
    o = _sorted(o)
    assert len(g) == len(o), f"{what}: {len(g)} GPU contributions, {len(o)} oracle contributions"
    assert len(o) > 0, f"{what}: no contribution to compare"
    for f in ("pixel", "sample", "vertex", "bin", "tri"):
        bad = np.flatnonzero(g[f] != o[f])
        assert bad.size == 0, (f"{what}: field {f} differs in {bad.size} of {len(o)} contributions; first: "
                               f"gpu {g[bad[:3]]}, oracle {o[bad[:3]]}")
    d_tof = _ulps(g["tof"], o["tof"])
    d_val = _ulps(g["value"], o["value"])
    print(f"[records] {what}: {len(o)} contributions, bins identical, tof max {d_tof.max()} ulp, "
          f"value max {d_val.max()} ulp ({np.mean(d_val == 0):.4f} bit-identical)", flush=True)
    assert d_tof.max() == 0, f"{what}: time of flight differs by up to {d_tof.max()} ulp"
    assert d_val.max() <= value_ulps, f"{what}: value differs by up to {d_val.max()} ulp"
    return len(o)


def _run(tr, oracle_mod, name, pixels, kernel, **kw):
    import torch
    sc = _scene(name)
    _announce(f"records {name} ({sc.n_tris} tris, {sc.width}x{sc.height}x{sc.n_bins}) {len(pixels)} pixels "
              f"{kernel} {kw}")
    with tr.upload(sc) as dev:
        g, steady, film, oow = tr.render_transient_records(dev, pixels, kernel=kernel, **kw)
        torch.cuda.synchronize()
        film = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
    if name not in _ORACLES:
        _ORACLES[name] = oracle_mod.Oracle(sc)
    O = _ORACLES[name]
    o = O.records(pixels, **{k: v for k, v in kw.items() if k in ("spp", "seed", "max_depth", "nlos_area",
                                                                   "pixel_centre", "sample_offset")})
    # the recording build renders the same film: every listed contribution
    # is in it (the film of the pixels equals the records' histogram)
    spp = kw.get("spp", sc.spp)
    for p in pixels[:4]:
        rp = o[(o["pixel"] == p) & (o["bin"] >= 0)]
        hist = np.zeros(sc.n_bins)
        np.add.at(hist, rp["bin"], rp["value"].astype(np.float64))
        hist /= spp
        nz = hist != 0
        assert np.array_equal(film[p] != 0, nz), f"pixel {p}: film bins differ from the record histogram's"
        if nz.any():
            np.testing.assert_allclose(film[p][nz], hist[nz], rtol=2e-5)
    return g, o, sc


def _pixels(n_pixels, n, seed):
    return np.sort(np.random.default_rng(seed).choice(n_pixels, size=n, replace=False)).astype(np.int64)


@pytest.mark.parametrize("kernel", KERNELS)
def test_records_box_full(tr, oracle_mod, kernel):
    """Box room at full size (64x64, 256 bins, 16 spp, depth 4), 64 pixels."""
    g, o, sc = _run(tr, oracle_mod, "box", _pixels(64 * 64, 64, 1), kernel)
    compare_records(g, o, what=f"box {kernel}")


@pytest.mark.parametrize("kernel", KERNELS)
def test_records_confocal_full(tr, oracle_mod, kernel):
    """Confocal NLOS at full size (64x64 scan, 9,680-triangle blob, 512 bins,
    4096 spp), 12 scan points."""
    g, o, sc = _run(tr, oracle_mod, "confocal", _pixels(64 * 64, 12, 2), kernel)
    compare_records(g, o, what=f"confocal {kernel}")


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_records_confocal_area_sampling(tr, oracle_mod, kernel):
    """Confocal NLOS at full size with NLOS area sampling, 8 scan points."""
    g, o, sc = _run(tr, oracle_mod, "confocal", _pixels(64 * 64, 8, 3), kernel, nlos_area=True)
    compare_records(g, o, what=f"confocal area sampling {kernel}")


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_records_area_sampling_compact_layout(tr, oracle_mod, kernel):
    """NLOS area sampling on a 40,000-triangle blob (32-bit links, compact
    layout: the sampled triangle is read from the 64-byte records through
    the caller-to-BVH-order map), cosine sampling too, 8 scan points."""
    for area in (True, False):
        g, o, sc = _run(tr, oracle_mod, "confocal_big", _pixels(16 * 16, 8, 12), kernel, nlos_area=area)
        compare_records(g, o, what=f"confocal 40k tris {kernel} area={area}")


@pytest.mark.parametrize("kernel", KERNELS)
def test_records_large_full(tr, oracle_mod, kernel):
    """The 998,608-triangle fogged terrain at full size (512x512, 1024 bins,
    64 spp, depth 8), 24 pixels; fog transmittance enters the values."""
    g, o, sc = _run(tr, oracle_mod, "large", _pixels(512 * 512, 24, 4), kernel)
    compare_records(g, o, value_ulps=4, what=f"large {kernel}")


@pytest.mark.parametrize("kernel", KERNELS)
def test_records_glass_delays(tr, oracle_mod, kernel):
    """Glass box (index 1.5) in the box room with scattering delays, depth 8."""
    g, o, sc = _run(tr, oracle_mod, "glass", _pixels(24 * 24, 48, 5), kernel, spp=16, max_depth=8)
    compare_records(g, o, value_ulps=0, what=f"glass {kernel}")


@pytest.mark.parametrize("kernel", KERNELS)
def test_records_fog_ggx(tr, oracle_mod, kernel):
    """Small terrain with GGX spheres in fog, depth 8, every pixel."""
    g, o, sc = _run(tr, oracle_mod, "fog_small", np.arange(40 * 30), kernel)
    compare_records(g, o, value_ulps=4, what=f"fog+GGX {kernel}")


def test_records_capacity_and_mask(tr):
    """Only marked pixels are listed; the count reports every contribution
    even when the buffer is too small."""
    import torch
    sc = scenes.box_scene(width=16, height=16, spp=4)
    _announce("records capacity")
    with tr.upload(sc) as dev:
        g, _, film, _ = tr.render_transient_records(dev, [3, 7])
        assert set(np.unique(g["pixel"])) <= {3, 7}
        n = len(g)
        assert n > 0
        with pytest.raises(ValueError):
            tr.render_transient_records(dev, [3, 7], capacity=max(1, n - 1))
        _, ref = tr.render_transient(dev)
        torch.cuda.synchronize()
        np.testing.assert_allclose(film.cpu().numpy(), ref.cpu().numpy(), rtol=1e-5, atol=0)


def test_records_deep_stacks(tr, oracle_mod):
    """262,144 stacked layers (524,288 triangles, 512 bins): the path form
    keeps the film in HBM and splits each lane's stack between 16 words of
    LDS and scratch memory.  Every camera ray crosses all layers' boxes, so
    its traversal holds about as many pending far children as the tree has
    levels and uses the scratch words on every ray; the contributions must
    still match the oracle's (own median-split BVH) bit for bit."""
    sc = _scene("layers")
    with tr.upload(sc) as dev:
        depth = dev.info()["bvh_depth"]
    assert 16 + 2 < depth <= 16 + 48, f"tree depth {depth}: the scene no longer reaches the scratch words"
    g, o, sc = _run(tr, oracle_mod, "layers", _pixels(sc.n_pixels, 32, 9), "path", spp=8)
    compare_records(g, o, what="layers path")
    _announce("layers: whole film against the LDS-stack path form")
    import torch
    with tr.upload(sc) as dev:
        _, film = tr.render_transient(dev, kernel="path")
        _, film_w = tr.render_transient(dev, kernel="wavefront")
        torch.cuda.synchronize()
        a, b = film.cpu().numpy(), film_w.cpu().numpy()
    assert np.count_nonzero(a) > 0
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * float(np.abs(b).max()))


def test_records_large_whole_lds_stacks(tr, oracle_mod, monkeypatch):
    """The 1M-triangle fog scene's path form with whole stacks in LDS
    (TRHIP_SPLIT_STACK=0: the kernel kept for trees deeper than the split
    stack holds), contribution by contribution against the oracle, and its
    film against the split-stack render's."""
    import torch
    monkeypatch.setenv("TRHIP_SPLIT_STACK", "0")
    g, o, sc = _run(tr, oracle_mod, "large", _pixels(512 * 512, 16, 10), "path")
    compare_records(g, o, value_ulps=4, what="large path, whole LDS stacks")
    _announce("large: film with whole LDS stacks against split stacks")
    with tr.upload(sc) as dev:
        _, a = tr.render_transient(dev, kernel="path", spp=8)
        monkeypatch.setenv("TRHIP_SPLIT_STACK", "1")
        _, b = tr.render_transient(dev, kernel="path", spp=8)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.count_nonzero(a) > 0
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * float(np.abs(b).max()))


@pytest.mark.parametrize("kernel", ["path", "deferred"])
def test_records_compact_layout_axis_rays(tr, oracle_mod, kernel):
    """The compact layout's node test orders each axis's two planes by the
    sign of the ray's direction (the FP16 pair rotated where it is
    negative).  Seen straight down the stacked layers through pixel
    centres of an odd-sized image, the middle row and column cast rays with
    a zero direction component, and the centre pixel a ray along the axis:
    every contribution must still match the oracle's."""
    import dataclasses
    base = scenes.layered_scene(n_layers=16385, width=15, height=15, spp=2)
    sc = dataclasses.replace(base, **scenes.look_at([0.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, -1.0], 50.0,
                                                      15, 15))
    assert sc.cam_fwd == (0.0, -1.0, 0.0) and sc.cam_right == (1.0, 0.0, 0.0)
    name = "layers_axis"
    _SCENES[name] = sc
    _announce(f"records compact layout, axis-aligned rays: {sc.n_tris} tris, {kernel}")
    g, o, _ = _run(tr, oracle_mod, name, np.arange(sc.n_pixels, dtype=np.int64), kernel, pixel_centre=True)
    centre = (sc.height // 2) * sc.width + sc.width // 2
    assert np.count_nonzero(o["pixel"] == centre) > 0
    compare_records(g, o, what=f"layers, axis-aligned rays ({kernel})")


@pytest.mark.parametrize("scale", [1e-5, 1e5])
def test_records_compact_layout_extreme_scales(tr, oracle_mod, scale):
    """The compact layout (scenes above 32,768 triangles) stores child boxes
    as FP16 rounded outward.  Scaled by 1e5, coordinates pass FP16's largest
    finite value (boxes become infinite); scaled by 1e-5, layers 1e-10 apart
    share their FP16 bounds.  Traversal gets slower, the result must not
    change: contributions identical to the oracle's."""
    import dataclasses
    base = scenes.layered_scene(n_layers=16385, spp=2)
    k = np.float32(scale)
    sc = dataclasses.replace(
        base, vertices=(base.vertices * k).astype(np.float32),
        cam_origin=tuple(float(np.float32(v) * k) for v in base.cam_origin),
        light_pos=tuple(float(np.float32(v) * k) for v in base.light_pos),
        bin_start=float(np.float32(base.bin_start) * k), bin_width=float(np.float32(base.bin_width) * k))
    _announce(f"records compact layout at scale {scale}: {sc.n_tris} tris")
    name = f"layers_scaled_{scale}"
    _SCENES[name] = sc
    g, o, _ = _run(tr, oracle_mod, name, _pixels(sc.n_pixels, 24, 11), "path")
    compare_records(g, o, what=f"layers x{scale:g}")
