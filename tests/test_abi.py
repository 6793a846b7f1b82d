"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/trhip.h declares, and rejects invalid
arguments before any HIP call."""
import copy
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2510_25660_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_2510_25660_amd import build
        build.build()
    return _binding


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "trhip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)   # drop comments
    return sorted(set(re.findall(r"\b(trhip_\w+)\s*\(", src)))


def test_exports_every_declared_symbol(B):
    L = B.lib()
    declared = _declared_symbols()
    assert len(declared) >= 8
    for name in declared:
        assert hasattr(L, name), f"{name} declared in trhip.h but not exported"
    assert set(B.EXPORTED_SYMBOLS) <= set(declared)


def test_version_and_status_strings(B):
    L = B.lib()
    assert b"gfx950" in L.trhip_version()
    for code, name in [(0, b"ok"), (1, b"invalid argument"), (5, b"bad handle")]:
        assert L.trhip_status_string(code) == name
    assert L.trhip_status_string(12345) == b"unknown status"


def _desc(sc):
    import paper_2510_25660_amd as tr
    return tr.make_scene_desc(sc)


def test_scene_create_validation(B):
    from paper_2510_25660_amd import scenes
    L = B.lib()
    h = C.c_void_p()
    assert L.trhip_scene_create(None, None, C.byref(h)) == 1
    sc = scenes.box_scene()
    d, keep = _desc(sc)
    assert L.trhip_scene_create(C.byref(d), None, None) == 1

    def expect_invalid(mutate, msg):
        d2, keep2 = _desc(copy.deepcopy(sc))
        mutate(d2, keep2)
        st = L.trhip_scene_create(C.byref(d2), None, C.byref(h))
        assert st == 1, (msg, st)
        assert msg in L.trhip_last_error().decode(), L.trhip_last_error()

    expect_invalid(lambda d, k: setattr(d, "n_bins", 0), "n_bins")
    expect_invalid(lambda d, k: setattr(d, "bin_width", 0.0), "bin_width")
    expect_invalid(lambda d, k: setattr(d, "bin_width", float("nan")), "bin_width")
    expect_invalid(lambda d, k: setattr(d, "width", 0), "no pixels")
    expect_invalid(lambda d, k: setattr(d, "sensor", 7), "unknown sensor")
    expect_invalid(lambda d, k: setattr(d, "n_triangles", 0), "empty scene")
    expect_invalid(lambda d, k: setattr(d, "sigma_t", -1.0), "sigma_t")
    expect_invalid(lambda d, k: setattr(d, "n_vertices", 3), "index out of range")

    def zero_area(d, k):
        k[0][k[1][0, 1]] = k[0][k[1][0, 0]]   # collapse one edge of triangle 0
    expect_invalid(zero_area, "zero area")

    def bad_albedo(d, k):
        k[3][5] = 0.0
    expect_invalid(bad_albedo, "albedo")

    def nan_vertex(d, k):
        k[0][3, 1] = np.nan
    expect_invalid(nan_vertex, "not finite")

    def bad_mat(d, k):
        k[2][0] = 9
    expect_invalid(bad_mat, "unknown material")


def test_dielectric_and_delay_validation(B):
    """Refractive indices and scattering delays are checked on the host
    before any device call."""
    from paper_2510_25660_amd import scenes
    L = B.lib()
    h = C.c_void_p()
    sc = scenes.glass_box_scene(delay_mean=0.05)

    def expect_invalid(mutate, msg):
        d, keep = _desc(copy.deepcopy(sc))
        mutate(d, keep)
        st = L.trhip_scene_create(C.byref(d), None, C.byref(h))
        assert st == 1, (msg, st)
        assert msg in L.trhip_last_error().decode(), L.trhip_last_error()

    expect_invalid(lambda d, k: setattr(d, "ior", None), "ior is NULL")

    def bad_ior(d, k):
        k[5][12] = 0.0           # a triangle of the glass box
    expect_invalid(bad_ior, "ior must lie")

    def nan_ior(d, k):
        k[5][12] = np.nan
    expect_invalid(nan_ior, "ior must lie")

    def bad_delay(d, k):
        k[6][0] = -1.0
    expect_invalid(bad_delay, "delay")

    def inf_delay(d, k):
        k[6][0] = np.inf
    expect_invalid(inf_delay, "delay")
    expect_invalid(lambda d, k: setattr(d, "medium_ior", -1.0), "medium_ior")
    expect_invalid(lambda d, k: setattr(d, "medium_ior", float("nan")), "medium_ior")


def test_confocal_validation(B):
    from paper_2510_25660_amd import scenes
    L = B.lib()
    h = C.c_void_p()
    sc = scenes.confocal_nlos(grid=4, n_tris=200)
    d, keep = _desc(sc)
    d.scan_points = None
    assert L.trhip_scene_create(C.byref(d), None, C.byref(h)) == 1
    assert b"scan_points" in L.trhip_last_error()
    d, keep = _desc(sc)
    d.camera_unwarp = 1
    assert L.trhip_scene_create(C.byref(d), None, C.byref(h)) == 1


def test_bad_handles(B):
    L = B.lib()
    r = B.RenderDesc()
    r.spp = 1
    r.max_depth = 2
    fake = C.c_void_p(0xdeadbeef)
    assert L.trhip_render_transient(fake, C.byref(r), C.c_void_p(16), None, None, None) == 5
    assert L.trhip_render_transient(None, C.byref(r), C.c_void_p(16), None, None, None) == 5
    assert L.trhip_render_transient_backward(fake, C.byref(r), None, None, None, None, None) == 5
    assert L.trhip_scene_destroy(fake) == 5
    assert L.trhip_scene_destroy(None) == 0
    info = B.SceneInfo()
    assert L.trhip_scene_get_info(fake, C.byref(info)) == 5


def test_poisson_noise_validation(B):
    """Invalid noise arguments are rejected on the host, before any HIP call."""
    L = B.lib()
    assert L.trhip_poisson_noise(None, None, 0, 1.0, 0, None) == 0
    assert L.trhip_poisson_noise(None, C.c_void_p(16), 4, 1.0, 0, None) == 1
    assert L.trhip_poisson_noise(C.c_void_p(16), None, 4, 1.0, 0, None) == 1
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        assert L.trhip_poisson_noise(C.c_void_p(16), C.c_void_p(16), 4, bad, 0, None) == 1
    assert b"scale" in L.trhip_last_error()


def test_product_path_has_no_oracle_or_fallback():
    """The package never imports the oracle and has no CPU rendering path."""
    pkg = os.path.join(ROOT, "paper_2510_25660_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.h" not in text, f


def test_records_and_probe_validation(B):
    """The recording render and the numerics probe reject invalid arguments
    on the host, before any HIP call."""
    L = B.lib()
    r = B.RenderDesc()
    r.spp = 1
    r.max_depth = 2
    n = C.c_uint64(0)
    fake = C.c_void_p(0xdeadbeef)
    assert L.trhip_render_transient_records(fake, C.byref(r), C.c_void_p(16), C.c_void_p(16), 4, C.byref(n),
                                            C.c_void_p(16), None, None, None) == 5
    assert L.trhip_numerics_probe(-1, None, C.c_void_p(16), 4, 0, None) == 1
    assert L.trhip_numerics_probe(5, None, C.c_void_p(16), 4, 0, None) == 1
    assert L.trhip_numerics_probe(0, None, None, 4, 0, None) == 1
    assert L.trhip_numerics_probe(2, None, C.c_void_p(16), 4, 0, None) == 1   # Philox needs its input
    assert L.trhip_numerics_probe(1, None, C.c_void_p(16), 16, (1 << 24) - 8, None) == 1
    assert b"2^24" in L.trhip_last_error()
    assert L.trhip_numerics_probe(3, None, None, 0, 0, None) == 0   # nothing to do
