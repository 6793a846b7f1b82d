"""trhip_render_transient_noalloc, called through the C ABI, against
trhip_render_transient on the same scenes: the same film, steady and
out-of-window images (identical non-zero bins, values to the 1e-4 bar),
for two calls in a row, the second on a smaller input; renders whose
scratch would not fit the static array are rejected."""
import ctypes as C
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


def _both(tr, sc, **kw):
    """(film, steady, oow) of trhip_render_transient_noalloc and of
    trhip_render_transient, each called through the C ABI."""
    import torch
    from paper_2510_25660_amd._binding import check, lib
    out = []
    with tr.upload(sc) as dev:
        r = tr.make_render_desc(dev, **kw)
        stream = torch.cuda.current_stream().cuda_stream
        for fn in (lib().trhip_render_transient_noalloc, lib().trhip_render_transient):
            film = torch.full((sc.n_pixels, sc.n_bins), float("nan"), device="cuda", dtype=torch.float32)
            steady = torch.full((sc.n_pixels,), float("nan"), device="cuda", dtype=torch.float32)
            oow = torch.full((sc.n_pixels,), float("nan"), device="cuda", dtype=torch.float32)
            check(fn(dev.handle, C.byref(r), film.data_ptr(), steady.data_ptr(), oow.data_ptr(), stream))
            torch.cuda.synchronize()
            out.append((film.cpu().numpy(), steady.cpu().numpy(), oow.cpu().numpy()))
    return out


def _check_pair(pair, what):
    (fa, sa, oa), (fb, sb, ob) = pair
    assert np.isfinite(fa).all() and np.isfinite(sa).all() and np.isfinite(oa).all(), f"{what}: unwritten output"
    assert fa.sum() > 0, what
    compare_films(fa, fb, what=f"{what} film")
    compare_vec(sa, sb, what=f"{what} steady")
    if np.abs(ob).max() > 0:
        compare_vec(oa, ob, what=f"{what} oow")


def test_noalloc_matches_render_two_calls(tr):
    # the full confocal scan: the deferred form splits each scan point's 4096
    # samples into two chunks, whose partial film goes through the static
    # scratch; then a smaller scan, which reuses the scratch's first part
    big = scenes.confocal_nlos()
    _announce("noalloc confocal 64x64x512 4096 spp (two sample chunks)")
    _check_pair(_both(tr, big), "confocal full")
    small = scenes.confocal_nlos(grid=24, n_tris=4000, n_bins=300, spp=4096)
    _announce("noalloc confocal 24x24x300 4096 spp")
    _check_pair(_both(tr, small), "confocal small")


def test_noalloc_other_forms(tr):
    """Forms without scratch (path per lane, deterministic) pass through."""
    sc = scenes.box_scene(width=32, height=32, spp=16)
    _announce("noalloc box path form and deterministic")
    _check_pair(_both(tr, sc), "box")
    (fa, sa, oa), (fb, sb, ob) = _both(tr, sc, deterministic=True)
    assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32))


def test_noalloc_rejects_oversized_scratch(tr):
    import torch
    from paper_2510_25660_amd._binding import lib
    sc = scenes.confocal_nlos(grid=64, n_tris=2000, n_bins=2048, spp=4096)  # 4096 x 2048 floats of partial film
    _announce("noalloc oversized")
    with tr.upload(sc) as dev:
        r = tr.make_render_desc(dev)
        film = torch.empty((sc.n_pixels, sc.n_bins), device="cuda", dtype=torch.float32)
        st = lib().trhip_render_transient_noalloc(dev.handle, C.byref(r), film.data_ptr(), None, None,
                                                  torch.cuda.current_stream().cuda_stream)
        assert st == 4, st  # UNSUPPORTED
        assert b"scratch" in lib().trhip_last_error()
