"""Batched persistent rendering (one graph launch for many confocal scenes of
uneven size) against the single-scene forward render and the oracle."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films

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


def _small_batch(n=10, spp=64):
    return scenes.batched_nlos(n_scenes=n, spp=spp, tri_range=(300, 6000), grid_range=(4, 12),
                               bins_range=(256, 1024))


@pytest.mark.parametrize("autotune,kernel", [(False, "path"), (False, "deferred"), (True, "auto")])
def test_batch_matches_single_renders(tr, autotune, kernel):
    import torch
    scs = _small_batch()
    _announce(f"batch of {len(scs)} autotune={autotune} kernel={kernel}")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=autotune, kernel=kernel) as b:
            info = b.info()
            assert info["n_scenes"] == len(scs)
            # every scene has at least one item, and no item is empty
            assert len(scs) <= info["n_items"] <= sum(s.n_pixels for s in scs)
            films = [f.clone() for f in b.render()]
            torch.cuda.synchronize()
        for d, f in zip(devs, films):
            _, ref = tr.render_transient(d)
            torch.cuda.synchronize()
            a, r = f.cpu().numpy(), ref.cpu().numpy()
            assert ((a != 0) == (r != 0)).all()
            np.testing.assert_allclose(a, r, rtol=1e-5, atol=0)
    finally:
        for d in devs:
            d.destroy()


def test_batch_matches_oracle(tr, oracle_mod):
    import torch
    scs = _small_batch(n=4, spp=128)
    _announce("batch vs oracle")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=False) as b:
            films = [f.cpu().numpy() for f in b.render()]
            torch.cuda.synchronize()
        for s, f in zip(scs, films):
            o_film, _, _ = oracle_mod.Oracle(s).render()
            compare_films(f.reshape(s.n_pixels, s.n_bins), o_film)
    finally:
        for d in devs:
            d.destroy()


def test_batch_graph_replays(tr):
    """Replays of the captured graph, with eager work in between, each equal
    the first replay."""
    import torch
    scs = _small_batch(n=6, spp=32)
    _announce("batch graph replays")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=False) as b:
            first = [f.clone() for f in b.render()]
            torch.cuda.synchronize()
            for rep in range(3):
                junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
                for f in b.films:
                    f.fill_(-1.0)
                torch.cuda.synchronize()
                out = b.render()
                torch.cuda.synchronize()
                for a, c in zip(first, out):
                    np.testing.assert_allclose(c.cpu().numpy(), a.cpu().numpy(), rtol=1e-5, atol=0)
                del junk
    finally:
        for d in devs:
            d.destroy()


def test_batch_rejects_bad_input(tr):
    import ctypes as C
    from paper_2510_25660_amd import _binding as B
    sc = scenes.confocal_nlos(grid=4, n_tris=200, spp=8)
    dev = tr.upload(sc)
    try:
        L = B.lib()
        h = C.c_void_p()
        descs = (B.RenderDesc * 1)(tr.make_render_desc(dev, frozen=True))
        handles = (C.c_void_p * 1)(dev.handle.value)
        films = (C.c_void_p * 1)(None)
        assert L.trhip_batch_create(handles, descs, 1, films, None, None, C.byref(h)) == 1
        assert L.trhip_batch_render(C.c_void_p(1234), None) == 5
        assert L.trhip_batch_destroy(C.c_void_p(1234)) == 5
    finally:
        dev.destroy()


@pytest.mark.parametrize("big", [32768, 32769])
def test_batch_mixed_link_widths(tr, big):
    """A batch holding a scene at or above the 16-bit stack link limit next to
    small scenes (the whole batch then takes the wider links) against the
    single-scene renders."""
    import torch
    scs = _small_batch(n=3, spp=32) + [scenes.cluttered_box(big)]
    _announce(f"batch with cluttered box nt={big}")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=False) as b:
            films = [f.clone() for f in b.render()]
            torch.cuda.synchronize()
        for d, f in zip(devs, films):
            _, ref = tr.render_transient(d)
            torch.cuda.synchronize()
            a, r = f.cpu().numpy(), ref.cpu().numpy()
            assert ((a != 0) == (r != 0)).all()
            np.testing.assert_allclose(a, r, rtol=1e-5, atol=0)
    finally:
        for d in devs:
            d.destroy()


def test_tune_cache_file_reused_by_another_process(tr, tmp_path, monkeypatch):
    """The tuner writes its choice per scene class to TRHIP_TUNE_CACHE; a new
    process creating the same batch loads it instead of tuning again, and
    renders the same films."""
    import os
    import subprocess
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TRHIP_TUNE_CACHE", str(cache))
    scs = _small_batch(n=6, spp=32)
    _announce("tune cache file")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=True) as b:
            info = b.info()
            films = [f.cpu().numpy() for f in b.render()]
            torch.cuda.synchronize()
    finally:
        for d in devs:
            d.destroy()
    assert info["candidates"] > 0 and info["n_classes"] >= 1
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == info["n_classes"]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "films.npz")
    code = (f"import sys, numpy as np, torch; sys.path.insert(0, {root!r});"
            "import paper_2510_25660_amd as tr; from tests.test_gpu_batch import _small_batch;"
            "scs = _small_batch(n=6, spp=32); devs = [tr.upload(s) for s in scs];"
            "b = tr.Batch(devs, autotune=True); i = b.info(); f = [x.cpu().numpy() for x in b.render()];"
            "torch.cuda.synchronize();"
            f"np.savez({out!r}, *f); print('CANDIDATES', i['candidates'])")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TRHIP_TUNE_CACHE=str(cache)))
    assert r.returncode == 0, r.stderr[-3000:]
    assert "CANDIDATES 0" in r.stdout, r.stdout
    other = np.load(out)
    for k, f in enumerate(films):
        a = other[f"arr_{k}"]
        assert ((a != 0) == (f != 0)).all()
        np.testing.assert_allclose(a, f, rtol=1e-5, atol=0)
