"""The batched workload at full size: all 256 confocal scenes (blob triangles
log-uniform in 1k-50k, so about a tenth of them above the 32,768 triangles of
16-bit stack links; scan grids 16^2-64^2; 256-1024 bins of 2.4 mm; 256 spp;
3 bounces) rendered by the tuned persistent graph launch.  Every scene's film
equals its single render (identical non-zero bins, 1e-4 on bins >= 1e-3 of
the peak), and sampled scan points of eight scenes (the most triangles, a
64^2 grid, the fewest triangles and five random ones) equal the oracle's."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_full_batch_against_single_renders_and_oracle(oracle_mod):
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    scs = scenes.batched_nlos()
    assert len(scs) == 256
    big = [i for i, s in enumerate(scs) if s.n_tris > 32768]
    assert big, "the batch must hold scenes above the 16-bit link limit"
    _announce(f"full batch: 256 scenes, {sum(s.n_tris for s in scs)} triangles, {len(big)} above 32,768")
    devs = [tr.upload(s) for s in scs]
    try:
        with tr.Batch(devs, autotune=True) as b:
            info = b.info()
            print(f"[batch] {info}", flush=True)
            films = [f.cpu().numpy() for f in b.render()]
            torch.cuda.synchronize()
        for i, (d, s) in enumerate(zip(devs, scs)):
            _, ref = tr.render_transient(d)
            torch.cuda.synchronize()
            compare_films(films[i].reshape(s.n_pixels, s.n_bins), ref.cpu().numpy().reshape(s.n_pixels, s.n_bins),
                          what=f"scene {i} ({s.n_tris} tris, {s.width}^2, {s.n_bins} bins)")
    finally:
        for d in devs:
            d.destroy()
    rng = np.random.default_rng(256)
    pick = [int(np.argmax([s.n_tris for s in scs])), int(np.argmin([s.n_tris for s in scs]))]
    pick += [i for i, s in enumerate(scs) if s.width == 64][:1]
    pick += [int(i) for i in rng.choice(len(scs), 5, replace=False)]
    for i in dict.fromkeys(pick):
        s = scs[i]
        pix = np.sort(rng.choice(s.n_pixels, 4, replace=False)).astype(np.int32)
        _announce(f"batch scene {i} vs oracle ({s.n_tris} tris, {s.width}^2, {s.n_bins} bins), 4 scan points")
        o_film, _, _ = oracle_mod.Oracle(s).render(pixels=pix)
        g = films[i].reshape(s.n_pixels, s.n_bins)[pix]
        if o_film.sum() > 0:
            compare_films(g, o_film, what=f"scene {i} vs oracle")
        else:
            assert not g.any()
