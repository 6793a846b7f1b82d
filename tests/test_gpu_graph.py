"""A render captured in a hipGraph (torch.cuda.graph) and replayed: every
replay, with eager work and synchronisations between the replays, equals the
eager render of the same samples (path and deferred forms; the deferred form
clears its sample-chunk film with a fill kernel, not a memset)."""
import sys

import numpy as np
import pytest

from paper_2510_25660_amd import scenes
from tests.parity import compare_films

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["box", "confocal"])
def test_graph_replays_equal_eager(name):
    import torch
    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    import paper_2510_25660_amd as tr
    sc = scenes.box_scene(width=32, height=32) if name == "box" else scenes.confocal_nlos(grid=8, n_tris=2000)
    _announce(f"graph replays {name}")
    with tr.upload(sc) as dev:
        eager_st, eager = tr.render_transient(dev)
        torch.cuda.synchronize()
        ref = eager.cpu().numpy().reshape(sc.n_pixels, -1).astype(np.float64)
        film = torch.empty_like(eager)
        steady = torch.empty_like(eager_st)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            tr.render_transient(dev, film=film, steady=steady)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            tr.render_transient(dev, film=film, steady=steady)
        for i in range(4):
            film.fill_(-1.0)
            _, other = tr.render_transient(dev, seed=99 + i)   # eager work between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            compare_films(film.cpu().numpy().reshape(sc.n_pixels, -1), ref, what=f"replay {i}")
        del graph
