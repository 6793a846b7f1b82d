"""GPU adjoint (path replay, through the C ABI) against the oracle's adjoint,
against central finite differences of GPU renders, and its replayed primal
film against the forward film."""
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


def _setup(sub=2, res=16, spp=64):
    sc = scenes.diff_scene(sub=sub, width=res, height=res, spp=spp)
    ta, trough = scenes.perturbed_params(sc, seed=5)
    return sc, ta, trough


def test_adjoint_matches_oracle(tr, oracle_mod):
    import torch
    sc, ta, trough = _setup()
    spp, seed = 64, 77
    _announce("adjoint vs oracle")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(spp=spp, seed=seed, stream_id=1, albedo=ta, roughness=trough)
    film_o, _, _ = O.render(spp=spp, seed=seed)
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta, spp=spp, seed=seed)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr, primal = tr.render_transient_backward(dev, d, spp=spp, seed=seed, primal=True)
        _, film = tr.render_transient(dev, spp=spp, seed=seed)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
        primal = primal.cpu().numpy()
        film = film.cpu().numpy()
    compare_films(primal.reshape(sc.n_pixels, -1), film_o, what="primal film")
    compare_films(film.reshape(sc.n_pixels, -1), film_o, what="forward film")
    scale_a = np.abs(ga_o).max()
    scale_r = np.abs(gr_o).max()
    assert scale_a > 0 and scale_r > 0
    assert np.abs(ga - ga_o).max() <= 1e-4 * scale_a, np.abs(ga - ga_o).max() / scale_a
    assert np.abs(gr - gr_o).max() <= 1e-4 * scale_r, np.abs(gr - gr_o).max() / scale_r
    assert (gr[sc.mat_type == scenes.MAT_LAMBERT] == 0).all()


def test_adjoint_matches_gpu_finite_differences(tr):
    """Central differences (eps = 1e-3) of the GPU loss L = sum (I - I*)^2 on
    32 seeded parameters with |g| >= 1e-3 max|g|: 16 albedo, 16 GGX
    roughness (frozen proposal, so directions do not move with alpha)."""
    import torch
    sc, ta, trough = _setup(sub=2, res=24, spp=256)
    spp, seed, eps = 256, 21, 1e-3
    _announce("adjoint vs GPU finite differences")
    with tr.upload(sc) as dev:
        a0 = torch.from_numpy(sc.albedo).cuda()
        r0 = torch.from_numpy(sc.roughness).cuda()
        _, target = tr.render_transient(dev, spp=spp, seed=seed, stream_id=1,
                                        albedo=torch.from_numpy(ta).cuda(), roughness=torch.from_numpy(trough).cuda())
        _, film = tr.render_transient(dev, spp=spp, seed=seed, frozen=True, albedo=a0, roughness=r0)
        delta = 2.0 * (film - target)
        ga, gr = tr.render_transient_backward(dev, delta, spp=spp, seed=seed, frozen=True, albedo=a0, roughness=r0)
        torch.cuda.synchronize()
        ga_n = ga.cpu().numpy().astype(np.float64)
        gr_n = gr.cpu().numpy().astype(np.float64)
        tgt = target.double()

        def loss_diff(which, k):
            out = []
            for sgn in (1, -1):
                a = a0.clone()
                r = r0.clone()
                (a if which == "a" else r)[k] += sgn * eps
                _, f = tr.render_transient(dev, spp=spp, seed=seed, frozen=True, albedo=a, roughness=r)
                out.append(f.double())
            fp, fm = out
            return float(((fp - fm) * (fp + fm - 2 * tgt)).sum().item() / (2 * eps))

        rng = np.random.default_rng(8)
        ggx = np.flatnonzero(sc.mat_type == scenes.MAT_GGX)
        cand_a = np.flatnonzero(np.abs(ga_n) >= 1e-3 * np.abs(ga_n).max())
        cand_r = ggx[np.abs(gr_n[ggx]) >= 1e-3 * np.abs(gr_n[ggx]).max()]
        worst = 0.0
        for k in rng.choice(cand_a, size=min(16, len(cand_a)), replace=False):
            fd = loss_diff("a", int(k))
            worst = max(worst, abs(fd - ga_n[k]) / np.abs(ga_n).max())
        for k in rng.choice(cand_r, size=min(16, len(cand_r)), replace=False):
            fd = loss_diff("r", int(k))
            worst = max(worst, abs(fd - gr_n[k]) / np.abs(gr_n).max())
    print(f"worst FD deviation / max|g| = {worst:.2e}")
    assert worst <= 5e-3


def test_autograd_function(tr):
    import torch
    sc, ta, trough = _setup(sub=1, res=16, spp=32)
    _announce("autograd")
    with tr.upload(sc) as dev:
        a = torch.from_numpy(sc.albedo).cuda().requires_grad_(True)
        r = torch.from_numpy(sc.roughness).cuda().requires_grad_(True)
        film = tr.TransientRender.apply(a, r, dev, {"spp": 32, "seed": 3})
        loss = (film ** 2).sum()
        loss.backward()
        ga, gr = tr.render_transient_backward(dev, 2 * film.detach(), spp=32, seed=3, albedo=a.detach(),
                                              roughness=r.detach())
        torch.cuda.synchronize()
        np.testing.assert_allclose(a.grad.cpu().numpy(), ga.cpu().numpy(), rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(r.grad.cpu().numpy(), gr.cpu().numpy(), rtol=1e-5, atol=1e-12)
