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


@pytest.mark.parametrize("mode", ["replay", "stash"])
@pytest.mark.parametrize("depth", [4, 6])
def test_adjoint_matches_oracle(tr, oracle_mod, mode, depth):
    """Single-trace (register stash) and path-replay adjoints against the
    oracle's adjoint, at 3 and 5 vertices per path."""
    import torch
    sc, ta, trough = _setup()
    spp, seed = 64, 77
    _announce(f"adjoint vs oracle {mode} depth {depth}")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(spp=spp, seed=seed, max_depth=depth, stream_id=1, albedo=ta, roughness=trough)
    film_o, _, _ = O.render(spp=spp, seed=seed, max_depth=depth)
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta, spp=spp, seed=seed, max_depth=depth)
    kernel = "path" if mode == "replay" else "auto"
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr, primal = tr.render_transient_backward(dev, d, spp=spp, seed=seed, max_depth=depth, primal=True,
                                                      kernel=kernel)
        _, film = tr.render_transient(dev, spp=spp, seed=seed, max_depth=depth)
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


def test_adjoint_full_size_sampled_pixels(tr, oracle_mod):
    """The differentiable workload at full size (9,826 triangles, 64x64, 256
    bins, 1024 spp, depth 4) in the launch the benchmark times, with
    dL/dfilm non-zero on 64 sampled pixels only, so that the oracle's adjoint
    over exactly those pixels is the reference."""
    import torch
    sc = scenes.diff_scene()
    ta, trough = scenes.perturbed_params(sc, seed=5)
    rng = np.random.default_rng(31)
    pix = np.sort(rng.choice(sc.n_pixels, 64, replace=False)).astype(np.int32)
    _announce("adjoint full size, sampled pixels")
    O = oracle_mod.Oracle(sc)
    tgt, _, _ = O.render(pixels=pix, stream_id=1, albedo=ta, roughness=trough)
    cur, _, _ = O.render(pixels=pix)
    delta = np.zeros((sc.n_pixels, sc.n_bins), np.float32)
    delta[pix] = 2.0 * (cur - tgt)
    ga_o, gr_o = O.backward(delta, pixels=pix)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr = tr.render_transient_backward(dev, d)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
    assert np.abs(ga - ga_o).max() <= 1e-4 * np.abs(ga_o).max()
    assert np.abs(gr - gr_o).max() <= 1e-4 * np.abs(gr_o).max()
    assert (np.abs(ga_o) > 0).sum() > 100


def test_adjoint_full_size_finite_differences(tr):
    """Full-size differentiable workload: GPU adjoint against central
    differences (eps 1e-3) of GPU renders on 32 seeded parameters with
    |g| >= 1e-3 max|g| (16 albedo, 16 GGX roughness, frozen proposal)."""
    import torch
    sc = scenes.diff_scene()
    ta, trough = scenes.perturbed_params(sc, seed=5)
    eps = 1e-3
    _announce("adjoint full size vs finite differences")
    with tr.upload(sc) as dev:
        a0 = torch.from_numpy(sc.albedo).cuda()
        r0 = torch.from_numpy(sc.roughness).cuda()
        _, target = tr.render_transient(dev, stream_id=1, albedo=torch.from_numpy(ta).cuda(),
                                        roughness=torch.from_numpy(trough).cuda())
        _, film = tr.render_transient(dev, frozen=True, albedo=a0, roughness=r0)
        ga, gr = tr.render_transient_backward(dev, 2.0 * (film - target), frozen=True, albedo=a0, roughness=r0)
        torch.cuda.synchronize()
        ga_n, gr_n = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
        tgt = target.double()

        def fd(which, k):
            out = []
            for sgn in (1, -1):
                a = a0.clone()
                r = r0.clone()
                (a if which == "a" else r)[k] += sgn * eps
                out.append(tr.render_transient(dev, frozen=True, albedo=a, roughness=r)[1].double())
            return float(((out[0] - out[1]) * (out[0] + out[1] - 2 * tgt)).sum().item() / (2 * eps))

        rng = np.random.default_rng(32)
        ggx = np.flatnonzero(sc.mat_type == scenes.MAT_GGX)
        cand_a = np.flatnonzero(np.abs(ga_n) >= 1e-3 * np.abs(ga_n).max())
        cand_r = ggx[np.abs(gr_n[ggx]) >= 1e-3 * np.abs(gr_n[ggx]).max()]
        worst = 0.0
        for k in rng.choice(cand_a, 16, replace=False):
            worst = max(worst, abs(fd("a", int(k)) - ga_n[k]) / np.abs(ga_n).max())
        for k in rng.choice(cand_r, 16, replace=False):
            worst = max(worst, abs(fd("r", int(k)) - gr_n[k]) / np.abs(gr_n).max())
    print(f"full-size worst FD deviation / max|g| = {worst:.2e}")
    assert worst <= 5e-3


@pytest.mark.parametrize("kernel", ["path", "auto"])
@pytest.mark.parametrize("n_tris", [32768, 32769])
def test_adjoint_stack_link_widths(tr, oracle_mod, n_tris, kernel):
    """Adjoint (replay and stash) on scenes either side of the 16-bit stack
    link limit, against the oracle's adjoint."""
    import torch
    sc = scenes.cluttered_box(n_tris)
    ta, trough = scenes.perturbed_params(sc, seed=6)
    _announce(f"adjoint cluttered box nt={n_tris} {kernel}")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(stream_id=1, albedo=ta, roughness=trough)
    film_o, _, _ = O.render()
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta)
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr = tr.render_transient_backward(dev, d, kernel=kernel)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
    assert np.abs(ga_o).max() > 0 and np.abs(gr_o).max() > 0
    assert np.abs(ga - ga_o).max() <= 1e-4 * np.abs(ga_o).max()
    assert np.abs(gr - gr_o).max() <= 1e-4 * np.abs(gr_o).max()


@pytest.mark.parametrize("kernel", ["path", "auto"])
def test_adjoint_gradient_table_overflow(tr, oracle_mod, kernel):
    """One workgroup renders the whole 16 x 16 image of a box cluttered with
    20,000 small triangles (8,192 paths), so its paths touch far more
    triangles than the workgroup's 512-slot LDS gradient table holds: the
    overflow goes to the global gradients directly.  Both adjoints against
    the oracle's."""
    import torch
    sc = scenes.cluttered_box(20000, width=16, height=16, n_bins=16, bin_width=0.16, spp=32)
    ta, trough = scenes.perturbed_params(sc, seed=7)
    _announce(f"adjoint gradient table overflow {kernel}")
    O = oracle_mod.Oracle(sc)
    target, _, _ = O.render(stream_id=1, albedo=ta, roughness=trough)
    film_o, _, _ = O.render()
    delta = (2.0 * (film_o - target)).astype(np.float32)
    ga_o, gr_o = O.backward(delta)
    assert np.count_nonzero(ga_o) > 2 * 512  # one tile touched them all
    with tr.upload(sc) as dev:
        d = torch.from_numpy(delta.reshape(sc.height, sc.width, sc.n_bins)).cuda()
        ga, gr = tr.render_transient_backward(dev, d, kernel=kernel, tile_pixels=sc.n_pixels, block_size=256)
        torch.cuda.synchronize()
        ga, gr = ga.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)
    assert np.abs(ga - ga_o).max() <= 1e-4 * np.abs(ga_o).max()
    assert np.abs(gr - gr_o).max() <= 1e-4 * np.abs(gr_o).max()
