"""GPU forward-mode derivative (trhip_render_transient_tangent) against the
oracle's (|d dfilm| <= 1e-4 max|dfilm|, the gradient bar), the adjoint
identity on the GPU, and torch forward-mode AD through TransientRender."""
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


def _directions(sc, seed):
    rng = np.random.default_rng(seed)
    va = rng.uniform(-1.0, 1.0, sc.n_tris).astype(np.float32)
    vr = (rng.uniform(-1.0, 1.0, sc.n_tris) * (sc.mat_type == scenes.MAT_GGX)).astype(np.float32)
    return va, vr


def _check(tr, oracle_mod, sc, va, vr, pixels=None, **kw):
    import torch
    with tr.upload(sc) as dev:
        ta = None if va is None else torch.from_numpy(va).cuda()
        trr = None if vr is None else torch.from_numpy(vr).cuda()
        st, film, dfilm = tr.render_transient_tangent(dev, ta, trr, **kw)
        torch.cuda.synchronize()
        g_film = film.cpu().numpy().reshape(sc.n_pixels, sc.n_bins)
        g_d = dfilm.cpu().numpy().reshape(sc.n_pixels, sc.n_bins).astype(np.float64)
    ora_kw = {k: v for k, v in kw.items() if k in ("spp", "seed", "max_depth", "frozen")}
    o_film, o_d, _ = oracle_mod.Oracle(sc).render_tangent(va, vr, pixels=pixels, **ora_kw)
    if pixels is not None:
        g_film, g_d = g_film[pixels], g_d[pixels]
    compare_films(g_film, o_film, what="primal film")
    scale = np.abs(o_d).max()
    assert scale > 0
    assert np.abs(g_d - o_d).max() <= 1e-4 * scale, np.abs(g_d - o_d).max() / scale


@pytest.mark.parametrize("which", ["albedo", "roughness", "both"])
def test_tangent_matches_oracle(tr, oracle_mod, which):
    sc = scenes.diff_scene(sub=2, width=24, height=24, spp=64)
    va, vr = _directions(sc, 7)
    _announce(f"tangent vs oracle {which}")
    _check(tr, oracle_mod, sc, None if which == "roughness" else va, None if which == "albedo" else vr,
           frozen=True, max_depth=5)


def test_tangent_full_size_sampled(tr, oracle_mod):
    """The differentiable workload at full size (9,826 triangles, 64x64, 1024
    spp): the derivative along the roughness of the two boxes (one parameter
    pi_i as an indicator direction), 48 sampled pixels."""
    sc = scenes.diff_scene()
    vr = (sc.mat_type == scenes.MAT_GGX).astype(np.float32)
    pix = np.sort(np.random.default_rng(12).choice(sc.n_pixels, 48, replace=False)).astype(np.int32)
    _announce("tangent full size sampled")
    _check(tr, oracle_mod, sc, None, vr, pixels=pix, frozen=True)


def test_tangent_confocal(tr, oracle_mod):
    """Confocal NLOS: the derivative along the hidden blob's albedo."""
    sc = scenes.confocal_nlos(grid=12, spp=256)
    va = np.zeros(sc.n_tris, np.float32)
    va[:-2] = 1.0  # the blob; the last two triangles are the relay wall
    _announce("tangent confocal")
    _check(tr, oracle_mod, sc, va, None)


def test_tangent_is_transpose_of_adjoint_on_gpu(tr):
    import torch
    sc = scenes.diff_scene(sub=2, width=24, height=24, spp=64)
    va, vr = _directions(sc, 8)
    _announce("tangent/adjoint identity")
    with tr.upload(sc) as dev:
        _, film, dfilm = tr.render_transient_tangent(dev, torch.from_numpy(va).cuda(), torch.from_numpy(vr).cuda(),
                                                     frozen=True)
        delta = torch.randn(film.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
        ga, gr = tr.render_transient_backward(dev, delta, frozen=True)
        torch.cuda.synchronize()
        lhs = float((delta.double() * dfilm.double()).sum())
        rhs = float((ga.double().cpu() * torch.from_numpy(va).double()).sum()
                    + (gr.double().cpu() * torch.from_numpy(vr).double()).sum())
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_torch_forward_mode_ad(tr):
    """torch.autograd.forward_ad through TransientRender (its jvp) equals the
    tangent render."""
    import torch
    import torch.autograd.forward_ad as fwAD
    sc = scenes.diff_scene(sub=1, width=16, height=16, spp=32)
    va, vr = _directions(sc, 9)
    _announce("torch forward-mode AD")
    with tr.upload(sc) as dev:
        a = torch.from_numpy(sc.albedo).cuda()
        r = torch.from_numpy(sc.roughness).cuda()
        opts = {"spp": 32, "seed": 5}
        with fwAD.dual_level():
            out = tr.TransientRender.apply(fwAD.make_dual(a, torch.from_numpy(va).cuda()),
                                           fwAD.make_dual(r, torch.from_numpy(vr).cuda()), dev, opts)
            primal, tangent = fwAD.unpack_dual(out)
            film, dfilm = primal.clone(), tangent.clone()
        _, film2, dfilm2 = tr.render_transient_tangent(dev, torch.from_numpy(va).cuda(), torch.from_numpy(vr).cuda(),
                                                       albedo=a, roughness=r, **opts)
        torch.cuda.synchronize()
        np.testing.assert_allclose(film.cpu().numpy(), film2.cpu().numpy(), rtol=1e-5, atol=0)
        np.testing.assert_allclose(dfilm.cpu().numpy(), dfilm2.cpu().numpy(), rtol=1e-5,
                                   atol=1e-6 * float(dfilm2.abs().max()))
