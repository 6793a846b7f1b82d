"""Pins of the oracle's forward-mode derivative (Sec. 4.4): the adjoint
identity <dL/dfilm, dfilm> = <grad, direction> against the (separately
written) adjoint, and central finite differences of the film along the
direction (common random numbers; frozen GGX proposal for roughness)."""
import numpy as np
import pytest

from paper_2510_25660_amd import scenes


def _scene():
    return scenes.diff_scene(sub=2, width=16, height=16, spp=32)


def test_forward_mode_is_the_transpose_of_the_adjoint(oracle_mod):
    sc = _scene()
    O = oracle_mod.Oracle(sc)
    rng = np.random.default_rng(3)
    va = rng.normal(size=sc.n_tris)
    vr = rng.normal(size=sc.n_tris) * (sc.mat_type == scenes.MAT_GGX)
    film, dfilm, _ = O.render_tangent(va, vr, spp=32, frozen=True)
    delta = rng.normal(size=film.shape).astype(np.float32)
    ga, gr = O.backward(delta, spp=32, frozen=True)
    lhs = float((delta.astype(np.float64) * dfilm).sum())
    rhs = float((ga * va).sum() + (gr * vr).sum())
    assert abs(lhs) > 1e-3
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    assert np.abs(dfilm[film == 0]).max() == 0.0


@pytest.mark.parametrize("which", ["albedo", "roughness"])
def test_forward_mode_matches_finite_differences(oracle_mod, which):
    """Along a seeded direction: (film(p + eps v) - film(p - eps v)) / 2 eps
    per pixel-bin; the film is a polynomial in the albedos (exact up to
    rounding) and smooth in the frozen-proposal roughness."""
    sc = _scene()
    O = oracle_mod.Oracle(sc)
    rng = np.random.default_rng(4)
    v = rng.uniform(-1.0, 1.0, sc.n_tris)
    if which == "roughness":
        v *= (sc.mat_type == scenes.MAT_GGX)
    eps = 1e-3
    base_a, base_r = sc.albedo.astype(np.float64), sc.roughness.astype(np.float64)
    kw = dict(spp=32, frozen=True)
    if which == "albedo":
        _, dfilm, _ = O.render_tangent(v, None, **kw)
        fp, _, _ = O.render(albedo=(base_a + eps * v).astype(np.float32), **kw)
        fm, _, _ = O.render(albedo=(base_a - eps * v).astype(np.float32), **kw)
        # the float32 parameters actually used: their step is not exactly 2 eps v
        step = ((base_a + eps * v).astype(np.float32).astype(np.float64)
                - (base_a - eps * v).astype(np.float32).astype(np.float64))
        _, dstep, _ = O.render_tangent(step, None, **kw)
        fd = (fp - fm)
        scale = np.abs(dstep).max()
        assert np.abs(fd - dstep).max() <= 1e-4 * scale
    else:
        _, dfilm, _ = O.render_tangent(None, v, **kw)
        rp = (base_r + eps * v).astype(np.float32)
        rm = (base_r - eps * v).astype(np.float32)
        fp, _, _ = O.render(roughness=rp, **kw)
        fm, _, _ = O.render(roughness=rm, **kw)
        step = rp.astype(np.float64) - rm.astype(np.float64)
        _, dstep, _ = O.render_tangent(None, step, **kw)
        fd = (fp - fm)
        scale = np.abs(dstep).max()
        assert np.abs(fd - dstep).max() <= 2e-3 * scale
    assert np.abs(dfilm).max() > 0
