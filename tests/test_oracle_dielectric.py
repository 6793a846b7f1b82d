"""Pins of the oracle's refractive indices, dielectric interface and
scattering delays (Eq. 3: a segment's time of flight is its length times
the index it runs in; Eq. 10: the delays of the path's vertices add to its
time of flight).

* Fresnel reflectance: normal incidence ((n-1)/(n+1))^2, Brewster's angle
  (the p amplitude vanishes: F = cos^2(2 theta_B) / 2), total internal
  reflection beyond the critical angle, reciprocity F(theta_i, 1->n) =
  F(theta_t, n->1), grazing incidence -> 1.
* A camera looking into a closed glass tank that holds a plane and the
  light: every pixel (pixel centre) has one non-zero bin, at the optical
  path |c-x1| + n |x1-x2| + n |x2-l| (Snell's law for x2), holding
  c / n^2 per transmitted sample (radiance leaving glass is divided by
  n^2); the count of transmitted samples is binomial with 1 - F.
* A camera looking through a glass slab at a plane: the ray leaves the slab
  parallel to its incident direction, shifted; value c per sample that
  crosses both faces (probability (1 - F)^2), time |c-x1| + n |x1-x2| +
  |x2-x3| + |x3-l|.
* Scattering delay with mean tau on a plane: the single-bounce contribution
  spreads over the bins as c (e^{-(a-t0)/tau} - e^{-(b-t0)/tau}) (chi-square
  over all pixels); the steady image is unchanged.
* An index eta around the meshes scales every time of flight by eta and
  leaves the steady image bit for bit unchanged.
* The adjoint with a glass box in the room equals central finite
  differences of the oracle's loss.
"""
import math

import numpy as np
import pytest

from paper_2510_25660_amd import scenes


def _pixel_dirs(sc):
    W, H = sc.width, sc.height
    ix, iy = np.meshgrid(np.arange(W), np.arange(H))
    sx = (2 * (ix.ravel() + 0.5) / W - 1) * sc.tan_x
    sy = (1 - 2 * (iy.ravel() + 0.5) / H) * sc.tan_y
    d = (np.asarray(sc.cam_fwd, np.float64)[None] + sx[:, None] * np.asarray(sc.cam_right, np.float64)[None]
         + sy[:, None] * np.asarray(sc.cam_up, np.float64)[None])
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _fresnel_angles(ti, n):
    """Fresnel's equations in angle form, light from index 1 into n."""
    tt = np.arcsin(np.sin(ti) / n)
    if np.isscalar(ti) and ti == 0:
        return ((n - 1) / (n + 1)) ** 2
    rs = -np.sin(ti - tt) / np.sin(ti + tt)
    rp = np.tan(ti - tt) / np.tan(ti + tt)
    return 0.5 * (rs**2 + rp**2)


def _refract_down(d, n):
    """Vector Snell's law for a ray going down (-z) into a horizontal
    interface from index 1 into n: the tangential part shrinks by 1/n."""
    tang = d[:, :2] / n
    z = -np.sqrt(1.0 - (tang**2).sum(1))
    return np.concatenate([tang, z[:, None]], 1)


def test_fresnel_special_values(oracle_mod):
    F = oracle_mod.lib().orc_fresnel
    for n in (1.33, 1.5, 2.4):
        assert abs(F(1.0, 1.0, n) - ((n - 1) / (n + 1)) ** 2) < 1e-6
        assert abs(F(1.0, n, 1.0) - ((n - 1) / (n + 1)) ** 2) < 1e-6
        tb = math.atan(n)                        # Brewster
        assert abs(F(math.cos(tb), 1.0, n) - 0.5 * math.cos(2 * tb) ** 2) < 2e-6
        tc = math.asin(1.0 / n)                  # critical angle from inside
        assert F(math.cos(tc + 1e-3), n, 1.0) == 1.0
        assert F(math.cos(tc - 1e-2), n, 1.0) < 1.0
        for ti in (0.2, 0.7, 1.2):               # reciprocity
            tt = math.asin(math.sin(ti) / n)
            assert abs(F(math.cos(ti), 1.0, n) - F(math.cos(tt), n, 1.0)) < 2e-6
            assert abs(F(math.cos(ti), 1.0, n) - _fresnel_angles(ti, n)) < 2e-6
        assert F(1e-4, 1.0, n) > 0.999           # grazing


def _one_bin_per_pixel(film, steady, value, q, spp):
    """Pixel-centre renders: each pixel holds value * k / spp in exactly one
    bin (k transmitted samples) -- returns k per pixel after checking the
    bin (away from edges) and that k is an integer."""
    ks = []
    checked = 0
    for p in range(film.shape[0]):
        nz = np.flatnonzero(film[p])
        if len(nz) == 0:
            ks.append(0)
            continue
        assert len(nz) == 1
        k = film[p, nz[0]] * spp / value[p]
        assert abs(k - round(k)) < 1e-3 * max(1.0, k), (p, k)
        assert abs(steady[p] - film[p, nz[0]]) <= 1e-9 * steady[p]
        ks.append(int(round(k)))
        # ray origins leaving a surface are offset by up to ~256 ulps of
        # the coordinates (3e-5 m here), which shifts the optical path of
        # the next segment: compare bins 0.1 bin (1e-4 m) away from an edge
        if abs(q[p] - round(q[p])) > 0.1:
            assert nz[0] == int(math.floor(q[p])), (p, nz[0], q[p])
            checked += 1
    assert checked > 0.7 * film.shape[0]
    return np.array(ks)


@pytest.mark.parametrize("n", [1.33, 1.5])
def test_glass_tank_closed_form(oracle_mod, n):
    sc = scenes.glass_tank_scene(ior=n)
    spp = 256
    film, steady, oow = oracle_mod.Oracle(sc).render(spp=spp, pixel_centre=True)
    d = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    t1 = (1.0 - o[2]) / d[:, 2]
    x1 = o[None] + t1[:, None] * d
    dt = _refract_down(d, n)
    s = (-0.5 - 1.0) / dt[:, 2]
    x2 = x1 + s[:, None] * dt
    r = np.linalg.norm(light[None] - x2, axis=1)
    cos_l = (light[2] - x2[:, 2]) / r
    value = (0.6 / math.pi) * cos_l / r**2 / n**2
    opl = t1 + n * s + n * r
    q = (opl - sc.bin_start) / sc.bin_width
    k = _one_bin_per_pixel(film, steady, value, q, spp)
    T = 1.0 - _fresnel_angles(np.arccos(-d[:, 2]), n)
    mean, var = spp * T.sum(), spp * (T * (1 - T)).sum()
    assert abs(k.sum() - mean) < 5 * math.sqrt(var) + 1, (k.sum(), mean)
    assert (oow == 0).all()


def test_glass_slab_closed_form(oracle_mod):
    n = 1.5
    sc = scenes.glass_slab_scene(ior=n)
    spp = 256
    film, steady, _ = oracle_mod.Oracle(sc).render(spp=spp, pixel_centre=True)
    d = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    t1 = (1.0 - o[2]) / d[:, 2]
    x1 = o[None] + t1[:, None] * d
    dt = _refract_down(d, n)
    s = (0.8 - 1.0) / dt[:, 2]
    x2 = x1 + s[:, None] * dt
    t3 = (0.0 - 0.8) / d[:, 2]          # leaves parallel to the incident ray
    x3 = x2 + t3[:, None] * d
    r = np.linalg.norm(light[None] - x3, axis=1)
    cos_l = (light[2] - x3[:, 2]) / r
    value = (0.5 / math.pi) * cos_l / r**2
    opl = t1 + n * s + t3 + r
    q = (opl - sc.bin_start) / sc.bin_width
    k = _one_bin_per_pixel(film, steady, value, q, spp)
    T2 = (1.0 - _fresnel_angles(np.arccos(-d[:, 2]), n)) ** 2
    mean, var = spp * T2.sum(), spp * (T2 * (1 - T2)).sum()
    assert abs(k.sum() - mean) < 5 * math.sqrt(var) + 1, (k.sum(), mean)


def test_scattering_delay_exponential(oracle_mod):
    tau = 0.05
    sc = scenes.plane_scene(h=1.0, albedo=0.6, width=8, height=8, n_bins=400, bin_width=0.005, bin_start=2.0)
    base_film, base_steady, _ = oracle_mod.Oracle(sc).render(spp=1, max_depth=2, pixel_centre=True)
    sc.delay = np.full(sc.n_tris, tau, np.float32)
    spp = 4096
    film, steady, oow = oracle_mod.Oracle(sc).render(spp=spp, max_depth=2, pixel_centre=True)
    c = base_steady                                   # every sample adds c, whatever its delay
    assert np.allclose(steady, c, rtol=1e-6)
    np.testing.assert_allclose(film.sum(1) + oow, steady, rtol=1e-9)
    d = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    t = -o[1] / d[:, 1]
    x = o[None] + t[:, None] * d
    t0 = t + np.linalg.norm(x - light[None], axis=1)
    edges = sc.bin_start + sc.bin_width * np.arange(sc.n_bins + 1)
    chi2, dof = 0.0, 0
    for p in range(sc.n_pixels):
        counts = film[p] * spp / c[p]
        assert np.allclose(counts, np.round(counts), atol=1e-3)
        cdf = 1.0 - np.exp(-np.maximum(edges - t0[p], 0.0) / tau)
        prob = np.diff(cdf)
        tail = 1.0 - cdf[-1]
        obs = np.append(np.round(counts), round(oow[p] * spp / c[p]))
        exp_ = spp * np.append(prob, tail)
        big = exp_ >= 5
        o_, e_ = np.append(obs[big], obs[~big].sum()), np.append(exp_[big], exp_[~big].sum())
        keep = e_ > 0
        chi2 += (((o_ - e_) ** 2)[keep] / e_[keep]).sum()
        dof += keep.sum() - 1
        # nothing before the undelayed arrival
        assert film[p, : max(0, int(math.floor((t0[p] - sc.bin_start) / sc.bin_width)) - 1)].sum() == 0
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof), (chi2, dof)


def test_medium_ior_scales_time(oracle_mod):
    eta = 1.33
    sc = scenes.plane_scene(h=1.0, albedo=0.6, n_bins=16384)
    film1, steady1, _ = oracle_mod.Oracle(sc).render(spp=1, max_depth=2, pixel_centre=True)
    sc.medium_ior = eta
    film, steady, oow = oracle_mod.Oracle(sc).render(spp=1, max_depth=2, pixel_centre=True)
    assert np.array_equal(steady, steady1)
    d = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    t = -o[1] / d[:, 1]
    x = o[None] + t[:, None] * d
    q = (eta * (t + np.linalg.norm(x - light[None], axis=1)) - sc.bin_start) / sc.bin_width
    checked = 0
    for p in range(sc.n_pixels):
        nz = np.flatnonzero(film[p])
        assert len(nz) == 1 and film[p, nz[0]] == steady[p]
        if abs(q[p] - round(q[p])) > 1e-2:
            assert nz[0] == int(math.floor(q[p]))
            checked += 1
    assert checked > 0.9 * sc.n_pixels


def test_adjoint_with_glass_matches_finite_differences(oracle_mod):
    """Albedo gradients of L = sum (I - I*)^2 on the room seen through and
    around the glass box (the film is a polynomial in the albedos at a fixed
    seed, so central differences are exact up to rounding)."""
    sc = scenes.glass_box_scene(width=12, height=12, spp=32, max_depth=6)
    O = oracle_mod.Oracle(sc)
    spp, seed = 32, 3
    rng = np.random.default_rng(2)
    ta = np.clip(sc.albedo + rng.uniform(-0.1, 0.1, sc.n_tris), 0.05, 0.95).astype(np.float32)
    target, _, _ = O.render(spp=spp, seed=seed, stream_id=1, albedo=ta)
    film, _, _ = O.render(spp=spp, seed=seed)
    ga, gr = O.backward((2.0 * (film - target)).astype(np.float32), spp=spp, seed=seed)
    assert (ga[sc.mat_type == scenes.MAT_DIELECTRIC] == 0).all() and (gr == 0).all()
    eps = 1e-3
    idx = [k for k in np.argsort(-np.abs(ga))[:8]]
    assert abs(ga[idx[0]]) > 0
    for k in idx:
        ap, am = sc.albedo.copy(), sc.albedo.copy()
        ap[k] += eps
        am[k] -= eps
        fp, _, _ = O.render(spp=spp, seed=seed, albedo=ap)
        fm, _, _ = O.render(spp=spp, seed=seed, albedo=am)
        fd = (((fp - fm) * (fp + fm - 2.0 * target)).sum()) / (2 * eps)
        assert abs(fd - ga[k]) <= 1e-4 * np.abs(ga).max() + 1e-3 * abs(ga[k]), (k, fd, ga[k])
