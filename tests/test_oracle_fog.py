"""Pins of the oracle's participating-medium branches (paper Sec. 4.1,
volumetric scattering with analog free flight; Eqs. 3-4 for the time of
flight, Eq. 8 for the connection factors).

* a plane inside homogeneous fog, one vertex per path at pixel centres: a
  path reaches the plane with probability exp(-sigma_t t) (t the camera ray's
  distance to the plane), and then contributes exactly
  rho I cos / (pi r^2) exp(-sigma_t r) at bin floor((t + r - b_start)/b_width);
  otherwise it scatters in the fog at s < t, distributed as the exponential
  law truncated to [0, t), and contributes alpha I exp(-sigma_t r_s) /
  (4 pi r_s^2) at time s + r_s;
* the medium's phase sampler draws directions uniformly on the sphere (z
  uniform in [-1, 1], azimuth uniform), checked by Kolmogorov-Smirnov;
* double scattering in fog without surfaces: the second vertex's mean
  contribution equals a 2-D quadrature of the exponential integral form
  (the average over isotropic directions and exponential distances from
  the first vertex, in closed form in the distance to the light).

Each pin is a function that raises AssertionError; the last tests compile
copies of the oracle with a planted mistake (the surface connection's
transmittance dropped, the free-flight decision reversed, the phase sampler
restricted to a hemisphere) and check that the pins fail on them.
"""
import math
import os
import re
import subprocess

import numpy as np
import pytest
from scipy import integrate, optimize, special, stats

from paper_2510_25660_amd import scenes

SIGMA_T, MED_ALB, RHO = 0.35, 0.8, 0.6


def _pixel_dirs(sc):
    W, H = sc.width, sc.height
    ix, iy = np.meshgrid(np.arange(W), np.arange(H))
    fx = ix.ravel() + 0.5
    fy = iy.ravel() + 0.5
    sx = (2 * fx / W - 1) * sc.tan_x
    sy = (1 - 2 * fy / H) * sc.tan_y
    d = (np.asarray(sc.cam_fwd, np.float64)[None] + sx[:, None] * np.asarray(sc.cam_right, np.float64)[None]
         + sy[:, None] * np.asarray(sc.cam_up, np.float64)[None])
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _fog_plane():
    return scenes.plane_scene(h=1.0, albedo=RHO, width=4, height=4, sigma_t=SIGMA_T, medium_albedo=MED_ALB)


def check_plane_in_fog(oracle_mod, pixels=(0, 5, 10, 15), n=3000):
    sc = _fog_plane()
    O = oracle_mod.Oracle(sc)
    d_all = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    hits, expect_hits, var_hits, pit = 0, 0.0, 0.0, []
    for p in pixels:
        d = d_all[p]
        t = -o[1] / d[1]
        x = o + t * d
        r = np.linalg.norm(x - light)
        v_surf = RHO * 1.0 * (light[1] / r) / (math.pi * r**2) * math.exp(-SIGMA_T * r)
        q = (t + r - sc.bin_start) / sc.bin_width
        p_reach = math.exp(-SIGMA_T * t)
        expect_hits += n * p_reach
        var_hits += n * p_reach * (1 - p_reach)

        def opl_of(s):
            return s + np.linalg.norm(o + s * d - light)

        for s_idx in range(n):
            path = O.trace(p, s_idx, max_depth=2, pixel_centre=True)
            assert len(path) == 1, path
            v = path[0]
            assert v["has_c"] == 1
            if v["tri"] >= 0:
                hits += 1
                assert abs(v["c"] - v_surf) <= 2e-5 * v_surf, ("surface value", p, v["c"], v_surf)
                assert abs(v["opl_c"] - (t + r)) <= 1e-5 * (t + r), ("surface time", p, v["opl_c"], t + r)
                if abs(q - round(q)) > 1e-2:
                    assert v["bin"] == int(math.floor(q)), ("surface bin", p, v["bin"], q)
            else:
                # scattered in the fog before the plane: recover s from the time
                assert v["opl_c"] <= t + r + 1e-5, ("medium time beyond the surface's", v["opl_c"], t + r)
                s = optimize.brentq(lambda z: opl_of(z) - v["opl_c"], 0.0, t, xtol=1e-12)
                rs = np.linalg.norm(o + s * d - light)
                c = MED_ALB * 1.0 * math.exp(-SIGMA_T * rs) / (4 * math.pi * rs**2)
                assert abs(v["c"] - c) <= 2e-4 * c, ("medium value", p, v["c"], c, s)
                pit.append((1 - math.exp(-SIGMA_T * s)) / (1 - math.exp(-SIGMA_T * t)))
    z = (hits - expect_hits) / math.sqrt(var_hits)
    assert abs(z) < 5, ("paths reaching the plane", hits, expect_hits, z)
    ks = stats.kstest(np.array(pit), "uniform")
    assert ks.pvalue > 1e-4, ("medium vertex distance law", ks)


def test_plane_in_fog(oracle_mod):
    check_plane_in_fog(oracle_mod)


def check_plane_in_fog_steady(oracle_mod, spp=20000):
    """The steady image's expectation per pixel: the surface term times the
    probability of reaching it, plus the single-scattering integral over
    the fog in front of the plane."""
    sc = _fog_plane()
    O = oracle_mod.Oracle(sc)
    film, steady, oow = O.render(spp=spp, max_depth=2, pixel_centre=True)
    d_all = _pixel_dirs(sc)
    o = np.asarray(sc.cam_origin, np.float64)
    light = np.asarray(sc.light_pos, np.float64)
    for p in range(sc.n_pixels):
        d = d_all[p]
        t = -o[1] / d[1]
        r = np.linalg.norm(o + t * d - light)
        v_surf = RHO * (light[1] / r) / (math.pi * r**2) * math.exp(-SIGMA_T * r)

        def c_med(s):
            rs = np.linalg.norm(o + s * d - light)
            return MED_ALB * math.exp(-SIGMA_T * rs) / (4 * math.pi * rs**2)

        dens = lambda s: SIGMA_T * math.exp(-SIGMA_T * s)
        m1 = math.exp(-SIGMA_T * t) * v_surf + integrate.quad(lambda s: dens(s) * c_med(s), 0, t)[0]
        m2 = math.exp(-SIGMA_T * t) * v_surf**2 + integrate.quad(lambda s: dens(s) * c_med(s) ** 2, 0, t)[0]
        se = math.sqrt((m2 - m1**2) / spp)
        assert abs(steady[p] - m1) < 5 * se, (p, steady[p], m1, se)
    np.testing.assert_allclose(film.sum(1) + oow, steady, rtol=1e-12)


def test_plane_in_fog_steady(oracle_mod):
    check_plane_in_fog_steady(oracle_mod)


def check_phase_sampler(oracle_mod, n=200_000):
    rng = np.random.default_rng(17)
    u0 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    w = oracle_mod.phase_sample_n(u0, u1).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=3e-7)
    assert stats.kstest(w[:, 2], "uniform", args=(-1.0, 2.0)).pvalue > 1e-4, "z not uniform in [-1, 1]"
    phi = np.mod(np.arctan2(w[:, 1], w[:, 0]), 2 * np.pi)
    assert stats.kstest(phi, "uniform", args=(0.0, 2 * np.pi)).pvalue > 1e-4, "azimuth not uniform"
    # uniform on the sphere: each coordinate is U[-1, 1] (Archimedes)
    for k in (0, 1):
        assert stats.kstest(w[:, k], "uniform", args=(-1.0, 2.0)).pvalue > 1e-4, f"coordinate {k}"


def test_phase_sampler_isotropic(oracle_mod):
    check_phase_sampler(oracle_mod)


def _second_order_mean(sigma_t, alb, light):
    """E[contribution of the second medium vertex] for the camera ray along
    -z from the origin in fog without surfaces, I = 1.  The average of
    exp(-sigma_t u) / (4 pi u^2) over an isotropic direction and an
    exponential distance s from a point at distance rho from the light is,
    with u^2 = rho^2 + s^2 + 2 rho s mu and du = rho s / u dmu,
    (E1(sigma_t |rho - s|) - E1(sigma_t (rho + s))) / (8 pi rho s)."""
    light = np.asarray(light, np.float64)

    def h(rho):
        f = lambda s: (sigma_t * math.exp(-sigma_t * s) *
                       (special.exp1(sigma_t * abs(rho - s)) - special.exp1(sigma_t * (rho + s))) /
                       (8 * math.pi * rho * s))
        a = integrate.quad(f, 0, rho, limit=200)[0]
        b = integrate.quad(f, rho, np.inf, limit=200)[0]
        return a + b

    def outer(s1):
        x1 = np.array([0.0, 0.0, -s1])
        return sigma_t * math.exp(-sigma_t * s1) * alb * alb * h(np.linalg.norm(x1 - light))

    return integrate.quad(outer, 0, np.inf, limit=200, epsabs=0, epsrel=1e-7)[0]


def check_double_scattering(oracle_mod, batches=16, spp=25_000):
    sigma_t, alb = 0.5, 0.8
    light = (0.0, 1.0, -2.0)
    sc = scenes.fog_only(sigma_t=sigma_t, albedo=alb, n_bins=512, bin_width=0.05, light=light)
    O = oracle_mod.Oracle(sc)
    second = []
    for b in range(batches):
        _, s3, _ = O.render(spp=spp, max_depth=3, pixel_centre=True, sample_offset=b * spp)
        _, s2, _ = O.render(spp=spp, max_depth=2, pixel_centre=True, sample_offset=b * spp)
        second.append(s3[0] - s2[0])  # the same paths: depth 3 adds the second vertex
    second = np.array(second)
    mean = second.mean()
    sem = second.std(ddof=1) / math.sqrt(batches)
    expect = _second_order_mean(sigma_t, alb, light)
    assert abs(mean - expect) < 5 * sem + 1e-4 * expect, ("second-order scattering", mean, expect, sem)


def test_double_scattering_quadrature(oracle_mod):
    check_double_scattering(oracle_mod)


# ---------------------------------------------------------------------------
# planted mistakes: each pin must fail on a copy of the oracle carrying one
# ---------------------------------------------------------------------------
PLANTS = {
    "surface_connection_without_transmittance": (
        r"if \(has_medium && !inside\) c = c \* expf\(-\(sc->sigma_t \* dist\)\);", "",
        [check_plane_in_fog]),
    "free_flight_decision_reversed": (
        r"if \(!hit \|\| t_ff < t_hit\) \{", "if (!hit || t_ff > t_hit) {",
        [check_plane_in_fog, check_plane_in_fog_steady]),
    "phase_sampler_hemisphere": (
        r"float z = 1\.0f - \(u0 \+ u0\);", "float z = 1.0f - u0;",
        [check_phase_sampler, check_double_scattering]),
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistake_is_caught(oracle_mod, tmp_path, plant):
    pattern, repl, checks = PLANTS[plant]
    src = open(oracle_mod.SRC_PATH).read()
    planted, n = re.subn(pattern, repl, src)
    assert n == 1, f"the planted line must occur exactly once ({n})"
    c_path = tmp_path / "oracle.c"
    c_path.write_text(planted)
    so = str(tmp_path / "liboracle_planted.so")
    inc = os.path.dirname(oracle_mod.SRC_PATH)
    subprocess.check_call(["gcc", *oracle_mod.CFLAGS, "-I", inc, "-o", so, str(c_path), "-lm"])
    with oracle_mod.using_library(so):
        for check in checks:
            with pytest.raises(AssertionError):
                check(oracle_mod)
