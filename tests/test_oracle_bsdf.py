"""Pins of the oracle's BSDFs by integral identities and consistency
conditions (no formula is re-typed here):

* cosine sampling: cos^2(theta) ~ U[0,1], azimuth ~ U[0, 2 pi), unit length;
* GGX visible-normal pdf: integrates to 1 over the sphere of reflected
  directions (upper-hemisphere quadrature + the sampler's below-horizon mass);
* the visible-normal sampler's histogram matches its pdf;
* sample weight == f cos / pdf (so sampler, pdf and f are mutually consistent);
* reciprocity f(a, b) == f(b, a); energy: integral of f cos <= F;
* d log f / d alpha == central finite difference of log f.
"""
import numpy as np
import pytest
from scipy import stats


def _dirs(theta):
    return np.stack([np.sin(theta), np.zeros_like(theta), np.cos(theta)], 1)


def test_cosine_sampling_distribution(oracle_mod):
    rng = np.random.default_rng(3)
    n = 200_000
    u0 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    w = oracle_mod.cosine_sample_n(u0, u1).astype(np.float64)
    assert np.abs(np.linalg.norm(w, axis=1) - 1.0).max() < 1e-6
    assert (w[:, 2] > 0).all()
    assert stats.kstest(w[:, 2] ** 2, "uniform").pvalue > 1e-3
    phi = (np.arctan2(w[:, 1], w[:, 0]) / (2 * np.pi)) % 1.0
    assert stats.kstest(phi, "uniform").pvalue > 1e-3


def _hemisphere_grid(n_mu=1500, n_phi=720):
    mu = (np.arange(n_mu) + 0.5) / n_mu
    phi = (np.arange(n_phi) + 0.5) / n_phi * 2 * np.pi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    s = np.sqrt(1 - M**2)
    wi = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
    dw = (1.0 / n_mu) * (2 * np.pi / n_phi)
    return wi, dw


@pytest.mark.parametrize("alpha,theta_o", [(0.2, 0.3), (0.5, 0.0), (0.5, 1.1), (0.35, 0.8)])
def test_ggx_pdf_normalisation_and_energy(oracle_mod, alpha, theta_o):
    wo = _dirs(np.array([theta_o]))[0]
    wi, dw = _hemisphere_grid()
    f, pdf = oracle_mod.ggx_eval_n(np.broadcast_to(wo, wi.shape), wi, alpha, 1.0)
    upper = pdf.astype(np.float64).sum() * dw
    # mass the sampler sends below the horizon (its weight is 0 there)
    rng = np.random.default_rng(5)
    n = 400_000
    u0 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    ws, wt = oracle_mod.ggx_sample_n(np.broadcast_to(wo, (n, 3)), alpha, 1.0, u0, u1)
    below = np.mean(ws[:, 2] <= 0)
    assert abs(upper + below - 1.0) < 3e-3, (upper, below)
    # energy: integral of f cos over the hemisphere is at most F = 1 and equals
    # the mean sample weight (an independent estimator of the same integral)
    albedo = (f.astype(np.float64) * wi[:, 2]).sum() * dw
    assert albedo <= 1.0 + 2e-3
    assert abs(albedo - wt.astype(np.float64).mean()) < 5e-3


def test_ggx_sampler_matches_pdf(oracle_mod):
    """Histogram of sampled cos(theta_i) against the integrated pdf."""
    alpha = 0.4
    wo = _dirs(np.array([0.6]))[0]
    rng = np.random.default_rng(9)
    n = 400_000
    u0 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    u1 = (rng.integers(0, 1 << 24, n) * 2.0**-24).astype(np.float32)
    ws, _ = oracle_mod.ggx_sample_n(np.broadcast_to(wo, (n, 3)), alpha, 1.0, u0, u1)
    mu = ws[:, 2].astype(np.float64)
    edges = np.linspace(0, 1, 21)
    counts, _ = np.histogram(mu[mu > 0], bins=edges)
    wi, dw = _hemisphere_grid(2000, 720)
    _, pdf = oracle_mod.ggx_eval_n(np.broadcast_to(wo, wi.shape), wi, alpha, 1.0)
    expect = np.histogram(wi[:, 2], bins=edges, weights=pdf.astype(np.float64) * dw)[0] * n
    m = expect > 50
    chi2 = ((counts[m] - expect[m]) ** 2 / expect[m]).sum()
    assert stats.chi2.sf(chi2, m.sum()) > 1e-4, (chi2, m.sum())


def test_ggx_weight_equals_f_cos_over_pdf(oracle_mod):
    rng = np.random.default_rng(10)
    n = 20_000
    th = rng.uniform(0, 1.4, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    wo = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1).astype(np.float32)
    alpha = rng.uniform(0.05, 0.5, n).astype(np.float32)
    F = rng.uniform(0.5, 0.8, n).astype(np.float32)
    u0 = rng.uniform(0, 1, n).astype(np.float32)
    u1 = rng.uniform(0, 1, n).astype(np.float32)
    wi, w = oracle_mod.ggx_sample_n(wo, alpha, F, u0, u1)
    ok = w > 0
    f, pdf = oracle_mod.ggx_eval_n(wo[ok], wi[ok], alpha[ok], F[ok])
    ref = f.astype(np.float64) * wi[ok, 2] / pdf
    np.testing.assert_allclose(w[ok], ref, rtol=2e-4)
    # frozen proposal with alpha_s == alpha computes f cos / pdf explicitly
    wi2, w2 = oracle_mod.ggx_sample_n(wo, alpha, F, u0, u1, alpha_s=alpha, frozen=True)
    np.testing.assert_array_equal(wi2, wi)
    np.testing.assert_allclose(w2[ok], w[ok], rtol=2e-4)
    # reflected directions are unit length
    assert np.abs(np.linalg.norm(wi[ok].astype(np.float64), axis=1) - 1).max() < 1e-5


def test_ggx_reciprocity(oracle_mod):
    rng = np.random.default_rng(11)
    n = 5000
    a = rng.normal(size=(n, 3))
    a[:, 2] = np.abs(a[:, 2])
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(n, 3))
    b[:, 2] = np.abs(b[:, 2])
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    alpha = rng.uniform(0.05, 0.5, n)
    f1, _ = oracle_mod.ggx_eval_n(a, b, alpha, 0.7)
    f2, _ = oracle_mod.ggx_eval_n(b, a, alpha, 0.7)
    np.testing.assert_allclose(f1, f2, rtol=1e-5)


def test_ggx_dlogf_dalpha_matches_finite_difference(oracle_mod):
    rng = np.random.default_rng(12)
    for _ in range(300):
        a = rng.normal(size=3)
        a[2] = abs(a[2]) + 0.2
        a /= np.linalg.norm(a)
        b = rng.normal(size=3)
        b[2] = abs(b[2]) + 0.2
        b /= np.linalg.norm(b)
        alpha = rng.uniform(0.08, 0.5)
        h = 1e-2 * alpha
        lf = [np.log(oracle_mod.ggx_f(a, b, alpha + k * h, 1.0)) for k in (-2, -1, 1, 2)]
        fd = (lf[0] - 8 * lf[1] + 8 * lf[2] - lf[3]) / (12 * h)  # five-point stencil
        an = oracle_mod.ggx_dlogf_dalpha(a.astype(np.float32), b.astype(np.float32), alpha)
        assert abs(fd - an) <= 2e-3 * max(1.0, abs(an)), (fd, an, alpha)
