"""Photon-count noise (trhip_poisson_noise) against the Poisson law itself:
chi-square of the empirical count distribution against the exact Poisson
pmf at fixed means, moments, determinism, and the scale convention."""
import sys

import numpy as np
import pytest
from scipy import stats

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


def _chi2_pvalue(counts, lam):
    """Chi-square of integer counts against Poisson(lam), cells merged so
    every expected count is >= 20."""
    n = counts.size
    lo, hi = int(stats.poisson.ppf(1e-7, lam)), int(stats.poisson.isf(1e-7, lam)) + 1
    ks = np.arange(lo, hi + 1)
    pmf = stats.poisson.pmf(ks, lam)
    pmf[0] += stats.poisson.cdf(lo - 1, lam)
    pmf[-1] += stats.poisson.sf(hi, lam)
    obs = np.bincount(np.clip(counts, lo, hi) - lo, minlength=len(ks)).astype(np.float64)
    exp = pmf * n
    # merge adjacent cells until each expects >= 20
    o_m, e_m, ao, ae = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        ao += o
        ae += e
        if ae >= 20:
            o_m.append(ao)
            e_m.append(ae)
            ao, ae = 0.0, 0.0
    if ae > 0:
        o_m[-1] += ao
        e_m[-1] += ae
    o_m, e_m = np.array(o_m), np.array(e_m)
    chi2 = ((o_m - e_m) ** 2 / e_m).sum()
    return stats.chi2.sf(chi2, len(o_m) - 1)


@pytest.mark.parametrize("lam", [0.05, 0.9, 4.5, 37.0, 255.0, 256.5, 900.0, 3000.0])
def test_counts_follow_poisson_law(tr, lam):
    """2^20 bins of one mean: the counts pass a chi-square test against the
    exact Poisson pmf, and mean and variance agree with lam."""
    import torch
    _announce(f"poisson lam={lam}")
    n = 1 << 20
    scale = 2.0
    film = torch.full((n,), lam / scale, device="cuda", dtype=torch.float32)
    out, s = tr.poisson_noise(film, scale=scale, seed=11)
    torch.cuda.synchronize()
    counts = out.cpu().numpy().astype(np.float64) * scale
    k = np.rint(counts).astype(np.int64)
    assert np.abs(counts - k).max() < 1e-3 and (k >= 0).all()
    lam32 = float(np.float32(lam / scale)) * scale  # the mean the kernel sees
    se = np.sqrt(lam32 / n)
    assert abs(k.mean() - lam32) < 6 * se
    assert abs(k.var() / lam32 - 1.0) < 6 * np.sqrt(2.0 / n) + 1e-3
    assert _chi2_pvalue(k, lam32) > 1e-4


def test_normal_regime_moments(tr):
    """Means above 2^16 use the normal approximation: mean and variance."""
    import torch
    _announce("poisson normal regime")
    n = 1 << 18
    lam = 200000.0
    film = torch.full((n,), lam, device="cuda", dtype=torch.float32)
    out, _ = tr.poisson_noise(film, scale=1.0, seed=3)
    torch.cuda.synchronize()
    k = out.cpu().numpy().astype(np.float64)
    assert abs(k.mean() - lam) < 6 * np.sqrt(lam / n)
    assert abs(k.var() / lam - 1.0) < 0.02


def test_noise_on_a_film(tr):
    """A confocal film: zero bins stay zero, the default scale puts the
    expected peak count at peak_count, same seed gives the same capture,
    another seed another one, and the capture's total matches the film's."""
    import torch
    from paper_2510_25660_amd import scenes
    _announce("poisson on confocal film")
    sc = scenes.confocal_nlos(grid=16, spp=512)
    with tr.upload(sc) as dev:
        _, film = tr.render_transient(dev)
        torch.cuda.synchronize()
    a, scale = tr.poisson_noise(film, peak_count=1000.0, seed=5)
    b, _ = tr.poisson_noise(film, peak_count=1000.0, seed=5)
    c, _ = tr.poisson_noise(film, peak_count=1000.0, seed=6)
    torch.cuda.synchronize()
    f, a, b, c = (x.cpu().numpy().astype(np.float64) for x in (film, a, b, c))
    assert scale == pytest.approx(1000.0 / f.max(), rel=1e-6)
    assert (a[f == 0] == 0).all()
    assert (a == b).all() and (a != c).any()
    total = f.sum() * scale
    assert abs(a.sum() * scale - total) < 6 * np.sqrt(total)
