"""The renderer's primitives on the device against independent host
implementations, bit for bit (the reason bin indices can agree exactly):
Philox4x32-10 against the oracle's, the sine/cosine and ln(1 - u)
approximations over every one of the 2^24 uniforms the renderer draws
against the oracle's, and FP32 division and square root over 2^28 random
bit patterns plus special values against the host's IEEE correctly rounded
operations (SSE)."""
import sys

import numpy as np
import pytest

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


def _same_bits(a, b):
    """Equal bit patterns, or both NaN."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


def test_sincos2pi_all_uniforms(tr, oracle_mod):
    import torch
    _announce("probe sincos2pi 2^24")
    n = 1 << 24
    g = tr.numerics_probe("sincos2pi", n=n)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    u = (np.arange(n, dtype=np.float64) * 2.0**-24).astype(np.float32)
    s, c = oracle_mod.sincos2pi(u)
    assert _same_bits(g[:, 0], s).all(), f"sin differs at {np.flatnonzero(~_same_bits(g[:, 0], s))[:5]}"
    assert _same_bits(g[:, 1], c).all(), f"cos differs at {np.flatnonzero(~_same_bits(g[:, 1], c))[:5]}"


def test_log1m_all_uniforms(tr, oracle_mod):
    import torch
    _announce("probe log1m 2^24")
    n = 1 << 24
    g = tr.numerics_probe("log1m", n=n)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    u = (np.arange(n, dtype=np.float64) * 2.0**-24).astype(np.float32)
    o = oracle_mod.log1m(u)
    bad = np.flatnonzero(~_same_bits(g, o))
    assert bad.size == 0, f"ln(1-u) differs at {bad[:5]}: gpu {g[bad[:5]]}, oracle {o[bad[:5]]}"


def test_philox_random_counters(tr, oracle_mod):
    import torch
    _announce("probe philox 2^20")
    n = 1 << 20
    rng = np.random.default_rng(2510)
    words = rng.integers(0, 1 << 32, size=(n, 6), dtype=np.uint64).astype(np.uint32)
    # small counters too, as the renderer uses them (pixel, sample, block, stream)
    words[: n // 4, 1:4] = rng.integers(0, 64, size=(n // 4, 3), dtype=np.uint64).astype(np.uint32)
    g = tr.numerics_probe("philox", torch.from_numpy(words.view(np.int32)).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().view(np.uint32)
    o = oracle_mod.philox(words[:, :4], words[:, 4:6])
    bad = np.flatnonzero((g != o).any(1))
    assert bad.size == 0, f"Philox differs at {bad[:5]}"


def _specials():
    v = [0.0, -0.0, 1.0, -1.0, 2.0, 0.5, 3.0, 1e-45, -1e-45, 1.1754942e-38, 1.1754944e-38, 3.4028235e38,
         -3.4028235e38, np.inf, -np.inf, np.nan, 7.0, 1e-30, 1e30, 0.1, 1.0000001, 0.99999994]
    v = np.array(v, np.float32)
    a, b = np.meshgrid(v, v)
    return a.ravel(), b.ravel()


@pytest.mark.parametrize("op", ["div", "sqrt"])
def test_correctly_rounded_div_sqrt(tr, op):
    """2^28 random FP32 bit patterns (every exponent, denormals included)
    and the special values, in chunks of 2^24."""
    import torch
    _announce(f"probe {op} 2^28")
    rng = np.random.default_rng(7 if op == "div" else 8)
    chunk = 1 << 24
    sa, sb = _specials()
    checked = 0
    for k in range(16):
        if op == "div":
            ab = rng.integers(0, 1 << 32, size=(chunk, 2), dtype=np.uint64).astype(np.uint32).view(np.float32)
            if k == 0:
                ab[: sa.size, 0] = sa
                ab[: sa.size, 1] = sb
            g = tr.numerics_probe("div", torch.from_numpy(ab).cuda())
            with np.errstate(all="ignore"):
                ref = ab[:, 0] / ab[:, 1]
        else:
            x = rng.integers(0, 1 << 31, size=chunk, dtype=np.uint64).astype(np.uint32).view(np.float32)
            if k == 0:
                x[: sa.size] = np.abs(sa)
                x[sa.size: 2 * sa.size] = -np.abs(sa)
            g = tr.numerics_probe("sqrt", torch.from_numpy(x).cuda())
            with np.errstate(all="ignore"):
                ref = np.sqrt(x)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
        bad = np.flatnonzero(~_same_bits(g, ref))
        assert bad.size == 0, f"{op}: {bad.size} results differ from the correctly rounded ones; first at {bad[:4]}"
        checked += chunk
    assert checked == 1 << 28


def test_probe_rejects_bad_arguments(tr):
    import torch
    with pytest.raises(tr.TrhipError):
        tr.numerics_probe("sincos2pi", n=16, first=(1 << 24) - 8)
    from paper_2510_25660_amd._binding import lib
    assert lib().trhip_numerics_probe(9, None, None, 4, 0, None) == 1  # unknown op: INVALID_ARG
    assert torch.cuda.is_available()
