"""Pins of the oracle's numerics against things other than itself:
rocRAND's Philox4x32-10 engine, and FP64 libm over every 24-bit uniform."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_ref_binary():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    out = os.path.join(tempfile.mkdtemp(prefix="rocrand_ref_"), "prr")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                           os.path.join(HERE, "support", "rocrand_philox_ref.cpp"), "-o", out],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, cwd=tempfile.gettempdir())
    return out


def test_philox_matches_rocrand(oracle_mod):
    """Philox4x32-10 (Salmon et al. 2011) against rocRAND's implementation,
    over random counters/keys covering all four counter words."""
    binary = _rocrand_ref_binary()
    rng = np.random.default_rng(7)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 29) - 1  # rocRAND's offset argument reaches counter word 1 below 2^30
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:10] = 0
    key[:5] = 0
    lines = "\n".join(" ".join(str(int(x)) for x in (*c, *k)) for c, k in zip(ctr, key)) + "\n"
    res = subprocess.run([binary], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(w) for w in ln.split()] for ln in res.stdout.strip().splitlines()], np.uint64)
    got = oracle_mod.philox(ctr, key).astype(np.uint64)
    assert ref.shape == got.shape
    np.testing.assert_array_equal(got, ref)


def _all_uniforms():
    return (np.arange(1 << 24, dtype=np.float64) * 2.0**-24).astype(np.float32)


def _ulp(x):
    x = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(x, 2.0**-126)))
    return 2.0 ** (e - 23)


def test_sincos2pi_exhaustive(oracle_mod):
    """sin/cos(2 pi u) for all 2^24 uniforms within 2 ulp of FP64 libm (or
    2^-25 absolute where the result is near zero)."""
    u = _all_uniforms()
    s, c = oracle_mod.sincos2pi(u)
    a = 2.0 * np.pi * u.astype(np.float64)
    for got, ref in ((s, np.sin(a)), (c, np.cos(a))):
        err = np.abs(got.astype(np.float64) - ref)
        tol = np.maximum(2.0 * _ulp(ref), 2.0**-25)
        bad = err > tol
        assert not bad.any(), (np.flatnonzero(bad)[:5], err[bad][:5])
    # exact special points
    assert s[0] == 0.0 and c[0] == 1.0
    q = 1 << 22
    assert s[q] == 1.0 and c[2 * q] == -1.0 and s[3 * q] == -1.0


def test_log1m_exhaustive(oracle_mod):
    """ln(1-u) for all 2^24 uniforms within 2 ulp of FP64 log1p(-u)."""
    u = _all_uniforms()
    got = oracle_mod.log1m(u).astype(np.float64)
    ref = np.log1p(-u.astype(np.float64))
    err = np.abs(got - ref)
    tol = 2.0 * _ulp(ref)
    tol[0] = 0.0
    bad = err > tol
    assert not bad.any(), (np.flatnonzero(bad)[:5], err[bad][:5])
    assert got[0] == 0.0


def test_uniform_mapping(oracle_mod):
    """u = (x >> 8) * 2^-24 is exact and lies in [0, 1 - 2^-24]."""
    L = oracle_mod.lib()
    L.orc_uniform.restype = __import__("ctypes").c_float
    L.orc_uniform.argtypes = [__import__("ctypes").c_uint32]
    assert L.orc_uniform(0) == 0.0
    assert L.orc_uniform(0xFFFFFFFF) == np.float32(1.0 - 2.0**-24)
    assert L.orc_uniform(0x80000000) == 0.5
