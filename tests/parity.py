"""Comparison helpers for GPU-vs-oracle parity (imported by the GPU tests)."""
import numpy as np

# Floating-point bar: 1e-4 relative on every pixel-bin holding at least 1e-3
# of the film's peak, and the set of non-zero bins must match exactly.  On
# films this is necessary, not sufficient, for identical bin indices: a
# contribution moved between two bins that both hold others would pass.  The
# bin of every single contribution is compared by tests/test_gpu_records.py,
# which diffs the recording build's (pixel, sample, vertex, bin, value, time)
# records against the oracle's.
REL_TOL = 1e-4
PEAK_FRACTION = 1e-3
# Every other bin (a sum of a few FP32 terms, added in LDS in arbitrary
# order on the GPU, in FP64 in path order on the oracle).
REL_TOL_SMALL = 2e-3


def compare_films(gpu_film, ora_film, what="film"):
    g = np.asarray(gpu_film, np.float64).reshape(ora_film.shape)
    o = np.asarray(ora_film, np.float64)
    gz = g != 0
    oz = o != 0
    mismatch = np.flatnonzero((gz != oz).ravel())
    assert mismatch.size == 0, (
        f"{what}: {mismatch.size} bins differ in being non-zero; first {mismatch[:8]}: gpu {g.ravel()[mismatch[:8]]}, "
        f"oracle {o.ravel()[mismatch[:8]]}")
    peak = np.abs(o).max() if o.size else 0.0
    if peak == 0:
        return 0.0
    big = np.abs(o) >= PEAK_FRACTION * peak
    rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-300)
    worst_big = rel[big].max() if big.any() else 0.0
    assert worst_big <= REL_TOL, f"{what}: max rel err {worst_big:.3e} on bins >= 1e-3 peak"
    nz = oz & ~big
    if nz.any():
        worst_small = rel[nz].max()
        assert worst_small <= REL_TOL_SMALL, f"{what}: max rel err {worst_small:.3e} on small bins"
    return float(worst_big)


def compare_vec(gpu, ora, rel=REL_TOL, what="vec"):
    g = np.asarray(gpu, np.float64).ravel()
    o = np.asarray(ora, np.float64).ravel()
    peak = np.abs(o).max()
    err = np.abs(g - o)
    bad = err > rel * np.maximum(np.abs(o), PEAK_FRACTION * peak)
    assert not bad.any(), f"{what}: {bad.sum()} entries off; worst {np.max(err / np.maximum(np.abs(o), 1e-300)):.3e}"
