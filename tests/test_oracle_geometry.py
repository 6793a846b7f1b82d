"""Pins of the oracle's ray-triangle test and BVH: FP64 exact intersection,
and BVH closest hit equal (bitwise) to brute force."""
import numpy as np

from paper_2510_25660_amd import scenes


def _fp64_hit(o, d, tri):
    v0, v1, v2 = tri[0:3].astype(np.float64), tri[3:6].astype(np.float64), tri[6:9].astype(np.float64)
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    e1, e2 = v1 - v0, v2 - v0
    n = np.cross(e1, e2)
    denom = d @ n
    if denom == 0:
        return None, 0.0, 0.0
    t = ((v0 - o) @ n) / denom
    x = o + t * d
    # barycentrics by area ratios
    A = n @ n
    b1 = np.cross(x - v0, e2) @ n / A
    b2 = np.cross(e1, x - v0) @ n / A
    margin = min(b1, b2, 1 - b1 - b2)
    grazing = abs(denom) / (np.linalg.norm(d) * np.sqrt(A))
    return (t if (t > 0 and margin >= 0) else None), margin, grazing


def test_moller_trumbore_vs_fp64(oracle_mod):
    rng = np.random.default_rng(11)
    disagreements = 0
    checked = 0
    for trial in range(60):
        sc = scenes.random_soup(rng, 1, extent=0.5, size=0.4)
        O = oracle_mod.Oracle(sc)
        tri = sc.triangles()[0]
        for _ in range(100):
            o = rng.uniform(-2, 2, 3).astype(np.float32)
            target = (tri[0:3] + (tri[3:6] - tri[0:3]) * rng.uniform(-0.2, 1.2)
                      + (tri[6:9] - tri[0:3]) * rng.uniform(-0.2, 1.2))
            d = (target - o).astype(np.float32)
            d = (d / np.linalg.norm(d)).astype(np.float32)
            t_o, k = O.closest_hit(o, d, use_bvh=False)
            t_r, margin, grazing = _fp64_hit(o, d, tri)
            checked += 1
            if (t_o is None) != (t_r is None):
                # only rays within a hair of an edge, or grazing, may disagree
                assert abs(margin) < 1e-5 or grazing < 1e-3, (trial, o, d, t_o, t_r, margin, grazing)
                disagreements += 1
            elif t_o is not None:
                # FP32 Moller-Trumbore: relative error grows like eps / sin(grazing angle)
                tol = (1e-6 + 64 * 2.0**-24 / grazing) * max(1.0, t_r)
                assert abs(t_o - t_r) <= tol, (t_o, t_r, grazing)
    assert checked == 6000
    assert disagreements < 10


def test_bvh_closest_equals_brute_force(oracle_mod):
    rng = np.random.default_rng(12)
    for trial in range(4):
        sc = scenes.random_soup(rng, 300 + 200 * trial, extent=1.0, size=0.15)
        O = oracle_mod.Oracle(sc)
        n_hits = 0
        for _ in range(600):
            o = rng.uniform(-1.5, 1.5, 3).astype(np.float32)
            d = rng.normal(size=3)
            d = (d / np.linalg.norm(d)).astype(np.float32)
            excl = int(rng.integers(-1, sc.n_tris))
            a = O.closest_hit(o, d, exclude=excl, use_bvh=True)
            b = O.closest_hit(o, d, exclude=excl, use_bvh=False)
            assert a[1] == b[1]
            if a[0] is not None:
                n_hits += 1
                assert np.float32(a[0]) == np.float32(b[0])
        assert n_hits > 100


def test_closed_room_is_watertight_enough(oracle_mod):
    """Rays from inside the closed box room hit a wall (the room quads share
    exact vertices; only exact-edge rays may leak)."""
    rng = np.random.default_rng(13)
    sc = scenes.box_scene()
    O = oracle_mod.Oracle(sc)
    miss = 0
    for _ in range(3000):
        o = rng.uniform(0.05, 0.95, 3).astype(np.float32)
        d = rng.normal(size=3)
        d[2] = -abs(d[2])  # the room is open at z = 1
        d = (d / np.linalg.norm(d)).astype(np.float32)
        t, k = O.closest_hit(o, d)
        miss += t is None
    assert miss <= 2
