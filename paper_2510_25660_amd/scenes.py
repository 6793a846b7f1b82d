"""Seeded synthetic scenes for transient rendering.

This module only builds input arrays (geometry, materials, sensor and film
parameters); it holds none of the rendering arithmetic.  Both the HIP path and
the CPU oracle consume what it produces.

The paper's own scenes (Cornell box, Staircase, Office, Bottle) are not
available, so the workloads below are synthetic stand-ins with the sizes and
structure of the paper's use cases (Sec. 3 and Sec. 4):

* ``box_scene``       -- a 34-triangle box room seen by a 64x64 pinhole camera
                          (the Cornell-box style use of Sec. 3 and Sec. 4.3);
* ``confocal_nlos``   -- a relay wall scanned at 64x64 points with a 9,680
                          triangle hidden blob (the NLOS capture of Sec. 4.5);
* ``large_scene``     -- ~1M-triangle terrain plus displaced spheres in fog
                          with Lambertian and GGX materials (Sec. 4.1);
* ``diff_scene``      -- the box room subdivided to 9,826 triangles with
                          per-triangle albedo and roughness parameters
                          (the backward-mode example of Sec. 4.4);
* ``batched_nlos``    -- many confocal scenes of uneven size (Sec. 4.5).

Distances are metres (c = 1): a segment's optical path length is its length
times the refractive index it runs in.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MAT_LAMBERT = 0
MAT_GGX = 1
MAT_DIELECTRIC = 2   # smooth interface; the mesh's inside lies against the winding normal e1 x e2

SENSOR_PINHOLE = 0
SENSOR_CONFOCAL = 1

BASE_SEED = 2510_25660


@dataclasses.dataclass
class Scene:
    vertices: np.ndarray            # float32 [nv, 3]
    indices: np.ndarray             # uint32 [nt, 3]
    mat_type: np.ndarray            # uint8 [nt]
    albedo: np.ndarray              # float32 [nt]
    roughness: np.ndarray           # float32 [nt]
    n_bins: int
    bin_width: float
    bin_start: float
    sensor: int = SENSOR_PINHOLE
    width: int = 64
    height: int = 64
    light_pos: tuple = (0.0, 0.0, 0.0)
    light_intensity: float = 1.0
    cam_origin: tuple = (0.0, 0.0, 0.0)
    cam_right: tuple = (1.0, 0.0, 0.0)
    cam_up: tuple = (0.0, 1.0, 0.0)
    cam_fwd: tuple = (0.0, 0.0, -1.0)
    tan_x: float = 0.0
    tan_y: float = 0.0
    scan_points: Optional[np.ndarray] = None   # float32 [height*width, 3]
    wall_normal: tuple = (0.0, 0.0, 1.0)
    wall_albedo: float = 1.0
    laser_power: float = 1.0
    sigma_t: float = 0.0
    medium_albedo: float = 0.0
    camera_unwarp: bool = False
    # refractive index inside dielectric meshes (per triangle), scattering
    # delay means in metres of OPL (per triangle), index of the surrounding space
    ior: Optional[np.ndarray] = None
    delay: Optional[np.ndarray] = None
    medium_ior: float = 1.0
    # default render settings of the workload
    spp: int = 16
    max_depth: int = 4
    seed: int = BASE_SEED
    name: str = ""

    @property
    def n_tris(self) -> int:
        return int(self.indices.shape[0])

    @property
    def n_pixels(self) -> int:
        return int(self.width * self.height)

    def triangles(self) -> np.ndarray:
        """Triangle soup float32 [nt, 9] (v0, v1, v2)."""
        return np.ascontiguousarray(self.vertices[self.indices].reshape(-1, 9), dtype=np.float32)


# --------------------------------------------------------------------------
# small helpers (host-side set-up arithmetic in float64, stored as float32)
# --------------------------------------------------------------------------
def _f32(v):
    return tuple(float(np.float32(x)) for x in v)


def look_at(origin, target, up_hint, vfov_deg, width, height):
    """Pinhole basis: unit right/up/forward vectors and tan of the half fovs."""
    o = np.asarray(origin, np.float64)
    f = np.asarray(target, np.float64) - o
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up_hint, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    tan_y = math.tan(math.radians(vfov_deg) * 0.5)
    tan_x = tan_y * width / height
    return dict(cam_origin=_f32(o), cam_right=_f32(r), cam_up=_f32(u), cam_fwd=_f32(f),
                tan_x=float(np.float32(tan_x)), tan_y=float(np.float32(tan_y)))


def quad(p0, p1, p2, p3):
    """Two triangles of the planar quad p0 p1 p2 p3 (in order)."""
    v = np.array([p0, p1, p2, p3], np.float64)
    return v, np.array([[0, 1, 2], [0, 2, 3]], np.int64)


def box_mesh(lo, hi):
    """12 triangles of an axis-aligned box."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    f = np.array([[0, 1, 2], [0, 2, 3],   # z0
                  [4, 6, 5], [4, 7, 6],   # z1
                  [0, 4, 5], [0, 5, 1],   # y0
                  [3, 2, 6], [3, 6, 7],   # y1
                  [0, 3, 7], [0, 7, 4],   # x0
                  [1, 5, 6], [1, 6, 2]],  # x1
                 np.int64)
    return v, f


def outward(verts, faces):
    """Rewinds the triangles of a mesh that is star-shaped about the centroid
    of the vertices it uses so that every winding normal e1 x e2 points away
    from it (the orientation a dielectric mesh needs: its inside lies against
    e1 x e2)."""
    v = np.asarray(verts, np.float64)
    f = np.array(faces, np.int64, copy=True)
    c = v[np.unique(f)].mean(axis=0)
    t = v[f]
    nrm = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    flip = np.einsum("ij,ij->i", nrm, t.mean(axis=1) - c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def merge(parts):
    verts, faces, off = [], [], 0
    for v, f in parts:
        verts.append(np.asarray(v, np.float64))
        faces.append(np.asarray(f, np.int64) + off)
        off += len(v)
    return np.concatenate(verts), np.concatenate(faces)


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    return v, f


def geodesic_sphere(freq: int):
    """Unit geodesic sphere of frequency ``freq``: 20*freq^2 triangles with
    shared (deduplicated) vertices."""
    iv, ifc = _icosahedron()
    n = int(freq)
    ii, jj = [], []
    for i in range(n + 1):
        for j in range(n + 1 - i):
            ii.append(i)
            jj.append(j)
    ii = np.array(ii)
    jj = np.array(jj)
    lut = -np.ones((n + 1, n + 1), np.int64)
    lut[ii, jj] = np.arange(len(ii))
    up, dn = [], []
    for i in range(n):
        for j in range(n - i):
            up.append([lut[i, j], lut[i + 1, j], lut[i, j + 1]])
            if i + j < n - 1:
                dn.append([lut[i + 1, j], lut[i + 1, j + 1], lut[i, j + 1]])
    local = np.array(up + dn, np.int64)
    A = iv[ifc[:, 0]][:, None, :]
    B = iv[ifc[:, 1]][:, None, :]
    C = iv[ifc[:, 2]][:, None, :]
    w0 = ((n - ii - jj) / n)[None, :, None]
    w1 = (ii / n)[None, :, None]
    w2 = (jj / n)[None, :, None]
    pts = A * w0 + B * w1 + C * w2
    pts /= np.linalg.norm(pts, axis=2, keepdims=True)
    npf = pts.shape[1]
    flat = pts.reshape(-1, 3)
    key = np.round(flat * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    verts = uniq.astype(np.float64) * 1e-9
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    faces = (local[None, :, :] + (np.arange(20) * npf)[:, None, None]).reshape(-1, 3)
    faces = inv.reshape(-1)[faces]
    return verts, faces


def geodesic_freq_for(n_tris: float) -> int:
    """Frequency of the geodesic sphere closest to ``n_tris`` triangles."""
    return max(1, int(round(math.sqrt(n_tris / 20.0))))


def noisy_blob(rng, freq, radius, centre, noise=0.1, n_waves=8):
    """Geodesic sphere with a smooth seeded radial displacement
    r(v) = R (1 + noise * n(v)), n a normalised sum of sinusoids."""
    v, f = geodesic_sphere(freq)
    dirs = rng.normal(size=(n_waves, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    freqs = rng.uniform(2.0, 6.0, size=n_waves)
    phase = rng.uniform(0.0, 2 * math.pi, size=n_waves)
    amp = rng.uniform(0.5, 1.0, size=n_waves)
    field = (amp[None, :] * np.sin((v @ dirs.T) * freqs[None, :] + phase[None, :])).sum(1) / amp.sum()
    r = radius * (1.0 + noise * field)
    return v * r[:, None] + np.asarray(centre, np.float64)[None, :], f


def _finish(verts, faces, mat, albedo, rough, **kw) -> Scene:
    return Scene(vertices=np.ascontiguousarray(verts, np.float32),
                 indices=np.ascontiguousarray(faces, np.uint32),
                 mat_type=np.ascontiguousarray(mat, np.uint8),
                 albedo=np.ascontiguousarray(albedo, np.float32),
                 roughness=np.ascontiguousarray(rough, np.float32), **kw)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def _box_room_parts():
    parts = [
        quad([0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1]),      # floor y=0
        quad([0, 1, 0], [0, 1, 1], [1, 1, 1], [1, 1, 0]),      # ceiling y=1
        quad([0, 0, 0], [0, 1, 0], [1, 1, 0], [1, 0, 0]),      # back z=0
        quad([0, 0, 0], [0, 0, 1], [0, 1, 1], [0, 1, 0]),      # left x=0
        quad([1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1]),      # right x=1
        box_mesh([0.13, 0.0, 0.37], [0.43, 0.3, 0.67]),        # short box
        box_mesh([0.55, 0.0, 0.10], [0.85, 0.6, 0.40]),        # tall box
    ]
    return parts


def box_scene(seed: int = BASE_SEED + 1, width=64, height=64, n_bins=256, bin_width=0.01,
              bin_start=0.0, spp=16, max_depth=4) -> Scene:
    """Box room (5 quads open at z=1) with two boxes: 34 Lambertian triangles,
    albedo U[0.5, 0.8] per triangle, isotropic point light at (0.5, 0.9, 0.5),
    pinhole at (0.5, 0.5, 1.5) looking down -z with a 40 degree vertical fov."""
    rng = np.random.default_rng(seed)
    v, f = merge(_box_room_parts())
    nt = len(f)
    albedo = rng.uniform(0.5, 0.8, nt)
    cam = look_at([0.5, 0.5, 1.5], [0.5, 0.5, 0.0], [0, 1, 0], 40.0, width, height)
    return _finish(v, f, np.zeros(nt), albedo, np.full(nt, 0.3), n_bins=n_bins, bin_width=bin_width,
                   bin_start=bin_start, width=width, height=height, light_pos=(0.5, 0.9, 0.5),
                   light_intensity=1.0, spp=spp, max_depth=max_depth, seed=seed, name="box", **cam)


def cluttered_box(n_tris: int, seed: int = BASE_SEED + 11, width=24, height=16, n_bins=128, bin_width=0.02,
                  spp=8, max_depth=4) -> Scene:
    """The box room filled up to exactly n_tris triangles with small random
    triangles (edge ~0.01) uniform in the room; every other one GGX with
    roughness U[0.1, 0.7].  Sizes either side of a power of two probe the
    traversal's index widths."""
    rng = np.random.default_rng(seed)
    v, f = merge(_box_room_parts())
    k = n_tris - len(f)
    assert k >= 0
    c = rng.uniform(0.02, 0.98, size=(k, 1, 3))
    cv = (c + rng.normal(scale=0.005, size=(k, 3, 3))).reshape(-1, 3)
    verts = np.concatenate([v, cv])
    faces = np.concatenate([f, len(v) + np.arange(3 * k).reshape(-1, 3)])
    mat = np.zeros(n_tris)
    mat[len(f) + 1::2] = MAT_GGX
    albedo = rng.uniform(0.3, 0.9, n_tris)
    rough = rng.uniform(0.1, 0.7, n_tris)
    cam = look_at([0.5, 0.5, 1.5], [0.5, 0.5, 0.0], [0, 1, 0], 40.0, width, height)
    return _finish(verts, faces, mat, albedo, rough, n_bins=n_bins, bin_width=bin_width, bin_start=0.0,
                   width=width, height=height, light_pos=(0.5, 0.9, 0.5), light_intensity=1.0, spp=spp,
                   max_depth=max_depth, seed=seed, name=f"cluttered_box_{n_tris}", **cam)


def subdivide(verts, faces, k: int):
    """Split every triangle into k^2 congruent sub-triangles (same geometry)."""
    ii, jj = [], []
    for i in range(k + 1):
        for j in range(k + 1 - i):
            ii.append(i)
            jj.append(j)
    ii = np.array(ii)
    jj = np.array(jj)
    lut = -np.ones((k + 1, k + 1), np.int64)
    lut[ii, jj] = np.arange(len(ii))
    tri = []
    for i in range(k):
        for j in range(k - i):
            tri.append([lut[i, j], lut[i + 1, j], lut[i, j + 1]])
            if i + j < k - 1:
                tri.append([lut[i + 1, j], lut[i + 1, j + 1], lut[i, j + 1]])
    tri = np.array(tri, np.int64)
    A = verts[faces[:, 0]][:, None, :]
    B = verts[faces[:, 1]][:, None, :]
    C = verts[faces[:, 2]][:, None, :]
    w0 = ((k - ii - jj) / k)[None, :, None]
    w1 = (ii / k)[None, :, None]
    w2 = (jj / k)[None, :, None]
    pts = (A * w0 + B * w1 + C * w2)
    npf = pts.shape[1]
    nv = pts.reshape(-1, 3)
    nf = (tri[None, :, :] + (np.arange(len(faces)) * npf)[:, None, None]).reshape(-1, 3)
    parent = np.repeat(np.arange(len(faces)), len(tri))
    return nv, nf, parent


def diff_scene(seed: int = BASE_SEED + 4, sub: int = 17, width=64, height=64, spp=1024) -> Scene:
    """The box room with every triangle split into sub^2 pieces (9,826
    triangles at sub=17): room Lambertian, both boxes GGX conductors; albedo
    U[0.5, 0.8] and roughness U[0.05, 0.5] per triangle."""
    rng = np.random.default_rng(seed)
    v, f = merge(_box_room_parts())
    parent_is_box = np.arange(len(f)) >= 10
    nv, nf, parent = subdivide(v, f, sub)
    nt = len(nf)
    mat = np.where(parent_is_box[parent], MAT_GGX, MAT_LAMBERT)
    albedo = rng.uniform(0.5, 0.8, nt)
    rough = rng.uniform(0.05, 0.5, nt)
    cam = look_at([0.5, 0.5, 1.5], [0.5, 0.5, 0.0], [0, 1, 0], 40.0, width, height)
    return _finish(nv, nf, mat, albedo, rough, n_bins=256, bin_width=0.01, bin_start=0.0,
                   width=width, height=height, light_pos=(0.5, 0.9, 0.5), light_intensity=1.0,
                   spp=spp, max_depth=4, seed=seed, name="diff", **cam)


def perturbed_params(scene: Scene, seed: int):
    """Target parameters: albedo + U(-0.1, 0.1) clipped to [0.05, 0.95],
    roughness + U(-0.1, 0.1) clipped to [0.05, 0.5]."""
    rng = np.random.default_rng(seed)
    a = np.clip(scene.albedo + rng.uniform(-0.1, 0.1, scene.n_tris), 0.05, 0.95).astype(np.float32)
    r = np.clip(scene.roughness + rng.uniform(-0.1, 0.1, scene.n_tris), 0.05, 0.5).astype(np.float32)
    return a, r


def relay_wall(nx: int, ny: int, half: float = 0.5):
    """Relay wall z=0 spanning [-half, half]^2 (2 triangles) and the scan
    points at its nx x ny cell centres, row-major (iy, ix)."""
    v, f = quad([-half, -half, 0], [half, -half, 0], [half, half, 0], [-half, half, 0])
    xs = -half + (np.arange(nx) + 0.5) * (2 * half / nx)
    ys = -half + (np.arange(ny) + 0.5) * (2 * half / ny)
    gx, gy = np.meshgrid(xs, ys)
    pts = np.stack([gx.ravel(), gy.ravel(), np.zeros(nx * ny)], 1).astype(np.float32)
    return (v, f), pts


def confocal_nlos(seed: int = BASE_SEED + 2, grid: int = 64, n_tris: int = 10_000, n_bins: int = 512,
                  bin_width: float = 0.0024, bin_start: float = 0.9, spp: int = 4096,
                  bounces: int = 3, albedo: float = 0.7) -> Scene:
    """Confocal NLOS: 1x1 m Lambertian relay wall (albedo 1) scanned at
    grid x grid points, laser and detector co-located at each point; hidden
    seeded noisy geodesic blob (R = 0.25 m, radial noise 0.1) centred 0.75 m
    in front of the wall, albedo 0.7."""
    rng = np.random.default_rng(seed)
    wall, pts = relay_wall(grid, grid)
    blob = noisy_blob(rng, geodesic_freq_for(n_tris), 0.25, (0.0, 0.0, 0.75))
    v, f = merge([wall, blob])
    nt = len(f)
    alb = np.full(nt, albedo)
    alb[:2] = 1.0
    return _finish(v, f, np.zeros(nt), alb, np.full(nt, 0.3), n_bins=n_bins, bin_width=bin_width,
                   bin_start=bin_start, sensor=SENSOR_CONFOCAL, width=grid, height=grid,
                   scan_points=pts, wall_normal=(0.0, 0.0, 1.0), wall_albedo=1.0, laser_power=1.0,
                   spp=spp, max_depth=bounces + 1, seed=seed, name="confocal")


def terrain(rng, cells: int = 512, half: float = 2.0, amplitude: float = 0.25, n_waves: int = 8):
    """Heightfield over x,z in [-half, half]: sum of seeded sinusoids scaled to
    the given amplitude; 2*cells^2 triangles."""
    kx = rng.uniform(-4.0, 4.0, n_waves)
    kz = rng.uniform(-4.0, 4.0, n_waves)
    ph = rng.uniform(0.0, 2 * math.pi, n_waves)
    am = rng.uniform(0.5, 1.0, n_waves)
    am = am * (amplitude / am.sum())

    def height(x, z):
        return (am[None, :] * np.sin(np.outer(x, kx) + np.outer(z, kz) + ph[None, :])).sum(1)

    g = np.linspace(-half, half, cells + 1)
    gx, gz = np.meshgrid(g, g)
    y = height(gx.ravel(), gz.ravel())
    verts = np.stack([gx.ravel(), y, gz.ravel()], 1)
    idx = np.arange((cells + 1) * (cells + 1)).reshape(cells + 1, cells + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[1:, :-1].ravel()
    faces = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return (verts, faces), height


def large_scene(seed: int = BASE_SEED + 3, cells: int = 512, sphere_freq: int = 22, grid: int = 7,
                width: int = 512, height: int = 512, n_bins: int = 1024, bin_width: float = 0.005,
                bin_start: float = 4.5, spp: int = 64, max_depth: int = 8, fog: bool = True) -> Scene:
    """Seeded terrain (524,288 triangles at cells=512) plus a jittered 7x7 grid
    of displaced geodesic spheres resting on it (474,320 triangles at
    freq 22); terrain Lambertian, each sphere Lambertian or GGX by coin flip;
    homogeneous fog sigma_t = 0.1/m with albedo 0.9."""
    rng = np.random.default_rng(seed)
    ter, hfun = terrain(rng, cells)
    parts = [ter]
    mats = [np.zeros(len(ter[1]))]
    alb = [rng.uniform(0.5, 0.8, len(ter[1]))]
    rough = [np.full(len(ter[1]), 0.3)]
    cell = 3.5 / grid
    for gi in range(grid):
        for gj in range(grid):
            cx = -1.75 + (gi + 0.5) * cell + rng.uniform(-0.15, 0.15)
            cz = -1.75 + (gj + 0.5) * cell + rng.uniform(-0.15, 0.15)
            R = rng.uniform(0.1, 0.3)
            cy = float(hfun(np.array([cx]), np.array([cz]))[0]) + R
            sv, sf = noisy_blob(rng, sphere_freq, R, (cx, cy, cz))
            parts.append((sv, sf))
            m = MAT_GGX if rng.uniform() < 0.5 else MAT_LAMBERT
            mats.append(np.full(len(sf), m))
            alb.append(rng.uniform(0.5, 0.8, len(sf)))
            rough.append(rng.uniform(0.05, 0.5, len(sf)))
    v, f = merge(parts)
    cam = look_at([0.0, 1.5, 3.5], [0.0, 0.0, 0.0], [0, 1, 0], 45.0, width, height)
    return _finish(v, f, np.concatenate(mats), np.concatenate(alb), np.concatenate(rough),
                   n_bins=n_bins, bin_width=bin_width, bin_start=bin_start, width=width, height=height,
                   light_pos=(0.0, 2.0, 0.0), light_intensity=1.0, sigma_t=0.1 if fog else 0.0,
                   medium_albedo=0.9 if fog else 0.0, spp=spp, max_depth=max_depth, seed=seed,
                   name="large", **cam)


def batched_nlos(n_scenes: int = 256, seed: int = BASE_SEED + 5, spp: int = 256,
                 tri_range=(1_000, 50_000), grid_range=(16, 64), bins_range=(256, 1024)) -> List[Scene]:
    """Confocal scenes of uneven size: triangle count log-uniform in
    tri_range, scan grid side uniform in grid_range, bin count uniform in
    bins_range; bin width 2.4 mm from 0.9 m; per-scene seed = seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_scenes):
        nt = math.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1])))
        g = int(rng.integers(grid_range[0], grid_range[1] + 1))
        nb = int(rng.integers(bins_range[0], bins_range[1] + 1))
        s = confocal_nlos(seed=seed + i, grid=g, n_tris=int(nt), n_bins=nb, spp=spp)
        s.name = f"batch{i}"
        out.append(s)
    return out


# --------------------------------------------------------------------------
# small analytic fixtures
# --------------------------------------------------------------------------
def plane_scene(h=1.0, albedo=0.6, half=50.0, width=16, height=16, n_bins=8192, bin_width=0.001,
                bin_start=0.0, cam_height=2.0, vfov=60.0, mat=MAT_LAMBERT, roughness=0.3,
                unwarp=False, sigma_t=0.0, medium_albedo=0.0) -> Scene:
    """Large plane y=0, point light at height h above the origin, pinhole
    looking straight down from cam_height (single-bounce closed form);
    optionally filled with homogeneous fog (sigma_t > 0)."""
    v, f = quad([-half, 0, -half], [-half, 0, half], [half, 0, half], [half, 0, -half])
    cam = look_at([0.3, cam_height, 0.2], [0.3, 0.0, 0.2], [0, 0, -1], vfov, width, height)
    return _finish(v, f, np.full(2, mat), np.full(2, albedo), np.full(2, roughness), n_bins=n_bins,
                   bin_width=bin_width, bin_start=bin_start, width=width, height=height,
                   light_pos=(0.0, h, 0.0), light_intensity=1.0, camera_unwarp=unwarp,
                   sigma_t=float(sigma_t), medium_albedo=float(medium_albedo),
                   spp=1, max_depth=2, name="plane", **cam)


def layered_scene(n_layers=2 ** 18, spacing=1e-5, half=4.0, width=16, height=16, n_bins=512, bin_width=0.01,
                  spp=4) -> Scene:
    """n_layers parallel quads y = -i * spacing under a point light, seen from
    above.  Every camera ray crosses the boxes of all layers, so its
    closest-hit traversal keeps a far child pending at nearly every level of
    the tree: the deepest traversal stacks any scene of this size produces."""
    v0, f0 = quad([-half, 0, -half], [-half, 0, half], [half, 0, half], [half, 0, -half])
    ys = 0.0 - spacing * np.arange(n_layers, dtype=np.float64)
    verts = np.tile(v0, (n_layers, 1))
    verts[:, 1] = np.repeat(ys, 4)
    faces = (f0[None, :, :] + 4 * np.arange(n_layers)[:, None, None]).reshape(-1, 3)
    nt = faces.shape[0]
    cam = look_at([0.1, 2.0, 0.05], [0.1, 0.0, 0.05], [0, 0, -1], 50.0, width, height)
    return _finish(verts, faces, np.full(nt, MAT_LAMBERT), np.full(nt, 0.7), np.full(nt, 0.3), n_bins=n_bins,
                   bin_width=bin_width, bin_start=2.0, width=width, height=height, light_pos=(0.5, 1.5, -0.3),
                   light_intensity=1.0, spp=spp, max_depth=3, name="layers", **cam)


def parallel_plane_confocal(d=0.5, half=40.0, grid=4, n_bins=2048, bin_width=0.0024,
                            bin_start=0.9, albedo=0.7, spp=4096) -> Scene:
    """Relay wall z=0 (scan grid over [-0.05, 0.05]^2) facing a large
    Lambertian plane z=d (confocal first-return closed form)."""
    (wv, wf), pts = relay_wall(grid, grid, half=0.05)
    pv, pf = quad([-half, -half, d], [half, -half, d], [half, half, d], [-half, half, d])
    v, f = merge([(wv, wf), (pv, pf)])
    alb = np.array([1.0, 1.0, albedo, albedo])
    return _finish(v, f, np.zeros(4), alb, np.full(4, 0.3), n_bins=n_bins, bin_width=bin_width,
                   bin_start=bin_start, sensor=SENSOR_CONFOCAL, width=grid, height=grid,
                   scan_points=pts, wall_normal=(0.0, 0.0, 1.0), wall_albedo=1.0,
                   laser_power=1.0, spp=spp, max_depth=4, name="parallel")


def sphere_furnace(radius=1.0, freq=40, albedo=1.0, width=8, height=8, n_bins=1024, bin_width=0.01,
                   max_depth=4) -> Scene:
    """Closed geodesic sphere shell of the given radius with camera and
    point light at its centre (white furnace when albedo = 1)."""
    v, f = geodesic_sphere(freq)
    v = v * radius
    nt = len(f)
    cam = look_at([0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0, 1, 0], 90.0, width, height)
    return _finish(v, f, np.zeros(nt), np.full(nt, albedo), np.full(nt, 0.3), n_bins=n_bins,
                   bin_width=bin_width, bin_start=0.0, width=width, height=height,
                   light_pos=(0.0, 0.0, 0.0), light_intensity=1.0, max_depth=max_depth,
                   name="furnace", **cam)


def fog_only(sigma_t=0.5, albedo=0.8, n_bins=512, bin_width=0.02, light=(0.0, 1.0, -2.0)) -> Scene:
    """Homogeneous fog with no reachable surface (one tiny triangle far
    behind the camera), a point light, a 1x1 pinhole."""
    v = np.array([[0, 0, 1000.0], [0.001, 0, 1000.0], [0, 0.001, 1000.0]])
    f = np.array([[0, 1, 2]])
    cam = look_at([0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0, 1, 0], 10.0, 1, 1)
    return _finish(v, f, np.zeros(1), np.full(1, 0.5), np.full(1, 0.3), n_bins=n_bins,
                   bin_width=bin_width, bin_start=0.0, width=1, height=1, light_pos=tuple(light),
                   light_intensity=1.0, sigma_t=sigma_t, medium_albedo=albedo, max_depth=2,
                   name="fog", **cam)


def random_soup(rng, n_tris, extent=1.0, size=0.3):
    """Random triangle soup in [-extent, extent]^3 for intersection tests."""
    c = rng.uniform(-extent, extent, size=(n_tris, 1, 3))
    v = c + rng.normal(scale=size, size=(n_tris, 3, 3))
    verts = v.reshape(-1, 3)
    faces = np.arange(3 * n_tris).reshape(-1, 3)
    return _finish(verts, faces, np.zeros(n_tris), np.full(n_tris, 0.5), np.full(n_tris, 0.3),
                   n_bins=16, bin_width=0.1, bin_start=0.0, name="soup")


CONFIGS = {
    "box": box_scene,
    "confocal": confocal_nlos,
    "large": large_scene,
    "diff": diff_scene,
}


def occluded_nlos_scene(grid=4, spp=4096, n_bins=512, bin_width=0.01, bin_start=0.4, bounces=4) -> Scene:
    """Confocal scan points near the origin of the relay wall z=0; a square
    occluder [-0.2,0.2]^2 at z=0.3 hides a square plane of the same size at
    z=0.6 from every scan point; a plane x=0.5 (|y| <= 1, 0 <= z <= 1) is in
    direct view.  Light reaches the hidden square only around the occluder,
    so a path drawn on it must carry the visibility of its first segment."""
    (wv, wf), pts = relay_wall(grid, grid, half=0.02)
    wv = wv * 50.0  # the wall itself spans [-1, 1]^2
    occ = quad([-0.2, -0.2, 0.3], [0.2, -0.2, 0.3], [0.2, 0.2, 0.3], [-0.2, 0.2, 0.3])
    hid = quad([-0.2, -0.2, 0.6], [0.2, -0.2, 0.6], [0.2, 0.2, 0.6], [-0.2, 0.2, 0.6])
    side = quad([0.5, -1.0, 0.0], [0.5, 1.0, 0.0], [0.5, 1.0, 1.0], [0.5, -1.0, 1.0])
    v, f = merge([(wv, wf), occ, hid, side])
    alb = np.array([1.0, 1.0, 0.6, 0.6, 0.8, 0.8, 0.7, 0.7])
    return _finish(v, f, np.zeros(8), alb, np.full(8, 0.3), n_bins=n_bins, bin_width=bin_width,
                   bin_start=bin_start, sensor=SENSOR_CONFOCAL, width=grid, height=grid, scan_points=pts,
                   wall_normal=(0.0, 0.0, 1.0), wall_albedo=1.0, laser_power=1.0, spp=spp,
                   max_depth=bounces + 1, name="occluded_nlos")


# --------------------------------------------------------------------------
# refractive indices and scattering delays (Eqs. 3 and 10)
# --------------------------------------------------------------------------
def glass_tank_scene(ior=1.5, width=16, height=16, n_bins=8192, bin_width=0.001, spp=256) -> Scene:
    """Closed dielectric box [-2,2]^2 x [-1,1] (index ior) holding a
    Lambertian plane z=-0.5 (albedo 0.6) and the point light (0.2, 0.1, 0.3);
    pinhole at (0.1, -0.05, 3) looking down -z, 30 degree vfov; max_depth 3:
    the camera ray refracts into the tank and the plane connects to the light
    inside it."""
    tank = outward(*box_mesh((-2.0, -2.0, -1.0), (2.0, 2.0, 1.0)))
    plane = quad([-1.5, -1.5, -0.5], [1.5, -1.5, -0.5], [1.5, 1.5, -0.5], [-1.5, 1.5, -0.5])
    v, f = merge([tank, plane])
    mat = np.array([MAT_DIELECTRIC] * 12 + [MAT_LAMBERT] * 2)
    alb = np.array([1.0] * 12 + [0.6] * 2)
    cam = look_at([0.1, -0.05, 3.0], [0.1, -0.05, 0.0], [0, 1, 0], 30.0, width, height)
    return _finish(v, f, mat, alb, np.full(14, 0.3), n_bins=n_bins, bin_width=bin_width, bin_start=0.0,
                   width=width, height=height, light_pos=(0.2, 0.1, 0.3), light_intensity=1.0,
                   ior=np.full(14, ior, np.float32), spp=spp, max_depth=3, name="tank", **cam)


def glass_slab_scene(ior=1.5, width=16, height=16, n_bins=8192, bin_width=0.001, spp=256) -> Scene:
    """Dielectric slab [-3,3]^2 x [0.8,1.0] (index ior) over a Lambertian
    plane z=0 (albedo 0.5); point light (0.3, 0.2, 0.4) between them; pinhole
    at (0.1, -0.05, 2.5) looking down -z, 30 degree vfov; max_depth 4: the
    camera ray crosses both faces of the slab before reaching the plane."""
    slab = outward(*box_mesh((-3.0, -3.0, 0.8), (3.0, 3.0, 1.0)))
    plane = quad([-4, -4, 0], [4, -4, 0], [4, 4, 0], [-4, 4, 0])
    v, f = merge([slab, plane])
    mat = np.array([MAT_DIELECTRIC] * 12 + [MAT_LAMBERT] * 2)
    alb = np.array([1.0] * 12 + [0.5] * 2)
    cam = look_at([0.1, -0.05, 2.5], [0.1, -0.05, 0.0], [0, 1, 0], 30.0, width, height)
    return _finish(v, f, mat, alb, np.full(14, 0.3), n_bins=n_bins, bin_width=bin_width, bin_start=0.0,
                   width=width, height=height, light_pos=(0.3, 0.2, 0.4), light_intensity=1.0,
                   ior=np.full(14, ior, np.float32), spp=spp, max_depth=4, name="slab", **cam)


def glass_box_scene(ior=1.5, seed: int = BASE_SEED + 12, width=64, height=64, n_bins=256, bin_width=0.01,
                    spp=16, max_depth=8, delay_mean=0.0) -> Scene:
    """The box room with its short box made of a dielectric of index ior
    (the setting of the paper's index-of-refraction example, Sec. 4.4);
    optionally every room triangle has a scattering delay of mean delay_mean
    (metres of OPL), the fluorescent-surface case of Eq. 10."""
    sc = box_scene(seed=seed, width=width, height=height, n_bins=n_bins, bin_width=bin_width, spp=spp,
                   max_depth=max_depth)
    nt = sc.n_tris
    short = slice(10, 22)  # the short box's 12 triangles follow the room's 10
    v = sc.vertices.astype(np.float64)
    f = sc.indices.astype(np.int64)
    _, bf = outward(v, f[short])
    f = f.copy()
    f[short] = bf
    mat = sc.mat_type.copy()
    mat[short] = MAT_DIELECTRIC
    ior_a = np.ones(nt, np.float32)
    ior_a[short] = ior
    delay = None
    if delay_mean > 0.0:
        delay = np.zeros(nt, np.float32)
        delay[:10] = delay_mean
    sc.indices = np.ascontiguousarray(f, np.uint32)
    sc.mat_type = mat
    sc.ior = ior_a
    sc.delay = delay
    sc.name = "glass_box"
    return sc

