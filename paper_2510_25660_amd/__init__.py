"""MI355X-native transient path tracer (arXiv 2510.25660, "mitransient").

Python front-end over the C ABI of libtrhip.so (include/trhip.h).  PyTorch
provides device memory and streams; every step of rendering runs in the HIP
kernels of the library.

    import paper_2510_25660_amd as tr
    from paper_2510_25660_amd import scenes
    dev = tr.upload(scenes.box_scene())
    steady, film = tr.render_transient(dev, spp=16)    # (H, W), (H, W, T)

``TransientRender`` is a ``torch.autograd.Function`` whose backward is the
library's path-replay adjoint (Sec. 4.4 of the paper).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import scenes
from ._binding import (FLAG_ACCUMULATE, FLAG_DETERMINISTIC, FLAG_FROZEN_PROPOSAL, FLAG_NLOS_AREA_SAMPLING,
                       FLAG_PIXEL_CENTRE, BatchInfo, BatchOpts, RenderDesc, SceneDesc, SceneInfo, TrhipError, check,
                       lib)

__all__ = [
    "scenes", "upload", "DeviceScene", "render_transient", "render_transient_backward", "render_transient_counted",
    "render_transient_tangent", "render_phasor", "poisson_noise", "render_transient_records", "numerics_probe",
    "TransientRender", "Batch",
    "TrhipError", "FLAG_PIXEL_CENTRE", "FLAG_ACCUMULATE", "FLAG_FROZEN_PROPOSAL", "FLAG_NLOS_AREA_SAMPLING",
    "FLAG_DETERMINISTIC",
    "version",
]


def version() -> str:
    return lib().trhip_version().decode()


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _f3(v):
    return (C.c_float * 3)(*[float(x) for x in v])


def make_scene_desc(sc: "scenes.Scene", builder="ploc"):
    """Fill a trhip_scene_desc from a Scene; returns (desc, keepalive)."""
    verts = np.ascontiguousarray(sc.vertices, np.float32)
    idx = np.ascontiguousarray(sc.indices, np.uint32)
    mat = np.ascontiguousarray(sc.mat_type, np.uint8)
    alb = np.ascontiguousarray(sc.albedo, np.float32)
    rough = np.ascontiguousarray(sc.roughness, np.float32)
    keep = [verts, idx, mat, alb, rough]
    d = SceneDesc()
    fp = C.POINTER(C.c_float)
    d.vertices = verts.ctypes.data_as(fp)
    d.n_vertices = verts.shape[0]
    d.indices = idx.ctypes.data_as(C.POINTER(C.c_uint32))
    d.n_triangles = idx.shape[0]
    d.mat_type = mat.ctypes.data_as(C.POINTER(C.c_uint8))
    d.albedo = alb.ctypes.data_as(fp)
    d.roughness = rough.ctypes.data_as(fp)
    d.light_pos = _f3(sc.light_pos)
    d.light_intensity = sc.light_intensity
    d.sensor = int(sc.sensor)
    d.width = sc.width
    d.height = sc.height
    d.cam_origin = _f3(sc.cam_origin)
    d.cam_right = _f3(sc.cam_right)
    d.cam_up = _f3(sc.cam_up)
    d.cam_fwd = _f3(sc.cam_fwd)
    d.tan_x = sc.tan_x
    d.tan_y = sc.tan_y
    if sc.scan_points is not None:
        scan = np.ascontiguousarray(sc.scan_points, np.float32)
        keep.append(scan)
        d.scan_points = scan.ctypes.data_as(fp)
    d.wall_normal = _f3(sc.wall_normal)
    d.wall_albedo = sc.wall_albedo
    d.laser_power = sc.laser_power
    d.sigma_t = sc.sigma_t
    d.medium_albedo = sc.medium_albedo
    d.n_bins = sc.n_bins
    d.bin_width = sc.bin_width
    d.bin_start = sc.bin_start
    d.camera_unwarp = int(bool(sc.camera_unwarp))
    from ._binding import BUILDERS
    d.bvh_builder = BUILDERS[builder] if isinstance(builder, str) else int(builder)
    for name in ("ior", "delay"):
        arr = getattr(sc, name, None)
        if arr is not None:
            arr = np.ascontiguousarray(arr, np.float32)
            keep.append(arr)
            setattr(d, name, arr.ctypes.data_as(fp))
    d.medium_ior = float(getattr(sc, "medium_ior", 1.0))
    return d, keep


class DeviceScene:
    """A scene uploaded to the GPU with its BVH (owns a trhip_scene*)."""

    def __init__(self, sc: "scenes.Scene", stream=None, builder="ploc"):
        self.scene = sc
        desc, keep = make_scene_desc(sc, builder)
        h = C.c_void_p()
        check(lib().trhip_scene_create(C.byref(desc), _stream_handle(stream), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise TrhipError(5, "scene destroyed")
        return self._h

    def info(self) -> dict:
        inf = SceneInfo()
        check(lib().trhip_scene_get_info(self.handle, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in SceneInfo._fields_}

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            check(lib().trhip_scene_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def upload(sc: "scenes.Scene", stream=None, builder="ploc") -> DeviceScene:
    """Upload a scene and build its BVH on the device (builder "ploc" or "lbvh")."""
    return DeviceScene(sc, stream, builder)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def make_render_desc(dev: DeviceScene, spp=None, seed=None, max_depth=None, sample_offset=0, norm_spp=0,
                     stream_id=0, pixel_centre=False, accumulate=False, frozen=False, albedo=None,
                     roughness=None, tile_pixels=0, block_size=0, kernel="auto", nlos_area=False,
                     deterministic=False) -> RenderDesc:
    sc = dev.scene
    r = RenderDesc()
    r.spp = int(sc.spp if spp is None else spp)
    r.sample_offset = int(sample_offset)
    r.norm_spp = int(norm_spp)
    r.max_depth = int(sc.max_depth if max_depth is None else max_depth)
    r.seed = int(sc.seed if seed is None else seed)
    r.stream_id = int(stream_id)
    r.flags = ((FLAG_PIXEL_CENTRE if pixel_centre else 0) | (FLAG_ACCUMULATE if accumulate else 0)
               | (FLAG_FROZEN_PROPOSAL if frozen else 0) | (FLAG_NLOS_AREA_SAMPLING if nlos_area else 0)
               | (FLAG_DETERMINISTIC if deterministic else 0))
    r.albedo_override = _ptr(albedo)
    r.roughness_override = _ptr(roughness)
    r.tile_pixels = int(tile_pixels)
    r.block_size = int(block_size)
    from ._binding import KERNELS
    r.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return r


def _check_param(t, n, name):
    torch = _torch()
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor with {n} elements")
    return t


def _out(t, shape, name, optional=False):
    """A caller-supplied output buffer (checked: the kernels write exactly
    prod(shape) floats through its pointer), or a new one."""
    torch = _torch()
    if t is None:
        return None if optional else torch.empty(shape, device="cuda", dtype=torch.float32)
    n = int(np.prod(shape))
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor with {n} elements")
    return t


def render_transient(dev: DeviceScene, spp=None, seed=None, max_depth=None, film=None, steady=None, oow=None,
                     stream=None, return_oow=False, **kw):
    """Forward transient render.  Returns (steady [H, W], film [H, W, T])
    (and oow [H, W] with return_oow) as float32 CUDA tensors."""
    torch = _torch()
    sc = dev.scene
    shape = (sc.height, sc.width)
    n = sc.n_tris
    kw["albedo"] = _check_param(kw.get("albedo"), n, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), n, "roughness")
    film = _out(film, shape + (sc.n_bins,), "film")
    steady = _out(steady, shape, "steady")
    oow = _out(oow, shape, "oow", optional=not return_oow)
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    check(lib().trhip_render_transient(dev.handle, C.byref(r), _ptr(film), _ptr(steady), _ptr(oow),
                                       _stream_handle(stream)))
    if return_oow:
        return steady, film, oow
    return steady, film


def render_phasor(dev: DeviceScene, freqs, spp=None, seed=None, max_depth=None, phasor=None, steady=None,
                  stream=None, **kw):
    """Frequency-space film (trhip_render_phasor): returns (steady [H, W],
    phasor [H, W, K] complex64) for the K frequencies `freqs` (cycles per
    metre of optical path): the mean over samples of c exp(-2 pi i f tof)."""
    torch = _torch()
    sc = dev.scene
    shape = (sc.height, sc.width)
    f = np.ascontiguousarray(np.asarray(freqs, dtype=np.float32).ravel())
    k = int(f.size)
    kw["albedo"] = _check_param(kw.get("albedo"), sc.n_tris, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), sc.n_tris, "roughness")
    phasor = _out(phasor, shape + (k, 2), "phasor")
    steady = _out(steady, shape, "steady")
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    check(lib().trhip_render_phasor(dev.handle, C.byref(r), f.ctypes.data_as(C.POINTER(C.c_float)), k,
                                    _ptr(phasor), _ptr(steady), _stream_handle(stream)))
    return steady, torch.view_as_complex(phasor)


def render_transient_tangent(dev: DeviceScene, tangent_albedo=None, tangent_roughness=None, spp=None, seed=None,
                             max_depth=None, film=None, dfilm=None, steady=None, stream=None, **kw):
    """Forward-mode derivative (trhip_render_transient_tangent): returns
    (steady [H, W], film [H, W, T], dfilm [H, W, T]) where dfilm is the
    derivative of the film along (tangent_albedo, tangent_roughness)."""
    torch = _torch()
    sc = dev.scene
    shape = (sc.height, sc.width)
    n = sc.n_tris
    kw["albedo"] = _check_param(kw.get("albedo"), n, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), n, "roughness")
    ta = _check_param(tangent_albedo, n, "tangent_albedo")
    trr = _check_param(tangent_roughness, n, "tangent_roughness")
    film = _out(film, shape + (sc.n_bins,), "film")
    dfilm = _out(dfilm, shape + (sc.n_bins,), "dfilm")
    steady = _out(steady, shape, "steady")
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    check(lib().trhip_render_transient_tangent(dev.handle, C.byref(r), _ptr(ta), _ptr(trr), _ptr(film), _ptr(dfilm),
                                               _ptr(steady), _stream_handle(stream)))
    return steady, film, dfilm


def render_transient_counted(dev: DeviceScene, spp=None, seed=None, max_depth=None, stream=None, **kw):
    """Same render as render_transient by the counting build of the kernel;
    returns (steady, film, counts) with counts a dict of work counters
    (BVH node visits, triangle tests, rays, shadow rays, vertices, Philox
    draws, contributions, per path) and of wave executions of node visits,
    triangle tests and vertices (their ratios are the mean active lanes).
    Synchronous."""
    torch = _torch()
    from ._binding import COUNT_NAMES
    sc = dev.scene
    shape = (sc.height, sc.width)
    kw["albedo"] = _check_param(kw.get("albedo"), sc.n_tris, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), sc.n_tris, "roughness")
    film = torch.empty(shape + (sc.n_bins,), device="cuda", dtype=torch.float32)
    steady = torch.empty(shape, device="cuda", dtype=torch.float32)
    counts = (C.c_uint64 * len(COUNT_NAMES))()
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    check(lib().trhip_render_transient_counted(dev.handle, C.byref(r), _ptr(film), _ptr(steady), None, counts,
                                               _stream_handle(stream)))
    return steady, film, dict(zip(COUNT_NAMES, [int(c) for c in counts]))


def render_transient_records(dev: DeviceScene, pixels, capacity=None, spp=None, seed=None, max_depth=None,
                             stream=None, **kw):
    """Same render as render_transient by the recording build of the kernel
    (trhip_render_transient_records): every next-event contribution of the
    listed pixels as a record (pixel, sample, vertex, bin, value, tof, tri).
    Returns (records numpy structured array, steady, film, oow); raises if
    the pixels made more than `capacity` contributions (default: 64 per
    path sample of the listed pixels).  Synchronous."""
    torch = _torch()
    from ._binding import RECORD_FIELDS
    sc = dev.scene
    shape = (sc.height, sc.width)
    kw["albedo"] = _check_param(kw.get("albedo"), sc.n_tris, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), sc.n_tris, "roughness")
    pix = np.unique(np.asarray(pixels, np.int64).ravel())
    if pix.size and (pix[0] < 0 or pix[-1] >= sc.n_pixels):
        raise ValueError("pixel index out of range")
    mask = torch.zeros(sc.n_pixels, device="cuda", dtype=torch.uint8)
    mask[torch.from_numpy(pix).cuda()] = 1
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    if capacity is None:
        capacity = max(1, 64 * int(pix.size) * int(r.spp))
    recs = torch.empty((int(capacity), 8), device="cuda", dtype=torch.int32)
    film = torch.empty(shape + (sc.n_bins,), device="cuda", dtype=torch.float32)
    steady = torch.empty(shape, device="cuda", dtype=torch.float32)
    oow = torch.empty(shape, device="cuda", dtype=torch.float32)
    n = C.c_uint64(0)
    check(lib().trhip_render_transient_records(dev.handle, C.byref(r), _ptr(mask), _ptr(recs), int(capacity),
                                               C.byref(n), _ptr(film), _ptr(steady), _ptr(oow),
                                               _stream_handle(stream)))
    if n.value > capacity:
        raise ValueError(f"{n.value} contributions exceed the record capacity {capacity}")
    out = recs[:n.value].cpu().numpy().view(np.dtype(RECORD_FIELDS)).reshape(-1)
    return out, steady, film, oow


def numerics_probe(op: str, inp=None, n=None, first=0, out=None, stream=None):
    """The renderer's primitives evaluated element by element on the device
    (trhip_numerics_probe): op "sincos2pi" / "log1m" over u = (first + i) 2^-24
    (n values; out float32 [n, 2] / [n]), "philox" (inp uint32 [n, 6] ->
    out [n, 4]), "div" (float32 [n, 2] -> [n]), "sqrt" ([n] -> [n])."""
    torch = _torch()
    from ._binding import PROBES
    code = PROBES[op]
    if op in ("sincos2pi", "log1m"):
        if n is None:
            raise ValueError("n is required")
        shape = (int(n), 2) if op == "sincos2pi" else (int(n),)
        out = torch.empty(shape, device="cuda", dtype=torch.float32) if out is None else out
        ip = None
    else:
        want = {"philox": (torch.int32, 6), "div": (torch.float32, 2), "sqrt": (torch.float32, 1)}[op]
        if not (inp.is_cuda and inp.is_contiguous() and inp.dtype == want[0] and inp.numel() % want[1] == 0):
            raise ValueError(f"{op}: input must be a contiguous CUDA {want[0]} tensor of rows of {want[1]}")
        n = inp.numel() // want[1]
        if out is None:
            out = (torch.empty((n, 4), device="cuda", dtype=torch.int32) if op == "philox"
                   else torch.empty(n, device="cuda", dtype=torch.float32))
        ip = _ptr(inp)
    check(lib().trhip_numerics_probe(code, ip, _ptr(out), int(n), int(first), _stream_handle(stream)))
    return out


def poisson_noise(film, scale=None, peak_count=1000.0, seed=0, out=None, stream=None):
    """One photon-count capture of a film: out = Poisson(scale * film) / scale
    (trhip_poisson_noise).  scale defaults to peak_count / max(film), so the
    brightest bin expects peak_count photons.  Returns (out, scale)."""
    torch = _torch()
    if not (film.is_cuda and film.dtype == torch.float32 and film.is_contiguous()):
        raise ValueError("film must be a contiguous float32 CUDA tensor")
    if scale is None:
        peak = float(film.max().item())
        if not peak > 0.0:
            raise ValueError("film has no positive bin; pass scale explicitly")
        scale = float(peak_count) / peak
    if out is None:
        out = torch.empty_like(film)
    check(lib().trhip_poisson_noise(_ptr(film), _ptr(out), film.numel(), float(scale), int(seed),
                                    _stream_handle(stream)))
    return out, scale


def render_transient_backward(dev: DeviceScene, grad_film, spp=None, seed=None, max_depth=None, primal=False,
                              stream=None, **kw):
    """Adjoint: returns (grad_albedo [nt], grad_roughness [nt]) (and the
    replayed primal film when primal=True)."""
    torch = _torch()
    sc = dev.scene
    n = sc.n_tris
    kw["albedo"] = _check_param(kw.get("albedo"), n, "albedo")
    kw["roughness"] = _check_param(kw.get("roughness"), n, "roughness")
    g = grad_film.contiguous()
    if g.numel() != sc.n_pixels * sc.n_bins or g.dtype != torch.float32 or not g.is_cuda:
        raise ValueError("grad_film must be a float32 CUDA tensor of the film's shape")
    ga = torch.empty(n, device="cuda", dtype=torch.float32)
    gr = torch.empty(n, device="cuda", dtype=torch.float32)
    pf = torch.empty((sc.height, sc.width, sc.n_bins), device="cuda", dtype=torch.float32) if primal else None
    r = make_render_desc(dev, spp, seed, max_depth, **kw)
    check(lib().trhip_render_transient_backward(dev.handle, C.byref(r), _ptr(g), _ptr(ga), _ptr(gr), _ptr(pf),
                                                _stream_handle(stream)))
    if primal:
        return ga, gr, pf
    return ga, gr


class Batch:
    """Many scenes rendered by one persistent, graph-captured launch
    (trhip_batch_*).  films[i] (allocated here unless given) receives what
    render_transient(devs[i], **renders[i]) would produce."""

    def __init__(self, devs, renders=None, films=None, block_size=0, tile_pixels=0, groups_per_cu=0,
                 kernel="auto", autotune=True, stream=None):
        torch = _torch()
        self.devs = list(devs)
        n = len(self.devs)
        renders = renders or [{} for _ in range(n)]
        if films is None:
            films = [None] * n
        films = [_out(f, (d.scene.height, d.scene.width, d.scene.n_bins), f"films[{i}]")
                 for i, (f, d) in enumerate(zip(films, self.devs))]
        self.films = films
        descs = (RenderDesc * n)()
        for i, (d, kw) in enumerate(zip(self.devs, renders)):
            descs[i] = make_render_desc(d, **kw)
        handles = (C.c_void_p * n)(*[d.handle.value for d in self.devs])
        fptrs = (C.c_void_p * n)(*[f.data_ptr() for f in films])
        from ._binding import KERNELS
        opts = BatchOpts(block_size, tile_pixels, groups_per_cu, KERNELS[kernel] if isinstance(kernel, str) else kernel,
                         1 if autotune else 0)
        h = C.c_void_p()
        check(lib().trhip_batch_create(handles, descs, n, fptrs, C.byref(opts), _stream_handle(stream),
                                       C.byref(h)))
        self._h = h

    def render(self, stream=None):
        check(lib().trhip_batch_render(self._h, _stream_handle(stream)))
        return self.films

    def info(self) -> dict:
        inf = BatchInfo()
        check(lib().trhip_batch_get_info(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in BatchInfo._fields_}

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            check(lib().trhip_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def _make_autograd():
    torch = _torch()

    class TransientRender(torch.autograd.Function):
        """film = TransientRender.apply(albedo, roughness, dev, opts) with opts a
        dict of render options (spp, seed, max_depth, ...).  The backward is
        the library's adjoint at the same seed; its forward-mode derivative
        (torch.autograd.forward_ad) is the library's tangent render."""

        @staticmethod
        def forward(albedo, roughness, dev, opts):
            _, film = render_transient(dev, albedo=albedo.contiguous(), roughness=roughness.contiguous(),
                                       **dict(opts or {}))
            return film

        @staticmethod
        def setup_context(ctx, inputs, output):
            albedo, roughness, dev, opts = inputs
            ctx.dev = dev
            ctx.opts = dict(opts or {})
            ctx.save_for_backward(albedo, roughness)
            ctx.save_for_forward(albedo, roughness)

        @staticmethod
        def jvp(ctx, d_albedo, d_roughness, _dev, _opts):
            albedo, roughness = ctx.saved_tensors
            ta = d_albedo.contiguous() if d_albedo is not None else None
            trr = d_roughness.contiguous() if d_roughness is not None else None
            _, _, dfilm = render_transient_tangent(ctx.dev, ta, trr, albedo=albedo.contiguous(),
                                                   roughness=roughness.contiguous(), **ctx.opts)
            return dfilm

        @staticmethod
        def backward(ctx, grad_film):
            albedo, roughness = ctx.saved_tensors
            ga, gr = render_transient_backward(ctx.dev, grad_film.contiguous(), albedo=albedo.contiguous(),
                                               roughness=roughness.contiguous(), **ctx.opts)
            return ga, gr, None, None

    return TransientRender


class _Lazy:
    _fn = None

    def __get__(self, obj, objtype=None):
        if _Lazy._fn is None:
            _Lazy._fn = _make_autograd()
        return _Lazy._fn


class _Namespace:
    TransientRender = _Lazy()


def __getattr__(name):
    if name == "TransientRender":
        return _Namespace.TransientRender
    raise AttributeError(name)
