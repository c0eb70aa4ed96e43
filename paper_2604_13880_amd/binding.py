"""Thin Python binding of libcg (ctypes).  Argument marshalling only:
every step of the cartogram path runs in the library's HIP kernels.
PyTorch supplies device memory and streams.

Names follow the C ABI (include/cg.h): rasterize, integral_image,
map_points, region_areas, step_series.  The binding raises when the
shared library has not been built or no GPU is usable; it never falls
back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcg.so")

F32, COMP, F64, F64ACC = 0, 1, 2, 3
DIRECT, CUMULATIVE = 0, 1
FRAMES_POSITIONS, FRAMES_VALUES = 0, 1
AREA_PIXEL, AREA_POLYGON = 0, 1
STATUS_CONVERGED, STATUS_STALLED, STATUS_MAXITER, STATUS_ERROR = 0, 1, 2, 3
FLAG_CONTESTED, FLAG_OVERFLOW, FLAG_FALLBACK, FLAG_BADVALUES = 1, 2, 4, 8


class CgInim(C.Structure):
    _fields_ = [("N", C.c_int32), ("precision", C.c_int32), ("pitch", C.c_int64),
                ("S", C.c_void_p), ("T", C.c_void_p), ("HA", C.c_void_p), ("HB", C.c_void_p)]


class CgSeriesDesc(C.Structure):
    _fields_ = [("map", C.c_void_p), ("xy0", C.c_void_p), ("N", C.c_int32), ("n_steps", C.c_int32),
                ("values", C.c_void_p), ("mode", C.c_int32), ("shape", C.c_float),
                ("area_source", C.c_int32), ("tol", C.c_float), ("patience", C.c_int32),
                ("max_iters", C.c_int32), ("fixed_iters", C.c_int32), ("precision", C.c_int32),
                ("frames", C.c_int32), ("extra", C.c_void_p), ("n_extra", C.c_int64),
                ("init_field", C.c_void_p), ("init_G", C.c_int32), ("area_min", C.c_float),
                ("area_max", C.c_float), ("mass_t0", C.c_int32), ("mass_t1", C.c_int32), ("frame_mode", C.c_int32)]


class CgNetConfig(C.Structure):
    _fields_ = [("base_channels", C.c_int32), ("levels", C.c_int32), ("height", C.c_int32),
                ("width", C.c_int32), ("max_batch", C.c_int32), ("out_scale", C.c_float), ("seed", C.c_uint64),
                ("in_channels", C.c_int32), ("residual_gain", C.c_float)]


class CgQualityOut(C.Structure):
    _fields_ = [("adjacency", C.c_void_p), ("overlap", C.c_void_p), ("pixels", C.c_void_p),
                ("shape", C.c_void_p), ("bary", C.c_void_p), ("summary", C.c_void_p)]


class CgSeriesOut(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("extra_xy", C.c_void_p), ("frames", C.c_void_p),
                ("iters", C.c_void_p), ("status", C.c_void_p), ("flags", C.c_void_p),
                ("eps", C.c_void_p), ("xi", C.c_void_p), ("warm_step", C.c_void_p),
                ("frame_iters", C.c_void_p), ("frame_xi", C.c_void_p)]


_lib = None


def lib():
    """The loaded libcg (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_13880_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "cg_create": (C.c_int, [C.c_int, C.POINTER(vp)]),
            "cg_destroy": (C.c_int, [vp]),
            "cg_last_error": (C.c_char_p, [vp]),
            "cg_stream": (vp, [vp]),
            "cg_map_build": (C.c_int, [vp, i32, i32, i32, vp, vp, vp, C.POINTER(vp)]),
            "cg_map_destroy": (C.c_int, [vp]),
            "cg_map_n_edges": (i32, [vp]),
            "cg_rasterize": (C.c_int, [vp, vp, vp, C.c_int, vp, vp, vp, vp]),
            "cg_inim_size": (C.c_int, [C.c_int, C.c_int, C.POINTER(i64), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
            "cg_integral_image": (C.c_int, [vp, C.c_int, vp, vp, i32, vp, C.c_int, C.POINTER(CgInim), vp]),
            "cg_integral_image_noalloc": (C.c_int, [vp, C.c_int, vp, vp, i32, vp, C.c_int, C.POINTER(CgInim), vp]),
            "cg_map_points": (C.c_int, [vp, C.POINTER(CgInim), vp, vp, i64, vp]),
            "cg_region_areas": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "cg_quality": (C.c_int, [vp, vp, C.c_int, vp, vp, vp, vp, C.POINTER(CgQualityOut), vp]),
            "cg_step_series": (C.c_int, [vp, C.POINTER(CgSeriesDesc), C.c_int, C.POINTER(CgSeriesOut), i32, vp]),
            "cg_tile_shape": (C.c_int, [vp, C.c_int, C.c_int, i64, C.POINTER(i32), C.POINTER(i32)]),
            "cg_autotune": (C.c_int, [vp, C.c_int, C.c_int, i32, C.c_char_p]),
            "cg_set_tile_shape": (C.c_int, [vp, C.c_int, C.c_int, i64, i32, i32]),
            "cg_profile_stage": (C.c_int, [vp, C.c_char_p, i32]),
            "cg_profile_read": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(i64)]),
            "cg_log_density": (C.c_int, [vp, C.c_int, vp, vp, vp, i32, C.c_float, vp, vp]),
            "cg_log_density_maps": (C.c_int, [vp, i32, vp, vp, C.c_int, vp, C.c_float, vp, vp]),
            "cg_tracer_field": (C.c_int, [vp, i32, vp, vp, vp]),
            "cg_field_pool": (C.c_int, [vp, i32, vp, i32, vp, vp]),
            "cg_net_create": (C.c_int, [vp, C.POINTER(CgNetConfig), C.POINTER(vp)]),
            "cg_net_destroy": (C.c_int, [vp]),
            "cg_net_n_params": (i64, [vp]),
            "cg_net_get_params": (C.c_int, [vp, vp, vp]),
            "cg_net_set_params": (C.c_int, [vp, vp, vp]),
            "cg_net_get_grads": (C.c_int, [vp, vp, vp]),
            "cg_net_zero_grads": (C.c_int, [vp, vp]),
            "cg_net_forward": (C.c_int, [vp, vp, i32, vp, vp]),
            "cg_net_backward": (C.c_int, [vp, vp, i32, vp, vp]),
            "cg_net_adam_step": (C.c_int, [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
            "cg_net_save": (C.c_int, [vp, C.c_char_p]),
            "cg_net_load": (C.c_int, [vp, C.c_char_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return ["cg_create", "cg_destroy", "cg_last_error", "cg_stream", "cg_map_build", "cg_map_destroy",
            "cg_map_n_edges", "cg_rasterize", "cg_inim_size", "cg_integral_image", "cg_integral_image_noalloc",
            "cg_map_points",
            "cg_region_areas", "cg_quality", "cg_step_series", "cg_tile_shape", "cg_set_tile_shape", "cg_autotune", "cg_profile_stage",
            "cg_profile_read", "cg_log_density", "cg_log_density_maps", "cg_tracer_field", "cg_field_pool", "cg_net_create", "cg_net_destroy",
            "cg_net_n_params", "cg_net_get_params", "cg_net_set_params", "cg_net_get_grads", "cg_net_zero_grads",
            "cg_net_forward", "cg_net_backward", "cg_net_adam_step", "cg_net_save", "cg_net_load"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    t = t.to(device="cuda", dtype=dtype).contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


class CartogramError(RuntimeError):
    pass


@dataclass
class Inim:
    N: int
    precision: int
    pitch: int
    S: torch.Tensor     # [(N+1), pitch]
    T: torch.Tensor
    HA: torch.Tensor    # [2N+1]
    HB: torch.Tensor

    def c(self) -> CgInim:
        return CgInim(self.N, self.precision, self.pitch, self.S.data_ptr(), self.T.data_ptr(),
                      self.HA.data_ptr(), self.HB.data_ptr())


class Map:
    """Map topology uploaded by cg_map_build (vertex positions stay with the caller)."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, n_vertices: int, n_regions: int):
        self.ctx = ctx
        self.handle = handle
        self.n_vertices = n_vertices
        self.n_regions = n_regions

    @property
    def n_edges(self) -> int:
        return lib().cg_map_n_edges(self.handle)

    def __del__(self):
        try:
            if self.handle:
                lib().cg_map_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise CartogramError("no GPU visible: the cartogram library runs on the GPU only")
        torch.cuda.set_device(device)
        h = C.c_void_p()
        rc = lib().cg_create(device, C.byref(h))
        if rc != 0:
            raise CartogramError(f"cg_create failed ({rc})")
        self.handle = h
        self.device = device

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().cg_last_error(self.handle).decode()
            raise CartogramError(f"{what} failed ({rc}): {msg}")

    def close(self):
        if getattr(self, "handle", None):
            lib().cg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- topology ------------------------------------------------------------
    def map_build(self, ring_off, ring_idx, ring_reg, n_vertices: int, n_regions: int) -> Map:
        ro = np.ascontiguousarray(ring_off, dtype=np.int32)
        ri = np.ascontiguousarray(ring_idx, dtype=np.int32)
        rr = np.ascontiguousarray(ring_reg, dtype=np.int32)
        h = C.c_void_p()
        rc = lib().cg_map_build(self.handle, int(n_vertices), int(n_regions), int(len(rr)),
                                ro.ctypes.data_as(C.c_void_p), ri.ctypes.data_as(C.c_void_p),
                                rr.ctypes.data_as(C.c_void_p), C.byref(h))
        self._check(rc, "cg_map_build")
        return Map(self, h, int(n_vertices), int(n_regions))

    def map_from(self, pm) -> Map:
        """Map from an object with ring_off / ring_idx / ring_reg / n_vertices / n_regions."""
        return self.map_build(pm.ring_off, pm.ring_idx, pm.ring_reg, pm.n_vertices, pm.n_regions)

    # -- the five steps ------------------------------------------------------
    def rasterize(self, m: Map, xy, N: int):
        xy = _dev(xy, torch.float32, (-1, 2))
        labels = torch.empty((N, N), dtype=torch.int16, device="cuda")
        counts = torch.empty(m.n_regions + 1, dtype=torch.int64, device="cuda")
        contested = torch.zeros(1, dtype=torch.int64, device="cuda")
        rc = lib().cg_rasterize(self.handle, m.handle, _ptr(xy), int(N), _ptr(labels), _ptr(counts),
                                _ptr(contested), _stream())
        self._check(rc, "cg_rasterize")
        return labels, counts, contested

    def inim_alloc(self, N: int, precision: int) -> Inim:
        pitch = C.c_int64()
        tb = C.c_size_t()
        mb = C.c_size_t()
        self._check(lib().cg_inim_size(int(N), int(precision), C.byref(pitch), C.byref(tb), C.byref(mb)),
                    "cg_inim_size")
        dt = torch.float64 if precision == F64 else torch.float32
        S = torch.empty((N + 1, pitch.value), dtype=dt, device="cuda")
        T = torch.empty((N + 1, pitch.value), dtype=dt, device="cuda")
        HA = torch.empty(2 * N + 1, dtype=dt, device="cuda")
        HB = torch.empty(2 * N + 1, dtype=dt, device="cuda")
        return Inim(int(N), int(precision), int(pitch.value), S, T, HA, HB)

    def integral_image(self, N: int, labels=None, lut=None, density=None, precision: int = F32,
                       out: Inim | None = None, noalloc: bool = False) -> Inim:
        """Step 4 through cg_integral_image, or through the allocation-free
        cg_integral_image_noalloc when `noalloc` (inputs and `out` must then
        already be device tensors for the call itself to allocate nothing)."""
        im = out or self.inim_alloc(N, precision)
        cim = im.c()
        name = "cg_integral_image_noalloc" if noalloc else "cg_integral_image"
        fn = getattr(lib(), name)
        if density is not None:
            dens = _dev(density, torch.float32, (N, N))
            rc = fn(self.handle, int(N), None, None, 0, _ptr(dens), int(precision), C.byref(cim), _stream())
        else:
            lab = labels if (isinstance(labels, torch.Tensor) and labels.is_cuda) else \
                torch.as_tensor(np.asarray(labels).astype(np.uint16).view(np.int16)).cuda()
            lab = lab.contiguous()
            lt = _dev(lut, torch.float32)
            rc = fn(self.handle, int(N), _ptr(lab), _ptr(lt), int(lt.numel()), None, int(precision), C.byref(cim),
                    _stream())
        self._check(rc, name)
        return im

    def map_points(self, im: Inim, xy_in, xy_out=None):
        xin = _dev(xy_in, torch.float32, (-1, 2))
        xout = xin if xy_out is None else xy_out
        cim = im.c()
        rc = lib().cg_map_points(self.handle, C.byref(cim), _ptr(xin), _ptr(xout), int(xin.shape[0]), _stream())
        self._check(rc, "cg_map_points")
        return xout

    def region_areas(self, m: Map, xy, values=None):
        xy = _dev(xy, torch.float32, (-1, 2))
        areas = torch.empty(m.n_regions + 1, dtype=torch.float64, device="cuda")
        vals = None if values is None else _dev(values, torch.float32)
        ex = None if values is None else torch.empty(2, dtype=torch.float64, device="cuda")
        rc = lib().cg_region_areas(self.handle, m.handle, _ptr(xy), _ptr(vals), _ptr(areas), _ptr(ex), _stream())
        self._check(rc, "cg_region_areas")
        return areas, ex

    def quality(self, m: Map, N: int, xy_map, xy_cart, labels_map=None, labels_cart=None) -> dict:
        """Geographic-distortion measures of the cartogram xy_cart against
        the map xy_map (cg_quality), from their label maps at texture size N
        (rasterised here through cg_rasterize when not given)."""
        xm = _dev(xy_map, torch.float32, (-1, 2))
        xc = _dev(xy_cart, torch.float32, (-1, 2))
        if labels_map is None:
            labels_map = self.rasterize(m, xm, N)[0]
        if labels_cart is None:
            labels_cart = self.rasterize(m, xc, N)[0]
        R = m.n_regions
        f64, i64 = torch.float64, torch.int64
        out = dict(adjacency=torch.empty(3, dtype=i64, device="cuda"),
                   overlap=torch.empty(R + 1, dtype=i64, device="cuda"),
                   pixels=torch.empty((2, R + 1), dtype=i64, device="cuda"),
                   shape=torch.empty(R + 1, dtype=f64, device="cuda"),
                   bary=torch.empty((2, R + 1, 2), dtype=f64, device="cuda"),
                   summary=torch.empty(4, dtype=f64, device="cuda"))
        q = CgQualityOut(*[C.c_void_p(out[k].data_ptr()) for k in
                           ("adjacency", "overlap", "pixels", "shape", "bary", "summary")])
        rc = lib().cg_quality(self.handle, m.handle, int(N), _ptr(labels_map.contiguous()),
                              _ptr(labels_cart.contiguous()), _ptr(xm), _ptr(xc), C.byref(q), _stream())
        self._check(rc, "cg_quality")
        s = out["summary"].cpu().numpy()
        out.update(tau=float(s[0]), shape_mean=float(s[1]), shape_max=float(s[2]), rel_pos=float(s[3]))
        return out

    def log_density(self, labels, counts, values, shape: float = 1.0):
        """log(d / mean d) of the Step-3 density from a label map and pixel counts."""
        N = int(labels.shape[-1])
        vals = _dev(values, torch.float32)
        out = torch.empty((N, N), dtype=torch.float32, device="cuda")
        rc = lib().cg_log_density(self.handle, N, _ptr(labels.contiguous()), _ptr(counts), _ptr(vals),
                                  int(vals.numel()), float(shape), _ptr(out), _stream())
        self._check(rc, "cg_log_density")
        return out

    def log_density_maps(self, maps, xys, N: int, values, shape: float = 1.0):
        """log(d / mean d) textures [n][N][N] of several maps in one call
        (device positions xys[k] [n_k][2] and values[k] [R_k])."""
        n = len(maps)
        xs = [_dev(x, torch.float32, (-1, 2)) for x in xys]
        vs = [_dev(v, torch.float32) for v in values]
        out = torch.empty((n, N, N), dtype=torch.float32, device="cuda")
        mp = (C.c_void_p * n)(*[m.handle for m in maps])
        xp = (C.c_void_p * n)(*[_ptr(x) for x in xs])
        vp_ = (C.c_void_p * n)(*[_ptr(v) for v in vs])
        rc = lib().cg_log_density_maps(self.handle, n, mp, xp, int(N), vp_, float(shape), _ptr(out), _stream())
        self._check(rc, "cg_log_density_maps")
        return out

    def tracer_grid(self, G: int):
        """Pixel-centre positions of a G x G grid, float32 [G*G, 2]."""
        out = torch.empty((G * G, 2), dtype=torch.float32, device="cuda")
        self._check(lib().cg_tracer_field(self.handle, int(G), None, _ptr(out), _stream()), "cg_tracer_field")
        return out

    def tracer_field(self, G: int, final_xy):
        """Displacement of moved tracers from their pixel centres, float32 [G, G, 2]."""
        fin = _dev(final_xy, torch.float32, (-1, 2))
        out = torch.empty((G, G, 2), dtype=torch.float32, device="cuda")
        self._check(lib().cg_tracer_field(self.handle, int(G), _ptr(fin), _ptr(out), _stream()), "cg_tracer_field")
        return out

    def field_pool(self, field, factor: int):
        """Box average of a [G, G, 2] field over factor x factor cells."""
        f = _dev(field, torch.float32)
        G = int(f.shape[0])
        out = torch.empty((G // factor, G // factor, 2), dtype=torch.float32, device="cuda")
        self._check(lib().cg_field_pool(self.handle, G, _ptr(f), int(factor), _ptr(out), _stream()), "cg_field_pool")
        return out

    def profile_stage(self, stage: str | None, every: int = 1):
        self._check(lib().cg_profile_stage(self.handle, (stage or "").encode(), int(every)), "cg_profile_stage")

    def profile_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(lib().cg_profile_read(self.handle, C.byref(ms), C.byref(n)), "cg_profile_read")
        return ms.value, n.value

    def tile_shape(self, N: int, precision: int, batch_pixels: int):
        tw, th = C.c_int32(), C.c_int32()
        self._check(lib().cg_tile_shape(self.handle, int(N), int(precision), int(batch_pixels),
                                        C.byref(tw), C.byref(th)), "cg_tile_shape")
        return tw.value, th.value

    def set_tile_shape(self, N: int, precision: int, batch_pixels: int, tw: int, th: int):
        self._check(lib().cg_set_tile_shape(self.handle, int(N), int(precision), int(batch_pixels), int(tw), int(th)),
                    "cg_set_tile_shape")

    def autotune(self, N: int, precision: int, batch: int = 1, cache_path: str | None = None):
        self._check(lib().cg_autotune(self.handle, int(N), int(precision), int(batch),
                                      None if cache_path is None else cache_path.encode()), "cg_autotune")
        return self.tile_shape(N, precision, int(N) * int(N) * int(batch))

    def step_series(self, series: list[dict], graph_iters: int = 8):
        """Run cartogram series.  Each dict: map (Map), xy0 (float32 [n,2]),
        N, values ([T,R] or [R]), and optional mode, shape, area_source,
        tol, patience, max_iters, fixed_iters, precision, frames, frame_mode
        ("positions" or "values"), area_fraction ((A_min, A_max) or
        (A_min, A_max, t0, t1): background mass of eq.(4)), extra ([m,2]
        tracer points), init_field ([G,G,2] warm-start displacement at
        pixel centres).  Returns one dict per series with xy [T,n,2],
        extra_xy, frames, iters, status, flags, eps, xi (host numpy for the
        scalars), and frame_iters / frame_xi [T-1,K-1] for value frames."""
        descs = (CgSeriesDesc * len(series))()
        outs = (CgSeriesOut * len(series))()
        keep, results = [], []
        for k, s in enumerate(series):
            m: Map = s["map"]
            vals = _dev(s["values"], torch.float32)
            if vals.dim() == 1:
                vals = vals.reshape(1, -1)
            T = int(vals.shape[0])
            xy0 = _dev(s["xy0"], torch.float32, (-1, 2))
            n = xy0.shape[0]
            extra = s.get("extra")
            extra = None if extra is None else _dev(extra, torch.float32, (-1, 2))
            field = s.get("init_field")
            field = None if field is None else _dev(field, torch.float32)
            K = int(s.get("frames", 0))
            xy = torch.empty((T, n, 2), dtype=torch.float32, device="cuda")
            exy = None if extra is None else torch.empty((T, extra.shape[0], 2), dtype=torch.float32, device="cuda")
            fr = torch.empty((max(T - 1, 0), K - 1, n, 2), dtype=torch.float32, device="cuda") if K >= 2 else None
            host = {key: np.zeros(T, dtype=np.int32) for key in ("iters", "status", "flags")}
            host.update({key: np.zeros(T, dtype=np.float64) for key in ("eps", "xi")})
            host["warm_step"] = np.zeros(T, dtype=np.float32)
            d = descs[k]
            d.map = m.handle
            d.xy0 = xy0.data_ptr()
            d.N = int(s["N"])
            d.n_steps = T
            d.values = vals.data_ptr()
            d.mode = int(s.get("mode", DIRECT))
            d.shape = float(s.get("shape", 1.0))
            d.area_source = int(s.get("area_source", AREA_PIXEL))
            d.tol = float(s.get("tol", 0.01))
            d.patience = int(s.get("patience", 32))
            d.max_iters = int(s.get("max_iters", 512))
            d.fixed_iters = int(s.get("fixed_iters", 0))
            d.precision = int(s.get("precision", F32))
            d.frames = K
            d.extra = 0 if extra is None else extra.data_ptr()
            d.n_extra = 0 if extra is None else int(extra.shape[0])
            d.init_field = 0 if field is None else field.data_ptr()
            d.init_G = 0 if field is None else int(field.shape[0])
            af = s.get("area_fraction")
            if af is not None:
                d.area_min, d.area_max = float(af[0]), float(af[1])
                d.mass_t0, d.mass_t1 = (int(af[2]), int(af[3])) if len(af) > 2 else (0, -1)
            else:
                d.mass_t0, d.mass_t1 = 0, -1
            fm = s.get("frame_mode", FRAMES_POSITIONS)
            d.frame_mode = {"positions": FRAMES_POSITIONS, "values": FRAMES_VALUES}.get(fm, fm) \
                if isinstance(fm, str) else int(fm)
            if K >= 2 and d.frame_mode == FRAMES_VALUES:
                host["frame_iters"] = np.zeros((max(T - 1, 0), K - 1), dtype=np.int32)
                host["frame_xi"] = np.zeros((max(T - 1, 0), K - 1), dtype=np.float64)
            o = outs[k]
            o.xy = xy.data_ptr()
            o.extra_xy = 0 if exy is None else exy.data_ptr()
            o.frames = 0 if fr is None else fr.data_ptr()
            for key in ("iters", "status", "flags", "eps", "xi", "warm_step", "frame_iters", "frame_xi"):
                if key in host:
                    setattr(o, key, host[key].ctypes.data)
            keep += [vals, xy0, extra, field, xy, exy, fr]
            results.append(dict(xy=xy, extra_xy=exy, frames=fr, **host))
        rc = lib().cg_step_series(self.handle, descs, len(series), outs, int(graph_iters), _stream())
        self._check(rc, "cg_step_series")
        return results


class Net:
    """Learned warm start (include/cg_net.h): U-Net trained and run by the
    library's own kernels."""

    def __init__(self, ctx: Context, base_channels: int = 32, levels: int = 4, height: int = 512,
                 width: int = 512, max_batch: int = 8, out_scale: float = 0.1, seed: int = 0,
                 in_channels: int = 1, residual_gain: float = 0.0):
        self.ctx = ctx
        cfg = CgNetConfig(int(base_channels), int(levels), int(height), int(width), int(max_batch),
                          float(out_scale), int(seed), int(in_channels), float(residual_gain))
        self.in_channels = int(in_channels)
        h = C.c_void_p()
        ctx._check(lib().cg_net_create(ctx.handle, C.byref(cfg), C.byref(h)), "cg_net_create")
        self.handle = h
        self.H, self.W, self.max_batch = int(height), int(width), int(max_batch)
        self.n_params = int(lib().cg_net_n_params(h))

    def close(self):
        if getattr(self, "handle", None):
            lib().cg_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self.ctx._check(lib().cg_net_get_params(self.handle, _ptr(out), _stream()), "cg_net_get_params")
        return out

    def set_params(self, p):
        p = _dev(p, torch.float32)
        if p.numel() != self.n_params:
            raise CartogramError(f"expected {self.n_params} parameters, got {p.numel()}")
        self.ctx._check(lib().cg_net_set_params(self.handle, _ptr(p), _stream()), "cg_net_set_params")
        torch.cuda.current_stream().synchronize()

    def grads(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self.ctx._check(lib().cg_net_get_grads(self.handle, _ptr(out), _stream()), "cg_net_get_grads")
        return out

    def zero_grads(self):
        self.ctx._check(lib().cg_net_zero_grads(self.handle, _stream()), "cg_net_zero_grads")

    def forward(self, x, out=None) -> torch.Tensor:
        """x: [B, H, W] (one channel) or [B, H, W, in_channels]."""
        x = _dev(x, torch.float32)
        B = int(x.shape[0])
        if x.numel() != B * self.H * self.W * self.in_channels:
            raise CartogramError(f"net input must hold {self.in_channels} channel(s) of {self.H}x{self.W}")
        if out is None:
            out = torch.empty((B, self.H, self.W, 2), dtype=torch.float32, device="cuda")
        self.ctx._check(lib().cg_net_forward(self.handle, _ptr(x), B, _ptr(out), _stream()), "cg_net_forward")
        return out

    def backward(self, target, loss=None):
        t = _dev(target, torch.float32)
        B = int(t.shape[0])
        self.ctx._check(lib().cg_net_backward(self.handle, _ptr(t), B, _ptr(loss), _stream()), "cg_net_backward")

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.ctx._check(lib().cg_net_adam_step(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                               _stream()), "cg_net_adam_step")

    def save(self, path: str):
        self.ctx._check(lib().cg_net_save(self.handle, path.encode()), "cg_net_save")

    def load(self, path: str):
        self.ctx._check(lib().cg_net_load(self.handle, path.encode()), "cg_net_load")
