"""Python binding of liblnr (include/lnr.h): locally non-rigid HDR registration
and deghosted merging on MI355X.

This module only marshals arguments: torch provides device memory and the
current HIP stream, and every step of the method runs in the library's HIP
kernels. Importing it without the built library raises (there is no CPU
fallback); build it with `python -m paper_1504_01441_amd.build`.

Typical use::

    import paper_1504_01441_amd as lnr
    ctx = lnr.Context()
    ref = lnr.Frame.from_numpy(y0, u0, v0, exposure=1.0)   # copies to the GPU
    src = lnr.Frame.from_numpy(y1, u1, v1, exposure=8.0)
    reg = lnr.register_pair(ctx, ref, src)
    hdr = lnr.merge(ctx, [ref, src], 0, [reg])              # [3][H][W] float32
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblnr.so")

LNR_Y8, LNR_I420, LNR_NV12 = 0, 1, 2
_STATUS = {0: "LNR_OK", -1: "LNR_E_ARG", -2: "LNR_E_UNSUPPORTED", -3: "LNR_E_TOO_SMALL",
           -4: "LNR_E_HIP", -5: "LNR_E_NOMEM", -6: "LNR_E_CAPTURE", -7: "LNR_E_WEIGHTS"}


class LnrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("tile", C.c_int32), ("patch_r", C.c_int32), ("corner_step", C.c_int32),
        ("corner_half", C.c_int32), ("quad_r", C.c_int32), ("corner_t", C.c_int32),
        ("max_levels", C.c_int32), ("min_level_dim", C.c_int32),
        ("radius_coarse", C.c_int32), ("radius0", C.c_int32), ("weed_iters", C.c_int32),
        ("weed_delta_min", C.c_int32), ("weed_delta_pct", C.c_int32), ("dt_iters", C.c_int32),
        ("weed_eps", C.c_double), ("sigma_s", C.c_double), ("sigma_r", C.c_double),
        ("n_min", C.c_double), ("ssim_sigma", C.c_double), ("ssim_radius", C.c_int32),
        ("search_frame", C.c_int32), ("ssim_c1", C.c_double), ("ssim_c2", C.c_double),
        ("sigma_e", C.c_double), ("seed", C.c_uint64),
        ("learned", C.c_int32), ("window_r", C.c_int32), ("conf_min", C.c_double),
    ]

    def __init__(self, **overrides):
        super().__init__()
        lib().lnr_default_params(C.byref(self))
        for k, v in overrides.items():
            if not any(k == f[0] for f in self._fields_):
                raise KeyError(k)
            setattr(self, k, v)


class _Frame(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("format", C.c_int32),
                ("reserved", C.c_int32), ("plane", C.c_void_p * 3), ("stride", C.c_int32 * 3),
                ("exposure", C.c_float)]


class _Sizes(C.Structure):
    _fields_ = [("levels", C.c_int32), ("tiles_total", C.c_int32), ("tile_off", C.c_int32 * 6),
                ("level_w", C.c_int32 * 5), ("level_h", C.c_int32 * 5),
                ("channels", C.c_int32), ("blend_levels", C.c_int32)]


class _TraceEntry(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("count", C.c_int32), ("reserved", C.c_int32),
                ("ms_total", C.c_double)]


class _Registration(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("corner_xy", "disp", "ssd", "flags", "counts", "H",
                                           "yeq_ref", "yeq_src", "warped0", "flow", "ntilde",
                                           "image", "yeq_warped")]


_lib = None


def lib():
    """The loaded liblnr.so; raises if it was not built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1504_01441_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.lnr_create.argtypes = [C.POINTER(vp), i32]
        L.lnr_destroy.argtypes = [vp]
        L.lnr_last_error.argtypes = [vp]
        L.lnr_last_error.restype = C.c_char_p
        L.lnr_default_params.argtypes = [C.POINTER(Params)]
        L.lnr_query_sizes.argtypes = [i32, i32, i32, C.POINTER(Params), C.POINTER(_Sizes)]
        L.lnr_register_pair.argtypes = [vp, C.POINTER(_Frame), C.POINTER(_Frame),
                                        C.POINTER(Params), C.POINTER(_Registration), vp]
        L.lnr_register_pair_noalloc.argtypes = [vp, C.POINTER(_Frame), C.POINTER(_Frame),
                                                C.POINTER(Params), C.POINTER(_Registration), vp]
        L.lnr_register_stack.argtypes = [vp, C.POINTER(_Frame), i32, C.POINTER(Params),
                                         C.POINTER(_Registration), C.POINTER(i32), vp]
        L.lnr_merge.argtypes = [vp, C.POINTER(_Frame), i32, i32, C.POINTER(_Registration),
                                C.POINTER(Params), vp, vp]
        L.lnr_merge_irradiance.argtypes = [vp, C.POINTER(_Frame), i32, i32, C.POINTER(_Registration),
                                C.POINTER(Params), vp, vp]
        L.lnr_stage_equalize.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
        L.lnr_stage_warp_q8.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        L.lnr_stage_search.argtypes = [vp, vp, vp, i32, i32, i32, C.POINTER(Params), vp, vp, vp,
                                       vp, vp]
        L.lnr_stage_weed_fit.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, C.POINTER(Params),
                                         vp, vp, vp, vp]
        L.lnr_stage_flow.argtypes = [vp, vp, vp, vp, i32, vp, i32, i32, C.POINTER(Params), vp,
                                     vp, vp]
        L.lnr_stage_backward_warp.argtypes = [vp, C.POINTER(_Frame), vp, vp, vp, vp, vp, vp]
        L.lnr_stage_frame_rgb.argtypes = [vp, C.POINTER(_Frame), vp, vp, vp, vp]
        L.lnr_stage_merge.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, C.POINTER(Params),
                                      vp, vp]
        L.lnr_meter.argtypes = [vp, vp, i32, i32, i32, i32, C.c_float, C.c_float, vp, vp]
        L.lnr_stage_irradiance.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, i32,
                                           C.POINTER(Params), vp, vp]
        L.lnr_stage_search_window.argtypes = [vp, vp, vp, i32, i32, i32, vp, C.POINTER(Params),
                                              vp, vp, vp, vp, vp]
        L.lnr_proposal_set.argtypes = [vp, vp, vp]
        L.lnr_proposal_get.argtypes = [vp, vp, vp]
        L.lnr_proposal_save.argtypes = [vp, C.c_char_p, vp]
        L.lnr_proposal_load.argtypes = [vp, C.c_char_p, vp]
        L.lnr_proposal_checkpoint_save.argtypes = [vp, C.c_char_p, C.c_uint64, vp]
        L.lnr_proposal_checkpoint_load.argtypes = [vp, C.c_char_p, C.POINTER(C.c_uint64), vp]
        L.lnr_proposal_inputs.argtypes = [vp, vp, vp, i32, i32, vp, vp]
        L.lnr_proposal_forward.argtypes = [vp, vp, i32, vp, vp]
        L.lnr_proposal_train_step.argtypes = [vp, vp, vp, i32, C.c_float, C.c_float, vp, vp, vp]
        L.lnr_register_batch.argtypes = [vp, C.POINTER(_Frame), C.POINTER(_Frame), i32,
                                         C.POINTER(Params), C.POINTER(_Registration), i32, vp]
        L.lnr_autotune_flow.argtypes = [vp, i32, i32, C.POINTER(Params), vp, vp]
        L.lnr_autotune_search.argtypes = [vp, i32, i32, C.POINTER(Params), vp, vp]
        L.lnr_set_flow_shape.argtypes = [vp, i32, i32, vp]
        L.lnr_set_search_shape.argtypes = [vp, i32, i32, i32, i32]
        L.lnr_flow_shapes.argtypes = [i32, i32, vp, i32]
        L.lnr_flow_shapes.restype = C.c_int32
        L.lnr_trace_enable.argtypes = [vp, i32]
        L.lnr_trace_read.argtypes = [vp, C.POINTER(_TraceEntry), i32]
        for name in ("lnr_trace_enable", "lnr_trace_read", "lnr_create", "lnr_query_sizes", "lnr_register_pair", "lnr_register_stack",
                     "lnr_register_pair_noalloc", "lnr_merge",
                     "lnr_proposal_checkpoint_save", "lnr_proposal_checkpoint_load", "lnr_stage_equalize", "lnr_stage_warp_q8", "lnr_stage_search",
                     "lnr_stage_weed_fit", "lnr_stage_flow", "lnr_stage_backward_warp",
                     "lnr_stage_frame_rgb", "lnr_stage_merge", "lnr_stage_search_window", "lnr_proposal_set",
                     "lnr_proposal_get", "lnr_proposal_inputs", "lnr_proposal_forward",
                     "lnr_proposal_train_step", "lnr_register_batch", "lnr_autotune_flow",
                     "lnr_autotune_search", "lnr_proposal_save", "lnr_proposal_load",
                     "lnr_merge_irradiance", "lnr_stage_irradiance", "lnr_meter",
                     "lnr_set_flow_shape", "lnr_set_search_shape"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


EXPORTED = ("lnr_create", "lnr_destroy", "lnr_last_error", "lnr_default_params",
            "lnr_query_sizes", "lnr_register_pair", "lnr_register_stack", "lnr_merge",
            "lnr_stage_equalize", "lnr_stage_warp_q8", "lnr_stage_search",
            "lnr_stage_weed_fit", "lnr_stage_flow", "lnr_stage_backward_warp",
            "lnr_stage_frame_rgb", "lnr_stage_merge", "lnr_trace_enable", "lnr_trace_read",
            "lnr_stage_search_window", "lnr_proposal_set", "lnr_proposal_get",
            "lnr_proposal_inputs", "lnr_proposal_forward", "lnr_proposal_train_step",
            "lnr_register_batch", "lnr_autotune_flow", "lnr_autotune_search",
            "lnr_proposal_save", "lnr_proposal_load", "lnr_merge_irradiance",
            "lnr_stage_irradiance", "lnr_meter", "lnr_set_flow_shape", "lnr_flow_shapes",
            "lnr_register_pair_noalloc", "lnr_proposal_checkpoint_save",
            "lnr_proposal_checkpoint_load", "lnr_set_search_shape")

BATCH_GRAPH, BATCH_AUTOTUNE = 1, 2

PROPOSAL_PARAMS = 30467
PROPOSAL_IN = 4   # network input channels


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context on one GPU (owns the workspace)."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        self.device = device
        rc = lib().lnr_create(C.byref(self._h), device)
        if rc:
            raise LnrError(rc, f"lnr_create(device={device}) failed")

    def check(self, rc):
        if rc:
            raise LnrError(rc, lib().lnr_last_error(self._h).decode())

    def trace(self, on: bool = True):
        """Start (or stop) per-kernel HIP-event timing; clears what was recorded."""
        self.check(lib().lnr_trace_enable(self._h, 1 if on else 0))

    def trace_read(self) -> dict:
        """{kernel name: (launches, total ms)} since trace(True); waits for the events."""
        buf = (_TraceEntry * 64)()
        n = lib().lnr_trace_read(self._h, buf, 64)
        if n < 0:
            self.check(n)
        return {buf[i].name.decode(): (buf[i].count, buf[i].ms_total) for i in range(min(n, 64))}

    def close(self):
        if self._h:
            lib().lnr_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Frame:
    """An 8-bit Y8, I420 or NV12 frame whose planes are uint8 tensors on the
    GPU (NV12: u holds the interleaved U, V plane [H/2, W] and v is None)."""
    y: torch.Tensor
    u: torch.Tensor | None = None
    v: torch.Tensor | None = None
    exposure: float = 1.0
    nv12: bool = False

    @staticmethod
    def from_numpy(y, u=None, v=None, exposure=1.0, device="cuda"):
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return Frame(t(y), t(u), t(v), float(exposure))

    @staticmethod
    def nv12_from_numpy(y, uv, exposure=1.0, device="cuda"):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return Frame(t(y), t(uv), None, float(exposure), True)

    @property
    def fmt(self):
        if self.u is None:
            return LNR_Y8
        return LNR_NV12 if self.nv12 else LNR_I420

    @property
    def width(self):
        return int(self.y.shape[1])

    @property
    def height(self):
        return int(self.y.shape[0])

    def _c(self) -> _Frame:
        f = _Frame()
        f.width, f.height, f.format = self.width, self.height, self.fmt
        planes = [self.y, self.u, self.v]
        for i, pl in enumerate(planes):
            if pl is None:
                f.plane[i] = None
                f.stride[i] = 0
            else:
                if pl.dtype != torch.uint8 or not pl.is_cuda or pl.stride(1) != 1:
                    raise ValueError("planes must be uint8 CUDA tensors with unit column stride")
                f.plane[i] = pl.data_ptr()
                f.stride[i] = pl.stride(0)
        f.exposure = self.exposure
        return f


def query_sizes(width, height, fmt=LNR_Y8, params=None):
    p = params or Params()
    s = _Sizes()
    rc = lib().lnr_query_sizes(width, height, fmt, C.byref(p), C.byref(s))
    if rc:
        raise LnrError(rc, "lnr_query_sizes")
    return s


@dataclass
class Registration:
    """Device outputs of one registration (see lnr_registration in lnr.h)."""
    corner_xy: torch.Tensor
    disp: torch.Tensor
    ssd: torch.Tensor
    flags: torch.Tensor
    counts: torch.Tensor
    H: torch.Tensor
    yeq_ref: torch.Tensor
    yeq_src: torch.Tensor
    warped0: torch.Tensor
    flow: torch.Tensor
    ntilde: torch.Tensor
    image: torch.Tensor
    yeq_warped: torch.Tensor
    levels: int = 1
    tile_off: list = field(default_factory=list)

    @staticmethod
    def alloc(width, height, fmt, params, device="cuda"):
        s = query_sizes(width, height, fmt, params)
        T, L, ch = max(s.tiles_total, 1), s.levels, s.channels
        e = lambda *shape, dt: torch.empty(*shape, dtype=dt, device=device)
        return Registration(
            corner_xy=e(T, 2, dt=torch.int32), disp=e(T, 2, dt=torch.int32),
            ssd=e(T, dt=torch.int32), flags=e(T, dt=torch.uint8),
            counts=torch.zeros(5, 4, dtype=torch.int32, device=device),
            H=e(L + 1, 9, dt=torch.float64), yeq_ref=e(height, width, dt=torch.uint8),
            yeq_src=e(height, width, dt=torch.uint8), warped0=e(height, width, dt=torch.uint8),
            flow=e(2, height, width, dt=torch.float32), ntilde=e(height, width, dt=torch.float32),
            image=e(ch, height, width, dt=torch.float32),
            yeq_warped=e(height, width, dt=torch.float32), levels=L,
            tile_off=list(s.tile_off)[:L + 1])

    def _c(self) -> _Registration:
        r = _Registration()
        for name, _ in _Registration._fields_:
            setattr(r, name, getattr(self, name).data_ptr())
        return r


def register_pair(ctx: Context, ref: Frame, src: Frame, params: Params | None = None,
                  out: Registration | None = None) -> Registration:
    """Register src to ref (paper Sec. 2.2 - 2.4); asynchronous on the current stream."""
    p = params or Params()
    out = out or Registration.alloc(ref.width, ref.height, ref.fmt, p, ref.y.device)
    rf, sf, rr = ref._c(), src._c(), out._c()
    ctx.check(lib().lnr_register_pair(ctx._h, C.byref(rf), C.byref(sf), C.byref(p),
                                      C.byref(rr), _stream()))
    return out


NOALLOC_SCRATCH_BYTES = 96 << 20


def register_pair_noalloc(ctx: Context, ref: Frame, src: Frame, params: Params | None = None,
                          out: Registration | None = None) -> Registration:
    """register_pair on the library's fixed device scratch (no allocation by
    the library; `out` is the caller's); calls on one GPU must not overlap."""
    p = params or Params()
    out = out or Registration.alloc(ref.width, ref.height, ref.fmt, p, ref.y.device)
    rf, sf, rr = ref._c(), src._c(), out._c()
    ctx.check(lib().lnr_register_pair_noalloc(ctx._h, C.byref(rf), C.byref(sf), C.byref(p),
                                              C.byref(rr), _stream()))
    return out


def register_stack(ctx: Context, frames, params: Params | None = None):
    """Register every frame to the shortest exposure; returns (registrations, ref_index)."""
    p = params or Params()
    n = len(frames)
    f0 = frames[0]
    regs = [Registration.alloc(f0.width, f0.height, f0.fmt, p, f0.y.device) for _ in range(n - 1)]
    FA = (_Frame * n)(*[f._c() for f in frames])
    RA = (_Registration * max(n - 1, 1))(*[r._c() for r in regs])
    ref_index = C.c_int32(-1)
    ctx.check(lib().lnr_register_stack(ctx._h, FA, n, C.byref(p), RA, C.byref(ref_index),
                                       _stream()))
    return regs, ref_index.value


def merge(ctx: Context, frames, ref_index: int, regs, params: Params | None = None,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """Error-tolerant exposure fusion (paper Sec. 2.5); returns [ch][H][W] float32."""
    p = params or Params()
    n = len(frames)
    f0 = frames[ref_index]
    ch = 1 if f0.fmt == LNR_Y8 else 3
    out = out if out is not None else torch.empty(ch, f0.height, f0.width, dtype=torch.float32,
                                                  device=f0.y.device)
    FA = (_Frame * n)(*[f._c() for f in frames])
    RA = (_Registration * max(n - 1, 1))(*[r._c() for r in regs])
    ctx.check(lib().lnr_merge(ctx._h, FA, n, ref_index, RA, C.byref(p), _ptr(out), _stream()))
    return out


def merge_irradiance(ctx: Context, frames, ref_index: int, regs, params: Params | None = None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """HDR irradiance map of the registered frames (reference units); see
    lnr_merge_irradiance."""
    p = params or Params()
    n = len(frames)
    f0 = frames[ref_index]
    ch = 1 if f0.fmt == LNR_Y8 else 3
    out = out if out is not None else torch.empty(ch, f0.height, f0.width, dtype=torch.float32,
                                                  device=f0.y.device)
    FA = (_Frame * n)(*[f._c() for f in frames])
    RA = (_Registration * max(n - 1, 1))(*[r._c() for r in regs])
    ctx.check(lib().lnr_merge_irradiance(ctx._h, FA, n, ref_index, RA, C.byref(p), _ptr(out),
                                         _stream()))
    return out


# ----------------------------------------------------------------- stage entry points

def stage_equalize(ctx, img: torch.Tensor):
    h, w = img.shape
    lut = torch.empty(256, dtype=torch.uint8, device=img.device)
    out = torch.empty(h, w, dtype=torch.uint8, device=img.device)
    ctx.check(lib().lnr_stage_equalize(ctx._h, _ptr(img), w, h, img.stride(0), _ptr(lut),
                                       _ptr(out), _stream()))
    return lut, out


def meter(ctx, y: torch.Tensor, dark=16, frac3=0.05, frac4=0.20):
    """(stops, under-exposed count) for the ETTR first frame's luma y
    (uint8 [h, w] on the GPU, unit column stride); see lnr_meter."""
    h, w = y.shape
    out = torch.zeros(2, dtype=torch.int32, device=y.device)
    ctx.check(lib().lnr_meter(ctx._h, _ptr(y), w, h, y.stride(0), int(dark), float(frac3),
                              float(frac4), _ptr(out), _stream()))
    o = out.cpu()
    return int(o[0]), int(o[1])


def stage_warp_q8(ctx, src: torch.Tensor, H: torch.Tensor):
    h, w = src.shape
    out = torch.empty_like(src)
    Hd = H.to(device=src.device, dtype=torch.float64).contiguous()
    ctx.check(lib().lnr_stage_warp_q8(ctx._h, _ptr(src), w, h, _ptr(Hd), _ptr(out), _stream()))
    return out


def stage_search(ctx, ref: torch.Tensor, warped: torch.Tensor, R: int, params=None):
    p = params or Params()
    h, w = ref.shape
    nt = max((w // p.tile) * (h // p.tile), 1)
    dev = ref.device
    cxy = torch.empty(nt, 2, dtype=torch.int32, device=dev)
    disp = torch.empty(nt, 2, dtype=torch.int32, device=dev)
    ssd = torch.empty(nt, dtype=torch.int32, device=dev)
    flags = torch.empty(nt, dtype=torch.uint8, device=dev)
    ctx.check(lib().lnr_stage_search(ctx._h, _ptr(ref), _ptr(warped), w, h, R, C.byref(p),
                                     _ptr(cxy), _ptr(disp), _ptr(ssd), _ptr(flags), _stream()))
    return cxy, disp, ssd, flags


def stage_weed_fit(ctx, corner_xy, disp, flags, w, h, level, H_prev, params=None):
    p = params or Params()
    dev = corner_xy.device
    flags = flags.clone()
    Hp = H_prev.to(device=dev, dtype=torch.float64).contiguous()
    Ho = torch.empty(9, dtype=torch.float64, device=dev)
    counts = torch.empty(4, dtype=torch.int32, device=dev)
    ctx.check(lib().lnr_stage_weed_fit(ctx._h, _ptr(corner_xy), _ptr(disp), _ptr(flags),
                                       flags.numel(), w, h, level, C.byref(p), _ptr(Hp), _ptr(Ho),
                                       _ptr(counts), _stream()))
    return flags, Ho, counts


def stage_flow(ctx, corner_xy, disp, flags, guide: torch.Tensor, params=None):
    p = params or Params()
    h, w = guide.shape
    flow = torch.empty(2, h, w, dtype=torch.float32, device=guide.device)
    ntilde = torch.empty(h, w, dtype=torch.float32, device=guide.device)
    nt = (w // p.tile) * (h // p.tile)
    ctx.check(lib().lnr_stage_flow(ctx._h, _ptr(corner_xy), _ptr(disp), _ptr(flags), nt,
                                   _ptr(guide), w, h, C.byref(p), _ptr(flow), _ptr(ntilde),
                                   _stream()))
    return flow, ntilde


def stage_backward_warp(ctx, src: Frame, yeq: torch.Tensor, H: torch.Tensor,
                        flow: torch.Tensor):
    ch = 1 if src.fmt == LNR_Y8 else 3
    dev = src.y.device
    img = torch.empty(ch, src.height, src.width, dtype=torch.float32, device=dev)
    yw = torch.empty(src.height, src.width, dtype=torch.float32, device=dev)
    Hd = H.to(device=dev, dtype=torch.float64).contiguous()
    sf = src._c()
    ctx.check(lib().lnr_stage_backward_warp(ctx._h, C.byref(sf), _ptr(yeq), _ptr(Hd),
                                            _ptr(flow.contiguous()), _ptr(img), _ptr(yw),
                                            _stream()))
    return img, yw


def stage_frame_rgb(ctx, f: Frame, yeq: torch.Tensor = None):
    """The merge's conversion of an unwarped frame: (image [ch][h][w],
    yeq / 255 or None)."""
    ch = 1 if f.fmt == LNR_Y8 else 3
    dev = f.y.device
    img = torch.empty(ch, f.height, f.width, dtype=torch.float32, device=dev)
    yo = None if yeq is None else torch.empty(f.height, f.width, dtype=torch.float32, device=dev)
    ff = f._c()
    ctx.check(lib().lnr_stage_frame_rgb(ctx._h, C.byref(ff), _ptr(yeq), _ptr(img), _ptr(yo),
                                        _stream()))
    return img, yo


def stage_merge(ctx, imgs, yeqs, ref_index, params=None):
    p = params or Params()
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = torch.empty(ch, h, w, dtype=torch.float32, device=imgs[0].device)
    IA = (C.c_void_p * n)(*[i.data_ptr() for i in imgs])
    YA = (C.c_void_p * n)(*[y.data_ptr() for y in yeqs])
    ctx.check(lib().lnr_stage_merge(ctx._h, n, ch, w, h, IA, YA, ref_index, C.byref(p),
                                    _ptr(out), _stream()))
    return out


def stage_irradiance(ctx, imgs, yeqs, exposures, ref_index, params=None):
    p = params or Params()
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = torch.empty(ch, h, w, dtype=torch.float32, device=imgs[0].device)
    IA = (C.c_void_p * n)(*[i.data_ptr() for i in imgs])
    YA = (C.c_void_p * n)(*[y.data_ptr() for y in yeqs])
    EA = (C.c_float * n)(*[float(e) for e in exposures])
    ctx.check(lib().lnr_stage_irradiance(ctx._h, n, ch, w, h, IA, YA, EA, ref_index, C.byref(p),
                                         _ptr(out), _stream()))
    return out


# --------------------------------------------------------------------------- learned proposal
# (an extension beyond the paper: a CNN proposes each level-0 tile's
# displacement; the library's kernels run inference and training)

def stage_search_window(ctx, ref: torch.Tensor, warped: torch.Tensor, R: int,
                        centre: torch.Tensor, params=None):
    """Search of stage_search restricted to centre[t] + [-R, R]^2 per tile."""
    p = params or Params()
    h, w = ref.shape
    nt = max((w // p.tile) * (h // p.tile), 1)
    dev = ref.device
    centre = centre.to(device=dev, dtype=torch.int32).contiguous()
    cxy = torch.empty(nt, 2, dtype=torch.int32, device=dev)
    disp = torch.empty(nt, 2, dtype=torch.int32, device=dev)
    ssd = torch.empty(nt, dtype=torch.int32, device=dev)
    flags = torch.empty(nt, dtype=torch.uint8, device=dev)
    ctx.check(lib().lnr_stage_search_window(ctx._h, _ptr(ref), _ptr(warped), w, h, R,
                                            _ptr(centre), C.byref(p), _ptr(cxy), _ptr(disp),
                                            _ptr(ssd), _ptr(flags), _stream()))
    return cxy, disp, ssd, flags


def proposal_set(ctx, params: torch.Tensor):
    """Load network parameters (float32 [PROPOSAL_PARAMS], device) and reset AdamW."""
    params = params.to(device="cuda", dtype=torch.float32).contiguous()
    assert params.numel() == PROPOSAL_PARAMS
    ctx.check(lib().lnr_proposal_set(ctx._h, _ptr(params), _stream()))


def proposal_get(ctx) -> torch.Tensor:
    out = torch.empty(PROPOSAL_PARAMS, dtype=torch.float32, device="cuda")
    ctx.check(lib().lnr_proposal_get(ctx._h, _ptr(out), _stream()))
    return out


def proposal_save(ctx, path: str):
    """Write the context's network to a file (the library's network file format)."""
    ctx.check(lib().lnr_proposal_save(ctx._h, os.fsencode(path), _stream()))


def proposal_load(ctx, path: str):
    """Load a network file written by proposal_save and reset AdamW."""
    ctx.check(lib().lnr_proposal_load(ctx._h, os.fsencode(path), _stream()))


def proposal_checkpoint_save(ctx, path: str, counter: int):
    """Write parameters, AdamW moments and step count, and `counter` (the
    caller's data-order position) to a checkpoint file."""
    ctx.check(lib().lnr_proposal_checkpoint_save(ctx._h, os.fsencode(path), int(counter),
                                                 _stream()))


def proposal_checkpoint_load(ctx, path: str) -> int:
    """Restore a checkpoint written by proposal_checkpoint_save; returns its counter."""
    c = C.c_uint64(0)
    ctx.check(lib().lnr_proposal_checkpoint_load(ctx._h, os.fsencode(path), C.byref(c),
                                                 _stream()))
    return int(c.value)


def proposal_inputs(ctx, ref: torch.Tensor, warped: torch.Tensor) -> torch.Tensor:
    """Network inputs of every full 32x32 tile: int16 view of bf16 [n, 4, 16, 16]."""
    h, w = ref.shape
    n = (w // 32) * (h // 32)
    x = torch.empty(max(n, 1), PROPOSAL_IN, 16, 16, dtype=torch.int16, device=ref.device)
    ctx.check(lib().lnr_proposal_inputs(ctx._h, _ptr(ref.contiguous()), _ptr(warped.contiguous()),
                                        w, h, _ptr(x), _stream()))
    return x[:n]


def proposal_forward(ctx, x: torch.Tensor) -> torch.Tensor:
    """[n, 3] outputs for bf16 inputs x (int16 bit patterns or bfloat16)."""
    x = x.contiguous()
    n = x.shape[0]
    out = torch.empty(max(n, 1), 3, dtype=torch.float32, device=x.device)
    ctx.check(lib().lnr_proposal_forward(ctx._h, _ptr(x), n, _ptr(out), _stream()))
    return out[:n]


def proposal_train_step(ctx, x: torch.Tensor, labels: torch.Tensor, lr: float, wd: float = 0.0,
                        want_loss: bool = True, want_grad: bool = False):
    """One AdamW step on a batch; returns (per-sample loss or None, gradient or None)."""
    x = x.contiguous()
    n = x.shape[0]
    labels = labels.to(device=x.device, dtype=torch.int32).contiguous()
    loss = torch.empty(n, dtype=torch.float32, device=x.device) if want_loss else None
    grad = torch.empty(PROPOSAL_PARAMS, dtype=torch.float32, device=x.device) if want_grad else None
    ctx.check(lib().lnr_proposal_train_step(
        ctx._h, _ptr(x), _ptr(labels), n, float(lr), float(wd),
        None if loss is None else _ptr(loss), None if grad is None else _ptr(grad), _stream()))
    return loss, grad


# --------------------------------------------------------------------------- batches

def register_batch(ctx: Context, refs, srcs, params: Params | None = None, outs=None,
                   graph: bool = False, autotune: bool = False):
    """Register len(refs) pairs of any sizes in one call (concurrent streams;
    optionally one cached HIP graph). Returns the list of Registrations."""
    p = params or Params()
    n = len(refs)
    assert n == len(srcs) and n > 0
    if outs is None:
        outs = [Registration.alloc(r.width, r.height, r.fmt, p) for r in refs]
    RA = (_Frame * n)(*[r._c() for r in refs])
    SA = (_Frame * n)(*[s._c() for s in srcs])
    OA = (_Registration * n)(*[o._c() for o in outs])
    flags = (BATCH_GRAPH if graph else 0) | (BATCH_AUTOTUNE if autotune else 0)
    ctx.check(lib().lnr_register_batch(ctx._h, RA, SA, n, C.byref(p), OA, flags, _stream()))
    return outs


def autotune_search(ctx: Context, w: int, h: int, params: Params | None = None):
    """Pick the fastest search workgroup shape (patch-row split) for each
    pyramid level of a w x h pair; returns the split per level."""
    p = params or Params()
    out = (C.c_int32 * 5)()
    ctx.check(lib().lnr_autotune_search(ctx._h, w, h, C.byref(p), out, _stream()))
    return tuple(v for v in out if v)


def flow_shapes(w: int, h: int):
    """The propagation kernel shapes that cover w x h (5-tuples)."""
    n = lib().lnr_flow_shapes(w, h, None, 0)
    buf = (C.c_int32 * (5 * max(n, 1)))()
    lib().lnr_flow_shapes(w, h, buf, n)
    return [tuple(buf[5 * i:5 * i + 5]) for i in range(n)]


SEARCH_KX12 = 16
SEARCH_MFMA = 32


def set_search_shape(ctx: Context, level_w: int, level_h: int, radius: int, shape: int):
    """Pin the search shape (split 1..7, plus SEARCH_KX12 for 12 candidates per
    lane or SEARCH_MFMA for matrix-core cross terms) for levels of that size
    and radius."""
    ctx.check(lib().lnr_set_search_shape(ctx._h, level_w, level_h, radius, shape))


def set_flow_shape(ctx: Context, w: int, h: int, shape):
    arr = (C.c_int32 * 5)(*[int(v) for v in shape])
    ctx.check(lib().lnr_set_flow_shape(ctx._h, w, h, arr))


def autotune_flow(ctx: Context, w: int, h: int, params: Params | None = None):
    """Pick the fastest domain-transform kernel shape for w x h; returns it
    (rows per thread, row block, rows per column segment, columns per block,
    segments per column)."""
    p = params or Params()
    out = (C.c_int32 * 5)()
    ctx.check(lib().lnr_autotune_flow(ctx._h, w, h, C.byref(p), out, _stream()))
    return tuple(out)
