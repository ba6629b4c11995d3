"""CPU oracle for locally non-rigid HDR registration -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product library (paper_1504_01441_amd) never does,
and this package imports nothing from it: the C sources here share no code
with the GPU path.

`build()` compiles lnr_oracle.c (the paper's method) and proposal_oracle.c
(the learned displacement proposal, an extension) with gcc into
liblnr_oracle.so next to them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lnr_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "proposal_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liblnr_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


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
    ]


class _Registration(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("tile_off", C.c_int32 * 6),
        ("corner_x", C.c_void_p), ("corner_y", C.c_void_p), ("dx", C.c_void_p),
        ("dy", C.c_void_p), ("ssd", C.c_void_p), ("flags", C.c_void_p),
        ("n_valid", C.c_void_p), ("n_inliers", C.c_void_p), ("best_iter", C.c_void_p),
        ("H", C.c_void_p),
        ("yeq_ref", C.c_void_p), ("yeq_src", C.c_void_p), ("warped0", C.c_void_p),
        ("flow_u", C.c_void_p), ("flow_v", C.c_void_p), ("ntilde", C.c_void_p),
        ("rgb", C.c_void_p), ("yeq_warped", C.c_void_p),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
                os.path.getmtime(f) for f in _SRCS + [os.path.join(_HERE, "lnr_oracle.h")]):
            build(force=True)
        _lib = C.CDLL(_LIB_PATH)
        _lib.lo_default_params.argtypes = [C.POINTER(Params)]
        _lib.lo_bf16.argtypes = [C.c_double]
        _lib.lo_bf16.restype = C.c_double
        _lib.lo_cnn_loss_grad.restype = C.c_double
        _lib.lo_adamw.argtypes = [C.c_void_p] * 4 + [C.c_int, C.c_int] + [C.c_double] * 5
        _lib.lo_num_levels.argtypes = [C.c_int, C.c_int, C.POINTER(Params)]
        _lib.lo_num_levels.restype = C.c_int
        _lib.lo_weed.restype = C.c_int
        _lib.lo_fit_level.restype = C.c_int
        _lib.lo_fit_level_absolute.restype = C.c_int
        _lib.lo_fit4.restype = C.c_int
        _lib.lo_weed_delta.restype = C.c_int
        _lib.lo_hypothesis_inliers.restype = C.c_int
        _lib.lo_register_pair.restype = C.c_int
        _lib.lo_merge.restype = C.c_int
        _lib.lo_irradiance.restype = C.c_int
        _lib.lo_fusion_weight_sum.restype = C.c_int
        _lib.lo_meter.restype = C.c_int
        _lib.lo_meter.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_float,
                                  C.c_float, C.c_void_p]
        _lib.lo_hat_weight.restype = C.c_double
        _lib.lo_hat_weight.argtypes = [C.c_double]
        _lib.lo_num_blend_levels.restype = C.c_int
    return _lib


def params(**overrides) -> Params:
    p = Params()
    lib().lo_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------- stages

def num_levels(w, h, p=None):
    p = p or params()
    return lib().lo_num_levels(w, h, C.byref(p))


def histogram(img):
    img = _c(img, np.uint8)
    hist = np.zeros(256, np.uint32)
    lib().lo_histogram(_p(img), img.shape[1], img.shape[0], img.shape[1], _p(hist))
    return hist


def equalize_lut(hist):
    hist = _c(hist, np.uint32)
    lut = np.zeros(256, np.uint8)
    lib().lo_equalize_lut(_p(hist), _p(lut))
    return lut


def equalize(img):
    img = _c(img, np.uint8)
    lut = equalize_lut(histogram(img))
    out = np.empty_like(img)
    lib().lo_apply_lut(_p(img), img.shape[1], img.shape[0], img.shape[1], _p(lut), _p(out))
    return out


def downsample(img):
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.zeros((h // 2, w // 2), np.uint8)
    lib().lo_downsample(_p(img), w, h, _p(out))
    return out


def corners(img, p=None):
    p = p or params()
    img = _c(img, np.uint8)
    h, w = img.shape
    nt = (w // p.tile) * (h // p.tile)
    cx = np.zeros(max(nt, 1), np.int32)
    cy = np.zeros(max(nt, 1), np.int32)
    has = np.zeros(max(nt, 1), np.uint8)
    lib().lo_corners(_p(img), w, h, C.byref(p), _p(cx), _p(cy), _p(has))
    return cx[:nt], cy[:nt], has[:nt]


def pixel_homography(H, w, h):
    H = _c(H, np.float64).reshape(9)
    Hp = np.zeros(9, np.float64)
    lib().lo_pixel_homography(_p(H), w, h, _p(Hp))
    return Hp.reshape(3, 3)


def warp_q8(src, Hp):
    src = _c(src, np.uint8)
    Hp = _c(Hp, np.float64).reshape(9)
    out = np.zeros_like(src)
    lib().lo_warp_q8(_p(src), src.shape[1], src.shape[0], _p(Hp), _p(out))
    return out


def search(ref, wimg, R, cx, cy, has, p=None):
    p = p or params()
    ref = _c(ref, np.uint8)
    wimg = _c(wimg, np.uint8)
    h, w = ref.shape
    nt = (w // p.tile) * (h // p.tile)
    cx, cy, has = _c(cx, np.int32), _c(cy, np.int32), _c(has, np.uint8)
    dx = np.zeros(max(nt, 1), np.int32)
    dy = np.zeros(max(nt, 1), np.int32)
    ssd = np.zeros(max(nt, 1), np.uint32)
    valid = np.zeros(max(nt, 1), np.uint8)
    lib().lo_search(_p(ref), _p(wimg), w, h, C.byref(p), R, _p(cx), _p(cy), _p(has),
                    _p(dx), _p(dy), _p(ssd), _p(valid))
    return dx[:nt], dy[:nt], ssd[:nt], valid[:nt]


def search_unwarped(ref, src, R, Hp, cx, cy, has, p=None):
    """The search of Eq. 3 as printed: around round(Hp x) in the unwarped
    source; returns absolute displacements (dx, dy), ssd, valid."""
    p = p or params()
    ref = _c(ref, np.uint8)
    src = _c(src, np.uint8)
    h, w = ref.shape
    nt = (w // p.tile) * (h // p.tile)
    Hp = _c(Hp, np.float64).reshape(9)
    cx, cy, has = _c(cx, np.int32), _c(cy, np.int32), _c(has, np.uint8)
    dx = np.zeros(max(nt, 1), np.int32)
    dy = np.zeros(max(nt, 1), np.int32)
    ssd = np.zeros(max(nt, 1), np.uint32)
    valid = np.zeros(max(nt, 1), np.uint8)
    lib().lo_search_unwarped(_p(ref), _p(src), w, h, C.byref(p), R, _p(Hp), _p(cx), _p(cy),
                             _p(has), _p(dx), _p(dy), _p(ssd), _p(valid))
    return dx[:nt], dy[:nt], ssd[:nt], valid[:nt]


def weed(cx, cy, dx, dy, valid, w, h, level, p=None, it0=0, it1=None, inM=None):
    """Returns (inM, N, best_count, best_iter)."""
    p = p or params()
    nt = len(cx)
    it1 = p.weed_iters if it1 is None else it1
    inM = np.zeros(max(nt, 1), np.uint8) if inM is None else _c(inM, np.uint8).copy()
    args = [_c(a, np.int32) for a in (cx, cy, dx, dy)]
    valid = _c(valid, np.uint8)
    bc, bi = C.c_int32(-1), C.c_int32(-1)
    n = lib().lo_weed(nt, *[_p(a) for a in args], _p(valid), w, h, level, C.byref(p),
                      it0, it1, _p(inM), C.byref(bc), C.byref(bi))
    return inM[:nt], n, bc.value, bi.value


def weed_delta(n, p=None):
    p = p or params()
    return lib().lo_weed_delta(n, C.byref(p))


def hypothesis_inliers(cx, cy, dx, dy, valid, w, h, level, it, p=None):
    p = p or params()
    nt = len(cx)
    sel = np.zeros(max(nt, 1), np.uint8)
    args = [_c(a, np.int32) for a in (cx, cy, dx, dy)]
    valid = _c(valid, np.uint8)
    cnt = lib().lo_hypothesis_inliers(nt, *[_p(a) for a in args], _p(valid), w, h, level,
                                      C.byref(p), it, _p(sel))
    return sel[:nt], cnt


def fit4(src_pts, dst_pts):
    s = _c(src_pts, np.float64)
    d = _c(dst_pts, np.float64)
    sx, sy = _c(s[:, 0], np.float64), _c(s[:, 1], np.float64)
    tx, ty = _c(d[:, 0], np.float64), _c(d[:, 1], np.float64)
    g = np.zeros(9, np.float64)
    ok = lib().lo_fit4(_p(sx), _p(sy), _p(tx), _p(ty), _p(g))
    return (g.reshape(3, 3) if ok else None)


def fit_level(cx, cy, dx, dy, sel, w, h, Hprev):
    args = [_c(a, np.int32) for a in (cx, cy, dx, dy)]
    inM = _c(sel, np.uint8)
    Hprev = _c(Hprev, np.float64).reshape(9)
    Hout = np.zeros(9, np.float64)
    m = lib().lo_fit_level(len(cx), *[_p(a) for a in args], _p(inM), w, h, _p(Hprev), _p(Hout))
    return Hout.reshape(3, 3), m


def fit_level_absolute(cx, cy, dx, dy, sel, w, h, Hprev):
    """Level homography fitted to absolute matches (Hprev kept on failure)."""
    args = [_c(a, np.int32) for a in (cx, cy, dx, dy)]
    inM = _c(sel, np.uint8)
    Hprev = _c(Hprev, np.float64).reshape(9)
    Hout = np.zeros(9, np.float64)
    m = lib().lo_fit_level_absolute(len(cx), *[_p(a) for a in args], _p(inM), w, h, _p(Hprev),
                                    _p(Hout))
    return Hout.reshape(3, 3), m


def sparse_to_dense(cx, cy, dx, dy, inM, guide, p=None):
    p = p or params()
    guide = _c(guide, np.uint8)
    h, w = guide.shape
    args = [_c(a, np.int32) for a in (cx, cy, dx, dy)]
    inM = _c(inM, np.uint8)
    fu = np.zeros((h, w), np.float64)
    fv = np.zeros((h, w), np.float64)
    nt = np.zeros((h, w), np.float64)
    lib().lo_sparse_to_dense(len(cx), *[_p(a) for a in args], _p(inM), _p(guide), w, h,
                             C.byref(p), _p(fu), _p(fv), _p(nt))
    return fu, fv, nt


def backward_warp(y, u, v, yeq, Hp, fu, fv):
    y, yeq = _c(y, np.uint8), _c(yeq, np.uint8)
    h, w = y.shape
    ch = 1 if u is None else 3
    uu = None if u is None else _c(u, np.uint8)
    vv = None if v is None else _c(v, np.uint8)
    Hp = _c(Hp, np.float64).reshape(9)
    fu, fv = _c(fu, np.float64), _c(fv, np.float64)
    rgb = np.zeros((ch, h, w), np.float64)
    yw = np.zeros((h, w), np.float64)
    lib().lo_backward_warp(_p(y), None if uu is None else _p(uu), None if vv is None else _p(vv),
                           _p(yeq), w, h, _p(Hp), _p(fu), _p(fv), _p(rgb), _p(yw))
    return rgb, yw


def frame_to_rgb(y, u=None, v=None):
    y = _c(y, np.uint8)
    h, w = y.shape
    ch = 1 if u is None else 3
    rgb = np.zeros((ch, h, w), np.float64)
    if u is None:
        lib().lo_frame_to_rgb(_p(y), None, None, w, h, _p(rgb))
    else:
        uu, vv = _c(u, np.uint8), _c(v, np.uint8)
        lib().lo_frame_to_rgb(_p(y), _p(uu), _p(vv), w, h, _p(rgb))
    return rgb


def ssim(a, b, p=None):
    p = p or params()
    a, b = _c(a, np.float64), _c(b, np.float64)
    out = np.zeros_like(a)
    lib().lo_ssim(_p(a), _p(b), a.shape[1], a.shape[0], C.byref(p), _p(out))
    return out


def fusion_weights(imgs, ssims, p=None):
    p = p or params()
    imgs = [_c(i, np.float64) for i in imgs]
    n = len(imgs)
    ch, h, w = imgs[0].shape
    ss = [None if s is None else _c(s, np.float64) for s in ssims]
    outs = [np.zeros((h, w), np.float64) for _ in range(n)]
    IA = (C.c_void_p * n)(*[_p(i) for i in imgs])
    SA = (C.c_void_p * n)(*[None if s is None else _p(s) for s in ss])
    OA = (C.c_void_p * n)(*[_p(o) for o in outs])
    lib().lo_fusion_weights(n, ch, w, h, IA, SA, C.byref(p), OA)
    return outs


def num_blend_levels(w, h):
    return lib().lo_num_blend_levels(w, h)


def reduce(img):
    """The blend's REDUCE step on one 2-D plane."""
    img = _c(img, np.float64)
    h, w = img.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2), np.float64)
    lib().lo_reduce(_p(img), w, h, _p(out))
    return out


def expand(coarse, w, h):
    """The blend's EXPAND step of a coarse 2-D plane to w x h."""
    coarse = _c(coarse, np.float64)
    ch_, cw = coarse.shape
    out = np.zeros((h, w), np.float64)
    lib().lo_expand(_p(coarse), cw, ch_, w, h, _p(out))
    return out


def pick_reference(exposures, ys):
    """Index of the stack's reference frame from its exposures and luma planes."""
    ys = [_c(y, np.uint8) for y in ys]
    n = len(ys)
    h, w = ys[0].shape
    ex = _c(exposures, np.float32)
    YA = (C.c_void_p * n)(*[_p(y) for y in ys])
    return lib().lo_pick_reference(n, _p(ex), YA, w, h, w)


def blend(imgs, weights):
    imgs = [_c(i, np.float64) for i in imgs]
    wts = [_c(x, np.float64) for x in weights]
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = np.zeros((ch, h, w), np.float64)
    IA = (C.c_void_p * n)(*[_p(i) for i in imgs])
    WA = (C.c_void_p * n)(*[_p(x) for x in wts])
    lib().lo_blend(n, ch, w, h, IA, WA, _p(out))
    return out


def merge(imgs, yeqs, ref_index, p=None):
    """imgs: list of [ch][H][W] float64 in [0, 1]; yeqs: list of [H][W] Y_eq/255."""
    p = p or params()
    imgs = [_c(i, np.float64) for i in imgs]
    yeqs = [_c(y, np.float64) for y in yeqs]
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = np.zeros((ch, h, w), np.float64)
    IA = (C.c_void_p * n)(*[_p(i) for i in imgs])
    YA = (C.c_void_p * n)(*[_p(y) for y in yeqs])
    rc = lib().lo_merge(n, ch, w, h, IA, YA, ref_index, C.byref(p), _p(out))
    if rc:
        raise ValueError("lo_merge failed")
    return out


def fusion_weight_sum(imgs, yeqs, ref_index, p=None):
    """[H][W] sum of the raw fusion weights before normalisation."""
    p = p or params()
    imgs = [_c(i, np.float64) for i in imgs]
    yeqs = [_c(y, np.float64) for y in yeqs]
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = np.zeros((h, w), np.float64)
    IA = (C.c_void_p * n)(*[_p(i) for i in imgs])
    YA = (C.c_void_p * n)(*[_p(y) for y in yeqs])
    if lib().lo_fusion_weight_sum(n, ch, w, h, IA, YA, ref_index, C.byref(p), _p(out)):
        raise ValueError("lo_fusion_weight_sum failed")
    return out


def irradiance(imgs, yeqs, exposures, ref_index, p=None):
    """HDR irradiance map (reference units) of frames imgs ([ch][H][W] in
    [0, 1]) with relative exposures, deghosted by SSIM of yeqs; see
    lo_irradiance."""
    p = p or params()
    imgs = [_c(i, np.float64) for i in imgs]
    yeqs = [_c(y, np.float64) for y in yeqs]
    ex = _c(np.asarray(exposures, np.float64), np.float64)
    n = len(imgs)
    ch, h, w = imgs[0].shape
    out = np.zeros((ch, h, w), np.float64)
    IA = (C.c_void_p * n)(*[_p(i) for i in imgs])
    YA = (C.c_void_p * n)(*[_p(y) for y in yeqs])
    rc = lib().lo_irradiance(n, ch, w, h, IA, YA, _p(ex), ref_index, C.byref(p), _p(out))
    if rc:
        raise ValueError("lo_irradiance failed")
    return out


def meter(y, dark=16, frac3=0.05, frac4=0.20):
    """(stops, under-exposed count) for the ETTR first frame's 8-bit luma y."""
    y = _c(y, np.uint8)
    h, w = y.shape
    n = C.c_longlong(0)
    stops = lib().lo_meter(_p(y), w, h, w, int(dark), float(frac3), float(frac4), C.byref(n))
    return stops, n.value


def hat_weight(v):
    return lib().lo_hat_weight(float(v))


# --------------------------------------------------------------------------- whole pair

def register_pair(ref, src, p=None, H_init=None):
    """ref, src: synth.Frame-like objects (y, u, v). Returns a dict of arrays."""
    p = p or params()
    ry, sy = _c(ref.y, np.uint8), _c(src.y, np.uint8)
    h, w = ry.shape
    L = num_levels(w, h, p)
    lw, lh = [w], [h]
    for _ in range(1, L):
        lw.append(lw[-1] // 2)
        lh.append(lh[-1] // 2)
    T = sum((a // p.tile) * (b // p.tile) for a, b in zip(lw, lh))
    T1 = max(T, 1)
    ch = 1 if src.u is None else 3
    o = dict(
        corner_x=np.zeros(T1, np.int32), corner_y=np.zeros(T1, np.int32),
        dx=np.zeros(T1, np.int32), dy=np.zeros(T1, np.int32), ssd=np.zeros(T1, np.uint32),
        flags=np.zeros(T1, np.uint8), n_valid=np.zeros(6, np.int32),
        n_inliers=np.zeros(6, np.int32), best_iter=np.zeros(6, np.int32), H=np.zeros((L + 1, 9), np.float64),
        yeq_ref=np.zeros((h, w), np.uint8), yeq_src=np.zeros((h, w), np.uint8),
        warped0=np.zeros((h, w), np.uint8), flow_u=np.zeros((h, w), np.float64),
        flow_v=np.zeros((h, w), np.float64), ntilde=np.zeros((h, w), np.float64),
        rgb=np.zeros((ch, h, w), np.float64), yeq_warped=np.zeros((h, w), np.float64),
    )
    r = _Registration()
    for k, v in o.items():
        setattr(r, k, v.ctypes.data)
    hi = None
    if H_init is not None:
        hi = _c(H_init, np.float64).reshape(9)
    if src.u is None:
        up = vp = None
    else:
        su, sv = _c(src.u, np.uint8), _c(src.v, np.uint8)
        up, vp = _p(su), _p(sv)
    rc = lib().lo_register_pair(_p(ry), _p(sy), up, vp, w, h, C.byref(p),
                                None if hi is None else _p(hi), C.byref(r))
    if rc:
        raise ValueError("lo_register_pair failed")
    o["levels"] = r.levels
    o["tile_off"] = np.array(list(r.tile_off)[:L + 1], np.int32)
    for k in ("corner_x", "corner_y", "dx", "dy", "ssd", "flags"):
        o[k] = o[k][:T]
    o["H"] = o["H"].reshape(L + 1, 3, 3)
    o["level_sizes"] = list(zip(lw, lh))
    return o


# --------------------------------------------------------------------------- learned proposal
# (an extension beyond the paper: a CNN proposes each level-0 tile's
# displacement so that the Sec. 2.2 search scans a small window)

CNN_PARAMS = 30467
CNN_IN = 4       # input channels: tile pair (1/2 resolution), window pair (1/4)


def bf16(v):
    """bfloat16 round-to-nearest-even of each value (as a float32 -> bf16 cast)."""
    a = np.asarray(v, dtype=np.float64)
    return np.vectorize(lambda t: lib().lo_bf16(float(t)), otypes=[np.float64])(a)


def cnn_tile_inputs(ref, warped, tiles, tile=32):
    """[n, 4, 16, 16] network inputs of the given level-0 tile indices."""
    ref = _c(ref, np.uint8)
    warped = _c(warped, np.uint8)
    h, w = ref.shape
    ntx = w // tile
    out = np.zeros((len(tiles), CNN_IN, 16, 16), np.float64)
    for k, t in enumerate(tiles):
        tx, ty = int(t) % ntx, int(t) // ntx
        lib().lo_cnn_tile_input(_p(ref), _p(warped), w, h, tx * tile, ty * tile,
                                _p(out[k]))
    return out


def cnn_forward(params, x, rnd=True):
    """[n, 3] network outputs (o0, o1, o2): prediction (8 o0, 8 o1), logit o2."""
    params = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, CNN_IN * 256)
    out = np.zeros((x.shape[0], 3), np.float64)
    lib().lo_cnn_forward(_p(params), _p(x), x.shape[0], int(rnd), _p(out))
    return out


def cnn_loss_grad(params, x, labels, rnd=True):
    """(mean loss, gradient over the flat parameter vector)."""
    params = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, CNN_IN * 256)
    lab = _c(labels, np.int32).reshape(-1, 2)
    g = np.zeros(CNN_PARAMS, np.float64)
    loss = lib().lo_cnn_loss_grad(_p(params), _p(x), _p(lab), x.shape[0], int(rnd), _p(g))
    return loss, g


def adamw(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step in place on float64 arrays w, m, v."""
    lib().lo_adamw(_p(w), _p(m), _p(v), _p(_c(g, np.float64)), len(w), int(t), float(lr),
                   float(b1), float(b2), float(eps), float(wd))


def search_window(ref, wimg, R, centre_x, centre_y, cx, cy, has, p=None):
    """Sec. 2.2 search restricted to centre + [-R, R]^2 per tile."""
    p = p or params()
    ref = _c(ref, np.uint8)
    wimg = _c(wimg, np.uint8)
    h, w = ref.shape
    nt = len(cx)
    dx = np.zeros(nt, np.int32)
    dy = np.zeros(nt, np.int32)
    ssd = np.zeros(nt, np.uint32)
    valid = np.zeros(nt, np.uint8)
    args = [_c(a, np.int32) for a in (centre_x, centre_y, cx, cy)]
    lib().lo_search_window(_p(ref), _p(wimg), w, h, C.byref(p), R, *[_p(a) for a in args],
                           _p(_c(has, np.uint8)), _p(dx), _p(dy), _p(ssd), _p(valid))
    return dx, dy, ssd, valid
