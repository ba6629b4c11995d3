"""Seeded synthetic HDR exposure stacks.

Scene model (radiance in reference DN):
    S(x) = base + sum of Gaussian blobs + per-pixel uniform texture in [-8, 8]
The reference frame samples S at integer pixels. Every other frame k sees the
scene through a planted homography H_k (rotation about the image centre,
translation, small perspective) composed with planted integer per-tile shifts
t_k(tile): the content at reference pixel x appears near H_k(x + t_k(tile(x))).
Frame k's pixel value is clip(round(ratio_k * S + noise)).

Chroma (I420) comes from two independent smooth blob fields around 128,
mapped the same way and not scaled by exposure.

Everything is a function of the seed; numpy's PCG64 generator is the only
source of randomness.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Frame:
    y: np.ndarray                   # uint8 [H][W]
    u: np.ndarray | None = None     # uint8 [H/2][W/2] (I420) or None (Y8)
    v: np.ndarray | None = None
    exposure: float = 1.0

    @property
    def fmt(self) -> str:
        return "y8" if self.u is None else "i420"

    @property
    def width(self) -> int:
        return int(self.y.shape[1])

    @property
    def height(self) -> int:
        return int(self.y.shape[0])


@dataclass
class Stack:
    frames: list
    H_true: list            # per frame: 3x3 float64, reference pixel -> frame pixel
    t_tile: list            # per frame: int32 [tiles_y][tiles_x][2] (dx, dy)
    tile: int = 32
    meta: dict = field(default_factory=dict)

    def gt_map(self, k: int):
        """Ground-truth position in frame k of every reference pixel (planted model)."""
        f0 = self.frames[0]
        W, H = f0.width, f0.height
        ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
        t = self.t_tile[k]
        ty = np.clip(ys.astype(np.int64) // self.tile, 0, t.shape[0] - 1)
        tx = np.clip(xs.astype(np.int64) // self.tile, 0, t.shape[1] - 1)
        X = xs + t[ty, tx, 0]
        Y = ys + t[ty, tx, 1]
        Hm = self.H_true[k]
        den = Hm[2, 0] * X + Hm[2, 1] * Y + Hm[2, 2]
        return ((Hm[0, 0] * X + Hm[0, 1] * Y + Hm[0, 2]) / den,
                (Hm[1, 0] * X + Hm[1, 1] * Y + Hm[1, 2]) / den)


# ----------------------------------------------------------------------------
# scene synthesis
# ----------------------------------------------------------------------------

def _blob_field(rng, W, H, n, amp, smin, smax):
    f = np.zeros((H, W), np.float64)
    cx = rng.uniform(0, W, n)
    cy = rng.uniform(0, H, n)
    sg = rng.uniform(smin, smax, n)
    am = rng.uniform(-amp, amp, n)
    for i in range(n):
        r = 4.0 * sg[i]
        x0, x1 = max(0, int(cx[i] - r)), min(W, int(cx[i] + r) + 1)
        y0, y1 = max(0, int(cy[i] - r)), min(H, int(cy[i] + r) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        gx = np.exp(-((np.arange(x0, x1) - cx[i]) ** 2) / (2 * sg[i] ** 2))
        gy = np.exp(-((np.arange(y0, y1) - cy[i]) ** 2) / (2 * sg[i] ** 2))
        f[y0:y1, x0:x1] += am[i] * np.outer(gy, gx)
    return f


def _bilinear(img, X, Y):
    """Sample img (float64 [h][w]) at float positions with edge clamping."""
    h, w = img.shape
    X = np.clip(X, 0.0, w - 1.0)
    Y = np.clip(Y, 0.0, h - 1.0)
    x0 = np.floor(X).astype(np.int64)
    y0 = np.floor(Y).astype(np.int64)
    x0 = np.minimum(x0, w - 2) if w > 1 else x0
    y0 = np.minimum(y0, h - 2) if h > 1 else y0
    ax = X - x0
    ay = Y - y0
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    return ((1 - ay) * ((1 - ax) * img[y0, x0] + ax * img[y0, x1])
            + ay * ((1 - ax) * img[y1, x0] + ax * img[y1, x1]))


def random_homography(rng, W, H, max_rot_deg, max_trans, max_persp_vga):
    """Reference pixel -> frame pixel homography about the image centre.

    The perspective bound is given per pixel at 640 px width and kept
    size-invariant (scaled by 640 / W) so every image size sees the same
    relative keystone.
    """
    th = math.radians(rng.uniform(-max_rot_deg, max_rot_deg))
    tx, ty = rng.uniform(-max_trans, max_trans, 2)
    p = max_persp_vga * 640.0 / W
    px, py = rng.uniform(-p, p, 2)
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    A = np.array([[math.cos(th), -math.sin(th), tx],
                  [math.sin(th), math.cos(th), ty],
                  [px, py, 1.0]])
    T = np.array([[1, 0, cx], [0, 1, cy], [0, 0, 1.0]])
    Ti = np.array([[1, 0, -cx], [0, 1, -cy], [0, 0, 1.0]])
    return T @ A @ Ti


def _render(rng, scene, chroma, m, W, H, Hm, t, tile, ratio, noise_sigma, fmt):
    """Render one frame of size W x H through homography Hm and shifts t."""
    Hi = np.linalg.inv(Hm)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)

    def inverse_map(X, Y):
        den = Hi[2, 0] * X + Hi[2, 1] * Y + Hi[2, 2]
        zx = (Hi[0, 0] * X + Hi[0, 1] * Y + Hi[0, 2]) / den
        zy = (Hi[1, 0] * X + Hi[1, 1] * Y + Hi[1, 2]) / den
        tyi = np.clip(np.floor(zy / tile).astype(np.int64), 0, t.shape[0] - 1)
        txi = np.clip(np.floor(zx / tile).astype(np.int64), 0, t.shape[1] - 1)
        return zx - t[tyi, txi, 0] + m, zy - t[tyi, txi, 1] + m

    sx, sy = inverse_map(xs, ys)
    val = _bilinear(scene, sx, sy) * ratio
    if noise_sigma > 0:
        n1 = rng.standard_normal(val.shape)
        n2 = rng.standard_normal(val.shape)
        val = val + np.sqrt(0.25 * np.maximum(val, 0.0)) * n1 + noise_sigma * n2
    y = np.clip(np.rint(val), 0, 255).astype(np.uint8)
    if fmt == "y8":
        return Frame(y=y, exposure=float(ratio))
    cys, cxs = np.mgrid[0:H // 2, 0:W // 2].astype(np.float64)
    csx, csy = inverse_map(2 * cxs + 0.5, 2 * cys + 0.5)
    u = np.clip(np.rint(_bilinear(chroma[0], csx, csy)), 0, 255).astype(np.uint8)
    v = np.clip(np.rint(_bilinear(chroma[1], csx, csy)), 0, 255).astype(np.uint8)
    return Frame(y=y, u=u, v=v, exposure=float(ratio))


def make_stack(W, H, seed, ratios=(1.0, 4.0), fmt="y8", tile=32,
               max_rot_deg=2.0, max_trans=10.0, max_persp_vga=1e-4,
               shift_range=6, mover_frac=0.0, mover_range=16,
               noise_sigma=0.0, sat_frac=0.0, n_blobs=200, ref_median=None,
               texture=8.0):
    """A stack of len(ratios) frames; frame 0 (ratio ratios[0]) is the reference geometry."""
    if fmt == "i420" and (W % 2 or H % 2):
        raise ValueError("I420 needs even width and height")
    if ref_median is None:
        # dark reference: the first source lands near mid-grey
        ref_median = 120.0 / (ratios[1] if len(ratios) > 1 else 4.0)
    rng = np.random.default_rng(seed)
    m = int(64 + 0.06 * max(W, H))
    CW, CH = W + 2 * m, H + 2 * m
    blobs = _blob_field(rng, CW, CH, n_blobs, 40.0, W / 100.0, W / 10.0)
    scene = blobs + rng.uniform(-texture, texture, (CH, CW))
    scene += ref_median - np.median(scene[m:m + H, m:m + W])
    if sat_frac > 0:
        yy, xx = np.mgrid[0:CH, 0:CW]
        target = sat_frac * W * H
        covered = np.zeros((CH, CW), bool)
        while covered[m:m + H, m:m + W].sum() < target:
            r = rng.uniform(W / 60.0, W / 20.0)
            cx, cy = rng.uniform(m, m + W), rng.uniform(m, m + H)
            covered |= (xx - cx) ** 2 + (yy - cy) ** 2 < r * r
        scene[covered] = 1e4
    chroma = None
    if fmt == "i420":
        chroma = [128.0 + _blob_field(rng, CW, CH, 60, 24.0, W / 40.0, W / 6.0)
                  for _ in range(2)]
    tx_n, ty_n = W // tile, H // tile
    frames, Hs, ts = [], [], []
    for k, ratio in enumerate(ratios):
        if k == 0:
            Hm = np.eye(3)
            t = np.zeros((max(ty_n, 1), max(tx_n, 1), 2), np.int32)
        else:
            Hm = random_homography(rng, W, H, max_rot_deg, max_trans, max_persp_vga)
            t = rng.integers(-shift_range, shift_range + 1,
                             (max(ty_n, 1), max(tx_n, 1), 2)).astype(np.int32)
            if mover_frac > 0:
                mv = rng.random((t.shape[0], t.shape[1])) < mover_frac
                mt = rng.integers(-mover_range, mover_range + 1, t.shape).astype(np.int32)
                t[mv] = mt[mv]
        frames.append(_render(rng, scene, chroma, m, W, H, Hm, t, tile, ratio,
                              noise_sigma, fmt))
        Hs.append(Hm)
        ts.append(t)
    return Stack(frames=frames, H_true=Hs, t_tile=ts, tile=tile,
                 meta=dict(W=W, H=H, seed=seed, ratios=tuple(ratios), fmt=fmt))


def make_pair(W, H, seed, ratio=4.0, **kw):
    return make_stack(W, H, seed, ratios=(1.0, ratio), **kw)


# Workload shapes: sizes, exposure ratios, planted motion and noise of each case.
CONFIGS = {
    # 640x480 Y8, exposure ratio 4, rotation <= 2 deg, translation <= 10 px,
    # perspective <= 1e-4, per-tile shifts in [-6, 6]; radius 8 at level 0
    "c1": dict(W=640, H=480, ratios=(1.0, 4.0), fmt="y8", shift_range=6,
               max_rot_deg=2.0, radius0=8),
    # 5 MP I420, ratio 8, Poisson-Gaussian noise sigma 2 DN, 10% mover tiles in [-16, 16]
    "c2": dict(W=2592, H=1944, ratios=(1.0, 8.0), fmt="i420", shift_range=6,
               mover_frac=0.10, mover_range=16, noise_sigma=2.0,
               max_rot_deg=2.0, radius0=16),
    # 12 MP 3-frame stack, ratios 1/4/16, rotation <= 3 deg, shifts in [-12, 12],
    # 5% saturated regions
    "c3": dict(W=4000, H=3000, ratios=(1.0, 4.0, 16.0), fmt="i420",
               shift_range=12, max_rot_deg=3.0, sat_frac=0.05, noise_sigma=2.0,
               radius0=16),
}


def make_config_pair(name, seed, scale=None):
    """Stack for a named workload; `scale` optionally shrinks W and H (tests)."""
    cfg = dict(CONFIGS[name])
    radius0 = cfg.pop("radius0")
    W, H = cfg.pop("W"), cfg.pop("H")
    if scale is not None:
        W = int(W * scale) // 2 * 2
        H = int(H * scale) // 2 * 2
    st = make_stack(W, H, seed, **cfg)
    st.meta["radius0"] = radius0
    st.meta["config"] = name
    return st


# Pixel-count sweep, VGA to 12 MP (4:3), for runtime against image size
SWEEP_SIZES = ((640, 480), (1280, 960), (2048, 1536), (2592, 1944), (3264, 2448), (4000, 3000))


def make_sweep_pair(W, H, seed):
    """The 5 MP pair's recipe (I420, ratio 8, noise sigma 2 DN, 10% mover
    tiles, radius 16) at another size."""
    cfg = dict(CONFIGS["c2"])
    radius0 = cfg.pop("radius0")
    cfg.pop("W")
    cfg.pop("H")
    st = make_stack(W, H, seed, **cfg)
    st.meta["radius0"] = radius0
    st.meta["config"] = "sweep"
    return st


def make_batch_pair(seed):
    """One pair of the batched workload: width and height drawn uniformly over
    even sizes from 640x480 to 4032x3024, 8-bit I420, exposure ratio in
    [2, 16], per-tile translations in [-16, 16]; search radius 16."""
    rng = np.random.default_rng(seed)
    W = int(rng.integers(320, 2017)) * 2
    H = int(rng.integers(240, 1513)) * 2
    ratio = float(rng.uniform(2.0, 16.0))
    st = make_stack(W, H, seed, ratios=(1.0, ratio), fmt="i420", shift_range=16,
                    max_rot_deg=2.0)
    st.meta["radius0"] = 16
    st.meta["config"] = "c4"
    return st


def make_texture(W, H, seed, lo=0, hi=256):
    """I.i.d. uniform 8-bit texture."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, (H, W)).astype(np.uint8)


def make_planted_shift_pair(W, H, seed, R, tile=32, patch_reach=14):
    """Reference texture plus a source into which, for every tile whose indices
    are both even, the reference block around the tile centre (the region that
    any candidate corner's patch can touch: centre +- patch_reach) is pasted
    at a planted integer shift in [-R, R]^2. Planted blocks never overlap
    (tiles are two tiles apart); everything else in the source is independent
    texture. Returns (ref, src, shifts[ty][tx][2], planted_mask[ty][tx])."""
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 256, (H, W)).astype(np.uint8)
    src = rng.integers(0, 256, (H, W)).astype(np.uint8)
    ty_n, tx_n = H // tile, W // tile
    shifts = np.zeros((ty_n, tx_n, 2), np.int32)
    planted = np.zeros((ty_n, tx_n), bool)
    c = tile // 2
    for ty in range(ty_n):
        for tx in range(tx_n):
            if tx % 2 or ty % 2:
                continue
            x0, y0 = tx * tile + c - patch_reach, ty * tile + c - patch_reach
            x1, y1 = tx * tile + c + patch_reach, ty * tile + c + patch_reach
            lo_x, hi_x = max(-R, -x0), min(R, W - 1 - x1)
            lo_y, hi_y = max(-R, -y0), min(R, H - 1 - y1)
            dx = int(rng.integers(lo_x, hi_x + 1))
            dy = int(rng.integers(lo_y, hi_y + 1))
            src[y0 + dy:y1 + dy + 1, x0 + dx:x1 + dx + 1] = ref[y0:y1 + 1, x0:x1 + 1]
            shifts[ty, tx] = (dx, dy)
            planted[ty, tx] = True
    return ref, src, shifts, planted
