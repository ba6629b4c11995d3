"""The allocation-free registration (lnr_register_pair_noalloc, fixed device
scratch) against lnr_register_pair on the same inputs: two calls in a row,
the second on a smaller pair, so the second runs on the scratch the first
left behind. Integer outputs bit-exact, float outputs within 1e-4 relative."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import assert_close, lnr, params_pair, to_gpu_frame

pytestmark = pytest.mark.gpu

INTS = ("corner_xy", "disp", "ssd", "flags", "counts", "H", "yeq_ref", "yeq_src", "warped0")
FLOATS = ("flow", "ntilde", "image", "yeq_warped")


def _check(got, want, tiles):
    for k in INTS:
        g, w = getattr(got, k), getattr(want, k)
        if k in ("corner_xy", "disp", "ssd", "flags"):
            g, w = g[:tiles], w[:tiles]
        assert torch.equal(g, w), k
    for k in FLOATS:
        assert_close(getattr(got, k).cpu().numpy(), getattr(want, k).cpu().numpy(), 1.0,
                     what=k)


@pytest.mark.parametrize("fmt", ["i420", "y8"])
def test_noalloc_matches_register_pair_twice(fmt):
    L = lnr()
    ctx = L.Context(0)
    cases = [(synth.make_stack(800, 600, 31, ratios=(1.0, 6.0), fmt=fmt, shift_range=6), 16),
             (synth.make_stack(330, 250, 32, ratios=(1.0, 4.0), fmt=fmt, shift_range=4), 8)]
    for st, R in cases:
        f0, f1 = st.frames
        print(f"noalloc {fmt} {f0.width}x{f0.height} R={R}", flush=True)
        p, _ = params_pair(radius0=R, min_level_dim=64)
        ref, src = to_gpu_frame(f0), to_gpu_frame(f1)
        fmt_id = L.LNR_I420 if fmt == "i420" else L.LNR_Y8
        got = L.Registration.alloc(f0.width, f0.height, fmt_id, p)
        got = L.register_pair_noalloc(ctx, ref, src, p, out=got)
        torch.cuda.synchronize()
        want = L.register_pair(ctx, ref, src, p)
        torch.cuda.synchronize()
        _check(got, want, want.tile_off[want.levels])


def test_noalloc_rejects_oversize_before_launch():
    L = lnr()
    ctx = L.Context(0)
    W, H = 4000, 3000
    y = torch.zeros(H, W, dtype=torch.uint8, device="cuda")
    f = L.Frame(y=y, u=None, v=None, exposure=1.0)
    p = L.Params(radius0=16)
    out = L.Registration.alloc(W, H, L.LNR_Y8, p)
    with pytest.raises(RuntimeError, match="scratch"):
        L.register_pair_noalloc(ctx, f, f, p, out=out)
