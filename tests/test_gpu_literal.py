"""The paper-literal search frame (search_frame 1, Eq. 3 as printed: every
level searches the unwarped source around round(Hp x), fits its homography
to the absolute matches, and the absolute level-0 flow is propagated) on the
GPU against the oracle: tiles, flags, SSDs and every level's H bit-exact,
flow and warped image within 1e-4 relative."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import lnr, params_pair, registration_parity, to_gpu_frame

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return lnr().Context(0)


CASES = [
    ("c1 640x480 y8", lambda: synth.make_config_pair("c1", 1), 8, 100),
    ("330x250 i420 ragged", lambda: synth.make_stack(330, 250, 41, ratios=(1.0, 4.0), fmt="i420",
                                                    shift_range=4), 8, 64),
    ("c2 2592x1944 i420", lambda: synth.make_config_pair("c2", 1), 16, 100),
]


@pytest.mark.parametrize("name,make,R,mind", CASES, ids=[c[0] for c in CASES])
def test_literal_registration_matches_oracle(ctx, name, make, R, mind):
    st = make()
    f0, f1 = st.frames
    print(f"literal search {name}", flush=True)
    p, op = params_pair(radius0=R, min_level_dim=mind, search_frame=1)
    reg = lnr().register_pair(ctx, to_gpu_frame(f0), to_gpu_frame(f1), p)
    torch.cuda.synchronize()
    o = oracle.register_pair(f0, f1, op)
    registration_parity(reg, o, warped0=False)
    # the mapping is the flow alone: H^1 is not applied
    assert (o["flags"] & 2).sum() > 0


def test_literal_equals_warped_search_for_identical_frames(ctx):
    """Identical frames: both search frames find d = 0 everywhere, so the
    two registrations agree (tiles exactly; H = I and the copied image up to
    the rounding of the level fits, which compose differently)."""
    st = synth.make_config_pair("c1", 2)
    f0 = st.frames[0]
    L = lnr()
    p0 = L.Params(radius0=8)
    p1 = L.Params(radius0=8, search_frame=1)
    a = L.register_pair(ctx, to_gpu_frame(f0), to_gpu_frame(f0), p0)
    b = L.register_pair(ctx, to_gpu_frame(f0), to_gpu_frame(f0), p1)
    torch.cuda.synchronize()
    T = a.tile_off[a.levels]
    for k in ("corner_xy", "disp", "ssd", "flags"):
        assert torch.equal(getattr(a, k)[:T], getattr(b, k)[:T]), k
    assert np.allclose(a.H.cpu().numpy(), b.H.cpu().numpy(), atol=1e-9)
    assert np.allclose(a.image.cpu().numpy(), b.image.cpu().numpy(), atol=1e-6)


def test_literal_rejects_learned(ctx):
    L = lnr()
    st = synth.make_config_pair("c1", 1)
    f0, f1 = st.frames
    p = L.Params(radius0=8, search_frame=1, learned=1)
    out = L.Registration.alloc(f0.width, f0.height, L.LNR_Y8, L.Params(radius0=8))
    with pytest.raises(RuntimeError, match="search_frame"):
        L.register_pair(ctx, to_gpu_frame(f0), to_gpu_frame(f1), p, out=out)
