"""The seeded generator: determinism and the planted model."""
import numpy as np

import synth


def test_generator_is_deterministic():
    a = synth.make_config_pair("c1", 5)
    b = synth.make_config_pair("c1", 5)
    c = synth.make_config_pair("c1", 6)
    assert np.array_equal(a.frames[1].y, b.frames[1].y)
    assert np.array_equal(a.H_true[1], b.H_true[1])
    assert not np.array_equal(a.frames[1].y, c.frames[1].y)


def test_shapes_and_formats():
    st = synth.make_stack(128, 96, 1, ratios=(1.0, 4.0, 16.0), fmt="i420", noise_sigma=2.0)
    assert len(st.frames) == 3
    for f in st.frames:
        assert f.y.shape == (96, 128) and f.u.shape == (48, 64) and f.v.shape == (48, 64)
        assert f.y.dtype == np.uint8
    assert [f.exposure for f in st.frames] == [1.0, 4.0, 16.0]
    assert st.t_tile[1].shape == (3, 4, 2)


def test_reference_frame_is_the_scene_geometry():
    st = synth.make_pair(96, 64, 2, shift_range=0)
    gx, gy = st.gt_map(0)
    ys, xs = np.mgrid[0:64, 0:96]
    assert np.allclose(gx, xs) and np.allclose(gy, ys)


def test_planted_shift_pair_pastes_reference_blocks():
    ref, src, shifts, planted = synth.make_planted_shift_pair(256, 192, 3, 12)
    for ty, tx in zip(*np.nonzero(planted)):
        dx, dy = shifts[ty, tx]
        x0, y0 = tx * 32 + 2, ty * 32 + 2
        assert np.array_equal(src[y0 + dy:y0 + dy + 29, x0 + dx:x0 + dx + 29],
                              ref[y0:y0 + 29, x0:x0 + 29])
