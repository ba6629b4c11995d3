"""The C ABI without a GPU: the library loads, exports every entry point that
include/lnr.h declares, and its host-side logic (defaults, sizes, argument
checks) agrees with the oracle and the header. No kernel is launched."""
import ctypes as C
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lnr.h")


@pytest.fixture(scope="module")
def lnr():
    import paper_1504_01441_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1504_01441_amd import build
        build.build()
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lnr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lnr):
    names = declared_functions()
    assert len(names) >= 15
    L = C.CDLL(lnr.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lnr.EXPORTED)


def test_defaults_agree_with_oracle(lnr):
    p, op = lnr.Params(), oracle.params()
    for name, _ in op._fields_:
        assert getattr(p, name) == getattr(op, name), name


@pytest.mark.parametrize("w,h", [(640, 480), (2592, 1944), (4000, 3000), (331, 257), (32, 32)])
def test_query_sizes_match_oracle_levels(lnr, w, h):
    s = lnr.query_sizes(w, h, lnr.LNR_I420)
    op = oracle.params()
    L = oracle.num_levels(w, h, op)
    assert s.levels == L
    tot, ww, hh = 0, w, h
    for l in range(L):
        assert (s.level_w[l], s.level_h[l]) == (ww, hh)
        assert s.tile_off[l] == tot
        tot += (ww // 32) * (hh // 32)
        ww, hh = ww // 2, hh // 2
    assert s.tiles_total == tot == s.tile_off[L]
    assert s.blend_levels == oracle.num_blend_levels(w, h)
    assert s.channels == 3


@pytest.mark.parametrize("bad", [dict(radius0=33), dict(patch_r=12), dict(tile=8),
                                 dict(corner_half=5), dict(max_levels=6), dict(dt_iters=0),
                                 dict(sigma_r=0.0), dict(weed_iters=0), dict(ssim_radius=9),
                                 dict(quad_r=14)])
def test_parameter_checks(lnr, bad):
    p = lnr.Params(**bad)
    s = lnr._Sizes()
    assert lnr.lib().lnr_query_sizes(640, 480, 0, C.byref(p), C.byref(s)) == -2


def test_create_without_device_fails_cleanly(lnr):
    h = C.c_void_p()
    rc = lnr.lib().lnr_create(C.byref(h), 1 << 20)
    assert rc == -1 and not h.value


def test_flow_shapes_cover_the_image(lnr):
    """Host-only listing of the propagation shapes: every listed shape covers
    the image (row segments x threads >= W, column segments x rows >= H), and
    the listing is exactly the covering subset of the shape table."""
    for w, h in [(640, 480), (2592, 1944), (6144, 1024), (1024, 6144)]:
        shapes = lnr.flow_shapes(w, h)
        assert shapes, (w, h)
        for seg, nt, rows, ncol, nseg in shapes:
            assert seg * nt >= w and rows * nseg >= h
    assert len(lnr.flow_shapes(640, 480)) == 49      # every row x column shape
    assert len(lnr.flow_shapes(2592, 1944)) == 20
