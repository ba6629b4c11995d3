"""Batches of uneven-size pairs (streams, cached HIP graphs, autotuning) give
exactly what one register_pair call per pair gives, and register_pair stays
within the oracle's tolerance after the domain-transform kernel shapes are
autotuned."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import registration_parity

pytestmark = pytest.mark.gpu

SIZES = [(640, 480), (354, 258), (512, 400), (290, 226), (800, 600), (418, 330)]


@pytest.fixture(scope="module")
def lnr():
    import paper_1504_01441_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(lnr):
    return lnr.Context(0)


def _pairs(lnr, seed0):
    out = []
    for i, (w, h) in enumerate(SIZES):
        st = synth.make_stack(w, h, seed0 + i, ratios=(1.0, 2.0 + 2 * i), fmt="i420",
                              shift_range=12)
        f0, f1 = st.frames
        out.append((f0, f1, lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure),
                    lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)))
    return out


FIELDS = ("corner_xy", "disp", "ssd", "flags", "counts", "H", "yeq_ref", "yeq_src", "warped0",
          "flow", "ntilde", "image", "yeq_warped")


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert torch.equal(x, y), f


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (True, True)])
def test_batch_equals_single_calls(lnr, ctx, graph, autotune):
    p = lnr.Params(radius0=12, min_level_dim=64)
    pairs = _pairs(lnr, 700)
    singles = [lnr.register_pair(ctx, r, s, p) for _, _, r, s in pairs]
    outs = lnr.register_batch(ctx, [q[2] for q in pairs], [q[3] for q in pairs], p,
                              graph=graph, autotune=autotune)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        _same(a, b)
    if graph:
        # replays of the cached graph, with other work and new contents in between
        for rep in range(3):
            for o in outs:
                o.flow.zero_()
                o.flags.fill_(255)
            singles[0].image.add_(1.0)
            lnr.register_batch(ctx, [q[2] for q in pairs], [q[3] for q in pairs], p, outs=outs,
                               graph=True, autotune=autotune)
            torch.cuda.synchronize()
            for a, b in zip(outs[1:], singles[1:]):
                _same(a, b)
            assert torch.equal(outs[0].flow, singles[0].flow)
            assert torch.equal(outs[0].flags, singles[0].flags)


def test_learned_batch_equals_single_calls(lnr, ctx):
    """The learned proposal inside a graph-captured batch (network inference
    and the windowed / fallback searches on the pairs' streams) gives exactly
    what one learned register_pair call per pair gives, over several replays."""
    from paper_1504_01441_amd import proposal as prop
    P, conf = prop.load()
    lnr.proposal_set(ctx, torch.from_numpy(P).cuda())
    p = lnr.Params(radius0=12, min_level_dim=64, learned=1, window_r=2, conf_min=conf)
    pairs = _pairs(lnr, 760)
    singles = [lnr.register_pair(ctx, r, s, p) for _, _, r, s in pairs]
    outs = lnr.register_batch(ctx, [q[2] for q in pairs], [q[3] for q in pairs], p, graph=True)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        _same(a, b)
    for rep in range(2):
        for o in outs:
            o.disp.zero_()
            o.flags.fill_(255)
        lnr.register_batch(ctx, [q[2] for q in pairs], [q[3] for q in pairs], p, outs=outs,
                           graph=True)
        torch.cuda.synchronize()
        for a, b in zip(outs, singles):
            _same(a, b)
    # some tiles took the window and some the fallback
    fl = np.concatenate([o.flags.cpu().numpy()[: o.tile_off[1]] for o in outs])
    cornered = (fl & 1) != 0
    assert (cornered & ((fl & 16) == 0)).any() and (cornered & ((fl & 16) != 0)).any()


def test_batch_matches_oracle(lnr, ctx):
    p = lnr.Params(radius0=12, min_level_dim=64)
    op = oracle.params(radius0=12, min_level_dim=64)
    pairs = _pairs(lnr, 720)[:3]
    outs = lnr.register_batch(ctx, [q[2] for q in pairs], [q[3] for q in pairs], p, graph=True)
    torch.cuda.synchronize()
    for (f0, f1, _, _), reg in zip(pairs, outs):
        registration_parity(reg, oracle.register_pair(f0, f1, op))


@pytest.mark.parametrize("w,h", [(640, 480), (1296, 972)])
def test_autotuned_flow_shape_keeps_parity(lnr, ctx, w, h):
    p = lnr.Params(radius0=12, min_level_dim=64)
    shape = lnr.autotune_flow(ctx, w, h, p)
    assert shape[0] * shape[1] >= w and shape[2] * shape[4] >= h
    st = synth.make_stack(w, h, 730, ratios=(1.0, 4.0), fmt="i420", shift_range=8)
    f0, f1 = st.frames
    reg = lnr.register_pair(ctx, lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure),
                            lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure), p)
    torch.cuda.synchronize()
    registration_parity(reg, oracle.register_pair(f0, f1, oracle.params(radius0=12,
                                                                        min_level_dim=64)))


@pytest.mark.parametrize("w,h,radius0", [(640, 480, 12), (1296, 972, 24)])
def test_autotuned_search_split_keeps_results(lnr, w, h, radius0):
    # a fresh context: the untuned run uses the default split, the second the tuned one
    c = lnr.Context(0)
    p = lnr.Params(radius0=radius0, min_level_dim=64)
    st = synth.make_stack(w, h, 750 + radius0, ratios=(1.0, 4.0), fmt="i420", shift_range=8)
    f0, f1 = st.frames
    F0 = lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
    F1 = lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
    before = lnr.register_pair(c, F0, F1, p)
    torch.cuda.synchronize()
    splits = lnr.autotune_search(c, w, h, p)
    # a split 1..7, plus 16 (12 candidates per lane) or 32 (matrix cores)
    assert len(splits) >= 2 and all(1 <= (s & 7) <= 7 and s & ~(16 | 32 | 7) == 0 and
                                    (s & 48) != 48 for s in splits)
    after = lnr.register_pair(c, F0, F1, p)
    torch.cuda.synchronize()
    _same(before, after)
    registration_parity(after, oracle.register_pair(
        f0, f1, oracle.params(radius0=radius0, min_level_dim=64)))


def test_nv12_equals_i420(lnr, ctx):
    # the same pixels as interleaved chroma (with a padded row stride) give the
    # same registration and merge, bit for bit
    w, h = 418, 330
    p = lnr.Params(radius0=12, min_level_dim=64)
    st = synth.make_stack(w, h, 760, ratios=(1.0, 4.0), fmt="i420", shift_range=8)
    f0, f1 = st.frames

    def nv12(f):
        uv = torch.zeros(h // 2, w + 64, dtype=torch.uint8)
        uv[:, 0:w:2] = torch.from_numpy(f.u)
        uv[:, 1:w:2] = torch.from_numpy(f.v)
        fr = lnr.Frame.nv12_from_numpy(f.y, np.zeros((1, 1), np.uint8), f.exposure)
        fr.u = uv.cuda()[:, :w]
        return fr

    I0 = lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
    I1 = lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
    N0, N1 = nv12(f0), nv12(f1)
    assert N0.fmt == lnr.LNR_NV12 and N0.u.stride(0) == w + 64
    a = lnr.register_pair(ctx, I0, I1, p)
    b = lnr.register_pair(ctx, N0, N1, p)
    torch.cuda.synchronize()
    _same(a, b)
    ha = lnr.merge(ctx, [I0, I1], 0, [a], p)
    hb = lnr.merge(ctx, [N0, N1], 0, [b], p)
    torch.cuda.synchronize()
    assert ha.shape == (3, h, w) and torch.equal(ha, hb)
    # mixed formats are rejected
    with pytest.raises(lnr.LnrError):
        lnr.register_pair(ctx, I0, N1, p)


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_register_pair_graph_capture(lnr):
    # a caller's own graph of one registration: a fresh context cannot grow its
    # workspace under capture (clean error, nothing enqueued); after one call
    # outside the capture, every replay equals the eager result, with other
    # eager work on the same context between the replays
    c = lnr.Context(0)
    w, h = 640, 480
    p = lnr.Params(radius0=12, min_level_dim=64)
    pairs = []
    for seed in (770, 771):
        st = synth.make_stack(w, h, seed, ratios=(1.0, 4.0), fmt="i420", shift_range=8)
        f0, f1 = st.frames
        pairs.append((lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure),
                      lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)))
    (A0, A1), (B0, B1) = pairs
    out = lnr.Registration.alloc(w, h, lnr.LNR_I420, p)
    g = torch.cuda.CUDAGraph()
    with pytest.raises(lnr.LnrError) as e:
        with torch.cuda.graph(g):
            lnr.register_pair(c, A0, A1, p, out=out)
    assert e.value.status == -6
    torch.cuda.synchronize()
    want_a = lnr.register_pair(c, A0, A1, p)
    want_b = lnr.register_pair(c, B0, B1, p)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lnr.register_pair(c, A0, A1, p, out=out)
    for _ in range(3):
        other = lnr.register_pair(c, B0, B1, p)
        torch.cuda.synchronize()
        _same(other, want_b)
        g.replay()
        torch.cuda.synchronize()
        _same(out, want_a)
    c.close()


def test_every_flow_shape_keeps_parity(lnr):
    """Each of the 49 propagation shapes (row segment x threads, column rows x
    columns x segments) pinned for a 640 x 480 pair gives the oracle's
    registration; shapes only regroup the recursions' scans."""
    c = lnr.Context(0)
    w, h = 640, 480
    p = lnr.Params(radius0=12, min_level_dim=64)
    st = synth.make_stack(w, h, 780, ratios=(1.0, 4.0), fmt="i420", shift_range=8)
    f0, f1 = st.frames
    F0 = lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
    F1 = lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
    o = oracle.register_pair(f0, f1, oracle.params(radius0=12, min_level_dim=64))
    shapes = lnr.flow_shapes(w, h)
    assert len(shapes) == 49
    for shp in shapes:
        lnr.set_flow_shape(c, w, h, shp)
        reg = lnr.register_pair(c, F0, F1, p)
        torch.cuda.synchronize()
        registration_parity(reg, o)
    with pytest.raises(lnr.LnrError):
        lnr.set_flow_shape(c, w, h, (5, 256, 8, 8, 128))    # not in the table
    with pytest.raises(lnr.LnrError):
        lnr.set_flow_shape(c, 4096, 480, (4, 256, 8, 8, 128))  # does not cover the width
    c.close()


def test_batch_rejects_bad_flags(lnr, ctx):
    import ctypes as C
    ref = _pairs(lnr, 740)[0][2]
    RA = (lnr._Frame * 1)(ref._c())
    out = lnr.Registration.alloc(ref.width, ref.height, lnr.LNR_I420, lnr.Params())
    OA = (lnr._Registration * 1)(out._c())
    rc = lnr.lib().lnr_register_batch(ctx._h, RA, RA, 1, C.byref(lnr.Params()), OA, 8,
                                      lnr._stream())
    assert rc == -1


# the batched workload's extremes and three sizes between them (the 64-pair
# batch draws widths from 640..4032 and heights from 480..3024)
C4_SIZES = [(4032, 3024), (640, 480), (2590, 1000), (1218, 2888), (3000, 2250)]


def test_c4_batch_full_range_matches_oracle(lnr, ctx):
    """A graph-captured, autotuned batch over the batched workload's whole
    size range (tile shifts +-16, exposure ratios 2-16, radius 16): every
    pair's registration against the oracle (tiles and H bit-exact, float
    outputs within 1e-4)."""
    p = lnr.Params(radius0=16)
    op = oracle.params(radius0=16)
    stacks = []
    for i, (w, h) in enumerate(C4_SIZES):
        stacks.append(synth.make_stack(w, h, 7100 + i, ratios=(1.0, 2.0 + 3.5 * i), fmt="i420",
                                       shift_range=16, max_rot_deg=2.0))
    refs = [lnr.Frame.from_numpy(s.frames[0].y, s.frames[0].u, s.frames[0].v, 1.0)
            for s in stacks]
    srcs = [lnr.Frame.from_numpy(s.frames[1].y, s.frames[1].u, s.frames[1].v,
                                 s.frames[1].exposure) for s in stacks]
    print("c4 batch sizes " + ", ".join(f"{w}x{h}" for w, h in C4_SIZES), flush=True)
    outs = lnr.register_batch(ctx, refs, srcs, p, graph=True, autotune=True)
    torch.cuda.synchronize()
    # a replay of the cached graph gives the same
    outs = lnr.register_batch(ctx, refs, srcs, p, outs=outs, graph=True)
    torch.cuda.synchronize()
    for st, reg, (w, h) in zip(stacks, outs, C4_SIZES):
        print(f"oracle {w}x{h}", flush=True)
        registration_parity(reg, oracle.register_pair(st.frames[0], st.frames[1], op))


def test_c5_learned_batch_full_size_equals_single_calls(lnr, ctx):
    """Three full 5 MP pairs of the benchmark recipe in one graph-captured
    learned batch give exactly what one learned register_pair call per pair
    gives."""
    from paper_1504_01441_amd import proposal as prop
    P, conf = prop.load()
    lnr.proposal_set(ctx, torch.from_numpy(P).cuda())
    p = lnr.Params(radius0=16, learned=1, window_r=2, conf_min=conf)
    stacks = [synth.make_config_pair("c2", s) for s in (21, 22, 23)]
    refs = [lnr.Frame.from_numpy(s.frames[0].y, s.frames[0].u, s.frames[0].v, 1.0)
            for s in stacks]
    srcs = [lnr.Frame.from_numpy(s.frames[1].y, s.frames[1].u, s.frames[1].v,
                                 s.frames[1].exposure) for s in stacks]
    singles = [lnr.register_pair(ctx, r, s, p) for r, s in zip(refs, srcs)]
    outs = lnr.register_batch(ctx, refs, srcs, p, graph=True, autotune=True)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        _same(a, b)
    outs = lnr.register_batch(ctx, refs, srcs, p, outs=outs, graph=True)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        _same(a, b)


@pytest.mark.parametrize("shape", [1, 3, 16 | 1, 16 | 2, 16 | 7, 32 | 1, 32 | 2, 32 | 5])
def test_every_search_shape_keeps_results(lnr, shape):
    """Each pinned search shape (patch-row split; 8 or 12 candidates per lane,
    or the matrix cores) at every level gives the untuned registration bit
    for bit."""
    p = lnr.Params(radius0=16)
    st = synth.make_stack(640, 480, 777, ratios=(1.0, 4.0), fmt="y8", shift_range=8)
    f0, f1 = st.frames
    F0, F1 = lnr.Frame.from_numpy(f0.y), lnr.Frame.from_numpy(f1.y)
    base = lnr.register_pair(lnr.Context(0), F0, F1, p)
    c = lnr.Context(0)
    s = lnr.query_sizes(640, 480, lnr.LNR_Y8, p)
    for l in range(s.levels):
        R = p.radius0 if l == 0 else p.radius_coarse
        lnr.set_search_shape(c, s.level_w[l], s.level_h[l], R, shape)
    got = lnr.register_pair(c, F0, F1, p)
    torch.cuda.synchronize()
    _same(base, got)


def test_search_shape_rejects_bad_shapes(lnr):
    c = lnr.Context(0)
    for bad in (0, 8, 16, 32, 16 | 32 | 1, 64, 64 | 1):
        with pytest.raises(lnr.LnrError):
            lnr.set_search_shape(c, 640, 480, 16, bad)
    # more than 64 KB of workgroup memory (radius 32, 12 candidates per lane,
    # two patch-row groups: ~69 KB) or more than 1024 threads (radius 32, 8
    # per lane, 2 groups; matrix cores, 4 groups)
    for bad in (16 | 2, 2, 32 | 4):
        with pytest.raises(lnr.LnrError):
            lnr.set_search_shape(c, 640, 480, 32, bad)
    lnr.set_search_shape(c, 640, 480, 32, 32 | 1)
    lnr.set_search_shape(c, 640, 480, 32, 32 | 3)  # (~56 KB, 960 threads)
