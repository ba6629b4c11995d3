"""GPU path vs the CPU oracle, through the C ABI (stage by stage on the
oracle's own intermediate inputs, then end to end). Integer outputs must be
bit-exact; FP32 outputs within 1e-4 relative (tests/gpu_util.py)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_close, assert_tiles_equal, lnr, params_pair,
                      registration_parity, to_gpu_frame)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lnr().Context(0)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sync():
    torch.cuda.synchronize()


# ------------------------------------------------------------------ stages

@pytest.mark.parametrize("shape", [(480, 640), (97, 133), (1, 5), (1944, 2592)])
def test_equalize(ctx, shape):
    rng = np.random.default_rng(shape[0])
    img = np.clip(rng.normal(40, 25, shape), 0, 255).astype(np.uint8)
    lut, out = lnr().stage_equalize(ctx, _t(img))
    _sync()
    assert np.array_equal(lut.cpu().numpy(), oracle.equalize_lut(oracle.histogram(img)))
    assert np.array_equal(out.cpu().numpy(), oracle.equalize(img))


def test_equalize_strided_and_constant(ctx):
    base = np.random.default_rng(3).integers(0, 256, (50, 90)).astype(np.uint8)
    t = _t(base)[:, 7:71]             # row stride 90, width 64
    lut, out = lnr().stage_equalize(ctx, t)
    _sync()
    assert np.array_equal(out.cpu().numpy(), oracle.equalize(base[:, 7:71]))
    flat = np.full((33, 47), 91, np.uint8)
    lut, out = lnr().stage_equalize(ctx, _t(flat))
    _sync()
    assert np.array_equal(out.cpu().numpy(), flat)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_warp_q8(ctx, seed):
    rng = np.random.default_rng(seed)
    h, w = [(480, 640), (121, 162), (243, 325)][seed]
    img = rng.integers(0, 256, (h, w)).astype(np.uint8)
    th = rng.uniform(-0.05, 0.05)
    H = np.array([[math.cos(th), -math.sin(th), rng.uniform(-0.05, 0.05)],
                  [math.sin(th), math.cos(th), rng.uniform(-0.05, 0.05)],
                  [rng.uniform(-0.03, 0.03), rng.uniform(-0.03, 0.03), 1.0]])
    got = lnr().stage_warp_q8(ctx, _t(img), torch.from_numpy(H.reshape(9)))
    _sync()
    want = oracle.warp_q8(img, oracle.pixel_homography(H, w, h))
    assert np.array_equal(got.cpu().numpy(), want)


def _eq_pair(cfg, seed, scale=None):
    st = synth.make_config_pair(cfg, seed, scale=scale)
    return st, oracle.equalize(st.frames[0].y), oracle.equalize(st.frames[1].y)


@pytest.mark.parametrize("R", [0, 3, 8, 10, 16, 32])
def test_search_vs_oracle(ctx, R):
    st, a, b = _eq_pair("c1", 4)
    p, op = params_pair()
    cx, cy, has = oracle.corners(a, op)
    dx, dy, ssd, valid = oracle.search(a, b, R, cx, cy, has, op)
    cxy, disp, gssd, flags = lnr().stage_search(ctx, _t(a), _t(b), R, p)
    _sync()
    c = cxy.cpu().numpy()
    assert np.array_equal(c[:, 0], np.where(has > 0, cx, -1))
    assert np.array_equal(c[:, 1], np.where(has > 0, cy, -1))
    d = disp.cpu().numpy()
    assert np.array_equal(d[:, 0], dx) and np.array_equal(d[:, 1], dy)
    assert np.array_equal(gssd.cpu().numpy().view(np.uint32), ssd)
    assert np.array_equal(flags.cpu().numpy(), has | (valid << 1))


def test_search_planted_shifts_and_ragged_size(ctx):
    R = 16
    ref, src, shifts, planted = synth.make_planted_shift_pair(335, 259, 21, R)
    p, op = params_pair()
    cxy, disp, ssd, flags = lnr().stage_search(ctx, _t(ref), _t(src), R, p)
    _sync()
    d = disp.cpu().numpy()
    ntx = 335 // 32
    cx, cy, has = oracle.corners(ref, op)
    dx, dy, ossd, valid = oracle.search(ref, src, R, cx, cy, has, op)
    assert np.array_equal(d[:, 0], dx) and np.array_equal(d[:, 1], dy)
    assert np.array_equal(ssd.cpu().numpy().view(np.uint32), ossd)
    hit = 0
    for t in range(len(d)):
        ty, tx = divmod(t, ntx)
        if planted[ty, tx] and has[t]:
            assert tuple(d[t]) == tuple(shifts[ty, tx])
            hit += 1
    assert hit > 10


def test_search_other_patch_and_grid(ctx):
    st, a, b = _eq_pair("c1", 6)
    kw = dict(tile=48, patch_r=7, corner_half=3, corner_step=3, quad_r=8, corner_t=1)
    p, op = params_pair(**kw)
    cx, cy, has = oracle.corners(a, op)
    dx, dy, ssd, valid = oracle.search(a, b, 12, cx, cy, has, op)
    cxy, disp, gssd, flags = lnr().stage_search(ctx, _t(a), _t(b), 12, p)
    _sync()
    d = disp.cpu().numpy()
    assert np.array_equal(d[:, 0], dx) and np.array_equal(d[:, 1], dy)
    assert np.array_equal(gssd.cpu().numpy().view(np.uint32), ssd)
    assert np.array_equal(flags.cpu().numpy(), has | (valid << 1))


@pytest.mark.parametrize("R,shape", [(0, 32 | 1), (3, 32 | 1), (3, 32 | 3), (8, 32 | 2), (12, 32 | 4),
                                     (10, 32 | 1), (10, 32 | 4), (16, 32 | 1), (16, 32 | 3),
                                     (32, 32 | 1), (32, 32 | 3), (24, 32 | 2)])
def test_search_mfma_vs_oracle(R, shape):
    """The matrix-core cross terms (window rows times the Toeplitz matrix of a
    patch row, int8 products of the centred pixels), pinned for the level's
    size, against the oracle's search: corners, displacements, SSDs and flags
    bit for bit, with and without the patch rows split over wave groups."""
    c = lnr().Context(0)
    st, a, b = _eq_pair("c1", 4)
    p, op = params_pair()
    h, w = a.shape
    lnr().set_search_shape(c, w, h, R, shape)
    cx, cy, has = oracle.corners(a, op)
    dx, dy, ssd, valid = oracle.search(a, b, R, cx, cy, has, op)
    cxy, disp, gssd, flags = lnr().stage_search(c, _t(a), _t(b), R, p)
    _sync()
    d = disp.cpu().numpy()
    assert np.array_equal(d[:, 0], dx) and np.array_equal(d[:, 1], dy)
    assert np.array_equal(gssd.cpu().numpy().view(np.uint32), ssd)
    assert np.array_equal(flags.cpu().numpy(), has | (valid << 1))
    c.close()


def test_search_mfma_other_patch_and_grid():
    c = lnr().Context(0)
    st, a, b = _eq_pair("c1", 6)
    kw = dict(tile=48, patch_r=7, corner_half=3, corner_step=3, quad_r=8, corner_t=1)
    p, op = params_pair(**kw)
    h, w = a.shape
    lnr().set_search_shape(c, w, h, 12, 32 | 2)
    cx, cy, has = oracle.corners(a, op)
    dx, dy, ssd, valid = oracle.search(a, b, 12, cx, cy, has, op)
    cxy, disp, gssd, flags = lnr().stage_search(c, _t(a), _t(b), 12, p)
    _sync()
    d = disp.cpu().numpy()
    assert np.array_equal(d[:, 0], dx) and np.array_equal(d[:, 1], dy)
    assert np.array_equal(gssd.cpu().numpy().view(np.uint32), ssd)
    assert np.array_equal(flags.cpu().numpy(), has | (valid << 1))
    c.close()


def _oracle_level0(cfg, seed, scale=None, **kw):
    st = synth.make_config_pair(cfg, seed, scale=scale)
    kw.setdefault("radius0", st.meta["radius0"])
    p, op = params_pair(**kw)
    return st, p, op, oracle.register_pair(st.frames[0], st.frames[1], op)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_weed_fit_vs_oracle(ctx, level):
    st, p, op, o = _oracle_level0("c1", 7)
    a, b = o["tile_off"][level], o["tile_off"][level + 1]
    w, h = o["level_sizes"][level]
    cxy = np.stack([o["corner_x"][a:b], o["corner_y"][a:b]], 1).astype(np.int32)
    disp = np.stack([o["dx"][a:b], o["dy"][a:b]], 1).astype(np.int32)
    flags = (o["flags"][a:b] & 3).astype(np.uint8)
    gf, Ho, counts = lnr().stage_weed_fit(ctx, _t(cxy), _t(disp), _t(flags), w, h, level,
                                          torch.from_numpy(o["H"][level + 1].reshape(9)), p)
    _sync()
    assert np.array_equal(gf.cpu().numpy(), o["flags"][a:b])
    c = counts.cpu().numpy()
    assert c[0] == o["n_valid"][level] and c[1] == o["n_inliers"][level]
    assert np.array_equal(Ho.cpu().numpy().reshape(3, 3), o["H"][level])


def test_weed_split_parity_many_iterations(ctx):
    """8,192 hypotheses run in parallel give the oracle's sequential union."""
    st, p, op, o = _oracle_level0("c1", 8)
    p.weed_iters = 8192
    op.weed_iters = 8192
    b = o["tile_off"][1]
    cxy = np.stack([o["corner_x"][:b], o["corner_y"][:b]], 1).astype(np.int32)
    disp = np.stack([o["dx"][:b], o["dy"][:b]], 1).astype(np.int32)
    valid = ((o["flags"][:b] & 2) > 0).astype(np.uint8)
    M, n, bc, bi = oracle.weed(cxy[:, 0], cxy[:, 1], disp[:, 0], disp[:, 1], valid, 640, 480, 0, op)
    gf, Ho, counts = lnr().stage_weed_fit(ctx, _t(cxy), _t(disp), _t(o["flags"][:b] & 3),
                                          640, 480, 0, torch.from_numpy(np.eye(3).reshape(9)), p)
    _sync()
    assert np.array_equal((gf.cpu().numpy() & 4) > 0, M > 0)
    assert counts.cpu().numpy()[3] == bi


def test_flow_vs_oracle(ctx):
    st, p, op, o = _oracle_level0("c1", 9)
    b = o["tile_off"][1]
    cxy = np.stack([o["corner_x"][:b], o["corner_y"][:b]], 1).astype(np.int32)
    disp = np.stack([o["dx"][:b], o["dy"][:b]], 1).astype(np.int32)
    flow, nt = lnr().stage_flow(ctx, _t(cxy), _t(disp), _t(o["flags"][:b]), _t(o["yeq_ref"]), p)
    _sync()
    mask = o["ntilde"] > 2e-30
    f = flow.cpu().numpy()
    assert_close(f[0], o["flow_u"], 1.0, mask=mask, what="flow u")
    assert_close(f[1], o["flow_v"], 1.0, mask=mask, what="flow v")


@pytest.mark.parametrize("sigma_r", [0.05, 1.0, 4.0])
def test_flow_sigma_r(ctx, sigma_r):
    st, p, op, o = _oracle_level0("c1", 10)
    b = o["tile_off"][1]
    p.sigma_r = op.sigma_r = sigma_r
    cx, cy = o["corner_x"][:b], o["corner_y"][:b]
    fu, fv, nt = oracle.sparse_to_dense(cx, cy, o["dx"][:b], o["dy"][:b],
                                        (o["flags"][:b] & 4) > 0, o["yeq_ref"], op)
    cxy = np.stack([cx, cy], 1).astype(np.int32)
    disp = np.stack([o["dx"][:b], o["dy"][:b]], 1).astype(np.int32)
    flow, gnt = lnr().stage_flow(ctx, _t(cxy), _t(disp), _t(o["flags"][:b]), _t(o["yeq_ref"]), p)
    _sync()
    mask = nt > 2e-30
    f = flow.cpu().numpy()
    assert_close(f[0], fu, 1.0, mask=mask, what="flow u")
    assert_close(f[1], fv, 1.0, mask=mask, what="flow v")


@pytest.mark.parametrize("fmt", ["y8", "i420"])
def test_backward_warp_vs_oracle(ctx, fmt):
    st = synth.make_stack(322, 250, 12, ratios=(1.0, 4.0), fmt=fmt)
    f1 = st.frames[1]
    rng = np.random.default_rng(12)
    fu = rng.uniform(-6, 6, (250, 322)).astype(np.float32)
    fv = rng.uniform(-6, 6, (250, 322)).astype(np.float32)
    th = 0.04
    H = np.array([[math.cos(th), -math.sin(th), 0.02], [math.sin(th), math.cos(th), -0.03],
                  [0.01, -0.02, 1.0]])
    yeq = oracle.equalize(f1.y)
    img, yw = lnr().stage_backward_warp(ctx, to_gpu_frame(f1), _t(yeq),
                                        torch.from_numpy(H.reshape(9)), _t(np.stack([fu, fv])))
    _sync()
    want, ywant = oracle.backward_warp(f1.y, f1.u, f1.v, yeq, oracle.pixel_homography(H, 322, 250),
                                       fu.astype(np.float64), fv.astype(np.float64))
    assert_close(img.cpu().numpy(), want, 1.0, what="image")
    assert_close(yw.cpu().numpy(), ywant, 1.0, what="Y_eq")


@pytest.mark.parametrize("n,ch,shape", [(2, 3, (480, 640)), (3, 3, (301, 411)), (2, 1, (97, 64)),
                                        (1, 3, (64, 80)), (4, 1, (7, 9))])
def test_merge_vs_oracle(ctx, n, ch, shape):
    rng = np.random.default_rng(n * 10 + ch)
    h, w = shape
    import scipy.ndimage as ndi
    imgs = [np.clip(ndi.gaussian_filter(rng.uniform(0, 1, (ch, h, w)), (0, 1.5, 1.5)) * 1.6 - 0.3,
                    0, 1) for _ in range(n)]
    yeqs = [np.clip(ndi.gaussian_filter(rng.uniform(0, 1, (h, w)), 1.0) * 2 - 0.5, 0, 1)
            for _ in range(n)]
    ref = n // 2
    p, op = params_pair()
    got = lnr().stage_merge(ctx, [_t(i.astype(np.float32)) for i in imgs],
                            [_t(y.astype(np.float32)) for y in yeqs], ref, p)
    _sync()
    want = oracle.merge([i.astype(np.float32).astype(np.float64) for i in imgs],
                        [y.astype(np.float32).astype(np.float64) for y in yeqs], ref, op)
    assert_close(got.cpu().numpy(), want, 1.0, what="merge")


@pytest.mark.parametrize("r,sigma", [(1, 0.7), (3, 1.0), (8, 2.5)])
def test_merge_ssim_window_sizes(ctx, r, sigma):
    """SSIM windows other than the default 11 x 11 (one kernel build per radius),
    on a width that leaves a ragged last column tile."""
    rng = np.random.default_rng(40 + r)
    h, w = 133, 517
    import scipy.ndimage as ndi
    imgs = [np.clip(ndi.gaussian_filter(rng.uniform(0, 1, (3, h, w)), (0, 1.2, 1.2)) * 1.6 - 0.3,
                    0, 1) for _ in range(2)]
    yeqs = [np.clip(ndi.gaussian_filter(rng.uniform(0, 1, (h, w)), 1.0) * 2 - 0.5, 0, 1)
            for _ in range(2)]
    p, op = params_pair(ssim_radius=r, ssim_sigma=sigma)
    got = lnr().stage_merge(ctx, [_t(i.astype(np.float32)) for i in imgs],
                            [_t(y.astype(np.float32)) for y in yeqs], 0, p)
    _sync()
    want = oracle.merge([i.astype(np.float32).astype(np.float64) for i in imgs],
                        [y.astype(np.float32).astype(np.float64) for y in yeqs], 0, op)
    assert_close(got.cpu().numpy(), want, 1.0, what="merge")


# ------------------------------------------------------------------ end to end

@pytest.mark.parametrize("seed", [1, 2])
def test_register_pair_c1(ctx, seed):
    st = synth.make_config_pair("c1", seed)
    p, op = params_pair(radius0=8)
    reg = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    _sync()
    o = oracle.register_pair(st.frames[0], st.frames[1], op)
    registration_parity(reg, o)


@pytest.mark.parametrize("size", [(330, 250), (129, 100), (64, 48), (32, 32)])
def test_register_pair_ragged_and_small(ctx, size):
    w, h = size
    fmt = "i420" if w % 2 == 0 and h % 2 == 0 else "y8"
    st = synth.make_stack(w, h, 13, ratios=(1.0, 2.0), fmt=fmt, shift_range=3)
    p, op = params_pair(radius0=8, min_level_dim=50)
    reg = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    _sync()
    o = oracle.register_pair(st.frames[0], st.frames[1], op)
    registration_parity(reg, o)


def test_register_identical_frames(ctx):
    st = synth.make_config_pair("c1", 14)
    f = st.frames[0]
    p, op = params_pair(radius0=8)
    reg = lnr().register_pair(ctx, to_gpu_frame(f), to_gpu_frame(f), p)
    _sync()
    o = oracle.register_pair(f, f, op)
    registration_parity(reg, o)
    assert not reg.disp.cpu().numpy()[: o["tile_off"][1]].any()
    assert np.abs(reg.flow.cpu().numpy()).max() == 0.0


def _gpu_merge_planes(ctx, frames, ref, regs):
    """The float32 planes lnr_merge consumes, on the GPU: the reference's RGB
    (a zero-flow identity backward warp runs the same conversion as the
    merge's own), the registered frames, and the luma maps. For checking
    lnr_merge against the merge stage (GPU against GPU); never an oracle input."""
    f = frames[ref]
    gref = to_gpu_frame(f)
    img_ref, _ = lnr().stage_backward_warp(ctx, gref, regs[0].yeq_ref,
                                           torch.from_numpy(np.eye(3).reshape(9)),
                                           torch.zeros(2, f.height, f.width, device="cuda"))
    yref = regs[0].yeq_ref.float() / 255.0
    imgs, yeqs, j = [], [], 0
    for k in range(len(frames)):
        if k == ref:
            imgs.append(img_ref)
            yeqs.append(yref)
        else:
            imgs.append(regs[j].image)
            yeqs.append(regs[j].yeq_warped)
            j += 1
    return imgs, yeqs


def _oracle_merge_planes(frames, ref, regs_o):
    """The oracle's own registered planes (its reference RGB, its warped frames
    and luma maps), rounded to float32 as a merge consumes them."""
    f = frames[ref]
    imgs, yeqs, j = [], [], 0
    for k in range(len(frames)):
        if k == ref:
            imgs.append(oracle.frame_to_rgb(f.y, f.u, f.v).astype(np.float32))
            yeqs.append((regs_o[0]["yeq_ref"] / 255.0).astype(np.float32))
        else:
            imgs.append(regs_o[j]["rgb"].astype(np.float32))
            yeqs.append(regs_o[j]["yeq_warped"].astype(np.float32))
            j += 1
    return imgs, yeqs


def _check_full_merge(ctx, frames, ref, regs, regs_o, out, p, op):
    """lnr_merge agrees with the merge stage on the same GPU planes (its
    workspace offsets differ, which can change the blend's vector path, so
    within the tolerance rather than bit for bit), and the merge stage on the
    oracle's registered planes equals the oracle's merge of those planes (the
    fusion divides weight sums near 1e-12, so the two merges are compared on
    identical inputs)."""
    gi, gy = _gpu_merge_planes(ctx, frames, ref, regs)
    again = lnr().stage_merge(ctx, gi, gy, ref, p)
    _sync()
    assert_close(out.cpu().numpy(), again.cpu().numpy(), 1.0, what="lnr_merge vs merge stage")
    oi, oy = _oracle_merge_planes(frames, ref, regs_o)
    got = lnr().stage_merge(ctx, [_t(i) for i in oi], [_t(y) for y in oy], ref, p)
    _sync()
    want = oracle.merge([i.astype(np.float64) for i in oi], [y.astype(np.float64) for y in oy],
                        ref, op)
    assert_close(got.cpu().numpy(), want, 1.0, what="merge")


def test_register_pair_c2_full_size(ctx):
    """The 5 MP benchmark workload, in the launch configuration bench.py times:
    the registration against the oracle's; lnr_merge against the merge stage,
    and the merge stage on the oracle's registered planes against the
    oracle's merge of them."""
    st = synth.make_config_pair("c2", 1)
    p, op = params_pair(radius0=16)
    g = [to_gpu_frame(f) for f in st.frames]
    reg = lnr().register_pair(ctx, g[0], g[1], p)
    hdr = lnr().merge(ctx, g, 0, [reg], p)
    _sync()
    o = oracle.register_pair(st.frames[0], st.frames[1], op)
    registration_parity(reg, o)
    _check_full_merge(ctx, st.frames, 0, [reg], [o], hdr, p, op)


@pytest.mark.parametrize("size", [(6144, 1024), (1024, 6144)])
def test_register_pair_maximum_side(ctx, size):
    """The largest supported side (6144) in each direction: rows wider than the
    default 64 KB of workgroup memory in the row propagation, the tallest
    column shape, 192 tiles per level-0 row or column."""
    w, h = size
    st = synth.make_stack(w, h, 21, ratios=(1.0, 4.0), fmt="i420", shift_range=6)
    p, op = params_pair(radius0=8)
    reg = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    _sync()
    o = oracle.register_pair(st.frames[0], st.frames[1], op)
    registration_parity(reg, o)


@pytest.mark.parametrize("size", [(1280, 960), (3264, 2448)])
def test_sweep_sizes_match_oracle(ctx, size):
    """Pairs of the pixel-count sweep (the 5 MP recipe at other sizes), in the
    autotuned launch configuration the sweep times."""
    w, h = size
    st = synth.make_sweep_pair(w, h, 1)
    p, op = params_pair(radius0=16)
    lnr().autotune_flow(ctx, w, h, p)
    lnr().autotune_search(ctx, w, h, p)
    reg = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    _sync()
    registration_parity(reg, oracle.register_pair(st.frames[0], st.frames[1], op))


@pytest.mark.parametrize("n,ch,shape,ref", [(2, 3, (37, 53), 0), (3, 3, (120, 203), 1),
                                             (5, 1, (64, 257), 2), (16, 3, (33, 70), 7)])
def test_irradiance_vs_oracle(ctx, n, ch, shape, ref):
    """Irradiance map of synthetic linear stacks (saturated and black samples,
    a ghost frame with anti-correlated luma), same float32 planes on both
    sides, on ragged sizes."""
    rng = np.random.default_rng(900 + n * 10 + ch)
    h, w = shape
    import scipy.ndimage as ndi
    E = ndi.gaussian_filter(rng.uniform(0, 1, (ch, h, w)), (0, 1.5, 1.5)) * 0.5 + 0.01
    rel = [2.0 ** (k - ref) for k in range(n)]
    expo = [0.5 * r for r in rel]                   # absolute; only ratios matter
    imgs = [np.clip(E * r + rng.normal(0, 0.003, E.shape), 0, 1).astype(np.float32)
            for r in rel]
    base = ndi.gaussian_filter(rng.uniform(0, 1, (h, w)), 1.0)
    yeqs = [np.clip(base + rng.normal(0, 0.02, (h, w)), 0, 1).astype(np.float32)
            for _ in range(n)]
    if n > 2:
        yeqs[0 if ref else 1] = (1.0 - yeqs[ref]).astype(np.float32)   # a ghost
    p, op = params_pair()
    got = lnr().stage_irradiance(ctx, [_t(i) for i in imgs], [_t(y) for y in yeqs], expo, ref, p)
    _sync()
    want = oracle.irradiance([i.astype(np.float64) for i in imgs],
                             [y.astype(np.float64) for y in yeqs], expo, ref, op)
    assert_close(got.cpu().numpy(), want, 1.0, what="irradiance")


def test_merge_irradiance_full_path(ctx):
    """A registered pair's irradiance map against the oracle's map of the
    oracle's own registration."""
    st = synth.make_config_pair("c2", 3, scale=0.25)
    p, op = params_pair(radius0=16)
    g = [to_gpu_frame(f) for f in st.frames]
    reg = lnr().register_pair(ctx, g[0], g[1], p)
    got = lnr().merge_irradiance(ctx, g, 0, [reg], p)
    _sync()
    o = oracle.register_pair(st.frames[0], st.frames[1], op)
    registration_parity(reg, o)
    f0 = st.frames[0]
    ref_rgb = oracle.frame_to_rgb(f0.y, f0.u, f0.v)
    want = oracle.irradiance([ref_rgb, o["rgb"]],
                             [o["yeq_ref"].astype(np.float64) / 255.0, o["yeq_warped"]],
                             [f.exposure for f in st.frames], 0, op)
    assert_close(got.cpu().numpy(), want, 1.0, what="irradiance map")
    # the map is in the reference's units: where the reference is neither black
    # nor saturated and no ghost, it is close to the reference's own values
    assert np.isfinite(got.cpu().numpy()).all()


@pytest.mark.parametrize("h,w,n_dark", [(40, 50, 0), (40, 50, 100), (40, 50, 101),
                                         (40, 50, 400), (40, 50, 401), (40, 50, 2000),
                                         (1944, 2592, 500000), (487, 613, 14000)])
def test_meter_vs_oracle(ctx, h, w, n_dark):
    """Metering decision and under-exposed count, exact, on padded rows."""
    rng = np.random.default_rng(h + n_dark)
    y = rng.integers(16, 256, (h, w)).astype(np.uint8)
    idx = rng.permutation(h * w)[:n_dark]
    y.reshape(-1)[idx] = rng.integers(0, 16, n_dark)
    buf = torch.zeros(h, w + 37, dtype=torch.uint8)
    buf[:, :w] = torch.from_numpy(y)
    got = lnr().meter(ctx, buf.cuda()[:, :w])
    assert got == oracle.meter(y)
    assert got[1] == n_dark
    for dark, f3, f4 in [(8, 0.01, 0.5), (64, 0.3, 0.3), (256, 0.0, 1.0)]:
        assert lnr().meter(ctx, buf.cuda()[:, :w], dark, f3, f4) == oracle.meter(y, dark, f3, f4)


def test_meter_rejects_bad_thresholds(ctx):
    y = torch.zeros(8, 8, dtype=torch.uint8, device="cuda")
    for dark, f3, f4 in [(-1, 0.05, 0.2), (257, 0.05, 0.2), (16, 0.3, 0.2), (16, -0.1, 0.2),
                         (16, 0.05, 1.5), (16, float("nan"), 0.2)]:
        with pytest.raises(lnr().LnrError):
            lnr().meter(ctx, y, dark, f3, f4)


def test_register_deterministic(ctx):
    st = synth.make_config_pair("c1", 15)
    p = lnr().Params(radius0=8)
    a = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    b = lnr().register_pair(ctx, to_gpu_frame(st.frames[0]), to_gpu_frame(st.frames[1]), p)
    _sync()
    for k in ("disp", "flags", "H", "flow", "image", "yeq_warped"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def test_stack_and_merge_three_frames(ctx):
    """A scaled-down 3-frame bracketed stack (ratios 1/4/16): register_stack
    picks the shortest exposure; each registration matches the oracle, and the
    merge is checked as in the 5 MP test. (Exposure fusion divides by weight
    sums as small as 1e-12: two merges of inputs that differ by float rounding
    differ by up to 1e-2 on these stacks, so the merges are compared on
    identical inputs, the oracle's registered planes.)"""
    st = synth.make_config_pair("c3", 2, scale=0.2)
    frames = st.frames[::-1]                # reference (shortest) last: index 2
    p, op = params_pair(radius0=16, min_level_dim=64)
    g = [to_gpu_frame(f) for f in frames]
    regs, ref = lnr().register_stack(ctx, g, p)
    out = lnr().merge(ctx, g, ref, regs, p)
    _sync()
    assert ref == 2
    j, regs_o = 0, []
    for k, f in enumerate(frames):
        if k != ref:
            regs_o.append(oracle.register_pair(frames[ref], f, op))
            registration_parity(regs[j], regs_o[-1])
            j += 1
    _check_full_merge(ctx, frames, ref, regs, regs_o, out, p, op)


def test_stack_reference_without_exposures(ctx):
    """Exposures unknown (all 0): register_stack takes the darkest frame (the
    oracle's pick, lowest mean luma) as the reference, and registers the
    others to it as the oracle does."""
    st = synth.make_config_pair("c3", 4, scale=0.2)
    frames = st.frames[::-1]                # darkest last: index 2
    p, op = params_pair(radius0=16, min_level_dim=64)
    g = [lnr().Frame.from_numpy(f.y, f.u, f.v, 0.0) for f in frames]
    regs, ref = lnr().register_stack(ctx, g, p)
    _sync()
    want = oracle.pick_reference([0.0] * 3, [f.y for f in frames])
    print(f"reference {ref}, oracle {want}", flush=True)
    assert ref == want == 2
    j = 0
    for k, f in enumerate(frames):
        if k != ref:
            registration_parity(regs[j], oracle.register_pair(frames[ref], f, op))
            j += 1


def test_stack_and_merge_three_frames_full_size(ctx):
    """The 12 MP 3-frame stack at its full size (4000x3000, ratios 1/4/16,
    rotation up to 3 degrees, shifts +-12, 5 % saturated discs): both
    registrations against the oracle's, and the merge checked as in the 5 MP
    test."""
    st = synth.make_config_pair("c3", 3)
    frames = st.frames
    p, op = params_pair(radius0=16)
    g = [to_gpu_frame(f) for f in frames]
    regs, ref = lnr().register_stack(ctx, g, p)
    out = lnr().merge(ctx, g, ref, regs, p)
    _sync()
    assert ref == 0
    j, regs_o = 0, []
    for k, f in enumerate(frames):
        if k != ref:
            regs_o.append(oracle.register_pair(frames[ref], f, op))
            registration_parity(regs[j], regs_o[-1])
            j += 1
    _check_full_merge(ctx, frames, ref, regs, regs_o, out, p, op)


def test_register_rejects_bad_arguments(ctx):
    st = synth.make_config_pair("c1", 16)
    a = to_gpu_frame(st.frames[0])
    small = lnr().Frame.from_numpy(st.frames[0].y[:100, :100])
    with pytest.raises(lnr().LnrError) as e:
        lnr().register_pair(ctx, a, small, lnr().Params(radius0=8))
    assert e.value.status == -1
    with pytest.raises(lnr().LnrError) as e:
        lnr().register_pair(ctx, a, a, lnr().Params(radius0=40))
    assert e.value.status == -2
    tiny = lnr().Frame.from_numpy(st.frames[0].y[:20, :20])
    with pytest.raises(lnr().LnrError) as e:
        lnr().register_pair(ctx, tiny, tiny, lnr().Params())
    assert e.value.status == -3
    # one pixel past the largest supported side
    wide = lnr().Frame.from_numpy(np.zeros((64, 6145), np.uint8))
    with pytest.raises(lnr().LnrError) as e:
        lnr().register_pair(ctx, wide, wide, lnr().Params(radius0=8))
    assert e.value.status == -2


@pytest.mark.parametrize("fmt,w,h", [("i420", 2592, 1944), ("i420", 330, 250), ("y8", 331, 251),
                                     ("nv12", 642, 482)])
def test_frame_rgb_vs_oracle(ctx, fmt, w, h):
    """The merge's conversion of the unwarped reference (k_frame_rgb4, four
    pixels per thread with a scalar tail) against the oracle's BT.601
    conversion, and yeq / 255, including ragged widths and a padded NV12
    chroma row."""
    L = lnr()
    rng = np.random.default_rng(w + h)
    y = rng.integers(0, 256, (h, w), np.uint8)
    yeq = rng.integers(0, 256, (h, w), np.uint8)
    if fmt == "y8":
        f = L.Frame.from_numpy(y)
        want = oracle.frame_to_rgb(y)
    else:
        u = rng.integers(0, 256, (h // 2, w // 2), np.uint8)
        v = rng.integers(0, 256, (h // 2, w // 2), np.uint8)
        want = oracle.frame_to_rgb(y, u, v)
        if fmt == "i420":
            f = L.Frame.from_numpy(y, u, v)
        else:
            uv = torch.zeros(h // 2, w + 64, dtype=torch.uint8)
            uv[:, 0:w:2] = torch.from_numpy(u)
            uv[:, 1:w:2] = torch.from_numpy(v)
            f = L.Frame.nv12_from_numpy(y, np.zeros((1, 1), np.uint8))
            f.u = uv.cuda()[:, :w]
    print(f"frame_rgb {fmt} {w}x{h}", flush=True)
    img, yo = L.stage_frame_rgb(ctx, f, _t(yeq))
    _sync()
    assert img.shape == want.shape
    assert_close(img.cpu().numpy(), want, 1.0, what=f"{fmt} rgb")
    assert_close(yo.cpu().numpy(), yeq / 255.0, 1.0, what="yeq / 255")
