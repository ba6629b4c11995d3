"""Pins of the learned-proposal oracle (oracle/proposal_oracle.c) against
things it does not compute itself: torch's bfloat16 cast, scipy's 2-D
correlation, central finite differences, AdamW's first-step closed form and
brute-force search. The proposal is an extension beyond the paper; the search
it narrows is the paper's Sec. 2.2 search."""
import numpy as np
import pytest
import scipy.signal
import torch

import oracle

NP = oracle.CNN_PARAMS


def _layout():
    """offsets of W1 b1 W2 b2 W3 b3 W4 b4 Wh bh in the flat vector"""
    cin = [oracle.CNN_IN, 32, 32, 32]
    off, o = {}, 0
    for l in range(4):
        off[f"W{l + 1}"] = (o, (32, cin[l], 3, 3))
        o += 32 * cin[l] * 9
        off[f"b{l + 1}"] = (o, (32,))
        o += 32
    off["Wh"] = (o, (3, 512))
    o += 1536
    off["bh"] = (o, (3,))
    o += 3
    assert o == NP
    return off


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(NP)
    for name, (o, shp) in _layout().items():
        fan = int(np.prod(shp[1:])) if len(shp) > 1 else 1
        s = scale * (np.sqrt(2.0 / fan) if name[0] == "W" else 0.05)
        P[o:o + int(np.prod(shp))] = rng.normal(0, s, int(np.prod(shp)))
    return P


def _tensor(P, name):
    o, shp = _layout()[name]
    return P[o:o + int(np.prod(shp))].reshape(shp)


def _conv_scipy(x, W, b, stride):
    """cross-correlation with zero padding 1, via scipy, then the stride"""
    co_n, ci_n = W.shape[:2]
    out = []
    for co in range(co_n):
        acc = np.full((x.shape[1], x.shape[2]), b[co])
        for ci in range(ci_n):
            acc = acc + scipy.signal.correlate2d(x[ci], W[co, ci], mode="same", boundary="fill")
        out.append(acc[::stride, ::stride])
    return np.stack(out)


def _forward_scipy(P, x):
    a = x
    for l, s in zip(range(1, 5), (1, 2, 1, 2)):
        a = np.maximum(_conv_scipy(a, _tensor(P, f"W{l}"), _tensor(P, f"b{l}"), s), 0.0)
    feat = a.transpose(1, 2, 0).reshape(-1)  # f = (y * 4 + x) * 32 + c
    return _tensor(P, "bh") + _tensor(P, "Wh") @ feat


def test_param_count():
    assert oracle.lib().lo_cnn_param_count() == NP == 30467


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-30, 50), [0.0, -0.0, 1.0, 3.0]])
    v = v.astype(np.float32)
    # exact halfway cases: low 16 bits 0x8000 with even and odd kept parts
    halves = np.array([0x3f808000, 0x3f818000, 0xbf808000, 0x40490000 | 0x8000],
                      np.uint32).view(np.float32)
    v = np.concatenate([v, halves])
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.bf16(v.astype(np.float64)), want)


def _bf16_np(v):
    return torch.from_numpy(np.asarray(v, np.float32)).to(torch.bfloat16).double().numpy()


def test_tile_input_brute_force():
    """Channels 0, 1: 2x2 sums of the tile; channels 2, 3: 4x4 sums of the
    64 x 64 window around it, the image padded by repeating its edge (numpy's
    'edge' mode), at interior, corner and edge tiles of a ragged image."""
    rng = np.random.default_rng(4)
    H, W = 100, 130
    ref = rng.integers(0, 256, (H, W), np.uint8)
    wrp = rng.integers(0, 256, (H, W), np.uint8)
    ntx = W // 32
    tiles = [0, 5, ntx - 1, 2 * ntx + 3]   # corner, interior, right edge, bottom-right
    x = oracle.cnn_tile_inputs(ref, wrp, tiles)
    assert x.shape == (4, 4, 16, 16)
    for k, t in enumerate(tiles):
        x0, y0 = (t % ntx) * 32, (t // ntx) * 32
        for c, img in enumerate((ref, wrp)):
            tl = img[y0:y0 + 32, x0:x0 + 32].astype(np.int64)
            s = tl[0::2, 0::2] + tl[1::2, 0::2] + tl[0::2, 1::2] + tl[1::2, 1::2]
            assert np.array_equal(x[k, c], _bf16_np((s - 510) / 512.0)), (t, c)
            pad = np.pad(img.astype(np.int64), 16, mode="edge")
            win = pad[y0:y0 + 64, x0:x0 + 64]        # window origin (x0 - 16, y0 - 16)
            s4 = win.reshape(16, 4, 16, 4).sum(axis=(1, 3))
            assert np.array_equal(x[k, 2 + c], _bf16_np((s4 - 2040) / 2048.0)), (t, c)


def test_tile_input_window_shows_a_shifted_tile():
    """A source that is the reference shifted by (8, -4) px: the source
    window channel equals the reference window channel shifted by (2, -1)
    quarter-resolution pixels where both stay inside the image."""
    rng = np.random.default_rng(9)
    big = rng.integers(0, 256, (200, 200), np.uint8)
    ref = big[40:168, 40:168].copy()
    src = big[40 - 4:168 - 4, 40 + 8:168 + 8].copy()    # src(x, y) = ref(x + 8, y - 4)
    x = oracle.cnn_tile_inputs(ref, src, [5])           # tile (1, 1) of a 4 x 4 grid
    a, b = x[0, 2], x[0, 3]
    assert np.array_equal(b[1:, :-2], a[:-1, 2:])


def test_forward_matches_scipy_correlation():
    P = _params(5)
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (3, oracle.CNN_IN, 16, 16))
    got = oracle.cnn_forward(P, x, rnd=False)
    for s in range(3):
        assert np.allclose(got[s], _forward_scipy(P, x[s]), rtol=1e-12, atol=1e-12)


def test_forward_rounded_close_to_exact():
    P = _params(7)
    x = oracle.bf16(np.random.default_rng(8).uniform(-1, 1, (4, oracle.CNN_IN, 16, 16)))
    a = oracle.cnn_forward(P, x, rnd=True)
    b = oracle.cnn_forward(P, x, rnd=False)
    assert np.all(np.abs(a - b) <= 0.05 * (1 + np.abs(b)))
    assert not np.array_equal(a, b)


def _rd(t):
    """bf16 round to nearest even (torch's cast, pinned above), kept in float64"""
    return t.float().to(torch.bfloat16).double()


def _torch_rounded(P, x, lab):
    """The rounded network written independently with torch's float64
    convolution primitives: weights and post-ReLU activations rounded to
    bf16, biases and the fp32 head unrounded; backward through the ReLUs with
    the gradient rounded where the kernels consume it (dz), then the weight,
    bias and input gradients of each convolution. Returns outputs and the
    flat gradient (same layout as the oracle)."""
    import torch.nn.grad as G
    import torch.nn.functional as F
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64))  # noqa: E731
    n = x.shape[0]
    Ws = [_rd(t(_tensor(P, f"W{l}"))) for l in range(1, 5)]
    bs = [t(_tensor(P, f"b{l}")) for l in range(1, 5)]
    Wh, bh = t(_tensor(P, "Wh")), t(_tensor(P, "bh"))
    strides = (1, 2, 1, 2)
    acts = [t(x)]
    for l in range(4):
        z = F.conv2d(acts[-1], Ws[l], bs[l], stride=strides[l], padding=1)
        acts.append(_rd(torch.clamp(z, min=0.0)))
    feat = acts[4].permute(0, 2, 3, 1).reshape(n, -1)  # f = (y * 4 + x) * 32 + c
    o = feat @ Wh.T + bh
    labt = t(lab.astype(np.float64))
    ex, ey = 8 * o[:, 0] - labt[:, 0], 8 * o[:, 1] - labt[:, 1]
    q = 1 / (1 + torch.exp(-4 * (2.5 - torch.maximum(ex.abs(), ey.abs()))))
    dO = torch.stack([8 * ex.clamp(-1, 1), 8 * ey.clamp(-1, 1), torch.sigmoid(o[:, 2]) - q],
                     1) / n
    grads = {"Wh": dO.T @ feat, "bh": dO.sum(0)}
    da = (dO @ Wh).reshape(n, 4, 4, 32).permute(0, 3, 1, 2)
    for l in range(3, -1, -1):
        dz = _rd(torch.where(acts[l + 1] > 0, da, torch.zeros_like(da)))
        grads[f"W{l + 1}"] = G.conv2d_weight(acts[l], Ws[l].shape, dz, stride=strides[l],
                                             padding=1)
        grads[f"b{l + 1}"] = dz.sum((0, 2, 3))
        if l:
            da = G.conv2d_input(acts[l].shape, Ws[l], dz, stride=strides[l], padding=1)
    g = np.zeros(NP)
    for name, (off, shp) in _layout().items():
        g[off:off + int(np.prod(shp))] = grads[name].numpy().reshape(-1)
    return o.numpy(), g


def test_forward_rounded_matches_torch():
    """The bf16-rounded forward pass against the independent torch version:
    the two sum in different orders (about 1e-16 apart before each rounding),
    so they agree to 1e-12 unless a sum falls on a bf16 rounding boundary."""
    P = _params(17)
    rng = np.random.default_rng(18)
    x = oracle.bf16(rng.uniform(-1, 1, (6, oracle.CNN_IN, 16, 16)))
    lab = rng.integers(-8, 9, (6, 2)).astype(np.int32)
    got = oracle.cnn_forward(P, x, rnd=True)
    want, _ = _torch_rounded(P, x, lab)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)
    # the rounding matters: the exact network differs by far more
    assert np.abs(oracle.cnn_forward(P, x, rnd=False) - want).max() > 1e-4


@pytest.mark.parametrize("seed", [19, 20])
def test_gradient_rounded_matches_torch(seed):
    """The bf16-rounded loss gradient (every parameter) against the
    independent torch version, to 1e-9 of the gradient's largest entry."""
    P = _params(seed)
    rng = np.random.default_rng(seed + 50)
    x = oracle.bf16(rng.uniform(-1, 1, (4, oracle.CNN_IN, 16, 16)))
    lab = rng.integers(-8, 9, (4, 2)).astype(np.int32)
    _, got = oracle.cnn_loss_grad(P, x, lab, rnd=True)
    _, want = _torch_rounded(P, x, lab)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    _, exact = oracle.cnn_loss_grad(P, x, lab, rnd=False)
    assert np.abs(exact - want).max() > 1e-6 * np.abs(want).max()


def _frozen_loss(P, x, lab, q0):
    o = oracle.cnn_forward(P, x, rnd=False)
    ex, ey = 8 * o[:, 0] - lab[:, 0], 8 * o[:, 1] - lab[:, 1]
    hub = lambda e: np.where(np.abs(e) <= 1, 0.5 * e * e, np.abs(e) - 0.5)  # noqa: E731
    z = o[:, 2]
    bce = np.maximum(z, 0) - q0 * z + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(hub(ex) + hub(ey) + bce))


@pytest.mark.parametrize("seed", [11, 12])
def test_gradient_matches_finite_differences(seed):
    """Backward pinned by central differences of the loss with the soft
    confidence target held at its current value (as the gradient defines)."""
    P = _params(seed)
    rng = np.random.default_rng(seed + 100)
    x = rng.uniform(-1, 1, (3, oracle.CNN_IN, 16, 16))
    lab = rng.integers(-6, 7, (3, 2)).astype(np.int32)
    o = oracle.cnn_forward(P, x, rnd=False)
    ex, ey = 8 * o[:, 0] - lab[:, 0], 8 * o[:, 1] - lab[:, 1]
    q0 = 1.0 / (1.0 + np.exp(-4.0 * (2.5 - np.maximum(np.abs(ex), np.abs(ey)))))
    loss, g = oracle.cnn_loss_grad(P, x, lab, rnd=False)
    assert abs(loss - _frozen_loss(P, x, lab, q0)) < 1e-12 * max(1.0, abs(loss))
    idx = []
    for name, (off, shp) in _layout().items():
        n = int(np.prod(shp))
        idx += list(off + rng.choice(n, size=min(n, 6), replace=False))
    eps = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += eps
        Pm[i] -= eps
        fd = (_frozen_loss(Pp, x, lab, q0) - _frozen_loss(Pm, x, lab, q0)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_gradient_rounded_close_to_exact():
    """Sanity bound only: weight gradients sum many terms that largely cancel,
    so the 2^-9 relative rounding of each activation and back-propagated
    gradient shows up enlarged (about 10-20 % here at random init)."""
    P = _params(13)
    rng = np.random.default_rng(14)
    x = oracle.bf16(rng.uniform(-1, 1, (4, oracle.CNN_IN, 16, 16)))
    lab = rng.integers(-8, 9, (4, 2)).astype(np.int32)
    _, ga = oracle.cnn_loss_grad(P, x, lab, rnd=True)
    _, gb = oracle.cnn_loss_grad(P, x, lab, rnd=False)
    assert np.linalg.norm(ga - gb) <= 0.3 * np.linalg.norm(gb)
    assert np.linalg.norm(ga[-1539:] - gb[-1539:]) <= 0.05 * np.linalg.norm(gb[-1539:])


def test_adamw_first_step_and_decay():
    rng = np.random.default_rng(15)
    n = 50
    w0 = rng.normal(0, 1, n)
    g = rng.normal(0, 1, n)
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    oracle.adamw(w, m, v, g, 1, 1e-3, eps=1e-12)
    # bias-corrected first moments are g and g^2: the step is lr * sign(g)
    assert np.allclose(w, w0 - 1e-3 * np.sign(g), rtol=0, atol=1e-12)
    # a second step with the same gradient is again lr * sign(g)
    oracle.adamw(w, m, v, g, 2, 1e-3, eps=1e-12)
    assert np.allclose(w, w0 - 2e-3 * np.sign(g), rtol=0, atol=1e-12)
    # zero gradient from zero moments: only the decoupled decay acts
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    oracle.adamw(w, m, v, np.zeros(n), 1, 1e-2, wd=0.1)
    assert np.allclose(w, w0 * (1 - 1e-3), rtol=1e-15, atol=0)


def _scene(seed, w=160, h=128):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 256, (h + 40, w + 40)).astype(np.float64)
    from scipy.ndimage import gaussian_filter
    img = gaussian_filter(base, 1.2)
    img = (img - img.min()) / (img.max() - img.min()) * 255
    return img


def test_window_search_equals_exhaustive_when_argmin_inside():
    img = _scene(16)
    ref = np.round(img[20:148, 20:180]).astype(np.uint8)
    wimg = np.round(img[23:151, 18:178]).astype(np.uint8)  # true shift (-2, 3)
    p = oracle.params(radius0=8)
    cx, cy, has = oracle.corners(ref, p)
    dx, dy, ssd, valid = oracle.search(ref, wimg, 8, cx, cy, has, p)
    # windows of radius 2 around the exhaustive result +- 1
    rng = np.random.default_rng(17)
    ox = rng.integers(-1, 2, len(cx))
    oy = rng.integers(-1, 2, len(cx))
    wdx, wdy, wssd, wvalid = oracle.search_window(ref, wimg, 2, dx + ox, dy + oy, cx, cy, has, p)
    m = valid.astype(bool)
    assert m.sum() > 5
    assert np.array_equal(wdx[m], dx[m]) and np.array_equal(wdy[m], dy[m])
    assert np.array_equal(wssd[m], ssd[m])
    # centre 0 with the full radius is the plain search
    z = np.zeros(len(cx), np.int32)
    a = oracle.search_window(ref, wimg, 8, z, z, cx, cy, has, p)
    assert all(np.array_equal(u, v) for u, v in zip(a, (dx, dy, ssd, valid)))


def test_window_search_brute_force():
    rng = np.random.default_rng(18)
    ref = rng.integers(0, 256, (64, 64), np.uint8)
    wimg = rng.integers(0, 256, (64, 64), np.uint8)
    p = oracle.params(radius0=4)
    cx = np.array([16, 48, 16, 48], np.int32)
    cy = np.array([16, 16, 48, 48], np.int32)
    has = np.ones(4, np.uint8)
    ccx = np.array([3, -5, 0, 7], np.int32)
    ccy = np.array([-2, 4, 9, -1], np.int32)
    dx, dy, ssd, valid = oracle.search_window(ref, wimg, 2, ccx, ccy, cx, cy, has, p)
    P = p.patch_r
    for t in range(4):
        best = None
        for ddy in range(ccy[t] - 2, ccy[t] + 3):
            for ddx in range(ccx[t] - 2, ccx[t] + 3):
                x, y = cx[t] + ddx, cy[t] + ddy
                if x - P < 0 or x + P > 63 or y - P < 0 or y + P > 63:
                    continue
                a = ref[cy[t] - P:cy[t] + P + 1, cx[t] - P:cx[t] + P + 1].astype(np.int64)
                b = wimg[y - P:y + P + 1, x - P:x + P + 1].astype(np.int64)
                k = (int(((a - b) ** 2).sum()), abs(ddx) + abs(ddy), ddy, ddx)
                best = k if best is None or k < best else best
        if best is None:
            assert valid[t] == 0
        else:
            assert valid[t] == 1 and (ssd[t], dy[t], dx[t]) == (best[0], best[2], best[3])
