"""Shared helpers for the GPU parity tests (GPU output vs the CPU oracle)."""
import numpy as np

# FP32 stages: |gpu - oracle| <= REL * (|oracle| + scale), scale 1 for [0, 1]
# planes and 1 px for flow (the bound the method's FP32 stages are held to).
REL = 1e-4


def lnr():
    import paper_1504_01441_amd as m
    return m


def to_gpu_frame(f):
    return lnr().Frame.from_numpy(f.y, f.u, f.v, f.exposure)


def params_pair(**kw):
    """The same parameter values for the library and the oracle."""
    import oracle
    return lnr().Params(**kw), oracle.params(**kw)


def assert_close(got, want, scale=1.0, rel=REL, mask=None, what=""):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want)
    tol = rel * (np.abs(want) + scale)
    bad = err > tol
    if mask is not None:
        bad &= mask
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(
            f"{what}: {bad.sum()} of {bad.size} values out of tolerance; worst "
            f"{(err / tol)[bad].max():.3g}x tol; first at {idx.tolist()}: got "
            f"{[got[tuple(i)] for i in idx]} want {[want[tuple(i)] for i in idx]}")


def tile_arrays(reg, T):
    """GPU per-tile outputs as numpy, cut to T tiles."""
    c = reg.corner_xy.cpu().numpy()[:T]
    d = reg.disp.cpu().numpy()[:T]
    return dict(corner_x=c[:, 0], corner_y=c[:, 1], dx=d[:, 0], dy=d[:, 1],
                ssd=reg.ssd.cpu().numpy().view(np.uint32)[:T], flags=reg.flags.cpu().numpy()[:T])


def assert_tiles_equal(reg, o):
    T = len(o["flags"])
    g = tile_arrays(reg, T)
    for k in ("flags", "corner_x", "corner_y", "dx", "dy", "ssd"):
        if not np.array_equal(g[k], o[k]):
            bad = np.nonzero(g[k] != o[k])[0]
            raise AssertionError(f"tile {k} differs at {len(bad)} tiles, first {bad[:8].tolist()}: "
                                 f"gpu {g[k][bad[:8]].tolist()} oracle {o[k][bad[:8]].tolist()}")


def registration_parity(reg, o, flow_mask_nmin=1e-30, warped0=True):
    """Everything register_pair produces, against the oracle (warped0: the
    level-0 Q8-warped source, which the unwarped-source search does not
    produce)."""
    assert_tiles_equal(reg, o)
    L = o["levels"]
    counts = reg.counts.cpu().numpy()
    for l in range(L):
        assert counts[l, 0] == o["n_valid"][l], f"level {l}: N differs"
        assert counts[l, 1] == o["n_inliers"][l], f"level {l}: fit count differs"
        if o["n_inliers"][l]:
            assert counts[l, 3] == o["best_iter"][l], f"level {l}: best iteration differs"
    H = reg.H.cpu().numpy().reshape(-1, 3, 3)
    if not np.array_equal(H, o["H"]):
        raise AssertionError(f"H differs (max abs {np.abs(H - o['H']).max():.3g})")
    assert np.array_equal(reg.yeq_ref.cpu().numpy(), o["yeq_ref"]), "Y_eq(ref) differs"
    assert np.array_equal(reg.yeq_src.cpu().numpy(), o["yeq_src"]), "Y_eq(src) differs"
    if warped0:
        assert np.array_equal(reg.warped0.cpu().numpy(), o["warped0"]), "Q8 warp differs"
    nt = o["ntilde"]
    mask = nt > 2 * flow_mask_nmin
    flow = reg.flow.cpu().numpy()
    assert_close(flow[0], o["flow_u"], 1.0, mask=mask, what="flow u")
    assert_close(flow[1], o["flow_v"], 1.0, mask=mask, what="flow v")
    # N~ as every FP32 plane (1e-4 of |N~| + 1), and besides that relative to
    # its own size down to 1e-20 (the float storage between the recursive
    # passes keeps about 1e-4 of that)
    ntg = reg.ntilde.cpu().numpy()
    assert_close(ntg, nt, 1.0, what="N~")
    assert_close(ntg, nt, 0.0, rel=1e-3, mask=nt > 1e-20, what="N~ (relative)")
    assert_close(reg.image.cpu().numpy(), o["rgb"], 1.0, what="warped image")
    assert_close(reg.yeq_warped.cpu().numpy(), o["yeq_warped"], 1.0, what="warped Y_eq")
