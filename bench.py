#!/usr/bin/env python3
"""Benchmark: registered MPix/s on the 5 MP pair (2592x1944 I420, exposure
ratio 8, sensor noise sigma 2 DN, 10% mover tiles, search radius 16).

A step is one pass of the whole path on one synthetic pair that is already
resident in HBM: register_pair (equalisation, pyramid, five matching levels
with weeding and homography fits, level-0 search, propagation, backward
warp) followed by the deghosted merge. `value` = W*H / step time.

Besides the JSON line's throughput, the run
  * times every kernel with HIP events on its launch stream over a second,
    traced pass of the same K steps (the library's lnr_trace_* calls), and
    reports the kernel with the largest time per step against its roofline
    (`roofline`; every modelled kernel in `rooflines`);
  * runs the CPU oracle on the same pair on every host core (one pair per
    process, started before the GPU is touched): the aggregate rate is
    `cpu_baseline`, and the oracle's tiles give the % of tiles equal to it;
  * reports the mean end-point error of the final mapping against the
    generator's ground truth, for the plain and the learned method.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       [--only-step] [--dt-shape a,b,c,d,e]
(--only-step: the timed and traced steps only, for profiler runs; --dt-shape:
pin the propagation kernel shape instead of autotuning it.)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 lanes x 2.4 GHz, 1 op/lane/clk
# one v_dot4_u32_u8 lane-instruction forms four byte products
DOT4_PEAK_TPS = 4 * INT_PEAK_TOPS
MAX_CPU_WORKERS = 16           # the host share of one GPU


def search_products(flags, tile_off, levels, radius0, radius_coarse, patch_r):
    """Pixel-candidate products of the exhaustive search of one pair, per
    level: cornered tiles x (2R + 1)^2 candidates x (2P + 1)^2 pixels."""
    out = []
    for l in range(levels):
        c = int((flags[tile_off[l]:tile_off[l + 1]] & 1).sum())
        R = radius0 if l == 0 else radius_coarse
        out.append(c * (2 * R + 1) ** 2 * (2 * patch_r + 1) ** 2)
    return out


def mean_epe(H1, flow, gt):
    """Mean distance between the final sample position Hp1(x + F(x)) and the
    generator's ground truth (planted homography and tile shifts), over
    pixels at least one tile from the border."""
    import numpy as np
    h, w = flow.shape[1:]
    B = np.array([[w, 0, w - 1], [0, w, h - 1], [0, 0, 2]], np.float64)
    Cm = np.array([[2, 0, -(w - 1)], [0, 2, -(h - 1)], [0, 0, w]], np.float64)
    Hp = B @ (H1.reshape(3, 3) @ Cm)
    ys, xs = np.mgrid[32:h - 32, 32:w - 32].astype(np.float64)
    X = xs + flow[0, 32:h - 32, 32:w - 32]
    Y = ys + flow[1, 32:h - 32, 32:w - 32]
    den = Hp[2, 0] * X + Hp[2, 1] * Y + Hp[2, 2]
    mx = (Hp[0, 0] * X + Hp[0, 1] * Y + Hp[0, 2]) / den
    my = (Hp[1, 0] * X + Hp[1, 1] * Y + Hp[1, 2]) / den
    gx, gy = gt
    return float(np.mean(np.hypot(mx - gx[32:h - 32, 32:w - 32], my - gy[32:h - 32, 32:w - 32])))


def _oracle_job(job):
    """One oracle registration + merge of the pair (runs in a child process)."""
    f0, f1, radius0 = job
    import oracle
    op = oracle.params(radius0=radius0)
    t0 = time.time()
    o = oracle.register_pair(f0, f1, op)
    ref_rgb = oracle.frame_to_rgb(f0.y, f0.u, f0.v)
    oracle.merge([ref_rgb, o["rgb"]], [o["yeq_ref"] / 255.0, o["yeq_warped"]], 0, op)
    return t0, time.time(), o["flags"], o["dx"], o["dy"]


def cpu_baseline(f0, f1, radius0):
    """The oracle on every host core: one copy of the pair per process, all
    started together; rate = copies x pixels / (last end - first start).
    Runs before the GPU is touched (children are spawned, not forked)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, MAX_CPU_WORKERS))
    with cf.ProcessPoolExecutor(cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(abs, range(cores)))        # start the workers first
        res = list(ex.map(_oracle_job, [(f0, f1, radius0)] * cores))
    t0 = min(r[0] for r in res)
    t1 = max(r[1] for r in res)
    mpix = f0.width * f0.height / 1e6
    return {"value": round(cores * mpix / (t1 - t0), 4), "unit": "MPix/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} copies of the full {f0.width}x{f0.height} pair (registration + "
                      f"merge), one per process on {cores} cores, {t1 - t0:.1f} s wall; "
                      f"single copy {min(r[1] - r[0] for r in res):.1f} s"}, res[0][2:]


def kernel_key(name):
    """Trace names are the launched expressions, e.g. "(k_dt_row<SEG, NT, true>)":
    return (base name, last template flag)."""
    n = name.strip("()")
    return n.split("<")[0], n.endswith("true>")


def algo_bytes_per_step(W, H, fmt_i420, n, ch, reg_sizes, blend_levels, launches):
    """Algorithmic HBM bytes of one whole-path step, per kernel base name: the
    bytes each launch must move at least (every input read once, every output
    written once), summed over that kernel's launches in the step.

    launches: {trace name: launches per step}. Only bandwidth-type kernels are
    modelled; the search is priced in pixel-candidate operations instead.
    """
    N = W * H
    chroma = 0.5 if fmt_i420 else 0.0
    # registration pyramid levels (equalised luma, u8)
    reg_px = [reg_sizes.level_w[i] * reg_sizes.level_h[i] for i in range(reg_sizes.levels)]
    # merge (Burt-Adelson) pyramid levels: sizes halve with rounding up
    mw, mh, mpx = W, H, []
    for _ in range(blend_levels):
        mpx.append(mw * mh)
        mw, mh = (mw + 1) // 2, (mh + 1) // 2
    out = {}

    def add(k, v):
        out[k] = out.get(k, 0) + v

    for name, cnt in launches.items():
        base, flag = kernel_key(name)
        if base == "k_hist":            # read both frames' luma
            add(base, 2 * N)
        elif base == "k_lut_pyr":       # read luma; write every pyramid level of both frames,
            # level 0 again into the outputs (yeq_ref, yeq_src), and the
            # reference's level 0 column-major for the propagation
            add(base, 2 * N + 2 * sum(reg_px) + 2 * N + N)
        elif base == "k_dt_row":        # first pass: guide in, 3 maps out; else 3 maps in/out
            add(base, cnt * (13 * N if flag else 25 * N))
        elif base == "k_dt_col":        # 3 maps + guide in; 3 maps (last: F and N~) out
            add(base, cnt * 25 * N)
        elif base == "k_bwarp":         # F, Y, UV, Y_eq in; RGB + warped Y_eq out
            add(base, cnt * (8 + 1 + chroma + 1 + 4 * ch + 4) * N)
        elif base == "k_frame_rgb4":    # reference YUV in, RGB out; equalised luma u8 in, f32 out
            add(base, cnt * (1 + chroma + 4 * ch + 1 + 4) * N)
        elif base == "k_ssim":          # two luma maps in, SSIM out
            add(base, cnt * 12 * N)
        elif base == "k_weights":       # all frames' planes + SSIM in, weights out
            add(base, cnt * (n * ch * 4 + (n - 1) * 4 + n * 4) * N)
        elif base == "k_reduce":        # every weight/image plane, level l-1 in, level l out
            add(base, sum(n * (ch + 1) * 4 * (mpx[l - 1] + mpx[l]) for l in range(1, blend_levels)))
        elif base == "k_blend":         # weights, images, coarse images, coarse result in; result out
            tot = 0
            for l in range(blend_levels):
                tot += (n * 4 + n * ch * 4 + ch * 4) * mpx[l]
                if l + 1 < blend_levels:
                    tot += (n * ch * 4 + ch * 4) * mpx[l + 1]
            add(base, tot)
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it has none or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_c2_5mp_pair.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel:
            src = os.path.join(ROOT, f[3])
            if not os.path.exists(src):
                return None
            h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            return int(f[2]) if h == f[4] else None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c4", "c5", "sweep", "flow-widths"],
                    help="c2: the 5 MP pair (default); c4: 64 uneven pairs in one batched call; "
                         "c5: 16 5 MP pairs in one batched call, learned proposal vs plain; "
                         "sweep: registration time from VGA to 12 MP; flow-widths: the "
                         "propagation passes at height 1944 and widths 512..4096")
    ap.add_argument("--pairs", type=int, default=64, help="pairs of the c4 batch")
    ap.add_argument("--only-step", action="store_true",
                    help="time and trace the steps only (no learned step, irradiance map, "
                         "search-only pass, metering or oracle): for profiler runs")
    ap.add_argument("--dt-shape", default=None,
                    help="pin the propagation kernel shape (five integers, as reported in "
                         "autotuned_dt_shape) instead of autotuning it")
    ap.add_argument("--calib-copy", action="store_true",
                    help="one 256 MiB device-to-device copy before the steps (the reference "
                         "transfer for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: pairs are independent units of "
              "work, so more GPUs would each take a share of the pairs.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return batch_main(args)
    if args.workload == "c5":
        return learned_batch_main(args)
    if args.workload == "sweep":
        return sweep_main(args)
    if args.workload == "flow-widths":
        return flow_widths_main(args)

    import numpy as np
    import torch

    import paper_1504_01441_amd as lnr
    import synth

    t_gen = time.time()
    st = synth.make_config_pair("c2", args.seed)
    f0, f1 = st.frames
    W, H = f0.width, f0.height
    print(f"[bench] generated 2592x1944 pair in {time.time() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    cpu = None
    if not args.no_cpu_baseline and not args.only_step:
        t_cpu = time.time()
        cpu = cpu_baseline(f0, f1, st.meta["radius0"])
        print(f"[bench] oracle on {cpu[0]['cores']} cores in {time.time() - t_cpu:.1f}s",
              file=sys.stderr, flush=True)
    ctx = lnr.Context(0)
    p = lnr.Params(radius0=st.meta["radius0"])
    ref = lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
    src = lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
    reg = lnr.Registration.alloc(W, H, lnr.LNR_I420, p)
    hdr = torch.empty(3, H, W, dtype=torch.float32, device="cuda")

    # the library's autotuners pick the propagation kernel shape and the
    # search's workgroup shape per level for this size
    if args.dt_shape:
        dt_shape = tuple(int(v) for v in args.dt_shape.split(","))
        lnr.set_flow_shape(ctx, W, H, dt_shape)
    else:
        dt_shape = lnr.autotune_flow(ctx, W, H, p)
    search_split = lnr.autotune_search(ctx, W, H, p)

    def step():
        lnr.register_pair(ctx, ref, src, p, out=reg)
        lnr.merge(ctx, [ref, src], 0, [reg], p, out=hdr)

    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole-path steps, untraced
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    mpix = W * H / 1e6
    value = mpix / (ms_step / 1e3)

    # registration alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lnr.register_pair(ctx, ref, src, p, out=reg)
    torch.cuda.synchronize()
    ms_reg = (time.perf_counter() - t0) / args.steps * 1e3

    # traced pass: per-kernel HIP-event durations on the launch stream
    ctx.trace(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tr = ctx.trace_read()
    ctx.trace(False)
    per_step = {k: (c / args.steps, ms / args.steps) for k, (c, ms) in tr.items()}
    kernels = sorted(per_step.items(), key=lambda kv: -kv[1][1])
    print("[bench] per-step kernel time (ms): " +
          ", ".join(f"{k} {v[1]:.3f} ({v[0]:.0f}x)" for k, v in kernels), file=sys.stderr,
          flush=True)
    sizes = lnr.query_sizes(W, H, lnr.LNR_I420, p)
    launches = {k: v[0] for k, v in per_step.items()}
    model = algo_bytes_per_step(W, H, True, 2, 3, sizes, sizes.blend_levels, launches)
    by_base = {}
    for name, (cnt, ms) in per_step.items():
        base, _ = kernel_key(name)
        c, t = by_base.get(base, (0.0, 0.0))
        by_base[base] = (c + cnt, t + ms)
    hbm = {}
    for base, (cnt, ms) in by_base.items():
        if base in model:
            gbs = model[base] / (ms / 1e3) / 1e9
            hbm[base] = {"ms": round(ms, 4), "launches": round(cnt, 2),
                         "algo_bytes": int(model[base]), "gbs": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # the search is priced in pixel-candidate products (dot4 peak) per level
    torch.cuda.synchronize()
    flags_all = reg.flags.cpu().numpy()
    prods = search_products(flags_all, reg.tile_off, reg.levels, p.radius0, p.radius_coarse,
                            p.patch_r)
    search_ops = prods[0]
    rooflines = {}
    for base, h in hbm.items():
        cnt = by_base[base][0]
        rooflines[base] = {"kernel": base, "bound": "hbm", "achieved": h["gbs"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": h["frac"],
                           "traffic": measured_traffic(base),
                           "avg_launch_us": round(by_base[base][1] / cnt * 1e3, 2),
                           "algo_bytes_per_launch": int(h["algo_bytes"] / cnt),
                           "ms_per_step": h["ms"], "launches_per_step": round(cnt, 2)}
    if "k_search" in by_base:
        cnt, ms = by_base["k_search"]
        ach = sum(prods) / (ms / 1e3) / 1e12
        rooflines["k_search"] = {
            "kernel": "k_search", "bound": "alu", "achieved": round(ach, 2),
            "peak": round(DOT4_PEAK_TPS, 2), "unit": "T pixel-candidate products/s (v_dot4)",
            "frac": round(ach / DOT4_PEAK_TPS, 4), "traffic": measured_traffic("k_search"),
            "avg_launch_us": round(ms / cnt * 1e3, 2),
            "products_per_launch": int(sum(prods) / cnt), "ms_per_step": round(ms, 4),
            "launches_per_step": round(cnt, 2), "products_per_level": prods}
    # the kernel with the largest time per step (all its launches)
    dom = max(by_base.items(), key=lambda kv: kv[1][1])[0] if by_base else None
    if dom in rooflines:
        roof = dict(rooflines[dom])
    else:
        best = max(rooflines.values(), key=lambda r: r["ms_per_step"]) if rooflines else None
        roof = None if best is None else dict(best, dominant_overall=dom)

    gt = st.gt_map(1)
    epe_plain = mean_epe(reg.H[1].cpu().numpy(), reg.flow.cpu().numpy().astype(np.float64), gt)

    # learned proposal: the same step with the level-0 search narrowed by the
    # network trained on the GPU (paper_1504_01441_amd.proposal)
    learned = None
    from paper_1504_01441_amd import proposal as prop
    if os.path.exists(prop.DEFAULT_WEIGHTS) and not args.only_step:
        P_net, conf_min = prop.load()
        lnr.proposal_set(ctx, torch.from_numpy(P_net))
        pq = lnr.Params(radius0=st.meta["radius0"], learned=1, window_r=2, conf_min=conf_min)
        reg_l = lnr.Registration.alloc(W, H, lnr.LNR_I420, pq)

        def step_l():
            lnr.register_pair(ctx, ref, src, pq, out=reg_l)
            lnr.merge(ctx, [ref, src], 0, [reg_l], pq, out=hdr)

        for _ in range(args.warmup):
            step_l()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_l()
        torch.cuda.synchronize()
        ms_l = (time.perf_counter() - t0) / args.steps * 1e3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lnr.register_pair(ctx, ref, src, pq, out=reg_l)
        torch.cuda.synchronize()
        ms_lr = (time.perf_counter() - t0) / args.steps * 1e3
        # per-kernel times of the learned registration (HIP events)
        ctx.trace(True)
        for _ in range(args.steps):
            lnr.register_pair(ctx, ref, src, pq, out=reg_l)
        torch.cuda.synchronize()
        tr_l = ctx.trace_read()
        ctx.trace(False)
        ker_l = sorted(((k, ms / args.steps) for k, (c, ms) in tr_l.items()), key=lambda kv: -kv[1])
        n0 = reg.tile_off[1]
        fl = reg_l.flags.cpu().numpy()[:n0]
        cornered = (fl & 1) != 0
        window = cornered & ((fl & 16) == 0)
        full = (2 * st.meta["radius0"] + 1) ** 2
        cand = int(window.sum()) * 25 + int(cornered.sum() - window.sum()) * full
        learned = {"value": round(mpix / (ms_l / 1e3), 2), "unit": "MPix/s",
                   "ms_per_step": round(ms_l, 4),
                   "registration_only": {"ms": round(ms_lr, 4),
                                         "mpix_s": round(mpix / (ms_lr / 1e3), 2)},
                   "conf_min": round(conf_min, 6),
                   "tiles_in_window_pct": round(100.0 * window.sum() / max(cornered.sum(), 1), 2),
                   "ssd_candidates_vs_plain": round(cand / max(int(cornered.sum()) * full, 1), 4),
                   "mean_epe_px": round(mean_epe(reg_l.H[1].cpu().numpy(),
                                                 reg_l.flow.cpu().numpy().astype(np.float64),
                                                 gt), 4),
                   "registration_kernels_ms": {k: round(v, 4) for k, v in ker_l},
                   "_flags": fl, "_disp": reg_l.disp.cpu().numpy()[:n0]}

    # the paper-literal search frame (Eq. 3 as printed): the same pair
    # registered with every level searching the unwarped source around its
    # prediction and the absolute flow propagated
    literal = None
    if not args.only_step:
        pt = lnr.Params(radius0=st.meta["radius0"], search_frame=1)
        reg_t = lnr.Registration.alloc(W, H, lnr.LNR_I420, pt)
        for _ in range(args.warmup):
            lnr.register_pair(ctx, ref, src, pt, out=reg_t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lnr.register_pair(ctx, ref, src, pt, out=reg_t)
        torch.cuda.synchronize()
        ms_t = (time.perf_counter() - t0) / args.steps * 1e3
        eye = np.eye(3).reshape(9)
        literal = {"registration_only": {"ms": round(ms_t, 4),
                                         "mpix_s": round(mpix / (ms_t / 1e3), 2)},
                   "mean_epe_px": round(mean_epe(eye, reg_t.flow.cpu().numpy().astype(np.float64),
                                                 gt), 4)}

    result = {
        "metric": "registered MPix/s on 5MP pairs, plain vs learned-proposal; % tiles = oracle",
        "value": round(value, 2),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8+f32",
        "data": "synthetic",
        "config": {"workload": "5MP pair 2592x1944 I420, exposure ratio 8, noise sigma 2 DN, "
                               "10% mover tiles, radius 16, plain method; step = register_pair "
                               "+ merge",
                   "width": W, "height": H, "seed": args.seed},
        "registration_only": {"ms": round(ms_reg, 4), "mpix_s": round(mpix / (ms_reg / 1e3), 2)},
        "mean_epe_px": round(epe_plain, 4),
        "autotuned_dt_shape": {"row_seg": dt_shape[0], "row_block": dt_shape[1],
                               "col_rows": dt_shape[2], "col_cols": dt_shape[3],
                               "col_segments": dt_shape[4]},
        "autotuned_search_split_per_level": list(search_split),
        "paper_literal_search": literal,
        "learned_proposal": None if learned is None else
        {k: v for k, v in learned.items() if not k.startswith("_")},
        "roofline": roof,
        "rooflines": rooflines,
        "search_level0": {"pixel_candidate_ops": search_ops,
                          "int_peak_tops": round(INT_PEAK_TOPS, 2)},
        "kernels_ms_per_step": {k: round(v[1], 4) for k, v in kernels},
        "hbm_kernels": hbm,
    }
    if "k_search" in by_base:
        # all five levels' searches; the level-0 share dominates
        result["search_level0"]["ms_all_levels"] = round(by_base["k_search"][1], 4)
    if args.only_step:
        print(json.dumps(result))
        return

    # the irradiance map of the registered pair (the alternative output to
    # the fusion): SSIM of the warped frame plus one pass over both frames
    irr = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
    lnr.register_pair(ctx, ref, src, p, out=reg)
    for _ in range(args.warmup):
        lnr.merge_irradiance(ctx, [ref, src], 0, [reg], p, out=irr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lnr.merge_irradiance(ctx, [ref, src], 0, [reg], p, out=irr)
    torch.cuda.synchronize()
    ms_irr = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.trace(True)
    for _ in range(args.steps):
        lnr.merge_irradiance(ctx, [ref, src], 0, [reg], p, out=irr)
    torch.cuda.synchronize()
    tri = {kernel_key(k)[0]: (c / args.steps, ms / args.steps) for k, (c, ms) in
           ctx.trace_read().items()}
    ctx.trace(False)
    irr_entry = {"ms": round(ms_irr, 4), "mpix_s": round(mpix / (ms_irr / 1e3), 2),
                 "kernels_ms": {k: round(v[1], 4) for k, v in tri.items()}}
    if "k_irradiance" in tri:
        # two frames of three float planes and one SSIM map in, three planes out
        b_irr = W * H * (2 * 3 * 4 + 4 + 3 * 4)
        gbs = b_irr / (tri["k_irradiance"][1] / tri["k_irradiance"][0] / 1e3) / 1e9
        irr_entry["k_irradiance"] = {"algo_bytes": b_irr, "gbs": round(gbs, 1),
                                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    result["irradiance_map"] = irr_entry

    # the level-0 search alone, on the registration's own level-0 inputs (the
    # equalised reference and the Q8-warped source), against the int VALU
    # peak: one v_dot4 lane-instruction forms four byte products, so the
    # cross-term peak is 4 x 39.3 T pixel-candidate products per second
    R0 = st.meta["radius0"]
    yq, wq = reg.yeq_ref.contiguous(), reg.warped0.contiguous()
    for _ in range(args.warmup):
        lnr.stage_search(ctx, yq, wq, R0, p)
    torch.cuda.synchronize()
    ctx.trace(True)
    for _ in range(args.steps):
        lnr.stage_search(ctx, yq, wq, R0, p)
    torch.cuda.synchronize()
    trs = {}
    for k, (c_, ms_) in ctx.trace_read().items():
        b_ = kernel_key(k)[0]
        c0, m0 = trs.get(b_, (0, 0.0))
        trs[b_] = (c0 + c_, m0 + ms_)
    ctx.trace(False)
    if "k_search" in trs:
        c_s, ms_s = trs["k_search"]
        t_l0 = ms_s / c_s / 1e3
        peak_pc = DOT4_PEAK_TPS
        ach = search_ops / t_l0 / 1e12
        result["search_roofline"] = {
            "kernel": "k_search (level 0)", "bound": "alu", "achieved": round(ach, 2),
            "peak": round(peak_pc, 2), "unit": "T pixel-candidate products/s",
            "frac": round(ach / peak_pc, 4), "avg_launch_us": round(t_l0 * 1e6, 2),
            "products_per_launch": search_ops}

    # metering of the second exposure from the first (reference) frame's luma
    for _ in range(args.warmup):
        stops = lnr.meter(ctx, ref.y)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stops = lnr.meter(ctx, ref.y)
    ms_meter = (time.perf_counter() - t0) / args.steps * 1e3
    result["metering"] = {"ms_with_readback": round(ms_meter, 4), "stops": stops[0],
                          "under_exposed": stops[1]}

    if cpu is not None:
        result["cpu_baseline"] = cpu[0]
        oflags, odx, ody = cpu[1]
        T = len(oflags)
        g = {"flags": reg.flags.cpu().numpy()[:T], "disp": reg.disp.cpu().numpy()[:T]}
        same = (g["flags"] == oflags) & (g["disp"][:, 0] == odx) & (g["disp"][:, 1] == ody)
        result["tiles_equal_oracle_pct"] = round(100.0 * same.mean(), 3)
        if learned is not None:
            n0 = len(learned["_flags"])
            sl = ((learned["_flags"] & 3) == (oflags[:n0] & 3)) & \
                 (learned["_disp"][:, 0] == odx[:n0]) & (learned["_disp"][:, 1] == ody[:n0])
            result["learned_proposal"]["tiles_equal_oracle_pct"] = round(100.0 * sl.mean(), 3)
    print(json.dumps(result))


def _batch_pair(seed):
    import synth
    return synth.make_batch_pair(seed)


def batch_main(args):
    """64 pairs of uneven sizes (640x480 .. 4032x3024 I420) registered by one
    lnr_register_batch call (concurrent streams, one cached HIP graph,
    autotuned concurrency) against one lnr_register_pair call per pair."""
    import concurrent.futures as cf
    t0 = time.time()
    seeds = list(range(7000, 7000 + args.pairs))
    # generated on the host before anything touches the GPU
    with cf.ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        stacks = list(ex.map(_batch_pair, seeds))
    print(f"[bench] generated {len(stacks)} pairs in {time.time() - t0:.0f} s", file=sys.stderr,
          flush=True)
    import numpy as np
    import torch
    import paper_1504_01441_amd as lnr
    ctx = lnr.Context(0)
    p = lnr.Params(radius0=16)
    refs, srcs, outs = [], [], []
    for st in stacks:
        f0, f1 = st.frames
        refs.append(lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure))
        srcs.append(lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure))
        outs.append(lnr.Registration.alloc(f0.width, f0.height, lnr.LNR_I420, p))
    mpix = sum(r.width * r.height for r in refs) / 1e6
    t0 = time.time()
    lnr.register_batch(ctx, refs, srcs, p, outs=outs, graph=True, autotune=True)
    torch.cuda.synchronize()
    t_setup = time.time() - t0

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / k * 1e3

    ms_b = timed(lambda: lnr.register_batch(ctx, refs, srcs, p, outs=outs, graph=True), args.steps)
    ms_s = timed(lambda: [lnr.register_pair(ctx, r, s_, p, out=o)
                          for r, s_, o in zip(refs, srcs, outs)], args.steps)
    result = {
        "metric": "registered MPix/s, 64 uneven pairs in one batched call",
        "value": round(mpix / (ms_b / 1e3), 2), "unit": "MPix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8+f32",
        "data": "synthetic",
        "config": {"workload": f"{len(refs)} pairs, sizes uniform over even 640x480 .. "
                               "4032x3024, I420, exposure ratio 2-16, tile shifts +-16, "
                               "radius 16; step = one register_batch call (graph replay)",
                   "total_mpix": round(mpix, 2)},
        "sequential_register_pair": {"ms": round(ms_s, 3),
                                     "mpix_s": round(mpix / (ms_s / 1e3), 2)},
        "first_call_s (autotune + capture)": round(t_setup, 2),
    }
    print(json.dumps(result))


def _sweep_pair(wh):
    import synth
    return synth.make_sweep_pair(wh[0], wh[1], 1)


def sweep_main(args):
    """Registration (and registration + merge) time of one pair at six sizes
    from VGA to 12 MP with the 5 MP pair's recipe, each size autotuned; the
    exponent of time against pixel count (least squares in log-log) says how
    the path scales (below 1: sublinear, fixed per-level costs dominate small
    images)."""
    import concurrent.futures as cf
    import synth
    t0 = time.time()
    sizes = list(synth.SWEEP_SIZES)
    with cf.ProcessPoolExecutor(min(6, os.cpu_count() or 1)) as ex:
        stacks = list(ex.map(_sweep_pair, sizes))
    print(f"[bench] generated {len(stacks)} pairs in {time.time() - t0:.0f} s", file=sys.stderr,
          flush=True)
    import numpy as np
    import torch
    import paper_1504_01441_amd as lnr
    ctx = lnr.Context(0)
    rows = []
    for st in stacks:
        f0, f1 = st.frames
        W, H = f0.width, f0.height
        p = lnr.Params(radius0=st.meta["radius0"])
        ref = lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
        src = lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
        reg = lnr.Registration.alloc(W, H, lnr.LNR_I420, p)
        hdr = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
        lnr.autotune_flow(ctx, W, H, p)
        lnr.autotune_search(ctx, W, H, p)

        def timed(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - a) / args.steps * 1e3

        ms_reg = timed(lambda: lnr.register_pair(ctx, ref, src, p, out=reg))
        ms_all = timed(lambda: (lnr.register_pair(ctx, ref, src, p, out=reg),
                                lnr.merge(ctx, [ref, src], 0, [reg], p, out=hdr)))
        mp = W * H / 1e6
        rows.append({"width": W, "height": H, "mpix": round(mp, 3),
                     "registration_ms": round(ms_reg, 4),
                     "registration_mpix_s": round(mp / (ms_reg / 1e3), 1),
                     "with_merge_ms": round(ms_all, 4),
                     "with_merge_mpix_s": round(mp / (ms_all / 1e3), 1)})
        print(f"[bench] {W}x{H}: registration {ms_reg:.3f} ms, with merge {ms_all:.3f} ms",
              file=sys.stderr, flush=True)
    x = np.log([r["mpix"] for r in rows])
    y = np.log([r["registration_ms"] for r in rows])
    slope = float(np.polyfit(x, y, 1)[0])
    ym = np.log([r["with_merge_ms"] for r in rows])
    slope_m = float(np.polyfit(x, ym, 1)[0])
    result = {
        "metric": "exponent of registration time against pixel count, VGA to 12 MP",
        "value": round(slope, 4), "unit": "d log t / d log N", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rows[-1]["registration_ms"], "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "u8+f32", "data": "synthetic",
        "config": {"workload": "one pair per size, 640x480 .. 4000x3000 I420, the 5 MP pair's "
                               "recipe (ratio 8, noise sigma 2 DN, 10% movers, radius 16), "
                               "seed 1; each size autotuned; ms_per_step is the 12 MP "
                               "registration"},
        "with_merge_exponent": round(slope_m, 4),
        "sizes": rows,
    }
    print(json.dumps(result))


def flow_widths_main(args):
    """The propagation alone (lnr_stage_flow, default kernel shapes) on a
    random guide of height 1944 at widths 512 .. 4096: per-launch times of the
    row and column passes. The column pass keeps a whole column strip in
    registers, so its time steps up once the strips no longer fit the chip in
    one round of resident workgroups."""
    import torch
    import paper_1504_01441_amd as lnr
    ctx = lnr.Context(0)
    p = lnr.Params()
    H = 1944
    rows = []
    for W in (512, 1024, 2048, 2304, 2592, 3072, 4096):
        g = torch.randint(0, 256, (H, W), dtype=torch.uint8,
                          generator=torch.Generator().manual_seed(W)).cuda()
        nt = (W // p.tile) * (H // p.tile)
        cxy = torch.zeros(nt, 2, dtype=torch.int32, device="cuda")
        d = torch.zeros(nt, 2, dtype=torch.int32, device="cuda")
        f = torch.zeros(nt, dtype=torch.uint8, device="cuda")
        for _ in range(args.warmup):
            lnr.stage_flow(ctx, cxy, d, f, g, p)
        torch.cuda.synchronize()
        ctx.trace(True)
        for _ in range(args.steps):
            lnr.stage_flow(ctx, cxy, d, f, g, p)
        torch.cuda.synchronize()
        tr = ctx.trace_read()
        ctx.trace(False)
        per = {}
        for k, (c, ms) in tr.items():
            base, flag = kernel_key(k)
            if base == "k_dt_col":
                key = "k_dt_col_last" if flag else "k_dt_col"
            elif base == "k_dt_row":
                key = "k_dt_row_first" if flag else "k_dt_row"
            else:
                key = base
            per[key] = round(ms / c * 1e3, 2)
        rows.append({"width": W, "height": H, "us_per_launch": per,
                     "column_blocks": (W + 3) // 4})
        print(f"[bench] {W}x{H}: {per}", file=sys.stderr, flush=True)
    result = {"metric": "propagation pass time against image width at height 1944",
              "value": rows[-3]["us_per_launch"].get("k_dt_col"), "unit": "us per column pass "
              "at 2592 wide", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": False, "data": "synthetic",
              "config": {"workload": "lnr_stage_flow on a random 8-bit guide, no matches, "
                                     "the default kernel shapes for each size (columns at "
                                     "height 1944: 4 columns x 128 segments of 16 rows)"},
              "widths": rows}
    print(json.dumps(result))


def _c2_pair(seed):
    import synth
    return synth.make_config_pair("c2", seed)


def learned_batch_main(args):
    """16 5 MP pairs (the 5 MP recipe, seeds 1-16) registered by one
    lnr_register_batch call with the learned proposal, against the same call
    with the plain method on the same pairs: MPix/s of both, the fraction of
    level-0 tiles searched in the +-2 window, and the fraction of level-0 tiles
    whose result equals the plain (exhaustive, oracle-exact) one."""
    import concurrent.futures as cf
    t0 = time.time()
    seeds = list(range(1, 17))
    with cf.ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        stacks = list(ex.map(_c2_pair, seeds))
    print(f"[bench] generated {len(stacks)} 5 MP pairs in {time.time() - t0:.0f} s",
          file=sys.stderr, flush=True)
    import numpy as np
    import torch
    import paper_1504_01441_amd as lnr
    from paper_1504_01441_amd import proposal as prop
    ctx = lnr.Context(0)
    P_net, conf_min = prop.load()
    lnr.proposal_set(ctx, torch.from_numpy(P_net))
    pp = lnr.Params(radius0=16)
    pq = lnr.Params(radius0=16, learned=1, window_r=2, conf_min=conf_min)
    refs, srcs, outs_p, outs_q = [], [], [], []
    for st in stacks:
        f0, f1 = st.frames
        refs.append(lnr.Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure))
        srcs.append(lnr.Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure))
        outs_p.append(lnr.Registration.alloc(f0.width, f0.height, lnr.LNR_I420, pp))
        outs_q.append(lnr.Registration.alloc(f0.width, f0.height, lnr.LNR_I420, pq))
    mpix = sum(r.width * r.height for r in refs) / 1e6
    lnr.register_batch(ctx, refs, srcs, pp, outs=outs_p, graph=True, autotune=True)
    lnr.register_batch(ctx, refs, srcs, pq, outs=outs_q, graph=True, autotune=True)
    torch.cuda.synchronize()

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / k * 1e3

    ms_p = timed(lambda: lnr.register_batch(ctx, refs, srcs, pp, outs=outs_p, graph=True),
                 args.steps)
    ms_q = timed(lambda: lnr.register_batch(ctx, refs, srcs, pq, outs=outs_q, graph=True),
                 args.steps)
    torch.cuda.synchronize()
    tiles = window = cornered = equal = 0
    for op_, oq in zip(outs_p, outs_q):
        n0 = op_.tile_off[1]
        fp, fq = op_.flags.cpu().numpy()[:n0], oq.flags.cpu().numpy()[:n0]
        dp, dq = op_.disp.cpu().numpy()[:n0], oq.disp.cpu().numpy()[:n0]
        c = (fq & 1) != 0
        tiles += n0
        cornered += int(c.sum())
        window += int((c & ((fq & 16) == 0)).sum())
        equal += int(((fp & 3) == (fq & 3)).__and__(np.all(dp == dq, axis=1)).sum())
    result = {
        "metric": "registered MPix/s, 16 5 MP pairs in one batched call, learned proposal",
        "value": round(mpix / (ms_q / 1e3), 2), "unit": "MPix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_q, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8+bf16+f32",
        "data": "synthetic",
        "config": {"workload": "16 pairs 2592x1944 I420 (5 MP recipe, seeds 1-16), radius 16, "
                               "learned proposal (+-2 window, exhaustive fallback); step = one "
                               "register_batch call (graph replay)",
                   "total_mpix": round(mpix, 2), "level0_tiles": tiles},
        "plain_same_pairs": {"ms": round(ms_p, 3), "mpix_s": round(mpix / (ms_p / 1e3), 2)},
        "conf_min": round(conf_min, 6),
        "tiles_in_window_pct": round(100.0 * window / max(cornered, 1), 2),
        "tiles_equal_plain_pct": round(100.0 * equal / max(tiles, 1), 3),
    }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
