"""Training pipeline of the learned displacement proposal (an extension beyond
the paper; the network narrows the Sec. 2.2 search).

Labels come from the method itself: the exhaustive level-0 search of
register_pair (plain mode) on synthetic pairs gives each valid tile's
displacement; the network input is the tile pair (equalised reference and the
level-0 source warped by H^1). Every step runs in the library's kernels
(lnr_proposal_inputs / lnr_proposal_train_step); torch only holds the tensors.

    python -m paper_1504_01441_amd.proposal --pairs 42    # -> proposal_weights.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

from . import (Context, Frame, Params, Registration, register_pair, proposal_inputs,
               proposal_set, proposal_get, proposal_forward, proposal_train_step, LNR_I420,
               LNR_Y8)

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "proposal_weights.npz")


def collect(ctx: Context, frames_pairs, params: Params | None = None):
    """(x [n, 4, 16, 16] bf16 bits as int16, labels [n, 2] int32) over the valid
    level-0 tiles of the given (ref, src) synth frame pairs."""
    p = params or Params()
    xs, ls = [], []
    for f0, f1 in frames_pairs:
        ref = Frame.from_numpy(f0.y, f0.u, f0.v, f0.exposure)
        src = Frame.from_numpy(f1.y, f1.u, f1.v, f1.exposure)
        fmt = LNR_I420 if f0.u is not None else LNR_Y8
        reg = Registration.alloc(f0.width, f0.height, fmt, p)
        register_pair(ctx, ref, src, p, out=reg)
        x = proposal_inputs(ctx, reg.yeq_ref, reg.warped0)
        n0 = reg.tile_off[1]
        ok = (reg.flags[:n0] & 2) != 0
        xs.append(x[ok])
        ls.append(reg.disp[:n0][ok])
    return torch.cat(xs), torch.cat(ls)


def _dihedral(x: torch.Tensor, lab: torch.Tensor, k: int):
    """One of the 8 flips / transposes of a batch of tile pairs, with the
    displacement labels mapped alike (a flip in x negates dx, ...)."""
    lab = lab.clone()
    if k & 1:
        x = x.flip(-1)
        lab[:, 0] = -lab[:, 0]
    if k & 2:
        x = x.flip(-2)
        lab[:, 1] = -lab[:, 1]
    if k & 4:
        x = x.transpose(-1, -2)
        lab = lab[:, [1, 0]]
    return x.contiguous(), lab.contiguous()


def train(ctx: Context, x: torch.Tensor, labels: torch.Tensor, epochs: int = 10,
          batch: int = 256, lr: float = 3e-3, wd: float = 1e-4, seed: int = 0,
          init: torch.Tensor | None = None, augment: bool = True, log=None,
          start_step: int = 0, stop_step: int | None = None):
    """AdamW training on the GPU (cosine learning-rate decay; with `augment`,
    each batch is one of the 8 flips / transposes of its tiles); returns the
    per-epoch mean loss.

    start_step / stop_step run only the global steps [start_step, stop_step)
    of this schedule: the data order, flips and learning rates are those of
    the whole run (replayed from the seed), so a run stopped at step k,
    checkpointed (proposal_checkpoint_save with counter k) and resumed with
    start_step = k after proposal_checkpoint_load ends with the same network
    bit for bit. With start_step > 0 the context must already hold the
    checkpoint (init is not applied)."""
    if start_step == 0:
        if init is None:
            from synth import proposal_params  # seeded initial parameters
            init = torch.from_numpy(proposal_params(seed))
        proposal_set(ctx, init.cuda())
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = x.shape[0]
    steps = epochs * ((n + batch - 1) // batch)
    k = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot = torch.zeros((), dtype=torch.float64, device="cuda")
        for i in range(0, n, batch):
            flip = int(torch.randint(8, (1,), generator=g)) if augment else 0
            if k < start_step or (stop_step is not None and k >= stop_step):
                k += 1
                continue
            idx = perm[i:i + batch]
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * k / max(steps, 1)))
            xb, lb = x[idx], labels[idx]
            if augment:
                xb, lb = _dihedral(xb, lb, flip)
            loss, _ = proposal_train_step(ctx, xb, lb, cur, wd)
            tot += loss.double().sum()
            k += 1
        hist.append(float(tot) / n)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def calibrate(ctx: Context, x: torch.Tensor, labels: torch.Tensor, window: int = 2,
              radius0: int = 16, budget: float = 0.005):
    """Confidence threshold conf_min for held-out tiles (x, labels): the most
    confident tiles are searched in the +-window box around the rounded,
    clamped prediction, as many as possible while the tiles whose exhaustive
    argmin falls outside their box stay within `budget` of all tiles (each
    such tile is a disagreement with the exhaustive search). Returns
    (conf_min, fraction of tiles searched in the window)."""
    o = proposal_forward(ctx, x).double().cpu().numpy()
    lab = labels.cpu().numpy()
    c = np.clip(np.floor(8.0 * o[:, :2] + 0.5), -(radius0 - window), radius0 - window)
    inside = np.all(np.abs(c - lab) <= window, axis=1)
    calibrate.inside_fraction = float(inside.mean())  # the most any threshold can window
    order = np.argsort(-o[:, 2], kind="stable")   # most confident first
    misses = np.cumsum(~inside[order])
    good = np.nonzero(misses <= budget * len(order))[0]
    if len(good) == 0:
        return 1.0 - 1e-9, 0.0
    k = int(good.max())
    # threshold halfway (in logit) to the next tile so that tile k is included
    z = o[order[k], 2] if k + 1 == len(order) else 0.5 * (o[order[k], 2] + o[order[k + 1], 2])
    conf = 1.0 / (1.0 + np.exp(-z))
    return float(min(max(conf, 1e-6), 1.0 - 1e-9)), (k + 1) / len(order)


def load(path: str = DEFAULT_WEIGHTS):
    """(parameters float32 [PROPOSAL_PARAMS], conf_min) of a saved network."""
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), float(z["conf_min"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=42)
    ap.add_argument("--scale", type=float, default=None, help="pair size factor (1 = 5 MP)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed0", type=int, default=100)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--budget", type=float, default=0.005,
                    help="held-out tiles whose argmin may fall outside their window")
    ap.add_argument("--lr", type=float, default=3e-3)
    args = ap.parse_args()
    import concurrent.futures as cf
    t0 = time.time()
    seeds = list(range(args.seed0, args.seed0 + args.pairs))
    # the synthetic pairs are generated on the host before anything touches
    # the GPU (worker processes are forked from a process without GPU state)
    with cf.ProcessPoolExecutor(args.workers) as ex:
        stacks = []
        for st in ex.map(_gen, [(s, args.scale) for s in seeds]):
            stacks.append(st)
            print(f"[train] generated pair {len(stacks)}/{len(seeds)} ({time.time() - t0:.0f} s)",
                  flush=True)
    ctx = Context(0)
    xs, ls = [], []
    for st in stacks:
        x, l = collect(ctx, [tuple(st.frames)])
        xs.append(x)
        ls.append(l)
    nh = max(1, args.pairs // 8)  # held-out pairs for the confidence threshold
    x, lab = torch.cat(xs[:-nh]), torch.cat(ls[:-nh])
    xh, lh = torch.cat(xs[-nh:]), torch.cat(ls[-nh:])
    print(f"[train] {x.shape[0]} labelled tiles, {xh.shape[0]} held out", flush=True)
    t1 = time.time()
    train(ctx, x, lab, epochs=args.epochs, lr=args.lr,
          log=lambda m: print("[train] " + m, flush=True))
    torch.cuda.synchronize()
    print(f"[train] {args.epochs} epochs in {time.time() - t1:.1f} s", flush=True)
    conf, frac = calibrate(ctx, xh, lh, budget=args.budget)
    print(f"[train] conf_min {conf:.6f}: {100 * frac:.1f} % of held-out tiles confident; "
          f"{100 * calibrate.inside_fraction:.1f} % have their argmin in the window",
          flush=True)
    np.savez(args.out, params=proposal_get(ctx).cpu().numpy(), conf_min=np.float64(conf))
    print(f"[train] saved {args.out}", flush=True)


def _gen(a):
    import synth
    seed, scale = a
    return synth.make_config_pair("c2", seed, scale=scale)


if __name__ == "__main__":
    sys.exit(main())
