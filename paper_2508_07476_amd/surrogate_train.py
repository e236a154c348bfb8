"""Training of the orientation surrogate's weights on the library's own
kernels: every forward and backward pass is st_surrogate_grad (bf16 MFMA
convolutions, float32 accumulation and master weights) and every update is
st_surrogate_adam.  This module only builds the data: labelled phantoms, the
patch set, the held-out evaluation.

The network is the one st_surrogate_infer evaluates (include/st.h): five 3x3x3
convolutions with 32 channels, ReLU and clamped faces, then a 1x1x1 head with
five outputs (fibre vector, FA logit, confidence logit).  The objective
(include/st.h, st_surrogate_grad) is

  mean(1 - (u . t)^2) + mean((sigmoid(h3) - FA_t)^2) + w_c BCE(h4, [angle(u, t) < 2 deg])

over the weighted voxels, u = h[0:3] / |h[0:3]|, t the label's unit vector,
w_c the confidence term's weight (--conf-weight, 0.1 by default).

Data: rod-lattice helical phantoms whose helix range, rod period and noise are
drawn per volume (helix angles of +-[30, 80] degrees across the wall, period
3..8 voxels, noise 0.01..0.2); half hold a whole, strongly curved annulus, half
a piece of a wide wall whose axis lies outside the volume.  Labels are
st_compute's e3 and FA at (sigma, rho) on the same volumes; voxels outside the
mask, degenerate voxels and voxels within the network's receptive radius of a
patch face carry weight 0.  The patch set is a fixed list of `--patches`
origins (32^3 patches holding at least `--min-weight` weighted voxels) visited
in a fresh order every epoch.  Held-out phantoms, drawn from other seeds, give
the reported angle error of st_surrogate_infer against st_compute and the
fallback fraction at the confidence threshold.

Usage (on a GPU machine; the defaults reproduce the shipped weights):
  python -m paper_2508_07476_amd.surrogate_train out.npy [--patches 100000] [--epochs E]
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

IN_SCALE = 4.0 / 65535.0
IN_OFFSET = -2.0
MARGIN = 5  # receptive radius of the network
CHANNELS = 32


def init_blob(rng) -> np.ndarray:
    """He-normal convolution weights, zero biases, small head: the blob layout
    of st_surrogate_infer (in_scale, in_offset, then per layer W[co][ci][27], b[co],
    then the head W[5][32], b[5])."""
    parts = [np.array([IN_SCALE, IN_OFFSET])]
    for layer in range(5):
        cin = 1 if layer == 0 else CHANNELS
        parts.append(rng.normal(scale=math.sqrt(2.0 / (27 * cin)), size=CHANNELS * cin * 27))
        parts.append(np.zeros(CHANNELS))
    parts.append(rng.normal(scale=math.sqrt(1.0 / CHANNELS), size=5 * CHANNELS))
    parts.append(np.zeros(5))
    return np.concatenate(parts).astype(np.float32)


def phantom_spec(helix, rng, shape, seed):
    a_in = float(rng.uniform(30, 80))
    a_out = -float(rng.uniform(30, 80))
    if rng.random() < 0.5:
        a_in, a_out = a_out, a_in
    centre = None
    if seed % 2 == 0:  # a whole, strongly curved annulus inside the volume
        r_out = min(shape[1], shape[2]) / 2 - 2
        r_in = float(rng.uniform(0.15, 0.4)) * r_out
    else:  # a piece of a wide, weakly curved wall: the axis lies outside the volume
        r_in = float(rng.uniform(60.0, 160.0))
        r_out = r_in + float(rng.uniform(60.0, 130.0))
        r_mid, th = 0.5 * (r_in + r_out), float(rng.uniform(0, 2 * np.pi))
        c = [(s - 1) / 2.0 for s in shape]
        centre = (c[0], c[1] - r_mid * np.sin(th), c[2] - r_mid * np.cos(th))
    return helix.PhantomSpec(shape=shape, annuli=(helix.Annulus(r_in, r_out, a_in, a_out),),
                             period=float(rng.uniform(3.0, 8.0)), noise=(float(rng.uniform(0.01, 0.2)),),
                             dtype="u16", seed=int(rng.integers(1 << 30)), with_mask=True, center=centre)


def make_pool(torch, st, helix, n, shape, sigma, rho, seed, dev):
    """n labelled volumes stacked: volume (n, S, S, S) (uint16 bytes held as int16), e3 (3, n, S, S, S),
    FA (n, S, S, S), weight (n, S, S, S) u8 (inside the mask, not degenerate)."""
    rng = np.random.default_rng(seed)
    vols = torch.empty((n,) + shape, dtype=torch.int16, device=dev)  # uint16 bytes
    e3 = torch.empty((3, n) + shape, dtype=torch.float32, device=dev)
    fa = torch.empty((n,) + shape, dtype=torch.float32, device=dev)
    good = torch.empty((n,) + shape, dtype=torch.uint8, device=dev)
    specs = []
    for i in range(n):
        spec = phantom_spec(helix, rng, shape, seed * 1000 + i)
        ph = helix.generate(spec, device=dev)
        lab = st.st_compute(ph["volume"], sigma, rho, mask=ph["mask"], outputs=("e3", "fa", "flags"))
        vols[i] = ph["volume"].view(torch.int16)
        e3[:, i] = lab["e3"]
        fa[i] = lab["fa"]
        good[i] = (lab["flags"] == 0).to(torch.uint8)
        specs.append(spec)
    torch.cuda.synchronize()
    return {"vol": vols, "e3": e3, "fa": fa, "good": good, "specs": specs}


def patch_origins(torch, pool, count, P, min_weight, seed):
    """`count` patch origins (volume, z, y, x) whose weighted interior holds at
    least min_weight voxels, drawn uniformly with a fixed seed."""
    n, S = pool["vol"].shape[0], pool["vol"].shape[1]
    # integral image of the weight: the interior [o + MARGIN, o + P - MARGIN) per axis
    c = torch.nn.functional.pad(pool["good"].to(torch.int32), (1, 0, 1, 0, 1, 0))
    c = c.cumsum(1).cumsum(2).cumsum(3)
    lim = S - P + 1
    a, b = MARGIN, MARGIN + lim
    e, f = P - MARGIN, P - MARGIN + lim
    box = (c[:, e:f, e:f, e:f] - c[:, a:b, e:f, e:f] - c[:, e:f, a:b, e:f] - c[:, e:f, e:f, a:b]
           + c[:, a:b, a:b, e:f] + c[:, a:b, e:f, a:b] + c[:, e:f, a:b, a:b] - c[:, a:b, a:b, a:b])
    box_cpu = box.cpu().numpy()
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        cand = rng.integers(0, [n, lim, lim, lim], size=(4 * count, 4))
        ok = box_cpu[cand[:, 0], cand[:, 1], cand[:, 2], cand[:, 3]] >= min_weight
        out.extend(cand[ok].tolist())
    return np.asarray(out[:count], dtype=np.int64)


class Gatherer:
    """Patch stacks gathered from the pool with one indexing kernel per tensor."""

    def __init__(self, torch, pool, P, batch, dev):
        self.t, self.pool, self.P = torch, pool, P
        S = pool["vol"].shape[1]
        r = torch.arange(P, device=dev)
        self.off = ((r[:, None, None] * S + r[None, :, None]) * S + r[None, None, :]).reshape(1, -1)
        m = torch.zeros((P, P, P), dtype=torch.uint8, device=dev)
        m[MARGIN:P - MARGIN, MARGIN:P - MARGIN, MARGIN:P - MARGIN] = 1
        self.margin = m.reshape(1, -1)
        self.S, self.n = S, pool["vol"].shape[0]
        self.flat = {k: pool[k].reshape(-1) for k in ("vol", "fa", "good")}
        self.e3 = pool["e3"].reshape(3, -1)

    def __call__(self, origins):
        t, P, S = self.t, self.P, self.S
        o = t.as_tensor(origins, device=self.off.device)
        base = ((o[:, 0] * S + o[:, 1]) * S + o[:, 2]) * S + o[:, 3]
        idx = (base[:, None] + self.off).reshape(-1)
        B = o.shape[0]
        shape = (B * P, P, P)
        vol = self.flat["vol"][idx].reshape(shape).view(t.uint16)
        fa = self.flat["fa"][idx].reshape(shape)
        w = (self.flat["good"][idx].reshape(B, -1) * self.margin).reshape(shape)
        e3 = self.e3[:, idx].reshape((3,) + shape)
        return vol, e3, fa, w


def evaluate(torch, st, helix, blob, count, shape, sigma, rho, seed, dev, thresholds=(0.9,)):
    """Angle error of st_surrogate_infer against st_compute (unit vectors up to
    sign) on held-out phantoms, over voxels inside the mask and not degenerate;
    for each threshold the fraction of those voxels below it (the fallback
    fraction) and the error of the rest."""
    rng = np.random.default_rng(seed)
    angs, confs = [], []
    for i in range(count):
        spec = phantom_spec(helix, rng, shape, seed * 1000 + i)
        ph = helix.generate(spec, device=dev)
        lab = st.st_compute(ph["volume"], sigma, rho, mask=ph["mask"], outputs=("e3", "flags"))
        out = st.st_surrogate_infer(ph["volume"], blob, 0.0, sigma, rho, mask=ph["mask"],
                                    outputs=("e3", "confidence"))
        sel = lab["flags"] == 0
        dot = (out["e3"] * lab["e3"]).sum(0).abs().clamp(max=1.0)
        angs.append(torch.rad2deg(torch.acos(dot[sel])).float().cpu())
        confs.append(out["confidence"][sel].float().cpu())
    ang, conf = torch.cat(angs).numpy(), torch.cat(confs).numpy()
    res = {"voxels": int(ang.size), "median_deg": float(np.median(ang)), "p90_deg": float(np.quantile(ang, 0.9)),
           "within_2deg": float((ang < 2.0).mean())}
    for thr in thresholds:
        keep = conf >= thr
        res[f"fallback_{thr}"] = float(1.0 - keep.mean())
        res[f"median_deg_conf_{thr}"] = float(np.median(ang[keep])) if keep.any() else float("nan")
    # reliability: per confidence bin, its share of the voxels and the share of
    # them within 2 degrees (a calibrated head has the second near the bin's value)
    edges = [0.0, 0.3, 0.5, 0.7, 0.8, 0.9, 1.0001]
    res["reliability"] = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (conf >= lo) & (conf < hi)
        res["reliability"].append({"conf": [lo, min(hi, 1.0)], "share": round(float(sel.mean()), 4),
                                   "within_2deg": round(float((ang[sel] < 2.0).mean()), 4) if sel.any() else None})
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--patches", type=int, default=100_000)
    ap.add_argument("--epochs", type=float, default=16.0)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--patch", type=int, default=32)
    ap.add_argument("--volumes", type=int, default=128)
    ap.add_argument("--shape", type=int, default=128)
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--rho", type=float, default=2.0)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--conf-weight", type=float, default=0.1, help="weight of the confidence term")
    ap.add_argument("--min-weight", type=int, default=2000)
    ap.add_argument("--eval-volumes", type=int, default=4)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--init", default=None, help="start from this blob (.npy) instead of a fresh one")
    args = ap.parse_args(argv)

    import torch

    import paper_2508_07476_amd as st
    from phantom import helix

    dev = torch.device("cuda:0")
    t0 = time.time()
    shape = (args.shape,) * 3
    pool = make_pool(torch, st, helix, args.volumes, shape, args.sigma, args.rho, args.seed, dev)
    origins = patch_origins(torch, pool, args.patches, args.patch, args.min_weight, args.seed + 1)
    print(f"pool of {args.volumes} labelled {shape} volumes, {len(origins)} patches in {time.time() - t0:.1f} s",
          flush=True)
    rng = np.random.default_rng(args.seed + 2)
    blob = np.load(args.init, allow_pickle=False).astype(np.float32) if args.init else init_blob(rng)
    params = torch.from_numpy(blob).to(dev)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    grad = torch.empty_like(params)
    stats = torch.empty(8, dtype=torch.float32, device=dev)
    ws = torch.empty(st.st_surrogate_grad_workspace_bytes(args.batch, args.patch), dtype=torch.uint8, device=dev)
    gather = Gatherer(torch, pool, args.patch, args.batch, dev)
    per_epoch = len(origins) // args.batch
    steps = max(1, int(round(args.epochs * per_epoch)))
    log_every = max(1, steps // 40)
    acc = torch.zeros(8, dtype=torch.float64, device=dev)
    since = 0
    order = rng.permutation(len(origins))
    pos = 0
    t1 = time.time()
    for step in range(1, steps + 1):
        if pos + args.batch > len(order):
            order, pos = rng.permutation(len(origins)), 0
        vol, e3, fa, w = gather(origins[order[pos:pos + args.batch]])
        pos += args.batch
        st.st_surrogate_grad(vol, e3, fa, w, params, grad=grad, stats=stats, workspace=ws, conf_weight=args.conf_weight)
        acc += stats.double()
        warm = min(1.0, step / args.warmup)
        lr = args.lr * warm * 0.5 * (1.0 + math.cos(math.pi * step / steps))
        st.st_surrogate_adam(params, grad, m, v, step, lr)
        since += 1
        if step % log_every == 0 or step == steps:
            a = (acc / since).cpu().numpy()
            acc.zero_()
            since = 0
            print(f"step {step}/{steps}: loss {a[3]:.4f} dir {a[0]:.4f} fa {a[1]:.5f} conf {a[2]:.4f} "
                  f"within 2 deg {a[5] / max(a[4], 1):.3f} mean angle {a[6]:.2f} deg "
                  f"lr {lr:.2e} ({time.time() - t1:.0f} s)", flush=True)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    out = params.cpu().numpy().astype(np.float32)
    np.save(args.out, out, allow_pickle=False)
    ev = evaluate(torch, st, helix, params, args.eval_volumes, shape, args.sigma, args.rho, args.seed + 1000, dev)
    meta = {"trainer": "st_surrogate_grad + st_surrogate_adam", "patches": int(len(origins)),
            "epochs": args.epochs, "steps": steps, "batch": args.batch, "patch": args.patch,
            "volumes": args.volumes, "shape": list(shape), "sigma": args.sigma, "rho": args.rho,
            "lr": args.lr, "warmup": args.warmup, "min_weight": args.min_weight, "seed": args.seed,
            "conf_weight": args.conf_weight,
            "in_scale": IN_SCALE, "in_offset": IN_OFFSET, "values": int(out.size),
            "train_seconds": round(train_s, 1), "ms_per_step": round(1e3 * train_s / steps, 3),
            "held_out": {"volumes": args.eval_volumes, "seed": args.seed + 1000, **ev},
            "seconds": round(time.time() - t0, 1)}
    with open(args.out + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
