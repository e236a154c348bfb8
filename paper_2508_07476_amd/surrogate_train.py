"""Offline training of the orientation surrogate's weights (not part of any
inference path: st_surrogate_infer evaluates the network in HIP kernels).

The network is the one st_surrogate_infer evaluates (include/st.h): five 3x3x3
convolutions with 32 channels, ReLU and clamped faces, then a 1x1x1 head with
five outputs (fibre vector, FA logit, confidence logit).  Training uses
PyTorch autograd in float32 on synthetic rod-lattice phantoms whose helix range,
rod period and noise are drawn per volume (helix angles of +-[30, 80] degrees
across the wall, period 3..8 voxels, noise 0.01..0.2); half the volumes hold a
whole, strongly curved annulus, half a piece of a wide wall (radii 60..290)
whose axis lies outside the volume.  Labels are the outputs
of the structure-tensor path, st_compute (sigma, rho as given), on the same
volumes:

  loss = mean(1 - (u . t)^2)                 (sign-invariant direction, u = h[0:3]/|h[0:3]|)
       + mean((sigmoid(h[3]) - FA_t)^2)
       + 0.1 * BCE(h[4], [angle(u, t) < 2 deg])   (confidence: "within 2 degrees")

over masked, non-degenerate voxels at least 5 voxels inside each training patch.
The result is written as the float32 blob the C ABI takes, with a JSON record of
the settings.

Usage (on a GPU machine):  python -m paper_2508_07476_amd.surrogate_train out.npy [--steps N]
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


def build_model(torch):
    nn = torch.nn
    layers = []
    cin = 1
    for _ in range(5):
        layers += [nn.Conv3d(cin, 32, 3, padding=1, padding_mode="replicate"), nn.ReLU()]
        cin = 32
    layers.append(nn.Conv3d(32, 5, 1))
    return nn.Sequential(*layers)


def export_blob(model) -> np.ndarray:
    """Flatten the model into the st_surrogate_infer weights layout."""
    convs = [m for m in model if m.__class__.__name__ == "Conv3d"]
    parts = [np.array([IN_SCALE, IN_OFFSET])]
    for c in convs[:5]:
        w = c.weight.detach().cpu().numpy()  # (co, ci, 3, 3, 3): tap 9 kz + 3 ky + kx
        parts += [w.reshape(w.shape[0], w.shape[1], 27).ravel(), c.bias.detach().cpu().numpy()]
    h = convs[5]
    parts += [h.weight.detach().cpu().numpy().reshape(5, 32).ravel(), h.bias.detach().cpu().numpy()]
    return np.concatenate(parts).astype(np.float32)


def make_pool(torch, st, helix, n, shape, sigma, rho, seed, dev):
    """n labelled volumes: (volume, target e3, target FA, weight mask)."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n):
        a_in = float(rng.uniform(30, 80))
        a_out = -float(rng.uniform(30, 80))
        if rng.random() < 0.5:
            a_in, a_out = a_out, a_in
        centre = None
        if i % 2 == 0:  # a whole, strongly curved annulus inside the volume
            r_out = min(shape[1], shape[2]) / 2 - 2
            r_in = float(rng.uniform(0.15, 0.4)) * r_out
        else:  # a piece of a wide, weakly curved wall: the axis lies outside the volume
            r_in = float(rng.uniform(60.0, 160.0))
            r_out = r_in + float(rng.uniform(60.0, 130.0))
            r_mid, th = 0.5 * (r_in + r_out), float(rng.uniform(0, 2 * np.pi))
            c = [(n - 1) / 2.0 for n in shape]
            centre = (c[0], c[1] - r_mid * np.sin(th), c[2] - r_mid * np.cos(th))
        spec = helix.PhantomSpec(shape=shape, annuli=(helix.Annulus(r_in, r_out, a_in, a_out),),
                                 period=float(rng.uniform(3.0, 8.0)), noise=(float(rng.uniform(0.01, 0.2)),),
                                 dtype="u16", seed=int(rng.integers(1 << 30)), with_mask=True, center=centre)
        ph = helix.generate(spec, device=dev)
        lab = st.st_compute(ph["volume"], sigma, rho, mask=ph["mask"], outputs=("e3", "fa", "flags"))
        good = (lab["flags"] == 0).float()  # inside the mask and not degenerate
        pool.append((ph["volume"], lab["e3"], lab["fa"], good))
    torch.cuda.synchronize()
    return pool


def sample(torch, pool, rng, batch, p):
    xs, ts, fs, ws = [], [], [], []
    for _ in range(batch):
        vol, e3, fa, good = pool[rng.integers(len(pool))]
        nz, ny, nx = vol.shape
        z, y, x = (int(rng.integers(0, s - p + 1)) for s in (nz, ny, nx))
        sl = (slice(z, z + p), slice(y, y + p), slice(x, x + p))
        xs.append(vol[sl].float() * IN_SCALE + IN_OFFSET)
        ts.append(e3[(slice(None),) + sl])
        fs.append(fa[sl])
        w = good[sl].clone()
        w[:MARGIN] = 0; w[-MARGIN:] = 0
        w[:, :MARGIN] = 0; w[:, -MARGIN:] = 0
        w[:, :, :MARGIN] = 0; w[:, :, -MARGIN:] = 0
        ws.append(w)
    return (torch.stack(xs)[:, None], torch.stack(ts), torch.stack(fs), torch.stack(ws))


def losses(torch, h, t, fa_t, w):
    u = h[:, :3]
    u = u / (u.norm(dim=1, keepdim=True) + 1e-12)
    dot = (u * t).sum(1)
    wsum = w.sum().clamp_min(1.0)
    l_dir = ((1 - dot * dot) * w).sum() / wsum
    l_fa = ((torch.sigmoid(h[:, 3]) - fa_t) ** 2 * w).sum() / wsum
    ang = torch.acos(dot.abs().clamp(max=1.0)).detach()
    good = (ang < math.radians(2.0)).float()
    l_conf = (torch.nn.functional.binary_cross_entropy_with_logits(h[:, 4], good, reduction="none") * w).sum() / wsum
    return l_dir, l_fa, l_conf, ang


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--patch", type=int, default=32)
    ap.add_argument("--volumes", type=int, default=24)
    ap.add_argument("--shape", type=int, default=96)
    ap.add_argument("--sigma", type=float, default=1.5)
    ap.add_argument("--rho", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args(argv)

    import torch

    import paper_2508_07476_amd as st
    from phantom import helix

    dev = torch.device("cuda:0")
    torch.manual_seed(args.seed)
    t0 = time.time()
    shape = (args.shape,) * 3
    pool = make_pool(torch, st, helix, args.volumes, shape, args.sigma, args.rho, args.seed, dev)
    print(f"pool of {len(pool)} labelled {shape} volumes in {time.time() - t0:.1f} s", flush=True)
    model = build_model(torch).to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=1e-3)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, args.steps)
    rng = np.random.default_rng(args.seed + 1)
    for step in range(1, args.steps + 1):
        x, t, fa_t, w = sample(torch, pool, rng, args.batch, args.patch)
        h = model(x)
        l_dir, l_fa, l_conf, ang = losses(torch, h, t, fa_t, w)
        loss = l_dir + l_fa + 0.1 * l_conf
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
        if step % 250 == 0 or step == 1:
            m = w > 0
            med = float(torch.quantile(ang[m][:200000], 0.5)) if m.any() else float("nan")
            print(f"step {step}: loss {float(loss.detach()):.4f} dir {float(l_dir):.4f} fa {float(l_fa):.5f} "
                  f"conf {float(l_conf):.4f} median angle {math.degrees(med):.2f} deg "
                  f"({time.time() - t0:.0f} s)", flush=True)
    blob = export_blob(model)
    np.save(args.out, blob, allow_pickle=False)
    meta = {"steps": args.steps, "batch": args.batch, "patch": args.patch, "volumes": args.volumes,
            "shape": shape, "sigma": args.sigma, "rho": args.rho, "seed": args.seed,
            "in_scale": IN_SCALE, "in_offset": IN_OFFSET, "values": int(blob.size),
            "seconds": round(time.time() - t0, 1)}
    with open(args.out + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
