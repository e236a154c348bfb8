"""Benchmark of the voxel-wise structure-tensor path on one MI355X.

Default workload: the 2048 x 1024 x 1024 uint16 two-annuli helical phantom
(2^31 voxels, noise 0.02 / 0.1 / 0.2 by z-thirds), sigma = 2, rho = 6
(truncate 4), outputs e3 + FA + HA + IA for every voxel.  One step = one
st_compute call over the whole volume, inputs, outputs and workspace resident
in HBM.  Prints one JSON line (see the "metric" key) with

  * "roofline": the dominant kernel against the roof that binds it, from HIP
    events recorded around every kernel on its launch stream inside the timed
    region; "traffic" comes from committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters (profiles/traffic_<workload>.json) when they belong to the current
    kernel sources, else null;
  * "cpu_baseline": the FP64 CPU oracle on 16 sampled 96^3 blocks (each padded
    by R_sigma + R_rho) of the same volume, one block per worker process, over
    the host cores given to this process (at most 16);
  * "headline512": the 512^3 uint16 phantom with its annulus mask (sigma 1.5,
    rho 4), timed after the main workload (not part of "value").

  python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
                  [--workload two_annuli|headline512] [--batch] [--surrogate]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gvoxels/s (HBM GB/s vs peak) plain vs surrogate at ≤2° fibre-angle error"
HBM_PEAK_GBS = 8000.0
TRUNCATE = 4.0
OUTPUTS = ("e3", "fa", "ha", "ia")

WORKLOADS = {
    "two_annuli": {
        "desc": "2048x1024x1024 uint16 two-annuli helical rod-lattice phantom (r 128-256: +60 to -60 deg, "
                "r 320-480: -60 to +60 deg; noise 0.02/0.1/0.2 by z-thirds), no mask, sigma=2, rho=6, "
                "truncate=4; outputs e3, FA, HA, IA",
        "shape": (2048, 1024, 1024), "sigma": 2.0, "rho": 6.0, "mask": False,
    },
    "headline512": {
        "desc": "512^3 uint16 helical rod-lattice phantom + annulus mask (r 96-224), sigma=1.5, rho=4, "
                "truncate=4; outputs e3, FA, HA, IA",
        "shape": (512, 512, 512), "sigma": 1.5, "rho": 4.0, "mask": True,
    },
}
SHAPE = WORKLOADS["headline512"]["shape"]  # the batch and surrogate workloads crop this phantom


def make_phantom(helix, workload, dev):
    spec = (helix.spec_two_annuli_u16(shape=WORKLOADS[workload]["shape"]) if workload == "two_annuli"
            else helix.spec_headline_u16(shape=WORKLOADS[workload]["shape"]))
    return helix.generate(spec, device=dev)


def alg_bytes_per_voxel(kernel, mask=False):
    """Algorithmic HBM bytes per voxel of one launch of ``kernel``: every input
    read once and every output written once, no halo re-reads (uint16 input,
    float32 intermediates, outputs e3 + FA + HA + IA)."""
    return {"grad_fused": 2 + 24,             # u16 in, 6 products out
            "grad_z": 2 + 8,                  # u16 in, G_z V and D_z V out
            "grad_y": (4 + 8 + 4 + 4) / 2,    # two launches: (1 in, 2 out) and (1 in, 1 out)
            "grad_x_outer": 12 + 24,          # 3 planes in, 6 products out
            "integrate_z": 24 + 24,
            "integrate_y": 24 + 24,
            "integrate_x_eigen": 24 + (1 if mask else 0) + 12 + 12,  # S (+ mask) in; e3, FA, HA, IA out
            }[kernel]


# Algorithmic vector-ALU operations per voxel (one FMA or one float32 op = one
# lane-operation = 2 flop-equivalents): separable filters 2R+1 FMAs per 1-D
# pass (8 gradient passes at sigma, 6 components per integration axis at rho),
# 6 products, about 220 for the eigen-decomposition, FA and angles.
EIGEN_ANGLE_OPS = 220


def alg_ops_per_voxel(kernel, rs, rr):
    return {"grad_fused": 8 * (2 * rs + 1) + 6,
            "integrate_z": 6 * (2 * rr + 1),
            "integrate_y": 6 * (2 * rr + 1),
            "integrate_x_eigen": 6 * (2 * rr + 1) + EIGEN_ANGLE_OPS}.get(kernel)


# vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-operations/s
# (float64 FMA and non-packed float32 issue at the same rate), i.e. 78.6 TFLOP/s
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12

# Sources the plain path is built from: kernels, their launch shapes and the
# host layer that enqueues them.  The HBM byte counts recorded under profiles/
# hold for the sources with this hash.
KERNEL_SOURCES = ["k_gradf.hip", "k_strided.hip", "k_strided_impl.h", "k_strided_inst.hip",
                  "k_xfinala.hip", "k_xfinalb.hip", "k_xpass.hip", "k_xpass_impl.h", "st_device.h", "st_internal.h",
                  "st_host.h", "st_api.hip"]


def strip_comments(text):
    """C/C++ source text without comments, whitespace runs collapsed (string and
    character literals are kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(read=None):
    """sha256 (16 hex digits) of the comment-stripped headline-path sources."""
    if read is None:
        def read(f):
            with open(os.path.join(ROOT, "paper_2508_07476_amd", "csrc", f), encoding="utf-8") as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode() + b"\0" + strip_comments(read(f)).encode() + b"\0")
    return h.hexdigest()[:16]


def traffic_path(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def traffic_for(kernel, workload="two_annuli"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    ``workload``, if it belongs to the current kernel sources (else None)."""
    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def kernel_report(kern, nvox, steps, rs, rr, mask=False, workload="two_annuli"):
    """Roofline object of the dominant kernel and per-kernel figures.

    kern maps a kernel name to (total ms, launches) over `steps` steps of an
    nvox-voxel volume; rs and rr are the gradient and integration radii; mask
    says whether the final pass reads a mask.  The dominant kernel is placed
    against whichever roof (HBM bytes or vector-ALU operations) it is closer to."""

    def roof_for(name, ms, launches):
        avg_s = ms / launches / 1e3
        gbs = alg_bytes_per_voxel(name, mask) * nvox / avg_s / 1e9
        ops = alg_ops_per_voxel(name, rs, rr)
        tflops = None if ops is None else ops * 2 * nvox / avg_s / 1e12
        return avg_s, gbs, ops, tflops

    dname, (dms, dlaunch) = max(kern.items(), key=lambda kv: kv[1][0])
    avg_s, gbs, ops, tflops = roof_for(dname, dms, dlaunch)
    hbm_frac = gbs / HBM_PEAK_GBS
    alu_frac = None if tflops is None else tflops / VALU_PEAK_TFLOPS
    traffic = traffic_for(dname, workload)
    common = {"traffic": traffic, "kernel": dname, "avg_launch_ms": round(avg_s * 1e3, 4),
              "traffic_source": (f"committed rocprofv3 FETCH_SIZE/WRITE_SIZE counters of this workload and "
                                 f"these kernel sources (profiles/traffic_{workload}.json), not measured in "
                                 "this run" if traffic is not None else
                                 "none: no committed counters for the current kernel sources")}
    if alu_frac is not None and alu_frac > hbm_frac:
        roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), **common,
                "alg_ops_per_voxel": ops, "hbm_achieved_GBps": round(gbs, 1),
                "hbm_frac": round(hbm_frac, 4), "alg_bytes_per_voxel": alg_bytes_per_voxel(dname, mask)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4), **common,
                "alg_bytes_per_voxel": alg_bytes_per_voxel(dname, mask)}
    per_kernel = {}
    for k, v in kern.items():
        a_s, g, o, t = roof_for(k, v[0], v[1])
        per_kernel[k] = {"avg_ms": round(a_s * 1e3, 4), "launches_per_step": v[1] / steps,
                         "alg_GBps": round(g, 1), "hbm_frac": round(g / HBM_PEAK_GBS, 4)}
        tb = traffic_for(k, workload)  # rocprofv3 bytes per launch, when current
        if tb is not None:
            per_kernel[k]["measured_GBps"] = round(tb / a_s / 1e9, 1)
            per_kernel[k]["measured_frac"] = round(tb / a_s / 1e9 / HBM_PEAK_GBS, 4)
        if t is not None:
            per_kernel[k]["alu_frac"] = round(t / VALU_PEAK_TFLOPS, 4)
    return roof, per_kernel


def _oracle_block(crop, mask, lo, sigma, rho, center, direction):
    """One padded block through the FP64 oracle (runs in a worker process)."""
    import oracle
    oracle.compute(crop, mask, sigma, rho, TRUNCATE, axis_center=center, axis_direction=direction,
                   origin=tuple(lo))
    return crop.size


def _warm_worker(_):
    """Imports the oracle in a worker process before the timed region."""
    import numpy  # noqa: F401
    import scipy.ndimage  # noqa: F401

    import oracle  # noqa: F401
    return os.getpid()


def host_cores():
    """(cores this process may run on, capped at 16: the host share of one GPU; CPU model)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, min(16, avail)), model


def block_origins(shape, B, halo, count=16, seed=5, annuli=((128.0, 256.0), (320.0, 480.0))):
    """``count`` B^3 block origins spread over the z-thirds (the noise bands) and
    over the annuli, each at least ``halo`` from the volume faces."""
    import numpy as np
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    c = (ny - 1) / 2.0
    out = []
    for i in range(count):
        band = i % 3
        zlo = max(halo, band * nz // 3)
        zhi = min(nz - B - halo, (band + 1) * nz // 3 - B)
        z = int(rng.integers(zlo, max(zlo + 1, zhi)))
        r_in, r_out = annuli[i % len(annuli)]
        r = rng.uniform(r_in + B / 2, r_out - B / 2) if r_out - r_in > B else 0.5 * (r_in + r_out)
        th = rng.uniform(0, 2 * np.pi)
        y = int(np.clip(c + r * np.sin(th) - B / 2, halo, ny - B - halo))
        x = int(np.clip(c + r * np.cos(th) - B / 2, halo, nx - B - halo))
        out.append((z, y, x))
    return out


def cpu_baseline(workload, vol, mask, center, direction, B=96, count=16):
    """FP64 oracle, timed on ``count`` sampled B^3 blocks of the same volume, each
    padded by R_sigma + R_rho (which makes every block's interior equal to the
    whole-volume result), one block per worker process over the host cores."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    w = WORKLOADS[workload]
    sigma, rho = w["sigma"], w["rho"]
    halo = int(TRUNCATE * sigma + 0.5) + int(TRUNCATE * rho + 0.5)
    annuli = ((128.0, 256.0), (320.0, 480.0)) if workload == "two_annuli" else ((96.0, 224.0),)
    s = vol.shape[1] / 1024.0 if workload == "two_annuli" else vol.shape[1] / 512.0
    annuli = tuple((a * s, b * s) for a, b in annuli)
    origins = block_origins(tuple(vol.shape), B, halo, count, annuli=annuli)
    jobs = []
    for org in origins:
        lo = [o - halo for o in org]
        sl = tuple(slice(lo[d], org[d] + B + halo) for d in range(3))
        jobs.append((vol[sl].cpu().numpy(), None if mask is None else mask[sl].cpu().numpy(), lo))
    cores, model = host_cores()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"  # one thread per worker process
    try:
        with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as pool:
            pids = set(pool.map(_warm_worker, range(cores)))  # start and import in every worker
            t0 = time.perf_counter()
            futs = [pool.submit(_oracle_block, c, m, lo, sigma, rho, center, direction) for c, m, lo in jobs]
            padded = sum(f.result() for f in futs)
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    nvox = count * B ** 3
    return {"value": nvox / wall / 1e9, "unit": "Gvoxels/s", "cores": min(cores, count), "kind": "oracle",
            "cpu_model": model, "os_cpu_count": os.cpu_count(), "workers": len(pids),
            "sample": f"{count} blocks of {B}^3 voxels of the same volume (z-thirds and annuli), each padded by "
                      f"R_sigma + R_rho = {halo} and run whole through the FP64 NumPy/SciPy oracle (tensor, eigen, "
                      f"FA, HA, IA), one block per single-threaded worker process; value counts the {nvox} "
                      f"interior voxels ({padded} computed with the halos) over {wall:.1f} s wall"}


def run_plain(args, torch, st, helix, dev, workload):
    """One st_compute call per step on the whole volume of ``workload`` (inputs,
    outputs and workspace resident); returns the JSON line as a dict."""
    w = WORKLOADS[workload]
    shape, sigma, rho = w["shape"], w["sigma"], w["rho"]
    t = time.perf_counter()
    ph = make_phantom(helix, workload, dev)
    torch.cuda.synchronize()
    print(f"bench: {workload} phantom {shape} generated in {time.perf_counter() - t:.1f} s", file=sys.stderr,
          flush=True)
    vol = ph["volume"]
    mask = ph["mask"] if w["mask"] else None
    nvox = vol.numel()
    out = {k: torch.empty(((3,) if k == "e3" else ()) + tuple(shape), dtype=torch.float32, device=dev)
           for k in OUTPUTS}
    ws = torch.empty(st.st_workspace_bytes(shape), dtype=torch.uint8, device=dev)

    def step():
        st.st_compute(vol, sigma, rho, TRUNCATE, mask=mask, axis_center=ph["center"],
                      axis_direction=ph["direction"], outputs=OUTPUTS, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    st.profile_reset()
    st.profile_enable(True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    st.profile_enable(False)
    kern = st.profile_read()
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    value = nvox * args.steps / (total_ms / 1e3) / 1e9
    rs, rr = int(TRUNCATE * sigma + 0.5), int(TRUNCATE * rho + 0.5)
    roof, per_kernel = kernel_report(kern, nvox, args.steps, rs, rr, w["mask"], workload)
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gvoxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "shape": list(shape), "sigma": sigma, "rho": rho, "input": "uint16",
                   "mask": w["mask"], "arithmetic": "f64", "intermediate_storage": "f32"},
        "roofline": roof,
        "kernels": per_kernel,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(workload, vol, mask, ph["center"], ph["direction"])
    del out, ws, vol, mask, ph
    torch.cuda.empty_cache()
    return line


SURROGATE_WEIGHTS = os.path.join(ROOT, "paper_2508_07476_amd", "surrogate_weights.npy")


SURROGATE_WORKLOAD = {
    "desc": "1024^3 uint16 helical rod-lattice phantom + annulus mask (r 192-448, helix +70 to -50 deg, "
            "period 5, noise 0.02/0.06/0.12 by z-thirds); learned surrogate (5x 3x3x3 conv, 32 ch, bf16 MFMA) "
            "against the structure-tensor path at its training labels' scales sigma=1, rho=2, truncate=4; "
            "fallback where confidence < 0.9; outputs e3, FA, HA, IA, confidence",
    "shape": (1024, 1024, 1024), "sigma": 1.0, "rho": 2.0, "min_confidence": 0.9,
}


def run_surrogate(args, torch, st, helix, dev):
    """The surrogate alone and with its fallback (confidence < 0.9 takes the
    structure-tensor result), against the plain path on the 1024^3 surrogate
    volume: throughput, the fibre-angle error w.r.t. the plain path inside the
    mask (non-degenerate voxels, every 7th voxel), the fallback fraction and
    what the fallback ran."""
    import numpy as np
    W = SURROGATE_WORKLOAD
    sigma, rho = W["sigma"], W["rho"]
    blob = np.load(args.weights or SURROGATE_WEIGHTS, allow_pickle=False).astype(np.float32)
    w = torch.from_numpy(blob).to(dev)
    ph = helix.generate(helix.spec_surrogate_u16(shape=W["shape"]), device=dev)
    vol, mask = ph["volume"], ph["mask"]
    nvox = vol.numel()
    kw = dict(mask=mask, axis_center=ph["center"], axis_direction=ph["direction"])
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        st.profile_reset()
        st.profile_enable(True)
        ev[0].record(stream)
        for _ in range(args.steps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        st.profile_enable(False)
        kern = {k: round(v[0] / v[1], 4) for k, v in st.profile_read().items()}
        return ev[0].elapsed_time(ev[1]) / args.steps, kern

    plain = {}
    pms, _ = timed(lambda: plain.update(st.st_compute(vol, sigma, rho, TRUNCATE, outputs=("e3", "fa", "flags"),
                                                      **kw)))
    sub = torch.arange(0, nvox, 7, device=dev)
    sel = (plain["flags"].reshape(-1)[sub] == 0)
    idx = sub[sel]
    ref = plain["e3"].reshape(3, -1)[:, idx]
    inside = mask != 0
    n_inside = float(inside.sum())
    del plain
    torch.cuda.empty_cache()  # the surrogate's activations (128 B per voxel) come from the device pool
    outs = ("e3", "fa", "ha", "ia", "confidence")
    res = {}
    for name, thr in (("surrogate", 0.0), ("with_fallback", W["min_confidence"])):
        out = {}
        ms, kern = timed(lambda: out.update(st.st_surrogate_infer(vol, w, thr, sigma, rho, TRUNCATE, outputs=outs,
                                                                  **kw)))
        info = st.st_surrogate_fallback_info()
        a = out["e3"].reshape(3, -1)[:, idx]
        ang = torch.rad2deg(torch.atan2(torch.linalg.cross(a, ref, dim=0).norm(dim=0), (a * ref).sum(0).abs()))
        q = torch.quantile(ang[::max(1, ang.numel() // 8_000_000)].float(),
                           torch.tensor([0.5, 0.9], device=dev))
        fell = float(((out["confidence"] < thr) & inside).sum()) / n_inside if thr else 0.0
        res[name] = {"ms_per_step": round(ms, 3), "value": round(nvox / ms / 1e6, 4), "unit": "Gvoxels/s",
                     "median_angle_deg": round(float(q[0]), 3), "p90_angle_deg": round(float(q[1]), 3),
                     "frac_within_2deg": round(float((ang <= 2.0).float().mean()), 4),
                     "fallback_fraction": round(fell, 4), "kernels": kern}
        if thr:
            res[name]["fallback"] = info
        del out, a, ang
    torch.cuda.empty_cache()
    return {"workload": W["desc"], "weights": os.path.basename(args.weights or SURROGATE_WEIGHTS),
            "surrogate": res["surrogate"], "surrogate_with_fallback": res["with_fallback"],
            "plain": {"ms_per_step": round(pms, 3), "value": round(nvox / pms / 1e6, 4), "unit": "Gvoxels/s"}}


def surrogate_line(args, rec):
    """The --surrogate run's own line: the surrogate with its fallback is the value."""
    f = rec["surrogate_with_fallback"]
    return {"metric": METRIC, "value": f["value"], "unit": "Gvoxels/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": rec["workload"], "weights": rec["weights"]}, **rec}


BATCH_SIGMA = 1.0
BATCH_OUTPUTS = ("e3", "fa", "ha", "ia", "flags")


def run_batch(args, torch, st, helix, dev):
    """Chunk-batch workload (200 halo-padded chunks): the autotuned batch is the
    line's value; beside it the untuned 8-chain graph, the untuned grouped
    launches (in the batch's own 8-slot workspace, and in one holding every
    chunk: a single round) and one st_compute per chunk on one stream.  Inputs
    resident; all share one set of output tensors."""
    spec = helix.spec_headline_u16(shape=SHAPE)
    ph = helix.generate(spec, device=dev)
    crops = helix.batch_crops(SHAPE)
    chunks = []
    for org, shp, rho in crops:
        sl = tuple(slice(org[d], org[d] + shp[d]) for d in range(3))
        chunks.append({"volume": ph["volume"][sl].contiguous(), "mask": ph["mask"][sl].contiguous(),
                       "rho": rho, "origin": org})
    del ph["volume"], ph["mask"]
    nvox = sum(c["volume"].numel() for c in chunks)
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    kw = dict(axis_center=ph["center"], axis_direction=ph["direction"], outputs=BATCH_OUTPUTS)
    results = None
    modes = {}
    for name, lanes in (("chains8", 0), ("grouped", st.ST_BATCH_GROUPED)):
        b = st.Batch(chunks, BATCH_SIGMA, TRUNCATE, lanes=lanes, results=results, **kw)
        results = b.results
        ms = timed(b.launch, args.steps)
        modes[name] = {"ms_per_step": round(ms, 4), "value": round(nvox / ms / 1e6, 4), "unit": "Gvoxels/s",
                       "config": b.config(), "plan": b.plan()}
        b.close()
        torch.cuda.empty_cache()
    # grouped launches with a workspace holding every chunk: one round, one
    # launch per pass kind (when the device has room for it)
    one = sum((st.st_workspace_bytes(tuple(c["volume"].shape)) + 255) // 256 * 256 for c in chunks)
    if torch.cuda.mem_get_info(dev)[0] > one + (8 << 30):
        ws1 = torch.empty(one, dtype=torch.uint8, device=dev)
        b = st.Batch(chunks, BATCH_SIGMA, TRUNCATE, lanes=st.ST_BATCH_GROUPED, results=results, workspace=ws1, **kw)
        ms = timed(b.launch, args.steps)
        modes["grouped_one_round"] = {"ms_per_step": round(ms, 4), "value": round(nvox / ms / 1e6, 4),
                                      "unit": "Gvoxels/s", "workspace_bytes": one, "plan": b.plan()}
        b.close()
        del ws1
        torch.cuda.empty_cache()
    else:
        modes["grouped_one_round"] = {"skipped": f"needs {one} workspace bytes"}
    b = st.Batch(chunks, BATCH_SIGMA, TRUNCATE, lanes=0, results=results, **kw)
    t0 = time.perf_counter()
    cfg = b.tune(reps=2)
    tune_s = time.perf_counter() - t0
    ms = timed(b.launch, args.steps)
    tiles = {}
    for i in range(len(chunks)):
        key = "rows%d_lanes%d" % b.tiles(i)
        tiles[key] = tiles.get(key, 0) + 1
    tuned = {"config": cfg, "plan": b.plan(), "tile_shapes": tiles, "tune_seconds": round(tune_s, 2)}
    b.close()
    torch.cuda.empty_cache()
    # unbatched reference: one st_compute per chunk, in order, on one stream
    ws = torch.empty(max(st.st_workspace_bytes(tuple(c["volume"].shape)) for c in chunks),
                     dtype=torch.uint8, device=dev)

    def sequential():
        for c, r in zip(chunks, results):
            center = [ph["center"][d] - c["origin"][d] for d in range(3)]
            st.st_compute(c["volume"], BATCH_SIGMA, c["rho"], TRUNCATE, mask=c["mask"], axis_center=center,
                          axis_direction=ph["direction"], outputs=BATCH_OUTPUTS, out=r, workspace=ws)

    seq_ms = timed(sequential, max(1, args.steps // 2))
    line = {
        "metric": METRIC, "value": round(nvox / ms / 1e6, 4), "unit": "Gvoxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(chunks)} uint16 halo-padded chunks of the 512^3 helical phantom + "
                               "mask: interior sides U{64..384} per axis, halo 3*rho, rho in {2,3,4}, "
                               f"sigma={BATCH_SIGMA}; outputs e3, FA, HA, IA, flags; autotuned",
                   "chunks": len(chunks), "voxels": nvox, "input": "uint16",
                   "arithmetic": "f64", "intermediate_storage": "f32"},
        "tuned": tuned,
        "untuned": modes,
        "unbatched": {"ms_per_step": round(seq_ms, 4), "value": round(nvox / seq_ms / 1e6, 4),
                      "unit": "Gvoxels/s", "how": "one st_compute call per chunk on one stream"},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="two_annuli",
                    help="volume timed for the line's value (default: the 2048x1024x1024 two-annuli volume)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned surrogate's 1024^3 leg of the default run")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 512^3 figure that follows the default workload")
    ap.add_argument("--path-only", nargs=4, metavar=("SHAPE", "SIGMA", "RHO", "CALLS"), default=None,
                    help="only call st_compute CALLS times on the 512^3-geometry phantom of SHAPE (e.g. "
                         "512x512x512) at SIGMA, RHO (for counter collection)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write elementwise kernel (for scaling HBM "
                         "byte counters)")
    ap.add_argument("--surrogate", action="store_true",
                    help="time the learned surrogate (bf16 3-D CNN) alone and with its fallback on the "
                         "1024^3 surrogate volume and report its fibre-angle error against the "
                         "structure-tensor path")
    ap.add_argument("--weights", default=None, help="surrogate weights (.npy, float32 blob)")
    ap.add_argument("--batch", action="store_true",
                    help="time the chunk-batch workload (200 uneven halo-padded uint16 crops of the "
                         "512^3 phantom, rho in {2,3,4}, sigma 1) instead of the headline volume")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the structure-tensor path here is built and timed on "
              "a single MI355X (multi-GPU z-slab sharding is a design note, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2508_07476_amd as st
    from phantom import helix

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        # a kernel that reads 1 GiB and writes 1 GiB (a same-type copy_ is a DMA
        # transfer, which the kernel counters do not see)
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}))
        return
    torch.cuda.set_device(dev)
    st.load_library()
    if args.path_only:
        shape = tuple(int(v) for v in args.path_only[0].split("x"))
        sigma, rho, calls = float(args.path_only[1]), float(args.path_only[2]), int(args.path_only[3])
        ph = helix.generate(helix.spec_headline_u16(shape=shape), device=dev)
        outs = ("e3", "fa", "ha", "ia")
        out = {k: torch.empty(((3,) if k == "e3" else ()) + shape, dtype=torch.float32, device=dev) for k in outs}
        ws = torch.empty(st.st_workspace_bytes(shape), dtype=torch.uint8, device=dev)
        for _ in range(calls):
            st.st_compute(ph["volume"], sigma, rho, TRUNCATE, mask=ph["mask"], axis_center=ph["center"],
                          axis_direction=ph["direction"], outputs=outs, out=out, workspace=ws)
        torch.cuda.synchronize()
        print(json.dumps({"path_only": {"shape": shape, "sigma": sigma, "rho": rho, "calls": calls}}))
        return
    if args.batch:
        return run_batch(args, torch, st, helix, dev)
    if args.surrogate:
        print(json.dumps(surrogate_line(args, run_surrogate(args, torch, st, helix, dev))), flush=True)
        return
    line = run_plain(args, torch, st, helix, dev, args.workload)
    if args.workload == "two_annuli" and not args.no_secondary:
        sec = argparse.Namespace(**vars(args))
        sec.no_cpu_baseline = True
        sub = run_plain(sec, torch, st, helix, dev, "headline512")
        line["headline512"] = {k: sub[k] for k in ("value", "unit", "ms_per_step", "steps")}
        line["headline512"]["workload"] = WORKLOADS["headline512"]["desc"]
        line["headline512"]["dominant_kernel"] = {k: sub["roofline"][k] for k in
                                                  ("kernel", "bound", "frac", "avg_launch_ms")}
    if args.workload == "two_annuli" and not args.no_surrogate:
        rec = run_surrogate(args, torch, st, helix, dev)
        line["surrogate"] = {"workload": rec["workload"], "weights": rec["weights"], "plain": rec["plain"]}
        for key in ("surrogate", "surrogate_with_fallback"):
            line["surrogate"][key] = {k: v for k, v in rec[key].items() if k != "kernels"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
