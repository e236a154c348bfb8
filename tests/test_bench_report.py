"""bench.py's report assembly on a machine without a GPU: the roofline object
and per-kernel figures built from kernel timings, and the source hash that
decides whether the committed HBM byte counts still apply."""

import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

NVOX = 512 ** 3
STEPS = 4
# (total ms over STEPS steps, launches) per kernel, in the shape the profiler reports
KERN = {"grad_fused": (6.0, 4), "integrate_z": (5.6, 4), "integrate_y": (5.4, 4),
        "integrate_x_eigen": (8.0, 4)}


def test_dominant_kernel_roofline():
    roof, per = bench.kernel_report(KERN, NVOX, STEPS, 6, 16, mask=True, workload="headline512")
    json.dumps({"roofline": roof, "kernels": per})  # the line must serialise
    assert roof["kernel"] == "integrate_x_eigen"
    avg_s = 8.0 / 4 / 1e3
    assert roof["avg_launch_ms"] == 2.0
    ops = bench.alg_ops_per_voxel("integrate_x_eigen", 6, 16)
    assert ops == 6 * 33 + bench.EIGEN_ANGLE_OPS
    tflops = ops * 2 * NVOX / avg_s / 1e12
    gbs = bench.alg_bytes_per_voxel("integrate_x_eigen", True) * NVOX / avg_s / 1e9
    assert bench.alg_bytes_per_voxel("integrate_x_eigen", True) == 49
    assert bench.alg_bytes_per_voxel("integrate_x_eigen", False) == 48
    # the final pass is closer to the vector-ALU roof than to the HBM roof
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    assert math.isclose(roof["achieved"], tflops, rel_tol=1e-3)
    assert math.isclose(roof["frac"], roof["achieved"] / roof["peak"], rel_tol=1e-3)
    assert math.isclose(roof["hbm_achieved_GBps"], gbs, rel_tol=1e-3)
    assert set(per) == set(KERN)
    for k, v in per.items():
        assert v["launches_per_step"] == 1.0
        assert math.isclose(v["avg_ms"], KERN[k][0] / KERN[k][1], rel_tol=1e-6)


def test_hbm_bound_kernel():
    roof, _ = bench.kernel_report({"integrate_z": (1.0, 1), "grad_z": (9.0, 1)}, NVOX, 1, 6, 16)
    assert roof["kernel"] == "grad_z" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    gbs = bench.alg_bytes_per_voxel("grad_z") * NVOX / 9e-3 / 1e9
    assert math.isclose(roof["achieved"], gbs, rel_tol=1e-3)
    assert roof["peak"] == bench.HBM_PEAK_GBS


def test_peaks():
    assert math.isclose(bench.VALU_PEAK_TFLOPS, 78.6432, rel_tol=1e-9)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_strip_comments():
    src = 'int a = 1; // one\n/* two\n lines */ char* s = "x // y /* z */";\nchar c = \'/\';'
    assert bench.strip_comments(src) == 'int a = 1; char* s = "x // y /* z */"; char c = \'/\';'
    # comments and layout do not move the hash; code does
    assert bench.strip_comments("a  =\n b; // c") == bench.strip_comments("a = b;")
    assert bench.strip_comments("a = b;") != bench.strip_comments("a = c;")


def test_source_hash_covers_the_kernel_sources():
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2508_07476_amd", "csrc", f)), f
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    for w in bench.WORKLOADS:
        path = bench.traffic_path(w)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            rec = json.load(fh)
        assert len(rec["source_hash"]) == 16
        assert all(k in ("grad_fused", "grad_z", "grad_y", "grad_x_outer", "integrate_z", "integrate_y",
                         "integrate_x_eigen") for k in rec["kernels"])


def test_stale_traffic_is_not_reported(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda read=None: "0" * 16)
    roof, per = bench.kernel_report(KERN, NVOX, STEPS, 6, 16, mask=True, workload="headline512")
    assert roof["traffic"] is None and "none" in roof["traffic_source"]
    assert all("measured_GBps" not in v for v in per.values())


def test_block_origins_stay_inside_and_cover_the_bands():
    shape, B, halo = (2048, 1024, 1024), 96, 32
    org = bench.block_origins(shape, B, halo, 16)
    assert len(org) == 16
    for o in org:
        for d in range(3):
            assert halo <= o[d] <= shape[d] - B - halo, o
    assert {o[0] * 3 // shape[0] for o in org} == {0, 1, 2}


def test_calls_to_bench_functions_match_their_signatures():
    """Every call in bench.py to one of its own functions binds to that function's
    signature (the GPU-only modes cannot run here, so a stale call would only
    show on the GPU)."""
    import ast
    import inspect

    with open(os.path.join(ROOT, "bench.py")) as fh:
        tree = ast.parse(fh.read())
    funcs = {n.name: getattr(bench, n.name) for n in tree.body if isinstance(n, ast.FunctionDef)}
    checked = 0
    for node in ast.walk(tree):
        if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id in funcs:
            if any(isinstance(a, ast.Starred) for a in node.args) or any(k.arg is None for k in node.keywords):
                continue
            sig = inspect.signature(funcs[node.func.id])
            try:
                sig.bind(*[None] * len(node.args), **{k.arg: None for k in node.keywords})
            except TypeError as e:
                raise AssertionError(f"bench.py line {node.lineno}: {node.func.id}: {e}") from None
            checked += 1
    assert checked >= 8
