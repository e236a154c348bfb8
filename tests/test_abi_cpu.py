"""The C-ABI library on a machine without a GPU: it loads, exports every symbol
the header declares, and rejects invalid arguments on the host before any HIP
call (fake non-null pointers are safe because validation fails first)."""

import ctypes
import os
import re

import pytest

import paper_2508_07476_amd as st
from paper_2508_07476_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "st.h")
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation first


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2508_07476_amd.csrc import build
        build.build()
    return st.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(st_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"st_compute", "st_angles", "st_surrogate_infer"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, n
    assert set(B.SIGNATURES) == set(names)


def test_version_radius_and_workspace(lib):
    assert lib.st_version() >= 10000
    assert [lib.st_filter_radius(s, 4.0) for s in (1.0, 1.5, 2.0, 3.0, 4.0, 6.0)] == [4, 6, 8, 12, 16, 24]
    assert lib.st_filter_radius(0.0, 4.0) == -1 and lib.st_filter_radius(1.0, float("nan")) == -1
    # 12 float planes of nz * ny * pitch elements, each rounded up to 256 bytes; the
    # row pitch is nx rounded up to a multiple of 32 above 32, else of 4
    def expected(nz, ny, nx):
        pitch = -(-nx // 32) * 32 if nx > 32 else -(-nx // 4) * 4
        return 12 * (-(-(nz * ny * pitch * 4) // 256) * 256)

    for shape, pitch in (((5, 7, 9), 12), ((3, 4, 32), 32), ((3, 4, 33), 64), ((2, 3, 392), 416),
                         ((1, 1, 1), 4), ((4, 4, 512), 512)):
        assert lib.st_workspace_bytes(*shape) == expected(*shape), shape
        assert expected(*shape) >= 12 * shape[0] * shape[1] * pitch * 4
    assert lib.st_workspace_bytes(5, 7, 9) == 21504
    assert lib.st_workspace_bytes(0, 7, 9) == 0
    assert lib.st_workspace_bytes(2 ** 31, 1, 1) == 0          # each size < 2^31
    assert lib.st_workspace_bytes(2 ** 30, 2 ** 30, 2 ** 30) == 0  # product overflow


def _compute(lib, **kw):
    a = dict(volume=FAKE, dtype=B.ST_DTYPE_U16, mask=None, nz=8, ny=8, nx=8, sigma=1.0, rho=2.0,
             truncate=4.0, center=None, direction=None, e3=FAKE, evals=None, fa=None, ha=None, ia=None,
             flags=None, ws=None, ws_bytes=0)
    a.update(kw)
    vec = lambda v: None if v is None else (ctypes.c_double * 3)(*v)  # noqa: E731
    code = lib.st_compute(a["volume"], a["dtype"], a["mask"], a["nz"], a["ny"], a["nx"], a["sigma"],
                          a["rho"], a["truncate"], vec(a["center"]), vec(a["direction"]), a["e3"],
                          a["evals"], a["fa"], a["ha"], a["ia"], a["flags"], a["ws"], a["ws_bytes"], None)
    return code, lib.st_last_error().decode()


@pytest.mark.parametrize("kw,code,text", [
    (dict(volume=None), B.ST_ERR_INVALID_ARG, "volume is NULL"),
    (dict(dtype=7), B.ST_ERR_INVALID_ARG, "dtype"),
    (dict(nz=0), B.ST_ERR_INVALID_ARG, "sizes"),
    (dict(nx=-3), B.ST_ERR_INVALID_ARG, "sizes"),
    (dict(nz=2 ** 31), B.ST_ERR_INVALID_ARG, "sizes"),
    (dict(nz=2 ** 30, ny=2 ** 30, nx=2 ** 30), B.ST_ERR_INVALID_ARG, "sizes"),
    (dict(sigma=0.0), B.ST_ERR_INVALID_ARG, "sigma"),
    (dict(rho=float("nan")), B.ST_ERR_INVALID_ARG, "sigma"),
    (dict(truncate=-1.0), B.ST_ERR_INVALID_ARG, "sigma"),
    (dict(sigma=0.1), B.ST_ERR_INVALID_ARG, "radius"),
    (dict(sigma=5.0), B.ST_ERR_UNSUPPORTED, "exceeds"),
    (dict(rho=8.2), B.ST_ERR_UNSUPPORTED, "exceeds"),
    (dict(center=(1, 2, 3)), B.ST_ERR_INVALID_ARG, "both"),
    (dict(center=(1, 2, 3), direction=(0, 0, 0)), B.ST_ERR_INVALID_ARG, "non-zero"),
    (dict(center=(1, float("inf"), 3), direction=(1, 0, 0)), B.ST_ERR_INVALID_ARG, "finite"),
    (dict(ha=FAKE), B.ST_ERR_INVALID_ARG, "need an axis"),
    (dict(e3=None), B.ST_ERR_INVALID_ARG, "no output"),
    (dict(ws=None, ws_bytes=64), B.ST_ERR_INVALID_ARG, "workspace is NULL"),
    (dict(ws=FAKE, ws_bytes=64), B.ST_ERR_INVALID_ARG, "workspace_bytes"),
])
def test_compute_rejects_invalid_arguments_on_host(lib, kw, code, text):
    got, msg = _compute(lib, **kw)
    assert got == code, msg
    assert text in msg


def test_angles_rejects_invalid_arguments_on_host(lib):
    c = (ctypes.c_double * 3)(1, 2, 3)
    d = (ctypes.c_double * 3)(1, 0, 0)
    z = (ctypes.c_double * 3)(0, 0, 0)
    assert lib.st_angles(None, None, 4, 4, 4, c, d, FAKE, FAKE, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_angles(FAKE, None, 4, 4, 4, None, None, FAKE, FAKE, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_angles(FAKE, None, 4, 4, 4, c, z, FAKE, FAKE, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_angles(FAKE, None, 4, 0, 4, c, d, FAKE, FAKE, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_angles(FAKE, None, 4, 4, 4, c, d, None, None, None, None) == B.ST_ERR_INVALID_ARG
    assert "no output" in lib.st_last_error().decode()


def _surrogate(lib, **kw):
    a = dict(volume=FAKE, dtype=B.ST_DTYPE_U16, mask=None, nz=8, ny=8, nx=8, weights=FAKE,
             wbytes=4 * B.ST_SURROGATE_WEIGHTS, minc=0.0, sigma=1.0, rho=2.0, truncate=4.0, center=None,
             direction=None, e3=FAKE, fa=None, ha=None, ia=None, conf=None)
    a.update(kw)
    vec = lambda v: None if v is None else (ctypes.c_double * 3)(*v)  # noqa: E731
    code = lib.st_surrogate_infer(a["volume"], a["dtype"], a["mask"], a["nz"], a["ny"], a["nx"], a["weights"],
                                  a["wbytes"], a["minc"], a["sigma"], a["rho"], a["truncate"], vec(a["center"]),
                                  vec(a["direction"]), a["e3"], a["fa"], a["ha"], a["ia"], a["conf"], None)
    return code, lib.st_last_error().decode()


@pytest.mark.parametrize("kw,code,text", [
    (dict(volume=None), B.ST_ERR_INVALID_ARG, "volume is NULL"),
    (dict(dtype=3), B.ST_ERR_INVALID_ARG, "dtype"),
    (dict(nz=0), B.ST_ERR_INVALID_ARG, "sizes"),
    (dict(weights=None), B.ST_ERR_INVALID_ARG, "weights is NULL"),
    (dict(wbytes=100), B.ST_ERR_INVALID_ARG, "weights_bytes"),
    (dict(minc=1.5), B.ST_ERR_INVALID_ARG, "min_confidence"),
    (dict(minc=float("nan")), B.ST_ERR_INVALID_ARG, "min_confidence"),
    (dict(minc=0.5, sigma=0.0), B.ST_ERR_INVALID_ARG, "sigma"),
    (dict(minc=0.5, rho=9.0), B.ST_ERR_UNSUPPORTED, "exceeds"),
    (dict(center=(1, 2, 3)), B.ST_ERR_INVALID_ARG, "both"),
    (dict(ha=FAKE), B.ST_ERR_INVALID_ARG, "need an axis"),
    (dict(e3=None), B.ST_ERR_INVALID_ARG, "no output"),
])
def test_surrogate_rejects_invalid_arguments_on_host(lib, kw, code, text):
    got, msg = _surrogate(lib, **kw)
    assert got == code, msg
    assert text in msg


def test_surrogate_scales_are_not_needed_without_fallback(lib):
    # min_confidence 0: sigma/rho are unused, so an invalid value passes host
    # validation and the call fails later, at the device-buffer check
    got, msg = _surrogate(lib, minc=0.0, sigma=0.0)
    assert "sigma" not in msg


def test_surrogate_weight_count_matches_oracle(lib):
    from oracle import surrogate
    assert B.ST_SURROGATE_WEIGHTS == surrogate.n_weights()


def test_error_message_is_per_call(lib):
    _compute(lib, dtype=9)
    assert "dtype" in lib.st_last_error().decode()
    _compute(lib, nz=0)
    assert "dtype" not in lib.st_last_error().decode()


def _chunks(*specs):
    arr = (B.StChunk * max(1, len(specs)))()
    for i, s in enumerate(specs):
        c = dict(volume=FAKE.value, dtype=B.ST_DTYPE_U16, nz=8, ny=8, nx=8, rho=2.0, e3=FAKE.value)
        c.update(s)
        arr[i].volume, arr[i].dtype = c["volume"], c["dtype"]
        arr[i].nz, arr[i].ny, arr[i].nx, arr[i].rho = c["nz"], c["ny"], c["nx"], c["rho"]
        arr[i].e3, arr[i].ha = c["e3"], c.get("ha")
    return arr


def test_batch_workspace_bytes(lib):
    arr = _chunks(dict(nz=5, ny=7, nx=9), dict(nz=10, ny=3, nx=4))
    # a slot holds the single-volume workspace of the largest chunk
    slot = max(lib.st_workspace_bytes(5, 7, 9), lib.st_workspace_bytes(10, 3, 4))
    assert slot == 21504
    assert lib.st_batch_workspace_bytes(arr, 2, 3) == 3 * slot
    assert lib.st_batch_workspace_bytes(arr, 2, 0) == B.ST_BATCH_MAX_LANES * slot
    assert lib.st_batch_workspace_bytes(arr, 2, B.ST_BATCH_GROUPED) == B.ST_BATCH_MAX_LANES * slot
    assert lib.st_batch_workspace_bytes(arr, 2, -2) == 0
    assert lib.st_batch_workspace_bytes(arr, 2, 9) == 0
    assert lib.st_batch_workspace_bytes(arr, 0, 1) == 0
    assert lib.st_batch_workspace_bytes(_chunks(dict(nz=0)), 1, 1) == 0
    assert st.Batch.workspace_bytes([(5, 7, 9), (10, 3, 4)], lanes=3) == 3 * slot


def _create(lib, arr, n, lanes=1, center=None, direction=None, ws=None, ws_bytes=0, out=True):
    vec = lambda v: None if v is None else (ctypes.c_double * 3)(*v)  # noqa: E731
    h = ctypes.c_void_p()
    code = lib.st_batch_create(arr, n, 1.0, 4.0, vec(center), vec(direction), lanes, ws, ws_bytes,
                               ctypes.byref(h) if out else None)
    assert not h.value  # nothing is created when validation fails
    return code, lib.st_last_error().decode()


@pytest.mark.parametrize("case,text", [
    (dict(out=False), "out is NULL"),
    (dict(n=0), "at least one chunk"),
    (dict(lanes=9), "lanes"),
    (dict(lanes=-2), "lanes"),
    (dict(center=(1, 2, 3)), "both"),
    (dict(specs=[{}, dict(rho=0.0)]), "chunk 1"),
    (dict(specs=[dict(nx=0)]), "sizes"),
    (dict(specs=[dict(dtype=5)]), "dtype"),
    (dict(specs=[dict(ha=FAKE.value)]), "need an axis"),
    (dict(specs=[dict(e3=None)]), "no output"),
    (dict(ws_bytes=64), "workspace is NULL"),
    (dict(ws=FAKE, ws_bytes=64), "workspace_bytes"),
])
def test_batch_create_rejects_invalid_arguments_on_host(lib, case, text):
    specs = case.pop("specs", [{}])
    n = case.pop("n", len(specs))
    code, msg = _create(lib, _chunks(*specs), n, **case)
    assert code == B.ST_ERR_INVALID_ARG, msg
    assert text in msg


def test_batch_calls_reject_null_handle(lib):
    assert lib.st_batch_launch(None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_batch_tune(None, None, 1) == B.ST_ERR_INVALID_ARG
    assert lib.st_batch_config(None, None, None, None, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_batch_tiles(None, 0, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_batch_plan(None, None, None, None) == B.ST_ERR_INVALID_ARG
    assert lib.st_batch_destroy(None) == B.ST_OK


# ---- forced allocation failure (ST_FAULT_INJECT=alloc) ----------------------
# With the hook set, each entry point that would allocate device memory reports
# ST_ERR_OUT_OF_MEMORY after host validation and before any HIP call, so the
# path runs on a machine without a GPU.  The outputs here are host buffers with
# a sentinel: the library must not write them.


def _sentinel(n):
    buf = (ctypes.c_float * n)(*([7.25] * n))
    return buf, ctypes.cast(buf, ctypes.c_void_p)


def _untouched(buf):
    return all(v == 7.25 for v in buf)


def test_fault_inject_alloc_compute(lib, monkeypatch):
    monkeypatch.setenv("ST_FAULT_INJECT", "alloc")
    buf, ptr = _sentinel(3 * 8 * 8 * 8)
    code, msg = _compute(lib, e3=ptr)  # workspace NULL: the library would allocate it
    assert code == B.ST_ERR_OUT_OF_MEMORY, msg
    assert "ST_FAULT_INJECT" in msg and _untouched(buf)
    # a caller workspace needs no allocation: the hook does not fire (the call
    # then fails at the device-buffer check, since nothing here is on a GPU)
    code, msg = _compute(lib, e3=ptr, ws=FAKE, ws_bytes=1 << 20)
    assert code != B.ST_ERR_OUT_OF_MEMORY and "ST_FAULT_INJECT" not in msg
    assert _untouched(buf)


def test_fault_inject_alloc_batch_create(lib, monkeypatch):
    monkeypatch.setenv("ST_FAULT_INJECT", "alloc")
    buf, ptr = _sentinel(3 * 8 * 8 * 8)
    code, msg = _create(lib, _chunks(dict(e3=ptr.value), dict(e3=ptr.value, nz=12)), 2, lanes=2)
    assert code == B.ST_ERR_OUT_OF_MEMORY, msg
    assert "ST_FAULT_INJECT" in msg and _untouched(buf)


def test_fault_inject_alloc_surrogate(lib, monkeypatch):
    monkeypatch.setenv("ST_FAULT_INJECT", "alloc")
    buf, ptr = _sentinel(3 * 8 * 8 * 8)
    cbuf, cptr = _sentinel(8 * 8 * 8)
    for minc in (0.0, 0.9):
        code, msg = _surrogate(lib, e3=ptr, conf=cptr, minc=minc)
        assert code == B.ST_ERR_OUT_OF_MEMORY, msg
        assert "ST_FAULT_INJECT" in msg and _untouched(buf) and _untouched(cbuf)


def test_fault_inject_needs_the_exact_value(lib, monkeypatch):
    monkeypatch.setenv("ST_FAULT_INJECT", "none")
    code, msg = _compute(lib)
    assert code != B.ST_ERR_OUT_OF_MEMORY and "ST_FAULT_INJECT" not in msg
