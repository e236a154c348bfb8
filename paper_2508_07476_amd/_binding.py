"""ctypes binding of libst.so: argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module checks
tensor types, allocates outputs and the workspace with PyTorch (device memory
and streams are all PyTorch is used for) and passes raw pointers.  If the
library is missing it raises -- there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libst.so")

ST_OK = 0
ST_ERR_INVALID_ARG = 1
ST_ERR_UNSUPPORTED = 2
ST_ERR_OUT_OF_MEMORY = 3
ST_ERR_DEVICE = 4
ST_DTYPE_U16 = 1
ST_DTYPE_F32 = 2
ST_FLAG_DEGENERATE = 1
ST_FLAG_OUTSIDE_MASK = 2
ST_FLAG_ON_AXIS = 4

ST_BATCH_MAX_LANES = 8
ST_BATCH_GROUPED = -1
ST_NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024


class StChunk(ctypes.Structure):
    """Mirror of ``st_chunk`` (include/st.h)."""
    _fields_ = [("volume", ctypes.c_void_p), ("dtype", ctypes.c_int), ("mask", ctypes.c_void_p),
                ("nz", ctypes.c_int64), ("ny", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("rho", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("e3", ctypes.c_void_p), ("evals", ctypes.c_void_p), ("fa", ctypes.c_void_p),
                ("ha", ctypes.c_void_p), ("ia", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


# exported symbols and their C signatures (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "st_version": (ctypes.c_int, []),
    "st_last_error": (ctypes.c_char_p, []),
    "st_filter_radius": (ctypes.c_int, [_D, _D]),
    "st_workspace_bytes": (_SZ, [_I64, _I64, _I64]),
    "st_compute": (ctypes.c_int, [_P, ctypes.c_int, _P, _I64, _I64, _I64, _D, _D, _D, _DP, _DP,
                                  _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "st_compute_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _I64, _I64, _I64, _D, _D, _D, _DP, _DP,
                                          _P, _P, _P, _P, _P, _P, _P]),
    "st_angles": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _DP, _DP, _P, _P, _P, _P]),
    "st_surrogate_infer": (ctypes.c_int, [_P, ctypes.c_int, _P, _I64, _I64, _I64, _P, _SZ, _D,
                                          _D, _D, _D, _DP, _DP, _P, _P, _P, _P, _P, _P]),
    "st_surrogate_grad_workspace_bytes": (_SZ, [_I64, _I64]),
    "st_surrogate_grad": (ctypes.c_int, [_P, ctypes.c_int, _I64, _I64, _P, _P, _P, _P, _D, _P, _P, _P, _SZ, _P]),
    "st_surrogate_adam": (ctypes.c_int, [_P, _P, _P, _P, _I64, _D, _D, _D, _D, _P]),
    "st_surrogate_fallback_info": (ctypes.c_int, [_P, _P, _P, _P]),
    "st_batch_workspace_bytes": (_SZ, [ctypes.POINTER(StChunk), ctypes.c_int, ctypes.c_int]),
    "st_batch_create": (ctypes.c_int, [ctypes.POINTER(StChunk), ctypes.c_int, _D, _D, _DP, _DP,
                                       ctypes.c_int, _P, _SZ, ctypes.POINTER(_P)]),
    "st_batch_launch": (ctypes.c_int, [_P, _P]),
    "st_batch_tune": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "st_batch_config": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(_I64), ctypes.POINTER(_I64), _DP]),
    "st_batch_plan": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int)]),
    "st_batch_tiles": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "st_batch_progress": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "st_batch_destroy": (ctypes.c_int, [_P]),
    "st_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "st_profile_reset": (ctypes.c_int, []),
    "st_profile_read": (ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, _SZ, _DP,
                                       ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


class StError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"st error {code}: {message}")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load libst.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_2508_07476_amd.csrc.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != ST_OK:
        msg = load_library().st_last_error()
        raise StError(code, msg.decode() if msg else "")


def _vec3(v) -> Optional[ctypes.Array]:
    if v is None:
        return None
    vals = [float(x) for x in v]
    if len(vals) != 3:
        raise ValueError("axis vectors have 3 (z, y, x) components")
    return (ctypes.c_double * 3)(*vals)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def st_version() -> int:
    return load_library().st_version()


def st_filter_radius(scale: float, truncate: float = 4.0) -> int:
    return load_library().st_filter_radius(scale, truncate)


def st_workspace_bytes(shape: Sequence[int]) -> int:
    nz, ny, nx = (int(s) for s in shape)
    return load_library().st_workspace_bytes(nz, ny, nx)


def _require_device_tensor(name, t, dtypes, shape=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device, got {t.device}")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} dtype {t.dtype} not in {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be C-contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


ALL_OUTPUTS = ("e3", "evals", "fa", "ha", "ia", "flags")


def _mask_arg(mask, shape):
    """The mask as a uint8 device tensor of ``shape`` (a bool mask is viewed as uint8), or None."""
    import torch
    if mask is None:
        return None
    _require_device_tensor("mask", mask, (torch.uint8, torch.bool), shape)
    return mask.view(torch.uint8) if mask.dtype == torch.bool else mask


def _outputs(outputs, out, shape, dev):
    """The requested st_compute outputs: tensors from ``out`` (checked) or new ones."""
    import torch
    outputs = tuple(outputs)
    res = {}
    out = out or {}
    for k in outputs:
        if k not in ALL_OUTPUTS:
            raise ValueError(f"unknown output {k!r}")
        shp = (3,) + tuple(shape) if k in ("e3", "evals") else tuple(shape)
        dt = torch.uint8 if k == "flags" else torch.float32
        if k in out:
            _require_device_tensor(k, out[k], (dt,), shp)
            res[k] = out[k]
        else:
            res[k] = torch.empty(shp, dtype=dt, device=dev)
    return res


def st_compute(volume, sigma: float, rho: float, truncate: float = 4.0, mask=None,
               axis_center=None, axis_direction=None,
               outputs: Iterable[str] = ("e3", "fa", "ha", "ia", "flags"),
               out: Optional[dict] = None, workspace=None):
    """Run the whole structure-tensor path on ``volume`` (nz, ny, nx) uint16/float32 CUDA tensor.

    Returns a dict with the requested outputs: ``e3`` / ``evals`` (3, nz, ny, nx)
    float32, ``fa`` / ``ha`` / ``ia`` (nz, ny, nx) float32, ``flags`` uint8.
    ``out`` may supply preallocated output tensors; ``workspace`` a uint8 tensor of
    at least ``st_workspace_bytes(volume.shape)`` bytes.  Work is enqueued on the
    current stream of the volume's device.
    """
    import torch
    lib = load_library()
    _require_device_tensor("volume", volume, (torch.uint16, torch.float32))
    if volume.dim() != 3:
        raise ValueError("volume must be 3-D (nz, ny, nx)")
    nz, ny, nx = volume.shape
    dev = volume.device
    dtype = ST_DTYPE_U16 if volume.dtype == torch.uint16 else ST_DTYPE_F32
    mask = _mask_arg(mask, (nz, ny, nx))
    res = _outputs(outputs, out, (nz, ny, nx), dev)
    if workspace is None:
        workspace = torch.empty(st_workspace_bytes((nz, ny, nx)), dtype=torch.uint8, device=dev)
    else:
        _require_device_tensor("workspace", workspace, (torch.uint8,))
    ws_bytes = workspace.numel()
    with torch.cuda.device(dev):
        code = lib.st_compute(_ptr(volume), dtype, _ptr(mask), nz, ny, nx, float(sigma), float(rho),
                              float(truncate), _vec3(axis_center), _vec3(axis_direction),
                              _ptr(res.get("e3")), _ptr(res.get("evals")), _ptr(res.get("fa")),
                              _ptr(res.get("ha")), _ptr(res.get("ia")), _ptr(res.get("flags")),
                              _ptr(workspace), ws_bytes, _stream_handle(dev))
    _check(code)
    return res


def st_compute_noalloc(volume, sigma: float, rho: float, truncate: float = 4.0, mask=None,
                       axis_center=None, axis_direction=None,
                       outputs: Iterable[str] = ("e3", "fa", "ha", "ia", "flags"),
                       out: Optional[dict] = None):
    """``st_compute`` with the library's own device scratch as workspace: the
    library allocates nothing (volumes up to about 128^3; see include/st.h).
    Outputs not supplied in ``out`` are allocated here by PyTorch."""
    import torch
    lib = load_library()
    _require_device_tensor("volume", volume, (torch.uint16, torch.float32))
    if volume.dim() != 3:
        raise ValueError("volume must be 3-D (nz, ny, nx)")
    nz, ny, nx = volume.shape
    dev = volume.device
    mask = _mask_arg(mask, (nz, ny, nx))
    res = _outputs(outputs, out, (nz, ny, nx), dev)
    with torch.cuda.device(dev):
        code = lib.st_compute_noalloc(_ptr(volume), ST_DTYPE_U16 if volume.dtype == torch.uint16 else ST_DTYPE_F32,
                                      _ptr(mask), nz, ny, nx, float(sigma), float(rho), float(truncate),
                                      _vec3(axis_center), _vec3(axis_direction), _ptr(res.get("e3")),
                                      _ptr(res.get("evals")), _ptr(res.get("fa")), _ptr(res.get("ha")),
                                      _ptr(res.get("ia")), _ptr(res.get("flags")), _stream_handle(dev))
    _check(code)
    return res


def st_angles(e3, axis_center, axis_direction, mask=None, outputs: Iterable[str] = ("ha", "ia"),
              out: Optional[dict] = None):
    """Helix / intrusion angles of a fibre field ``e3`` (3, nz, ny, nx) about a new axis."""
    import torch
    lib = load_library()
    _require_device_tensor("e3", e3, (torch.float32,))
    if e3.dim() != 4 or e3.shape[0] != 3:
        raise ValueError("e3 must be (3, nz, ny, nx)")
    _, nz, ny, nx = e3.shape
    dev = e3.device
    if mask is not None:
        _require_device_tensor("mask", mask, (torch.uint8, torch.bool), (nz, ny, nx))
        if mask.dtype == torch.bool:
            mask = mask.view(torch.uint8)
    res = {}
    out = out or {}
    for k in outputs:
        if k not in ("ha", "ia", "flags"):
            raise ValueError(f"unknown output {k!r}")
        dt = torch.uint8 if k == "flags" else torch.float32
        if k in out:
            _require_device_tensor(k, out[k], (dt,), (nz, ny, nx))
            res[k] = out[k]
        else:
            res[k] = torch.empty((nz, ny, nx), dtype=dt, device=dev)
    with torch.cuda.device(dev):
        code = lib.st_angles(_ptr(e3), _ptr(mask), nz, ny, nx, _vec3(axis_center), _vec3(axis_direction),
                             _ptr(res.get("ha")), _ptr(res.get("ia")), _ptr(res.get("flags")),
                             _stream_handle(dev))
    _check(code)
    return res


ST_SURROGATE_WEIGHTS = 111783
SURROGATE_OUTPUTS = ("e3", "fa", "ha", "ia", "confidence")


def st_surrogate_infer(volume, weights, min_confidence: float = 0.0, sigma: float = 1.5,
                       rho: float = 4.0, truncate: float = 4.0, mask=None, axis_center=None,
                       axis_direction=None, outputs: Iterable[str] = ("e3", "fa", "confidence"),
                       out: Optional[dict] = None):
    """Learned orientation surrogate (dense 3-D CNN on the bf16 matrix cores).

    ``weights``: float32 CUDA tensor of ``ST_SURROGATE_WEIGHTS`` values (see
    include/st.h for the layout).  Voxels inside the mask whose confidence is
    below ``min_confidence`` take st_compute's outputs (sigma, rho, truncate).
    Returns a dict of the requested outputs.
    """
    import torch
    lib = load_library()
    _require_device_tensor("volume", volume, (torch.uint16, torch.float32))
    if volume.dim() != 3:
        raise ValueError("volume must be 3-D (nz, ny, nx)")
    _require_device_tensor("weights", weights, (torch.float32,))
    nz, ny, nx = volume.shape
    dev = volume.device
    if mask is not None:
        _require_device_tensor("mask", mask, (torch.uint8, torch.bool), (nz, ny, nx))
        if mask.dtype == torch.bool:
            mask = mask.view(torch.uint8)
    outputs = tuple(outputs)
    for k in outputs:
        if k not in SURROGATE_OUTPUTS:
            raise ValueError(f"unknown output {k!r}")
    out = out or {}
    res = {}
    for k in outputs:
        shape = (3, nz, ny, nx) if k == "e3" else (nz, ny, nx)
        if k in out:
            _require_device_tensor(k, out[k], (torch.float32,), shape)
            res[k] = out[k]
        else:
            res[k] = torch.empty(shape, dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        code = lib.st_surrogate_infer(_ptr(volume), ST_DTYPE_U16 if volume.dtype == torch.uint16 else ST_DTYPE_F32,
                                      _ptr(mask), nz, ny, nx, _ptr(weights), weights.numel() * 4,
                                      float(min_confidence), float(sigma), float(rho), float(truncate),
                                      _vec3(axis_center), _vec3(axis_direction), _ptr(res.get("e3")),
                                      _ptr(res.get("fa")), _ptr(res.get("ha")), _ptr(res.get("ia")),
                                      _ptr(res.get("confidence")), _stream_handle(dev))
    _check(code)
    return res


def st_surrogate_grad(patches, target_e3, target_fa, weight, params, grad=None, stats=None, workspace=None,
                      conf_weight: float = 0.1):
    """Gradient of the surrogate's training objective (see include/st.h) for a
    stack of patches (npatch * P, P, P) uint16/float32 CUDA tensor, P <= 32.
    target_e3 (3, npatch * P, P, P), target_fa (npatch * P, P, P) float32,
    weight (npatch * P, P, P) uint8/bool, params float32[ST_SURROGATE_WEIGHTS].
    conf_weight: weight of the confidence term of the objective.
    Returns (grad, stats) float32 CUDA tensors (stats: 8 values)."""
    import torch
    lib = load_library()
    _require_device_tensor("patches", patches, (torch.uint16, torch.float32))
    if patches.dim() != 3 or patches.shape[1] != patches.shape[2] or patches.shape[0] % patches.shape[1]:
        raise ValueError("patches must be a stack (npatch * P, P, P)")
    P = patches.shape[1]
    npatch = patches.shape[0] // P
    shape = tuple(patches.shape)
    dev = patches.device
    _require_device_tensor("target_e3", target_e3, (torch.float32,), (3,) + shape)
    _require_device_tensor("target_fa", target_fa, (torch.float32,), shape)
    weight = _mask_arg(weight, shape)
    _require_device_tensor("params", params, (torch.float32,), (ST_SURROGATE_WEIGHTS,))
    if grad is None:
        grad = torch.empty(ST_SURROGATE_WEIGHTS, dtype=torch.float32, device=dev)
    if stats is None:
        stats = torch.empty(8, dtype=torch.float32, device=dev)
    _require_device_tensor("grad", grad, (torch.float32,), (ST_SURROGATE_WEIGHTS,))
    _require_device_tensor("stats", stats, (torch.float32,), (8,))
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        _require_device_tensor("workspace", workspace, (torch.uint8,))
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    with torch.cuda.device(dev):
        code = lib.st_surrogate_grad(_ptr(patches), ST_DTYPE_U16 if patches.dtype == torch.uint16 else ST_DTYPE_F32,
                                     npatch, P, _ptr(target_e3), _ptr(target_fa), _ptr(weight), _ptr(params),
                                     float(conf_weight), _ptr(grad), _ptr(stats), ws_ptr, ws_bytes,
                                     _stream_handle(dev))
    _check(code)
    return grad, stats


def st_surrogate_fallback_info() -> dict:
    """What this thread's last st_surrogate_infer did for its fallback: mode
    0 (none), 1 (flagged tiles) or 2 (whole volume), the tile edge, the crop
    count and the voxels the structure-tensor path ran on."""
    mode, edge = ctypes.c_int(0), ctypes.c_int(0)
    tiles, voxels = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().st_surrogate_fallback_info(ctypes.byref(mode), ctypes.byref(edge), ctypes.byref(tiles),
                                                     ctypes.byref(voxels)))
    return {"mode": mode.value, "tile_edge": edge.value, "tiles": tiles.value, "voxels": voxels.value}


def st_surrogate_grad_workspace_bytes(npatch: int, patch: int) -> int:
    return load_library().st_surrogate_grad_workspace_bytes(int(npatch), int(patch))


def st_surrogate_adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                      eps: float = 1e-8):
    """One Adam step on the surrogate's float32 weights (in place; see include/st.h)."""
    import torch
    lib = load_library()
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _require_device_tensor(name, t, (torch.float32,), (ST_SURROGATE_WEIGHTS,))
    with torch.cuda.device(params.device):
        code = lib.st_surrogate_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                                     float(beta2), float(eps), _stream_handle(params.device))
    _check(code)


def profile_enable(on: bool = True):
    _check(load_library().st_profile_enable(1 if on else 0))


def profile_reset():
    _check(load_library().st_profile_reset())


def profile_read() -> dict:
    """{kernel name: (total milliseconds, launches)} accumulated since the last reset."""
    lib = load_library()
    n = lib.st_profile_read(-1, None, 0, None, None)
    if n < 0:
        _check(-n)
    out = {}
    for i in range(n):
        buf = ctypes.create_string_buffer(64)
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        lib.st_profile_read(i, buf, 64, ctypes.byref(ms), ctypes.byref(cnt))
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out


class Batch:
    """A batch of independent volumes (e.g. halo-padded chunks of one scan) run
    through the st_compute path as one captured, replayable unit (``st_batch_*``).

    ``chunks``: sequence of dicts with ``volume`` (3-D uint16/float32 CUDA
    tensor), ``rho``, optional ``origin`` (z, y, x) of ``volume[0, 0, 0]`` in the
    axis' coordinates (default 0) and optional ``mask``.  Outputs (``outputs``
    names) are allocated here, or taken from ``results`` (one dict per chunk),
    and returned per chunk by :attr:`results`.
    ``lanes`` is the number of concurrent chains (1..ST_BATCH_MAX_LANES); 0 takes
    ST_BATCH_MAX_LANES chains with graph replay; ST_BATCH_GROUPED (-1) takes
    grouped launches (each pass one kernel over a round of chunks).
    """

    def __init__(self, chunks, sigma: float, truncate: float = 4.0, axis_center=None,
                 axis_direction=None, outputs: Iterable[str] = ("e3", "fa", "ha", "ia", "flags"),
                 lanes: int = 0, workspace=None, results=None):
        import torch
        lib = load_library()
        outputs = tuple(outputs)
        for k in outputs:
            if k not in ALL_OUTPUTS:
                raise ValueError(f"unknown output {k!r}")
        n = len(chunks)
        if n < 1:
            raise ValueError("need at least one chunk")
        arr = (StChunk * n)()
        self._keep = []
        self.results = []
        dev = None
        for i, c in enumerate(chunks):
            vol = c["volume"]
            _require_device_tensor(f"chunks[{i}].volume", vol, (torch.uint16, torch.float32))
            if vol.dim() != 3:
                raise ValueError("chunk volumes must be 3-D (nz, ny, nx)")
            dev = vol.device if dev is None else dev
            if vol.device != dev:
                raise ValueError("all chunks must be on one device")
            nz, ny, nx = vol.shape
            mask = c.get("mask")
            if mask is not None:
                _require_device_tensor(f"chunks[{i}].mask", mask, (torch.uint8, torch.bool), (nz, ny, nx))
                if mask.dtype == torch.bool:
                    mask = mask.view(torch.uint8)
            res = {}
            for k in outputs:
                shape = (3, nz, ny, nx) if k in ("e3", "evals") else (nz, ny, nx)
                dt = torch.uint8 if k == "flags" else torch.float32
                if results is not None:  # caller-supplied output tensors (e.g. another batch's)
                    _require_device_tensor(f"results[{i}][{k!r}]", results[i][k], (dt,), shape)
                    res[k] = results[i][k]
                else:
                    res[k] = torch.empty(shape, dtype=dt, device=dev)
            self.results.append(res)
            self._keep += [vol, mask]
            org = c.get("origin", (0.0, 0.0, 0.0))
            arr[i] = StChunk(vol.data_ptr(), ST_DTYPE_U16 if vol.dtype == torch.uint16 else ST_DTYPE_F32,
                             _ptr(mask), nz, ny, nx, float(c["rho"]), (ctypes.c_double * 3)(*map(float, org)),
                             _ptr(res.get("e3")), _ptr(res.get("evals")), _ptr(res.get("fa")),
                             _ptr(res.get("ha")), _ptr(res.get("ia")), _ptr(res.get("flags")))
        self.device = dev
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            _require_device_tensor("workspace", workspace, (torch.uint8,))
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
            self._keep.append(workspace)
        handle = ctypes.c_void_p()
        with torch.cuda.device(dev):
            code = lib.st_batch_create(arr, n, float(sigma), float(truncate), _vec3(axis_center),
                                       _vec3(axis_direction), int(lanes), ws_ptr, ws_bytes,
                                       ctypes.byref(handle))
        _check(code)
        self._h = handle

    @staticmethod
    def workspace_bytes(shapes, lanes: int = 0) -> int:
        """Workspace a batch of volumes of these (nz, ny, nx) shapes needs."""
        arr = (StChunk * len(shapes))()
        for i, (nz, ny, nx) in enumerate(shapes):
            arr[i].nz, arr[i].ny, arr[i].nx = int(nz), int(ny), int(nx)
        return load_library().st_batch_workspace_bytes(arr, len(shapes), int(lanes))

    def _handle(self):
        if self._h is None:
            raise RuntimeError("batch is closed")
        return self._h

    def launch(self):
        """Enqueue the batch on the device's current stream."""
        _check(load_library().st_batch_launch(self._handle(), _stream_handle(self.device)))

    def tune(self, reps: int = 2) -> dict:
        """Autotune tile shapes (per chunk), chain count, split targets and graph
        vs direct enqueue on the real chunks (synchronises); returns :meth:`config`."""
        _check(load_library().st_batch_tune(self._handle(), _stream_handle(self.device), int(reps)))
        return self.config()

    def plan(self) -> dict:
        """{"grouped": bool, "rounds": grouped-mode rounds, "kernels": launches per batch launch}."""
        g, r, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load_library().st_batch_plan(self._handle(), ctypes.byref(g), ctypes.byref(r), ctypes.byref(k)))
        return {"grouped": bool(g.value), "rounds": r.value, "kernels": k.value}

    def tiles(self, chunk: int) -> tuple:
        """(gradient tile rows, final-pass segment lanes) of a chunk; 0 = library default."""
        rows, lanes = ctypes.c_int(), ctypes.c_int()
        _check(load_library().st_batch_tiles(self._handle(), int(chunk), ctypes.byref(rows), ctypes.byref(lanes)))
        return rows.value, lanes.value

    def progress(self) -> tuple:
        """(done, launches): done[c] is True when chunk c's outputs of the latest
        launch are complete (read without waiting for the GPU)."""
        n = len(self.results)
        done = (ctypes.c_uint8 * n)()
        launches = ctypes.c_int64()
        _check(load_library().st_batch_progress(self._handle(), done, n, ctypes.byref(launches)))
        return [bool(d) for d in done], launches.value

    def config(self) -> dict:
        lanes, graph = ctypes.c_int(), ctypes.c_int()
        gb, sw, ms = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(load_library().st_batch_config(self._handle(), ctypes.byref(lanes), ctypes.byref(graph),
                                              ctypes.byref(gb), ctypes.byref(sw), ctypes.byref(ms)))
        return {"lanes": lanes.value, "graph": bool(graph.value), "grad_min_blocks": gb.value,
                "strided_min_waves": sw.value, "best_ms": ms.value}

    def close(self):
        if self._h is not None:
            _check(load_library().st_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
