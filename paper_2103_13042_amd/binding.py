"""ctypes binding of libspamm.so.

Argument marshalling only: every step of the SpAMM path runs in the library's
HIP kernels.  torch provides device memory (tensors) and the stream (the
current torch stream of the tensors' device).  If the library is not built,
importing this module raises ImportError: there is no fallback path.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "libspamm.so"

if not LIB_PATH.exists():
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_2103_13042_amd.build` (hipcc, gfx950) first"
    )

_lib = ctypes.CDLL(str(LIB_PATH))

_i64, _i32, _f64, _vp, _sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
_st = ctypes.c_int

_SIGS = {
    "spamm_bdim": (_i64, [_i64, _i32]),
    "spamm_levels": (_i32, [_i64, _i32]),
    "spamm_pyramid_size": (_i64, [_i64, _i32]),
    "spamm_leaf_supported": (_i32, [_i32]),
    "spamm_workspace_bytes": (_sz, [_i64, _i32]),
    "spamm_norms": (_st, [_vp, _i64, _i32, _vp, _vp]),
    "spamm_pyramid": (_st, [_vp, _i64, _i32, _vp, _vp, _sz, _vp]),
    "spamm_plan": (_st, [_vp, _vp, _i64, _i32, _f64, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_execute": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_schedule": (_st, [_vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "spamm_execute_scheduled": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_prepare": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_multiply": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _vp, _sz, _vp]),
    "spamm_search_valid_ratio": (_st, [_vp, _vp, _i64, _i32, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_strerror": (ctypes.c_char_p, [_st]),
    "spamm_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

STATUS = {0: "SPAMM_OK", 1: "SPAMM_EINVAL", 2: "SPAMM_ENOSPACE", 3: "SPAMM_EDEVICE", 4: "SPAMM_EUNSUPPORTED"}


class SpammError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _lib.spamm_last_error().decode()
        msg = _lib.spamm_strerror(status).decode()
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg}) {detail}".rstrip())


def _check(status: int, where: str) -> None:
    if status != 0:
        raise SpammError(status, where)


def library():
    """The loaded ctypes library (for tests of the raw C ABI)."""
    return _lib


# -- geometry (host only) ---------------------------------------------------


def bdim(n: int, leaf: int) -> int:
    return int(_lib.spamm_bdim(n, leaf))


def levels(n: int, leaf: int) -> int:
    return int(_lib.spamm_levels(n, leaf))


def pyramid_size(n: int, leaf: int) -> int:
    return int(_lib.spamm_pyramid_size(n, leaf))


def leaf_supported(leaf: int) -> bool:
    return bool(_lib.spamm_leaf_supported(leaf))


def workspace_bytes(n: int, leaf: int) -> int:
    return int(_lib.spamm_workspace_bytes(n, leaf))


# -- marshalling helpers ----------------------------------------------------


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p | None:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _square_f32(x: torch.Tensor, name: str) -> int:
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32 or x.dim() != 2 or x.shape[0] != x.shape[1] or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous square float32 matrix")
    return int(x.shape[0])


_WS: dict = {}


def workspace(n: int, leaf: int, device: torch.device) -> torch.Tensor:
    """A cached device workspace of at least workspace_bytes(n, leaf) bytes."""
    need = workspace_bytes(n, leaf)
    if need == 0:
        raise ValueError(f"no GPU workspace for n={n}, leaf={leaf} (size or tile grid out of range)")
    key = (device.index if device.index is not None else torch.cuda.current_device())
    ws = _WS.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        _WS[key] = ws
    return ws


# -- the entry points ---------------------------------------------------------


def norms(x: torch.Tensor, leaf: int) -> torch.Tensor:
    """Leaf-tile Frobenius norms, FP64 [bdim, bdim] (spamm_norms)."""
    n = _square_f32(x, "x")
    b = bdim(n, leaf)
    out = torch.empty((b, b), dtype=torch.float64, device=x.device)
    _check(_lib.spamm_norms(_ptr(x), n, leaf, _ptr(out), _stream(x.device)), "spamm_norms")
    return out


def pyramid(x: torch.Tensor, leaf: int, *, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Flat FP64 norm pyramid, level l at (4^l - 1)/3 (spamm_pyramid)."""
    n = _square_f32(x, "x")
    ws = workspace(n, leaf, x.device) if ws is None else ws
    out = torch.empty(pyramid_size(n, leaf), dtype=torch.float64, device=x.device)
    _check(
        _lib.spamm_pyramid(_ptr(x), n, leaf, _ptr(out), _ptr(ws), ws.numel(), _stream(x.device)),
        "spamm_pyramid",
    )
    return out


def pyramid_levels(flat: torch.Tensor, n: int, leaf: int) -> list[torch.Tensor]:
    """Split a flat pyramid into [2^l, 2^l] views, root first."""
    out, off = [], 0
    for l in range(levels(n, leaf) + 1):
        s = 1 << l
        out.append(flat[off : off + s * s].view(s, s))
        off += s * s
    return out


def plan(pyr_a: torch.Tensor, pyr_b: torch.Tensor, n: int, leaf: int, tau: float, *, ws: torch.Tensor | None = None):
    """Pruning plan: (offsets int32 [T+1], klist int32 [bdim^3], pairs int64 [1]) (spamm_plan)."""
    dev = pyr_a.device
    ws = workspace(n, leaf, dev) if ws is None else ws
    offsets, klist, pairs = plan_buffers(n, leaf, dev)
    _check(
        _lib.spamm_plan(
            _ptr(pyr_a), _ptr(pyr_b), n, leaf, float(tau), _ptr(offsets), _ptr(klist), klist.numel(),
            _ptr(pairs), _ptr(ws), ws.numel(), _stream(dev),
        ),
        "spamm_plan",
    )
    return offsets, klist, pairs


def plan_buffers(n: int, leaf: int, device: torch.device):
    """Output buffers of a plan: offsets [T+1], klist [bdim^3] (int32), pairs [1] (int64)."""
    b = bdim(n, leaf)
    return (
        torch.empty(b * b + 1, dtype=torch.int32, device=device),
        torch.empty(max(1, b**3), dtype=torch.int32, device=device),
        torch.empty(1, dtype=torch.int64, device=device),
    )


def prepare(a, b, tau: float, leaf: int, *, bufs=None, ws=None):
    """Norms, pyramids and plan of A and B (spamm_prepare): (offsets, klist, pairs)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    offsets, klist, pairs = plan_buffers(n, leaf, a.device) if bufs is None else bufs
    ws = workspace(n, leaf, a.device) if ws is None else ws
    _check(
        _lib.spamm_prepare(
            _ptr(a), _ptr(b), n, float(tau), leaf, _ptr(offsets), _ptr(klist), klist.numel(), _ptr(pairs),
            _ptr(ws), ws.numel(), _stream(a.device),
        ),
        "spamm_prepare",
    )
    return offsets, klist, pairs


def _check_plan(offsets, klist, n: int, leaf: int, dev) -> None:
    b = bdim(n, leaf)
    for name, t, need in (("offsets", offsets, b * b + 1), ("klist", klist, 1)):
        if t.dtype != torch.int32 or t.device != dev or not t.is_contiguous() or t.numel() < need:
            raise ValueError(f"{name}: expected a contiguous int32 tensor on {dev} with >= {need} entries")


def _mul_operands(a, b, leaf, offsets, klist, c, ws):
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n or b.device != a.device:
        raise ValueError("a and b must have the same size and device")
    _check_plan(offsets, klist, n, leaf, a.device)
    c = torch.empty_like(a) if c is None else c
    if _square_f32(c, "c") != n or c.device != a.device:
        raise ValueError("c must match a")
    ws = workspace(n, leaf, a.device) if ws is None else ws
    return n, c, ws


def execute(a, b, leaf: int, offsets, klist, *, c=None, ws=None) -> torch.Tensor:
    """Multiply the kept pairs of a plan into C (spamm_execute)."""
    n, c, ws = _mul_operands(a, b, leaf, offsets, klist, c, ws)
    _check(
        _lib.spamm_execute(
            _ptr(a), _ptr(b), n, leaf, _ptr(offsets), _ptr(klist), _ptr(c), _ptr(ws), ws.numel(), _stream(a.device)
        ),
        "spamm_execute",
    )
    return c


def schedule(offsets, klist, n: int, leaf: int, *, ws=None) -> None:
    """First launch step of execute: the multiply schedule into the workspace (spamm_schedule)."""
    dev = offsets.device
    _check_plan(offsets, klist, n, leaf, dev)
    ws = workspace(n, leaf, dev) if ws is None else ws
    _check(_lib.spamm_schedule(_ptr(offsets), _ptr(klist), n, leaf, _ptr(ws), ws.numel(), _stream(dev)),
           "spamm_schedule")


def execute_scheduled(a, b, leaf: int, offsets, klist, *, c=None, ws=None) -> torch.Tensor:
    """Second launch step of execute: the multiply kernel alone (spamm_execute_scheduled)."""
    n, c, ws = _mul_operands(a, b, leaf, offsets, klist, c, ws)
    _check(
        _lib.spamm_execute_scheduled(
            _ptr(a), _ptr(b), n, leaf, _ptr(offsets), _ptr(klist), _ptr(c), _ptr(ws), ws.numel(), _stream(a.device)
        ),
        "spamm_execute_scheduled",
    )
    return c


def multiply(a, b, tau: float, leaf: int, *, c=None, pairs=None, ws=None, sync: bool = True):
    """The whole hot path (spamm_multiply).  Returns (C, pairs); pairs is an int
    when sync is True (one device-to-host read), else the int64 device tensor."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    c = torch.empty_like(a) if c is None else c
    _square_f32(c, "c")
    pairs = torch.empty(1, dtype=torch.int64, device=a.device) if pairs is None else pairs
    ws = workspace(n, leaf, a.device) if ws is None else ws
    _check(
        _lib.spamm_multiply(
            _ptr(a), _ptr(b), n, float(tau), leaf, _ptr(c), _ptr(pairs), _ptr(ws), ws.numel(), _stream(a.device)
        ),
        "spamm_multiply",
    )
    return (c, int(pairs.item())) if sync else (c, pairs)


def search_valid_ratio(pyr_a, pyr_b, n: int, leaf: int, target: float, tol: float = 0.01, max_iters: int = 20,
                       *, ws=None):
    """tau for a requested valid ratio (spamm_search_valid_ratio): (tau, pairs, bisections)."""
    dev = pyr_a.device
    size = pyramid_size(n, leaf)
    for name, p in (("pyr_a", pyr_a), ("pyr_b", pyr_b)):
        if p.dtype != torch.float64 or not p.is_cuda or not p.is_contiguous() or p.numel() != size:
            raise ValueError(f"{name}: expected a contiguous CUDA float64 pyramid of {size} entries")
    ws = workspace(n, leaf, dev) if ws is None else ws
    tau = ctypes.c_double(0.0)
    pairs = ctypes.c_int64(0)
    iters = ctypes.c_int32(0)
    _check(
        _lib.spamm_search_valid_ratio(
            _ptr(pyr_a), _ptr(pyr_b), n, leaf, float(target), float(tol), int(max_iters), ctypes.byref(tau),
            ctypes.byref(pairs), ctypes.byref(iters), _ptr(ws), ws.numel(), _stream(dev),
        ),
        "spamm_search_valid_ratio",
    )
    return tau.value, pairs.value, iters.value
