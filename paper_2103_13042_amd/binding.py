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
_f32 = ctypes.c_float

_SIGS = {
    "spamm_bdim": (_i64, [_i64, _i32]),
    "spamm_levels": (_i32, [_i64, _i32]),
    "spamm_pyramid_size": (_i64, [_i64, _i32]),
    "spamm_leaf_supported": (_i32, [_i32]),
    "spamm_release": (_st, []),
    "spamm_workspace_bytes": (_sz, [_i64, _i32]),
    "spamm_norms": (_st, [_vp, _i64, _i32, _vp, _vp]),
    "spamm_pyramid": (_st, [_vp, _i64, _i32, _vp, _vp, _sz, _vp]),
    "spamm_plan": (_st, [_vp, _vp, _i64, _i32, _f64, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_execute": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_schedule": (_st, [_vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "spamm_execute_scheduled": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_prepare": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_multiply": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _vp, _sz, _vp]),
    "spamm_prepare_schedule": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_search_valid_ratio": (_st, [_vp, _vp, _i64, _i32, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_mlp_param_count": (_i64, []),
    "spamm_mlp_acts_floats": (_i64, [_i32]),
    "spamm_tau_features": (_st, [_vp, _vp, _i64, _i32, _f64, _vp, _vp]),
    "spamm_mlp_forward": (_st, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "spamm_mlp_loss_grad": (_st, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "spamm_mlp_adam": (_st, [_vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _vp]),
    "spamm_sumsq_scratch_bytes": (_sz, []),
    "spamm_sumsq": (_st, [_vp, _i64, _vp, _vp, _sz, _vp]),
    "spamm_error_for_tau": (_st, [_vp, _vp, _i64, _i32, _f64, _vp, _vp, _f64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_search_tau_for_error": (
        _st, [_vp, _vp, _i64, _i32, _f64, _f64, _i32, _vp, _vp, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_split_bytes": (_sz, [_i64, _i32]),
    "spamm_split": (_st, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "spamm_execute_split": (_st, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_execute_split_scheduled": (_st, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_split_scales": (_st, [_vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "spamm_prepare_scales": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp, _sz, _vp]),
    "spamm_prepare_schedule_scales": (_st, [_vp, _vp, _i64, _f64, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp, _sz,
                                            _vp]),
    "spamm_execute_f16x3_scheduled": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_execute_bf16_scheduled": (_st, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_prepare_split": (_st, [_vp, _vp, _i64, _f64, _i32, _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp, _sz, _vp]),
    "spamm_multiply_precision": (_st, [_vp, _vp, _i64, _f64, _i32, _i32, _vp, _vp, _vp, _sz, _vp, _sz, _vp]),
    "spamm_batch_workspace_bytes": (_sz, [_i32, _vp, _vp]),
    "spamm_batch_setup": (_st, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spamm_batch_run": (_st, [_i32, _vp, _vp, _vp, _sz, _vp]),
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


def release() -> None:
    """Free the library's cached per-device workspaces (spamm_release)."""
    _check(_lib.spamm_release(), "spamm_release")


# passed as ws= to multiply(): the library's own cached workspace of the device
# (a NULL workspace pointer at the C ABI)
LIBRARY_WORKSPACE = "library"


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


def prepare(a, b, tau: float, leaf: int, *, bufs=None, ws=None, schedule: bool = False):
    """Norms, pyramids and plan of A and B (spamm_prepare; with schedule=True
    also the multiply schedule, spamm_prepare_schedule): (offsets, klist, pairs)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    offsets, klist, pairs = plan_buffers(n, leaf, a.device) if bufs is None else bufs
    ws = workspace(n, leaf, a.device) if ws is None else ws
    fn, name = ((_lib.spamm_prepare_schedule, "spamm_prepare_schedule") if schedule
                else (_lib.spamm_prepare, "spamm_prepare"))
    _check(
        fn(
            _ptr(a), _ptr(b), n, float(tau), leaf, _ptr(offsets), _ptr(klist), klist.numel(), _ptr(pairs),
            _ptr(ws), ws.numel(), _stream(a.device),
        ),
        name,
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
    if isinstance(ws, str) and ws == LIBRARY_WORKSPACE:
        ws_ptr, ws_bytes = None, 0
    else:
        ws = workspace(n, leaf, a.device) if ws is None else ws
        ws_ptr, ws_bytes = _ptr(ws), ws.numel()
    _check(
        _lib.spamm_multiply(
            _ptr(a), _ptr(b), n, float(tau), leaf, _ptr(c), _ptr(pairs), ws_ptr, ws_bytes, _stream(a.device)
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


# -- threshold for an error target, and the network that predicts it -------


def mlp_param_count() -> int:
    return int(_lib.spamm_mlp_param_count())


def _dev_f32(t, name: str, numel: int | None = None):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous CUDA float32 tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs >= {numel} entries")


def mlp_acts(batch: int, device) -> torch.Tensor:
    return torch.empty(int(_lib.spamm_mlp_acts_floats(batch)), dtype=torch.float32, device=device)


def tau_features(pyr_a, pyr_b, n: int, leaf: int, target: float, *, out=None) -> torch.Tensor:
    """FP32 [129] features of one problem (spamm_tau_features)."""
    dev = pyr_a.device
    out = torch.empty(129, dtype=torch.float32, device=dev) if out is None else out
    _dev_f32(out, "out", 129)
    _check(_lib.spamm_tau_features(_ptr(pyr_a), _ptr(pyr_b), n, leaf, float(target), _ptr(out), _stream(dev)),
           "spamm_tau_features")
    return out


def mlp_forward(params, x, *, y=None, acts=None) -> torch.Tensor:
    """Predicted log10(tau) for rows x [B, 129] (spamm_mlp_forward)."""
    batch = x.shape[0]
    _dev_f32(params, "params", mlp_param_count())
    _dev_f32(x, "x", batch * 129)
    y = torch.empty(batch, dtype=torch.float32, device=x.device) if y is None else y
    acts = mlp_acts(batch, x.device) if acts is None else acts
    _dev_f32(y, "y", batch)
    _dev_f32(acts, "acts", int(_lib.spamm_mlp_acts_floats(batch)))
    _check(_lib.spamm_mlp_forward(_ptr(params), _ptr(x), batch, _ptr(y), _ptr(acts), _stream(x.device)),
           "spamm_mlp_forward")
    return y


def mlp_loss_grad(params, x, t, *, acts=None, grad=None, loss=None):
    """(loss [1], grad [P]) of the mean squared log10(tau) error (spamm_mlp_loss_grad)."""
    batch = x.shape[0]
    _dev_f32(params, "params", mlp_param_count())
    _dev_f32(x, "x", batch * 129)
    _dev_f32(t, "t", batch)
    acts = mlp_acts(batch, x.device) if acts is None else acts
    grad = torch.empty_like(params) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=x.device) if loss is None else loss
    _dev_f32(acts, "acts", int(_lib.spamm_mlp_acts_floats(batch)))
    _dev_f32(grad, "grad", mlp_param_count())
    _dev_f32(loss, "loss", 1)
    _check(_lib.spamm_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(t), batch, _ptr(acts), _ptr(grad), _ptr(loss),
                                    _stream(x.device)), "spamm_mlp_loss_grad")
    return loss, grad


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8) -> None:
    """One Adam step in place on params, m, v (spamm_mlp_adam)."""
    p = mlp_param_count()
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _dev_f32(t, name, p)
    _check(_lib.spamm_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(params.device)), "spamm_mlp_adam")


def sumsq(x, *, out=None, scratch=None) -> torch.Tensor:
    """Sum of squares of an FP32 tensor in FP64, as a device tensor [1] (spamm_sumsq)."""
    _dev_f32(x, "x")
    dev = x.device
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    nb = int(_lib.spamm_sumsq_scratch_bytes())
    scratch = torch.empty(nb, dtype=torch.uint8, device=dev) if scratch is None else scratch
    _check(_lib.spamm_sumsq(_ptr(x), x.numel(), _ptr(out), _ptr(scratch), scratch.numel(), _stream(dev)),
           "spamm_sumsq")
    return out


def _tau_args(a, b, leaf, pyr_a, pyr_b, e, ws):
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    size = pyramid_size(n, leaf)
    for name, p in (("pyr_a", pyr_a), ("pyr_b", pyr_b)):
        if p.dtype != torch.float64 or not p.is_cuda or not p.is_contiguous() or p.numel() != size:
            raise ValueError(f"{name}: expected a contiguous CUDA float64 pyramid of {size} entries")
    e = torch.empty_like(a) if e is None else e
    _square_f32(e, "e")
    ws = workspace(n, leaf, a.device) if ws is None else ws
    return n, e, ws


def error_for_tau(a, b, tau: float, leaf: int, pyr_a, pyr_b, ab_sumsq: float, *, e=None, ws=None):
    """(||AB - SpAMM||_F / ||AB||_F, dropped triples) at tau (spamm_error_for_tau)."""
    n, e, ws = _tau_args(a, b, leaf, pyr_a, pyr_b, e, ws)
    err = ctypes.c_double(0.0)
    dropped = ctypes.c_int64(0)
    _check(_lib.spamm_error_for_tau(_ptr(a), _ptr(b), n, leaf, float(tau), _ptr(pyr_a), _ptr(pyr_b),
                                    float(ab_sumsq), _ptr(e), ctypes.byref(err), ctypes.byref(dropped), _ptr(ws),
                                    ws.numel(), _stream(a.device)), "spamm_error_for_tau")
    return err.value, dropped.value


def search_tau_for_error(a, b, leaf: int, target: float, pyr_a, pyr_b, ab_sumsq: float, *, guess: float = 0.0,
                         max_evals: int = 64, e=None, ws=None):
    """Largest norm product tau with relative error <= target: (tau, err, pairs, evals)
    (spamm_search_tau_for_error)."""
    n, e, ws = _tau_args(a, b, leaf, pyr_a, pyr_b, e, ws)
    tau, err = ctypes.c_double(0.0), ctypes.c_double(0.0)
    pairs, evals = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(_lib.spamm_search_tau_for_error(
        _ptr(a), _ptr(b), n, leaf, float(target), float(guess), int(max_evals), _ptr(pyr_a), _ptr(pyr_b),
        float(ab_sumsq), _ptr(e), ctypes.byref(tau), ctypes.byref(err), ctypes.byref(pairs), ctypes.byref(evals),
        _ptr(ws), ws.numel(), _stream(a.device)), "spamm_search_tau_for_error")
    return tau.value, err.value, pairs.value, evals.value


# -- reduced-precision leaf products -----------------------------------------

PRECISIONS = {"fp32": 0, "bf16": 1, "f16x3": 2}


def _prec(precision) -> int:
    if isinstance(precision, str):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[precision]
    return int(precision)


def split_bytes(n: int, precision) -> int:
    return int(_lib.spamm_split_bytes(n, _prec(precision)))


def split_buffer(n: int, precision, device) -> torch.Tensor:
    """A device buffer for the split operands (torch allocations are 256-byte aligned)."""
    nb = split_bytes(n, precision)
    if nb == 0:
        raise ValueError("no split operands for this precision")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def split_views(buf: torch.Tensor, n: int, precision):
    """(exps int32 [2], planes: list of int16 [n, n] views: A hi, [A lo], Bt hi, [Bt lo])."""
    p = _prec(precision)
    exps = buf[:8].view(torch.int32)
    plane = (n * n * 2 + 255) // 256 * 256
    count = 4 if p == 2 else 2
    planes = [buf[256 + q * plane : 256 + q * plane + n * n * 2].view(torch.int16).view(n, n) for q in range(count)]
    return exps, planes


def split(a, b, leaf: int, precision, pyr_a, pyr_b, *, out=None) -> torch.Tensor:
    """Split operands of A and B (spamm_split)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    out = split_buffer(n, precision, a.device) if out is None else out
    _check(_lib.spamm_split(_ptr(a), _ptr(b), n, leaf, _prec(precision), _ptr(pyr_a), _ptr(pyr_b), _ptr(out),
                            out.numel(), _stream(a.device)), "spamm_split")
    return out


def execute_split(split_buf, n: int, leaf: int, precision, offsets, klist, *, c=None, ws=None,
                  scheduled: bool = False) -> torch.Tensor:
    """Reduced-precision multiply of a plan (spamm_execute_split, or with
    scheduled=True spamm_execute_split_scheduled after schedule())."""
    dev = split_buf.device
    _check_plan(offsets, klist, n, leaf, dev)
    c = torch.empty((n, n), dtype=torch.float32, device=dev) if c is None else c
    if _square_f32(c, "c") != n:
        raise ValueError("c must be n x n")
    ws = workspace(n, leaf, dev) if ws is None else ws
    fn = _lib.spamm_execute_split_scheduled if scheduled else _lib.spamm_execute_split
    _check(fn(_ptr(split_buf), n, leaf, _prec(precision), _ptr(offsets), _ptr(klist), _ptr(c), _ptr(ws), ws.numel(),
              _stream(dev)), "spamm_execute_split")
    return c


def split_scales(pyr_a, pyr_b, n: int, leaf: int, header=None) -> torch.Tensor:
    """The f16x3 scale exponents into a 256-byte header (spamm_split_scales)."""
    dev = pyr_a.device
    header = torch.empty(256, dtype=torch.uint8, device=dev) if header is None else header
    _check(_lib.spamm_split_scales(_ptr(pyr_a), _ptr(pyr_b), n, leaf, _ptr(header), header.numel(), _stream(dev)),
           "spamm_split_scales")
    return header


def prepare_scales(a, b, tau: float, leaf: int, header, *, bufs=None, ws=None, schedule: bool = False):
    """spamm_prepare + spamm_split_scales on the workspace pyramids (with
    schedule=True spamm_prepare_schedule_scales: also the multiply schedule,
    from the one-launch plan): (offsets, klist, pairs)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    dev = a.device
    ws = workspace(n, leaf, dev) if ws is None else ws
    offsets, klist, pairs = plan_buffers(n, leaf, dev) if bufs is None else bufs
    fn, name = ((_lib.spamm_prepare_schedule_scales, "spamm_prepare_schedule_scales") if schedule
                else (_lib.spamm_prepare_scales, "spamm_prepare_scales"))
    _check(fn(_ptr(a), _ptr(b), n, float(tau), leaf, _ptr(offsets), _ptr(klist), klist.numel(), _ptr(pairs),
              _ptr(header), header.numel(), _ptr(ws), ws.numel(), _stream(dev)),
           name)
    return offsets, klist, pairs


def execute_f16x3(a, b, leaf: int, header, offsets, klist, *, c=None, ws=None) -> torch.Tensor:
    """f16x3 products straight from the FP32 inputs after schedule()
    (spamm_execute_f16x3_scheduled)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    dev = a.device
    _check_plan(offsets, klist, n, leaf, dev)
    c = torch.empty_like(a) if c is None else c
    if _square_f32(c, "c") != n:
        raise ValueError("c must be n x n")
    ws = workspace(n, leaf, dev) if ws is None else ws
    _check(_lib.spamm_execute_f16x3_scheduled(_ptr(a), _ptr(b), n, leaf, _ptr(header), _ptr(offsets), _ptr(klist),
                                              _ptr(c), _ptr(ws), ws.numel(), _stream(dev)),
           "spamm_execute_f16x3_scheduled")
    return c


def execute_bf16(a, b, leaf: int, offsets, klist, *, c=None, ws=None) -> torch.Tensor:
    """BF16 products straight from the FP32 inputs after prepare() and
    schedule() (spamm_execute_bf16_scheduled)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    dev = a.device
    _check_plan(offsets, klist, n, leaf, dev)
    c = torch.empty_like(a) if c is None else c
    if _square_f32(c, "c") != n:
        raise ValueError("c must be n x n")
    ws = workspace(n, leaf, dev) if ws is None else ws
    _check(_lib.spamm_execute_bf16_scheduled(_ptr(a), _ptr(b), n, leaf, _ptr(offsets), _ptr(klist), _ptr(c),
                                             _ptr(ws), ws.numel(), _stream(dev)),
           "spamm_execute_bf16_scheduled")
    return c


def multiply_precision(a, b, tau: float, leaf: int, precision, *, c=None, pairs=None, split_buf=None, ws=None,
                       sync: bool = True):
    """The whole path with reduced-precision products (spamm_multiply_precision): (C, pairs)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    dev = a.device
    p = _prec(precision)
    c = torch.empty_like(a) if c is None else c
    pairs = torch.empty(1, dtype=torch.int64, device=dev) if pairs is None else pairs
    ws = workspace(n, leaf, dev) if ws is None else ws
    if split_buf is None and p in (1, 2):
        split_buf = split_buffer(n, p, dev)
    _check(_lib.spamm_multiply_precision(_ptr(a), _ptr(b), n, float(tau), leaf, p, _ptr(c), _ptr(pairs),
                                         _ptr(split_buf), split_buf.numel() if split_buf is not None else 0,
                                         _ptr(ws), ws.numel(), _stream(dev)), "spamm_multiply_precision")
    return (c, int(pairs.item())) if sync else (c, pairs)


def prepare_split(a, b, tau: float, leaf: int, precision, split_buf, *, bufs=None, ws=None):
    """spamm_prepare + spamm_split on the workspace pyramids: (offsets, klist, pairs)."""
    n = _square_f32(a, "a")
    if _square_f32(b, "b") != n:
        raise ValueError("a and b must have the same size")
    dev = a.device
    ws = workspace(n, leaf, dev) if ws is None else ws
    offsets, klist, pairs = plan_buffers(n, leaf, dev) if bufs is None else bufs
    _check(_lib.spamm_prepare_split(_ptr(a), _ptr(b), n, float(tau), leaf, _prec(precision), _ptr(offsets),
                                    _ptr(klist), klist.numel(), _ptr(pairs), _ptr(split_buf), split_buf.numel(),
                                    _ptr(ws), ws.numel(), _stream(dev)), "spamm_prepare_split")
    return offsets, klist, pairs


# -- batches of independent products ------------------------------------------


class Batch:
    """A batch bound to its device matrices (spamm_batch_setup); run() enqueues
    the whole batch (spamm_batch_run) and can be captured in a graph."""

    def __init__(self, a_list, b_list, leaves, taus, *, c_list=None):
        count = len(a_list)
        if not (len(b_list) == len(leaves) == len(taus) == count) or count == 0:
            raise ValueError("a, b, leaves and taus must have the same non-zero length")
        dev = a_list[0].device
        ns = []
        for i, (a, b) in enumerate(zip(a_list, b_list)):
            n = _square_f32(a, f"a[{i}]")
            if _square_f32(b, f"b[{i}]") != n or a.device != dev or b.device != dev:
                raise ValueError(f"product {i}: a and b must be square of the same size on one device")
            ns.append(n)
        self.a, self.b = list(a_list), list(b_list)
        self.c = [torch.empty_like(a) for a in a_list] if c_list is None else list(c_list)
        self.count, self.device = count, dev
        self._n = (ctypes.c_int64 * count)(*ns)
        self._leaf = (ctypes.c_int32 * count)(*[int(v) for v in leaves])
        self._tau = (ctypes.c_double * count)(*[float(v) for v in taus])
        nb = int(_lib.spamm_batch_workspace_bytes(count, self._n, self._leaf))
        if nb == 0:
            _check(_lib.spamm_batch_setup(count, None, None, None, self._n, self._leaf, self._tau, None, None, 0,
                                          None), "spamm_batch_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.pairs = torch.zeros(count, dtype=torch.int64, device=dev)
        ptrs = lambda ts: (ctypes.c_void_p * count)(*[t.data_ptr() for t in ts])
        _check(_lib.spamm_batch_setup(count, ptrs(self.a), ptrs(self.b), ptrs(self.c), self._n, self._leaf,
                                      self._tau, _ptr(self.pairs), _ptr(self.ws), self.ws.numel(), _stream(dev)),
               "spamm_batch_setup")

    def run(self):
        _check(_lib.spamm_batch_run(self.count, self._n, self._leaf, _ptr(self.ws), self.ws.numel(),
                                    _stream(self.device)), "spamm_batch_run")
        return self.c
