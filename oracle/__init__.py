"""FP64 CPU oracle for SpAMM (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path never does.  The arithmetic lives in
``spamm_oracle.c`` (plain C, FP64); this module marshals numpy arrays to it.

Functions follow the paper's section 2.1: Eq. 1 (quadtree), Eq. 2 (Frobenius
norm of a node) and Algorithm 1 (recursive SpAMM, with the root pair tested).
"""

from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
# SPAMM_ORACLE_LIB selects another build of the same source (the sanitizer
# variant of oracle/build.py, for running the pin tests under ASan/UBSan)
LIB_PATH = Path(os.environ.get("SPAMM_ORACLE_LIB", _HERE / "libspamm_oracle.so"))
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        from . import build as _build

        _build.build_oracle()
    return _bind(ctypes.CDLL(str(LIB_PATH)))


def use_native_build() -> Path:
    """Switch to the -O3 -march=native build of the oracle, compiled now on the
    host that runs it (a build from another host may use instructions this one
    lacks): for timing it as a CPU baseline.  The arithmetic is the same C
    source with the same FP flags."""
    global _lib
    from . import build as _build

    path = _build.build_oracle(native=True)
    _lib = None
    _lib = _bind(ctypes.CDLL(str(path)))
    return path


def _bind(lib):
    global _lib
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    vp = ctypes.c_void_p
    lib.oracle_bdim.argtypes = [i64, i32]
    lib.oracle_bdim.restype = i64
    lib.oracle_levels.argtypes = [i64, i32]
    lib.oracle_levels.restype = i32
    lib.oracle_pyramid_size.argtypes = [i64, i32]
    lib.oracle_pyramid_size.restype = i64
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = i32
    lib.oracle_pyramid.argtypes = [vp, i64, i32, vp]
    lib.oracle_pyramid.restype = ctypes.c_int
    lib.oracle_spamm_tiles.argtypes = [vp, vp, i64, i32, f64, vp, vp, vp, i64, vp, vp, vp]
    lib.oracle_spamm_tiles.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _as_f32(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim != 2 or x.shape[0] != x.shape[1]:
        raise ValueError("expected a square matrix")
    return x


def bdim(n: int, leaf: int) -> int:
    """ceil(N / leaf): leaf tiles per side."""
    return int(_load().oracle_bdim(n, leaf))


def levels(n: int, leaf: int) -> int:
    """Lv = ceil(log2(bdim)): depth of the quadtree (Eq. 1) above the leaf tiles."""
    return int(_load().oracle_levels(n, leaf))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def pyramid(x, leaf: int) -> list[np.ndarray]:
    """Frobenius norm (Eq. 2) of every quadtree node (Eq. 1), root first.

    Level l is a 2^l x 2^l array; the last level is the leaf-tile grid padded to a
    power of two (padding tiles have norm 0).  Every node is summed directly from
    the matrix elements.
    """
    x = _as_f32(x)
    n = x.shape[0]
    lib = _load()
    flat = np.zeros(int(lib.oracle_pyramid_size(n, leaf)), dtype=np.float64)
    if lib.oracle_pyramid(_ptr(x), n, leaf, _ptr(flat)) != 0:
        raise ValueError("oracle_pyramid: bad arguments")
    out, off = [], 0
    for l in range(levels(n, leaf) + 1):
        side = 1 << l
        out.append(flat[off : off + side * side].reshape(side, side))
        off += side * side
    return out


def _flat(pyr: list[np.ndarray]) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([p.ravel() for p in pyr]), dtype=np.float64)


def leaf_norms(x, leaf: int) -> np.ndarray:
    """Frobenius norm of every leaf tile, bdim x bdim (padding tiles excluded)."""
    x = _as_f32(x)
    b = bdim(x.shape[0], leaf)
    return pyramid(x, leaf)[-1][:b, :b].copy()


def spamm_tiles(a, b, tau: float, leaf: int, tiles, *, products: bool = True, pyr_a=None, pyr_b=None):
    """Algorithm 1 restricted to the listed output leaf tiles.

    Returns (ctiles [ntiles, leaf, leaf] FP64 or None, counts [ntiles], mask
    [ntiles, bdim] bool).  mask[t, k] is True when the leaf pair
    (A[ti,k], B[k,tj]) was multiplied.
    """
    a, b = _as_f32(a), _as_f32(b)
    n = a.shape[0]
    if b.shape[0] != n:
        raise ValueError("A and B must have the same size")
    tiles = np.ascontiguousarray(np.asarray(tiles, dtype=np.int64).reshape(-1, 2))
    nt = tiles.shape[0]
    bd = bdim(n, leaf)
    pa = _flat(pyr_a if pyr_a is not None else pyramid(a, leaf))
    pb = _flat(pyr_b if pyr_b is not None else pyramid(b, leaf))
    ctiles = np.zeros((nt, leaf, leaf), dtype=np.float64) if products else None
    mask = np.zeros((nt, bd), dtype=np.uint8)
    counts = np.zeros(nt, dtype=np.int64)
    rc = _load().oracle_spamm_tiles(
        _ptr(a), _ptr(b), n, leaf, float(tau), _ptr(pa), _ptr(pb), _ptr(tiles), nt,
        _ptr(ctiles), _ptr(mask), _ptr(counts),
    )
    if rc != 0:
        raise ValueError(f"oracle_spamm_tiles failed with code {rc}")
    return ctiles, counts, mask.astype(bool)


def all_tiles(n: int, leaf: int) -> np.ndarray:
    b = bdim(n, leaf)
    ii, jj = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1)


def spamm(a, b, tau: float, leaf: int, *, products: bool = True):
    """Full SpAMM of A and B (Algorithm 1 with the root pair tested).

    Returns (C [N, N] FP64 or None, pairs, mask [bdim, bdim, bdim] bool indexed
    (i, j, k)).
    """
    a = _as_f32(a)
    n = a.shape[0]
    bd = bdim(n, leaf)
    tiles = all_tiles(n, leaf)
    ct, counts, mask = spamm_tiles(a, b, tau, leaf, tiles, products=products)
    c = None
    if products:
        p = bd * leaf
        full = ct.reshape(bd, bd, leaf, leaf).transpose(0, 2, 1, 3).reshape(p, p)
        c = np.ascontiguousarray(full[:n, :n])
    return c, int(counts.sum()), mask.reshape(bd, bd, bd)


def tiles_to_matrix_view(ctiles: np.ndarray, tiles: np.ndarray, n: int, leaf: int):
    """Crop each tile to the real N x N region: list of (r0, c0, block)."""
    out = []
    for t, (ti, tj) in enumerate(np.asarray(tiles).reshape(-1, 2)):
        r0, c0 = int(ti) * leaf, int(tj) * leaf
        r1, c1 = min(n, r0 + leaf), min(n, c0 + leaf)
        out.append((r0, c0, ctiles[t, : r1 - r0, : c1 - c0]))
    return out


def threads_env() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v and v.isdigit() else max_threads()


def mean_norm_product(a, b, leaf: int) -> float:
    """Mean of nA[i,k] * nB[k,j] over every leaf triple (i, k, j) of the real
    bdim^3 grid: the `ave` of the valid-ratio search (section 3.5.2)."""
    na, nb = leaf_norms(a, leaf), leaf_norms(b, leaf)
    prods = na[:, :, None] * nb[None, :, :]  # [i, k, j]
    return float(prods.sum() / prods.size)


def valid_ratio(a, b, tau: float, leaf: int, *, pyr_a=None, pyr_b=None) -> tuple[float, int]:
    """Fraction of leaf triples multiplied at tau, and their number (section 3.5.2)."""
    a = _as_f32(a)
    n = a.shape[0]
    bd = bdim(n, leaf)
    _, counts, _ = spamm_tiles(a, b, tau, leaf, all_tiles(n, leaf), products=False, pyr_a=pyr_a, pyr_b=pyr_b)
    c = int(counts.sum())
    return c / bd**3, c


def search_tau_for_valid_ratio(a, b, leaf: int, target: float, tol: float = 0.01, max_iters: int = 20,
                               max_expand: int = 1024):
    """The valid-ratio search of section 3.5.2: the first tau tried is ave (the
    mean norm product); while the ratio at the upper bound k*ave is still above
    the target (plus tol), k grows to k+1 (at most max_expand); then tau is
    bisected in [0, k*ave] until the ratio is within tol of the target or
    max_iters bisections ran.
    Returns (tau, pairs, bisections)."""
    pa, pb = pyramid(a, leaf), pyramid(b, leaf)
    ave = mean_norm_product(a, b, leaf)

    def ratio(t):
        return valid_ratio(a, b, t, leaf, pyr_a=pa, pyr_b=pb)

    k = 1
    hi = k * ave
    r, cnt = ratio(hi)
    while r > target + tol and k < max_expand:
        k += 1
        hi = k * ave
        r, cnt = ratio(hi)
    tau = hi
    lo = 0.0
    it = 0
    while abs(r - target) > tol and it < max_iters:
        mid = 0.5 * (lo + hi)
        r, cnt = ratio(mid)
        tau = mid
        it += 1
        if r > target:
            lo = mid
        else:
            hi = mid
    return tau, cnt, it
