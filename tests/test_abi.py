"""The C ABI of libspamm.so on the host: every declared symbol is exported, the
host-only geometry queries are right, and argument checks reject bad calls
before anything is enqueued (these calls never reach the GPU)."""

from __future__ import annotations

import ctypes
import math
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADERS = sorted((ROOT / "include").glob("*.h"))


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names |= set(re.findall(r"\b(spamm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2103_13042_amd import binding

    return binding.library()


def test_header_declares_the_hot_path():
    names = _declared()
    for want in ("spamm_norms", "spamm_pyramid", "spamm_plan", "spamm_prepare", "spamm_execute", "spamm_multiply"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    assert len(HEADERS) >= 2
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    for want in ("spamm_search_valid_ratio", "spamm_search_tau_for_error", "spamm_mlp_loss_grad", "spamm_schedule"):
        assert want in _declared()


def test_geometry_queries(lib):
    from paper_2103_13042_amd import binding as b

    assert b.bdim(1024, 32) == 32 and b.bdim(1000, 64) == 16 and b.bdim(5, 8) == 1 and b.bdim(0, 32) == 0
    assert b.levels(1024, 32) == 5 and b.levels(1000, 64) == 4 and b.levels(5, 8) == 0 and b.levels(8192, 64) == 7
    assert b.pyramid_size(8192, 64) == sum(4**l for l in range(8)) == 21845
    assert b.pyramid_size(1100, 32) == sum(4**l for l in range(7))  # bdim 35 -> padded to 64
    assert [b.leaf_supported(x) for x in (16, 32, 64, 128, 48, 8)] == [True, True, True, True, False, False]
    ws = b.workspace_bytes(8192, 64)
    assert ws >= 4 * 128**3  # the worst-case k-list alone
    assert b.workspace_bytes(8192, 4) == 0  # 2048 tiles per side is over the limit
    assert b.workspace_bytes(-1, 64) == 0


def test_strerror(lib):
    for code in range(5):
        assert lib.spamm_strerror(code)
    assert lib.spamm_last_error() is not None


_FAKE_A, _FAKE_B, _FAKE_C, _FAKE_WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def _mul(lib, n=64, tau=1e-3, leaf=32, a=_FAKE_A, b=_FAKE_B, c=_FAKE_C, ws=_FAKE_WS, wsb=None):
    from paper_2103_13042_amd import binding as bd

    if wsb is None:
        wsb = bd.workspace_bytes(n, leaf) if n > 0 else 0
    vp = ctypes.c_void_p
    return lib.spamm_multiply(vp(a), vp(b), n, tau, leaf, vp(c), None, vp(ws), wsb, None)


def test_multiply_argument_checks(lib):
    # each case fails host-side validation, so the fake pointers are never used
    assert _mul(lib, n=0) == 1
    assert _mul(lib, tau=math.nan) == 1
    assert _mul(lib, tau=-1.0) == 1
    assert _mul(lib, a=0) == 1
    assert _mul(lib, c=_FAKE_A) == 1  # C aliases A
    assert _mul(lib, c=_FAKE_B + 4) == 1  # C overlaps B
    assert b"overlaps" in lib.spamm_last_error()
    assert _mul(lib, leaf=48, wsb=1 << 30) == 4  # no multiply kernel for this leaf
    assert _mul(lib, leaf=48, ws=0) == 4  # checked before a NULL workspace is resolved
    assert _mul(lib, wsb=16) == 2  # workspace too small
    assert b"needed" in lib.spamm_last_error()


def test_plan_capacity_check(lib):
    from paper_2103_13042_amd import binding as bd

    vp = ctypes.c_void_p
    n, leaf = 256, 32
    cap = bd.bdim(n, leaf) ** 3
    args = dict(wsb=bd.workspace_bytes(n, leaf))
    st = lib.spamm_plan(vp(1 << 28), vp(2 << 28), n, leaf, 1e-3, vp(3 << 28), vp(4 << 28), cap - 1, vp(5 << 28),
                        vp(6 << 28), args["wsb"], None)
    assert st == 2
    st = lib.spamm_plan(vp(1 << 28), vp(2 << 28), n, leaf, math.nan, vp(3 << 28), vp(4 << 28), cap, vp(5 << 28),
                        vp(6 << 28), args["wsb"], None)
    assert st == 1


def test_prepare_schedule_scales_checks_the_header_first(lib):
    # every case fails host-side validation before anything is enqueued, so
    # the fake pointers are never used
    from paper_2103_13042_amd import binding as bd

    vp = ctypes.c_void_p
    n, leaf = 1024, 64
    cap, wsb = bd.bdim(n, leaf) ** 3, bd.workspace_bytes(n, leaf)

    def call(header, header_bytes=256, n=n, leaf=leaf, a=_FAKE_A):
        return lib.spamm_prepare_schedule_scales(vp(a), vp(_FAKE_B), n, 1e-6, leaf, vp(3 << 28), vp(4 << 28), cap,
                                                 vp(5 << 28), vp(header), header_bytes, vp(_FAKE_WS), wsb, None)

    assert call(0) == 1  # null header
    assert call((6 << 28) + 16) == 1  # not 256-byte aligned
    assert call(6 << 28, header_bytes=255) == 2  # too small
    assert call(_FAKE_A + 4096) == 1  # inside A (4 MiB at n = 1024)
    assert b"overlaps" in lib.spamm_last_error()
    assert call(6 << 28, leaf=32) == 4  # FP16 hi+lo products need leaf 64
    assert call(6 << 28, n=1000) == 4  # and n a multiple of 128


def test_binding_rejects_cpu_tensors():
    import torch

    from paper_2103_13042_amd import binding as bd

    x = torch.zeros(8, 8)
    with pytest.raises(TypeError):
        bd.norms(x, 4)


def test_gfx950_code_has_no_packed_fp32_instructions():
    # v_pk_{fma,mul,add}_f32 are kept out of the library (the device pass gets
    # -packed-fp32-ops); checked on the gfx950 code objects of the last build
    from paper_2103_13042_amd import build as b

    if not list(b.BUILD.glob("*.hipfb")):
        pytest.skip("no device bundles in the build folder (library not built here)")
    assert b.packed_fp32_instructions() == []
