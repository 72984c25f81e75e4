"""spamm_multiply_noalloc (include/spamm_noalloc.h) through the C ABI: the same
C and pair count as spamm_multiply with a caller workspace, on two calls in a
row whose second input is smaller (the static scratch keeps the first call's
contents), and ENOSPACE above the scratch size."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from paper_2103_13042_amd import binding as sp
from paper_2103_13042_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
SCRATCH_BYTES = 64 << 20


def _entry():
    fn = sp.library().spamm_multiply_noalloc
    vp = ctypes.c_void_p
    fn.restype = ctypes.c_int
    fn.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    return fn


def _noalloc(fn, a, b, tau, leaf):
    n = a.shape[0]
    c = torch.full_like(a, float("nan"))
    pairs = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    st = fn(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, tau, leaf,
            ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(pairs.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    assert st == 0, sp.library().spamm_last_error()
    torch.cuda.synchronize()
    return c, int(pairs.item())


@pytest.mark.parametrize("first,second", [((8192, 64, 1e-6, "alg"), (1000, 32, 1e-6, "exp")),
                                          ((4096, 32, 1e-6, "exp"), (1024, 16, 1e-5, "exp"))])
def test_noalloc_equals_multiply_on_two_calls(first, second):
    fn = _entry()
    for n, leaf, tau, kind in (first, second):  # the second input is smaller
        assert sp.workspace_bytes(n, leaf) <= SCRATCH_BYTES
        if kind == "alg":
            a, b = inputs.algebraic_decay_signed(n, 0), inputs.algebraic_decay_signed(n, 1)
        else:
            a, b = inputs.exp_decay(n, 0.05, 2), inputs.exp_decay(n, 0.05, 3)
        ga, gb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
        c_ref, p_ref = sp.multiply(ga, gb, tau, leaf)
        c, p = _noalloc(fn, ga, gb, tau, leaf)
        print(f"n={n} leaf={leaf} tau={tau:g}: pairs {p} (spamm_multiply {p_ref})", flush=True)
        assert p == p_ref
        # same kernels, same workspace layout and launch shapes: bitwise the same C
        assert torch.equal(c, c_ref)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    fn = _entry()
    a = torch.zeros(64, 64, device=DEV)
    n, leaf = 8192, 32  # 151 MiB of workspace
    assert sp.workspace_bytes(n, leaf) > SCRATCH_BYTES
    vp = ctypes.c_void_p
    st = fn(vp(a.data_ptr()), vp(a.data_ptr()), n, 1e-6, leaf, vp(a.data_ptr() + 4 * 64 * 64), None, None)
    assert st == 2  # ENOSPACE, checked before anything is enqueued
    assert b"static scratch" in sp.library().spamm_last_error()
