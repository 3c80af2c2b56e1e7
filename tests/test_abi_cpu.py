"""CPU checks of the C-ABI library: it loads, exports every declared entry point and
its struct layouts match the binding (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "celeste.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(celeste_[a-z_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = _declared()
    for n in ("celeste_elbo_eval", "celeste_newton_fit", "celeste_batch_fit", "celeste_ctx_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1611_03404_amd import celeste as cb
    lib = cb.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layouts_match_binding():
    from paper_1611_03404_amd import celeste as cb
    lib = cb.load()            # raises if sizes differ
    assert lib.celeste_struct_size(0) == 320
    assert lib.celeste_struct_size(99) == 0


def test_defaults_and_null_context_errors():
    from paper_1611_03404_amd import celeste as cb
    lib = cb.load()
    o = cb.default_opts()
    assert o.max_iter == 50 and o.delta0 == 1.0 and o.eta == pytest.approx(0.1)
    assert lib.celeste_ctx_set_option(None, 1, 4096) == cb.E_INVALID
    assert b"context" in lib.celeste_last_error()
    b = cb.CBatch()
    assert lib.celeste_elbo_eval(None, ctypes.byref(b), None, None, None, None, None) == cb.E_INVALID
    assert lib.celeste_elbo_eval_noalloc(None, ctypes.byref(b), None, None, None, None, None) == cb.E_INVALID
    assert lib.celeste_batch_fit(None, ctypes.byref(b), None, None, None, None) == cb.E_INVALID
    assert lib.celeste_autotune(None, ctypes.byref(b), None, 0, None, None) == cb.E_INVALID
    for opt, bad in ((cb.OPT_TILE_W, 12), (cb.OPT_VALUE_BLOCK, 64), (cb.OPT_VALUE_TILE_W, 4)):
        assert lib.celeste_ctx_set_option(None, opt, bad) == cb.E_INVALID
