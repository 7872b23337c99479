"""The C-ABI library loads and exports every entry point include/ssa.h
declares; host-side argument checks work without a GPU."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssa.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssa_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2602_19775_amd import ssa
    if not os.path.exists(ssa.LIB_PATH):
        from paper_2602_19775_amd import build
        build.build()
    return ssa.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header():
    from paper_2602_19775_amd import ssa
    assert set(ssa.EXPORTS) == set(declared_functions())


def test_status_strings_and_defaults(L):
    from paper_2602_19775_amd import ssa
    for code in range(0, -8, -1):
        assert L.ssa_status_string(code)
    cfg = ssa._Cfg()
    L.ssa_config_default(C.byref(cfg))
    assert cfg.n_steps == 2 ** 31 - 1 and math.isinf(cfg.t_end) and cfg.ckpt_every == 256
    assert abs(cfg.temperature - 0.5) < 1e-7


def test_host_side_argument_errors(L):
    from paper_2602_19775_amd import ssa
    h = C.c_void_p()
    assert L.ssa_net_create(None, C.byref(h)) == -1
    d = ssa._Desc()
    d.n_networks = 0
    assert L.ssa_net_create(C.byref(d), C.byref(h)) == -1
    assert b"n_networks" in L.ssa_last_error()
    # NULL handles are rejected before any device work
    cfg = ssa._Cfg()
    L.ssa_config_default(C.byref(cfg))
    assert L.ssa_forward(None, C.byref(cfg), *([None] * 7), 0, None, None, None, 0, None) == -1
    assert L.ssa_backward(None, C.byref(cfg), *([None] * 6), 0, None, None, None, None, 0, None) == -1
    assert L.ssa_selftest_neglog(0, 1 << 24, None, None) == -1


def test_struct_sizes_match_header(L):
    """ctypes mirrors of the public structs have the C layout."""
    from paper_2602_19775_amd import ssa
    assert C.sizeof(ssa._Cfg) == 72
    assert ssa.TIE_DTYPE.itemsize == 24
    assert C.sizeof(ssa._Layout) == 40


def test_grn_host_side_checks(L):
    from paper_2602_19775_amd import ssa
    assert C.sizeof(ssa._GrnDesc) == 28
    h = C.c_void_p()
    d = ssa._GrnDesc(784, 128, 10, 4, 2, 10.0, 0.25)
    assert L.ssa_grn_create(C.byref(d), C.byref(h)) == -2          # hidden layer must be 256 wide
    assert b"256" in L.ssa_last_error()
    d = ssa._GrnDesc(784, 256, 17, 4, 2, 10.0, 0.25)
    assert L.ssa_grn_create(C.byref(d), C.byref(h)) == -2          # at most 16 output genes
    d = ssa._GrnDesc(784, 256, 10, 0, 2, 10.0, 0.25)
    assert L.ssa_grn_create(C.byref(d), C.byref(h)) == -1
    d = ssa._GrnDesc(784, 256, 10, 4, 2, -1.0, 0.25)
    assert L.ssa_grn_create(C.byref(d), C.byref(h)) == -1
    cfg = ssa._Cfg()
    L.ssa_config_default(C.byref(cfg))
    tb, wb = C.c_size_t(), C.c_size_t()
    assert L.ssa_grn_buffer_sizes(None, C.byref(cfg), C.byref(tb), C.byref(wb)) == -1
    assert L.ssa_grn_forward(None, C.byref(cfg), *([None] * 9), 0, None, None, None) == -1
    assert L.ssa_grn_backward(None, C.byref(cfg), *([None] * 7), 0, None, None, None, None, 0, None) == -1
