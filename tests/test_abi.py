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
    assert cfg.d_temperature is None and cfg.d_epoch is None and cfg.selection == 0
    assert cfg.obs_layout == 0 and cfg.dobs_shared == 0


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


def test_struct_sizes_match_header(L, tmp_path):
    """ctypes mirrors of the public structs have the C layout: a C program
    built against include/ssa.h prints every size and field offset."""
    import shutil
    import subprocess
    from paper_2602_19775_amd import ssa
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"ssa_network_desc": ssa._Desc, "ssa_net_layout_t": ssa._Layout, "ssa_config": ssa._Cfg,
               "ssa_grn_desc": ssa._GrnDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#define __HIP_PLATFORM_AMD__ 1", '#include "ssa.h"',
             "int main(void) {"]
    for name, st in mirrors.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    for f in ssa.TIE_DTYPE.names:
        lines.append(f'printf("ssa_tie.{f} %zu\\n", offsetof(ssa_tie, {f}));')
    lines.append('printf("ssa_tie %zu\\n", sizeof(ssa_tie));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for name, st in mirrors.items():
        assert int(got[name]) == C.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)
    assert int(got["ssa_tie"]) == ssa.TIE_DTYPE.itemsize
    for f in ssa.TIE_DTYPE.names:
        assert int(got[f"ssa_tie.{f}"]) == ssa.TIE_DTYPE.fields[f][1], f


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
