"""Every name that a function of the benchmark, the entry point, the package
or the oracle reads as a global is bound at module level or is a builtin (the
parser alone does not check this: a function that reads a name nothing binds
fails only when that line runs)."""
import builtins
import os
import symtable

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["bench.py", "__graft_entry__.py"] + [
    os.path.join(d, f) for d in ("paper_2602_19775_amd", "oracle")
    for f in sorted(os.listdir(os.path.join(ROOT, d))) if f.endswith(".py")]


def _unbound_globals(path):
    top = symtable.symtable(open(path).read(), path, "exec")
    bound = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    bound |= set(dir(builtins)) | {"__file__", "__name__", "__doc__"}
    out = []

    def walk(t):
        for c in t.get_children():
            if c.get_type() == "function":
                for s in c.get_symbols():
                    if (s.is_global() or (s.is_referenced() and not s.is_local() and not s.is_free())) \
                            and s.is_referenced() and s.get_name() not in bound:
                        out.append(f"{c.get_name()}:{c.get_lineno()}: {s.get_name()}")
            walk(c)
    walk(top)
    return out


@pytest.mark.parametrize("rel", FILES)
def test_globals_are_bound(rel):
    assert _unbound_globals(os.path.join(ROOT, rel)) == []
