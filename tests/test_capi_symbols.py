"""The C-ABI library loads and exports every function include/bem.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(bem_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("bem_create", "bem_destroy", "bem_last_error", "bem_check",
              "bem_assemble_nearfield", "bem_assemble_coupling", "bem_eval_entries"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1510_07244_amd as pk
    lib = ctypes.CDLL(pk.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the binding's ctypes structs equal those
    the C compiler gives the header's structs."""
    import subprocess
    import paper_1510_07244_amd as pk
    structs = [pk.bem_mesh, pk.bem_op, pk.bem_blocks, pk.bem_batch, pk.bem_tune]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bem.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append(f'  printf("{n} %zu\\n", sizeof({n}));')
        for f in st._fields_:
            lines.append(f'  printf("{n}.{f[0]} %zu\\n", offsetof({n}, {f[0]}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for st in structs:
        n = st.__name__
        assert int(got[n]) == ctypes.sizeof(st), n
        for f in st._fields_:
            assert int(got[f"{n}.{f[0]}"]) == getattr(st, f[0]).offset, (n, f[0])


def test_calls_reject_null_context_without_gpu():
    import paper_1510_07244_amd as pk
    lib = pk.lib()
    assert lib.bem_check(None, None) == pk.BEM_EINVAL
    assert lib.bem_assemble_nearfield(None, None, None, None, None, 0, None) == pk.BEM_EINVAL
    assert lib.bem_assemble_nearfield_both(None, None, None, None, None, None, 0,
                                           None) == pk.BEM_EINVAL
    assert lib.bem_eval_entries(None, None, None, 0, None, None, None, None) == pk.BEM_EINVAL
    assert lib.bem_last_error(None) == b"no context"
    assert lib.bem_plan_batched(None, None, 0, None, None, None, None, None) == pk.BEM_EINVAL
    assert lib.bem_run_batched(None, None) == pk.BEM_EINVAL
    assert lib.bem_plan_tiles(None) == 0
    lib.bem_destroy(None)
    lib.bem_plan_destroy(None)


def test_oracle_is_not_reachable_from_the_product_package():
    pkg = os.path.join(ROOT, "paper_1510_07244_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
