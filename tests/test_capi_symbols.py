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


def test_struct_layouts_match_header():
    import paper_1510_07244_amd as pk
    assert ctypes.sizeof(pk.bem_mesh) == 32
    assert ctypes.sizeof(pk.bem_op) == 6 * 4 + 2 * 8 + 4 * 4
    assert ctypes.sizeof(pk.bem_blocks) == 64


def test_calls_reject_null_context_without_gpu():
    import paper_1510_07244_amd as pk
    lib = pk.lib()
    assert lib.bem_check(None, None) == pk.BEM_EINVAL
    assert lib.bem_assemble_nearfield(None, None, None, None, None, 0, None) == pk.BEM_EINVAL
    assert lib.bem_eval_entries(None, None, None, 0, None, None, None, None) == pk.BEM_EINVAL
    assert lib.bem_last_error(None) == b"no context"
    lib.bem_destroy(None)


def test_oracle_is_not_reachable_from_the_product_package():
    pkg = os.path.join(ROOT, "paper_1510_07244_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
