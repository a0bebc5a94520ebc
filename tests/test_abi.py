"""C-ABI checks that need no GPU: the library loads and exports every entry
point that include/ipc.h declares; the struct layouts match the binding."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "ipc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\*?\s*(ipc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("ipc_create", "ipc_step", "ipc_energy_grad_hess", "ipc_destroy", "ipc_get_pairs", "ipc_ccd",
              "ipc_pcg", "ipc_begin_step", "ipc_get_state", "ipc_set_state", "ipc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2609_25653_amd import _lib
    if not os.path.exists(_lib.SO_PATH):
        pytest.skip("library not built")
    # RTLD_NOW: every symbol the library needs must resolve at load time
    L = ctypes.CDLL(_lib.SO_PATH, mode=os.RTLD_NOW)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layout_matches_header(tmp_path):
    """Every field offset and the size of the ctypes records equal the C
    compiler's for include/ipc.h."""
    import subprocess
    from paper_2609_25653_amd import _lib
    recs = {"ipc_scene_desc": _lib.SceneDesc, "ipc_stats": _lib.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ipc.h"', "int main(void) {"]
    for cname, cls in recs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        rec, name, val = line.split()
        got[(rec, name)] = int(val)
    for cname, cls in recs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2609_25653_amd import _lib
    monkeypatch.setattr(_lib, "SO_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
