"""C-ABI checks that need no GPU: the library loads and exports every entry
point that the headers in include/ declare; the headers compile as C; the
struct layouts match the binding."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names.update(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(ipc_\w+)\s*\(", src, re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("ipc_create", "ipc_step", "ipc_energy_grad_hess", "ipc_destroy", "ipc_get_pairs", "ipc_ccd",
              "ipc_pcg", "ipc_begin_step", "ipc_get_state", "ipc_set_state", "ipc_last_error",
              "ipc_dualmesh_create", "ipc_dualmesh_apply", "ipc_dualmesh_weights", "ipc_dualmesh_destroy"):
        assert n in names


def test_headers_compile_as_c(tmp_path):
    import subprocess
    src = tmp_path / "h.c"
    src.write_text('#include "ipc.h"\n#include "ipc_dualmesh.h"\nint main(void) { return IPC_DM_NNZ - 3; }\n')
    exe = tmp_path / "h"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    assert subprocess.run([str(exe)]).returncode == 0


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
