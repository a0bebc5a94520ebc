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


def test_struct_layout_matches_header():
    from paper_2609_25653_amd import _lib
    # 11 int32 sizes, 30 pointers, 11 doubles (h, g[3], dhat, kappa, mu, eps_v, newton_tol, pcg_tol, ccd_s), 2 int32
    assert ctypes.sizeof(_lib.SceneDesc) == 11 * 4 + 4 + 30 * 8 + 11 * 8 + 2 * 4
    assert ctypes.sizeof(_lib.Stats) == 8 * 4 + 2 * 8


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2609_25653_amd import _lib
    monkeypatch.setattr(_lib, "SO_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
