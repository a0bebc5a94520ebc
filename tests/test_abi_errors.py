"""Error statuses of the C-ABI that the host reaches before any device work
(no GPU needed): ipc_create rejects bad scene data with IPC_E_INVALID and a
message, and leaves *out NULL.  The GPU-side statuses (capacity,
intersecting, not converged, line search, indefinite) are in
test_gpu_errors.py."""
import ctypes
import os

import numpy as np
import pytest

import ipcscenes as S


def _lib():
    from paper_2609_25653_amd import _lib
    if not os.path.exists(_lib.SO_PATH):
        pytest.skip("library not built")
    return _lib


def _create(scenes):
    L = _lib()
    keep = []
    arr = (L.SceneDesc * max(len(scenes), 1))(*[L.make_desc(s, keep) for s in scenes])
    h = ctypes.c_void_p(123)
    rc = L.lib().ipc_create(arr, len(scenes), None, ctypes.byref(h))
    return rc, h, L.lib().ipc_last_error(None).decode()


def _bad(mutate):
    sc = S.tiny_scene("cube", h=0.01, n_steps=2)
    mutate(sc)
    return sc


def _flip(sc):
    t = sc["tets"].copy()
    t[3, [1, 2]] = t[3, [2, 1]]
    sc["tets"] = t


CASES = {
    "poisson ratio 0.5": (lambda sc: sc["tet_nu"].__setitem__(5, 0.5), "invalid material at tet 5"),
    "negative Young's modulus": (lambda sc: sc["tet_E"].__setitem__(0, -1.0), "invalid material at tet 0"),
    "inverted tet": (_flip, "tet 3 is inverted or degenerate"),
    "NaN position": (lambda sc: sc["X"].__setitem__((7, 2), np.nan), "non-finite FEM state"),
    "tet index out of range": (lambda sc: sc["tets"].__setitem__((2, 1), len(sc["X"])), "tet index out of range"),
    "time step 0": (lambda sc: sc.__setitem__("h", np.asarray(0.0)), "invalid parameters"),
    "ccd fraction 1": (lambda sc: sc.__setitem__("ccd_s", np.asarray(1.0)), "invalid parameters"),
    "half-space normal of length 2": (lambda sc: sc.__setitem__("half_space", np.array([0.0, 0.0, 2.0, 0.0])),
                                      "half-space normal is not a unit vector"),
    "NaN half-space offset": (lambda sc: sc.__setitem__("half_space", np.array([0.0, 0.0, 1.0, np.nan])), "invalid half-space"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_create_rejects_bad_scene(name):
    mutate, msg = CASES[name]
    rc, h, err = _create([_bad(mutate)])
    assert rc == 1, (name, rc, err)            # IPC_E_INVALID
    assert h.value is None                      # *out is NULL
    assert msg in err, (name, err)


def test_create_names_the_scene_of_a_batch():
    good = S.tiny_scene("cube", h=0.01, n_steps=2)
    rc, _, err = _create([good, good, _bad(CASES["inverted tet"][0])])
    assert rc == 1 and err.startswith("scene 2:"), err


def test_create_rejects_no_scene():
    rc, h, err = _create([])
    assert rc == 1 and h.value is None and "at least one scene" in err


def test_missing_array_is_rejected():
    """A NULL array behind a nonzero count is reported, not dereferenced."""
    L = _lib()
    sc = S.tiny_scene("cube", h=0.01, n_steps=2)
    keep = []
    d = L.make_desc(sc, keep)
    d.tet_rho = ctypes.cast(None, L._D)
    arr = (L.SceneDesc * 1)(d)
    h = ctypes.c_void_p(123)
    rc = L.lib().ipc_create(arr, 1, None, ctypes.byref(h))
    assert rc == 1 and "missing array tet_rho" in L.lib().ipc_last_error(None).decode()
