"""ctypes binding of the C-ABI in include/ipc.h (argument marshalling only).

Every computation runs in the HIP library ``libipc_hip.so``; this module only
converts scene dictionaries to ``ipc_scene_desc`` records and passes device
pointers and the current torch stream.  Importing it without the built
library raises immediately: there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libipc_hip.so")

IPC_OK = 0
IPC_E_INVALID = 1
IPC_E_CAPACITY = 2
IPC_E_NOT_CONVERGED = 3
IPC_E_LINESEARCH = 4
IPC_E_INTERSECTING = 5
IPC_E_INDEFINITE = 6
IPC_E_DEVICE = 7
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "CAPACITY", 3: "NOT_CONVERGED", 4: "LINESEARCH", 5: "INTERSECTING",
                6: "INDEFINITE", 7: "DEVICE"}

IPC_PSD_PROJECT = 1
IPC_WITH_FRICTION = 2

Q_NDOF, Q_NSCENES, Q_NDRIVEN, Q_NTRI, Q_NEDGE, Q_NNODES, Q_NTETS, Q_NLOCAL, Q_NPAIRS, Q_NTETS_EXT, Q_COARSE, Q_WS_BYTES, Q_WS_PEAK, \
    Q_SPMV_LANES, Q_FEM_BLOCKS, Q_PCG_FUSED = range(16)

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


class SceneDesc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("nv", "nt", "nb", "nbv", "nbt", "nsv", "nst", "nobj", "nex", "ns", "nd")] + [
        ("X", _D), ("V", _D), ("tets", _I), ("tet_E", _D), ("tet_nu", _D), ("tet_rho", _D), ("vobj", _I),
        ("body_q", _D), ("body_qdot", _D), ("body_mass", _D), ("body_S", _D), ("body_vol", _D), ("body_kappa", _D),
        ("body_ext", _D), ("body_obj", _I), ("bv_xbar", _D), ("bv_body", _I), ("btri", _I), ("sv_x", _D),
        ("stri", _I), ("obj_kind", _I), ("excl", _I), ("sp_ka", _I), ("sp_ia", _I), ("sp_xa", _D), ("sp_kb", _I),
        ("sp_ib", _I), ("sp_xb", _D), ("sp_k", _D), ("driven_body", _I),
        ("h", ctypes.c_double), ("g", ctypes.c_double * 3), ("dhat", ctypes.c_double), ("kappa", ctypes.c_double),
        ("mu", ctypes.c_double), ("eps_v", ctypes.c_double), ("newton_tol", ctypes.c_double),
        ("pcg_tol", ctypes.c_double), ("ccd_s", ctypes.c_double), ("max_newton", ctypes.c_int32),
        ("max_pcg", ctypes.c_int32), ("nj", ctypes.c_int32), ("joint_spring", _I), ("half_space", ctypes.c_double * 4)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("newton_iters", ctypes.c_int32), ("pcg_iters_total", ctypes.c_int32),
                ("pcg_iters_max", ctypes.c_int32), ("n_pt_max", ctypes.c_int32), ("n_ee_max", ctypes.c_int32),
                ("n_lag", ctypes.c_int32), ("n_cand_max", ctypes.c_int32), ("alpha_min", ctypes.c_double),
                ("energy", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"HIP library not built: {SO_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(SO_PATH)
        P = ctypes.c_void_p
        L.ipc_create.argtypes = [ctypes.POINTER(SceneDesc), ctypes.c_int, P, ctypes.POINTER(P)]
        L.ipc_plan.argtypes = [ctypes.POINTER(SceneDesc), ctypes.c_int, ctypes.POINTER(Capacity), ctypes.POINTER(ctypes.c_size_t)]
        L.ipc_create_ws.argtypes = [ctypes.POINTER(SceneDesc), ctypes.c_int, ctypes.POINTER(Capacity), P, ctypes.c_size_t, P,
                                    ctypes.POINTER(P)]
        L.ipc_hessian_bsr.argtypes = [P, P, ctypes.c_uint32, P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.ipc_destroy.argtypes = [P]
        L.ipc_last_error.restype = ctypes.c_char_p
        L.ipc_last_error.argtypes = [P]
        L.ipc_query.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.ipc_scene_scalars.argtypes = [P, ctypes.c_int, _D, _D, _D]
        L.ipc_get_state.argtypes = [P, P, P]
        L.ipc_set_state.argtypes = [P, P, P]
        L.ipc_begin_step.argtypes = [P, P]
        L.ipc_energy_grad_hess.argtypes = [P, P, P, P, P, P, ctypes.c_uint32]
        L.ipc_get_pairs.argtypes = [P, P, ctypes.c_int, _I, _I, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]
        L.ipc_ccd.argtypes = [P, P, P, P]
        L.ipc_pcg.argtypes = [P, P, P, P, ctypes.c_double, _I]
        L.ipc_step.argtypes = [P, P, ctypes.POINTER(Stats)]
        L.ipc_set_params.argtypes = [P, P, _D]
        L.ipc_step_vjp.argtypes = [P, P, P, P, P, P, P, P, P, P, P, ctypes.c_double, _I]
        L.ipc_profile.argtypes = [P, ctypes.c_int]
        L.ipc_kernel_time.argtypes = [P, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int64), _D]
        L.ipc_time_kernel.argtypes = [P, ctypes.c_int, ctypes.c_int, _D, _D]
        L.ipc_autotune.argtypes = [P, ctypes.c_int, _D, _I]
        L.ipc_set_timestep.argtypes = [P, _D]
        L.ipc_set_friction_lag.argtypes = [P, ctypes.c_int]
        L.ipc_set_kappa_adaptive.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.ipc_dualmesh_create.argtypes = [_I, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.POINTER(P)]
        L.ipc_dualmesh_destroy.argtypes = [P]
        L.ipc_dualmesh_destroy.restype = None
        L.ipc_dualmesh_last_error.argtypes = [P]
        L.ipc_dualmesh_last_error.restype = ctypes.c_char_p
        L.ipc_dualmesh_query.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.ipc_dualmesh_fine_tris.argtypes = [P, _I]
        L.ipc_dualmesh_weights.argtypes = [P, _I, _I, _D]
        L.ipc_dualmesh_apply.argtypes = [P, P, P, ctypes.c_int32]
        L.ipc_dualmesh_time.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, _D, _D]
        for n in ("ipc_dualmesh_create", "ipc_dualmesh_query", "ipc_dualmesh_fine_tris", "ipc_dualmesh_weights",
                  "ipc_dualmesh_apply", "ipc_dualmesh_time"):
            getattr(L, n).restype = ctypes.c_int
        for n in ("ipc_create", "ipc_destroy", "ipc_query", "ipc_scene_scalars", "ipc_get_state", "ipc_set_state",
                  "ipc_begin_step", "ipc_energy_grad_hess", "ipc_get_pairs", "ipc_ccd", "ipc_pcg", "ipc_step",
                  "ipc_set_params", "ipc_step_vjp", "ipc_profile", "ipc_kernel_time", "ipc_time_kernel",
                  "ipc_autotune", "ipc_set_timestep", "ipc_set_friction_lag", "ipc_set_kappa_adaptive"):
            getattr(L, n).restype = ctypes.c_int
        _lib = L
    return _lib


class Capacity(ctypes.Structure):
    """ipc_capacity of include/ipc.h."""
    _fields_ = [("max_pairs", ctypes.c_int64), ("max_candidates", ctypes.c_int64), ("max_local_blocks", ctypes.c_int64)]


def make_desc(sc, keep):
    """Fill an ipc_scene_desc from a scene dict; arrays are kept alive in ``keep``."""
    d = SceneDesc()
    sizes = dict(nv=len(sc["X"]), nt=len(sc["tets"]), nb=len(sc["body_q"]), nbv=len(sc["bv_xbar"]),
                 nbt=len(sc["btri"]), nsv=len(sc["sv_x"]), nst=len(sc["stri"]), nobj=len(sc["obj_kind"]),
                 nex=len(sc["excl"]), ns=len(sc["sp_k"]), nd=len(sc["driven_body"]), nj=len(sc["joint_spring"]))
    for k, v in sizes.items():
        setattr(d, k, int(v))
    for name, typ in SceneDesc._fields_:
        if typ is _D or typ is _I:
            dt = np.float64 if typ is _D else np.int32
            a = np.ascontiguousarray(sc[name], dtype=dt)
            keep.append(a)
            setattr(d, name, a.ctypes.data_as(typ))
    d.h = float(sc["h"])
    for k in range(3):
        d.g[k] = float(sc["g"][k])
    for k in ("dhat", "kappa", "mu", "eps_v", "newton_tol", "pcg_tol", "ccd_s"):
        setattr(d, k, float(sc[k]))
    d.max_newton = int(sc["max_newton"])
    d.max_pcg = int(sc["max_pcg"])
    hs = np.asarray(sc.get("half_space", np.zeros(4)), np.float64).ravel()
    for k in range(4):
        d.half_space[k] = float(hs[k])
    return d
