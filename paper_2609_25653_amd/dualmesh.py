"""ctypes binding of the dual-mesh mapping in include/ipc_dualmesh.h
(argument marshalling only): the fine render mesh of a deformable object as
L levels of Loop subdivision of its coarse simulation mesh, W X^c per frame
(Sec. III-D, Eq. (6)-(7)).  W is built by the library on the host; the product
runs in the library's HIP kernel."""
import ctypes

import numpy as np

from . import _lib
from ._lib import lib

DM_NCOARSE, DM_NFINE, DM_NTRI, DM_NNZ, DM_MAXROW = range(5)


class DualMesh:
    def __init__(self, tri, n_vert, levels, stream=None):
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._keep = tri
        h = ctypes.c_void_p()
        if stream is None:   # the current torch stream, as for Sim (none on a machine without a GPU)
            import torch
            stream = torch.cuda.current_stream() if torch.cuda.is_available() else None
        s = ctypes.c_void_p(stream.cuda_stream if stream is not None else None)
        rc = lib().ipc_dualmesh_create(tri.ctypes.data_as(_lib._I), len(tri), int(n_vert), int(levels), s, ctypes.byref(h))
        if rc != 0:
            raise RuntimeError(f"ipc_dualmesh_create: {_lib.STATUS_NAMES.get(rc, rc)}: "
                               f"{lib().ipc_dualmesh_last_error(None).decode()}")
        self._h = h
        self.n_coarse = self._query(DM_NCOARSE)
        self.n_fine = self._query(DM_NFINE)
        self.n_tri = self._query(DM_NTRI)
        self.nnz = self._query(DM_NNZ)
        self.max_row = self._query(DM_MAXROW)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ipc_dualmesh_destroy(self._h)
            self._h = None

    def _query(self, what):
        v = ctypes.c_int64()
        self._check(lib().ipc_dualmesh_query(self._h, what, ctypes.byref(v)))
        return v.value

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(f"dual mesh: {_lib.STATUS_NAMES.get(rc, rc)}: {lib().ipc_dualmesh_last_error(self._h).decode()}")

    def fine_tris(self):
        t = np.zeros((self.n_tri, 3), np.int32)
        self._check(lib().ipc_dualmesh_fine_tris(self._h, t.ctypes.data_as(_lib._I)))
        return t

    def weights(self):
        """W as (row_ptr, col, val), columns ascending per row."""
        rp = np.zeros(self.n_fine + 1, np.int32)
        col = np.zeros(max(self.nnz, 1), np.int32)
        val = np.zeros(max(self.nnz, 1), np.float64)
        self._check(lib().ipc_dualmesh_weights(self._h, rp.ctypes.data_as(_lib._I), col.ctypes.data_as(_lib._I),
                                               val.ctypes.data_as(_lib._D)))
        return rp, col[:self.nnz], val[:self.nnz]

    def apply(self, xc, out=None):
        """X^f = W X^c for every frame: xc a float64 CUDA tensor of shape
        (frames, N_c, 3) or (N_c, 3); returns (frames, N_f, 3) (or (N_f, 3))."""
        import torch
        if not (xc.is_cuda and xc.dtype == torch.float64 and xc.is_contiguous()):
            raise ValueError("xc must be a contiguous float64 CUDA tensor")
        single = xc.dim() == 2
        x = xc.unsqueeze(0) if single else xc
        if x.shape[1:] != (self.n_coarse, 3):
            raise ValueError(f"xc must have shape (frames, {self.n_coarse}, 3)")
        if out is None:
            out = torch.empty((x.shape[0], self.n_fine, 3), dtype=torch.float64, device=x.device)
        self._check(lib().ipc_dualmesh_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.shape[0]))
        return out[0] if single else out

    def apply_noalloc(self, xc, out):
        """As apply, through the entry point that allocates nothing (W staged
        in the library's fixed device array); ``out`` is required."""
        import torch
        if not (xc.is_cuda and xc.dtype == torch.float64 and xc.is_contiguous() and xc.dim() == 3):
            raise ValueError("xc must be a contiguous float64 CUDA tensor of shape (frames, N_c, 3)")
        if xc.shape[1:] != (self.n_coarse, 3) or out.shape != (xc.shape[0], self.n_fine, 3) or not out.is_contiguous():
            raise ValueError("shape mismatch")
        self._check(lib().ipc_dualmesh_apply_noalloc(self._h, ctypes.c_void_p(xc.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                     xc.shape[0]))
        return out

    def time(self, xc, out, reps=20):
        """Average launch duration (us) of apply and its algorithmic bytes."""
        us, by = ctypes.c_double(), ctypes.c_double()
        self._check(lib().ipc_dualmesh_time(self._h, ctypes.c_void_p(xc.data_ptr()), ctypes.c_void_p(out.data_ptr()), xc.shape[0],
                                            int(reps), ctypes.byref(us), ctypes.byref(by)))
        return us.value, by.value
