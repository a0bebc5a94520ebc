"""MI355X-native IPC Newton step of the PhyVisGen arm-gripper system.

``Sim`` wraps one context of the HIP library (one or more scenes stepped
together).  Tensors are torch CUDA (HIP) float64 tensors in the external DOF
layout: per scene, FEM vertices (x, y, z) then 12 numbers per affine body
(p, A[:,0], A[:,1], A[:,2]).  All work is done by the library's kernels on the
current torch stream; torch only provides device memory and the stream.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (IPC_PSD_PROJECT, IPC_WITH_FRICTION, STATUS_NAMES, Stats, lib)  # noqa: F401


class IPCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the IPC library needs a ROCm GPU (torch.cuda is not available)")
    return torch


def _ptr(t):
    if t is None:
        return None
    if t.dtype != _torch().float64 or not t.is_contiguous():
        raise TypeError("device buffers must be contiguous float64 tensors")
    return ctypes.c_void_p(t.data_ptr())


def plan(scenes, capacity):
    """Device bytes of a context over ``scenes`` created over a workspace with
    ``capacity`` = (max_pairs, max_candidates, max_local_blocks) (host work only)."""
    if isinstance(scenes, dict):
        scenes = [scenes]
    keep = []
    arr = (_lib.SceneDesc * len(scenes))(*[_lib.make_desc(s, keep) for s in scenes])
    cap = _lib.Capacity(*[int(x) for x in capacity])
    out = ctypes.c_size_t()
    rc = lib().ipc_plan(arr, len(scenes), ctypes.byref(cap), ctypes.byref(out))
    if rc != 0:
        raise IPCError(rc, lib().ipc_last_error(None).decode())
    return out.value


class Sim:
    """A context over ``scenes`` (a scene dict or a list of them).  With
    ``capacity`` = (max_pairs, max_candidates, max_local_blocks) the context is
    created over a workspace that torch allocates (``workspace_bytes``, default
    the planned size): the library then allocates no device memory."""

    def __init__(self, scenes, device="cuda", capacity=None, workspace_bytes=None):
        torch = _torch()
        if isinstance(scenes, dict):
            scenes = [scenes]
        self.scenes = list(scenes)
        self.device = torch.device(device)
        L = lib()
        keep = []
        arr = (_lib.SceneDesc * len(self.scenes))(*[_lib.make_desc(s, keep) for s in self.scenes])
        h = ctypes.c_void_p()
        self._stream = torch.cuda.current_stream(self.device)
        self._ws = None
        if capacity is None:
            rc = L.ipc_create(arr, len(self.scenes), ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        else:
            nbytes = plan(self.scenes, capacity) if workspace_bytes is None else int(workspace_bytes)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)   # torch owns the memory
            cap = _lib.Capacity(*[int(x) for x in capacity])
            rc = L.ipc_create_ws(arr, len(self.scenes), ctypes.byref(cap), ctypes.c_void_p(self._ws.data_ptr()), nbytes,
                                 ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise IPCError(rc, L.ipc_last_error(None).decode())
        self._h = h
        self.ndof = self._query(_lib.Q_NDOF)
        self.n_scenes = self._query(_lib.Q_NSCENES)
        self.n_driven = self._query(_lib.Q_NDRIVEN)
        self.dof_offsets = np.cumsum([0] + [3 * (len(s["X"]) + 4 * len(s["body_q"])) for s in self.scenes])
        self.step_index = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            try:
                lib().ipc_destroy(h)
            except Exception:   # interpreter shutdown: the process releases the device anyway
                pass

    def _query(self, what):
        v = ctypes.c_int64()
        self._check(lib().ipc_query(self._h, what, ctypes.byref(v)))
        return v.value

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise IPCError(rc, lib().ipc_last_error(self._h).decode())
        return rc

    def _vec(self, n=None):
        torch = _torch()
        return torch.empty(self.ndof if n is None else n, dtype=torch.float64, device=self.device)

    def _as_dev(self, a, n=None):
        torch = _torch()
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def hessian_bsr(self, y, project=True, friction=True):
        """The assembled Hessian at y as (row_ptr, col, val) device tensors
        (external nodes, 3x3 blocks, val of shape (nnzb, 3, 3))."""
        torch = _torch()
        y = self._as_dev(y, self.ndof)
        nodes = self.ndof // 3
        rp = torch.empty(nodes + 1, dtype=torch.int32, device=self.device)
        n = ctypes.c_int64()
        flags = (IPC_PSD_PROJECT if project else 0) | (IPC_WITH_FRICTION if friction else 0)
        rc = lib().ipc_hessian_bsr(self._h, _ptr(y), flags, ctypes.c_void_p(rp.data_ptr()), None, None, 0, ctypes.byref(n))
        self._check(rc, allow=(_lib.IPC_E_CAPACITY,))
        col = torch.empty(max(n.value, 1), dtype=torch.int32, device=self.device)
        val = torch.empty((max(n.value, 1), 3, 3), dtype=torch.float64, device=self.device)
        self._check(lib().ipc_hessian_bsr(self._h, _ptr(y), flags, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                                          ctypes.c_void_p(val.data_ptr()), n.value, ctypes.byref(n)))
        return rp, col[:n.value], val[:n.value]

    def scene_scalars(self, s=0):
        k, L, t = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().ipc_scene_scalars(self._h, s, ctypes.byref(k), ctypes.byref(L), ctypes.byref(t)))
        return dict(kappa=k.value, L=L.value, newton_threshold=t.value)

    def state(self):
        y, v = self._vec(), self._vec()
        self._check(lib().ipc_get_state(self._h, _ptr(y), _ptr(v)))
        return y, v

    def set_state(self, y, ydot):
        y = self._as_dev(y, self.ndof); v = self._as_dev(ydot, self.ndof)
        self._check(lib().ipc_set_state(self._h, _ptr(y), _ptr(v)))

    def targets(self, n):
        """Targets of step n: the drive targets of all scenes (nd x 12), then the
        joint-spring points of all scenes (nj x 3), concatenated."""
        parts = [s["drive_q"][n].ravel() for s in self.scenes if s["drive_q"].shape[1] > 0]
        parts += [s["joint_xbar"][n].ravel() for s in self.scenes if s["joint_xbar"].shape[1] > 0]
        if not parts:
            return None
        return self._as_dev(np.concatenate(parts, 0))

    def begin_step(self, n=None):
        t = self.targets(self.step_index if n is None else n)
        self._check(lib().ipc_begin_step(self._h, _ptr(t)))

    def energy_grad_hess(self, y, v=None, project=True, friction=True, energy=True, grad=True):
        """Energies per scene, gradient and H v at y (external layout)."""
        torch = _torch()
        y = self._as_dev(y, self.ndof)
        E = torch.empty(self.n_scenes, dtype=torch.float64, device=self.device) if energy else None
        g = self._vec() if grad else None
        vv = self._as_dev(v, self.ndof) if v is not None else None
        Hv = self._vec() if v is not None else None
        flags = (IPC_PSD_PROJECT if project else 0) | (IPC_WITH_FRICTION if friction else 0)
        rc = self._check(lib().ipc_energy_grad_hess(self._h, _ptr(y), _ptr(E), _ptr(g), _ptr(vv), _ptr(Hv), flags),
                         allow=(_lib.IPC_E_INTERSECTING,))
        return E, g, Hv, rc

    def pairs(self, y, scene=0, cap=1 << 20):
        y = self._as_dev(y, self.ndof)
        while True:
            pt = np.zeros((cap, 4), np.int32); ee = np.zeros((cap, 4), np.int32)
            npt, nee = ctypes.c_int64(), ctypes.c_int64()
            rc = lib().ipc_get_pairs(self._h, _ptr(y), scene, pt.ctypes.data_as(_lib._I), ee.ctypes.data_as(_lib._I),
                                     cap, ctypes.byref(npt), ctypes.byref(nee))
            if rc == _lib.IPC_E_CAPACITY:
                cap = max(npt.value, nee.value)
                continue
            self._check(rc)
            return pt[:npt.value].copy(), ee[:nee.value].copy()

    def ccd(self, y, p):
        torch = _torch()
        y = self._as_dev(y, self.ndof); p = self._as_dev(p, self.ndof)
        a = torch.empty(self.n_scenes, dtype=torch.float64, device=self.device)
        self._check(lib().ipc_ccd(self._h, _ptr(y), _ptr(p), _ptr(a)))
        return a

    def pcg(self, y, b, eta):
        y = self._as_dev(y, self.ndof); b = self._as_dev(b, self.ndof)
        x = self._vec()
        it = np.zeros(self.n_scenes, np.int32)
        self._check(lib().ipc_pcg(self._h, _ptr(y), _ptr(b), _ptr(x), float(eta), it.ctypes.data_as(_lib._I)))
        return x, it

    def step(self, n=None, allow_status=()):
        t = self.targets(self.step_index if n is None else n)
        st = (Stats * self.n_scenes)()
        rc = lib().ipc_step(self._h, _ptr(t), st)
        self._check(rc, allow=allow_status)
        self.step_index += 1
        return rc, [s.as_dict() for s in st]

    def step_targets(self, targets, allow_status=()):
        """One step towards explicit targets (the layout of targets(n)); the
        step index does not move."""
        t = None if targets is None else self._as_dev(targets)
        st = (Stats * self.n_scenes)()
        rc = lib().ipc_step(self._h, _ptr(t), st)
        self._check(rc, allow=allow_status)
        return rc, [s.as_dict() for s in st]

    def set_timestep(self, h):
        """New time step per scene (a scalar applies to every scene; entries
        <= 0 keep a scene's step)."""
        hh = np.broadcast_to(np.asarray(h, np.float64), (self.n_scenes,)).copy()
        self._check(lib().ipc_set_timestep(self._h, hh.ctypes.data_as(_lib._D)))

    def set_friction_lag(self, passes):
        """Friction lag passes per step (1: lagged once at the step start)."""
        self._check(lib().ipc_set_friction_lag(self._h, int(passes)))

    def set_kappa_adaptive(self, frac, factor=100.0):
        """Adaptive barrier stiffness: after an accepted Newton update a
        scene's kappa doubles when its smallest active-pair distance is below
        frac dhat and below the previous iterate's, capped at factor times
        its kappa at this call (frac = 0: off)."""
        self._check(lib().ipc_set_kappa_adaptive(self._h, float(frac), float(factor)))

    def step_adaptive(self, max_depth=3):
        """One step of a single-scene context with sub-stepping on failure:
        if Newton does not converge (status 3) the step is taken again from
        its start as two steps of h/2, the first towards the mean of the
        previous and this step's targets, each retried the same way down to
        h / 2^max_depth.  Returns (status of the last piece, pieces taken)."""
        if self.n_scenes != 1:
            raise ValueError("step_adaptive steps a single-scene context")
        n = self.step_index
        h = float(self.scenes[0]["h"])
        t1 = self.targets(n)
        t0 = self.targets(n - 1 if n > 0 else 0)
        st = (Stats * 1)()

        def run(y, v, hh, ta, tb, depth):
            self.set_state(y, v)
            self.set_timestep(hh)
            rc = lib().ipc_step(self._h, _ptr(tb), st)
            self._check(rc, allow=(3,))
            if rc != 3 or depth >= max_depth:
                return rc, 1
            tm = None if tb is None else 0.5 * (ta + tb)
            rc1, k1 = run(y, v, 0.5 * hh, ta, tm, depth + 1)
            if rc1 != 0:
                return rc1, k1
            y2, v2 = self.state()
            rc2, k2 = run(y2, v2, 0.5 * hh, tm, tb, depth + 1)
            return rc2, k1 + k2

        y, v = self.state()
        rc, pieces = run(y, v, h, t0, t1, 0)
        self.set_timestep(h)
        self.step_index += 1
        return rc, pieces

    def autotune(self, reps=20):
        """Pick the product's lanes per row on the current matrix and the FEM
        assembly's workgroup sizes on the current state (see fem_blocks);
        returns (lanes, {lanes: microseconds})."""
        us = np.zeros(5)
        L = ctypes.c_int32()
        self._check(lib().ipc_autotune(self._h, int(reps), us.ctypes.data_as(_lib._D), ctypes.byref(L)))
        return L.value, dict(zip((1, 2, 4, 8, 16), us.tolist()))

    @property
    def pcg_coarse(self):
        """Whether the PCG preconditioner applies its coarse correction."""
        return bool(self._query(_lib.Q_COARSE))

    @property
    def pcg_fused(self):
        """Whether a PCG iteration applies the coarse correction inside its
        update launch (same bits as the two-launch form)."""
        return bool(self._query(_lib.Q_PCG_FUSED))

    @property
    def spmv_lanes(self):
        """Lanes per row of the Hessian product (the autotuner's choice, or
        the one tuned earlier in this process for a context of this size)."""
        return int(self._query(_lib.Q_SPMV_LANES))

    @property
    def fem_blocks(self):
        """Workgroup sizes of the FEM assembly's three kernels (element
        blocks, slot gather, gradient gather): the autotuner's choice, or the
        one tuned earlier in this process for a context of this size."""
        v = int(self._query(_lib.Q_FEM_BLOCKS))
        return (v >> 32) & 0xffff, (v >> 16) & 0xffff, v & 0xffff

    # ---- adjoint --------------------------------------------------------------
    @property
    def n_tets(self):
        return self._query(_lib.Q_NTETS_EXT)

    def set_params(self, E=None, mu=None):
        """Young's moduli of all tets (scenes concatenated) and/or the friction
        coefficient of every scene (a scalar applies to all)."""
        e = self._as_dev(E, self.n_tets) if E is not None else None
        m = None
        if mu is not None:
            m = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, np.float64), (self.n_scenes,)))
        self._check(lib().ipc_set_params(self._h, _ptr(e), m.ctypes.data_as(_lib._D) if m is not None else None))

    def step_vjp(self, y_prev, ydot_prev, n, y_next, ybar_next, vbar_next, Ebar=None, mubar=None, eta=1e-12):
        """Adjoint of step n (from (y_prev, ydot_prev) to y_next).  Returns
        (ybar_prev, vbar_prev, pcg_iters); Ebar (n_tets) and mubar (n_scenes)
        tensors, when given, are accumulated in place."""
        a = [self._as_dev(v, self.ndof) for v in (y_prev, ydot_prev, y_next, ybar_next, vbar_next)]
        t = self.targets(n)
        yb, vb = self._vec(), self._vec()
        it = np.zeros(self.n_scenes, np.int32)
        self._check(lib().ipc_step_vjp(self._h, _ptr(a[0]), _ptr(a[1]), _ptr(t), _ptr(a[2]), _ptr(a[3]), _ptr(a[4]),
                                       _ptr(yb), _ptr(vb), _ptr(Ebar), _ptr(mubar), float(eta),
                                       it.ctypes.data_as(_lib._I)))
        return yb, vb, it
