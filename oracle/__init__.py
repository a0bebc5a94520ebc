"""Oracle binding (test infrastructure only).

A ctypes wrapper around ``ipc_oracle.c``, the plain FP64 CPU implementation of
one IPC Newton step.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libipc_oracle.so")
_SRC = os.path.join(_HERE, "ipc_oracle.c")

PTR_KEYS = ("X", "V", "tets", "tet_E", "tet_nu", "tet_rho", "vobj",
            "body_q", "body_qdot", "body_mass", "body_S", "body_vol", "body_kappa",
            "body_ext", "body_obj", "bv_xbar", "bv_body", "btri", "sv_x", "stri",
            "obj_kind", "excl", "sp_ka", "sp_ia", "sp_xa", "sp_kb", "sp_ib", "sp_xb",
            "sp_k", "driven_body", "joint_spring")


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, OpenMP over elements)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    # build under a private name, then rename: processes that build at the same
    # time never load a half-written library
    tmp = f"{_SO}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        L.or_create.restype = P
        L.or_create.argtypes = [I, ctypes.POINTER(P), D]
        L.or_destroy.argtypes = [P]
        L.or_count.restype = ctypes.c_int
        L.or_count.argtypes = [P, ctypes.c_int]
        L.or_scalar.restype = ctypes.c_double
        L.or_scalar.argtypes = [P, ctypes.c_int]
        for n in ("or_get_mass",):
            getattr(L, n).argtypes = [P, D]
        L.or_get_tris.argtypes = [P, I]
        L.or_get_edges.argtypes = [P, I]
        L.or_get_state.argtypes = [P, D, D]
        L.or_set_state.argtypes = [P, D, D]
        L.or_world.argtypes = [P, D, D]
        L.or_begin_step.argtypes = [P, D]
        L.or_energy.restype = ctypes.c_double
        L.or_energy.argtypes = [P, D, D]
        L.or_gradient.argtypes = [P, D, D, D]
        L.or_hessian_matvec.argtypes = [P, D, ctypes.c_int, D, D]
        L.or_hessian_matvec_abs.argtypes = [P, D, ctypes.c_int, ctypes.c_int, D, D, D]
        L.or_hessian_dense.argtypes = [P, D, ctypes.c_int, ctypes.c_int, D, D]
        L.or_pairs.restype = ctypes.c_int
        L.or_pairs.argtypes = [P, D, I, ctypes.c_int, I, ctypes.c_int, I, I]
        L.or_ccd.restype = ctypes.c_double
        L.or_ccd.argtypes = [P, D, D]
        L.or_pcg.restype = ctypes.c_int
        L.or_pcg.argtypes = [P, D, D, D, ctypes.c_double]
        L.or_step.restype = ctypes.c_int
        L.or_step.argtypes = [P, D, ctypes.POINTER(OStats)]
        L.or_dist2_pt.restype = ctypes.c_double
        L.or_dist2_pt.argtypes = [D, I]
        L.or_dist2_ee.restype = ctypes.c_double
        L.or_dist2_ee.argtypes = [D, I]
        L.or_dist2_derivs.restype = ctypes.c_double
        L.or_dist2_derivs.argtypes = [ctypes.c_int, D, D, D]
        L.or_accd.restype = ctypes.c_double
        L.or_accd.argtypes = [ctypes.c_int, D, D, ctypes.c_double]
        L.or_snh.restype = ctypes.c_double
        L.or_snh.argtypes = [D, ctypes.c_double, ctypes.c_double, D, D]
        L.or_psd_project.argtypes = [D, ctypes.c_int]
        L.or_barrier3.argtypes = [ctypes.c_double, ctypes.c_double, D]
        L.or_set_params.argtypes = [P, D, ctypes.c_double]
        L.or_set_timestep.argtypes = [P, ctypes.c_double]
        L.or_set_timestep.restype = None
        L.or_set_friction_lag.argtypes = [P, ctypes.c_int]
        L.or_set_friction_lag.restype = None
        L.or_set_kappa_adaptive.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.or_set_kappa_adaptive.restype = None
        L.or_set_kappa.argtypes = [P, ctypes.c_double]
        L.or_set_kappa.restype = None
        L.or_dG_dyn_T.argtypes = [P, D, D, D, D, D, D]
        L.or_dG_dtheta_T.restype = ctypes.c_double
        L.or_dG_dtheta_T.argtypes = [P, D, D, D, D, D, D]
        L.or_step_vjp.restype = ctypes.c_int
        L.or_step_vjp.argtypes = [P, D, D, D, D, D, D, D, D, D, D, ctypes.c_double, I]
        _lib = L
    return _lib


class OStats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("pcg_iters_total", ctypes.c_int),
                ("pcg_iters_max", ctypes.c_int), ("n_pt_max", ctypes.c_int), ("n_ee_max", ctypes.c_int),
                ("n_lag", ctypes.c_int), ("status", ctypes.c_int), ("alpha_min", ctypes.c_double),
                ("energy", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def scene_sizes(sc):
    return [len(sc["X"]), len(sc["tets"]), len(sc["body_q"]), len(sc["bv_xbar"]), len(sc["btri"]),
            len(sc["sv_x"]), len(sc["stri"]), len(sc["obj_kind"]), len(sc["excl"]), len(sc["sp_k"]),
            len(sc["driven_body"]), len(sc["joint_spring"])]


def scene_params(sc):
    g = sc["g"]
    return [float(sc["h"]), float(g[0]), float(g[1]), float(g[2]), float(sc["dhat"]), float(sc["kappa"]),
            float(sc["mu"]), float(sc["eps_v"]), float(sc["newton_tol"]), float(sc["max_newton"]),
            float(sc["pcg_tol"]), float(sc["max_pcg"]), float(sc["ccd_s"])] + \
        [float(v) for v in np.asarray(sc.get("half_space", np.zeros(4)), np.float64).ravel()[:4]]


class Oracle:
    """One scene held by the oracle."""

    def __init__(self, scene):
        L = lib()
        self.scene = scene
        sizes = np.array(scene_sizes(scene), np.int32)
        arrs = [np.ascontiguousarray(scene[k]) for k in PTR_KEYS]
        ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        prm = np.array(scene_params(scene), np.float64)
        self._h = L.or_create(_i(sizes), ptrs, _d(prm))
        self._keep = arrs
        self.ndof = L.or_count(self._h, 0)
        self.nnodes = L.or_count(self._h, 1)
        self.ncv = L.or_count(self._h, 2)
        self.ntri = L.or_count(self._h, 3)
        self.nedge = L.or_count(self._h, 4)
        self.step_index = 0

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    # scalars
    @property
    def kappa(self):
        return lib().or_scalar(self._h, 0)

    @property
    def L(self):
        return lib().or_scalar(self._h, 1)

    @property
    def newton_threshold(self):
        return lib().or_scalar(self._h, 3)

    def mass(self):
        m = np.zeros(len(self.scene["X"]))
        lib().or_get_mass(self._h, _d(m))
        return m

    def tris(self):
        t = np.zeros((self.ntri, 3), np.int32)
        lib().or_get_tris(self._h, _i(t))
        return t

    def edges(self):
        e = np.zeros((self.nedge, 2), np.int32)
        lib().or_get_edges(self._h, _i(e))
        return e

    def state(self):
        y = np.zeros(self.ndof)
        v = np.zeros(self.ndof)
        lib().or_get_state(self._h, _d(y), _d(v))
        return y, v

    def set_state(self, y, v):
        y = _f64(y); v = _f64(v)
        lib().or_set_state(self._h, _d(y), _d(v))

    def world(self, y):
        y = _f64(y)
        x = np.zeros((self.ncv, 3))
        lib().or_world(self._h, _d(y), _d(x))
        return x

    def targets(self, n):
        """Drive targets of step n (nd x 12) followed by the joint-spring points (nj x 3)."""
        dq, jx = self.scene["drive_q"], self.scene["joint_xbar"]
        if dq.shape[1] == 0 and jx.shape[1] == 0:
            return None
        return np.ascontiguousarray(np.concatenate([dq[n].ravel(), jx[n].ravel()]))

    def begin_step(self, n=None):
        n = self.step_index if n is None else n
        t = self.targets(n)
        lib().or_begin_step(self._h, _d(t) if t is not None else None)

    def energy(self, y):
        y = _f64(y)
        terms = np.zeros(7)
        E = lib().or_energy(self._h, _d(y), _d(terms))
        return E, terms

    def gradient(self, y):
        y = _f64(y)
        g = np.zeros(self.ndof)
        ga = np.zeros(self.ndof)
        lib().or_gradient(self._h, _d(y), _d(g), _d(ga))
        return g, ga

    def hess_matvec(self, y, v, project=True, with_abs=False, friction=True):
        """H(y) v (friction=False: without the lagged friction terms);
        with_abs=True also returns |P|^T |H| |P| |v| per entry (the scale of
        the operands that form it)."""
        y = _f64(y); v = _f64(v)
        out = np.zeros(self.ndof)
        scale = np.zeros(self.ndof) if with_abs else None
        lib().or_hessian_matvec_abs(self._h, _d(y), int(project), int(friction), _d(v), _d(out),
                                    _d(scale) if with_abs else None)
        return (out, scale) if with_abs else out

    def hessian_dense(self, y, project=True, friction=True):
        """(H, |H|-scale) as dense ndof x ndof arrays (small scenes only)."""
        y = _f64(y)
        H = np.zeros((self.ndof, self.ndof)); A = np.zeros((self.ndof, self.ndof))
        lib().or_hessian_dense(self._h, _d(y), int(project), int(friction), _d(H), _d(A))
        return H, A

    def pairs(self, y, cap=1 << 22):
        y = _f64(y)
        while True:
            pt = np.zeros((cap, 4), np.int32)
            ee = np.zeros((cap, 4), np.int32)
            npt = ctypes.c_int(); nee = ctypes.c_int()
            rc = lib().or_pairs(self._h, _d(y), _i(pt), cap, _i(ee), cap, ctypes.byref(npt), ctypes.byref(nee))
            if rc == 0:
                return pt[:npt.value].copy(), ee[:nee.value].copy()
            cap = max(npt.value, nee.value)

    def ccd(self, y, p):
        y = _f64(y); p = _f64(p)
        return lib().or_ccd(self._h, _d(y), _d(p))

    def pcg(self, y, b, eta):
        y = _f64(y); b = _f64(b)
        x = np.zeros(self.ndof)
        it = lib().or_pcg(self._h, _d(y), _d(b), _d(x), eta)
        return x, it

    def step(self):
        t = self.targets(self.step_index)
        st = OStats()
        rc = lib().or_step(self._h, _d(t) if t is not None else None, ctypes.byref(st))
        self.step_index += 1
        return rc, st.as_dict()

    def step_targets(self, t):
        """One step towards explicit targets (the layout of targets(n))."""
        st = OStats()
        t = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
        rc = lib().or_step(self._h, _d(t) if t is not None else None, ctypes.byref(st))
        return rc, st.as_dict()

    def set_timestep(self, h):
        lib().or_set_timestep(self._h, float(h))

    def set_friction_lag(self, passes):
        lib().or_set_friction_lag(self._h, int(passes))

    def set_kappa_adaptive(self, frac, factor=100.0):
        """Adaptive barrier stiffness: kappa doubles after an accepted Newton
        update whose smallest active-pair distance is below frac dhat and
        below the previous iterate's, capped at factor times the kappa at
        this call (frac = 0: off)."""
        lib().or_set_kappa_adaptive(self._h, float(frac), float(factor))

    def set_kappa(self, kappa):
        lib().or_set_kappa(self._h, float(kappa))

    def step_adaptive(self, max_depth=3):
        """One step with sub-stepping on failure (the recovery policy of the
        robustness variants): if the step ends without Newton convergence
        (status 3), it is taken again from its start as two steps of h/2, the
        first towards the mean of the previous and this step's targets, each
        retried the same way down to h / 2^max_depth.  Returns (status of the
        last piece, number of pieces)."""
        n = self.step_index
        h = float(self.scene["h"])
        t1 = self.targets(n)
        t0 = self.targets(n - 1 if n > 0 else 0)

        def run(y, v, hh, ta, tb, depth):
            self.set_state(y, v)
            self.set_timestep(hh)
            st = OStats()
            rc = lib().or_step(self._h, _d(tb) if tb is not None else None, ctypes.byref(st))
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

    # adjoint (one converged step n: y_prev -> y_next)
    def set_params(self, E=None, mu=None):
        """Replace the per-tet Young's moduli and/or the friction coefficient."""
        e = _f64(E) if E is not None else None
        lib().or_set_params(self._h, _d(e) if e is not None else None, -1.0 if mu is None else float(mu))

    def _t(self, n):
        t = self.targets(n)
        return _d(t) if t is not None else None

    def dG_dyn_T(self, y_prev, yd_prev, n, y_next, w):
        a = [_f64(v) for v in (y_prev, yd_prev, y_next, w)]
        out = np.zeros(self.ndof)
        lib().or_dG_dyn_T(self._h, _d(a[0]), _d(a[1]), self._t(n), _d(a[2]), _d(a[3]), _d(out))
        return out

    def dG_dtheta_T(self, y_prev, yd_prev, n, y_next, w):
        a = [_f64(v) for v in (y_prev, yd_prev, y_next, w)]
        eb = np.zeros(len(self.scene["tets"]))
        mb = lib().or_dG_dtheta_T(self._h, _d(a[0]), _d(a[1]), self._t(n), _d(a[2]), _d(a[3]), _d(eb))
        return eb, mb

    def step_vjp(self, y_prev, yd_prev, n, y_next, ybar_next, vbar_next, eta=1e-12):
        """Returns (status, ybar_prev, vbar_prev, Ebar, mubar, pcg_iters) for
        one step, with Ebar and mubar the parameter adjoints of this step alone."""
        a = [_f64(v) for v in (y_prev, yd_prev, y_next, ybar_next, vbar_next)]
        yb = np.zeros(self.ndof); vb = np.zeros(self.ndof)
        eb = np.zeros(len(self.scene["tets"])); mb = np.zeros(1); it = ctypes.c_int()
        rc = lib().or_step_vjp(self._h, _d(a[0]), _d(a[1]), self._t(n), _d(a[2]), _d(a[3]), _d(a[4]),
                               _d(yb), _d(vb), _d(eb), _d(mb), float(eta), ctypes.byref(it))
        return rc, yb, vb, eb, float(mb[0]), it.value


def rollout_loss(scene, y0, yd0, first_step, n_steps, tracked, target, E=None, mu=None, grad=False,
                 checkpoint_every=10, eta=1e-12):
    """Roll the scene from (y0, yd0) at step first_step over n_steps steps with
    parameters (E, mu) and return the loss sum_i |x_i - target_i|^2 over the
    tracked FEM vertices at the last step; with grad=True also dL/dE (per tet)
    and dL/dmu by the per-step adjoint, recomputing each checkpoint segment."""
    o = Oracle(scene)
    o.set_params(E, mu)
    y0 = _f64(y0); yd0 = _f64(yd0)
    idx = (3 * np.asarray(tracked)[:, None] + np.arange(3)[None, :]).ravel()
    ckpt = {}
    o.set_state(y0, yd0)
    for k in range(n_steps):
        if k % checkpoint_every == 0:
            ckpt[k] = o.state()
        o.step_index = first_step + k
        rc, _ = o.step()
        if rc != 0:
            raise RuntimeError(f"oracle step {first_step + k} returned {rc}")
    y, _ = o.state()
    diff = y[idx] - np.asarray(target, np.float64).ravel()
    loss = float(diff @ diff)
    if not grad:
        return loss
    ybar = np.zeros(o.ndof); ybar[idx] = 2.0 * diff
    vbar = np.zeros(o.ndof)
    Ebar = np.zeros(len(scene["tets"])); mubar = 0.0
    for c0 in sorted(ckpt, reverse=True):
        c1 = min(c0 + checkpoint_every, n_steps)
        states = [ckpt[c0]]
        o.set_state(*ckpt[c0])
        for k in range(c0, c1):
            o.step_index = first_step + k
            o.step()
            states.append(o.state())
        for k in range(c1 - 1, c0 - 1, -1):
            yp, vp = states[k - c0]
            yn, _ = states[k - c0 + 1]
            rc, ybar, vbar, eb, mb, _ = o.step_vjp(yp, vp, first_step + k, yn, ybar, vbar, eta)
            if rc != 0:
                raise RuntimeError(f"oracle adjoint of step {first_step + k} returned {rc}")
            Ebar += eb; mubar += mb
    return loss, Ebar, mubar


# single-pair helpers for unit pins
def dist2_pt(x):
    x = _f64(x); t = ctypes.c_int()
    return lib().or_dist2_pt(_d(x), ctypes.byref(t)), t.value


def dist2_ee(x):
    x = _f64(x); t = ctypes.c_int()
    return lib().or_dist2_ee(_d(x), ctypes.byref(t)), t.value


def dist2_derivs(kind, x):
    x = _f64(x)
    g = np.zeros(12); H = np.zeros(144)
    d2 = lib().or_dist2_derivs(kind, _d(x), _d(g), _d(H))
    return d2, g, H.reshape(12, 12)


def accd(kind, x, p, s=0.1):
    x = _f64(x); p = _f64(p)
    return lib().or_accd(kind, _d(x), _d(p), s)


def snh(F, mu, lam):
    """F as a 3x3 matrix; returns (Psi, P 3x3, dP/dF as 9x9 over column-major vec)."""
    Fv = _f64(np.asarray(F).T.ravel())
    P = np.zeros(9); H = np.zeros(81)
    psi = lib().or_snh(_d(Fv), mu, lam, _d(P), _d(H))
    return psi, P.reshape(3, 3).T, H.reshape(9, 9)


def barrier3(d, dhat):
    out = np.zeros(3)
    lib().or_barrier3(float(d), float(dhat), _d(out))
    return out


def psd_project(A):
    A = _f64(A).copy()
    lib().or_psd_project(_d(A), A.shape[0])
    return A
