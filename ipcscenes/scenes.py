"""Seeded synthetic scenes shaped like soft-gripper manipulation (PhyVisGen, Sec. III-C).

Everything here is input construction only: grids, tetrahedra, orientation of
the input mesh, body boxes, spring anchor points and drive trajectories.  No
energy, derivative, contact or solver arithmetic lives here, so both the HIP
library and the oracle can consume the same bits.

Scene dictionary layout (all arrays C-contiguous; float64 unless noted)
----------------------------------------------------------------------
FEM (deformable tetrahedra)
  X         (nv,3)   rest positions, also the initial positions (rest = initial)
  V         (nv,3)   initial velocities
  tets      (nt,4)   int32, positively oriented: det[X1-X0, X2-X0, X3-X0] > 0
  tet_E, tet_nu, tet_rho  (nt,)  Young's modulus, Poisson ratio, density
  vobj      (nv,)    int32 object id of every FEM vertex
Affine bodies (12 DOF: p, then the three columns of A)
  body_q, body_qdot (nb,12)
  body_mass (nb,)    body_S (nb,3,3) second moment about the centroid frame
  body_vol  (nb,)    body_kappa (nb,) orthogonality stiffness
  body_ext  (nb,3)   half extents of the body box (convergence measure)
  body_obj  (nb,)    int32 object id
Body contact geometry (positions in the body frame)
  bv_xbar (nbv,3), bv_body (nbv,) int32, btri (nbt,3) int32 into the body-vertex list
Static contact geometry (world positions)
  sv_x (nsv,3), stri (nst,3) int32 into the static-vertex list
Objects
  obj_kind (nobj,) int32: 0 = FEM mesh, 1 = affine body, 2 = static
  excl     (nex,2) int32 object pairs that never collide
Springs, E = 1/2 k |a - b|^2 (times h^2 in the incremental potential)
  sp_ka, sp_kb (ns,) int32 side kind: 0 FEM vertex, 1 body point, 2 drive target
  sp_ia, sp_ib (ns,) int32 vertex / body / driven-link slot
  sp_xa, sp_xb (ns,3) body-frame point (kind 1) or link-frame anchor (kind 2)
  sp_k (ns,)
Drives
  driven_body (nd,) int32 body driven by slot d
  drive_q (n_steps, nd, 12) target affine state of every driven link at t_{n+1}
Joint springs (joint-space drives: both sides body points, the b side's
body-frame point follows the joint reference)
  joint_spring (nj,) int32 spring index of every joint slot
  joint_xbar (n_steps, nj, 3) the b-side body-frame point of slot j at t_{n+1}
Scalars (0-d arrays): h, dhat, kappa (0 = automatic), mu, eps_v, newton_tol,
  max_newton, pcg_tol, max_pcg, ccd_s, n_steps; g (3,)
"""
import numpy as np

SCENE_KEYS = (
    "X", "V", "tets", "tet_E", "tet_nu", "tet_rho", "vobj",
    "body_q", "body_qdot", "body_mass", "body_S", "body_vol", "body_kappa",
    "body_ext", "body_obj",
    "bv_xbar", "bv_body", "btri", "sv_x", "stri",
    "obj_kind", "excl",
    "sp_ka", "sp_ia", "sp_xa", "sp_kb", "sp_ib", "sp_xb", "sp_k",
    "driven_body", "drive_q", "joint_spring", "joint_xbar",
    "h", "g", "dhat", "kappa", "mu", "eps_v", "newton_tol", "max_newton",
    "pcg_tol", "max_pcg", "ccd_s", "n_steps", "half_space",
)

INT_KEYS = {"tets", "vobj", "body_obj", "bv_body", "btri", "stri", "obj_kind",
            "excl", "sp_ka", "sp_ia", "sp_kb", "sp_ib", "driven_body", "joint_spring"}


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def hex_tets(nx, ny, nz):
    """Five-tetrahedron split of an nx*ny*nz hex grid with conforming faces.

    Grid vertex (i,j,k) has id (i*(ny+1)+j)*(nz+1)+k.  In each cell the four
    corners of odd global parity (i+j+k odd) form the central tetrahedron and
    every even corner with its three cell neighbours forms a corner
    tetrahedron, so the face diagonals of neighbouring cells agree.
    Orientation is not fixed here (see ``orient``).
    """
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()

    def vid(a, b, c):
        return ((I + a) * (ny + 1) + (J + b)) * (nz + 1) + (K + c)

    out = []
    cell_par = (I + J + K) % 2
    for par in (0, 1):
        sel = cell_par == par
        corners = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        odd = [cr for cr in corners if (par + sum(cr)) % 2 == 1]
        even = [cr for cr in corners if (par + sum(cr)) % 2 == 0]
        tl = [np.stack([vid(*cr)[sel] for cr in odd], axis=1)]
        for e in even:
            nb = [tuple(e[m] ^ (1 if m == q else 0) for m in range(3)) for q in range(3)]
            tl.append(np.stack([vid(*e)[sel]] + [vid(*n)[sel] for n in nb], axis=1))
        out.append(np.stack(tl, axis=1).reshape(-1, 4))
    return np.concatenate(out, axis=0).astype(np.int32)


def grid_vertices(nx, ny, nz, origin, spacing):
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    idx = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    return np.asarray(origin, np.float64) + idx * np.asarray(spacing, np.float64)


def orient(X, tets):
    """Swap two vertices of every tetrahedron with a negative signed volume."""
    t = tets.copy()
    a = X[t[:, 1]] - X[t[:, 0]]
    b = X[t[:, 2]] - X[t[:, 0]]
    c = X[t[:, 3]] - X[t[:, 0]]
    s = np.einsum("ij,ij->i", a, np.cross(b, c))
    neg = s < 0
    t[neg, 1], t[neg, 2] = tets[neg, 2], tets[neg, 1]
    return t


def box_surface(half):
    """8 corners and 12 outward triangles of an axis-aligned box centred at 0."""
    hx, hy, hz = half
    V = np.array([[sx * hx, sy * hy, sz * hz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                 np.float64)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    T = []
    for q in quads:
        for tri in ((q[0], q[1], q[2]), (q[0], q[2], q[3])):
            n = np.cross(V[tri[1]] - V[tri[0]], V[tri[2]] - V[tri[0]])
            c = V[list(tri)].mean(axis=0)
            T.append(tri if np.dot(n, c) > 0 else (tri[0], tri[2], tri[1]))
    return V, np.array(T, np.int32)


def ground_quad(half=1.0, z=0.0):
    """Two upward triangles over [-half, half]^2 split along the line y = -x."""
    V = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float64)
    T = np.array([[0, 1, 3], [1, 2, 3]], np.int32)
    return V, T


def ground_patch(center, size, spacing, z=0.0):
    """Finely triangulated static square patch, upward normals."""
    n = int(round(size / spacing))
    xs = center[0] - size / 2 + spacing * np.arange(n + 1)
    ys = center[1] - size / 2 + spacing * np.arange(n + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = (i * (n + 1) + j).ravel()
    v10 = v00 + (n + 1)
    v01 = v00 + 1
    v11 = v10 + 1
    T = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 0)
    return V, T.astype(np.int32)


def cylinder_mesh(radius, height, n_disk, n_layers, center_xy, z0):
    """Square grid mapped to a disk, extruded in layers; five tets per hex."""
    X = grid_vertices(n_disk, n_disk, n_layers, (-1.0, -1.0, 0.0), (2.0 / n_disk, 2.0 / n_disk, 1.0 / n_layers))
    u, v, w = X[:, 0], X[:, 1], X[:, 2]
    x = u * np.sqrt(1.0 - v * v / 2.0)
    y = v * np.sqrt(1.0 - u * u / 2.0)
    P = np.stack([center_xy[0] + radius * x, center_xy[1] + radius * y, z0 + height * w], axis=1)
    T = orient(P, hex_tets(n_disk, n_disk, n_layers))
    return P, T


def rotz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_axis(u, a):
    """Rotation by angle a about the unit axis u (Rodrigues' formula)."""
    u = np.asarray(u, np.float64) / np.linalg.norm(u)
    K = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return np.eye(3) + np.sin(a) * K + (1.0 - np.cos(a)) * (K @ K)


# --------------------------------------------------------------------------
# builder
# --------------------------------------------------------------------------
class _Builder:
    def __init__(self):
        self.X, self.tets, self.E, self.nu, self.rho, self.vobj = [], [], [], [], [], []
        self.nv = 0
        self.obj_kind = []
        self.excl = []
        self.bodies = []
        self.bv_xbar, self.bv_body, self.btri = [], [], []
        self.nbv = 0
        self.sv_x, self.stri = [], []
        self.nsv = 0
        self.springs = []
        self.driven = []
        self.joints = []   # (spring index, (n_steps, 3) b-side body-frame points)

    def add_fem(self, X, tets, E, nu, rho):
        obj = len(self.obj_kind)
        self.obj_kind.append(0)
        off = self.nv
        nt = len(tets)
        self.X.append(np.asarray(X, np.float64))
        self.tets.append(np.asarray(tets, np.int32) + off)
        self.E.append(np.broadcast_to(np.asarray(E, np.float64), (nt,)).copy())
        self.nu.append(np.full(nt, nu, np.float64))
        self.rho.append(np.full(nt, rho, np.float64))
        self.vobj.append(np.full(len(X), obj, np.int32))
        self.nv += len(X)
        return obj, off

    def add_body(self, center, size, mass, kappa=1e8, contact=False):
        size = np.asarray(size, np.float64)
        b = len(self.bodies)
        obj = len(self.obj_kind)
        self.obj_kind.append(1)
        q = np.concatenate([np.asarray(center, np.float64), np.eye(3).T.ravel()])
        S = mass / 12.0 * np.diag(size ** 2)
        self.bodies.append(dict(q=q, mass=mass, S=S, vol=float(np.prod(size)), kappa=kappa,
                                ext=size / 2, obj=obj))
        if contact:
            V, T = box_surface(size / 2)
            self.bv_xbar.append(V)
            self.bv_body.append(np.full(len(V), b, np.int32))
            self.btri.append(T + self.nbv)
            self.nbv += len(V)
        return b

    def add_static(self, V, T):
        obj = len(self.obj_kind)
        self.obj_kind.append(2)
        self.sv_x.append(np.asarray(V, np.float64))
        self.stri.append(np.asarray(T, np.int32) + self.nsv)
        self.nsv += len(V)
        return obj

    def body_center(self, b):
        return self.bodies[b]["q"][:3]

    def add_spring(self, a, b, k):
        self.springs.append((a, b, float(k)))

    def add_joint_spring(self, child, parent_body, xbar_traj, k):
        """A spring from a child side (kind, index, point) to a point of the
        parent body whose body-frame coordinates follow xbar_traj[n] at step n."""
        xbar_traj = np.asarray(xbar_traj, np.float64)
        self.joints.append((len(self.springs), xbar_traj))
        self.springs.append((child, (1, parent_body, xbar_traj[0]), float(k)))

    def add_driven(self, body):
        self.driven.append(body)
        return len(self.driven) - 1

    def finish(self, params, drive_q):
        d = {}
        cat = lambda L, shape, dt: (np.concatenate(L, 0).astype(dt) if L else np.zeros(shape, dt))
        d["X"] = cat(self.X, (0, 3), np.float64)
        d["V"] = np.zeros_like(d["X"])
        d["tets"] = cat(self.tets, (0, 4), np.int32)
        d["tet_E"] = cat(self.E, (0,), np.float64)
        d["tet_nu"] = cat(self.nu, (0,), np.float64)
        d["tet_rho"] = cat(self.rho, (0,), np.float64)
        d["vobj"] = cat(self.vobj, (0,), np.int32)
        nb = len(self.bodies)
        d["body_q"] = np.array([bd["q"] for bd in self.bodies], np.float64).reshape(nb, 12)
        d["body_qdot"] = np.zeros((nb, 12))
        d["body_mass"] = np.array([bd["mass"] for bd in self.bodies], np.float64)
        d["body_S"] = np.array([bd["S"] for bd in self.bodies], np.float64).reshape(nb, 3, 3)
        d["body_vol"] = np.array([bd["vol"] for bd in self.bodies], np.float64)
        d["body_kappa"] = np.array([bd["kappa"] for bd in self.bodies], np.float64)
        d["body_ext"] = np.array([bd["ext"] for bd in self.bodies], np.float64).reshape(nb, 3)
        d["body_obj"] = np.array([bd["obj"] for bd in self.bodies], np.int32)
        d["bv_xbar"] = cat(self.bv_xbar, (0, 3), np.float64)
        d["bv_body"] = cat(self.bv_body, (0,), np.int32)
        d["btri"] = cat(self.btri, (0, 3), np.int32)
        d["sv_x"] = cat(self.sv_x, (0, 3), np.float64)
        d["stri"] = cat(self.stri, (0, 3), np.int32)
        d["obj_kind"] = np.array(self.obj_kind, np.int32)
        d["excl"] = np.array(self.excl, np.int32).reshape(-1, 2)
        ns = len(self.springs)
        ka = np.zeros(ns, np.int32); ia = np.zeros(ns, np.int32); xa = np.zeros((ns, 3))
        kb = np.zeros(ns, np.int32); ib = np.zeros(ns, np.int32); xb = np.zeros((ns, 3))
        kk = np.zeros(ns)
        for s, (a, b, k) in enumerate(self.springs):
            for (kind, idx, xbar), K, I_, XB in ((a, ka, ia, xa), (b, kb, ib, xb)):
                K[s] = kind; I_[s] = idx; XB[s] = xbar
            kk[s] = k
        d.update(sp_ka=ka, sp_ia=ia, sp_xa=xa, sp_kb=kb, sp_ib=ib, sp_xb=xb, sp_k=kk)
        d["driven_body"] = np.array(self.driven, np.int32)
        d["drive_q"] = np.asarray(drive_q, np.float64).reshape(int(params["n_steps"]), len(self.driven), 12)
        nst = int(params["n_steps"])
        d["joint_spring"] = np.array([j for j, _ in self.joints], np.int32)
        d["joint_xbar"] = (np.stack([t[:nst] for _, t in self.joints], 1) if self.joints else np.zeros((nst, 0, 3))).astype(np.float64)
        d["joint_xbar"] = np.ascontiguousarray(d["joint_xbar"])
        for k, v in params.items():
            d[k] = np.asarray(v, np.float64)
        validate_scene(d)
        return d


def _params(**kw):
    p = dict(h=0.01, g=np.array([0.0, 0.0, -9.81]), dhat=1e-3, kappa=0.0, mu=0.3, eps_v=1e-3,
             newton_tol=1e-6, max_newton=100, pcg_tol=1e-4, max_pcg=20000, ccd_s=0.1, n_steps=20,
             half_space=np.zeros(4))
    p.update(kw)
    return p


def validate_scene(d):
    for k in SCENE_KEYS:
        if k not in d:
            raise KeyError(f"scene is missing {k}")
        want = np.int32 if k in INT_KEYS else np.float64
        if d[k].dtype != want:
            raise TypeError(f"{k}: dtype {d[k].dtype}, expected {want}")
        if not d[k].flags.c_contiguous:
            raise ValueError(f"{k} is not contiguous")
    return d


# --------------------------------------------------------------------------
# the gripper (Sec. III-C.2): pads stitched to rigid bases, bases fixed to
# fingers, fingers / hand / arm links driven toward kinematic targets
# --------------------------------------------------------------------------
def _pad(cells, size, lo):
    nx, ny, nz = cells
    X = grid_vertices(nx, ny, nz, lo, (size[0] / nx, size[1] / ny, size[2] / nz))
    return X, orient(X, hex_tets(nx, ny, nz))


def _add_gripper(b, rng, *, center_xy, z_mid, inner_half_gap, pad_cells, pad_E, pad_nu,
                 k_c=1e4, k_F=1e6, k_J=1e5, n_steps, h, t_close, v_close, v_lift, pert=True):
    """Two pads + bases + fingers + hand + two arm links; returns the drive trajectory."""
    cx, cy = center_xy
    psize = np.array([0.04, 0.02, 0.02])
    pads = []
    for side in (-1, 1):
        ylo = cy + inner_half_gap if side > 0 else cy - inner_half_gap - psize[1]
        lo = (cx - psize[0] / 2, ylo, z_mid - psize[2] / 2)
        X, T = _pad(pad_cells, psize, lo)
        obj, off = b.add_fem(X, T, pad_E, pad_nu, 1000.0)
        # the attachment set: the outer face (far from the object)
        outer = np.isclose(X[:, 1], ylo + (0.0 if side < 0 else psize[1]))
        pads.append((obj, off, X, np.nonzero(outer)[0], side, ylo))
    fingers, bases = [], []
    for obj, off, X, att, side, ylo in pads:
        y_face = ylo + (0.0 if side < 0 else psize[1])
        base_c = np.array([cx, y_face + side * 0.002, z_mid])
        base = b.add_body(base_c, (0.04, 0.004, 0.02), 0.05)
        for i in att:
            b.add_spring((0, off + i, np.zeros(3)), (1, base, X[i] - base_c), k_c)
        fing_c = np.array([cx, y_face + side * 0.009, z_mid + 0.01])
        fing = b.add_body(fing_c, (0.02, 0.01, 0.04), 0.1)
        for a in (np.zeros(3), 0.01 * np.eye(3)[0], 0.01 * np.eye(3)[1], 0.01 * np.eye(3)[2]):
            P = base_c + a
            b.add_spring((1, base, P - base_c), (1, fing, P - fing_c), k_F)
        bases.append(base)
        fingers.append((fing, fing_c, side))
    hand_c = np.array([cx, cy, z_mid + 0.05])
    hand = b.add_body(hand_c, (0.1, 0.04, 0.03), 0.5)
    arm = [b.add_body(hand_c + np.array([0, 0, 0.12 * (k + 1)]), (0.06, 0.06, 0.1), 1.0) for k in range(2)]
    links = [(f, c, s) for f, c, s in fingers] + [(hand, hand_c, 0)] + [(a, b.body_center(a).copy(), 0) for a in arm]
    anchors = [np.zeros(3), 0.01 * np.eye(3)[0], 0.01 * np.eye(3)[1], 0.01 * np.eye(3)[2]]
    for body, _, _ in links:
        slot = b.add_driven(body)
        for a in anchors:
            b.add_spring((1, body, a), (2, slot, a), k_J)
    # seeded hand perturbation: sum of three sines in x, y and yaw
    amp = rng.uniform(0.0, 1e-3, size=(3, 3)) if pert else np.zeros((3, 3))
    amp[2] = rng.uniform(0.0, np.deg2rad(1.0), size=3) if pert else 0.0
    freq = rng.uniform(0.5, 2.0, size=(3, 3))
    phase = rng.uniform(0.0, 2 * np.pi, size=(3, 3))
    nd = len(links)
    drive = np.zeros((n_steps, nd, 12))
    for n in range(n_steps):
        t = (n + 1) * h
        pert_v = [np.sum(amp[c] * (np.sin(2 * np.pi * freq[c] * t + phase[c]) - np.sin(phase[c]))) for c in range(3)]
        R = rotz(pert_v[2])
        shift = np.array([pert_v[0], pert_v[1], v_lift * max(0.0, t - t_close)])
        for d_, (body, c0, side) in enumerate(links):
            rel = c0 - hand_c
            if side != 0:
                rel = rel + np.array([0.0, -side * v_close * min(t, t_close), 0.0])
            p = hand_c + shift + R @ rel
            drive[n, d_] = np.concatenate([p, R.T.ravel()])  # columns of R
    return drive, [p[0] for p in pads], bases


# vertices of a regular tetrahedron of circumradius 1 cm centred on the origin:
# four spring points whose first moment vanishes and whose second moment is
# isotropic
TETRA_PTS = 0.01 / np.sqrt(3.0) * np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])


def _add_arm_gripper(b, rng, *, center_xy, z_mid, inner_half_gap, pad_cells, pad_E, pad_nu,
                     k_c=1e4, k_F=1e6, k_J=1e5, n_steps, h, t_close, v_close, v_lift, pert=True, link_len=0.1):
    """The gripper of _add_gripper on a joint-space arm: the fingers ride on
    prismatic joints of the hand, the hand on a revolute wrist of a 7-link
    revolute chain whose top link is anchored to the world (the only drive
    target).  Each revolute joint is two springs on its axis at +-1 cm from
    the joint centre (k_F) and two springs at +-1 cm along a normal of the
    axis whose parent-side points follow the joint angle (k_J); each prismatic
    joint, the finger mounts and the anchor are four springs on a regular
    tetrahedron centred on the body (TETRA_PTS), whose parent-side points
    follow the joint offset.  Every point set is centred on its joint, so a
    load through the joint centre moves the bodies without turning them.  The chain hangs above the hand (axes z, x, z, x, z,
    x, z from the top); the lift bends joints 2, 4, 6 by phi, -2 phi, phi so
    the hand rises without turning; joints 1, 3, 5, 7 carry seeded yaw
    perturbations.  Returns the drive trajectory (anchor only)."""
    cx, cy = center_xy
    psize = np.array([0.04, 0.02, 0.02])
    pads = []
    for side in (-1, 1):
        ylo = cy + inner_half_gap if side > 0 else cy - inner_half_gap - psize[1]
        lo = (cx - psize[0] / 2, ylo, z_mid - psize[2] / 2)
        X, T = _pad(pad_cells, psize, lo)
        obj, off = b.add_fem(X, T, pad_E, pad_nu, 1000.0)
        outer = np.isclose(X[:, 1], ylo + (0.0 if side < 0 else psize[1]))
        pads.append((obj, off, X, np.nonzero(outer)[0], side, ylo))
    fingers, bases = [], []
    for obj, off, X, att, side, ylo in pads:
        y_face = ylo + (0.0 if side < 0 else psize[1])
        base_c = np.array([cx, y_face + side * 0.002, z_mid])
        base = b.add_body(base_c, (0.04, 0.004, 0.02), 0.05)
        for i in att:
            b.add_spring((0, off + i, np.zeros(3)), (1, base, X[i] - base_c), k_c)
        fing_c = np.array([cx, y_face + side * 0.009, z_mid + 0.01])
        fing = b.add_body(fing_c, (0.02, 0.01, 0.04), 0.1)
        for a in TETRA_PTS:
            P = fing_c + a
            b.add_spring((1, base, P - base_c), (1, fing, P - fing_c), k_F)
        bases.append(base)
        fingers.append((fing, fing_c, side))
    hand_c = np.array([cx, cy, z_mid + 0.05])
    hand = b.add_body(hand_c, (0.1, 0.04, 0.03), 0.5)
    chain = [(b.add_body(hand_c + np.array([0.0, 0.0, link_len * (7 - k)]), (0.06, 0.06, 0.1), 1.0),
              hand_c + np.array([0.0, 0.0, link_len * (7 - k)])) for k in range(7)] + [(hand, hand_c)]
    ex, ey, ez = np.eye(3)
    axes = [ez, ex, ez, ex, ez, ex, ez]
    # joint references at t_{n+1}
    t = (np.arange(n_steps) + 1) * h
    dz = v_lift * np.maximum(0.0, t - t_close)
    phi = np.arccos(np.clip(1.0 - dz / (4.0 * link_len), -1.0, 1.0))
    theta = np.zeros((n_steps, 7))
    theta[:, 1], theta[:, 3], theta[:, 5] = phi, -2.0 * phi, phi
    amp = rng.uniform(0.0, np.deg2rad(0.5), size=(4, 3)) if pert else np.zeros((4, 3))
    freq = rng.uniform(0.5, 2.0, size=(4, 3))
    phase = rng.uniform(0.0, 2 * np.pi, size=(4, 3))
    for i, j in enumerate((0, 2, 4, 6)):
        theta[:, j] += np.sum(amp[i] * (np.sin(2 * np.pi * freq[i] * t[:, None] + phase[i]) - np.sin(phase[i])), 1)
    for j in range(7):
        (P, cP), (C, cC) = chain[j], chain[j + 1]
        O = 0.5 * (cP + cC)
        u = axes[j]
        v = ey if u is not ey else ez
        v = v - u * (v @ u); v = v / np.linalg.norm(v)
        for a in (O + 0.01 * u, O - 0.01 * u):
            b.add_spring((1, C, a - cC), (1, P, a - cP), k_F)
        for a in (O + 0.01 * v, O - 0.01 * v):
            traj = np.array([(O - cP) + rot_axis(u, th) @ (a - O) for th in theta[:, j]])
            b.add_joint_spring((1, C, a - cC), P, traj, k_J)
    d_close = v_close * np.minimum(t, t_close)
    for fing, fing_c, side in fingers:
        inward = -side * ey
        for a in fing_c + TETRA_PTS:
            traj = (a - hand_c)[None, :] + d_close[:, None] * inward[None, :]
            b.add_joint_spring((1, fing, a - fing_c), hand, traj, k_J)
    top, c_top = chain[0]
    slot = b.add_driven(top)
    for a in TETRA_PTS:
        b.add_spring((1, top, a), (2, slot, a), k_J)
    drive = np.zeros((n_steps, 1, 12))
    drive[:, 0] = np.concatenate([c_top, np.eye(3).T.ravel()])
    return drive, [p[0] for p in pads], bases


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def block_drop(seed=0, n_steps=20, ground="triangles"):
    """Soft 5x5x5-cell block (625 tets) dropped 2 mm onto a static plane:
    two static triangles (ground="triangles") or the analytic half-space
    z >= 0 (ground="half_space")."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder()
    n = 5
    X = grid_vertices(n, n, n, (0.3 - 0.025, 0.3 - 0.025, 0.002), (0.01, 0.01, 0.01))
    X = X + rng.uniform(-1e-4, 1e-4, size=X.shape)
    b.add_fem(X, orient(X, hex_tets(n, n, n)), 1e5, 0.45, 1000.0)
    hs = _ground(b, ground)
    p = _params(h=0.01, dhat=1e-3, mu=0.3, n_steps=n_steps, half_space=hs)
    return b.finish(p, np.zeros((n_steps, 0, 12)))


def _ground(b, ground):
    """The ground at z = 0: two static triangles, or the half-space (its
    (n, c) is returned; zeros for triangles)."""
    if ground == "triangles":
        b.add_static(*ground_quad())
        return np.zeros(4)
    if ground == "half_space":
        return np.array([0.0, 0.0, 1.0, 0.0])
    raise ValueError(ground)


def gripper_squeeze(seed=0, n_steps=200, pad_cells=(20, 10, 10), pad_E=2e5, mu=0.5, h=0.005):
    """Two soft pads on rigid fingers squeezing a free 4 cm, 0.2 kg box, then lifting it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder()
    cxy = (0.3, 0.3)
    box = b.add_body((cxy[0], cxy[1], 0.02 + 5e-4), (0.04, 0.04, 0.04), 0.2, contact=True)
    drive, _, _ = _add_gripper(b, rng, center_xy=cxy, z_mid=0.02 + 5e-4, inner_half_gap=0.022,
                               pad_cells=pad_cells, pad_E=pad_E, pad_nu=0.47, n_steps=n_steps, h=h,
                               t_close=0.5, v_close=0.01, v_lift=0.02)
    b.add_static(*ground_quad())
    del box
    p = _params(h=h, dhat=1e-3, mu=mu, n_steps=n_steps)
    return b.finish(p, drive)


def arm_squeeze(seed=0, n_steps=200, pad_cells=(20, 10, 10), pad_E=2e5, mu=0.5, h=0.005):
    """The squeeze of gripper_squeeze on a joint-space arm (see _add_arm_gripper):
    the box is squeezed by fingers on prismatic joints and lifted by bending
    the chain, whose top link alone is anchored."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder()
    cxy = (0.3, 0.3)
    b.add_body((cxy[0], cxy[1], 0.02 + 5e-4), (0.04, 0.04, 0.04), 0.2, contact=True)
    drive, _, _ = _add_arm_gripper(b, rng, center_xy=cxy, z_mid=0.02 + 5e-4, inner_half_gap=0.022,
                                   pad_cells=pad_cells, pad_E=pad_E, pad_nu=0.47, n_steps=n_steps, h=h,
                                   t_close=0.5, v_close=0.01, v_lift=0.02)
    b.add_static(*ground_quad())
    p = _params(h=h, dhat=1e-3, mu=mu, n_steps=n_steps)
    return b.finish(p, drive)


def contact_rich(seed=0, n_steps=100, s_g=8e-4, n_disk=30, n_layers=40):
    """Two pads squeezing a ~180k-tet soft cylinder that rests on a finely meshed ground patch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder()
    cxy = (0.3, 0.3)
    r, H = 0.03, 0.1
    P, T = cylinder_mesh(r, H, n_disk, n_layers, cxy, 2.5e-4)
    E = 5e4 * np.exp(0.3 * rng.standard_normal(len(T)) - 0.045)
    b.add_fem(P, T, E, 0.45, 1000.0)
    drive, _, _ = _add_gripper(b, rng, center_xy=cxy, z_mid=2.5e-4 + H / 2, inner_half_gap=r + 1e-3,
                               pad_cells=(20, 10, 10), pad_E=2e5, pad_nu=0.47, n_steps=n_steps, h=0.005,
                               t_close=0.2, v_close=0.01, v_lift=0.05)
    b.add_static(*ground_patch(cxy, 0.1, s_g))
    p = _params(h=0.005, dhat=5e-4, mu=0.5, n_steps=n_steps)
    return b.finish(p, drive)


def batched_squeeze(seed=0, n_scenes=256, n_steps=100):
    """Uneven squeeze scenes: pad resolution, stiffness and friction drawn per scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(n_scenes):
        Ns = float(np.exp(rng.uniform(np.log(1e3), np.log(4e4))))
        ny = max(2, int(round((Ns / 20.0) ** (1.0 / 3.0))))
        nx = max(2, int(round(Ns / (10.0 * ny * ny))))
        E = float(rng.uniform(5e4, 5e5))
        mu = float(rng.uniform(0.2, 0.8))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        out.append(gripper_squeeze(seed=sub, n_steps=n_steps, pad_cells=(nx, ny, ny), pad_E=E, mu=mu))
    return out


def adjoint_squeeze(seed=0):
    """The squeeze scene plus the seeded tracked nodes of the differentiation workload."""
    d = gripper_squeeze(seed=seed, n_steps=90)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    # 64 tracked pad surface vertices (any pad vertex on the box-facing face)
    X = d["X"]
    inner = np.nonzero(np.isclose(np.abs(X[:, 1] - 0.3), 0.022))[0]
    tracked = np.sort(rng.choice(inner, size=64, replace=False)).astype(np.int32)
    z_E = rng.standard_normal(len(d["tets"]))
    return d, dict(first_step=40, n_steps=50, tracked=tracked, target_E_scale=np.exp(0.2 * z_E),
                   target_mu_scale=1.1, checkpoint_every=10)


def tiny_scene(kind="tet", seed=0, **kw):
    """Small scenes for unit checks.

    tet      one tetrahedron, free (no contact geometry besides its own surface)
    two_tets two tetrahedra sharing a face
    cube     a 2x2x2-cell block resting above the 2-triangle ground
    edge_tet one tetrahedron on an edge nearly parallel to the ground's diagonal
             edge (an active edge-edge mollifier)
    pad_box  a 2x1x1-cell pad squeezing a small affine box (springs, bodies, contact)
    arm_box  pad_box's squeeze on the joint-space arm (joint springs)
    free_body one affine box (4 cm, 0.2 kg) with contact geometry and nothing to touch

    ground="half_space" replaces the two ground triangles of cube, edge_tet,
    pad_box and arm_box by the analytic half-space z >= 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder()
    drive = None
    ground = kw.pop("ground", "triangles")
    p = _params(n_steps=kw.pop("n_steps", 4), **kw)
    if kind == "tet":
        X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64) * 0.01 + 0.3
        b.add_fem(X, np.array([[0, 1, 2, 3]], np.int32), 1e5, 0.4, 1000.0)
    elif kind == "two_tets":
        X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], np.float64) * 0.01 + 0.3
        T = orient(X, np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32))
        b.add_fem(X, T, 1e5, 0.4, 1000.0)
    elif kind == "cube":
        X = grid_vertices(2, 2, 2, (0.29, 0.29, 0.0015), (0.01, 0.01, 0.01))
        X = X + rng.uniform(-1e-4, 1e-4, size=X.shape)
        b.add_fem(X, orient(X, hex_tets(2, 2, 2)), 1e5, 0.45, 1000.0)
        p["half_space"] = _ground(b, ground)
    elif kind == "edge_tet":
        # one tetrahedron resting on an edge 0.6 mm above the ground's diagonal
        # edge and about 1 degree off parallel to it
        X = np.array([[0.005, -0.005, 0.0], [-0.005, 0.005 + 2.5e-4, 0.0],
                      [0.005, 0.005, 0.008], [-0.005, -0.005, 0.008]], np.float64) + [0.0, 0.0, 6e-4]
        b.add_fem(X, orient(X, np.array([[0, 1, 2, 3]], np.int32)), 1e5, 0.4, 1000.0)
        p["half_space"] = _ground(b, ground)
    elif kind == "free_body":
        b.add_body((0.3, 0.3, 0.5), (0.04, 0.04, 0.04), 0.2, contact=True)
    elif kind == "arm_box":
        b.add_body((0.3, 0.3, 0.01 + 5e-4), (0.02, 0.02, 0.02), 0.05, contact=True)
        drive, _, _ = _add_arm_gripper(b, rng, center_xy=(0.3, 0.3), z_mid=0.01 + 5e-4, inner_half_gap=0.0115,
                                       pad_cells=(4, 2, 2), pad_E=1e5, pad_nu=0.45, n_steps=int(p["n_steps"]),
                                       h=p["h"], t_close=0.5, v_close=0.01, v_lift=0.02)
        p["half_space"] = _ground(b, ground)
    elif kind == "pad_box":
        b.add_body((0.3, 0.3, 0.01 + 5e-4), (0.02, 0.02, 0.02), 0.05, contact=True)
        drive, _, _ = _add_gripper(b, rng, center_xy=(0.3, 0.3), z_mid=0.01 + 5e-4, inner_half_gap=0.0115,
                                   pad_cells=(4, 2, 2), pad_E=1e5, pad_nu=0.45, n_steps=int(p["n_steps"]),
                                   h=p["h"], t_close=0.5, v_close=0.01, v_lift=0.02)
        p["half_space"] = _ground(b, ground)
    else:
        raise ValueError(kind)
    if drive is None:
        drive = np.zeros((int(p["n_steps"]), 0, 12))
    return b.finish(p, drive)


def tet_surface(P, T):
    """Boundary triangles of a tet mesh, oriented outward, on surface-local
    vertex numbers: (surface positions, triangles, volume index of every
    surface vertex)."""
    P = np.asarray(P, np.float64)
    T = np.asarray(T, np.int64).copy()
    vol = np.einsum("ij,ij->i", np.cross(P[T[:, 1]] - P[T[:, 0]], P[T[:, 2]] - P[T[:, 0]]), P[T[:, 3]] - P[T[:, 0]])
    neg = vol < 0
    T[neg, 1], T[neg, 2] = T[neg, 2].copy(), T[neg, 1].copy()
    a, b, c, d = T.T
    faces = np.stack([np.stack(f, 1) for f in ((b, c, d), (a, d, c), (a, b, d), (a, c, b))], 1).reshape(-1, 3)
    _, inv, cnt = np.unique(np.sort(faces, 1), axis=0, return_inverse=True, return_counts=True)
    bnd = faces[cnt[inv.ravel()] == 1]
    verts = np.unique(bnd.ravel())
    local = np.full(len(P), -1, np.int64)
    local[verts] = np.arange(len(verts))
    tri = local[bnd].astype(np.int32)
    return P[verts].copy(), tri, verts.astype(np.int32)


def dualmesh_frames(seed=0, n_frames=100, n_disk=30, n_layers=40, radius=0.03, height=0.1):
    """Coarse render input of the dual-mesh mapping: the surface of the soft
    cylinder of contact_rich (6602 vertices, 13200 triangles at the default
    resolution) and n_frames of its positions under a seeded smooth
    deformation (a squeeze that varies along the height, a twist and a
    sway), as a trajectory of simulated states would give them.  Returns
    (triangles (m, 3) int32, frames (n_frames, n, 3) float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P, T = cylinder_mesh(radius, height, n_disk, n_layers, (0.3, 0.3), 2.5e-4)
    X0, tri, _ = tet_surface(P, T)
    c = np.array([0.3, 0.3, 0.0])
    rel = X0 - c
    zeta = (X0[:, 2] - X0[:, 2].min()) / height
    amp = rng.uniform(0.05, 0.15, size=3)
    phase = rng.uniform(0.0, 2 * np.pi, size=3)
    frames = np.empty((n_frames,) + X0.shape)
    for f in range(n_frames):
        s = f / max(n_frames - 1, 1)
        sq = 1.0 - amp[0] * np.sin(np.pi * s + phase[0]) ** 2 * np.sin(np.pi * zeta)
        tw = amp[1] * s * zeta
        sway = amp[2] * 0.01 * np.sin(2 * np.pi * s + phase[2]) * zeta ** 2
        x = rel[:, 0] * np.cos(tw) - rel[:, 1] * np.sin(tw)
        y = rel[:, 0] * np.sin(tw) + rel[:, 1] * np.cos(tw)
        frames[f, :, 0] = c[0] + sq * x + sway
        frames[f, :, 1] = c[1] + sq * y
        frames[f, :, 2] = X0[:, 2]
    return tri, frames
