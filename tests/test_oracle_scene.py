"""Scene-level pins of the oracle: finite differences of the whole incremental
potential, brute-force pair sets, LAPACK for the linear solve, closed-form
dynamics and exact-rational non-penetration.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import ipcscenes as S
import oracle as O

rng = np.random.default_rng(7)


def advanced(scene, n):
    o = O.Oracle(scene)
    for _ in range(n):
        rc, _ = o.step()
        assert rc == 0
    return o


@pytest.fixture(scope="module")
def cube_contact():
    o = advanced(S.tiny_scene("cube", h=0.01, n_steps=8), 6)
    o.begin_step()
    y, _ = o.state()
    pt, ee = o.pairs(y)
    assert len(pt) > 0
    return o, y


@pytest.fixture(scope="module")
def padbox_contact():
    o = advanced(S.tiny_scene("pad_box", h=0.01, n_steps=40), 30)
    o.begin_step()
    y, _ = o.state()
    pt, ee = o.pairs(y)
    assert len(pt) > 0 and len(ee) > 0
    return o, y


def _fd_gradient(o, y, h):
    g = np.zeros_like(y)
    for i in range(len(y)):
        e = np.zeros_like(y); e[i] = h
        g[i] = (o.energy(y + e)[0] - o.energy(y - e)[0]) / (2 * h)
    return g


@pytest.mark.parametrize("fx", ["cube_contact", "padbox_contact"])
def test_gradient_fd(fx, request):
    o, y = request.getfixturevalue(fx)
    y = y + 1e-6 * rng.standard_normal(len(y)) * (np.arange(len(y)) < 3 * len(o.scene["X"]))
    g, gabs = o.gradient(y)
    gfd = _fd_gradient(o, y, 1e-8)
    err = np.abs(g - gfd)
    assert np.all(err <= 1e-4 * gabs + 1e-13), np.max(err / (gabs + 1e-30))


@pytest.mark.parametrize("fx", ["cube_contact", "padbox_contact"])
def test_hessian_fd(fx, request):
    o, y = request.getfixturevalue(fx)
    # move off zero slip: the friction mollifier has a |u|^3 term whose Hessian
    # is continuous but not differentiable at u = 0
    y = y + 1e-6 * rng.standard_normal(len(y)) * (np.arange(len(y)) < 3 * len(o.scene["X"]))
    for _ in range(3):
        v = rng.standard_normal(len(y))
        Hv = o.hess_matvec(y, v, project=False)
        h = 1e-9
        fd = (o.gradient(y + h * v)[0] - o.gradient(y - h * v)[0]) / (2 * h)
        assert np.linalg.norm(Hv - fd) <= 1e-5 * np.linalg.norm(Hv)


@pytest.mark.parametrize("fx", ["cube_contact", "padbox_contact"])
def test_projected_hessian_psd(fx, request):
    o, y = request.getfixturevalue(fx)
    for _ in range(5):
        v = rng.standard_normal(len(y))
        Hv = o.hess_matvec(y, v, project=True)
        assert v @ Hv > 0
    # projection only ever adds: v^T [H]+ v >= v^T H v
    v = rng.standard_normal(len(y))
    assert v @ o.hess_matvec(y, v, True) >= v @ o.hess_matvec(y, v, False) - 1e-12 * abs(v @ o.hess_matvec(y, v, True))


def _brute_pairs(o, y):
    x = o.world(y)
    tris = o.tris(); edges = o.edges()
    sc = o.scene
    nv, nbv = len(sc["X"]), len(sc["bv_xbar"])
    obj = np.concatenate([sc["vobj"], sc["body_obj"][sc["bv_body"]] if nbv else np.zeros(0, np.int32),
                          np.full(len(sc["sv_x"]), int(np.nonzero(sc["obj_kind"] == 2)[0][0]) if len(sc["sv_x"]) else -1, np.int32)])
    kind = sc["obj_kind"]

    def allowed(a, b):
        if kind[a] == 2 and kind[b] == 2:
            return False
        if a == b and kind[a] == 1:
            return False
        return True

    dh2 = float(sc["dhat"]) ** 2
    surf = np.unique(tris)
    pt = []
    for v in surf:
        for t in tris:
            if v in t or not allowed(obj[v], obj[t[0]]):
                continue
            if O.dist2_pt(np.concatenate([x[v], x[t[0]], x[t[1]], x[t[2]]]))[0] < dh2:
                pt.append((v, *t))
    ee = []
    for i in range(len(edges)):
        for j in range(i + 1, len(edges)):
            a, b = edges[i], edges[j]
            if len({*a, *b}) < 4 or not allowed(obj[a[0]], obj[b[0]]):
                continue
            if O.dist2_ee(np.concatenate([x[a[0]], x[a[1]], x[b[0]], x[b[1]]]))[0] < dh2:
                ee.append((*a, *b))
    return sorted(pt), sorted(ee)


@pytest.mark.parametrize("fx", ["cube_contact", "padbox_contact"])
def test_pairs_brute_force(fx, request):
    o, y = request.getfixturevalue(fx)
    pt, ee = o.pairs(y)
    bpt, bee = _brute_pairs(o, y)
    assert [tuple(r) for r in pt] == bpt
    assert [tuple(r) for r in ee] == bee


def test_pcg_matches_lapack(padbox_contact):
    o, y = padbox_contact
    n = len(y)
    H = np.stack([o.hess_matvec(y, e, True) for e in np.eye(n)], 1)
    b = rng.standard_normal(n)
    x, it = o.pcg(y, b, 1e-13)
    ref = np.linalg.solve(H, b)
    assert it > 0
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_surface_counts_of_block():
    o = O.Oracle(S.block_drop())
    assert o.ntri == 300 + 2 and o.nedge == 450 + 5
    m = o.mass()
    assert m.sum() == pytest.approx(0.125, rel=1e-3)   # the jittered mesh changes the volume slightly


def test_free_fall_closed_form():
    sc = S.tiny_scene("tet", n_steps=6, h=0.01)
    o = O.Oracle(sc)
    x0 = sc["X"].copy()
    g = sc["g"]
    for n in range(1, 7):
        assert o.step()[0] == 0
        y, _ = o.state()
        ref = x0 + 0.01 ** 2 * g * n * (n + 1) / 2
        assert np.abs(y.reshape(-1, 3) - ref).max() <= 1e-5 * 0.01 * o.L


def test_momentum_conserved_without_gravity():
    # its own generator: the velocities must not depend on the tests run before
    # (some draws leave the Newton measure above its tolerance at the energy's
    # rounding floor; this one converges)
    sc = S.tiny_scene("two_tets", n_steps=5, h=0.01)
    sc["g"] = np.zeros(3)
    sc["V"] = 0.05 * np.random.default_rng(0).standard_normal(sc["V"].shape)
    o = O.Oracle(sc)
    m = o.mass()
    p0 = (m[:, None] * sc["V"]).sum(0)
    for _ in range(5):
        assert o.step()[0] == 0
        _, v = o.state()
        p = (m[:, None] * v.reshape(-1, 3)).sum(0)
        assert np.abs(p - p0).max() <= 1e-6 * np.abs(m[:, None] * sc["V"]).sum()


def test_kappa_auto_closed_form():
    """Automatic barrier stiffness: 10 times the mean lumped FEM vertex mass
    times |g| h^2 / dhat.  The lumped masses sum to the mesh's mass, so the
    mean is rho * (sum of tet volumes) / nv, with volumes from the rest
    positions; for the 625-tet block (0.125 kg over 216 vertices, h = 0.01,
    dhat = 1e-3) that is about 5.7e-3."""
    sc = S.block_drop(n_steps=2)
    o = O.Oracle(sc)
    X, T = sc["X"], sc["tets"]
    D = np.stack([X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]], X[T[:, 3]] - X[T[:, 0]]], -1)
    vol = np.linalg.det(D) / 6.0
    mass = float(np.sum(sc["tet_rho"] * vol))
    want = 10.0 * mass / len(X) * np.linalg.norm(sc["g"]) * float(sc["h"]) ** 2 / float(sc["dhat"])
    assert mass == pytest.approx(0.125, rel=1e-2)
    assert o.kappa == pytest.approx(want, rel=1e-12)
    assert o.kappa == pytest.approx(5.68e-3, rel=1e-2)


def _rotation(a, u):
    u = np.asarray(u, np.float64) / np.linalg.norm(u)
    K = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return np.eye(3) + np.sin(a) * K + (1.0 - np.cos(a)) * (K @ K)


@pytest.mark.parametrize("gravity", [False, True])
def test_affine_body_free_flight(gravity):
    """A free affine body whose frame is a fixed rotation R (A = R, dA/dt = 0)
    and whose translation moves with v0: the orthogonality energy and its
    gradient vanish at any rotation, so implicit Euler reduces to
    p_{n+1} = p_n + h v_n + h^2 g, i.e. p_n = p_0 + n h v0 + h^2 g n(n+1)/2
    and v_n = v0 + n h g, while A and its rate stay exactly as they were."""
    n = 6
    sc = S.tiny_scene("free_body", n_steps=n, h=0.01)
    if not gravity:
        sc["g"] = np.zeros(3)
    R = _rotation(0.7, [1.0, -2.0, 0.5])
    p0 = sc["body_q"][0, :3].copy()
    v0 = np.array([0.1, -0.05, 0.2])
    sc["body_q"][0, 3:] = R.T.ravel()          # columns of A, one after another
    sc["body_qdot"][0, :3] = v0
    o = O.Oracle(sc)
    g, h = sc["g"], float(sc["h"])
    for k in range(1, n + 1):
        rc, st = o.step()
        assert rc == 0
        y, v = o.state()
        p_want = p0 + k * h * v0 + h * h * g * k * (k + 1) / 2.0
        assert np.abs(y[:3] - p_want).max() <= 1e-12 * (np.abs(p0).max() + 1.0)
        assert np.abs(v[:3] - (v0 + k * h * g)).max() <= 1e-9 * (np.abs(v0).max() + 1.0)
        assert np.abs(y[3:] - R.T.ravel()).max() <= 1e-13
        assert np.abs(v[3:]).max() <= 1e-10
        if not gravity:
            assert np.abs(v[:3] - v0).max() <= 1e-9 * np.abs(v0).max()
    E, terms = o.energy(y)
    assert terms[2] == pytest.approx(0.0, abs=1e-20)   # orthogonality energy zero at a rotation


def test_resting_block_contact_force():
    """At rest on the plane the barrier force balances the weight: d E_B / dz = -M g h^2."""
    sc = S.block_drop(n_steps=40)
    o = advanced(sc, 40)
    o.begin_step()
    y, v = o.state()
    assert np.abs(v).max() < 1e-3
    ez = np.zeros_like(y); ez[2::3] = 1.0
    dz = 1e-9
    dEb = (o.energy(y + dz * ez)[1][4] - o.energy(y - dz * ez)[1][4]) / (2 * dz)
    W = 0.125 * 9.81 * 0.01 ** 2
    assert dEb == pytest.approx(-W, rel=2e-2)


def test_coulomb_deceleration():
    """A block sliding on the plane loses mu g h of speed per step (lagged IPC friction)."""
    sc = S.block_drop(n_steps=60)
    o = advanced(sc, 40)
    y, v = o.state()
    v = v.reshape(-1, 3)
    v[:, 0] = 0.1
    o.set_state(y, v.ravel())
    vx = []
    for _ in range(3):
        assert o.step()[0] == 0
        vx.append(o.state()[1].reshape(-1, 3)[:, 0].mean())
    dv = -np.diff([0.1] + vx)
    assert np.allclose(dv, 0.3 * 9.81 * 0.01, rtol=2e-2)


def _orient(a, b, c, d):
    m = [[b[i] - a[i] for i in range(3)], [c[i] - a[i] for i in range(3)], [d[i] - a[i] for i in range(3)]]
    det = (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
           + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    return (det > 0) - (det < 0)


def _seg_tri_intersect(p, q, a, b, c):
    """Exact rational segment/triangle intersection (coplanar touching counts)."""
    s1, s2 = _orient(a, b, c, p), _orient(a, b, c, q)
    if s1 == s2 and s1 != 0:
        return False
    if s1 == 0 and s2 == 0:
        return False  # coplanar: reported by the positive-distance check instead
    o1, o2, o3 = _orient(p, q, a, b), _orient(p, q, b, c), _orient(p, q, c, a)
    return (o1 >= 0 and o2 >= 0 and o3 >= 0) or (o1 <= 0 and o2 <= 0 and o3 <= 0)


def test_no_interpenetration_exact():
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=40)
    o = O.Oracle(sc)
    tris = o.tris(); edges = o.edges()
    for step in range(40):
        assert o.step()[0] == 0
        if step % 5 != 4:
            continue
        y, _ = o.state()
        x = o.world(y)
        lo = np.minimum.reduce([x[tris[:, k]] for k in range(3)])
        hi = np.maximum.reduce([x[tris[:, k]] for k in range(3)])
        elo = np.minimum(x[edges[:, 0]], x[edges[:, 1]])
        ehi = np.maximum(x[edges[:, 0]], x[edges[:, 1]])
        X = [[Fraction(float(c)) for c in r] for r in x]
        for ei, (a, b) in enumerate(edges):
            near = np.nonzero(np.all(elo[ei] <= hi, 1) & np.all(ehi[ei] >= lo, 1))[0]
            for t in near:
                tv = tris[t]
                if a in tv or b in tv:
                    continue
                assert not _seg_tri_intersect(X[a], X[b], X[tv[0]], X[tv[1]], X[tv[2]]), (step, a, b, tv)
        pt, ee = o.pairs(y)
        for r in pt:
            assert O.dist2_pt(x[r].ravel())[0] > 0
        for r in ee:
            assert O.dist2_ee(x[r].ravel())[0] > 0


def test_coulomb_deceleration_with_lag_passes():
    """Three friction lag passes per step: the block still loses mu g h of
    speed per step.  The passes retake weights, normals and normal forces at
    the solution but keep measuring the slip from the step start (measured
    from the re-lag point, the second pass would see almost no slip and the
    deceleration would collapse)."""
    sc = S.block_drop(n_steps=60)
    o = advanced(sc, 40)
    o.set_friction_lag(3)
    y, v = o.state()
    v = v.reshape(-1, 3)
    v[:, 0] = 0.1
    o.set_state(y, v.ravel())
    vx = []
    for _ in range(3):
        rc, st = o.step()
        assert rc == 0 and st["newton_iters"] >= 3
        vx.append(o.state()[1].reshape(-1, 3)[:, 0].mean())
    dv = -np.diff([0.1] + vx)
    assert np.allclose(dv, 0.3 * 9.81 * 0.01, rtol=2e-2)
