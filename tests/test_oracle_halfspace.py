"""The analytic half-space ground in the oracle (CPU).

Pins, none of which uses the half-space code to check itself:
* a block over the half-space z >= 0 and the same block over the two ground
  triangles of z = 0 have the same energy terms, gradient, Hessian products
  and friction lag at any state whose vertices project inside the triangles
  (the point-triangle distance there is the height);
* the same trajectory while no CCD bound binds;
* rotating the whole scene (mesh, gravity, half-space normal) rotates the
  trajectory (the normal enters the barrier, friction and CCD);
* the CCD bound of a straight fall is the closed form (1 - s) d0 / |p_z| of
  the closest vertex, and no smaller than the additive CCD of the triangles;
* at rest the half-space carries the block's weight, and a sliding block
  loses mu g h of speed per step (lagged Coulomb friction).
The adjoint through the half-space's friction lag is pinned against finite
differences with the other adjoint pins (test_oracle_adjoint.py, "cube_hs")."""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O


def _pair(**kw):
    a = S.tiny_scene("cube", ground="triangles", **kw)
    b = S.tiny_scene("cube", ground="half_space", **kw)
    return a, b


def _contact_state(sc, n=6):
    o = O.Oracle(sc)
    for _ in range(n):
        assert o.step()[0] == 0
    return o.state()


def test_same_terms_as_the_ground_triangles():
    tri, hs = _pair(h=0.01, n_steps=8)
    y, v = _contact_state(tri)
    ot, oh = O.Oracle(tri), O.Oracle(hs)
    for o in (ot, oh):
        o.set_state(y, v)
        o.begin_step(6)
    nv = len(tri["X"])
    assert np.sort(y[:3 * nv].reshape(-1, 3)[:, 2])[0] < float(tri["dhat"])     # in contact
    rng = np.random.default_rng(3)
    for k in range(4):
        yq = y.copy()
        if k:   # slide and press a little: friction and barrier both vary
            yq[:3 * nv] += 2e-5 * rng.standard_normal(3 * nv) * np.tile([1.0, 1.0, 0.1], nv)
        Et, tt = ot.energy(yq)
        Eh, th = oh.energy(yq)
        assert th[4] > 0.0 and th[5] > 0.0
        np.testing.assert_allclose(th, tt, rtol=1e-12, atol=0.0)
        # per entry, against the sum of the absolute contributions: the two
        # distance formulas round differently (the pair barrier goes through
        # the derivatives of d^2, whose chain rule cancels near contact)
        gt, gabs = ot.gradient(yq)
        gh, _ = oh.gradient(yq)
        assert np.all(np.abs(gh - gt) <= 1e-11 * gabs)
        # unprojected: a pair's projection acts on its 12x12 Hessian, static
        # triangle corners included, and so changes the moving vertex's block
        w = rng.standard_normal(len(y))
        Ht, Habs = ot.hess_matvec(yq, w, project=False, with_abs=True)
        Hh = oh.hess_matvec(yq, w, project=False)
        assert np.all(np.abs(Hh - Ht) <= 1e-11 * Habs)


def test_same_trajectory_as_the_ground_triangles():
    tri, hs = _pair(h=0.01, n_steps=16)
    ot, oh = O.Oracle(tri), O.Oracle(hs)
    for k in range(16):
        rt, st = ot.step()
        rh, sh = oh.step()
        assert rt == rh == 0
        assert st["n_lag"] == sh["n_lag"]
        assert np.abs(oh.state()[0] - ot.state()[0]).max() <= 1e-9 * ot.L, k


def _rotation(a, u):
    u = np.asarray(u, np.float64) / np.linalg.norm(u)
    K = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return np.eye(3) + np.sin(a) * K + (1.0 - np.cos(a)) * (K @ K)


def test_rotated_scene_rotates_the_trajectory():
    """The block on the half-space, and the same scene turned by R about a
    point of the plane (vertices, gravity, normal), with a sideways push so
    that friction acts: positions stay R times the upright ones."""
    sc = S.tiny_scene("cube", ground="half_space", h=0.01, n_steps=12)
    sc["V"] = np.tile([0.05, -0.02, 0.0], (len(sc["X"]), 1))
    R = _rotation(0.6, [1.0, 2.0, -0.5])
    rot = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    rot["X"] = sc["X"] @ R.T
    rot["V"] = sc["V"] @ R.T
    rot["g"] = R @ sc["g"]
    n = R @ np.array([0.0, 0.0, 1.0])
    rot["half_space"] = np.array([n[0], n[1], n[2], 0.0])
    assert abs(n @ n - 1.0) <= 1e-15
    a, b = O.Oracle(sc), O.Oracle(rot)
    nv = len(sc["X"])
    for k in range(12):
        assert a.step()[0] == 0 and b.step()[0] == 0
        ya = a.state()[0][:3 * nv].reshape(-1, 3)
        yb = b.state()[0][:3 * nv].reshape(-1, 3)
        # the two Newton solves stop at 1e-6 h L per update on different
        # iterates: a few of those apart (a misused normal moves the block by
        # its contact gap, ~1e-3 L)
        assert np.abs(yb - ya @ R.T).max() <= 1e-7 * a.L, k
    assert a.step()[1]["n_lag"] > 0


def test_ccd_closed_form_for_a_fall():
    tri, hs = _pair(h=0.01, n_steps=2)
    ot, oh = O.Oracle(tri), O.Oracle(hs)
    y, _ = oh.state()
    nv = len(hs["X"])
    p = np.zeros_like(y)
    p[2:3 * nv:3] = -0.004                      # every vertex 4 mm down: through the plane
    z0 = y[:3 * nv].reshape(-1, 3)[:, 2].min()
    want = (1.0 - float(hs["ccd_s"])) * z0 / 0.004
    assert oh.ccd(y, p) == pytest.approx(want, rel=1e-14)
    assert ot.ccd(y, p) <= oh.ccd(y, p) * (1.0 + 1e-12)       # the additive CCD is conservative
    p[2:3 * nv:3] = 0.004                       # moving away: no bound
    assert oh.ccd(y, p) == 1.0


def test_resting_weight_and_coulomb_on_the_half_space():
    sc = S.block_drop(n_steps=60, ground="half_space")
    o = O.Oracle(sc)
    for _ in range(40):
        assert o.step()[0] == 0
    o.begin_step()
    y, v = o.state()
    assert np.abs(v).max() < 1e-3
    ez = np.zeros_like(y); ez[2::3] = 1.0
    dz = 1e-9
    dEb = (o.energy(y + dz * ez)[1][4] - o.energy(y - dz * ez)[1][4]) / (2 * dz)
    assert dEb == pytest.approx(-0.125 * 9.81 * 0.01 ** 2, rel=2e-2)
    v = v.reshape(-1, 3)
    v[:, 0] = 0.1
    o.set_state(y, v.ravel())
    vx = []
    for _ in range(3):
        assert o.step()[0] == 0
        vx.append(o.state()[1].reshape(-1, 3)[:, 0].mean())
    assert np.allclose(-np.diff([0.1] + vx), 0.3 * 9.81 * 0.01, rtol=2e-2)


def test_tilted_half_space_hessian_by_differences():
    """On a tilted half-space (normal off every axis) the unprojected
    Hessian product equals central differences of the gradient, barrier and
    lagged friction included: a wrong n n^T or tangent projection would not
    show in a trajectory (Newton still finds the minimiser), but shows here."""
    sc = S.tiny_scene("cube", ground="half_space", h=0.01, n_steps=8)
    sc["V"] = np.tile([0.05, -0.02, 0.0], (len(sc["X"]), 1))
    R = _rotation(0.6, [1.0, 2.0, -0.5])
    sc["X"] = sc["X"] @ R.T
    sc["V"] = sc["V"] @ R.T
    sc["g"] = R @ sc["g"]
    n = R @ np.array([0.0, 0.0, 1.0])
    sc["half_space"] = np.array([n[0], n[1], n[2], 0.0])
    o = O.Oracle(sc)
    for _ in range(5):
        assert o.step()[0] == 0
    o.begin_step()
    y, _ = o.state()
    E, terms = o.energy(y)
    assert terms[4] > 0.0
    rng = np.random.default_rng(7)
    nv = len(sc["X"])
    for _ in range(3):
        yq = y.copy()
        yq[:3 * nv] += 1e-5 * rng.standard_normal(3 * nv)         # slip: friction in its sliding branch too
        v = rng.standard_normal(len(y))
        Hv, Habs = o.hess_matvec(yq, v, project=False, with_abs=True)
        eps = 1e-9
        fd = (o.gradient(yq + eps * v)[0] - o.gradient(yq - eps * v)[0]) / (2 * eps)
        assert np.abs(fd - Hv).max() <= 1e-5 * np.abs(Habs).max(), np.abs(fd - Hv).max() / np.abs(Habs).max()
