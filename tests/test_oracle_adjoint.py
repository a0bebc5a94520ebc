"""Pins of the oracle's adjoint of one converged step.

The step solves G(y^{n+1}; y^n, ydot^n, theta) = grad E_n = 0 (Sec. III-C,
Eq. (3)); its adjoint follows from the implicit function theorem with the
friction lag held as a function of y^n.  Every quantity the oracle returns is
checked against finite differences of the oracle's own forward quantities
(gradient, full steps, whole rollouts), which share none of the adjoint code:
  * the partial (dG/dy^n)^T w, including the lag's dependence on y^n through
    the closest-point weights, the normal, the offset and the normal force
    (with the edge-edge mollifier active in one scene);
  * the partials w . dG/dE_e and w . dG/dmu;
  * the state adjoints of one step;
  * dL/dE and dL/dmu of a multi-step rollout with checkpoint recomputation.
"""
import numpy as np
import pytest

import ipcscenes
import oracle as O


def _scene(kind):
    if kind in ("cube", "cube_hs"):   # on the ground triangles / the half-space z >= 0
        sc = ipcscenes.tiny_scene("cube", n_steps=12, ground="half_space" if kind == "cube_hs" else "triangles")
        vel = (0.05, 0.02)
    elif kind == "edge_tet":
        sc = ipcscenes.tiny_scene("edge_tet", n_steps=6)
        vel = (0.03, 0.01)
    else:
        return ipcscenes.tiny_scene("pad_box", n_steps=30)
    sc["V"] = np.array(sc["V"])
    sc["V"][:, 0], sc["V"][:, 1] = vel
    return sc


PRE = {"cube": 6, "cube_hs": 6, "edge_tet": 2, "pad_box": 20}
_CACHE = {}


def _step_data(kind):
    """(oracle, scene, n, y^n, ydot^n, y^{n+1}) for a step with lagged friction."""
    if kind not in _CACHE:
        sc = _scene(kind)
        o = O.Oracle(sc)
        for _ in range(PRE[kind]):
            o.step()
        n = o.step_index
        yp, vp = o.state()
        rc, st = o.step()
        assert rc == 0 and st["n_lag"] > 0
        yn, _ = o.state()
        _CACHE[kind] = (o, sc, n, yp, vp, yn)
    return _CACHE[kind]


def _phi(o, n, y_prev, v_prev, y_next, w):
    """w . G(y_next) with the step set up (predictor and lag) at (y_prev, v_prev)."""
    o.set_state(y_prev, v_prev)
    o.begin_step(n)
    g, _ = o.gradient(y_next)
    return float(g @ w)


@pytest.mark.parametrize("kind", ["cube", "cube_hs", "edge_tet", "pad_box"])
def test_dG_dyn_matches_fd(kind):
    o, sc, n, yp, vp, yn = _step_data(kind)
    rng = np.random.default_rng(11)
    for _ in range(2):
        w = rng.standard_normal(o.ndof)
        d = rng.standard_normal(o.ndof)
        an = o.dG_dyn_T(yp, vp, n, yn, w) @ d
        # Richardson-extrapolated central difference: the lag is smooth in y^n
        # but curved on the scale of the gap, so plain differences need eps
        # so small that rounding shows
        eps = 2e-8
        f = lambda t: _phi(o, n, yp + t * d, vp, yn, w)
        d1 = (f(eps) - f(-eps)) / (2 * eps)
        d2 = (f(eps / 2) - f(-eps / 2)) / eps
        fd = (4 * d2 - d1) / 3
        assert abs(fd - an) <= 2e-6 * abs(an), (fd, an)


def test_edge_tet_has_mollified_lag_pair():
    """The edge-edge mollifier is active for one lagged pair of the edge_tet
    scene, so the FD pin above covers its derivative."""
    o, sc, n, yp, vp, yn = _step_data("edge_tet")
    _, ee = o.pairs(yp)
    xw = o.world(yp)
    rest = np.concatenate([sc["X"], sc["bv_xbar"], sc["sv_x"]])
    ratios = []
    for a0, a1, b0, b1 in ee:
        c = np.sum(np.cross(xw[a1] - xw[a0], xw[b1] - xw[b0]) ** 2)
        ex = 1e-3 * np.sum((rest[a1] - rest[a0]) ** 2) * np.sum((rest[b1] - rest[b0]) ** 2)
        ratios.append(c / ex)
    assert min(ratios) < 0.9


@pytest.mark.parametrize("kind", ["cube", "cube_hs", "pad_box"])
def test_dG_dtheta_matches_fd(kind):
    o, sc, n, yp, vp, yn = _step_data(kind)
    rng = np.random.default_rng(12)
    w = rng.standard_normal(o.ndof)
    Eb, mb = o.dG_dtheta_T(yp, vp, n, yn, w)
    E0 = np.array(sc["tet_E"], np.float64)
    mu0 = float(sc["mu"])
    d = rng.standard_normal(len(E0)) * E0
    h = 1e-3
    o.set_params(E0 + h * d)
    fp = _phi(o, n, yp, vp, yn, w)
    o.set_params(E0 - h * d)
    fm = _phi(o, n, yp, vp, yn, w)
    o.set_params(E0)
    # G is linear in E and in mu, so the difference quotient is exact up to rounding
    assert abs((fp - fm) / (2 * h) - Eb @ d) <= 1e-8 * np.abs(Eb) @ np.abs(d)
    o.set_params(None, mu0 * (1 + h))
    fp = _phi(o, n, yp, vp, yn, w)
    o.set_params(None, mu0 * (1 - h))
    fm = _phi(o, n, yp, vp, yn, w)
    o.set_params(None, mu0)
    assert abs((fp - fm) / (2 * h * mu0) - mb) <= 1e-8 * abs(mb)


@pytest.mark.parametrize("kind", ["cube", "cube_hs", "pad_box"])
def test_step_vjp_state_matches_fd(kind):
    """ybar^n and vbar^n of one step against differences of full steps.

    The difference quotients see the Newton stopping error of each perturbed
    step amplified by the conditioning of the pad_box scene's stiff bodies,
    so this check re-runs the step with a tighter stopping tolerance."""
    _, sc, n, yp, vp, _ = _step_data(kind)
    sc = dict(sc)
    sc["newton_tol"] = np.asarray(3e-8)
    sc["pcg_tol"] = np.asarray(1e-10)
    o = O.Oracle(sc)
    h = float(sc["h"])

    def step_from(y0, v0):
        o.set_state(y0, v0)
        o.step_index = n
        rc, _ = o.step()
        assert rc == 0
        return o.state()[0]

    yn = step_from(yp, vp)
    rng = np.random.default_rng(13)
    a = rng.standard_normal(o.ndof)
    b = rng.standard_normal(o.ndof)
    rc, yb, vb, _, _, it = o.step_vjp(yp, vp, n, yn, a, b)
    assert rc == 0 and it > 0

    def loss(y0, v0):
        y1 = step_from(y0, v0)
        return a @ y1 + b @ ((y1 - y0) / h)

    d = rng.standard_normal(o.ndof)
    ev = 1e-4   # m/s
    fd_v = (loss(yp, vp + ev * d) - loss(yp, vp - ev * d)) / (2 * ev)
    assert abs(fd_v - vb @ d) <= 2e-5 * np.abs(vb) @ np.abs(d), (fd_v, vb @ d)
    ey = 1e-7   # m: the lag is curved on the scale of the contact gaps
    fd_y = (loss(yp + ey * d, vp) - loss(yp - ey * d, vp)) / (2 * ey)
    assert abs(fd_y - yb @ d) <= 2e-5 * np.abs(yb) @ np.abs(d), (fd_y, yb @ d)


ROLLOUT = {"cube": (5, 4, 1e-5), "cube_hs": (5, 4, 1e-5), "pad_box": (16, 4, 3e-5)}


@pytest.mark.parametrize("kind", ["cube", "cube_hs", "pad_box"])
def test_rollout_gradient_matches_fd(kind):
    """dL/dE and dL/dmu of a 4-step rollout against central differences.

    The forward steps stop at |p|_inf <= 1e-6 h L, so each converged state
    carries an error of that size; on the pad_box scene, whose contact gaps
    are ~1e-4 m, that shows as a ~1e-5 relative difference between the exact
    derivative at the stopped iterate and the difference quotient."""
    sc = _scene(kind)
    first, nst, tol = ROLLOUT[kind]
    o = O.Oracle(sc)
    for _ in range(first):
        o.step()
    y0, v0 = o.state()
    rng = np.random.default_rng(3)
    tracked = np.sort(rng.choice(len(sc["X"]), 8, replace=False))
    target = sc["X"][tracked] + rng.normal(0.0, 1e-3, (8, 3))
    E0 = np.array(sc["tet_E"], np.float64)
    mu0 = float(sc["mu"])
    run = lambda E, mu, **kw: O.rollout_loss(sc, y0, v0, first, nst, tracked, target, E, mu, **kw)
    loss, Eb, mb = run(E0, mu0, grad=True, checkpoint_every=2)
    d = rng.standard_normal(len(E0)) * E0
    h = 1e-3
    fd = (run(E0 + h * d, mu0) - run(E0 - h * d, mu0)) / (2 * h)
    assert abs(fd - Eb @ d) <= tol * abs(Eb @ d), (fd, Eb @ d)
    fd = (run(E0, mu0 * (1 + h)) - run(E0, mu0 * (1 - h))) / (2 * h * mu0)
    assert abs(fd - mb) <= tol * abs(mb), (fd, mb)
    # recomputation from checkpoints reproduces the stored forward exactly
    loss3, Eb3, mb3 = run(E0, mu0, grad=True, checkpoint_every=3)
    assert loss3 == loss and np.array_equal(Eb3, Eb) and mb3 == mb


def test_adjoint_indefinite_status():
    """A strongly compressed stiff tetrahedron: M + h^2 H (unprojected) is
    indefinite, and the adjoint PCG reports it (status 6) instead of a
    solution, at every compression tried, inverted included."""
    sc = ipcscenes.tiny_scene("tet", n_steps=2, h=0.1)
    sc["tet_E"] = np.array([1e9])
    sc["g"] = np.zeros(3)
    o = O.Oracle(sc)
    y0, v0 = o.state()
    X = sc["X"]
    c = X.mean(0)
    H = np.zeros((12, 12))
    for f in (0.5, 0.3, -0.2):
        yn = (c + f * (X - c)).ravel()
        for j in range(12):
            e = np.zeros(12); e[j] = 1.0
            o.set_state(y0, v0); o.begin_step(0)
            H[:, j] = o.hess_matvec(yn, e, project=False)
        assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() < 0          # indefinite indeed
        rc = o.step_vjp(y0, v0, 0, yn, np.ones(12), np.zeros(12))[0]
        assert rc == 6, f
