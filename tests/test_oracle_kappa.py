"""Adaptive barrier stiffness in the oracle (CPU), a robustness variant of
the barrier term of Eq. (3): kappa doubles after an accepted Newton update
whose smallest active-pair distance is below frac * dhat and below the
previous iterate's, capped at factor * kappa0.

The pins predict the rule from geometry the oracle does not compute: a 2x2x2
block above the two-triangle ground at z = 0 has no active pair but its
vertices over the ground, whose distances are their heights z.  With one
Newton update per step (max_newton = 1) every step is one update, so the
kappa after each step follows from the heights of consecutive states."""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O


def _heights(y, nv, dhat):
    z = y[:3 * nv].reshape(-1, 3)[:, 2]
    z = z[z < dhat]
    return float(z.min()) if len(z) else np.inf


def _predict_and_step(frac, factor, n_steps):
    sc = S.tiny_scene("cube", h=0.01, n_steps=n_steps, max_newton=1)
    nv, dhat = len(sc["X"]), float(sc["dhat"])
    o = O.Oracle(sc)
    k0 = o.kappa
    o.set_kappa_adaptive(frac, factor)
    kap, fired, capped = k0, 0, 0
    dprev = _heights(o.state()[0], nv, dhat)
    for k in range(n_steps):
        o.step()                                  # one update: status 3 (not converged) is expected
        d = _heights(o.state()[0], nv, dhat)
        if d < frac * dhat and d < dprev:
            kap = min(2.0 * kap, factor * k0)
            fired += 1
            capped += kap == factor * k0
        dprev = d
        assert o.kappa == kap, (k, o.kappa / k0, kap / k0)
    return o, k0, fired, capped


def test_adaptive_kappa_rule_from_heights():
    """The block falls onto the ground and settles; kappa after every update
    is the one the rule gives from the block's heights, and it fires."""
    o, k0, fired, capped = _predict_and_step(0.8, 100.0, 30)
    assert fired >= 2 and capped == 0
    assert np.log2(o.kappa / k0) == int(np.log2(o.kappa / k0))    # a power of two times kappa0


def test_adaptive_kappa_cap():
    """With every active distance below the threshold the rule doubles at
    each decrease until factor * kappa0, then stays there."""
    o, k0, fired, capped = _predict_and_step(1e6, 3.0, 30)
    assert capped >= 1 and o.kappa == 3.0 * k0


def test_adaptive_kappa_enters_the_barrier():
    """The barrier term after the rule has fired is kappa (as reported) times
    the barrier of Sec. III-C.1 summed over the vertices' heights."""
    o, k0, fired, _ = _predict_and_step(0.8, 100.0, 20)
    assert o.kappa > k0
    y, _ = o.state()
    nv, dh = len(o.scene["X"]), float(o.scene["dhat"])
    z = y[:3 * nv].reshape(-1, 3)[:, 2]
    z = z[z < dh]
    want = o.kappa * np.sum(-(z - dh) ** 2 * np.log(z / dh))
    assert o.energy(y)[1][4] == pytest.approx(want, rel=1e-10)


def test_kappa_fixed_by_default():
    sc = S.block_drop(n_steps=12)
    o = O.Oracle(sc)
    k0 = o.kappa
    for _ in range(12):
        assert o.step()[0] == 0
    assert o.kappa == k0


def test_adaptive_kappa_compares_with_the_step_start():
    """The first update of a step compares with the distance at the step's
    own start state: after the block has settled (threshold 0.5 dhat), the
    threshold is raised to 0.95 dhat and the block moved up to 0.9 dhat with a
    downward speed, so the next update's distance is below the new start's
    (the rule fires) though above the settled gap."""
    sc = S.tiny_scene("cube", h=0.01, n_steps=30, max_newton=1)
    nv, dhat = len(sc["X"]), float(sc["dhat"])
    o = O.Oracle(sc)
    o.set_kappa_adaptive(0.5, 100.0)
    for _ in range(20):
        o.step()
    o.set_kappa_adaptive(0.95, 100.0)
    k1 = o.kappa
    y, v = o.state()
    settled = _heights(y, nv, dhat)
    z = y[:3 * nv].reshape(-1, 3)
    z[:, 2] += 0.9 * dhat - z[:, 2].min()
    v = np.zeros_like(v)
    v[2:3 * nv:3] = -0.005
    o.set_state(y, v)
    start = _heights(y, nv, dhat)
    o.step()
    d = _heights(o.state()[0], nv, dhat)
    assert settled < d < start < 0.95 * dhat
    assert o.kappa == 2.0 * k1
