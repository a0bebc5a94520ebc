"""Sub-stepping on failure (the dt-halving retry of the robustness
variants) and the time-step change it relies on: oracle pins (CPU).

Pins: implicit Euler free fall at a changed step follows its closed form;
linear momentum without gravity is conserved across the sub-steps of a
retried step (the internal and contact forces cancel at every piece); a step
that converges is the plain step, bit for bit.  Without the retry, 11 of
these 40 random velocity draws end a step with Newton unconverged at 100
iterations (the Newton measure stalls at the energy's rounding floor)."""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O


def _two_tets(seed):
    sc = S.tiny_scene("two_tets", n_steps=5, h=0.01)
    sc["g"] = np.zeros(3)
    sc["V"] = 0.05 * np.random.default_rng(seed).standard_normal(sc["V"].shape)
    return sc


def test_free_fall_at_a_changed_step():
    sc = S.tiny_scene("tet", n_steps=6, h=0.01)
    o = O.Oracle(sc)
    o.set_timestep(0.004)
    x0 = sc["X"].copy()
    for n in range(1, 7):
        assert o.step()[0] == 0
        y, _ = o.state()
        ref = x0 + 0.004 ** 2 * sc["g"] * n * (n + 1) / 2
        assert np.abs(y.reshape(-1, 3) - ref).max() <= 1e-5 * 0.004 * o.L


def test_retry_completes_every_draw_and_conserves_momentum():
    retried = 0
    for seed in range(40):
        sc = _two_tets(seed)
        plain = O.Oracle(sc)
        o = O.Oracle(sc)
        m = o.mass()
        p0 = (m[:, None] * sc["V"]).sum(0)
        for k in range(5):
            rc, pieces = o.step_adaptive()
            assert rc == 0, (seed, k)
            retried += pieces > 1
            _, v = o.state()
            p = (m[:, None] * v.reshape(-1, 3)).sum(0)
            assert np.abs(p - p0).max() <= 1e-6 * np.abs(m[:, None] * sc["V"]).sum(), (seed, k)
    assert retried >= 10


def test_converging_step_is_the_plain_step():
    sc = _two_tets(0)
    a, b = O.Oracle(sc), O.Oracle(sc)
    for _ in range(5):
        rc, pieces = a.step_adaptive()
        assert rc == 0 and pieces == 1
        assert b.step()[0] == 0
        assert np.array_equal(a.state()[0], b.state()[0])
