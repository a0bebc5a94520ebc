"""Parity of the HIP library with the oracle at identical inputs (needs a GPU).

Bars: contact-pair sets and CCD step bounds bit-exact; energies within 1e-10
of the sum of the absolute terms; gradients within 1e-10 of the per-entry sum
of absolute contributions; Hessian products within 1e-9 of the per-entry
absolute product scale |P|^T |H| |P| |v|, also for the friction blocks alone
(the product with friction minus the one without); trajectories within 1e-6
of the scene's bounding-box diagonal at every step.
"""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O
from gpu_util import assert_grad_close, assert_hv_close, energy_tol, oracle_states, to_np

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]

rng = np.random.default_rng(99)

def _rotation(a, u):
    u = np.asarray(u, np.float64) / np.linalg.norm(u)
    K = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return np.eye(3) + np.sin(a) * K + (1.0 - np.cos(a)) * (K @ K)


def tilted_cube(n_steps):
    """The block on the half-space, turned by a rotation off every axis
    (mesh, gravity and normal) and pushed sideways, so that the barrier,
    friction and CCD of the half-space see a general normal."""
    sc = S.tiny_scene("cube", ground="half_space", h=0.01, n_steps=n_steps)
    R = _rotation(0.6, [1.0, 2.0, -0.5])
    sc["V"] = np.tile([0.05, -0.02, 0.0], (len(sc["X"]), 1)) @ R.T
    sc["X"] = sc["X"] @ R.T
    sc["g"] = R @ sc["g"]
    n = R @ np.array([0.0, 0.0, 1.0])
    sc["half_space"] = np.array([n[0], n[1], n[2], 0.0])
    return sc


CASES = {
    "block": (lambda: S.block_drop(n_steps=8), [0, 2, 6]),
    "cube": (lambda: S.tiny_scene("cube", h=0.01, n_steps=8), [0, 6]),
    "pad_box": (lambda: S.tiny_scene("pad_box", h=0.01, n_steps=34), [0, 20, 32]),
    "arm_box": (lambda: S.tiny_scene("arm_box", h=0.01, n_steps=17), [0, 8, 16]),
    # the analytic half-space ground in place of the ground triangles
    "cube_hs": (lambda: S.tiny_scene("cube", ground="half_space", h=0.01, n_steps=8), [0, 6]),
    "tilted_hs": (lambda: tilted_cube(8), [0, 3, 6]),
    "pad_box_hs": (lambda: S.tiny_scene("pad_box", ground="half_space", h=0.01, n_steps=34), [0, 20, 32]),
}


@pytest.fixture(scope="module")
def states():
    out = {}
    for name, (mk, steps) in CASES.items():
        sc = mk()
        _, traj = oracle_states(sc, max(steps))
        out[name] = (sc, [(k, traj[k]) for k in steps])
    return out


def _pair(sim, o, sc, k, y, v):
    sim.set_state(y, v)
    sim.begin_step(k)
    o.set_state(y, v)
    o.begin_step(k)


@pytest.mark.parametrize("name", list(CASES))
def test_energy_gradient_hessian(name, states):
    from paper_2609_25653_amd import Sim
    sc, st = states[name]
    sim = Sim(sc)
    o = O.Oracle(sc)
    assert sim.ndof == o.ndof
    assert sim.scene_scalars()["kappa"] == pytest.approx(o.kappa, rel=1e-13)
    for k, (y, v) in st:
        _pair(sim, o, sc, k, y, v)
        yq = y + 1e-7 * rng.standard_normal(len(y)) * (np.arange(len(y)) < 3 * len(sc["X"]))
        E_or, terms = o.energy(yq)
        g_or, gabs = o.gradient(yq)
        for project in (True, False):
            vv = rng.standard_normal(len(y))
            E, g, Hv, rc = sim.energy_grad_hess(yq, vv, project=project, friction=True)
            assert rc == 0
            assert abs(to_np(E)[0] - E_or) <= energy_tol(terms), (k, to_np(E)[0], E_or)
            assert_grad_close(to_np(g), g_or, gabs)
            Hv_or, sc_or = o.hess_matvec(yq, vv, project, with_abs=True)
            assert_hv_close(to_np(Hv), Hv_or, sc_or, what=f"{name} step {k} project={project}")
            # the friction blocks alone: the product without friction, subtracted
            _, _, Hv0, rc = sim.energy_grad_hess(yq, vv, project=project, friction=False, energy=False, grad=False)
            assert rc == 0
            Hv0_or, sc0_or = o.hess_matvec(yq, vv, project, with_abs=True, friction=False)
            d_gpu, d_or = to_np(Hv) - to_np(Hv0), Hv_or - Hv0_or
            # scale: the friction terms' own absolute product, plus the rounding
            # of the two full products the difference cancels (each a sum of
            # tens of terms: a few 1e-16 of its absolute scale)
            sc_fr = (sc_or - sc0_or) + 1e-5 * sc_or
            assert_hv_close(d_gpu, d_or, sc_fr, what=f"{name} step {k} friction blocks project={project}")


@pytest.mark.parametrize("name", list(CASES))
def test_pairs_bit_exact(name, states):
    from paper_2609_25653_amd import Sim
    sc, st = states[name]
    sim = Sim(sc)
    o = O.Oracle(sc)
    for k, (y, v) in st:
        pt, ee = sim.pairs(y)
        opt, oee = o.pairs(y)
        assert np.array_equal(pt, opt), (name, k, len(pt), len(opt))
        assert np.array_equal(ee, oee), (name, k, len(ee), len(oee))


@pytest.mark.parametrize("name", list(CASES))
def test_ccd(name, states):
    from paper_2609_25653_amd import Sim
    sc, st = states[name]
    sim = Sim(sc)
    o = O.Oracle(sc)
    for k, (y, v) in st:
        for scale in (1e-4, 3e-3):
            p = scale * rng.standard_normal(len(y))
            a = to_np(sim.ccd(y, p))[0]
            a_or = o.ccd(y, p)
            # both sides evaluate every candidate's additive CCD with the same
            # operations in the same order, unfused: the bound is bit-exact
            assert a == a_or, (name, k, scale, a, a_or)


@pytest.mark.parametrize("coarse", [False, True])
@pytest.mark.parametrize("name", ["block", "pad_box", "arm_box", "pad_box_hs"])
def test_pcg(name, coarse, states, monkeypatch):
    """The solution of H x = b agrees with the oracle's PCG.  With the block-
    Jacobi preconditioner alone (the coarse correction switched off) the
    iteration counts agree too; with the coarse correction they may only
    drop."""
    from paper_2609_25653_amd import Sim
    monkeypatch.setenv("IPC_PCG_COARSE", "1" if coarse else "0")
    sc, st = states[name]
    sim = Sim(sc)
    o = O.Oracle(sc)
    k, (y, v) = st[-1]
    _pair(sim, o, sc, k, y, v)
    b = rng.standard_normal(len(y))
    x, it = sim.pcg(y, b, 1e-12)
    x_or, it_or = o.pcg(y, b, 1e-12)
    assert np.linalg.norm(to_np(x) - x_or) <= 1e-9 * np.linalg.norm(x_or)
    if coarse:
        assert int(it[0]) <= it_or + 2, (int(it[0]), it_or)
    else:
        assert abs(int(it[0]) - it_or) <= max(2, it_or // 20)


@pytest.mark.parametrize("coarse", [False, True])
@pytest.mark.parametrize("name,n", [("block", 20), ("pad_box", 34), ("arm_box", 30), ("block_hs", 20), ("tilted_hs", 16),
                                    ("pad_box_hs", 34)])
def test_trajectory(name, n, coarse, monkeypatch):
    """Steps agree with the oracle with the PCG's coarse correction switched
    off and on (these small scenes leave it off by default)."""
    from paper_2609_25653_amd import Sim
    monkeypatch.setenv("IPC_PCG_COARSE", "1" if coarse else "0")
    if name in ("block", "block_hs"):
        sc = S.block_drop(n_steps=n, ground="half_space" if name == "block_hs" else "triangles")
    elif name == "tilted_hs":
        sc = tilted_cube(n)
    elif name == "pad_box_hs":
        sc = S.tiny_scene("pad_box", ground="half_space", h=0.01, n_steps=n)
    else:
        sc = S.tiny_scene(name, h=0.01, n_steps=n)
    sim = Sim(sc)
    assert sim.pcg_coarse == coarse
    o = O.Oracle(sc)
    L = o.L
    for k in range(n):
        rc, stats = sim.step()
        rco, so = o.step()
        assert rc == 0 and rco == 0, (k, stats, so)
        y = to_np(sim.state()[0])
        yo, _ = o.state()
        err = np.abs(y - yo).max()
        assert err <= 1e-6 * L, (name, k, err / L, stats[0], so)


def test_graph_replay_matches_eager(monkeypatch):
    """PCG iterations replayed from a captured HIP graph (several replays per
    solve, eager work and host reads in between) match eager launches."""
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=30)
    monkeypatch.setenv("IPC_NO_GRAPH", "0")
    g = Sim(sc)
    monkeypatch.setenv("IPC_NO_GRAPH", "1")
    e = Sim(sc)
    L = O.Oracle(sc).L
    for k in range(30):
        rg, sg = g.step()
        re, se = e.step()
        assert rg == 0 and re == 0
        yg, ye = to_np(g.state()[0]), to_np(e.state()[0])
        assert np.abs(yg - ye).max() <= 1e-9 * L, (k, sg, se)


def test_half_steps_match_oracle():
    """The pieces of a retried step: from the state after 12 steps of the
    driven squeeze, two steps of h/2 towards the mean of steps 11 and 12's
    targets and then step 12's, on both sides (1e-6 L)."""
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=14)
    sim = Sim(sc)
    o = O.Oracle(sc)
    for k in range(12):
        assert sim.step()[0] == 0 and o.step()[0] == 0
    tm = 0.5 * (o.targets(11) + o.targets(12))
    sim.set_timestep(0.005)
    o.set_timestep(0.005)
    for t in (tm, o.targets(12)):
        assert sim.step_targets(t)[0] == 0 and o.step_targets(t)[0] == 0
        assert np.abs(to_np(sim.state()[0]) - o.state()[0]).max() <= 1e-6 * o.L
    assert sim.scene_scalars()["newton_threshold"] == pytest.approx(o.newton_threshold, rel=1e-14)


def _two_tet_draws(floor_stop):
    """40 random velocity draws of two free tets, 5 steps each through
    step_adaptive; returns the number of steps that needed the retry.  With
    floor_stop False the Newton loop has no stop at the energy's rounding
    floor (IPC_NO_FLOOR_STOP=1 at create), as in the oracle."""
    import os
    from paper_2609_25653_amd import Sim
    retried = 0
    for seed in range(40):
        sc = S.tiny_scene("two_tets", n_steps=5, h=0.01)
        sc["g"] = np.zeros(3)
        sc["V"] = 0.05 * np.random.default_rng(seed).standard_normal(sc["V"].shape)
        old = os.environ.get("IPC_NO_FLOOR_STOP")
        os.environ["IPC_NO_FLOOR_STOP"] = "0" if floor_stop else "1"
        try:
            sim = Sim(sc)
        finally:
            if old is None:
                del os.environ["IPC_NO_FLOOR_STOP"]
            else:
                os.environ["IPC_NO_FLOOR_STOP"] = old
        m = O.Oracle(sc).mass()
        p0 = (m[:, None] * sc["V"]).sum(0)
        for k in range(5):
            rc, pieces = sim.step_adaptive()
            assert rc == 0, (seed, k)
            retried += pieces > 1
            v = to_np(sim.state()[1]).reshape(-1, 3)
            assert np.abs((m[:, None] * v).sum(0) - p0).max() <= 1e-6 * np.abs(m[:, None] * sc["V"]).sum(), (seed, k)
    return retried


def test_step_adaptive_completes_and_conserves_momentum():
    """Without the rounding-floor stop, as in the oracle, some plain steps of
    these draws end unconverged (11 of them on the oracle): every draw still
    completes its 5 steps with the retry, and linear momentum is conserved
    across every piece."""
    assert _two_tet_draws(floor_stop=False) >= 1


def test_rounding_floor_stop_converges_the_plain_steps():
    """With the rounding-floor stop (the default), the same draws need no
    retry: the steps that stalled with the measure just above its stop and
    the energy unable to resolve a further decrease now end converged, and
    momentum is conserved."""
    assert _two_tet_draws(floor_stop=True) == 0


def test_changed_timestep_free_fall():
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("tet", n_steps=6, h=0.01)
    sim = Sim(sc)
    sim.set_timestep(0.004)
    x0 = sc["X"].copy()
    L = sim.scene_scalars()["L"]
    for n in range(1, 7):
        assert sim.step()[0] == 0
        ref = x0 + 0.004 ** 2 * sc["g"] * n * (n + 1) / 2
        assert np.abs(to_np(sim.state()[0]).reshape(-1, 3) - ref).max() <= 1e-5 * 0.004 * L


def test_friction_lag_passes_trajectory():
    """Two friction lag passes per step on the squeeze with a box (sticking
    and sliding contacts): the same trajectory as the oracle's two passes."""
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=30)
    sim = Sim(sc)
    o = O.Oracle(sc)
    sim.set_friction_lag(2)
    o.set_friction_lag(2)
    for k in range(30):
        rc, st = sim.step()
        rco, so = o.step()
        assert rc == 0 and rco == 0, (k, st, so)
        assert np.abs(to_np(sim.state()[0]) - o.state()[0]).max() <= 1e-6 * o.L, k


def test_friction_lag_passes_coulomb_and_adjoint_guard():
    """A block sliding on the ground with three lag passes still loses
    mu g h of speed per step; the adjoint refuses a multi-pass context."""
    from paper_2609_25653_amd import Sim, IPCError
    sc = S.block_drop(n_steps=60)
    sim = Sim(sc)
    for _ in range(40):
        assert sim.step()[0] == 0
    sim.set_friction_lag(3)
    y, v = sim.state()
    v = to_np(v).reshape(-1, 3)
    v[:, 0] = 0.1
    sim.set_state(y, v.ravel())
    vx = []
    for _ in range(3):
        assert sim.step()[0] == 0
        vx.append(to_np(sim.state()[1]).reshape(-1, 3)[:, 0].mean())
    dv = -np.diff([0.1] + vx)
    assert np.allclose(dv, 0.3 * 9.81 * 0.01, rtol=2e-2)
    yp, vp = sim.state()
    with pytest.raises(IPCError):
        sim.step_vjp(yp, vp, 43, yp, np.zeros(sim.ndof), np.zeros(sim.ndof))
