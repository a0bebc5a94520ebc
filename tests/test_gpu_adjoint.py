"""Parity of the library's one-step adjoint and of IPCRollout (needs a GPU).

The adjoint solves H w = ybar' with PCG to a relative residual of 1e-12 on
both sides; the two solves round differently, and the difference in w is
bounded by the residual times the conditioning of H along the slow
directions (stiff affine bodies against soft pads).  The bar for the one-step
outputs is therefore 1e-7 of the largest entry of each reference vector, and
for rollout gradients (whose forward trajectories already differ within the
1e-6 L trajectory bar) 1e-5 relative, with central finite differences of
the library's own rollouts as a second reference.
"""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O
from gpu_util import to_np

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def _scene(kind):
    if kind in ("pad_box", "pad_box_hs"):
        return S.tiny_scene("pad_box", n_steps=30, ground="half_space" if kind == "pad_box_hs" else "triangles")
    if kind == "cube_hs":   # the block sliding on the analytic half-space
        sc = S.tiny_scene("cube", n_steps=12, ground="half_space")
    else:
        sc = S.tiny_scene(kind, n_steps=12)
    sc["V"] = np.array(sc["V"])
    sc["V"][:, 0], sc["V"][:, 1] = (0.05, 0.02) if kind in ("cube", "cube_hs") else (0.03, 0.01)
    return sc


PRE = {"cube": 6, "cube_hs": 6, "edge_tet": 2, "pad_box": 20, "pad_box_hs": 20}


def _close(a, ref, rel):
    a, ref = np.asarray(a), np.asarray(ref)
    scale = np.max(np.abs(ref)) + 1e-300
    err = np.max(np.abs(a - ref))
    print(f"  max err / max |ref| = {err / scale:.3g}")
    assert err <= rel * scale, f"max err {err:.3g} vs scale {scale:.3g} ({err / scale:.3g} relative)"


@pytest.mark.parametrize("kind", ["cube", "edge_tet", "pad_box", "cube_hs", "pad_box_hs"])
def test_step_vjp_matches_oracle(kind):
    from paper_2609_25653_amd import Sim
    sc = _scene(kind)
    o = O.Oracle(sc)
    for _ in range(PRE[kind]):
        o.step()
    n = o.step_index
    yp, vp = o.state()
    rc, st = o.step()
    assert rc == 0 and st["n_lag"] > 0
    yn, _ = o.state()
    rng = np.random.default_rng(5)
    a = rng.standard_normal(o.ndof)
    b = rng.standard_normal(o.ndof)
    rc, yb_o, vb_o, Eb_o, mb_o, it_o = o.step_vjp(yp, vp, n, yn, a, b)
    assert rc == 0
    sim = Sim(sc)
    Eb = torch.zeros(sim.n_tets, dtype=torch.float64, device="cuda")
    mb = torch.zeros(1, dtype=torch.float64, device="cuda")
    yb, vb, it = sim.step_vjp(yp, vp, n, yn, a, b, Eb, mb)
    print(f"{kind}: pcg iterations oracle {it_o} gpu {it[0]}")
    _close(to_np(vb), vb_o, 1e-7)
    _close(to_np(yb), yb_o, 1e-7)
    _close(to_np(Eb), Eb_o, 1e-7)
    assert abs(to_np(mb)[0] - mb_o) <= 1e-7 * abs(mb_o)
    # the state is left at (y_prev, ydot_prev)
    y, v = sim.state()
    assert np.array_equal(to_np(y), yp) and np.array_equal(to_np(v), vp)


def test_step_vjp_batched_matches_single():
    """Two scenes in one context: each scene's adjoint equals its own."""
    from paper_2609_25653_amd import Sim
    scs = [_scene("cube"), _scene("pad_box")]
    data = []
    for sc, pre in zip(scs, (PRE["cube"], PRE["pad_box"])):
        o = O.Oracle(sc)
        for _ in range(pre):
            o.step()
        yp, vp = o.state()
        o.step()
        data.append((o.step_index - 1, yp, vp, o.state()[0]))
    rng = np.random.default_rng(6)
    single = []
    for sc, (n, yp, vp, yn) in zip(scs, data):
        sim = Sim(sc)
        a, b = rng.standard_normal(sim.ndof), rng.standard_normal(sim.ndof)
        Eb = torch.zeros(sim.n_tets, dtype=torch.float64, device="cuda")
        mb = torch.zeros(1, dtype=torch.float64, device="cuda")
        yb, vb, _ = sim.step_vjp(yp, vp, n, yn, a, b, Eb, mb)
        single.append((a, b, to_np(yb), to_np(vb), to_np(Eb), to_np(mb)))
    # both scenes share one step index only if their drive targets agree on it;
    # the cube has no driven links, so step the pair at the pad_box's index
    n = data[1][0]
    sim = Sim(scs)
    cat = lambda i: np.concatenate([data[0][i], data[1][i]])
    a = np.concatenate([single[0][0], single[1][0]])
    b = np.concatenate([single[0][1], single[1][1]])
    Eb = torch.zeros(sim.n_tets, dtype=torch.float64, device="cuda")
    mb = torch.zeros(2, dtype=torch.float64, device="cuda")
    yb, vb, _ = sim.step_vjp(cat(1), cat(2), n, cat(3), a, b, Eb, mb)
    off = sim.dof_offsets
    nt0 = len(scs[0]["tets"])
    for s in range(2):
        _close(to_np(yb)[off[s]:off[s + 1]], single[s][2], 1e-9)
        _close(to_np(vb)[off[s]:off[s + 1]], single[s][3], 1e-9)
        _close(to_np(Eb)[:nt0] if s == 0 else to_np(Eb)[nt0:], single[s][4], 1e-9)
        assert abs(to_np(mb)[s] - single[s][5][0]) <= 1e-9 * abs(single[s][5][0])


def _rollout_setup():
    sc = _scene("pad_box")
    first = 16
    o = O.Oracle(sc)
    for _ in range(first):
        o.step()
    y0, v0 = o.state()
    rng = np.random.default_rng(3)
    tracked = np.sort(rng.choice(len(sc["X"]), 8, replace=False))
    target = sc["X"][tracked] + rng.normal(0.0, 1e-3, (8, 3))
    return sc, first, y0, v0, tracked, target


def test_rollout_gradient_matches_oracle_and_fd():
    from paper_2609_25653_amd import Sim
    from paper_2609_25653_amd.rollout import rollout
    sc, first, y0, v0, tracked, target = _rollout_setup()
    nst = 4
    E0 = np.array(sc["tet_E"], np.float64)
    mu0 = float(sc["mu"])
    loss_o, Eb_o, mb_o = O.rollout_loss(sc, y0, v0, first, nst, tracked, target, E0, mu0, grad=True,
                                        checkpoint_every=2)
    sim = Sim(sc)
    idx = torch.as_tensor((3 * tracked[:, None] + np.arange(3)[None, :]).ravel(), device="cuda")
    tgt = torch.as_tensor(target.ravel(), dtype=torch.float64, device="cuda")
    y0t = torch.as_tensor(y0, device="cuda")
    v0t = torch.as_tensor(v0, device="cuda")

    def loss_of(E, mu, grad):
        E = torch.as_tensor(E, dtype=torch.float64, device="cuda").clone().requires_grad_(grad)
        mu = torch.tensor([mu], dtype=torch.float64, device="cuda", requires_grad=grad)
        y, _ = rollout(sim, E, mu, y0t, v0t, first, nst, checkpoint_every=2)
        L = ((y[idx] - tgt) ** 2).sum()
        if grad:
            L.backward()
            return float(L.detach()), to_np(E.grad), float(mu.grad[0])
        return float(L)

    loss, Eb, mb = loss_of(E0, mu0, True)
    assert abs(loss - loss_o) <= 1e-6 * loss_o
    rng = np.random.default_rng(8)
    for _ in range(2):
        d = rng.standard_normal(len(E0)) * E0
        assert abs(Eb @ d - Eb_o @ d) <= 1e-5 * abs(Eb_o @ d), (Eb @ d, Eb_o @ d)
        h = 1e-3
        fd = (loss_of(E0 + h * d, mu0, False) - loss_of(E0 - h * d, mu0, False)) / (2 * h)
        assert abs(fd - Eb @ d) <= 3e-5 * abs(Eb @ d), (fd, Eb @ d)
    assert abs(mb - mb_o) <= 1e-5 * abs(mb_o), (mb, mb_o)
    h = 1e-3
    fd = (loss_of(E0, mu0 * (1 + h), False) - loss_of(E0, mu0 * (1 - h), False)) / (2 * h * mu0)
    assert abs(fd - mb) <= 3e-5 * abs(mb), (fd, mb)


def test_observed_trajectory_loss_matches_chained_steps():
    """A loss over every step's tracked vertices through one checkpointed
    rollout (observe=...) equals the same loss through one rollout per step."""
    from paper_2609_25653_amd import Sim
    from paper_2609_25653_amd.rollout import rollout
    sc, first, y0, v0, tracked, target = _rollout_setup()
    nst = 4
    sim = Sim(sc)
    idx = torch.as_tensor((3 * tracked[:, None] + np.arange(3)[None, :]).ravel(), device="cuda")
    tgt = torch.as_tensor(target.ravel(), dtype=torch.float64, device="cuda")
    y0t = torch.as_tensor(y0, device="cuda")
    v0t = torch.as_tensor(v0, device="cuda")
    E0 = torch.as_tensor(sc["tet_E"], dtype=torch.float64, device="cuda")
    out = []
    for chained in (False, True):
        E = E0.clone().requires_grad_(True)
        mu = torch.tensor([float(sc["mu"])], dtype=torch.float64, device="cuda", requires_grad=True)
        if chained:
            y, v, L = y0t, v0t, 0.0
            for k in range(nst):
                y, v = rollout(sim, E, mu, y, v, first + k, 1)
                L = L + ((y[idx] - tgt) ** 2).sum()
        else:
            _, _, Y = rollout(sim, E, mu, y0t, v0t, first, nst, checkpoint_every=3, observe=idx)
            L = ((Y - tgt) ** 2).sum()
        L.backward()
        out.append((float(L.detach()), to_np(E.grad), float(mu.grad[0])))
    (La, Ea, ma), (Lb, Eb, mb) = out
    # the two forwards differ only by the order of FP64 atomic additions
    assert abs(La - Lb) <= 1e-9 * abs(Lb)
    _close(Ea, Eb, 1e-7)
    assert abs(ma - mb) <= 1e-7 * abs(mb)
