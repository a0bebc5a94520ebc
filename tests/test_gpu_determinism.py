"""Bit-for-bit reproducibility of the HIP library (needs a GPU).

Every sum the library forms has an order fixed by its inputs: reductions are
per wavefront in a fixed order, and the scatters of spring, barrier and
friction gradients, of contact and friction blocks into the matrix, of the
constant spring blocks and of the coarse preconditioner's blocks go through
sorted run sums instead of floating-point atomics.  Two contexts created from
the same scene therefore produce identical bits: states after every step,
energies, gradients, Hessian products and adjoints.
"""
import numpy as np
import pytest

import ipcscenes as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def _run(sc, n, coarse, monkeypatch):
    from paper_2609_25653_amd import Sim
    monkeypatch.setenv("IPC_PCG_COARSE", "1" if coarse else "0")
    sim = Sim(sc)
    out = []
    for _ in range(n):
        rc, st = sim.step()
        assert rc == 0, st
        y, v = sim.state()
        out.append((y.clone(), v.clone()))
    return sim, out


@pytest.mark.parametrize("coarse", [False, True])
@pytest.mark.parametrize("name,n", [("pad_box", 24), ("arm_box", 12), ("cube", 8)])
def test_trajectory_bitwise(name, n, coarse, monkeypatch):
    sc = S.tiny_scene(name, h=0.01, n_steps=n)
    _, a = _run(sc, n, coarse, monkeypatch)
    _, b = _run(sc, n, coarse, monkeypatch)
    for k, ((ya, va), (yb, vb)) in enumerate(zip(a, b)):
        assert torch.equal(ya, yb) and torch.equal(va, vb), (name, coarse, k)


def test_evaluation_bitwise(monkeypatch):
    """Energy, gradient and Hessian products at a contact-rich state, with
    friction, projected and not: two contexts, and twice on one context."""
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=30)
    sim, traj = _run(sc, 24, True, monkeypatch)
    y, v = traj[-1]
    other = Sim(sc)
    rng = np.random.default_rng(5)
    vv = torch.as_tensor(rng.standard_normal(sim.ndof), device="cuda")
    for s in (sim, other):
        s.set_state(y, v)
        s.begin_step(24)
    for project in (True, False):
        res = [s.energy_grad_hess(y, vv, project=project, friction=True) for s in (sim, other, sim)]
        for r in res[1:]:
            for a, b in zip(res[0][:3], r[:3]):
                assert torch.equal(a, b), project


def test_batched_bitwise(monkeypatch):
    from paper_2609_25653_amd import Sim
    monkeypatch.setenv("IPC_PCG_COARSE", "1")
    scenes = [S.tiny_scene("pad_box", seed=s, h=0.01, n_steps=10) for s in range(3)] + [S.block_drop(n_steps=10)]
    runs = []
    for _ in range(2):
        sim = Sim(scenes)
        states = []
        for _ in range(10):
            sim.step()
            states.append(sim.state()[0].clone())
        runs.append(states)
    for k, (a, b) in enumerate(zip(*runs)):
        assert torch.equal(a, b), k


def test_adjoint_bitwise(monkeypatch):
    """The one-step adjoint twice (fresh contexts): identical state and
    parameter adjoints."""
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=30)
    _, traj = _run(sc, 21, False, monkeypatch)
    (yp, vp), (yn, _) = traj[-2], traj[-1]
    rng = np.random.default_rng(9)
    a = torch.as_tensor(rng.standard_normal(yp.numel()), device="cuda")
    b = torch.as_tensor(rng.standard_normal(yp.numel()), device="cuda")
    outs = []
    for _ in range(2):
        sim = Sim(sc)
        Eb = torch.zeros(sim.n_tets, dtype=torch.float64, device="cuda")
        mb = torch.zeros(1, dtype=torch.float64, device="cuda")
        yb, vb, _ = sim.step_vjp(yp, vp, 20, yn, a, b, Eb, mb)
        outs.append((yb, vb, Eb, mb))
    for x, y in zip(*outs):
        assert torch.equal(x, y)


@pytest.mark.parametrize("name,n", [("pad_box", 24), ("arm_box", 12), ("block", 6), ("squeeze", 3)])
def test_one_launch_pcg_step_matches_two_launches(name, n, monkeypatch):
    """With the coarse correction on, a one-scene context applies it inside
    the PCG's update launch (each domain a contiguous node range: the
    update's workgroups recompute the new residual of the domain's other
    nodes, and of the bodies whose translation is grouped).  It is written
    to give the bits of the update followed by the correction's own launch:
    the trajectories of the two forms are compared bit for bit, over scenes
    with affine bodies (grouped with FEM vertices) and without."""
    from paper_2609_25653_amd import Sim
    if name == "block":
        sc = S.block_drop(n_steps=n)
    elif name == "squeeze":   # two pads of 12k tets and the gripper's bodies: several domains
        sc = S.gripper_squeeze(n_steps=n)
    else:
        sc = S.tiny_scene(name, h=0.01, n_steps=n)
    monkeypatch.setenv("IPC_PCG_COARSE", "1")
    runs = []
    for split in ("1", "0"):
        monkeypatch.setenv("IPC_NO_FUSED_PCG", split)
        sim = Sim(sc)
        assert sim.pcg_coarse and sim.pcg_fused == (split == "0")
        states = []
        for _ in range(n):
            rc, st = sim.step()
            assert rc == 0, st
            y, v = sim.state()
            states.append((y.clone(), v.clone(), sum(s["pcg_iters_total"] for s in st)))
        runs.append(states)
    for k, ((ya, va, ia), (yb, vb, ib)) in enumerate(zip(*runs)):
        assert ia == ib and torch.equal(ya, yb) and torch.equal(va, vb), (name, k)
