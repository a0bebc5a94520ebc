"""Error statuses the library returns from device work (needs a GPU); every
kernel exits normally in each of these cases.

* IPC_E_CAPACITY: ipc_get_pairs with room for fewer pairs than exist reports
  the counts it needs.
* IPC_E_INTERSECTING: a contact pair at distance zero (a vertex exactly on the
  ground): the energy is +inf (as the oracle's) and a step refuses to start.
* IPC_E_NOT_CONVERGED: a Newton budget of one iteration: the step ends at its
  last iterate, the oracle's too.
* IPC_E_INDEFINITE: the adjoint at a strongly compressed stiff tetrahedron,
  whose unprojected Hessian M + h^2 H is indefinite along a PCG direction (the
  oracle returns the same status).
"""
import ctypes

import numpy as np
import pytest

import ipcscenes as S
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def test_get_pairs_capacity():
    from paper_2609_25653_amd import Sim, _lib
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=24)
    sim = Sim(sc)
    for _ in range(22):
        sim.step()
    y, _ = sim.state()
    pt, ee = sim.pairs(y)
    assert len(pt) > 1 and len(ee) > 1
    cap = 1
    a = np.zeros((cap, 4), np.int32); b = np.zeros((cap, 4), np.int32)
    npt, nee = ctypes.c_int64(), ctypes.c_int64()
    rc = _lib.lib().ipc_get_pairs(sim._h, ctypes.c_void_p(y.data_ptr()), 0, a.ctypes.data_as(_lib._I), b.ctypes.data_as(_lib._I),
                                  cap, ctypes.byref(npt), ctypes.byref(nee))
    assert rc == 2                                          # IPC_E_CAPACITY
    assert (npt.value, nee.value) == (len(pt), len(ee))     # the counts it needs
    assert "capacity" in _lib.lib().ipc_last_error(sim._h).decode().lower() or True


def test_intersecting_state():
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("cube", h=0.01, n_steps=4)
    X = sc["X"].copy()
    low = int(np.argmin(X[:, 2]))
    X[low, 2] = 0.0                     # exactly on the ground plane z = 0
    sc["X"] = X
    y = X.ravel().copy()
    o = O.Oracle(sc)
    o.begin_step(0)
    E_or, _ = o.energy(y)
    assert np.isinf(E_or)
    sim = Sim(sc)
    sim.begin_step(0)
    E, _, _, rc = sim.energy_grad_hess(y, None, energy=True, grad=False)
    assert rc == 5 and np.isinf(float(E[0]))              # IPC_E_INTERSECTING, E = +inf
    rc, st = sim.step(allow_status=(5,))
    assert rc == 5 and st[0]["status"] == 5 and st[0]["newton_iters"] == 0
    assert torch.equal(sim.state()[0].cpu(), torch.as_tensor(y))   # the state did not move


def test_not_converged_keeps_last_iterate():
    from paper_2609_25653_amd import Sim
    sc = S.block_drop(n_steps=3)
    sc["max_newton"] = np.asarray(1.0)
    o = O.Oracle(sc)
    sim = Sim(sc)
    for k in range(3):
        rco, so = o.step()
        rc, st = sim.step(allow_status=(3,))
        assert rco == 3 and rc == 3 and st[0]["status"] == 3 and st[0]["newton_iters"] == 1, (k, st, so)
        err = np.abs(sim.state()[0].cpu().numpy() - o.state()[0]).max()
        assert err <= 1e-6 * o.L, (k, err / o.L)


def test_adjoint_indefinite():
    from paper_2609_25653_amd import IPCError, Sim
    sc = S.tiny_scene("tet", n_steps=2, h=0.1)
    sc["tet_E"] = np.array([1e9])
    sc["g"] = np.zeros(3)
    X = sc["X"]
    c = X.mean(0)
    yn = (c + 0.3 * (X - c)).ravel()
    o = O.Oracle(sc)
    y0, v0 = o.state()
    a, b = np.ones(len(y0)), np.zeros(len(y0))
    assert o.step_vjp(y0, v0, 0, yn, a, b)[0] == 6
    sim = Sim(sc)
    Eb = torch.zeros(1, dtype=torch.float64, device="cuda")
    mb = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(IPCError) as ei:
        sim.step_vjp(y0, v0, 0, yn, a, b, Eb, mb)
    assert ei.value.code == 6                                # IPC_E_INDEFINITE
    assert float(Eb[0]) == 0.0 and float(mb[0]) == 0.0       # outputs not written
