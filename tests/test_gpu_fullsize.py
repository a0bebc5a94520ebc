"""Parity at the benchmark's full size (needs a GPU): the 200k-tet
contact-rich squeeze (two pads and a soft cylinder on a 0.8 mm ground
patch), in the configuration the bench times (one context, the coarse
correction on by size).  From the scene's own initial state, already in
contact, plus a seeded perturbation: contact pair sets bit-exact, the
energy, the gradient and the projected and unprojected Hessian products
against the oracle to the same bars as the small cases (energy 1e-10 of
the summed terms, gradient 1e-10 of the per-entry absolute contributions,
Hessian products 1e-9 relative)."""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O
from gpu_util import assert_grad_close, energy_tol, to_np

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def test_contact_rich_200k_energy_gradient_hessian_pairs():
    from paper_2609_25653_amd import Sim
    sc = S.contact_rich(n_steps=2, s_g=8e-4)
    assert len(sc["tets"]) == 200_000
    sim = Sim(sc)
    assert sim.pcg_coarse        # the bench's configuration at this size
    o = O.Oracle(sc)
    y, v = o.state()
    sim.set_state(y, v)
    sim.begin_step(0)
    o.begin_step(0)

    pt, ee = sim.pairs(y)
    opt, oee = o.pairs(y)
    assert np.array_equal(pt, opt) and np.array_equal(ee, oee), (len(pt), len(opt), len(ee), len(oee))
    assert len(pt) + len(ee) > 10_000     # contact-rich from the first step

    rng = np.random.default_rng(2609)
    n_fem = 3 * len(sc["X"])
    yq = y + 1e-7 * rng.standard_normal(len(y)) * (np.arange(len(y)) < n_fem)
    E_or, terms = o.energy(yq)
    g_or, gabs = o.gradient(yq)
    for project in (True, False):
        vv = rng.standard_normal(len(y))
        E, g, Hv, rc = sim.energy_grad_hess(yq, vv, project=project, friction=True)
        assert rc == 0
        assert abs(to_np(E)[0] - E_or) <= energy_tol(terms), (to_np(E)[0], E_or)
        assert_grad_close(to_np(g), g_or, gabs)
        Hv_or = o.hess_matvec(yq, vv, project)
        err = np.linalg.norm(to_np(Hv) - Hv_or)
        assert err <= 1e-9 * np.linalg.norm(Hv_or), (project, err / np.linalg.norm(Hv_or))
