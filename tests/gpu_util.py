"""Shared helpers of the GPU parity tests (GPU path against the oracle)."""
import numpy as np

import oracle as O


def oracle_states(scene, n_steps):
    """Oracle trajectory: list of (y, ydot) before each step 0..n_steps."""
    o = O.Oracle(scene)
    out = [o.state()]
    for _ in range(n_steps):
        rc, _ = o.step()
        assert rc == 0
        out.append(o.state())
    return o, out


def energy_tol(terms):
    """|dE| <= 1e-10 * sum |terms| (every term is non-negative)."""
    return 1e-10 * np.sum(np.abs(terms[:6])) + 1e-300


def assert_grad_close(g_gpu, g_or, gabs, rel=1e-10):
    err = np.abs(g_gpu - g_or)
    tol = rel * gabs + 1e-14 * (np.abs(gabs).max() + 1e-300)
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, f"{len(bad)} gradient entries off; worst {np.max(err / (tol + 1e-300)):.3g}x tol at {bad[:5]}"


def to_np(t):
    return t.detach().cpu().numpy() if t is not None else None
