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
    """Per entry: |g_gpu - g_or| <= rel * gabs, gabs the oracle's sum of the
    absolute values of the operands that form the entry (no global floor)."""
    err = np.abs(g_gpu - g_or)
    tol = rel * gabs + 1e-300
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, f"{len(bad)} gradient entries off; worst {np.max(err / tol):.3g}x tol at {bad[:5]}"


def assert_hv_close(hv_gpu, hv_or, scale, rel=1e-9, what=""):
    """Per entry: |Hv_gpu - Hv_or| <= rel * (|P|^T |H| |P| |v|)_i, the
    oracle's absolute product scale of that entry."""
    err = np.abs(hv_gpu - hv_or)
    tol = rel * scale + 1e-300
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, f"{what}: {len(bad)} Hessian-product entries off; worst {np.max(err / tol):.3g}x tol at {bad[:5]}"


def to_np(t):
    return t.detach().cpu().numpy() if t is not None else None
