"""The boundary's memory and matrix contracts (needs a GPU).

* ipc_plan + ipc_create_ws: a context over a workspace that torch allocates
  steps exactly as one that allocates its own memory (bit for bit: every sum
  has a fixed order), uses at most the planned bytes, and reports a capacity
  or workspace that is too small with IPC_E_CAPACITY instead of growing.
* ipc_hessian_bsr: the exported block-CSR matrix times v is the library's own
  Hessian product, and its blocks are the oracle's Hessian entry by entry
  (1e-9 of the entry's absolute term scale |P|^T |H| |P|, or of 1e-4 of its
  row's largest such scale, whichever is larger), projected or not.
"""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]

CAP = (4000, 40000, 40000)


@pytest.mark.parametrize("name,n", [("pad_box", 24), ("arm_box", 16), ("cube", 8)])
def test_workspace_context_steps_like_the_plain_one(name, n):
    from paper_2609_25653_amd import Sim, _lib, plan
    sc = S.tiny_scene(name, h=0.01, n_steps=n)
    a, b = Sim(sc), Sim(sc, capacity=CAP)
    nbytes = plan(sc, CAP)
    assert b._query(_lib.Q_WS_BYTES) == nbytes
    for k in range(n):
        ra, sa = a.step()
        rb, sb = b.step()
        assert ra == rb == 0
        assert torch.equal(a.state()[0], b.state()[0]) and torch.equal(a.state()[1], b.state()[1]), (name, k)
    peak = b._query(_lib.Q_WS_PEAK)
    assert 0 < peak <= nbytes
    print(f"{name}: planned {nbytes} bytes, peak {peak}")


def test_workspace_batched_and_full_size():
    """A batch of mixed scenes, and the 200k-tet contact-rich scene over two
    steps at a capacity sized for it: the plan bounds the peak."""
    from paper_2609_25653_amd import Sim, _lib
    scenes = [S.tiny_scene("pad_box", seed=s, h=0.01, n_steps=6) for s in range(2)] + [S.block_drop(n_steps=6)]
    a, b = Sim(scenes), Sim(scenes, capacity=CAP)
    for _ in range(6):
        a.step(); b.step()
        assert torch.equal(a.state()[0], b.state()[0])
    assert b._query(_lib.Q_WS_PEAK) <= b._query(_lib.Q_WS_BYTES)
    sc = S.contact_rich(n_steps=3)
    big = Sim(sc, capacity=(150000, 600000, 400000))
    for _ in range(2):
        rc, st = big.step()
        assert rc == 0
    peak, nbytes = big._query(_lib.Q_WS_PEAK), big._query(_lib.Q_WS_BYTES)
    assert peak <= nbytes
    print(f"contact-rich: planned {nbytes / 2**20:.1f} MiB, peak {peak / 2**20:.1f} MiB")


def test_capacity_and_workspace_errors():
    from paper_2609_25653_amd import IPCError, Sim, plan
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=24)
    small = Sim(sc, capacity=(2, 8, 8))      # fewer pairs than the squeeze meets
    with pytest.raises(IPCError) as ei:
        for _ in range(24):
            small.step()
    assert ei.value.code == 2 and "capacity" in str(ei.value)
    with pytest.raises(IPCError) as ei:       # a workspace below the plan
        Sim(sc, capacity=CAP, workspace_bytes=plan(sc, CAP) // 8)
    assert ei.value.code == 2 and "workspace exhausted" in str(ei.value)


@pytest.mark.parametrize("name,k", [("pad_box", 20), ("arm_box", 12), ("block", 6)])
def test_hessian_bsr(name, k):
    from paper_2609_25653_amd import Sim
    sc = S.block_drop(n_steps=k + 2) if name == "block" else S.tiny_scene(name, h=0.01, n_steps=k + 2)
    o = O.Oracle(sc)
    for _ in range(k):
        o.step()
    y, v = o.state()
    o.begin_step(k)
    sim = Sim(sc)
    sim.set_state(y, v)
    sim.begin_step(k)
    rng = np.random.default_rng(k)
    for project in (True, False):
        rp, col, val = sim.hessian_bsr(y, project=project)
        rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
        n = len(y)
        H = np.zeros((n, n))
        for i in range(n // 3):
            for q in range(rp[i], rp[i + 1]):
                j = col[q]
                H[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[q]
        assert np.all(np.diff(col[rp[0]:rp[1]]) > 0)
        vv = rng.standard_normal(n)
        _, _, Hv, _ = sim.energy_grad_hess(y, vv, project=project, friction=True, energy=False, grad=False)
        Hv = Hv.cpu().numpy()
        assert np.abs(H @ vv - Hv).max() <= 1e-12 * np.abs(H).dot(np.abs(vv)).max()
        Ho, Ao = o.hessian_dense(y, project=project)
        err = np.abs(H - Ho)
        # the PSD projections and the reduced contact bases round in norm, per
        # term: an entry far below its row's largest term contribution is
        # compared at 1e-4 of that (1e-13 of the row's scale)
        scale = np.maximum(Ao, 1e-4 * Ao.max(axis=1, keepdims=True))
        bad = err > 1e-9 * scale + 1e-300
        assert not bad.any(), (name, project, int(bad.sum()), float((err / (Ao + 1e-300)).max()))
        # the pattern: every nonzero of the oracle's Hessian is in a stored block
        stored = np.zeros((n // 3, n // 3), bool)
        for i in range(n // 3):
            stored[i, col[rp[i]:rp[i + 1]]] = True
        nz = np.abs(Ho).reshape(n // 3, 3, n // 3, 3).max(axis=(1, 3)) > 0
        assert not (nz & ~stored).any()


def test_autotuned_lanes_carry_over_to_contexts_of_the_same_size():
    """The autotuner's lane count is kept per size bucket for the process: a
    second context of the same scene starts with it, and a context of a
    different size keeps the default until tuned itself."""
    from paper_2609_25653_amd import Sim
    # a batch of two free tetrahedra: a bucket no other test tunes
    pair = [S.tiny_scene("tet", h=0.01, n_steps=4), S.tiny_scene("tet", seed=1, h=0.01, n_steps=4)]
    a = Sim(pair)
    a.step()
    lanes, us = a.autotune(5)
    assert lanes in (1, 2, 4, 8, 16) and a.spmv_lanes == lanes and len(us) == 5
    b = Sim(pair)
    assert b.spmv_lanes == lanes
    other = Sim(pair[0])          # one scene: another bucket, not tuned
    assert other.spmv_lanes == 8


def test_autotuned_fem_blocks_carry_over_and_change_no_result():
    """The autotuner also picks the FEM assembly's workgroup sizes (64, 128
    or 256 each), keeps them for the size bucket, and no result depends on
    them: a tuned context and an untuned one step the pad squeeze bit for bit
    alike."""
    import os
    from paper_2609_25653_amd import Sim
    sc = S.tiny_scene("pad_box", h=0.01, n_steps=12)
    # the product's lane count changes the order of its sums, so it is fixed
    # here: only the FEM workgroup sizes differ between the two contexts
    old = os.environ.get("IPC_SPMV_LANES")
    os.environ["IPC_SPMV_LANES"] = "8"
    try:
        ref = Sim(sc)               # created before this bucket is tuned: default sizes
        assert ref.fem_blocks == (256, 256, 256)
        a = Sim(sc)
        a.step()
        a.autotune(5)
        blocks = a.fem_blocks
        assert all(b in (64, 128, 256) for b in blocks)
        b = Sim(sc)                 # same bucket: starts with the tuned sizes
    finally:
        if old is None:
            del os.environ["IPC_SPMV_LANES"]
        else:
            os.environ["IPC_SPMV_LANES"] = old
    assert b.fem_blocks == blocks and b.spmv_lanes == ref.spmv_lanes == 8
    for k in range(6):
        assert b.step()[0] == 0 and ref.step()[0] == 0
        yb, vb = b.state()
        yr, vr = ref.state()
        assert torch.equal(yb, yr) and torch.equal(vb, vr), k
