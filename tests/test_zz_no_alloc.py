"""The dual-mesh product through the entry point that allocates nothing
(ipc_dualmesh_apply_noalloc: W staged in the library's fixed device array)
against ipc_dualmesh_apply on the same inputs: identical bits, over two calls
in a row whose second call has a smaller input (another mesh, fewer levels
and frames), and a W too large for the array rejected (needs a GPU)."""
import numpy as np
import pytest

import ipcscenes as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def _mesh(n_disk, n_layers):
    tri, frames = S.dualmesh_frames(n_frames=6, n_disk=n_disk, n_layers=n_layers)
    return tri, frames


def test_noalloc_matches_apply_twice():
    from paper_2609_25653_amd.dualmesh import DualMesh
    # first call: a 12x12-disk cylinder surface, 2 levels, 6 frames; second: a
    # 6x6-disk one, 1 level, 2 frames (a smaller W and input)
    for (nd, nl, levels, nf) in ((12, 16, 2, 6), (6, 8, 1, 2)):
        tri, frames = _mesh(nd, nl)
        dm = DualMesh(tri, frames.shape[1], levels)
        xc = torch.as_tensor(frames[:nf], device="cuda").contiguous()
        ref = dm.apply(xc)
        out = torch.full_like(ref, float("nan"))
        dm.apply_noalloc(xc, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (nd, levels, nf)


def test_noalloc_alternating_handles_and_capacity():
    """Two handles alternating on one GPU: each call stages its own W again.
    A W beyond the array's size is rejected with IPC_E_CAPACITY."""
    from paper_2609_25653_amd.dualmesh import DualMesh
    tri_a, fr_a = _mesh(8, 10)
    tri_b, fr_b = _mesh(10, 6)
    a, b = DualMesh(tri_a, fr_a.shape[1], 2), DualMesh(tri_b, fr_b.shape[1], 1)
    xa = torch.as_tensor(fr_a[:3], device="cuda").contiguous()
    xb = torch.as_tensor(fr_b[:4], device="cuda").contiguous()
    ra, rb = a.apply(xa), b.apply(xb)
    for _ in range(2):
        oa, ob = torch.empty_like(ra), torch.empty_like(rb)
        a.apply_noalloc(xa, oa)
        b.apply_noalloc(xb, ob)
        torch.cuda.synchronize()
        assert torch.equal(oa, ra) and torch.equal(ob, rb)
    tri, frames = _mesh(30, 40)     # the bench's cylinder: W at 3 levels is far beyond 16 MiB
    big = DualMesh(tri, frames.shape[1], 3)
    xc = torch.as_tensor(frames[:1], device="cuda").contiguous()
    out = torch.empty((1, big.n_fine, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="CAPACITY"):
        big.apply_noalloc(xc, out)
