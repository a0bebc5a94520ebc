"""Dual-mesh mapping (Sec. III-D, Eq. (6)-(7)): the library's host-built W and
fine triangles against the oracle, which subdivides positions level by
level.  Host work only (no GPU): W X^c is formed here with numpy from the
library's W, and compared with the oracle's fine positions."""
import numpy as np
import pytest
import scipy.sparse as sp

import ipcscenes as S
from oracle.loop_subdiv import loop_subdivide
from paper_2609_25653_amd.dualmesh import DualMesh
from test_oracle_loop import hexagon_fan, icosahedron, octahedron, torus


def _w(dm):
    rp, col, val = dm.weights()
    return sp.csr_matrix((val, col, rp), shape=(dm.n_fine, dm.n_coarse))


@pytest.mark.parametrize("mesh", [octahedron, icosahedron, lambda: torus(jitter=0.05), hexagon_fan])
@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_weights_reproduce_the_oracle(mesh, levels):
    V, F = mesh()
    dm = DualMesh(F, len(V), levels)
    Vf, Ff = loop_subdivide(V, F, levels)
    assert dm.n_fine == len(Vf) and dm.n_tri == len(Ff)
    assert np.array_equal(dm.fine_tris(), Ff)                      # the numbering convention, bit-exact
    W = _w(dm)
    assert np.abs(W @ V - Vf).max() <= 1e-14 * np.abs(V).max()
    assert np.abs(np.asarray(W.sum(1)).ravel() - 1.0).max() < 1e-14   # affine: rows sum to one
    rp, col, _ = dm.weights()
    assert all(np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0) for r in range(dm.n_fine))


def test_cylinder_surface_at_full_size():
    """The render workload's mesh (6602 vertices, 13200 triangles), three
    levels: W X^c against the oracle on one frame of the trajectory."""
    tri, frames = S.dualmesh_frames(n_frames=3)
    dm = DualMesh(tri, frames.shape[1], 3)
    Vf, Ff = loop_subdivide(frames[2], tri, 3)
    assert dm.n_fine == 422402 and np.array_equal(dm.fine_tris(), Ff)
    assert np.abs(_w(dm) @ frames[2] - Vf).max() <= 1e-14 * np.abs(frames[2]).max()


@pytest.mark.parametrize("tri,msg", [
    ([[0, 1, 2], [0, 1, 3], [0, 1, 4]], "more than two triangles"),
    ([[0, 1, 1]], "repeats a vertex"),
    ([[0, 1, 9]], "out of range"),
    ([[0, 1, 2], [0, 3, 4]], "more than two boundary edges"),
])
def test_rejects_invalid_meshes(tri, msg):
    with pytest.raises(RuntimeError, match=msg):
        DualMesh(np.array(tri), 5, 1)


def test_rejects_bad_levels():
    with pytest.raises(RuntimeError, match="levels"):
        DualMesh(np.array([[0, 1, 2]]), 3, 7)
