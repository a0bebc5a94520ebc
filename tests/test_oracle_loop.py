"""Pins of the dual-mesh mapping oracle (Loop subdivision, Eq. (6)-(7)),
each against something other than the oracle's own rules: Loop's published
weights, the limit masks of the scheme's eigen-analysis (a vertex's limit
point does not change when the mesh is subdivided), the uniform cubic
B-spline of scipy for the boundary, Euler's formula for the counts, and
affine invariance.  CPU only."""
import math

import numpy as np
import pytest

from oracle.loop_subdiv import loop_beta, loop_level, loop_subdivide


def octahedron():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]])
    return V, F


def icosahedron():
    p = (1 + 5 ** 0.5) / 2
    V = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0], [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], float)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11],
                  [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    return V, F


def torus(nu=8, nv=6, R=1.0, r=0.35, jitter=0.0, seed=0):
    """Regular triangulation of a torus: every vertex has valence 6."""
    rng = np.random.default_rng(seed)
    V = []
    for i in range(nu):
        for j in range(nv):
            u, v = 2 * math.pi * i / nu, 2 * math.pi * j / nv
            V.append([(R + r * math.cos(v)) * math.cos(u), (R + r * math.cos(v)) * math.sin(u), r * math.sin(v)])
    V = np.array(V) + jitter * rng.standard_normal((nu * nv, 3))
    idx = lambda i, j: (i % nu) * nv + (j % nv)
    F = []
    for i in range(nu):
        for j in range(nv):
            F.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)])
            F.append([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)])
    return V, np.array(F)


def hexagon_fan(seed=0):
    """A planar hexagon split into 6 triangles around its centre: one
    interior vertex of valence 6, six boundary vertices."""
    rng = np.random.default_rng(seed)
    rim = [[math.cos(k * math.pi / 3), math.sin(k * math.pi / 3), 0.0] for k in range(6)]
    V = np.array([[0.0, 0.0, 0.0]] + rim) + 0.05 * rng.standard_normal((7, 3)) * np.array([1, 1, 0])
    F = np.array([[0, 1 + k, 1 + (k + 1) % 6] for k in range(6)])
    return V, F


def one_ring(F, i):
    nb = set()
    for t in F:
        t = [int(v) for v in t]
        if i in t:
            nb.update(v for v in t if v != i)
    return sorted(nb)


def limit_mask(V, F, i):
    """Limit point of interior vertex i: (1 - n chi) v + chi sum(nbrs) with
    chi = 1 / (n + 3 / (8 beta)), the left eigenvector of Loop's local
    subdivision matrix for the eigenvalue 1 (Hoppe et al. 1994)."""
    nb = one_ring(F, i)
    n = len(nb)
    chi = 1.0 / (n + 3.0 / (8.0 * loop_beta(n)))
    return (1.0 - n * chi) * V[i] + chi * V[nb].sum(0)


def test_beta_matches_loops_published_weights():
    # Loop (1987): valence 3 -> 3/16; valence 4 -> 31/256; the regular case
    # (valence 6) is the quartic box spline, whose vertex mask is 10/16 of the
    # vertex and 1/16 of each neighbour
    assert loop_beta(3) == pytest.approx(3.0 / 16.0, rel=1e-15)
    assert loop_beta(4) == pytest.approx(31.0 / 256.0, rel=1e-15)
    assert loop_beta(6) == pytest.approx(1.0 / 16.0, rel=1e-15)
    assert 1.0 - 6 * loop_beta(6) == pytest.approx(10.0 / 16.0, rel=1e-15)


@pytest.mark.parametrize("mesh", [octahedron, icosahedron, lambda: torus(jitter=0.05)])
def test_limit_point_is_invariant_under_subdivision(mesh):
    """The limit mask evaluated on the subdivided mesh equals the one on the
    coarse mesh for every old vertex: it holds only if the vertex rule and the
    edge rule (which forms the new one-ring) carry Loop's weights."""
    V, F = mesh()
    V1, F1 = loop_level(V, F)
    V2, F2 = loop_level(V1, F1)
    for i in range(len(V)):
        p0 = limit_mask(V, F, i)
        assert np.abs(limit_mask(V1, F1, i) - p0).max() < 1e-14
        assert np.abs(limit_mask(V2, F2, i) - p0).max() < 1e-14


def test_regular_limit_is_the_box_spline_mask():
    """On a regular torus (valence 6 everywhere) the limit mask is the quartic
    box spline's: 1/2 of the vertex and 1/12 of each neighbour."""
    V, F = torus(jitter=0.03, seed=4)
    V3, F3 = loop_subdivide(V, F, 3)
    for i in range(len(V)):
        nb = one_ring(F3, i)
        assert len(nb) == 6
        box = 0.5 * V3[i] + V3[nb].sum(0) / 12.0
        assert np.abs(box - limit_mask(V, F, i)).max() < 1e-14


def test_boundary_follows_the_cubic_bspline():
    """A boundary curve subdivides as the uniform cubic B-spline of the
    boundary polygon: the B-spline limit mask (1, 4, 1) / 6 of an old rim
    vertex is the same on every level, and equals scipy's periodic cubic
    B-spline of the rim polygon at that vertex's knot."""
    from scipy.interpolate import BSpline
    V, F = hexagon_fan(seed=2)
    rim = V[1:]
    # scipy: periodic cubic B-spline with the rim as control points (uniform knots)
    k = 3
    ctrl = np.vstack([rim, rim[:k]])
    t = np.arange(len(ctrl) + k + 1, dtype=float)
    spl = BSpline(t, ctrl, k)
    V1, F1 = loop_level(V, F)
    V2, F2 = loop_level(V1, F1)

    def bmask(VV, FF, i):
        # the two boundary neighbours of rim vertex i on this level
        nb = []
        for a in one_ring(FF, i):
            cnt = sum(1 for tri in FF if i in tri and a in tri)
            if cnt == 1:
                nb.append(a)
        assert len(nb) == 2
        return (VV[nb[0]] + 4 * VV[i] + VV[nb[1]]) / 6.0

    for m in range(6):
        i = 1 + m
        # at integer knot j the curve is (c[j-3] + 4 c[j-2] + c[j-1]) / 6: rim
        # point m is c[m] (and c[6] for m = 0), inside the valid span [3, 9]
        ref = spl(m + 2 if m >= 1 else 8)
        prev = rim[m - 1]
        nxt = rim[(m + 1) % 6]
        assert np.abs((prev + 4 * rim[m] + nxt) / 6.0 - ref).max() < 1e-14
        assert np.abs(bmask(V, F, i) - ref).max() < 1e-14
        assert np.abs(bmask(V1, F1, i) - ref).max() < 1e-14
        assert np.abs(bmask(V2, F2, i) - ref).max() < 1e-14


@pytest.mark.parametrize("mesh", [octahedron, icosahedron, torus])
def test_counts_follow_euler(mesh):
    """Every level: F' = 4 F, V' = V + E, E' = 2 E + 3 F; the Euler
    characteristic is kept; every directed edge appears once (a consistently
    oriented closed manifold)."""
    V, F = mesh()

    def edges(F):
        return {tuple(sorted((int(t[a]), int(t[(a + 1) % 3])))) for t in F for a in range(3)}

    chi = len(V) - len(edges(F)) + len(F)
    for _ in range(3):
        E = len(edges(F))
        V1, F1 = loop_level(V, F)
        assert len(F1) == 4 * len(F) and len(V1) == len(V) + E and len(edges(F1)) == 2 * E + 3 * len(F)
        assert len(V1) - len(edges(F1)) + len(F1) == chi
        directed = [(int(t[a]), int(t[(a + 1) % 3])) for t in F1 for a in range(3)]
        assert len(set(directed)) == len(directed)
        V, F = V1, F1


def test_affine_invariance():
    """The weights of every rule sum to one: subdividing A X + b gives
    A S(X) + b."""
    V, F = icosahedron()
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    Vf, _ = loop_subdivide(V, F, 2)
    Vg, _ = loop_subdivide(V @ A.T + b, F, 2)
    assert np.abs(Vg - (Vf @ A.T + b)).max() < 1e-13


def test_rejects_non_manifold_edges():
    V = np.zeros((5, 3))
    F = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]])
    with pytest.raises(ValueError):
        loop_level(V, F)
