"""Oracle of the dual-mesh mapping (Sec. III-D, Eq. (6)-(7)): L levels of Loop
subdivision of a coarse triangle mesh, computed directly on vertex positions,
one level at a time, in plain Python loops.  Test infrastructure only: it is
used by the tests and by bench.py's CPU baseline, never by the library.

The paper obtains the fine render mesh of a deformable object by L-level
Loop subdivision of the coarse simulation mesh.  Because every level is a
linear map of the positions, the fine positions are W X^c with W the product
of the per-level maps (Eq. (6)); applying the levels one after the other to
the positions (as here) gives the same fine positions up to rounding.

Rules of one level (Loop's scheme; the paper names it without weights):
  * edge vertex of an edge shared by two triangles: 3/8 of each end plus 1/8
    of each of the two opposite corners;
  * edge vertex of a boundary edge (one triangle): the midpoint;
  * old interior vertex of valence n: (1 - n beta) of itself plus beta of
    each neighbour, beta = (5/8 - (3/8 + cos(2 pi / n) / 4)^2) / n;
  * old boundary vertex (two boundary edges): 3/4 of itself plus 1/8 of each
    of its two boundary neighbours;
  * a vertex in no triangle keeps its position.
An edge in more than two triangles, or a vertex on more than two boundary
edges, is not a manifold configuration and is rejected.

Numbering of one level's output (shared with the library as a convention,
not as code): the old vertices keep their indices; edges are numbered in the
order in which they are first met when the triangles are scanned in order,
each triangle (a, b, c) contributing (a, b), (b, c), (c, a); the vertex of
edge e gets index n_old + e.  Triangle (a, b, c) with edge vertices ab, bc,
ca becomes, in this order, (a, ab, ca), (b, bc, ab), (c, ca, bc),
(ab, bc, ca).
"""
import math

import numpy as np


def loop_beta(n):
    """Weight of each neighbour of an interior vertex of valence n."""
    return (5.0 / 8.0 - (3.0 / 8.0 + 0.25 * math.cos(2.0 * math.pi / n)) ** 2) / n


def loop_level(V, F):
    """One level of Loop subdivision: (V (n, 3), F (m, 3)) -> (V', F')."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    n = len(V)
    edge_id = {}            # (min, max) -> edge index
    edge_ends = []          # (a, b) as first met
    edge_opp = []           # opposite corners of the triangles on the edge
    for t in range(len(F)):
        a, b, c = (int(v) for v in F[t])
        for u, w, o in ((a, b, c), (b, c, a), (c, a, b)):
            key = (min(u, w), max(u, w))
            e = edge_id.get(key)
            if e is None:
                e = len(edge_ends)
                edge_id[key] = e
                edge_ends.append((u, w))
                edge_opp.append([])
            edge_opp[e].append(o)
    # neighbours and boundary neighbours of the old vertices
    nbrs = [set() for _ in range(n)]
    bnd = [[] for _ in range(n)]
    for e, (u, w) in enumerate(edge_ends):
        if len(edge_opp[e]) > 2:
            raise ValueError(f"edge {u}-{w} is shared by {len(edge_opp[e])} triangles")
        nbrs[u].add(w)
        nbrs[w].add(u)
        if len(edge_opp[e]) == 1:
            bnd[u].append(w)
            bnd[w].append(u)
    out = np.zeros((n + len(edge_ends), 3))
    for i in range(n):
        if len(bnd[i]) > 2:
            raise ValueError(f"vertex {i} lies on {len(bnd[i])} boundary edges")
        if len(bnd[i]) == 2:
            out[i] = 0.75 * V[i] + 0.125 * (V[bnd[i][0]] + V[bnd[i][1]])
        elif nbrs[i]:
            k = len(nbrs[i])
            beta = loop_beta(k)
            s = np.zeros(3)
            for j in sorted(nbrs[i]):
                s += V[j]
            out[i] = (1.0 - k * beta) * V[i] + beta * s
        else:
            out[i] = V[i]
    for e, (u, w) in enumerate(edge_ends):
        opp = edge_opp[e]
        if len(opp) == 2:
            out[n + e] = 0.375 * (V[u] + V[w]) + 0.125 * (V[opp[0]] + V[opp[1]])
        else:
            out[n + e] = 0.5 * (V[u] + V[w])
    Fo = np.zeros((4 * len(F), 3), dtype=np.int64)
    for t in range(len(F)):
        a, b, c = (int(v) for v in F[t])
        ab = n + edge_id[(min(a, b), max(a, b))]
        bc = n + edge_id[(min(b, c), max(b, c))]
        ca = n + edge_id[(min(c, a), max(c, a))]
        Fo[4 * t] = (a, ab, ca)
        Fo[4 * t + 1] = (b, bc, ab)
        Fo[4 * t + 2] = (c, ca, bc)
        Fo[4 * t + 3] = (ab, bc, ca)
    return out, Fo


def loop_subdivide(V, F, levels):
    """L levels of Loop subdivision: the fine positions and triangles."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    for _ in range(levels):
        V, F = loop_level(V, F)
    return V, F


def loop_limit_point(V, F, i):
    """Limit position of interior vertex i under repeated subdivision: the
    eigen-analysis of the scheme's local subdivision matrix gives
    (1 - n chi) v + chi sum(neighbours), chi = 1 / (n + 3 / (8 beta))
    (Hoppe et al. 1994).  Independent of the rules' code above: a pin."""
    nb = set()
    for t in F:
        t = [int(v) for v in t]
        if i in t:
            nb.update(v for v in t if v != i)
    n = len(nb)
    chi = 1.0 / (n + 3.0 / (8.0 * loop_beta(n)))
    return (1.0 - n * chi) * np.asarray(V[i], float) + chi * np.sum([V[j] for j in sorted(nb)], axis=0)
