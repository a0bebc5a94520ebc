"""Pins of the oracle's pointwise formulas against mathematics that does not
depend on the oracle: finite differences, closed forms, invariants, LAPACK and
exhaustive KKT enumeration.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle as O

rng = np.random.default_rng(1234)


def rand_rot(r):
    q, _ = np.linalg.qr(r.standard_normal((3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


# ---------------------------------------------------------------- SNH (C3)
def test_snh_zero_at_rest_and_rotations():
    mu, lam = 3.4e4, 2.2e5
    for F in [np.eye(3)] + [rand_rot(rng) for _ in range(5)]:
        psi, P, _ = O.snh(F, mu, lam)
        assert abs(psi) < 1e-10 * mu
        assert np.abs(P).max() < 1e-10 * mu


def test_snh_small_strain_limit():
    """Rest-stable SNH with lh = lam + mu linearises to mu eps:eps + lam/2 tr(eps)^2."""
    mu, lam = 1.0e4, 3.0e4
    G = rng.standard_normal((3, 3))
    for eps in (1e-3, 1e-4):
        F = np.eye(3) + eps * G
        psi, _, _ = O.snh(F, mu, lam)
        e = eps * 0.5 * (G + G.T)
        ref = mu * np.sum(e * e) + 0.5 * lam * np.trace(e) ** 2
        assert abs(psi - ref) < 50 * eps * abs(ref)


@pytest.mark.parametrize("scale", [0.05, 0.4])
def test_snh_derivatives_fd(scale):
    mu, lam = 2.0e4, 5.0e4
    for _ in range(4):
        F = np.eye(3) + scale * rng.standard_normal((3, 3))
        psi, P, H = O.snh(F, mu, lam)
        Fv = F.T.ravel()
        h = 1e-6
        Pfd = np.zeros(9)
        Hfd = np.zeros((9, 9))
        for i in range(9):
            d = np.zeros(9); d[i] = h
            Fp = (Fv + d).reshape(3, 3).T
            Fm = (Fv - d).reshape(3, 3).T
            Pfd[i] = (O.snh(Fp, mu, lam)[0] - O.snh(Fm, mu, lam)[0]) / (2 * h)
            Hfd[:, i] = (O.snh(Fp, mu, lam)[1].T.ravel() - O.snh(Fm, mu, lam)[1].T.ravel()) / (2 * h)
        assert np.allclose(P.T.ravel(), Pfd, rtol=1e-7, atol=1e-7 * mu)
        assert np.allclose(H, Hfd, rtol=1e-6, atol=1e-6 * mu)
        assert np.allclose(H, H.T, atol=1e-9 * mu)


# ---------------------------------------------------------------- PSD (C11)
@pytest.mark.parametrize("n", [3, 9, 12])
def test_psd_projection_matches_lapack(n):
    for _ in range(5):
        A = rng.standard_normal((n, n)); A = A + A.T
        w, Q = np.linalg.eigh(A)
        ref = (Q * np.maximum(w, 0)) @ Q.T
        got = O.psd_project(A)
        assert np.allclose(got, ref, atol=1e-12 * np.abs(A).max())
        assert np.linalg.eigvalsh(got).min() > -1e-12 * np.abs(A).max()


def test_psd_projection_identity_on_psd():
    B = rng.standard_normal((12, 7))
    A = B @ B.T
    assert np.allclose(O.psd_project(A), A, atol=1e-12 * np.abs(A).max())


# ---------------------------------------------------------------- barrier (C8)
def test_barrier_vanishes_at_and_beyond_dhat():
    dh = 1e-3
    assert np.all(O.barrier3(dh, dh) == 0)
    assert np.all(O.barrier3(2 * dh, dh) == 0)
    b = O.barrier3(dh * (1 - 1e-6), dh)
    assert abs(b[0]) < 1e-16 and abs(b[1]) < 1e-12 and abs(b[2]) < 1e-4


def test_barrier_derivatives_fd():
    dh = 1e-3
    for d in (1e-5, 2e-4, 7e-4, 9.9e-4):
        h = 1e-7 * d
        b = O.barrier3(d, dh)
        bp = O.barrier3(d + h, dh); bm = O.barrier3(d - h, dh)
        assert np.isclose((bp[0] - bm[0]) / (2 * h), b[1], rtol=1e-6)
        assert np.isclose((bp[1] - bm[1]) / (2 * h), b[2], rtol=1e-6)
        assert b[0] > 0 and b[1] < 0 and b[2] > 0


# ---------------------------------------------------------------- distances (C7)
def _kkt_min(r0, D, cons):
    """Exact convex QP min |r0 + D s|^2 subject to linear inequality rows
    (a, b): a.s >= b, by enumerating every active set (KKT brute force)."""
    m = D.shape[1]
    best = np.inf
    for k in range(0, m + 1):
        for act in itertools.combinations(range(len(cons)), k):
            # minimise with the active constraints as equalities (Lagrange system)
            A = np.array([cons[i][0] for i in act]).reshape(k, m)
            b = np.array([cons[i][1] for i in act])
            K = np.zeros((m + k, m + k))
            K[:m, :m] = 2 * D.T @ D
            K[:m, m:] = -A.T
            K[m:, :m] = A
            rhs = np.concatenate([-2 * D.T @ r0, b])
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            s = sol[:m]
            if all(np.dot(a, s) >= bb - 1e-12 for a, bb in cons):
                best = min(best, float(np.sum((r0 + D @ s) ** 2)))
    return best


def ref_pt(x):
    p, t0, t1, t2 = x.reshape(4, 3)
    D = np.stack([t1 - t0, t2 - t0], 1)
    cons = [(np.array([1.0, 0.0]), 0.0), (np.array([0.0, 1.0]), 0.0), (np.array([-1.0, -1.0]), -1.0)]
    return _kkt_min(t0 - p, D, cons)


def ref_ee(x):
    a0, a1, b0, b1 = x.reshape(4, 3)
    D = np.stack([a1 - a0, -(b1 - b0)], 1)
    cons = [(np.array([1.0, 0.0]), 0.0), (np.array([-1.0, 0.0]), -1.0),
            (np.array([0.0, 1.0]), 0.0), (np.array([0.0, -1.0]), -1.0)]
    return _kkt_min(a0 - b0, D, cons)


def test_distance_pt_random():
    for _ in range(400):
        x = rng.standard_normal(12)
        d2, t = O.dist2_pt(x)
        ref = ref_pt(x)
        assert abs(d2 - ref) <= 1e-10 * max(ref, 1e-3), (d2, ref, t)


def test_distance_ee_random():
    for _ in range(400):
        x = rng.standard_normal(12)
        d2, t = O.dist2_ee(x)
        ref = ref_ee(x)
        assert abs(d2 - ref) <= 1e-10 * max(ref, 1e-3), (d2, ref, t)


def test_distance_special_cases():
    # point above a triangle interior: plane type, exact height
    x = np.array([0.2, 0.2, 0.7, 0, 0, 0, 1, 0, 0, 0, 1, 0], float)
    d2, t = O.dist2_pt(x)
    assert t == 6 and d2 == pytest.approx(0.49, rel=1e-15)
    # point beyond a vertex: point-point
    x = np.array([-1, -1, 0.5, 0, 0, 0, 1, 0, 0, 0, 1, 0], float)
    d2, t = O.dist2_pt(x)
    assert t == 0 and d2 == pytest.approx(2.25, rel=1e-15)
    # crossing edges at height 0.3: line-line
    x = np.array([-1, 0, 0, 1, 0, 0, 0, -1, 0.3, 0, 1, 0.3], float)
    d2, t = O.dist2_ee(x)
    assert t == 8 and d2 == pytest.approx(0.09, rel=1e-14)
    # parallel edges, overlapping span: distance between the lines
    x = np.array([0, 0, 0, 1, 0, 0, 0.5, 0.2, 0, 1.5, 0.2, 0], float)
    d2, t = O.dist2_ee(x)
    assert d2 == pytest.approx(0.04, rel=1e-14) and t in (4, 5, 6, 7)
    # collinear disjoint edges: endpoint gap
    x = np.array([0, 0, 0, 1, 0, 0, 1.5, 0, 0, 3, 0, 0], float)
    d2, t = O.dist2_ee(x)
    assert d2 == pytest.approx(0.25, rel=1e-14)


def test_distance_parallel_coplanar_edges_with_rounding():
    """Parallel face diagonals on one face of a generated pad: their
    coordinates are not exact in binary, so A C - B^2 is a rounding residue;
    the edges must still be treated as parallel (distance from the
    point-segment cases), not as crossing lines at distance 0."""
    import ipcscenes
    def seg_d2(p, a, b):
        t = np.clip(np.dot(p - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
        q = a + t * (b - a)
        return float(np.dot(p - q, p - q))
    X = ipcscenes.scenes.grid_vertices(10, 5, 5, (0.28, 0.258, 0.0105), (0.004, 0.004, 0.004))
    vid = lambda i, j, k: (i * 6 + j) * 6 + k
    n_checked = 0
    for j in range(4):
        for k in range(4):
            # diagonal (j,k+1)-(j+1,k) and its neighbour shifted by one cell in y and z
            a0, a1 = X[vid(0, j, k + 1)], X[vid(0, j + 1, k)]
            for dj, dk in ((1, 1), (1, 0), (0, 1)):
                if j + 1 + dj > 5 or k + 1 + dk > 5:
                    continue
                b0, b1 = X[vid(0, j + dj, k + 1 + dk)], X[vid(0, j + 1 + dj, k + dk)]
                if any(np.array_equal(p, q) for p in (a0, a1) for q in (b0, b1)):
                    continue
                d2, t = O.dist2_ee(np.concatenate([a0, a1, b0, b1]))
                ref = min(seg_d2(a0, b0, b1), seg_d2(a1, b0, b1), seg_d2(b0, a0, a1), seg_d2(b1, a0, a1))
                assert t != 8 and d2 == pytest.approx(ref, rel=1e-12), (j, k, dj, dk, d2, ref, t)
                n_checked += 1
    assert n_checked > 20


def test_generated_squeeze_scenes_start_separated():
    """Regression: the batched squeeze generator's scenes start with every
    contact pair at a positive distance (finite energy)."""
    import ipcscenes
    for sc in ipcscenes.batched_squeeze(n_scenes=16, n_steps=2):
        o = O.Oracle(sc)
        o.begin_step(0)
        y, _ = o.state()
        assert np.isfinite(o.energy(y)[0])


@pytest.mark.parametrize("kind", [0, 1])
def test_distance_derivatives_fd(kind):
    f = O.dist2_pt if kind == 0 else O.dist2_ee
    n = 0
    while n < 60:
        x = rng.standard_normal(12)
        d2, g, H = O.dist2_derivs(kind, x)
        h = 1e-6
        # stay inside one distance type for the finite-difference stencil
        types = {f(x + h * e)[1] for e in np.eye(12)} | {f(x - h * e)[1] for e in np.eye(12)}
        if len(types) > 1:
            continue
        n += 1
        gfd = np.array([(f(x + h * e)[0] - f(x - h * e)[0]) / (2 * h) for e in np.eye(12)])
        Hfd = np.stack([(O.dist2_derivs(kind, x + h * e)[1] - O.dist2_derivs(kind, x - h * e)[1]) / (2 * h)
                        for e in np.eye(12)], 1)
        sc = max(1.0, np.abs(g).max())
        assert np.allclose(g, gfd, atol=1e-6 * sc)
        assert np.allclose(H, Hfd, atol=1e-5 * max(1.0, np.abs(H).max()))
        assert np.allclose(H, H.T, atol=1e-10 * max(1.0, np.abs(H).max()))


# ---------------------------------------------------------------- CCD (C13)
def test_accd_point_onto_triangle_bounds():
    s = 0.1
    for _ in range(50):
        z0 = rng.uniform(0.1, 2.0)
        speed = rng.uniform(0.2, 5.0) * z0
        x = np.array([0.2, 0.3, z0, 0, 0, 0, 1, 0, 0, 0, 1, 0], float)
        p = np.zeros(12); p[2] = -speed
        toi = z0 / speed
        t = O.accd(0, x, p, s)
        if toi >= 1.0:
            assert t == 1.0 or t <= toi
        else:
            assert (1 - s) * toi * (1 - 1e-12) <= t <= toi


def test_accd_separating_motion_is_free():
    x = np.array([0.2, 0.3, 0.5, 0, 0, 0, 1, 0, 0, 0, 1, 0], float)
    p = np.zeros(12); p[2] = 1.0
    assert O.accd(0, x, p) == 1.0
    x = np.array([0, 0, 0, 1, 0, 0, 0, -1, 0.3, 0, 1, 0.3], float)
    p = np.zeros(12)
    assert O.accd(1, x, p) == 1.0


def test_accd_keeps_positive_distance():
    for kind in (0, 1):
        f = O.dist2_pt if kind == 0 else O.dist2_ee
        for _ in range(200):
            x = rng.standard_normal(12)
            p = 3.0 * rng.standard_normal(12)
            t = O.accd(kind, x, p)
            assert 0.0 <= t <= 1.0
            # distance stays positive along [0, t] (dense sampling)
            for a in np.linspace(0.0, t, 41):
                assert f(x + a * p)[0] > 0.0
