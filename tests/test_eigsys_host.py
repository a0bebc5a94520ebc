"""The FEM and affine-body kernels project the Hessians of the Stable
Neo-Hookean density (Sec. III-C.1) and of the orthogonality energy
kv |A A^T - I|^2 (Sec. III-C.2) to PSD with the energies' closed-form
eigensystems on a signed SVD instead of a 9x9 eigensolver.  The same header,
built for the host with g++, is checked against the definition of the
projection (numpy eigh, negative eigenvalues clamped to zero) on matrices
that stress the SVD: inverted, repeated and zero singular values, rank one,
the rest state; the orthogonality Hessian itself against finite differences
of its energy.  CPU only."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2609_25653_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    so = str(tmp_path_factory.mktemp("eigsys") / "eigsys.so")
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-I", CSRC, os.path.join(HERE, "eigsys_host_harness.cpp"),
                           "-o", so])
    L = ctypes.CDLL(so)
    P = ctypes.POINTER(ctypes.c_double)
    L.hess_c.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int, P]
    L.ortho_c.argtypes = [P, ctypes.c_double, P, ctypes.c_int]
    return L


def _call(L, F, mu, lh, proj):
    P = ctypes.POINTER(ctypes.c_double)
    F = np.ascontiguousarray(F, float)
    H = np.zeros(45)
    s = np.zeros(21)
    L.hess_c(F.ctypes.data_as(P), mu, lh, H.ctypes.data_as(P), proj, s.ctypes.data_as(P))
    M = np.zeros((9, 9))
    M[np.triu_indices(9)] = H
    return M + M.T - np.diag(np.diag(M)), s[:9].reshape(3, 3), s[9:18].reshape(3, 3), s[18:]


def _rot(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return Q


def _cases(n, seed=3):
    rng = np.random.default_rng(seed)
    for k in range(n):
        kind = k % 8
        if kind == 0:
            F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
        elif kind == 1:
            F = rng.standard_normal((3, 3))
        elif kind == 2:
            F = _rot(rng) @ np.diag(rng.choice([0.5, 1.0, 1.3], 3)) @ _rot(rng)
        elif kind == 3:
            F = np.eye(3) + 1e-9 * rng.standard_normal((3, 3))
        elif kind == 4:
            F = _rot(rng) @ np.diag([1.2, 0.9, rng.choice([1e-3, -1e-3, 1e-6, 0.0])]) @ _rot(rng)
        elif kind == 5:
            F = np.diag(rng.uniform(0.3, 2.0, 3)) * rng.choice([1.0, -1.0], 3)
        elif kind == 6:
            F = np.eye(3)
        else:
            F = np.outer(rng.standard_normal(3), rng.standard_normal(3)) if k % 16 == 7 else np.zeros((3, 3))
        mu = 10 ** rng.uniform(3, 7)
        yield F, mu, mu * 10 ** rng.uniform(-0.5, 2.5)


def test_projection_matches_the_clamped_eigendecomposition(lib):
    neg = 0
    for F, mu, lh in _cases(4000):
        M0, _, _, _ = _call(lib, F, mu, lh, 0)
        M1, _, _, _ = _call(lib, F, mu, lh, 1)
        w, Q = np.linalg.eigh(M0)
        ref = (Q * np.maximum(w, 0.0)) @ Q.T
        neg += w.min() < 0
        assert np.abs(M1 - ref).max() <= 1e-13 * np.abs(M0).max(), (F, mu, lh)
        assert np.linalg.eigvalsh(M1).min() >= -1e-13 * np.abs(M0).max()
    assert neg > 1000      # the cases exercise the correction, not only the early exit


def test_signed_svd_is_a_factorisation_with_rotations(lib):
    for F, mu, lh in _cases(800, seed=4):
        _, U, V, s = _call(lib, F, mu, lh, 0)
        assert np.abs(U @ np.diag(s) @ V.T - F).max() <= 1e-14 * max(np.abs(F).max(), 1.0)
        for R in (U, V):
            assert np.abs(R.T @ R - np.eye(3)).max() < 1e-14 and abs(np.linalg.det(R) - 1.0) < 1e-14
        tol = 1e-14 * max(abs(s[0]), 1e-300)      # singular values at rounding level have no order
        assert s[0] >= 0 and s[1] >= 0 and abs(s[0]) >= abs(s[1]) - tol and abs(s[1]) >= abs(s[2]) - tol
        # the sign of the last singular value is the sign of det F
        d = np.linalg.det(F)
        if abs(d) > 1e-12:
            assert np.sign(s[2]) == np.sign(d)


def test_psd_hessian_is_kept_bit_for_bit(lib):
    """Every mode is positive when |lh (J - 1) - mu| s_k < mu for all k (here
    J = 1.01: lh (J - 1) is close to mu): the projection must leave the formed
    Hessian untouched."""
    F = np.diag([1.004, 1.003, 1.003])
    M0, _, _, _ = _call(lib, F, 1e5, 1e7, 0)
    assert np.linalg.eigvalsh(M0).min() > 0
    M1, _, _, _ = _call(lib, F, 1e5, 1e7, 1)
    assert np.array_equal(M0, M1)


def _ortho(L, A, kv, proj):
    P = ctypes.POINTER(ctypes.c_double)
    A = np.ascontiguousarray(A, float)
    H = np.zeros(45)
    L.ortho_c(A.ctypes.data_as(P), kv, H.ctypes.data_as(P), proj)
    M = np.zeros((9, 9))
    M[np.triu_indices(9)] = H
    return M + M.T - np.diag(np.diag(M))


def test_orthogonality_hessian_matches_finite_differences(lib):
    rng = np.random.default_rng(7)
    kv = 3.0

    def energy(a):
        A = a.reshape(3, 3, order="F")
        return kv * np.sum((A @ A.T - np.eye(3)) ** 2)

    for _ in range(20):
        A = np.eye(3) + 0.4 * rng.standard_normal((3, 3))
        M = _ortho(lib, A, kv, 0)
        a = A.ravel(order="F")      # vec index 3 * column + row
        h = 1e-4
        FD = np.zeros((9, 9))
        for r in range(9):
            for c in range(9):
                er, ec = np.eye(9)[r] * h, np.eye(9)[c] * h
                FD[r, c] = (energy(a + er + ec) - energy(a + er - ec) - energy(a - er + ec) + energy(a - er - ec)) / (4 * h * h)
        assert np.abs(M - FD).max() <= 1e-6 * np.abs(M).max()


def test_orthogonality_projection_matches_the_clamped_eigendecomposition(lib):
    neg = 0
    for k, (A, _, _) in enumerate(_cases(3000, seed=9)):
        kv = 10 ** np.random.default_rng(k).uniform(-2, 6)
        M0 = _ortho(lib, A, kv, 0)
        M1 = _ortho(lib, A, kv, 1)
        w, Q = np.linalg.eigh(M0)
        ref = (Q * np.maximum(w, 0.0)) @ Q.T
        neg += w.min() < 0
        scale = max(np.abs(M0).max(), 4.0 * kv)
        assert np.abs(M1 - ref).max() <= 1e-13 * scale, (A, kv)
    assert neg > 1000
