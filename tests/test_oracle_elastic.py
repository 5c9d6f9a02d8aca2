"""Oracle elasticity and PSD projection against closed forms, finite
differences and numpy's symmetric eigensolver."""
import numpy as np
import pytest

import oracle as O

MU, LAM = O.lame(0.3e6, 0.45)


def rand_F(rng, jmin=0.5, jmax=2.0):
    while True:
        F = np.eye(3) + 0.4 * rng.standard_normal((3, 3))
        J = np.linalg.det(F)
        if jmin <= J <= jmax:
            return F


def rand_rot(rng):
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def test_rest_state_zero():
    assert O.nh_psi(np.eye(3), MU, LAM) == 0.0
    assert np.abs(O.nh_pk1(np.eye(3), MU, LAM)).max() == 0.0


def test_lame_from_E_nu():
    assert abs(MU - 103448.27586206897) < 1e-6
    assert abs(LAM - 931034.4827586205) < 1e-6


def test_hessian_at_identity_is_linear_elastic_tensor():
    H = O.nh_hessian(np.eye(3), MU, LAM)
    d = np.eye(3)
    C = (MU * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
         + LAM * np.einsum("ij,kl->ijkl", d, d)).reshape(9, 9)
    assert np.abs(H - C).max() <= 1e-9 * np.abs(C).max()


def test_inverted_is_infinite():
    F = np.diag([1.0, 1.0, -0.5])
    assert np.isinf(O.nh_psi(F, MU, LAM))


def test_rotation_invariance():
    rng = np.random.default_rng(1)
    for _ in range(20):
        F = rand_F(rng)
        R = rand_rot(rng)
        a, b = O.nh_psi(F, MU, LAM), O.nh_psi(R @ F, MU, LAM)
        assert abs(a - b) <= 1e-10 * abs(a) + 1e-6
        assert np.abs(O.nh_pk1(R @ F, MU, LAM) - R @ O.nh_pk1(F, MU, LAM)).max() <= 1e-8 * MU


def test_fd_stress_and_tangent():
    rng = np.random.default_rng(2)
    h = 1e-7
    for _ in range(10):
        F = rand_F(rng)
        P = O.nh_pk1(F, MU, LAM).ravel()
        H = O.nh_hessian(F, MU, LAM)
        Pfd = np.zeros(9)
        Hfd = np.zeros((9, 9))
        for k in range(9):
            e = np.zeros(9)
            e[k] = h
            Fp, Fm = (F.ravel() + e).reshape(3, 3), (F.ravel() - e).reshape(3, 3)
            Pfd[k] = (O.nh_psi(Fp, MU, LAM) - O.nh_psi(Fm, MU, LAM)) / (2 * h)
            Hfd[:, k] = (O.nh_pk1(Fp, MU, LAM).ravel() - O.nh_pk1(Fm, MU, LAM).ravel()) / (2 * h)
        assert np.abs(P - Pfd).max() <= 1e-6 * np.abs(P).max()
        assert np.abs(H - Hfd).max() <= 1e-6 * np.abs(H).max()
        assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()


def test_sym_eig_matches_numpy():
    rng = np.random.default_rng(3)
    for n in (3, 9, 12):
        A = rng.standard_normal((n, n))
        A = A + A.T
        w, V = O.sym_eig(A)
        assert np.allclose(np.sort(w), np.linalg.eigvalsh(A), atol=1e-12 * np.abs(A).max())
        assert np.abs(V @ np.diag(w) @ V.T - A).max() <= 1e-12 * np.abs(A).max()
        assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13


def test_psd_projection_unique_idempotent():
    rng = np.random.default_rng(4)
    for n in (9, 12):
        for _ in range(10):
            A = rng.standard_normal((n, n))
            A = A + A.T
            P = O.psd_project(A)
            w, V = np.linalg.eigh(A)
            ref = (V * np.maximum(w, 0)) @ V.T
            assert np.abs(P - ref).max() <= 1e-12 * np.abs(A).max()
            assert np.linalg.eigvalsh(P).min() >= -1e-12 * np.abs(A).max()
            assert np.abs(O.psd_project(P) - P).max() <= 1e-12 * np.abs(A).max()
        B = rng.standard_normal((n, n))
        S = B @ B.T
        assert np.array_equal(O.psd_project(S), S)  # no-op on PSD input


def _tet(rng):
    Xr = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float) * 1e-3
    Xr = Xr + 1e-4 * rng.standard_normal((4, 3))
    Dm = np.stack([Xr[1] - Xr[0], Xr[2] - Xr[0], Xr[3] - Xr[0]], axis=1)
    assert np.linalg.det(Dm) > 0
    return Xr, np.linalg.inv(Dm), np.linalg.det(Dm) / 6.0


def test_tet_fd_gradient_and_hessian():
    rng = np.random.default_rng(5)
    for trial in range(8):
        Xr, Bm, vol = _tet(rng)
        # small deformation keeps d2Psi/dF2 PSD so the projection is a no-op
        while True:
            x = Xr + (0.02 if trial < 4 else 0.2) * 1e-3 * rng.standard_normal((4, 3))
            F = (np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1)) @ Bm
            if np.linalg.det(F) > 0.3:
                break
        E, g, H = O.tet_elastic(x.ravel(), Bm.ravel(), vol, MU, LAM)
        h = 1e-7 * 1e-3
        gfd = np.zeros(12)
        Hfd = np.zeros((12, 12))
        for k in range(12):
            e = np.zeros(12)
            e[k] = h
            Ep, gp, _ = O.tet_elastic(x.ravel() + e, Bm.ravel(), vol, MU, LAM)
            Em, gm, _ = O.tet_elastic(x.ravel() - e, Bm.ravel(), vol, MU, LAM)
            gfd[k] = (Ep - Em) / (2 * h)
            Hfd[:, k] = (gp - gm) / (2 * h)
        assert np.abs(g - gfd).max() <= 1e-6 * np.abs(g).max()
        assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
        assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.abs(H).max()
        if np.linalg.eigvalsh(O.nh_hessian(F, MU, LAM)).min() > 0:
            assert np.abs(H - Hfd).max() <= 1e-6 * np.abs(H).max()
        # translation: gradient sums to zero per component
        assert np.abs(g.reshape(4, 3).sum(0)).max() <= 1e-9 * np.abs(g).max()


def test_tet_projected_hessian_compression():
    """Under strong compression the NH tangent is indefinite; the element
    Hessian must be V D^T Pi+(d2Psi/dF2) D, checked against numpy eigh."""
    rng = np.random.default_rng(6)
    Xr, Bm, vol = _tet(rng)
    x = Xr.copy()
    x[:, 2] *= 0.3  # 70% compression along z
    x[:, 0] *= 1.6
    F = (np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1)) @ Bm
    Hf = O.nh_hessian(F, MU, LAM)
    w, V = np.linalg.eigh(Hf)
    assert w.min() < 0  # the case exercises the projection
    Pp = (V * np.maximum(w, 0)) @ V.T
    # D: d vec(F) / d x
    q = np.zeros((4, 3))
    q[1:] = Bm
    q[0] = -Bm.sum(0)
    D = np.zeros((9, 12))
    for i in range(3):
        for j in range(3):
            for a in range(4):
                D[i * 3 + j, a * 3 + i] = q[a, j]
    ref = vol * D.T @ Pp @ D
    _, _, H = O.tet_elastic(x.ravel(), Bm.ravel(), vol, MU, LAM)
    assert np.abs(H - ref).max() <= 1e-10 * np.abs(ref).max()
