"""Pins of the oracle's precompute against closed forms, library routines and
invariants (CPU only)."""
import numpy as np
import pytest

import scenegen
from oracle import model as M


def small(n=8, seed=0, jitter=0.05):
    sc = scenegen.hanging_cloth(n, seed=seed, r=6, jitter=jitter)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    return sc, m


def polygon_area_xz(sc):
    n = sc.n_side
    ring = [i for i in range(n)] + [i * n + n - 1 for i in range(1, n)] + \
        [(n - 1) * n + j for j in range(n - 2, -1, -1)] + [i * n for i in range(n - 2, 0, -1)]
    P = sc.rest.astype(np.float64)[ring][:, [0, 2]]
    x, z = P[:, 0], P[:, 1]
    return 0.5 * abs(np.dot(x, np.roll(z, -1)) - np.dot(z, np.roll(x, -1)))


def test_mass_sums_to_density_times_area():
    sc, m = small(9)
    # shoelace area of the (jittered) boundary polygon, independent of triangles
    assert np.isclose(m.mass.sum(), sc.density * polygon_area_xz(sc), rtol=1e-12)


def test_triangle_quadratic_form_matches_metric_closed_form():
    """x^T H_tri x = sum_t w_t ||F_t||_F^2 with ||F||^2 = tr(D_s^T D_s (E^T E)^{-1}),
    E the 3x2 rest edge matrix: independent of the 2-D frame used in the oracle."""
    sc, m = small(7)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((m.nv, 3))
    X = m.rest
    tot = 0.0
    for t, (i, j, k) in enumerate(m.tris):
        E = np.stack([X[j] - X[i], X[k] - X[i]], 1)
        Ds = np.stack([x[j] - x[i], x[k] - x[i]], 1)
        tot += m.w_tri[t] * np.trace(Ds.T @ Ds @ np.linalg.inv(E.T @ E))
    # rebuild H without mass and bending
    mt = M.build_model(sc.tris, sc.rest, sc.pinned, 1.0, 0.0, sc.k_stretch, 0.0)
    q = sum(x[:, d] @ (mt.H @ x[:, d]) for d in range(3))
    assert np.isclose(q, tot, rtol=1e-11)


def test_bending_stencil_closed_form_and_affine_null():
    """K = [k0, k1, -|e|/h_A, -|e|/h_B] with k0, k1 fixed by sum K = 0 and
    sum K X = 0 (rest hinge is planar); bending energy vanishes on affine maps."""
    sc, m = small(8)
    X = m.rest
    for e in range(0, len(m.hinges), 7):
        x0, x1, x2, x3 = m.hinges[e]
        el = np.linalg.norm(X[x1] - X[x0])
        hA = np.linalg.norm(np.cross(X[x1] - X[x0], X[x2] - X[x0])) / el
        hB = np.linalg.norm(np.cross(X[x1] - X[x0], X[x3] - X[x0])) / el
        k2, k3 = -el / hA, -el / hB
        assert np.isclose(m.K[e, 2], k2, rtol=1e-12)
        assert np.isclose(m.K[e, 3], k3, rtol=1e-12)
        # solve for k0, k1 from sum = 0 and in-plane moment = 0 (x and z)
        A = np.array([[1, 1], [X[x0, 0], X[x1, 0]], [X[x0, 2], X[x1, 2]]])
        rhs = -np.array([k2 + k3, k2 * X[x2, 0] + k3 * X[x3, 0], k2 * X[x2, 2] + k3 * X[x3, 2]])
        k01 = np.linalg.lstsq(A, rhs, rcond=None)[0]
        assert np.allclose(m.K[e, :2], k01, rtol=1e-9)
    rng = np.random.default_rng(3)
    Aff = rng.standard_normal((3, 3))
    xa = X @ Aff.T + rng.standard_normal(3)
    s = np.einsum("ek,ekd->ed", m.K, xa[m.hinges])
    Eb = (m.w_hinge * (s * s).sum(1)).sum()
    scale = (m.w_hinge * (np.abs(m.K).sum(1) * np.abs(xa).max()) ** 2).sum()
    assert Eb <= 1e-24 * scale
    assert np.all(m.rest_bend == 0.0)


def test_system_matrix_invariants():
    sc, m = small(10)
    H = m.H
    assert abs(H - H.T).max() <= 1e-14 * abs(H).max()
    # constants: elastic part annihilates them, so H 1 = M/h^2 1
    one = np.ones(m.nv)
    assert np.allclose(H @ one, m.mass / m.h ** 2, rtol=1e-10, atol=1e-9 * m.diagH.max())
    w = np.linalg.eigvalsh(H.toarray())
    # elastic part is PSD and annihilates constants: min(m)/h^2 <= lambda_min <= mean(m)/h^2
    mh = m.mass / m.h ** 2
    assert mh.min() * (1 - 1e-12) <= w.min() <= mh.mean() * (1 + 1e-12)


def test_eigenbasis_library_special_case():
    """U^T H U is diagonal and equals numpy eigh's eigenvalues (FP64 U)."""
    sc, m = small(9)
    lam, U = M.eigenbasis(m, 6)
    free = ~m.pinned
    ref = np.linalg.eigvalsh(m.H.toarray()[np.ix_(free, free)])[:6]
    assert np.allclose(lam, ref, rtol=1e-10)
    L = M.reduced_matrix(m, U)
    assert np.allclose(L, np.diag(ref), atol=1e-9 * ref.max())
    assert np.allclose(U.T @ U, np.eye(6), atol=1e-12)
    assert np.all(U[m.pinned] == 0)
    # the sparse path (shift-invert) agrees with the dense path
    lam2, U2 = M.eigenbasis(m, 6, dense_limit=0)
    assert np.allclose(lam2, ref, rtol=1e-9)
    assert np.allclose(np.abs(U2.T @ U), np.eye(6), atol=1e-6)


def test_bf16_rounding_against_torch():
    import torch
    rng = np.random.default_rng(0)
    a = rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 4, 10000)
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(a), ref)
