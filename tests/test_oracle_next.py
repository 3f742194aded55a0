"""Pins of the oracle's modal warm start and residual forwarding (Algorithm 1
before the first full CCD and after the exiting filter; section 6)."""
import numpy as np
import scipy.linalg as sla

import scenegen
from oracle import model as M
from oracle import step as S


def linear_setup(n=10, r=8):
    sc = scenegen.hanging_cloth(n, seed=2, r=r)
    # k_stretch = 0: with a flat rest shape the local step adds nothing, b does not depend on x
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, 0.0, 1e-3, k_contact=50.0)
    lam, U = M.eigenbasis(m, r)
    return sc, m, lam, U


def test_warm_start_is_galerkin_solve_in_span():
    sc, m, lam, U = linear_setup()
    p = S.Params(1, 5, 0.9, 0.8, warm_iters=1, self_contact=False)
    o = S.Oracle(m, U, p, sc.gravity)
    rng = np.random.default_rng(0)
    z = m.rest + 0.01 * rng.standard_normal(m.rest.shape)
    z[m.pinned] = m.rest[m.pinned]
    inertia = (m.mass / m.h ** 2)[:, None] * z
    x1 = o.warm_start(z, inertia)
    b = inertia
    # closed form with the diagonal eigenvalue matrix (library eigenvalues)
    ref = z + U @ ((U.T @ (b - m.H @ z)) / lam[:, None])
    assert np.allclose(x1, ref, atol=1e-12)
    assert np.abs(U.T @ (b - m.H @ x1)).max() <= 1e-9 * np.abs(b).max()
    # Galerkin: x1 minimises the quadratic energy over z + span(U)
    def energy(x):
        return 0.5 * np.einsum("ij,ij->", x, m.H @ x) - np.einsum("ij,ij->", b, x)
    for _ in range(20):
        q = rng.standard_normal((U.shape[1], 3)) * 1e-3
        assert energy(x1) <= energy(x1 + U @ q) + 1e-12


def test_warm_start_converges_in_the_nonlinear_case():
    sc = scenegen.hanging_cloth(10, seed=2, r=8)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    _, U = M.eigenbasis(m, 8)
    o = S.Oracle(m, U, S.Params(1, 5, 0.9, 0.8, warm_iters=30, self_contact=False), sc.gravity)
    z = m.rest + np.array([0, -0.01, 0])
    z[m.pinned] = m.rest[m.pinned]
    inertia = (m.mass / m.h ** 2)[:, None] * z
    x = o.warm_start(z, inertia)
    r = inertia + S.elastic_rhs(m, x) - m.H @ x
    r[m.pinned] = 0
    assert np.abs(U.T @ r).max() <= 1e-8 * np.abs(inertia).max()


def test_forwarded_residual_enters_the_next_predictor():
    """k_s = k_b = 0, no contact: the step returns z exactly, so with a
    forwarded dx the next position is x + h v + h^2 g + 2 dx (Eq. (z_rf) with
    delta f = 2 M dx / h^2)."""
    sc = scenegen.hanging_cloth(8, seed=1, r=6)
    m = M.build_model(sc.tris, sc.rest, np.zeros(sc.nv, np.uint8), sc.dt, sc.density, 0.0, 0.0,
                      k_contact=10.0)
    _, U = M.eigenbasis(m, 6)
    o = S.Oracle(m, U, S.Params(1, 4, 0.5, 1.0, self_contact=False), sc.gravity)
    rng = np.random.default_rng(1)
    x0 = sc.x0.astype(np.float64)
    v0 = 0.1 * rng.standard_normal(x0.shape)
    o.set_state(x0, v0)
    dx = 1e-3 * rng.standard_normal(x0.shape)
    o.rf_dx = dx.copy()
    o.step()
    h = sc.dt
    assert np.allclose(o.x, x0 + h * v0 + h * h * np.array(sc.gravity) + 2 * dx, atol=1e-13)
    assert np.all(o.rf_dx == 0)


def test_residual_forwarding_uses_weight_k_and_no_filter():
    sc = scenegen.drop_cloth(14, seed=4, obstacle="sphere", r=6, steps=1, drop=0.001, d_hat=2e-3)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend,
                      k_contact=80.0)
    _, U = M.eigenbasis(m, 6)
    p = S.Params(1, 4, 0.95, 0.6, d_hat=sc.d_hat, rf_iters=3, rf_toi=1.5)
    obs = [S.Obst(0, np.array(o_.center), o_.radius, np.array(o_.axis)) for o_ in sc.obstacles]
    o = S.Oracle(m, U, p, sc.gravity, obs)
    x = sc.x0.astype(np.float64) - np.array([0, 0.0008, 0])
    v = np.array([[0, -0.5, 0.0]]) * np.ones_like(x)
    C = S.Constraints()
    verts = np.flatnonzero(S.obstacle_phi(obs[0], x)[0] < 5e-3).astype(np.int32)
    assert len(verts) > 0
    C.ob = np.stack([verts, np.zeros_like(verts)], 1)
    C.a_ob = np.full(len(verts), 7, np.int32)
    o._freeze(C, x)
    inertia = (m.mass / m.h ** 2)[:, None] * (x + m.h * v)
    dx = o.residual_forward(x, C, inertia)
    W = o.trace["W"]
    assert np.all(C.a_ob == 7)                       # the block's spans are untouched
    assert np.allclose(W[verts], m.k_contact)        # every collision weight is k
    assert np.all(dx[m.pinned] == 0) and np.abs(dx).max() > 0


def test_warm_start_uses_its_own_wider_basis():
    """The warm start takes its own basis (r_warm = 2 r modes): with the
    exact eigenvectors its Galerkin matrix is the diagonal of eigenvalues
    (library special case), one warm iteration is the closed-form modal
    solve in the wide span, and the correction leaves span(U) of the reuse
    basis."""
    sc, m, lam, U = linear_setup(r=8)
    lam_w, Uw = M.eigenbasis(m, 16)
    p = S.Params(1, 5, 0.9, 0.8, warm_iters=1, self_contact=False)
    o = S.Oracle(m, U, p, sc.gravity, Uw=Uw)
    assert np.allclose(o.Lw, np.diag(lam_w), atol=1e-9 * lam_w.max())
    rng = np.random.default_rng(4)
    z = m.rest + 0.01 * rng.standard_normal(m.rest.shape)
    z[m.pinned] = m.rest[m.pinned]
    inertia = (m.mass / m.h ** 2)[:, None] * z
    x1 = o.warm_start(z, inertia)
    ref = z + Uw @ ((Uw.T @ (inertia - m.H @ z)) / lam_w[:, None])
    assert np.allclose(x1, ref, atol=1e-12)
    d = x1 - z
    outside = d - U @ (U.T @ d)
    assert np.abs(outside).max() > 1e-3 * np.abs(d).max()
    # the default warm basis is the reuse basis
    o2 = S.Oracle(m, U, p, sc.gravity)
    x2 = o2.warm_start(z, inertia)
    assert np.allclose(x2 - z, U @ (U.T @ (x2 - z)), atol=1e-12)
