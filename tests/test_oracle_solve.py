"""Pins of the oracle's PD iteration: closed forms, the direct-solve fixed
point, monotone PD energy, rest equilibrium, exact subspace cancellation,
Eq. (uu), the Chebyshev weights and the NDB weights/targets (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import scenegen
from oracle import model as M
from oracle import step as S


def make(n=10, k_s=160.0, k_b=3e-4, r=6, pinned=True, seed=0, gamma=0.9, iters=10, outer=1):
    sc = scenegen.hanging_cloth(n, seed=seed, r=r)
    pin = sc.pinned if pinned else np.zeros_like(sc.pinned)
    m = M.build_model(sc.tris, sc.rest, pin, sc.dt, sc.density, k_s, k_b, k_contact=100.0)
    lam, U = M.eigenbasis(m, r)
    rho = M.spectral_radius(m, U, gamma, 200) if (k_s > 0 or k_b > 0) else 0.5
    p = S.Params(iters_outer=outer, iters_inner=iters, cheb_rho=min(0.999 * rho, 0.999),
                 cheb_gamma=gamma, cheb_delay=3, self_contact=False)
    return sc, m, U, p


def test_free_fall_closed_form():
    """k_s = k_b = 0, no contact: x_n = x_0 + n h v_0 + h^2 g n(n+1)/2."""
    sc, m, U, p = make(8, k_s=0.0, k_b=0.0, pinned=False, gamma=1.0)
    o = S.Oracle(m, U, p, sc.gravity)
    rng = np.random.default_rng(0)
    x0 = sc.x0.astype(np.float64)
    v0 = rng.standard_normal(x0.shape) * 0.1
    o.set_state(x0, v0)
    h = sc.dt
    g = np.array(sc.gravity)
    for n in range(1, 6):
        o.step()
        ref = x0 + n * h * v0 + h * h * g * n * (n + 1) / 2
        assert np.allclose(o.x, ref, rtol=0, atol=1e-13)


def test_rest_state_stays_at_rest():
    sc, m, U, p = make(10)
    o = S.Oracle(m, U, p, (0.0, 0.0, 0.0))
    o.set_state(m.rest, np.zeros_like(m.rest))
    for _ in range(3):
        o.step()
    assert np.abs(o.x - m.rest).max() <= 1e-13


def test_global_iteration_converges_to_direct_solve():
    """(a) With b and W frozen, coarse correction + Chebyshev-Jacobi converges
    to the sparse direct solution of (H + diag W) x = b on the free rows."""
    sc, m, U, p = make(12, r=8, iters=400)
    o = S.Oracle(m, U, p, sc.gravity)
    rng = np.random.default_rng(2)
    W = np.where(rng.random(m.nv) < 0.2, rng.uniform(10, 1000, m.nv), 0.0)
    p.cheb_rho = 0.999 * M.spectral_radius(m, U, p.cheb_gamma, 200)
    o = S.Oracle(m, U, p, sc.gravity)
    xb = m.rest + 0.01 * rng.standard_normal(m.rest.shape)
    b = rng.standard_normal((m.nv, 3)) * m.diagH[:, None] * 0.01
    free = ~m.pinned
    Hp = (m.H + __import__("scipy.sparse", fromlist=["diags"]).diags(W)).tocsr()
    Hff = Hp[free][:, free]
    rhs = b[free] - Hp[free][:, ~free] @ xb[~free]
    ref = xb.copy()
    ref[free] = spla.spsolve(Hff.tocsc(), rhs)
    xk = xb.copy()
    xkm1 = xb.copy()
    for k in range(400):
        xk1 = o.iterate(xk, xkm1, k, S.Constraints(), None, None, frozen=(b, W))
        xkm1, xk = xk, xk1
    assert np.abs(xk - ref).max() <= 1e-10 * np.abs(ref).max()


def test_rank2_a_jacobi_converges_to_direct_solve_and_doubles_the_sweeps():
    """The rank-2 A-Jacobi variant (sec. 8.1, two Jacobi steps per
    iteration): with b and W frozen it converges to the sparse direct
    solution, and per iteration it reduces the error more than a single
    damped sweep does."""
    sc, m, U, p = make(12, r=8, iters=300)
    rng = np.random.default_rng(3)
    W = np.where(rng.random(m.nv) < 0.2, rng.uniform(10, 1000, m.nv), 0.0)
    b = rng.standard_normal((m.nv, 3)) * m.diagH[:, None] * 0.01
    xb = m.rest + 0.01 * rng.standard_normal(m.rest.shape)
    free = ~m.pinned
    Hp = (m.H + __import__("scipy.sparse", fromlist=["diags"]).diags(W)).tocsr()
    ref = xb.copy()
    ref[free] = spla.spsolve(Hp[free][:, free].tocsc(), b[free] - Hp[free][:, ~free] @ xb[~free])
    p.smoother = "ajacobi2"
    p.cheb_gamma = 0.6
    o = S.Oracle(m, U, p, sc.gravity)
    xk = xb.copy()
    for k in range(300):
        xk = o.iterate(xk, xk, k, S.Constraints(), None, None, frozen=(b, W))
    assert np.abs(xk - ref).max() <= 1e-10 * np.abs(ref).max()
    # per iteration it reduces the error more than one damped sweep with the
    # same subspace correction (omega = 1, no Chebyshev blend)
    p1 = S.Params(**{**p.__dict__, "smoother": "chebyshev", "cheb_rho": 0.0})
    one = S.Oracle(m, U, p1, sc.gravity)
    one.omega[:] = 1.0
    xa = xb.copy()
    xr = xb.copy()
    for k in range(20):
        xa = one.iterate(xa, xa, k, S.Constraints(), None, None, frozen=(b, W))
        xr = o.iterate(xr, xr, k, S.Constraints(), None, None, frozen=(b, W))
    ea, er = np.abs(xa - ref).max(), np.abs(xr - ref).max()
    assert er < 0.5 * ea


def _true_energy(m, x, z):
    """Implicit-Euler energy with exact distances to the constraint sets:
    rotations for triangles (via SVD), the flat target for hinges."""
    e = 0.5 * (m.mass[:, None] / m.h ** 2 * (x - z) ** 2).sum()
    F = np.einsum("tcd,tci->tdi", x[m.tris], m.g)
    s = np.linalg.svd(F, compute_uv=False)
    e += 0.5 * (m.w_tri * ((s - 1.0) ** 2).sum(1)).sum()
    sb = np.einsum("ek,ekd->ed", m.K, x[m.hinges])
    e += 0.5 * (m.w_hinge * (sb * sb).sum(1)).sum()
    return e


def test_pd_energy_monotone_with_exact_global_step():
    """(b) Local projection + exact global solve never increases the energy."""
    sc, m, U, p = make(10, k_b=1e-3)
    rng = np.random.default_rng(4)
    z = m.rest + 0.05 * rng.standard_normal(m.rest.shape)
    z[m.pinned] = m.rest[m.pinned]
    x = z.copy()
    free = ~m.pinned
    Hff = m.H[free][:, free].tocsc()
    lu = spla.splu(Hff)
    E = [_true_energy(m, x, z)]
    for it in range(15):
        b = (m.mass / m.h ** 2)[:, None] * z + S.elastic_rhs(m, x)
        rhs = b[free] - m.H[free][:, ~free] @ x[~free]
        x = x.copy()
        x[free] = lu.solve(rhs)
        E.append(_true_energy(m, x, z))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    assert E[-1] < E[0]


def test_polar_projection_matches_svd():
    rng = np.random.default_rng(5)
    F = rng.standard_normal((200, 3, 2))
    T = S.polar_3x2(F)
    u, s, vt = np.linalg.svd(F, full_matrices=False)
    ref = u @ vt
    assert np.allclose(T, ref, atol=1e-12)
    assert np.allclose(np.einsum("tdi,tdj->tij", T, T), np.eye(2), atol=1e-12)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    assert np.allclose(S.polar_3x2(Q[None] @ F), Q[None] @ T, atol=1e-12)
    O = np.linalg.qr(rng.standard_normal((50, 3, 2)))[0]
    assert np.allclose(S.polar_3x2(O), O, atol=1e-13)


def test_subspace_correction_cancels_residual_in_span():
    """(d) b := (H + diag W)(x + U q0): the coarse step alone gives x~ = x + U q0
    and r1 = 0, for any W."""
    sc, m, U, p = make(10, r=6)
    o = S.Oracle(m, U, p, sc.gravity)
    rng = np.random.default_rng(6)
    W = rng.uniform(0, 500, m.nv) * (rng.random(m.nv) < 0.3)
    x = m.rest + 0.01 * rng.standard_normal(m.rest.shape)
    q0 = rng.standard_normal((6, 3))
    target = x + U @ q0
    b = m.H @ target + W[:, None] * target
    o.iterate(x, x, 0, S.Constraints(), None, None, frozen=(b, W))
    tr = o.trace
    assert np.allclose(tr["xt"], target, atol=1e-12)
    assert np.abs(tr["r1"]).max() <= 1e-9 * np.abs(b).max()


def test_eq_uu_rank_one_sum():
    sc, m, U, p = make(9, r=5)
    rng = np.random.default_rng(7)
    W = rng.uniform(0, 10, m.nv) * (rng.random(m.nv) < 0.5)
    ref = np.zeros((5, 5))
    for j in range(m.nv):
        if W[j]:
            ref += W[j] * np.outer(U[j], U[j])
    assert np.allclose(U.T @ (W[:, None] * U), ref, atol=1e-13)


def test_chebyshev_weights_limit_and_start():
    rho = 0.95
    w = S.chebyshev_weights(300, rho, 3)
    assert np.all(w[:3] == 1.0)
    assert w[3] == 2.0 / (2.0 - rho * rho)
    assert np.isclose(w[-1], 2.0 / (1.0 + np.sqrt(1.0 - rho * rho)), rtol=1e-12)


def test_ndb_weight_exact_power_of_two():
    sc, m, U, p = make(8)
    o = S.Oracle(m, U, p, sc.gravity)
    a = np.arange(0, 21, dtype=np.int32)
    w = o._weights(a)
    assert np.array_equal(w, np.array([m.k_contact * 2.0 ** int(i) for i in a]))
    w32 = np.ldexp(np.float32(m.k_contact), a)
    assert np.array_equal(w32.astype(np.float64), np.float32(m.k_contact).astype(np.float64) * 2.0 ** a)


def test_half_space_target_is_minimum_norm_projection():
    rng = np.random.default_rng(8)
    P = 50
    ids = np.arange(4 * P).reshape(P, 4)
    x = rng.standard_normal((4 * P, 3))
    coef = rng.standard_normal((P, 4))
    nrm = rng.standard_normal((P, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mov = np.ones(4 * P)
    mov[::7] = 0.0
    W = np.zeros(4 * P)
    WY = np.zeros((4 * P, 3))
    dh = 0.3
    S.Oracle._half_space(ids, coef, nrm, np.ones(P), x, mov, dh, W, WY)
    y = WY  # unit weights: WY holds the targets
    gx = np.einsum("pk,pkd,pd->p", coef, x[ids], nrm) - dh
    gy = np.einsum("pk,pkd,pd->p", coef, y[ids], nrm) - dh
    viol = gx < 0
    assert np.allclose(gy[viol], 0, atol=1e-12)
    assert np.array_equal(y[ids][~viol], x[ids][~viol])
    assert np.array_equal(y[mov == 0], x[mov == 0])
    # no feasible point is closer: random feasible perturbations of the target
    for p_ in np.flatnonzero(viol)[:10]:
        d0 = np.linalg.norm(y[ids[p_]] - x[ids[p_]])
        for _ in range(200):
            cand = y[ids[p_]] + 0.05 * rng.standard_normal((4, 3)) * mov[ids[p_]][:, None]
            if np.einsum("k,kd,d->", coef[p_], cand, nrm[p_]) - dh >= 0:
                assert np.linalg.norm(cand - x[ids[p_]]) >= d0 - 1e-12
