"""Pins of the oracle's loop conditions (Algorithm 1, section 7) and of its
strain-limited projection.

Loop conditions: a tolerance run is the fixed-budget run cut where the
condition first holds.  The inner loop stops after iteration K when the
change of iteration K-1 is below tol_inner, so a block run with that
tolerance equals the block run with a budget of K iterations; the outer loop
likewise equals the run with a budget of as many blocks.  A zero tolerance
is the fixed budget; a huge one leaves one iteration per block and one block
per step.

Strain limits: T = U clamp(Sigma) V^T is the nearest matrix with singular
values in [sigma_min, sigma_max] (checked against random feasible matrices),
keeps F when F is feasible, and is the rotation for limits (1, 1).
"""
import copy

import numpy as np

import scenegen
from oracle import model as M
from oracle import step as S


def make(iters_inner=10, iters_outer=3, tol_inner=0.0, tol_outer=0.0, n=10, seed=0):
    sc = scenegen.hanging_cloth(n, seed=seed, r=6)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    _, U = M.eigenbasis(m, sc.r)
    p = S.Params(iters_outer=iters_outer, iters_inner=iters_inner, cheb_rho=0.9, cheb_gamma=0.8, cheb_delay=3,
                 self_contact=False, tol_inner=tol_inner, tol_outer=tol_outer)
    o = S.Oracle(m, U, p, sc.gravity)
    v0 = np.tile(np.array([0.3, -1.0, 0.2]), (sc.nv, 1))
    v0[sc.pinned.astype(bool)] = 0
    o.set_state(sc.x0, v0)
    return o


def test_zero_tolerances_are_the_fixed_budget():
    a = make()
    b = make(tol_inner=0.0, tol_outer=0.0)
    for _ in range(2):
        sa, sb = a.step(), b.step()
        assert np.array_equal(a.x, b.x)
        assert sa.inner_iters == 30 and sa.outer_iters == 3 and sb.dx == sa.dx


def test_huge_tolerances_leave_one_iteration_per_block_and_one_block():
    o = make(tol_inner=1e9)
    st = o.step()
    assert st.inner_iters == 3 and st.outer_iters == 3
    o = make(tol_outer=1e9)
    st = o.step()
    assert st.outer_iters == 1 and st.inner_iters == 10
    ref = make(iters_outer=1)
    ref.step()
    assert np.array_equal(o.x, ref.x)


def test_inner_condition_equals_the_cut_budget():
    """With one block, tol_inner between consecutive changes stops the block
    exactly where the fixed run first falls below it."""
    full = make(iters_inner=12, iters_outer=1)
    st = full.step()
    dx = np.array(st.dx)
    for K in range(2, 11):
        tol = dx[K - 1] * 1.0001
        if not (dx[:K - 1] >= tol).all():
            continue   # an earlier change is below it already
        o = make(iters_inner=12, iters_outer=1, tol_inner=tol)
        so = o.step()
        assert so.inner_iters == K
        cut = make(iters_inner=K, iters_outer=1)
        cut.step()
        assert np.array_equal(o.x, cut.x), K


def test_outer_condition_equals_the_cut_budget():
    full = make(iters_inner=5, iters_outer=4)
    st = full.step()
    odx = np.array(st.outer_dx)
    assert len(odx) == 4 and (np.diff(odx) < 0).all()
    for B in (1, 2, 3):
        tol = odx[B - 1] * 1.0001
        o = make(iters_inner=5, iters_outer=4, tol_outer=tol)
        so = o.step()
        assert so.outer_iters == B and so.inner_iters == 5 * B
        cut = make(iters_inner=5, iters_outer=B)
        cut.step()
        assert np.array_equal(o.x, cut.x), B


def test_outer_change_is_the_change_of_x_over_the_block():
    o = make(iters_inner=4, iters_outer=2)
    x_before = o.x.copy()
    # run the same step by hand with one block, then compare the first norm
    one = make(iters_inner=4, iters_outer=1)
    one.step()
    st = o.step()
    # block 1 ends where the one-block run ends; its change is measured from
    # the filtered start of the block (the initial filter keeps z here)
    h = o.m.h
    v0 = np.tile(np.array([0.3, -1.0, 0.2]), (o.m.nv, 1))
    v0[o.m.pinned] = 0
    z = x_before + h * v0 + h * h * o.g
    z[o.m.pinned] = x_before[o.m.pinned]
    want = np.linalg.norm(one.x - z, axis=1).max()
    assert np.isclose(st.outer_dx[0], want, rtol=1e-12, atol=0)


# ------------------------------------------------------------ strain limits

def test_strain_limited_projection_is_the_nearest_feasible_matrix():
    rng = np.random.default_rng(31)
    F = rng.standard_normal((200, 3, 2)) * rng.uniform(0.5, 1.5, (200, 1, 1))
    for smin, smax in ((0.9, 1.1), (0.8, 1.0), (1.0, 1.3)):
        T = S.strain_limited_3x2(F, smin, smax)
        sv = np.linalg.svd(T, compute_uv=False)
        assert (sv >= smin - 1e-12).all() and (sv <= smax + 1e-12).all()
        d0 = np.linalg.norm(T - F, axis=(1, 2))
        for t in range(0, 200, 20):
            for _ in range(100):
                # a random feasible matrix near T
                Q, _ = np.linalg.qr(rng.standard_normal((3, 2)))
                R, _ = np.linalg.qr(rng.standard_normal((2, 2)))
                cand = T[t] + 0.3 * (Q @ np.diag(rng.uniform(smin, smax, 2)) @ R - T[t])
                svc = np.linalg.svd(cand, compute_uv=False)
                if (svc >= smin).all() and (svc <= smax).all():
                    assert np.linalg.norm(cand - F[t]) >= d0[t] - 1e-12


def test_strain_limited_projection_special_cases():
    rng = np.random.default_rng(32)
    F = rng.standard_normal((100, 3, 2))
    # limits (1, 1): the polar factor
    assert np.allclose(S.strain_limited_3x2(F, 1.0, 1.0), S.polar_3x2(F), atol=1e-12)
    # feasible F is kept
    Q, _ = np.linalg.qr(rng.standard_normal((3, 2)))
    R, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    G = Q @ np.diag([0.95, 1.04]) @ R
    assert np.allclose(S.strain_limited_3x2(G[None], 0.9, 1.1)[0], G, atol=1e-14)
    # rotation equivariance
    Rot, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    T = S.strain_limited_3x2(F, 0.9, 1.1)
    assert np.allclose(S.strain_limited_3x2(np.einsum("ij,tjk->tik", Rot, F), 0.9, 1.1),
                       np.einsum("ij,tjk->tik", Rot, T), atol=1e-12)


def test_strain_limited_step_moves_less_than_the_rigid_projection_allows():
    """A stretched cloth relaxes less toward rest when strains within
    [sigma_min, sigma_max] cost nothing: with limits the elastic right-hand
    side of a uniformly stretched rest state (stretch inside the range) is
    the one of an undeformed state, zero in the interior."""
    sc = scenegen.hanging_cloth(8, seed=1, r=6)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend,
                      sigma_min=0.9, sigma_max=1.1)
    x = sc.rest.astype(np.float64) * 1.05
    rhs = S.elastic_rhs(m, x)
    # with the stretch inside the limits each triangle's target is F itself,
    # so sum_t w_t G_t^T T_t^T = sum_t w_t G_t^T F_t^T = (H_elastic x) rows
    m1 = copy.copy(m)
    m1.sigma_min = m1.sigma_max = 1.0
    rhs1 = S.elastic_rhs(m1, x)
    Hel = m.H - np.diag(m.mass / m.h ** 2)
    assert np.allclose(rhs, np.asarray(Hel @ x) - _bending(m, x), atol=1e-9)
    assert np.abs(rhs - rhs1).max() > 1e-3


def _bending(m, x):
    out = np.zeros_like(x)
    kx = np.einsum("ek,ekd->ed", m.K, x[m.hinges])
    np.add.at(out, m.hinges.ravel(), (m.w_hinge[:, None, None] * m.K[:, :, None] * kx[:, None, :]).reshape(-1, 3))
    return out
