"""Pins of the oracle's variants of the method: the lagged obstacle friction
(section 8.4 drapes with a lagged friction Hessian; the model is the
smoothed Coulomb law documented in oracle.step.obstacle_friction) and the
partial-CCD sample density adapted to the change of rho* (end of section
4.1).  CPU only."""
import numpy as np

import scenegen
from oracle import model as M
from oracle import step as S


def _band_points(rng, ob, n, d_hat):
    """Points in the contact band of a sphere (signed distance in [-d, d))."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    dist = rng.uniform(-d_hat, d_hat, n)
    return ob.center + d * (ob.radius + dist)[:, None], d, dist


def test_friction_force_follows_the_smoothed_coulomb_law():
    """Force wf |u_T| equals mu lambda while slipping (|u_T| >= eps), stays
    below it while sticking and vanishes with the slip; u_T is tangent; the
    law is continuous at eps; no friction outside the band or with mu = 0."""
    rng = np.random.default_rng(0)
    ob = S.Obst(0, np.array([0.1, -0.2, 0.3]), 0.25, np.array([1.0, 0.0, 0.0]))
    h, dh, mu, ev = 1 / 200, 1e-3, 0.4, 1e-3
    eps = ev * h
    x, n, dist = _band_points(rng, ob, 400, dh)
    w = rng.uniform(1.0, 1e4, 400)
    slip = rng.normal(size=(400, 3)) * np.exp(rng.uniform(np.log(1e-9), np.log(1e-3), 400))[:, None]
    xs = x - slip
    wf, uT = S.obstacle_friction(ob, x, xs, w, h, dh, mu, ev)
    lam = w * (dh - dist)                       # w (R + d_hat - |x - c|)
    assert np.all(lam > 0)
    assert np.allclose(np.sum(uT * n, axis=1), 0.0, atol=1e-15)
    y = np.linalg.norm(uT, axis=1)
    force = wf * y
    slipping = y >= eps
    assert slipping.sum() > 50 and (~slipping).sum() > 50
    assert np.allclose(force[slipping], mu * lam[slipping], rtol=1e-12)
    assert np.all(force[~slipping] <= mu * lam[~slipping] * (1 + 1e-12))
    tiny = y < 1e-3 * eps
    assert tiny.any() and np.allclose(wf[tiny], 2 * mu * lam[tiny] / eps, rtol=2e-3)
    # continuity of the law at eps: one point just below, one just above
    t = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    top = ob.center + np.array([[0.0, ob.radius, 0.0], [0.0, ob.radius, 0.0]])
    wf2, _ = S.obstacle_friction(ob, top, top - t * np.array([[eps * (1 - 1e-9)], [eps * (1 + 1e-9)]]),
                                 np.ones(2), h, dh, mu, ev)
    assert abs(wf2[0] * eps - wf2[1] * eps) < 1e-6 * mu * dh
    # outside the band, or without friction: nothing
    far = ob.center + n * (ob.radius + 2 * dh)
    assert not S.obstacle_friction(ob, far, far - slip, w, h, dh, mu, ev)[0].any()
    assert not S.obstacle_friction(ob, x, xs, w, h, dh, 0.0, ev)[0].any()


def test_spinning_cylinder_pulls_a_resting_vertex_along_its_surface():
    """A vertex resting on top of a cylinder (axis +x) spinning at omega > 0
    sees the surface move along +z (omega R (axis x n), n = +y), so its slip
    relative to the surface is along -z and the friction target x - u_T lies
    on the +z side; with the spin reversed it is on the -z side."""
    h, dh = 1 / 200, 1e-3
    for om, sign in ((2.0, 1.0), (-2.0, -1.0)):
        ob = S.Obst(1, np.zeros(3), 0.2, np.array([1.0, 0.0, 0.0]), omega=om)
        x = np.array([[0.05, 0.2 + 0.5 * dh, 0.0]])
        wf, uT = S.obstacle_friction(ob, x, x.copy(), np.array([100.0]), h, dh, 0.5, 1e-3)
        assert wf[0] > 0
        target = x - uT
        assert np.sign(target[0, 2] - x[0, 2]) == sign
        assert np.allclose(uT[0], [0.0, 0.0, -om * 0.2 * h], rtol=1e-12, atol=1e-18)


def _cloth_on(obstacle, omega, v0, mu, steps, n=9):
    """A small flat cloth laid just above the top of an obstacle (inside the
    contact band), with an initial velocity, stepped by the oracle."""
    sc = scenegen.drop_cloth(n, seed=2, obstacle=obstacle, r=8, steps=steps, drop=0.0, d_hat=1e-3,
                             side=0.05, iters_outer=2, iters_inner=6)
    ob0 = sc.obstacles[0]
    x0 = sc.rest.astype(np.float64).copy()
    x0[:, 1] = ob0.radius + 0.5e-3          # flat, half d_hat above the top line
    # on a cylinder the flat sheet leaves the band away from the top line,
    # so keep the sheet narrow across the axis
    m = M.build_model(sc.tris, x0, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    _, U = M.eigenbasis(m, sc.r)
    p = S.Params(iters_outer=2, iters_inner=6, cheb_rho=0.9, cheb_gamma=0.6, d_hat=sc.d_hat,
                 self_contact=False, friction=mu)
    ob = S.Obst(ob0.kind, np.array(ob0.center, float), ob0.radius, np.array(ob0.axis, float), omega=omega)
    o = S.Oracle(m, U, p, sc.gravity, [ob])
    o.set_state(x0, np.tile(np.asarray(v0, float), (sc.nv, 1)))
    for _ in range(steps):
        o.step()
    return o


def test_friction_slows_a_sliding_cloth_and_a_spinning_cylinder_drags_one():
    """Oracle steps: a cloth sliding over a sphere's top at 0.3 m/s keeps
    less of its speed with friction than without; a cloth resting on a
    cylinder spinning at 2 rad/s picks up velocity along the surface motion
    (+z at the top) with friction and none without."""
    free = _cloth_on("sphere", 0.0, (0.3, 0.0, 0.0), 0.0, 4)
    fric = _cloth_on("sphere", 0.0, (0.3, 0.0, 0.0), 0.6, 4)
    assert fric.v[:, 0].mean() < free.v[:, 0].mean() - 0.02
    still = _cloth_on("cylinder", 2.0, (0.0, 0.0, 0.0), 0.0, 4)
    drag = _cloth_on("cylinder", 2.0, (0.0, 0.0, 0.0), 0.6, 4)
    assert abs(still.v[:, 2].mean()) < 1e-6
    assert drag.v[:, 2].mean() > 0.01


def _cover_radius(smp, vt, grid=120):
    """Largest distance from a point of the parameter domain to its nearest
    sample (the sample interval of the set), by brute force on a grid."""
    g = (np.arange(grid) + 0.5) / grid
    P = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    if vt:
        P = P[P.sum(1) <= 1.0]
    d = np.linalg.norm(P[:, None, :] - smp[None, :, :], axis=2).min(1)
    return d.max()


def test_refined_sample_sets_cover_the_domain_at_an_interval_shrinking_like_1_over_m():
    """Adaptive partial-CCD density (end of section 4.1): the refined set of
    level m has m^2 points inside the parameter domain (barycentric triangle
    for VT, unit square for EE), and its sample interval scales like 1/m."""
    for vt in (True, False):
        base = S.refined_samples(S.ADAPT_M0, vt)
        r0 = _cover_radius(base, vt)
        for m in (3, 4, 6, 8):
            smp = S.refined_samples(m, vt)
            assert len(smp) == m * m and len(np.unique(np.round(smp, 12), axis=0)) == m * m
            assert np.all(smp > 0) and np.all(smp < 1)
            if vt:
                assert np.all(smp.sum(1) < 1)
            r = _cover_radius(smp, vt)
            assert r <= r0 * S.ADAPT_M0 / m * 1.15 + 2e-2 and r >= r0 * S.ADAPT_M0 / m * 0.6


def test_rho_star_ratio_is_one_at_rest_and_falls_with_stretch_and_motion():
    """rho* of Eq. (sample_bound) changes with the longest edge L and the
    largest point distance H1: the ratio is 1 without motion, at most 1 for
    any motion, and falls monotonically as a triangle is stretched or the
    vertex moves farther; the level rises as the ratio falls."""
    rng = np.random.default_rng(1)
    for vt in (True, False):
        q0 = rng.normal(size=(300, 4, 3))
        q1 = q0 + rng.normal(scale=0.3, size=q0.shape)
        assert np.allclose(S.rho_star_ratio(q0, q0.copy(), vt), 1.0)
        r = S.rho_star_ratio(q0, q1, vt)
        assert np.all(r > 0) and np.all(r <= 1.0)
    tri = np.array([[0.3, 0.3, 0.01], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    prev = 1.0
    for s in (1.0, 1.5, 2.0, 4.0):                  # stretch the triangle about its corner
        q1 = tri.copy()
        q1[1:] = tri[1:] * s
        r = S.rho_star_ratio(tri[None], q1[None], True)[0]
        assert r <= prev
        prev = r
    levels = []
    for dz in (0.0, 0.5, 2.0, 8.0, 40.0):          # move the vertex farther through the plane
        q1 = tri.copy()
        q1[0, 2] -= dz
        levels.append(int(S.adaptive_level(S.rho_star_ratio(tri[None], q1[None], True))[0]))
    assert levels[0] == S.ADAPT_M0 and levels == sorted(levels) and levels[-1] == S.ADAPT_MMAX
