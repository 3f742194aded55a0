"""Pins of oracle functions that the collision side and the Chebyshev set-up
rest on, each against something other than the oracle itself:

  * closest points (og_frozen_vt / og_frozen_ee): a bounded least-squares
    library solve and a dense parameter grid, in the face, edge and vertex
    regions, with parallel and zero-length segments;
  * the life-span rule of Oracle._partial_ccd: constructed collisions whose
    outcome is fixed by Eq. (collision_judge), separating motions whose Q is
    positive by construction, an exact tie, the cap a_max and the obstacle
    branch;
  * the constraint-set carry-over (_merge, _outer_ccd): hand-built previous
    and candidate sets and a brute-force set computation;
  * query_ee: Eq. (collision_judge) for edge-edge collisions;
  * collision targets: the obstacle target on the offset surface along the
    radial line, and half-space targets of penetrating VT / EE pairs that
    sit exactly d_hat apart along the frozen normal;
  * spectral_radius: the dense spectrum of the error operator.
"""
import types

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize

from oracle import model as M
from oracle import native
from oracle import step as S


# ----------------------------------------------------------------- helpers

def bare_oracle(tris, edges, nv, pinned=None, d_hat=1e-2, obs=(), a_max=20, k_contact=1.0):
    """An Oracle whose mesh data are given directly (no system matrix): only
    the per-constraint methods are called on it."""
    o = object.__new__(S.Oracle)
    o.m = types.SimpleNamespace(tris=np.asarray(tris, np.int32).reshape(-1, 3),
                                edges=np.asarray(edges, np.int32).reshape(-1, 2), nv=nv,
                                k_contact=k_contact)
    o.p = S.Params(iters_outer=1, iters_inner=1, cheb_rho=0.5, d_hat=d_hat, a_max=a_max)
    o.obs = list(obs)
    o.free = np.ones(nv, bool) if pinned is None else ~np.asarray(pinned, bool)
    return o


def tri_point(P, lam):
    return P[0] + lam[0] * (P[1] - P[0]) + lam[1] * (P[2] - P[0])


def brute_tri(p, a, b, c):
    """Closest point of the closed triangle to p by (i) SLSQP on the
    barycentric simplex and (ii) a 401 x 401 parameter grid refined around
    its best point; returns (params of the best, its distance)."""
    E = np.stack([b - a, c - a], 1)

    def f(l):
        d = a + E @ l - p
        return d @ d

    res = minimize(f, np.array([1 / 3, 1 / 3]), method="SLSQP", jac=lambda l: 2 * E.T @ (a + E @ l - p),
                   bounds=[(0, 1), (0, 1)], constraints=[{"type": "ineq", "fun": lambda l: 1 - l[0] - l[1],
                                                          "jac": lambda l: np.array([-1.0, -1.0])}],
                   options={"ftol": 1e-16, "maxiter": 500})
    best = [(f(np.clip(res.x, 0, 1)), np.clip(res.x, 0, 1))] if res.x.sum() <= 1 + 1e-12 else []
    g = np.linspace(0, 1, 401)
    L1, L2 = np.meshgrid(g, g, indexing="ij")
    m = L1 + L2 <= 1 + 1e-15
    ll = np.stack([L1[m], L2[m]], 1)
    d = ((a + ll @ E.T - p) ** 2).sum(1)
    l0 = ll[np.argmin(d)]
    h = 2.0 / 400
    g1 = np.linspace(max(l0[0] - h, 0), min(l0[0] + h, 1), 401)
    g2 = np.linspace(max(l0[1] - h, 0), min(l0[1] + h, 1), 401)
    L1, L2 = np.meshgrid(g1, g2, indexing="ij")
    m = L1 + L2 <= 1 + 1e-15
    ll = np.stack([L1[m], L2[m]], 1)
    d = ((a + ll @ E.T - p) ** 2).sum(1)
    best.append((d.min(), ll[np.argmin(d)]))
    dmin, lbest = min(best, key=lambda z: z[0])
    return lbest, np.sqrt(dmin)


def brute_seg(p1, p2, p3, p4):
    """Closest parameters of two segments: bounded least squares (BVLS) of
    [d1, -d2] (s, t) = p3 - p1 over the unit square, and the distance."""
    A = np.stack([p2 - p1, -(p4 - p3)], 1)
    res = lsq_linear(A, p3 - p1, bounds=(0, 1), method="bvls", tol=1e-15)
    s, t = res.x
    return (s, t), np.linalg.norm(p1 + s * (p2 - p1) - p3 - t * (p4 - p3))


def rand_tri(rng):
    while True:
        P = rng.standard_normal((3, 3))
        n = np.cross(P[1] - P[0], P[2] - P[0])
        if np.linalg.norm(n) > 0.3:
            return P


# ---------------------------------------------------------- closest points

def _vt_cases(rng):
    """Points in each Voronoi region of random triangles: face (above/below),
    the three edges, the three corners, and in-plane points."""
    cases = []
    for _ in range(12):
        P = rand_tri(rng)
        a, b, c = P
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        h = rng.uniform(-0.7, 0.7)
        lam = rng.dirichlet([2, 2, 2])[1:]
        cases.append((P, tri_point(P, lam) + h * n, "face"))
        for (i, j, k) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            e = P[j] - P[i]
            mid = P[i] + rng.uniform(0.2, 0.8) * e
            out = np.cross(e, n)
            if out @ (P[k] - P[i]) > 0:
                out = -out
            out /= np.linalg.norm(out)
            cases.append((P, mid + rng.uniform(0.05, 1.0) * out + h * n, "edge"))
            # corner region: beyond the vertex, away from both incident edges
            away = 2 * P[i] - 0.5 * (P[j] + P[k])
            cases.append((P, away + h * n, "corner"))
        cases.append((P, tri_point(P, rng.uniform(-0.5, 1.2, 2)), "plane"))
    return cases


def test_closest_point_on_triangle_against_bounded_least_squares():
    rng = np.random.default_rng(11)
    regions = {"face": 0, "edge": 0, "corner": 0, "plane": 0}
    for P, p, kind in _vt_cases(rng):
        xm = np.vstack([p, P])
        lam, nrm = native.frozen_vt(xm, np.array([[1, 2, 3]]), np.array([[0, 0]]))
        l1, l2 = lam[0]
        assert l1 >= 0 and l2 >= 0 and l1 + l2 <= 1 + 1e-15
        q = tri_point(P, lam[0])
        d = np.linalg.norm(q - p)
        lb, db = brute_tri(p, *P)
        scale = 1.0 + np.abs(P).max() + np.abs(p).max()
        # optimal: no sampled point of the triangle is closer, and it agrees
        # with the library solve (the minimiser of a point-to-triangle
        # distance is unique)
        assert d <= db + 1e-12 * scale, (kind, d, db)
        assert d >= db - 1e-6 * scale, (kind, d, db)
        assert np.allclose(lam[0], lb, atol=2e-5), (kind, lam[0], lb)
        # normal: unit, orthogonal to the triangle, on the vertex side
        n = nrm[0]
        assert abs(np.linalg.norm(n) - 1) < 1e-14
        assert abs(n @ (P[1] - P[0])) < 1e-12 and abs(n @ (P[2] - P[0])) < 1e-12
        assert n @ (p - P[0]) >= -1e-14
        regions[kind] += 1
    # which region the parameters fell in (vertex / edge / interior)
    assert all(v > 0 for v in regions.values())


def test_closest_point_regions_are_reached():
    """Parameters land on the corners, on each edge and inside, as the
    constructed points demand."""
    P = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    pts = {
        (0.0, 0.0): [-1.0, 0.3, -1.0],     # beyond corner a
        (1.0, 0.0): [3.0, -0.2, -0.5],     # beyond corner b
        (0.0, 1.0): [-0.5, 0.1, 3.0],      # beyond corner c
        (0.25, 0.0): [0.5, 0.4, -1.0],     # edge ab
        (0.0, 0.75): [-1.0, -0.3, 1.5],    # edge ac
        (0.5, 0.5): [1.5, 0.2, 1.5],       # edge bc (x + z = 2 at the foot)
        (0.25, 0.25): [0.5, 0.7, 0.5],     # face
    }
    for want, p in pts.items():
        xm = np.vstack([np.array(p), P])
        lam, nrm = native.frozen_vt(xm, np.array([[1, 2, 3]]), np.array([[0, 0]]))
        assert np.allclose(lam[0], want, atol=1e-15), (want, lam[0])
        assert np.allclose(np.abs(nrm[0]), [0, 1, 0])
        assert np.sign(nrm[0][1]) == (np.sign(p[1]) if p[1] != 0 else 1)


def test_vertex_in_triangle_plane_keeps_positive_normal():
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    xm = np.vstack([np.array([0.2, 0.0, 0.2]), P])
    lam, nrm = native.frozen_vt(xm, np.array([[1, 2, 3]]), np.array([[0, 0]]))
    n = np.cross(P[1] - P[0], P[2] - P[0])
    assert np.allclose(nrm[0], n / np.linalg.norm(n))
    assert np.allclose(lam[0], [0.2, 0.2])


def _ee_frozen(p1, p2, p3, p4):
    xm = np.vstack([p1, p2, p3, p4])
    lam, nrm = native.frozen_ee(xm, np.array([[0, 1], [2, 3]]), np.array([[0, 1]]))
    return lam[0], nrm[0]


def test_closest_points_of_segments_against_bounded_least_squares():
    rng = np.random.default_rng(12)
    interior = clamped = 0
    for i in range(300):
        p1, p2, p3, p4 = rng.standard_normal((4, 3))
        if i % 3 == 0:   # shorter second edge: more clamped cases
            p4 = p3 + 0.2 * (p4 - p3)
        (s, t), n = _ee_frozen(p1, p2, p3, p4)
        assert 0 <= s <= 1 and 0 <= t <= 1
        q1, q2 = p1 + s * (p2 - p1), p3 + t * (p4 - p3)
        d = np.linalg.norm(q2 - q1)
        (sb, tb), db = brute_seg(p1, p2, p3, p4)
        assert d <= db + 1e-12 and d >= db - 1e-12, (d, db)
        assert np.allclose([s, t], [sb, tb], atol=1e-9), ([s, t], [sb, tb])
        assert np.allclose(n, (q2 - q1) / d, atol=1e-12)
        if 0 < s < 1 and 0 < t < 1:
            interior += 1
        else:
            clamped += 1
    assert interior > 20 and clamped > 20


def test_closest_points_of_parallel_and_degenerate_segments():
    rng = np.random.default_rng(13)
    for _ in range(100):
        p1 = rng.standard_normal(3)
        d = rng.standard_normal(3)
        off = rng.standard_normal(3)
        off -= (off @ d) / (d @ d) * d
        a0, a1, b0, b1 = np.sort(rng.uniform(-1, 2, 4))[[0, 2, 1, 3]] if rng.random() < 0.5 else \
            rng.uniform(-1, 2, 4)
        # parallel: the minimiser is not unique, the distance is
        p2 = p1 + d
        p3 = p1 + b0 * d + off
        p4 = p1 + b1 * d + off
        if abs(b1 - b0) < 1e-3:
            continue
        (s, t), n = _ee_frozen(p1, p2, p3, p4)
        assert 0 <= s <= 1 and 0 <= t <= 1
        q1, q2 = p1 + s * (p2 - p1), p3 + t * (p4 - p3)
        _, db = brute_seg(p1, p2, p3, p4)
        assert abs(np.linalg.norm(q2 - q1) - db) < 1e-12
        assert np.allclose(n, (q2 - q1) / np.linalg.norm(q2 - q1), atol=1e-12)
    # zero-length first / second / both segments
    p = rng.standard_normal((4, 3))
    for a, b, c, e in ((p[0], p[0], p[2], p[3]), (p[0], p[1], p[2], p[2]), (p[0], p[0], p[2], p[2])):
        (s, t), n = _ee_frozen(a, b, c, e)
        q1, q2 = a + s * (b - a), c + t * (e - c)
        _, db = brute_seg(a, b, c, e)
        assert abs(np.linalg.norm(q2 - q1) - db) < 1e-12
        assert abs(np.linalg.norm(n) - 1) < 1e-14


def test_crossing_segments_fall_back_to_edge_cross_normal():
    p1, p2 = np.array([-1.0, 0, 0]), np.array([1.0, 0, 0])
    p3, p4 = np.array([0.0, 0, -1]), np.array([0.0, 0, 1])
    (s, t), n = _ee_frozen(p1, p2, p3, p4)
    assert (s, t) == (0.5, 0.5)
    assert np.allclose(np.abs(n), [0, 1, 0])
    # collinear overlapping segments: no distance direction, no cross product
    (s, t), n = _ee_frozen(p1, p2, np.array([0.0, 0, 0]), np.array([2.0, 0, 0]))
    assert np.allclose(n, [0, 1, 0])


# ------------------------------------------------------- query_ee identity

def ee_collision(rng, t_star):
    """Edges (p1,p2), (p3,p4) whose points at parameters (l1*, l2*) meet at
    time t*; rows at t=0 and t=1."""
    P0 = rng.standard_normal((4, 3))
    P1 = P0 + 0.4 * rng.standard_normal((4, 3))
    l1, l2 = rng.uniform(0.05, 0.95, 2)
    at = lambda i: P0[i] + t_star * (P1[i] - P0[i])
    m = at(0) + l1 * (at(1) - at(0))
    p3_star = (m - l2 * at(3)) / (1 - l2)
    P1[2] = P0[2] + (p3_star - P0[2]) / t_star
    return P0, P1, np.array([l1, l2])


def test_query_ee_identity_collision_judge():
    """Q(lambda*) = ((t*-1)/t*) |p2^0(l2*) - p1^0(l1*)|^2 for constructed EE
    collisions (Eq. (collision_judge) with the EE parametrisation)."""
    rng = np.random.default_rng(14)
    for _ in range(60):
        t_star = rng.uniform(0.05, 1.0)
        P0, P1, lam = ee_collision(rng, t_star)
        # the construction meets at t*
        at = lambda i: P0[i] + t_star * (P1[i] - P0[i])
        assert np.allclose(at(0) + lam[0] * (at(1) - at(0)), at(2) + lam[1] * (at(3) - at(2)), atol=1e-10)
        Q = S.query_ee(P0, P1, np.array([[0, 1]]), np.array([[2, 3]]), lam[None, None, :])[0, 0]
        d0 = P0[2] + lam[1] * (P0[3] - P0[2]) - P0[0] - lam[0] * (P0[1] - P0[0])
        ref = (t_star - 1) / t_star * (d0 @ d0)
        assert np.isclose(Q, ref, rtol=1e-8, atol=1e-12)
        # and the distance at the other parameters of the same pair is not
        # what Q measures: swapping the two parameters changes Q
        if abs(lam[0] - lam[1]) > 0.1:
            Qs = S.query_ee(P0, P1, np.array([[0, 1]]), np.array([[2, 3]]), lam[None, None, ::-1])[0, 0]
            assert not np.isclose(Qs, ref, rtol=1e-6)


def test_query_ee_separating_edges_positive():
    """Edges that translate apart along a common normal keep Q > 0 at every
    parameter pair."""
    rng = np.random.default_rng(15)
    g = np.linspace(0, 1, 11)
    lam = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(1, -1, 2)
    for _ in range(30):
        P0 = rng.standard_normal((4, 3))
        P0[:2, 1] = 0.0
        P0[2:, 1] = rng.uniform(0.1, 1.0)
        P1 = P0.copy()
        P1[2:, 1] += rng.uniform(0.1, 1.0)
        Q = S.query_ee(P0, P1, np.array([[0, 1]]), np.array([[2, 3]]), lam)
        assert (Q > 0).all()


# -------------------------------------------------------- life-span rule

def vt_collision(rng, t_star, lam=None):
    """Vertex (row 0) meeting the triangle (rows 1-3) at barycentric lam at t*."""
    tri0 = rand_tri(rng)
    tri1 = tri0 + 0.3 * rng.standard_normal((3, 3))
    lam = rng.dirichlet([1, 1, 1])[1:] if lam is None else np.asarray(lam, float)
    q = tri_point(tri0 + t_star * (tri1 - tri0), lam)
    d = rng.standard_normal(3)
    p0 = q - t_star * d
    return np.vstack([p0, tri0]), np.vstack([p0 + d, tri1]), lam


def vt_separating(rng):
    """Static triangle, vertex above it moving straight away: Q > 0 for all
    parameters (Q = |d0|^2 + h0 (h1 - h0) along the normal)."""
    tri = rand_tri(rng)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    p0 = tri_point(tri, rng.dirichlet([1, 1, 1])[1:]) + 0.3 * n + 0.2 * rng.standard_normal(3)
    p0 += (0.3 - (p0 - tri[0]) @ n) * n
    return np.vstack([p0, tri]), np.vstack([p0 + 0.5 * n, tri])


def test_partial_ccd_life_span_rule_vt_and_ee():
    """a <- active ? min(a + 1, a_max) : 0 with active iff some sample has
    Q <= 0: constructed collisions (active by Eq. (collision_judge) at the
    frozen parameters), separating motions (inactive), an exact tie Q = 0
    (active), and the cap."""
    rng = np.random.default_rng(16)
    a_max = 20
    X0, X1, tris, vt, lam_vt, a_vt, want_vt = [], [], [], [], [], [], []

    def add_vt(P0, P1, lam, a, want):
        base = 4 * len(vt)
        X0.append(P0)
        X1.append(P1)
        tris.append([base + 1, base + 2, base + 3])
        vt.append([base, len(tris) - 1])
        lam_vt.append(lam)
        a_vt.append(a)
        want_vt.append(want)

    for a in (0, 5, a_max - 1, a_max):
        P0, P1, lam = vt_collision(rng, rng.uniform(0.1, 0.95))
        add_vt(P0, P1, lam, a, min(a + 1, a_max))
    for a in (0, 7, a_max):
        P0, P1 = vt_separating(rng)
        add_vt(P0, P1, rng.dirichlet([1, 1, 1])[1:], a, 0)
    # a collision through a fixed sample point (2/3, 1/6) while the frozen
    # parameters sit elsewhere: still active
    P0, P1, _ = vt_collision(rng, 0.5, lam=[2 / 3, 1 / 6])
    add_vt(P0, P1, np.array([0.05, 0.05]), 3, 4)
    # exact tie: the vertex lands on the triangle point (1, 0, 1) at t = 1
    tri = np.array([[0.0, 0, 0], [4.0, 0, 0], [0.0, 0, 4]])
    add_vt(np.vstack([[1.0, 1.0, 1.0], tri]), np.vstack([[1.0, 0.0, 1.0], tri]),
           np.array([0.25, 0.25]), 2, 3)
    nvt_vertices = 4 * len(vt)

    # EE pairs after the VT vertices
    e_rows, ee, lam_ee, a_ee, want_ee = [], [], [], [], []

    def add_ee(P0, P1, lam, a, want):
        base = nvt_vertices + 4 * len(ee)
        X0.append(P0)
        X1.append(P1)
        e_rows.extend([[base, base + 1], [base + 2, base + 3]])
        ee.append([len(e_rows) - 2, len(e_rows) - 1])
        lam_ee.append(lam)
        a_ee.append(a)
        want_ee.append(want)

    for a in (0, 9, a_max):
        P0, P1, lam = ee_collision(rng, rng.uniform(0.1, 0.95))
        add_ee(P0, P1, lam, a, min(a + 1, a_max))
    for a in (0, 4):
        P0 = rng.standard_normal((4, 3))
        P0[:2, 1] = 0.0
        P0[2:, 1] = 0.5
        P1 = P0.copy()
        P1[2:, 1] += 0.3
        add_ee(P0, P1, rng.uniform(0, 1, 2), a, 0)

    xm = np.vstack(X0)
    xp = np.vstack(X1)
    o = bare_oracle(tris, e_rows, xm.shape[0], a_max=a_max)
    C = S.Constraints(vt=np.array(vt, np.int32), ee=np.array(ee, np.int32),
                      a_vt=np.array(a_vt, np.int32), a_ee=np.array(a_ee, np.int32),
                      lam_vt=np.array(lam_vt), lam_ee=np.array(lam_ee))
    o._partial_ccd(C, xm, xp)
    assert C.a_vt.tolist() == want_vt
    assert C.a_ee.tolist() == want_ee


def test_partial_ccd_obstacle_branch():
    """Obstacle constraints are active iff the end position is closer than
    d_hat to the surface (inside counts), with the same counter rule."""
    dh = 0.01
    R = 0.5
    sph = S.Obst(0, np.zeros(3), R, np.array([1.0, 0, 0]))
    cyl = S.Obst(1, np.array([0.0, -2.0, 0.0]), R, np.array([1.0, 0, 0]))
    u = np.array([0.6, 0.8, 0.0])
    radial = np.array([0.0, 0.6, 0.8])
    pts = [R + 0.5 * dh, R + 2 * dh, R - 0.1, R + 0.999 * dh, R + 1.001 * dh]
    x = [sph.center + d * u for d in pts] + [cyl.center + np.array([3.0, 0, 0]) + d * radial for d in pts]
    x = np.array(x)
    n = len(pts)
    ob = np.array([[i, 0] for i in range(n)] + [[n + i, 1] for i in range(n)], np.int32)
    a0 = np.array([3, 3, 20, 0, 5] * 2, np.int32)
    want = [4, 0, 20, 1, 0] * 2
    o = bare_oracle(np.zeros((0, 3)), np.zeros((0, 2)), len(x), d_hat=dh, obs=[sph, cyl])
    C = S.Constraints(ob=ob, a_ob=a0.copy())
    o._partial_ccd(C, x, x)
    assert C.a_ob.tolist() == want


# ------------------------------------------------- constraint-set carry-over

def test_merge_hand_built_sets():
    cand = np.array([[0, 5], [1, 2], [1, 7], [3, 3], [4, 0]], np.int32)
    hit = np.array([False, True, False, False, True])
    prev = np.array([[1, 7], [2, 2], [3, 3], [4, 0]], np.int32)
    prev_a = np.array([4, 9, 11, 6], np.int32)
    rows, a = S._merge(cand, hit, prev, prev_a)
    # [0,5]: neither hit nor previous -> dropped; [1,2]: new hit -> 0;
    # [1,7], [3,3]: carried; [4,0]: hit and previous -> keeps its span;
    # [2,2]: previous but no longer a candidate -> dropped
    assert rows.tolist() == [[1, 2], [1, 7], [3, 3], [4, 0]]
    assert a.tolist() == [0, 4, 11, 6]
    # empty previous set: hits only, all new
    rows, a = S._merge(cand, hit, np.zeros((0, 2), np.int32), np.zeros(0, np.int32))
    assert rows.tolist() == [[1, 2], [4, 0]] and a.tolist() == [0, 0]
    # no candidates: empty, whatever the previous set
    rows, a = S._merge(np.zeros((0, 2), np.int32), np.zeros(0, bool), prev, prev_a)
    assert rows.shape == (0, 2) and a.shape == (0,)


def test_merge_against_brute_force_sets():
    rng = np.random.default_rng(17)
    for _ in range(200):
        allp = {(int(i), int(j)) for i, j in rng.integers(0, 12, (40, 2))}
        cand = sorted(p for p in allp if rng.random() < 0.6)
        prev = sorted(p for p in allp if rng.random() < 0.4)
        pa = {p: int(rng.integers(0, 21)) for p in prev}
        hit = {p: bool(rng.random() < 0.3) for p in cand}
        want = [(p, pa.get(p, 0)) for p in cand if hit[p] or p in pa]
        rows, a = S._merge(np.array(cand, np.int32).reshape(-1, 2), np.array([hit[p] for p in cand], bool),
                           np.array(prev, np.int32).reshape(-1, 2), np.array([pa[p] for p in prev], np.int32))
        assert [tuple(r) for r in rows.tolist()] == [w[0] for w in want]
        assert a.tolist() == [w[1] for w in want]


def test_outer_ccd_membership_on_a_small_scene():
    """Three separate triangles, one falling through another and one resting
    beside it: the new set is the hitting candidates plus the previous
    members still among the candidates, with carried spans; obstacle members
    are free vertices that cross the surface or start or end within d_hat of
    it."""
    tris = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    low = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 1]])
    up0 = np.array([[0.1, 0.05, 0.1], [0.6, 0.05, 0.1], [0.1, 0.05, 0.6]])
    up1 = up0 - np.array([0, 0.1, 0])
    side = np.array([[1.0003, 0.0005, 0.0], [1.5, 0.0005, 0.0], [1.5, 0.0005, 0.5]])
    # vertices 9..13 probe the obstacle rule around a sphere far away
    sph = S.Obst(0, np.array([5.0, -3.0, 5.0]), 1.0, np.array([1.0, 0, 0]))
    dh = 1e-3
    c = sph.center
    probe0 = np.array([c + [0, 1.5, 0], c + [0, 1 + 0.5 * dh, 0], c + [0, 1.2, 0], c + [0, 1.5, 0],
                       c + [0, 1 + 0.5 * dh, 0]])
    probe1 = np.array([c + [0, 0.8, 0], c + [0, 1.2, 0], c + [0, 1 + 0.5 * dh, 0], c + [0, 1.4, 0],
                       c + [0, 1 + 0.5 * dh, 0]])
    xm = np.vstack([low, up0, side, probe0])
    xp = np.vstack([low, up1, side, probe1])
    pinned = np.zeros(len(xm), bool)
    pinned[-1] = True   # a pinned vertex near the surface is no member
    edges = M.unique_edges(tris)
    o = bare_oracle(tris, edges, len(xm), pinned=pinned, d_hat=dh, obs=[sph])
    o.p.self_contact = True
    vt, ee = native.broad_phase(xm.astype(np.float32), xp.astype(np.float32), edges, tris, dh, True)
    tv, te, _ = native.toi_pairs(xm, xp, tris, edges, vt, ee)
    # previous set: a pair still a candidate but not hitting, and a pair
    # that is no longer a candidate, each with a span
    miss_c = [tuple(p) for p, t in zip(vt.tolist(), tv) if t > 1.0]
    hit_c = [tuple(p) for p, t in zip(vt.tolist(), tv) if t <= 1.0]
    assert hit_c and miss_c
    gone = (9, 0)
    assert gone not in {tuple(p) for p in vt.tolist()}
    prev_vt = sorted([miss_c[0], gone])
    prev_a = {miss_c[0]: 7, gone: 3}
    prev = S.Constraints(vt=np.array(prev_vt, np.int32), a_vt=np.array([prev_a[p] for p in prev_vt], np.int32),
                         ob=np.array([[10, 0]], np.int32), a_ob=np.array([5], np.int32))
    st = S.StepStats()
    s, C = o._outer_ccd(xm, xp, prev, st)
    want = sorted(set(hit_c) | {miss_c[0]})
    assert [tuple(p) for p in C.vt.tolist()] == want
    assert C.a_vt.tolist() == [prev_a.get(p, 0) for p in want]
    hit_e = [tuple(p) for p, t in zip(ee.tolist(), te) if t <= 1.0]
    assert [tuple(p) for p in C.ee.tolist()] == hit_e and not C.a_ee.any()
    # obstacle members: 9 crosses, 10 starts within d_hat (span carried),
    # 11 ends within d_hat, 12 never near, 13 pinned
    assert C.ob.tolist() == [[9, 0], [10, 0], [11, 0]]
    assert C.a_ob.tolist() == [0, 5, 0]
    tmin = min(tv.min(), te.min(initial=2.0), S.obstacle_toi(sph, xm, xp).min())
    assert tmin <= 1.0 and s == 0.8 * tmin


# ------------------------------------------------------------ targets

def test_obstacle_target_on_offset_surface_along_radial_line():
    rng = np.random.default_rng(18)
    dh = 0.02
    for kind in (0, 1):
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        ob = S.Obst(kind, rng.standard_normal(3), 0.7, axis)
        dirs = rng.standard_normal((40, 3))
        dist = rng.uniform(0.3, 0.9, 40)
        x = ob.center + dirs / np.linalg.norm(dirs, axis=1)[:, None] * dist[:, None]
        o = bare_oracle(np.zeros((0, 3)), np.zeros((0, 2)), len(x), d_hat=dh, obs=[ob])
        C = S.Constraints(ob=np.stack([np.arange(len(x)), np.zeros(len(x), int)], 1).astype(np.int32),
                          a_ob=np.zeros(len(x), np.int32))
        W, WY = o._collision_terms(C, x)
        assert np.array_equal(W, np.ones(len(x)))
        y = WY
        rel_x = x - ob.center
        rel_y = y - ob.center
        if kind == 1:   # radial = component normal to the axis; axial part unchanged
            assert np.allclose(rel_y @ axis, rel_x @ axis, atol=1e-14)
            rel_x = rel_x - np.outer(rel_x @ axis, axis)
            rel_y = rel_y - np.outer(rel_y @ axis, axis)
        rx = np.linalg.norm(rel_x, axis=1)
        ry = np.linalg.norm(rel_y, axis=1)
        inside = rx < ob.radius + dh
        assert inside.any() and (~inside).any()
        assert np.allclose(ry[inside], ob.radius + dh, atol=1e-14)
        # same radial direction
        cosang = np.einsum("ij,ij->i", rel_x[inside], rel_y[inside]) / (rx[inside] * ry[inside])
        assert np.allclose(cosang, 1.0, atol=1e-14)
        assert np.array_equal(y[~inside], x[~inside])


def _one_constraint_targets(kind, X, lam, nrm, pinned=None, dh=0.05):
    if kind == "vt":
        o = bare_oracle([[1, 2, 3]], [[0, 1]], 4, pinned=pinned, d_hat=dh)
        C = S.Constraints(vt=np.array([[0, 0]], np.int32), a_vt=np.zeros(1, np.int32),
                          lam_vt=lam[None], n_vt=nrm[None])
    else:
        o = bare_oracle(np.zeros((0, 3)), [[0, 1], [2, 3]], 4, pinned=pinned, d_hat=dh)
        C = S.Constraints(ee=np.array([[0, 1]], np.int32), a_ee=np.zeros(1, np.int32),
                          lam_ee=lam[None], n_ee=nrm[None])
    W, WY = o._collision_terms(C, X)
    assert np.array_equal(W, np.ones(4))
    return WY


def test_penetrating_vt_and_ee_targets_sit_d_hat_apart():
    """A penetrating pair is projected so that, along the frozen normal, the
    vertex (or the second edge point) sits exactly d_hat beyond the frozen
    triangle (first edge) point; every vertex moves along the normal only;
    pinned vertices stay; separated pairs keep their positions."""
    rng = np.random.default_rng(19)
    dh = 0.05
    n_pen = 0
    for _ in range(40):
        # VT frozen at a configuration with the vertex above the triangle
        tri = rand_tri(rng)
        nn = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        nn /= np.linalg.norm(nn)
        xm = np.vstack([tri_point(tri, rng.dirichlet([2, 2, 2])[1:]) + 0.1 * nn, tri])
        lam, nrm = native.frozen_vt(xm, np.array([[1, 2, 3]]), np.array([[0, 0]]))
        lam, nrm = lam[0], nrm[0]
        # current positions: vertex pushed through the triangle
        X = xm + 0.05 * rng.standard_normal((4, 3))
        X[0] -= rng.uniform(0.0, 0.3) * nrm
        for pinned in (None, np.array([False, True, False, False]), np.array([True, False, False, False])):
            y = _one_constraint_targets("vt", X, lam, nrm, pinned, dh)
            sep_x = nrm @ (X[0] - tri_point(X[1:], lam))
            sep_y = nrm @ (y[0] - tri_point(y[1:], lam))
            if sep_x < dh:
                n_pen += 1
                assert abs(sep_y - dh) < 1e-12
            else:
                assert np.array_equal(y, X)
            mv = y - X
            assert np.allclose(mv - np.outer(mv @ nrm, nrm), 0, atol=1e-14)
            if pinned is not None:
                assert np.array_equal(y[pinned], X[pinned])
        # EE: edges crossing over each other
        P = rng.standard_normal((4, 3))
        lam, nrm = native.frozen_ee(P, np.array([[0, 1], [2, 3]]), np.array([[0, 1]]))
        lam, nrm = lam[0], nrm[0]
        X = P + 0.05 * rng.standard_normal((4, 3))
        X[2:] -= rng.uniform(0.0, 2.0) * np.linalg.norm(P[2] + lam[1] * (P[3] - P[2]) - P[0]
                                                        - lam[0] * (P[1] - P[0])) * nrm
        for pinned in (None, np.array([False, False, True, False])):
            y = _one_constraint_targets("ee", X, lam, nrm, pinned, dh)
            pt = lambda Z: (Z[2] + lam[1] * (Z[3] - Z[2])) - (Z[0] + lam[0] * (Z[1] - Z[0]))
            if nrm @ pt(X) < dh:
                n_pen += 1
                assert abs(nrm @ pt(y) - dh) < 1e-12
            else:
                assert np.array_equal(y, X)
            mv = y - X
            assert np.allclose(mv - np.outer(mv @ nrm, nrm), 0, atol=1e-14)
            if pinned is not None:
                assert np.array_equal(y[pinned], X[pinned])
    assert n_pen > 60


# ------------------------------------------------------- spectral radius

@pytest.mark.parametrize("gamma", [0.9, 0.7])
def test_spectral_radius_against_dense_spectrum(gamma):
    """spectral_radius is the largest |eigenvalue| of the coarse-corrected
    damped Jacobi error operator E = (I - gamma D^{-1} H)(I - U A^{-1} U^T H)
    on the free rows, computed here as a dense matrix."""
    import scenegen
    sc = scenegen.hanging_cloth(10, seed=5, r=6)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    _, U = M.eigenbasis(m, sc.r)
    Us = M.stored_basis(U, "fp32")
    H = m.H.toarray()
    n = m.nv
    A = Us.T @ H @ Us
    Pc = np.eye(n) - Us @ np.linalg.solve(A, Us.T @ H)
    J = np.eye(n) - gamma * H / m.diagH[:, None]
    E = J @ Pc
    f = ~m.pinned
    ev = np.linalg.eigvals(E[np.ix_(f, f)])
    want = np.abs(ev).max()
    got = M.spectral_radius(m, Us, gamma, iters=3000)
    assert got == pytest.approx(want, rel=1e-6)
    # the coarse correction matters at these dampings: without it the
    # radius is the one of the low modes, much closer to 1
    ev0 = np.abs(np.linalg.eigvals(J[np.ix_(f, f)])).max()
    assert ev0 > want + 1e-3


# ------------------------------------------------- exact tangle arithmetic

def test_exact_integer_scaling_preserves_orientation_signs():
    """The exact tangle check scales FP32 coordinates to integers by 2^149:
    every orientation sign equals the one of the rational determinant, also
    for tiny, subnormal and exactly coplanar inputs."""
    from fractions import Fraction

    from oracle import exact
    rng = np.random.default_rng(41)

    def frac_orient(a, b, c, d):
        ab = [b[i] - a[i] for i in range(3)]
        ac = [c[i] - a[i] for i in range(3)]
        ad = [d[i] - a[i] for i in range(3)]
        det = (ab[0] * (ac[1] * ad[2] - ac[2] * ad[1]) - ab[1] * (ac[0] * ad[2] - ac[2] * ad[0])
               + ab[2] * (ac[0] * ad[1] - ac[1] * ad[0]))
        return (det > 0) - (det < 0)

    cases = []
    for _ in range(300):
        P = rng.standard_normal((4, 3)).astype(np.float32)
        cases.append(P)
        Q = P.copy()
        Q[3] = (Q[0] + np.float32(0.5) * (Q[1] - Q[0])).astype(np.float32)   # near the line / plane
        cases.append(Q)
        cases.append((P * np.float32(1e-38)).astype(np.float32))            # subnormal range
        R = P.copy()
        R[:, 2] = np.float32(0.25)                                           # exactly coplanar
        cases.append(R)
    zeros = 0
    for P in cases:
        F = [[Fraction(float(v)) for v in row] for row in P]
        I = [[exact._exact_int(v) for v in row] for row in P]
        want = frac_orient(*F)
        assert exact._orient(*I) == want
        zeros += want == 0
    assert zeros >= 300
