"""Pins of the oracle's collision side: Eq. (collision_judge), the no-miss
bound of Eq. (sample_bound), the gradient bound Eq. (derivative_bound), the
broad phase against brute force, TOI against dense time sampling, obstacle
TOI, the tangle checker, and a contact simulation that stays tangle-free."""
import numpy as np
import pytest

import scenegen
from oracle import exact, native
from oracle import model as M
from oracle import step as S


def rand_unit(rng, n=None):
    v = rng.standard_normal((n, 3) if n else 3)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def vt_collision(rng, t_star):
    """A VT pair whose vertex meets the triangle point at barycentric lambda*
    at time t*; returns positions at t=0 and t=1 (rows v, a, b, c) and lambda*."""
    a0, b0, c0 = rng.standard_normal((3, 3))
    lam = rng.dirichlet([1, 1, 1])[1:]
    va, vb, vc = 0.3 * rng.standard_normal((3, 3))
    tri0 = np.stack([a0, b0, c0])
    tri1 = tri0 + np.stack([va, vb, vc])
    meet = lambda tri: tri[0] + lam[0] * (tri[1] - tri[0]) + lam[1] * (tri[2] - tri[0])
    q_star = tri0 + t_star * (tri1 - tri0)
    m_star = meet(q_star)
    d = rng.standard_normal(3)
    p0 = m_star - t_star * d
    p1 = p0 + d
    return np.vstack([p0, tri0]), np.vstack([p1, tri1]), lam


def test_query_identity_collision_judge():
    """Q(lambda*) = ((t*-1)/t*) |p2^0 - p1^0|^2 for a known collision."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        t_star = rng.uniform(0.05, 1.0)
        P0, P1, lam = vt_collision(rng, t_star)
        Q = S.query_vt(P0, P1, np.array([0]), np.array([[1, 2, 3]]), lam[None, None, :])[0, 0]
        p2_0 = P0[1] + lam[0] * (P0[2] - P0[1]) + lam[1] * (P0[3] - P0[1])
        ref = (t_star - 1) / t_star * np.sum((p2_0 - P0[0]) ** 2)
        assert np.isclose(Q, ref, rtol=1e-9, atol=1e-12)
        assert Q <= 1e-12


def _grad_bound_pair(rng, L):
    """Random EE pair with edge lengths <= L (both times)."""
    P0 = rng.uniform(-1, 1, (4, 3))
    P1 = P0 + 0.5 * rng.standard_normal((4, 3))
    for P in (P0, P1):
        for (i, j) in ((0, 1), (2, 3)):
            d = P[j] - P[i]
            n = np.linalg.norm(d)
            if n > L:
                P[j] = P[i] + d * (L / n)
    return P0, P1


def test_derivative_bound():
    """|dQ/dlambda_i| <= 2 L (H1 + 2L), Eq. (derivative_bound), for EE pairs:
    L bounds edge lengths, H1 the distance at t=1 over the domain."""
    rng = np.random.default_rng(1)
    e1 = np.array([[0, 1]])
    e2 = np.array([[2, 3]])
    g = np.linspace(0, 1, 21)
    lam = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(1, -1, 2)
    for _ in range(200):
        L = rng.uniform(0.1, 1.0)
        P0, P1 = _grad_bound_pair(rng, L)
        p1 = P1[0] + lam[0, :, :1] * (P1[1] - P1[0])
        p2 = P1[2] + lam[0, :, 1:] * (P1[3] - P1[2])
        H1 = np.linalg.norm(p2 - p1, axis=1).max()
        eps = 1e-6
        for i in range(2):
            dl = np.zeros(2)
            dl[i] = eps
            Qp = S.query_ee(P0, P1, e1, e2, lam + dl)
            Qm = S.query_ee(P0, P1, e1, e2, lam - dl)
            dq = np.abs(Qp - Qm) / (2 * eps)
            assert dq.max() <= 2 * L * (H1 + 2 * L) * (1 + 1e-6)


def test_dense_samples_never_miss():
    """With sample interval below rho* (Eq. (sample_bound)) and t* <= alpha,
    some sample has Q <= 0 for every constructed VT collision."""
    rng = np.random.default_rng(2)
    alpha = 0.8
    tested = 0
    for _ in range(200):
        t_star = rng.uniform(0.1, alpha)
        P0, P1, lam = vt_collision(rng, t_star)
        # scale down motion so that the bound is moderate
        edges0 = [np.linalg.norm(P0[i] - P0[j]) for i, j in ((1, 2), (2, 3), (3, 1))]
        edges1 = [np.linalg.norm(P1[i] - P1[j]) for i, j in ((1, 2), (2, 3), (3, 1))]
        L = max(edges0 + edges1)
        g = np.linspace(0, 1, 201)
        ll = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
        ll = ll[ll.sum(1) <= 1]
        q1 = P1[1] + ll[:, :1] * (P1[2] - P1[1]) + ll[:, 1:] * (P1[3] - P1[1])
        q0 = P0[1] + ll[:, :1] * (P0[2] - P0[1]) + ll[:, 1:] * (P0[3] - P0[1])
        H1 = np.linalg.norm(q1 - P1[0], axis=1).max()
        H0 = np.linalg.norm(q0 - P0[0], axis=1).min()
        rho_star = (1 / alpha - 1) * H0 ** 2 / (2 * np.sqrt(2) * L * (H1 + 2 * L))
        h = rho_star * np.sqrt(2) * 0.999   # a square grid of spacing h has interval h/sqrt(2)
        if h < 4e-3:
            continue
        tested += 1
        gg = np.arange(0, 1 + h, h)
        samp = np.stack(np.meshgrid(gg, gg, indexing="ij"), -1).reshape(-1, 2)
        samp = samp[samp.sum(1) <= 1 + 1e-12]
        Q = S.query_vt(P0, P1, np.array([0]), np.array([[1, 2, 3]]), samp[None])[0]
        assert Q.min() <= 0
    assert tested >= 10


def brute_pairs(xm, xp, edges, tris, dhat):
    def boxes(idx):
        pts = np.concatenate([xm[idx], xp[idx]], axis=1)
        lo = pts.min(1) - np.float32(dhat)
        hi = pts.max(1) + np.float32(dhat)
        return lo.astype(np.float32), hi.astype(np.float32)
    nv = xm.shape[0]
    vl, vh = boxes(np.arange(nv)[:, None])
    tl, th = boxes(tris)
    el, eh = boxes(edges)
    ov = np.all((vl[:, None] <= th[None]) & (tl[None] <= vh[:, None]), axis=2)
    share = (tris[None, :, :] == np.arange(nv)[:, None, None]).any(2)
    vt = np.argwhere(ov & ~share)
    oe = np.all((el[:, None] <= eh[None]) & (el[None] <= eh[:, None]), axis=2)
    sh = (edges[:, None, :, None] == edges[None, :, None, :]).any((2, 3))
    up = np.triu(np.ones_like(oe), 1)
    ee = np.argwhere(oe & ~sh & up)
    return vt.astype(np.int32), ee.astype(np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_broad_phase_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    sc = scenegen.drop_cloth(12, seed=seed, obstacle="sphere", r=4, steps=1, d_hat=2e-3)
    tris = sc.tris
    edges = M.unique_edges(tris)
    xm = sc.x0.copy()
    # crumple: random displacements of a few edge lengths
    xm = (xm + rng.normal(0, 0.05, xm.shape)).astype(np.float32)
    xp = (xm + rng.normal(0, 0.03, xm.shape)).astype(np.float32)
    vt, ee = native.broad_phase(xm, xp, edges, tris, 2e-3)
    bvt, bee = brute_pairs(xm, xp, edges, tris, 2e-3)
    assert np.array_equal(vt, bvt)
    assert np.array_equal(ee, bee)
    assert len(vt) > 100 and len(ee) > 100


def sampled_toi(kind, P0, P1, n=100000):
    """Dense time sampling of the coplanarity sign plus bisection; the first
    coplanar time with contact (inside test on the exact in-plane geometry)."""
    t = np.linspace(0, 1, n + 1)
    P = P0[None] + t[:, None, None] * (P1 - P0)[None]

    def f(P):
        if kind == "vt":
            return np.einsum("...d,...d->...", np.cross(P[..., 2, :] - P[..., 1, :], P[..., 3, :] - P[..., 1, :]),
                             P[..., 0, :] - P[..., 1, :])
        return np.einsum("...d,...d->...", np.cross(P[..., 1, :] - P[..., 0, :], P[..., 3, :] - P[..., 2, :]),
                         P[..., 2, :] - P[..., 0, :])

    def inside(Q):
        if kind == "vt":
            p, a, b, c = Q
            n_ = np.cross(b - a, c - a)
            u = np.cross(b - p, c - p) @ n_
            v = np.cross(c - p, a - p) @ n_
            w = np.cross(a - p, b - p) @ n_
            return u >= -1e-9 * abs(n_ @ n_) and v >= -1e-9 * abs(n_ @ n_) and w >= -1e-9 * abs(n_ @ n_)
        p1, p2, p3, p4 = Q
        d1, d2, r = p2 - p1, p4 - p3, p3 - p1
        n_ = np.cross(d1, d2)
        nn = n_ @ n_
        s1 = np.cross(r, d2) @ n_ / nn
        s2 = np.cross(r, d1) @ n_ / nn
        return -1e-9 <= s1 <= 1 + 1e-9 and -1e-9 <= s2 <= 1 + 1e-9

    F = f(P)
    idx = np.flatnonzero(np.sign(F[:-1]) != np.sign(F[1:]))
    for i in idx:
        lo, hi = t[i], t[i + 1]
        flo = f(P0 + lo * (P1 - P0))
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            fm = f(P0 + mid * (P1 - P0))
            if np.sign(fm) == np.sign(flo):
                lo, flo = mid, fm
            else:
                hi = mid
        if inside(P0 + lo * (P1 - P0)):
            return lo
    return 2.0


@pytest.mark.parametrize("kind", ["vt", "ee"])
def test_toi_matches_dense_time_sampling(kind):
    rng = np.random.default_rng(3 if kind == "vt" else 4)
    hits = 0
    for it in range(60):
        if kind == "vt" and it % 2:
            P0, P1, _ = vt_collision(rng, rng.uniform(0.05, 1.0))
        else:
            P0 = rng.uniform(-1, 1, (4, 3))
            P1 = P0 + rng.normal(0, 0.8, (4, 3))
        ref = sampled_toi(kind, P0, P1)
        got, fb = (native.toi_vt if kind == "vt" else native.toi_ee)(P0, P1)
        assert fb == 0
        if ref > 1:
            assert got > 1
        else:
            hits += 1
            assert abs(got - ref) <= 1e-6
    assert hits >= 5


def test_toi_known_cases():
    # vertex moving straight through a static triangle: TOI = d0 / (d0 + d1)
    tri = np.array([[0.0, 0, 0], [1, 0, 0], [0, 0, 1]])
    for d0, d1 in ((0.3, 0.7), (0.01, 2.0), (1.0, 1e-3)):
        P0 = np.vstack([[0.2, d0, 0.2], tri])
        P1 = np.vstack([[0.2, -d1, 0.2], tri])
        t, fb = native.toi_vt(P0, P1)
        assert abs(t - d0 / (d0 + d1)) <= 1e-12
    # passing beside the triangle: no hit
    P0 = np.vstack([[2.0, 0.3, 2.0], tri])
    P1 = np.vstack([[2.0, -0.3, 2.0], tri])
    assert native.toi_vt(P0, P1)[0] > 1
    # crossing edges: edge 1 static along x, edge 2 along z moving down through it
    e0 = np.array([[-1.0, 0, 0], [1, 0, 0], [0.25, 0.5, -1], [0.25, 0.5, 1]])
    e1 = e0.copy()
    e1[2:, 1] = -1.5
    t, _ = native.toi_ee(e0, e1)
    assert abs(t - 0.25) <= 1e-12
    # coplanar motion (degenerate cubic) uses the sampled fallback
    P0 = np.vstack([[0.2, 0.0, 2.0], tri])
    P1 = np.vstack([[0.2, 0.0, -1.0], tri])
    t, fb = native.toi_vt(P0, P1)
    assert fb == 1 and abs(t - 0.4) < 1e-9  # enters across x + z = 1 at z = 0.8


def test_obstacle_toi_closed_form():
    ob = S.Obst(0, np.array([0.0, 0.0, 0.0]), 0.5, np.array([1.0, 0, 0]))
    xm = np.array([[0.0, 1.0, 0.0], [0.3, 0.9, 0.0], [2.0, 1.0, 0.0]])
    xp = np.array([[0.0, 0.0, 0.0], [0.3, -0.9, 0.0], [2.0, -1.0, 0.0]])
    toi = S.obstacle_toi(ob, xm, xp)
    assert abs(toi[0] - 0.5) < 1e-15
    yhit = np.sqrt(0.25 - 0.09)
    assert abs(toi[1] - (0.9 - yhit) / 1.8) < 1e-14
    assert toi[2] > 1
    cyl = S.Obst(1, np.array([0.0, 0.0, 0.0]), 0.5, np.array([1.0, 0, 0]))
    xm = np.array([[7.0, 1.0, 0.0]])
    xp = np.array([[-3.0, 0.0, 0.0]])
    assert abs(S.obstacle_toi(cyl, xm, xp)[0] - 0.5) < 1e-15


def test_tangle_checker():
    tris = np.array([[0, 1, 2], [3, 4, 5]])
    A = [[0, 0, 0], [1, 0, 0], [0, 0, 1]]
    cross = np.array(A + [[0.2, -1, 0.2], [0.2, 1, 0.2], [0.4, 1, 0.3]], np.float32)
    apart = np.array(A + [[0.2, 0.1, 0.2], [0.2, 1, 0.2], [0.4, 1, 0.3]], np.float32)
    touch = np.array(A + [[0.2, 0.0, 0.2], [0.2, 1, 0.2], [0.4, 1, 0.3]], np.float32)
    assert exact.count_tangles(cross, tris) == 1
    assert exact.count_tangles(apart, tris) == 0
    assert exact.count_tangles(touch, tris) == 1  # closed sets: touching counts
    sc = scenegen.drop_cloth(16, seed=0, obstacle="sphere", r=4, steps=1)
    assert exact.count_tangles(sc.x0, sc.tris) == 0


def test_tangle_exact_predicate_brute():
    rng = np.random.default_rng(9)
    for _ in range(300):
        P = rng.integers(-3, 4, (6, 3)).astype(np.float32)
        tris = np.array([[0, 1, 2], [3, 4, 5]])
        hits, und, nund, _ = native.tangles(P, tris)
        ex = exact.tri_tri_exact(P[:3], P[3:])
        if nund == 0:
            assert bool(hits) == ex


def test_contact_simulation_stays_tangle_free():
    """(f) A cloth dropped onto a sphere with self-contact: zero intersecting
    triangle pairs after every step."""
    sc = scenegen.drop_cloth(20, seed=5, obstacle="sphere", r=8, steps=12, drop=0.004,
                             d_hat=1e-3)
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    lam, U = M.eigenbasis(m, sc.r)
    rho = M.spectral_radius(m, U, 0.9, 150)
    p = S.Params(iters_outer=3, iters_inner=5, cheb_rho=0.999 * rho, cheb_gamma=0.9,
                 d_hat=sc.d_hat)
    obs = [S.Obst(0, np.array(o.center), o.radius, np.array(o.axis)) for o in sc.obstacles]
    o = S.Oracle(m, U, p, sc.gravity, obs)
    o.set_state(sc.x0, sc.v0)
    ncons = 0
    for _ in range(sc.steps):
        st = o.step()
        ncons += st.n_constraints
        assert exact.count_tangles(o.x.astype(np.float32), m.tris) == 0
        phi, _, _ = S.obstacle_phi(obs[0], o.x)
        assert phi.min() > 0
    assert ncons > 0
