"""Oracle time step: the inner projective-dynamics iteration with subspace
reuse, the non-distance barrier and partial CCD, and the per-block full CCD
filter, in FP64 on the CPU (TEST INFRASTRUCTURE ONLY).

Paper passages followed, in the order the step takes them:
  * predictor z = x* + h v* + h^2 g ............................ Eq. (z)
  * initial full CCD and filter on (x*, z) .............. Algorithm 1 (start)
  * per outer block, I inner iterations of:
      local step: triangle strain projection, hinge bending target,
        collision targets weighted by w = k K^a (K = 2) ... Eq. (local), (exp)
      residual r0 = b - (H + diag W) x ....................... Eq. (global)
      subspace reuse (Lambda~ + U^T diag W U) q = U^T r0,
        x~ = x + U q ......... Eq. (subspace_collision), Eq. (uu), section 5.1
      Jacobi sweep on the residual of x~ ..... Eq. (high_frequency_residual)
        with Chebyshev acceleration (the semi-iterative weights of Wang 2015)
      partial CCD on (x-, x^{k+1}) -> life spans a_p ....... Eq. (query)
    then full CCD on (x-, x+), constraint set update and the filter
      x = x- + s (x+ - x-), s = alpha t_TOI or 1 ......... section 6, 7
  * v = (x - x*) / h.

Readings where the paper is silent are listed in the repository's design
notes (strain model, collision target, life-span cap, sample set, filter).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from . import native
from .model import Model

NO_HIT = 2.0
VT_SAMPLES = np.array([[1 / 6, 1 / 6], [2 / 3, 1 / 6], [1 / 6, 2 / 3]])
EE_SAMPLES = np.array([[0.25, 0.25], [0.5, 0.5], [0.75, 0.75]])


@dataclass
class Params:
    iters_outer: int
    iters_inner: int
    cheb_rho: float
    cheb_gamma: float = 1.0
    cheb_delay: int = 3
    d_hat: float = 1e-3
    alpha: float = 0.8
    K_base: float = 2.0
    a_max: int = 20
    self_contact: bool = True
    tol_inner: float = 0.0     # Algorithm 1 inner loop condition (<= 0: the budget alone)
    tol_outer: float = 0.0     # Algorithm 1 outer loop condition (<= 0: the budget alone)
    warm_iters: int = 0        # modal warm-start iterations (0 = start from z)
    rf_iters: int = 0          # residual-forwarding iterations (0 = off)
    rf_toi: float = 0.5        # forward the residual when the exiting t_TOI is below this
    friction: float = 0.0      # friction coefficient mu of obstacle contacts (0 = frictionless)
    smoother: str = "chebyshev"    # or "ajacobi2": rank-2 A-Jacobi, two damped Jacobi steps per iteration
    adaptive_samples: bool = False   # partial-CCD sample density from the change of rho* (Eq. (sample_bound))
    friction_eps_v: float = 1e-3   # sticking velocity threshold (m/s)


@dataclass
class Obst:
    kind: int          # 0 sphere, 1 cylinder (infinite along its axis)
    center: np.ndarray
    radius: float
    axis: np.ndarray
    omega: float = 0.0   # spin about the axis (rad/s): the surface moves at omega R (axis x n)


@dataclass
class Constraints:
    """Constraint set C of one outer block (sorted lists, life spans a)."""
    vt: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    ee: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    ob: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))  # (vertex, obstacle)
    a_vt: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    a_ee: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    a_ob: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    # frozen at x- of the block
    lam_vt: np.ndarray = None
    n_vt: np.ndarray = None
    lam_ee: np.ndarray = None
    n_ee: np.ndarray = None


@dataclass
class StepStats:
    dx: List[float] = field(default_factory=list)
    min_toi: float = NO_HIT
    n_candidates: int = 0
    n_constraints: int = 0
    fallbacks: int = 0
    t_exit: float = NO_HIT     # t_TOI of the step's last (exiting) filter
    outer_dx: List[float] = field(default_factory=list)   # change of x over each outer block run
    inner_iters: int = 0       # inner iterations run
    outer_iters: int = 0       # outer blocks run
    block_iters: List[int] = field(default_factory=list)   # inner iterations of each block run


def chebyshev_weights(n: int, rho: float, delay: int) -> np.ndarray:
    """omega_{k+1} for k = 0..n-1: 1 before the delay S, 2/(2 - rho^2) at S,
    then 4/(4 - rho^2 omega_k)."""
    w = np.ones(n)
    for k in range(n):
        if k < delay:
            w[k] = 1.0
        elif k == delay:
            w[k] = 2.0 / (2.0 - rho * rho)
        else:
            w[k] = 4.0 / (4.0 - rho * rho * w[k - 1])
    return w


def polar_3x2(F: np.ndarray) -> np.ndarray:
    """Closest matrix with orthonormal columns to each 3x2 F (rows of a
    stack): T = F (F^T F)^{-1/2}, with the 2x2 square root in closed form
    sqrt(S) = (S + sqrt(det S) I) / sqrt(tr S + 2 sqrt(det S)).
    Near-degenerate F (det S <= 1e-20) is returned unchanged."""
    S = np.einsum("tdi,tdj->tij", F, F)
    det = S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0]
    ok = det > 1e-20
    sd = np.sqrt(np.where(ok, det, 1.0))
    den = np.sqrt(S[:, 0, 0] + S[:, 1, 1] + 2 * sd)
    R = (S + sd[:, None, None] * np.eye(2)) / den[:, None, None]
    detR = sd  # det sqrt(S) = sqrt(det S)
    Rinv = np.empty_like(R)
    Rinv[:, 0, 0] = R[:, 1, 1] / detR
    Rinv[:, 1, 1] = R[:, 0, 0] / detR
    Rinv[:, 0, 1] = -R[:, 0, 1] / detR
    Rinv[:, 1, 0] = -R[:, 1, 0] / detR
    T = np.einsum("tdi,tij->tdj", F, Rinv)
    T[~ok] = F[~ok]
    return T


def strain_limited_3x2(F: np.ndarray, smin: float, smax: float) -> np.ndarray:
    """Closest 3x2 matrix to each F whose singular values lie in
    [smin, smax]: T = U clamp(Sigma) V^T from the thin SVD F = U Sigma V^T
    (the strain-limiting projection of a triangle's deformation gradient;
    smin = smax = 1 is the rotation of polar_3x2)."""
    Uf, sv, Vt = np.linalg.svd(F, full_matrices=False)
    return np.einsum("tdi,ti,tij->tdj", Uf, np.clip(sv, smin, smax), Vt)


def elastic_rhs(model: Model, x: np.ndarray) -> np.ndarray:
    """sum_t w_t G_t^T T_t^T + sum_e w_e K_e y_e (local step, Eq. (local)) as
    a per-vertex 3-vector; T is the projection of the deformation gradient
    onto rotations, or onto the strain-limited set when the model's limits
    are not (1, 1)."""
    xs = x[model.tris]                                      # (T,3,3) corners x xyz
    F = np.einsum("tcd,tci->tdi", xs, model.g)              # (T,3,2)
    if model.sigma_min == 1.0 and model.sigma_max == 1.0:
        T = polar_3x2(F)
    else:
        T = strain_limited_3x2(F, model.sigma_min, model.sigma_max)
    contrib = np.einsum("tdi,tci->tcd", T, model.g) * model.w_tri[:, None, None]
    rhs = np.zeros_like(x)
    np.add.at(rhs, model.tris.ravel(), contrib.reshape(-1, 3))
    curved = model.rest_bend > 0
    if curved.any():
        hg = model.hinges[curved]
        K = model.K[curved]
        s = np.einsum("ek,ekd->ed", K, x[hg])
        sn = np.linalg.norm(s, axis=1)
        y = np.where(sn[:, None] > 0, s * (model.rest_bend[curved] / np.where(sn > 0, sn, 1))[:, None], 0)
        c = K[:, :, None] * (model.w_hinge[curved][:, None] * 1.0)[:, :, None] * y[:, None, :]
        np.add.at(rhs, hg.ravel(), c.reshape(-1, 3))
    return rhs


def query_vt(xm, xp, v, tri, lam):
    """Q(lambda) = (p2^1(lambda) - p1^1) . (p2^0(lambda) - p1^0), Eq. (query),
    for a vertex p1 = x_v and the triangle point p2 = x1 + l1 (x2-x1) + l2 (x3-x1);
    lam has shape (P, S, 2); returns (P, S)."""
    def p2(x):
        a, b, c = x[tri[:, 0]], x[tri[:, 1]], x[tri[:, 2]]
        return a[:, None] + lam[..., :1] * (b - a)[:, None] + lam[..., 1:] * (c - a)[:, None]
    return np.einsum("psd,psd->ps", p2(xp) - xp[v][:, None], p2(xm) - xm[v][:, None])


def query_ee(xm, xp, e1, e2, lam):
    """Q(lambda) for edges p1 = x1 + l1 (x2 - x1), p2 = x3 + l2 (x4 - x3)."""
    def diff(x):
        p1 = x[e1[:, 0]][:, None] + lam[..., :1] * (x[e1[:, 1]] - x[e1[:, 0]])[:, None]
        p2 = x[e2[:, 0]][:, None] + lam[..., 1:] * (x[e2[:, 1]] - x[e2[:, 0]])[:, None]
        return p2 - p1
    return np.einsum("psd,psd->ps", diff(xp), diff(xm))


ADAPT_M0, ADAPT_MMAX = 2, 8


def _norm3(d):
    """|d| per row, summed in the order x, y, z."""
    return np.sqrt((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2])


def rho_star_ratio(q0, q1, vt):
    """Change ratio of the threshold sample interval rho* of Eq.
    (sample_bound) over an inner iteration, for pairs with corner points q0
    (at x-) and q1 (at the iterate), shape (P, 4, 3); VT: vertex 0 against
    triangle (1, 2, 3); EE: edge (0, 1) against edge (2, 3).  rho* is
    proportional to (H0)^2 / (L (H1 + 2 L)); H0 (the distance at t = 0) is
    the same for both, L is the longest primitive edge and H1 the largest
    distance between a point of one primitive and a point of the other over
    the motion.  Both are convex in time along straight-line motion, so
    their maxima over t are the larger of the two end values; the reference
    takes them at x- alone (no motion).  The ratio is at most 1."""
    if vt:
        edges = [(1, 2), (2, 3), (3, 1)]
        pairs = [(0, 1), (0, 2), (0, 3)]
    else:
        edges = [(0, 1), (2, 3)]
        pairs = [(0, 2), (0, 3), (1, 2), (1, 3)]
    L0 = np.max([_norm3(q0[:, i] - q0[:, j]) for i, j in edges], axis=0)
    L1 = np.maximum(L0, np.max([_norm3(q1[:, i] - q1[:, j]) for i, j in edges], axis=0))
    H0 = np.max([_norm3(q0[:, i] - q0[:, j]) for i, j in pairs], axis=0)
    H1 = np.maximum(H0, np.max([_norm3(q1[:, i] - q1[:, j]) for i, j in pairs], axis=0))
    return (L0 * (H0 + 2.0 * L0)) / (L1 * (H1 + 2.0 * L1))


def adaptive_level(ratio):
    """Subdivision level m of the refined sample set: the base interval
    (level ADAPT_M0) scaled by the ratio, m = min(ADAPT_MMAX, floor(M0 /
    ratio)); m <= M0 keeps the fixed base samples."""
    with np.errstate(divide="ignore"):
        m = np.floor(ADAPT_M0 / ratio)
    return np.minimum(m, ADAPT_MMAX).astype(np.int64)


def refined_samples(m, vt):
    """The refined sample set of level m: VT, the centroids of the m^2
    sub-triangles of the m-subdivision of the barycentric triangle; EE, the
    centres of the m x m cells of the parameter square."""
    out = []
    if vt:
        for i in range(m):
            for j in range(m - i):
                out.append(((i + 1.0 / 3) / m, (j + 1.0 / 3) / m))
                if i + j <= m - 2:
                    out.append(((i + 2.0 / 3) / m, (j + 2.0 / 3) / m))
    else:
        for i in range(m):
            for j in range(m):
                out.append(((i + 0.5) / m, (j + 0.5) / m))
    return np.array(out)


def obstacle_phi(ob: Obst, x: np.ndarray):
    """Signed distance to the obstacle surface and the radial vector used by
    the projection (sphere: x - c; cylinder: its component normal to the axis)."""
    o = x - ob.center
    if ob.kind == 1:
        o = o - np.outer(o @ ob.axis, ob.axis)
    rad = np.linalg.norm(o, axis=1)
    return rad - ob.radius, o, rad


def obstacle_toi(ob: Obst, xm: np.ndarray, xp: np.ndarray) -> np.ndarray:
    """Entering root in [0,1] of |radial(x- + t (x+ - x-))| = R; NO_HIT for
    vertices already inside or never reaching the surface."""
    d = xp - xm
    o = xm - ob.center
    if ob.kind == 1:
        d = d - np.outer(d @ ob.axis, ob.axis)
        o = o - np.outer(o @ ob.axis, ob.axis)
    a = np.einsum("ij,ij->i", d, d)
    b = 2 * np.einsum("ij,ij->i", o, d)
    c = np.einsum("ij,ij->i", o, o) - ob.radius ** 2
    disc = b * b - 4 * a * c
    toi = np.full(xm.shape[0], NO_HIT)
    ok = (c > 0) & (b < 0) & (disc >= 0) & (a > 0)
    q = 0.5 * (-b[ok] + np.sqrt(disc[ok]))
    t = c[ok] / q
    t = np.where(t <= 1.0, t, NO_HIT)
    toi[ok] = t
    return toi


def obstacle_friction(ob: Obst, x: np.ndarray, xs: np.ndarray, w: np.ndarray, h: float, d_hat: float,
                      mu: float, eps_v: float):
    """Lagged friction of obstacle contacts (section 8.4: a lagged friction
    Hessian at every local/global iteration), a smoothed Coulomb law.  For a
    vertex in the contact band (signed distance below d_hat) with unit
    normal n, normal force lambda = w (R + d_hat - |radial|) of its barrier
    weight w, and tangential slip u_T: the tangential part of the motion over
    the step (x - xs) relative to the surface, which moves by
    h omega R (axis x n), the friction term is a weight
        wf = mu lambda f1(|u_T|) / |u_T|,
        f1(y) = 2 y / eps - y^2 / eps^2 for y < eps = eps_v h, 1 beyond,
    pulling toward x - u_T, so its force wf |u_T| is mu lambda while
    slipping and grows linearly from zero while sticking.  Returns (wf, u_T);
    wf = 0 outside the band."""
    phi, o, rad = obstacle_phi(ob, x)
    band = (phi < d_hat) & (rad > 0)
    wf = np.zeros(len(x))
    uT = np.zeros_like(x)
    if mu <= 0 or not band.any():
        return wf, uT
    n = o[band] / rad[band, None]
    vs_h = h * ob.omega * ob.radius * np.cross(ob.axis, n)
    u = (x[band] - xs[band]) - vs_h
    ut = u - np.sum(u * n, axis=1)[:, None] * n
    y = np.linalg.norm(ut, axis=1)
    eps = eps_v * h
    f = np.where(y < eps, 2.0 / eps - y / eps ** 2, 1.0 / np.where(y > 0, y, 1.0))
    lam = w[band] * (ob.radius + d_hat - rad[band])
    wf[band] = mu * lam * f
    uT[band] = ut
    return wf, uT


class Oracle:
    """FP64 reference solver for one scene; state is (x, v)."""

    def __init__(self, model: Model, Us: np.ndarray, params: Params, gravity,
                 obstacles: Optional[List[Obst]] = None, Uw: Optional[np.ndarray] = None):
        """Us: the stored basis of the subspace reuse (section 5); Uw: the
        stored basis of the modal warm start (Algorithm 1 before the first
        full CCD), by default Us (the paper uses a wider one there, 120
        modes against 30, section 8.1)."""
        self.m = model
        self.U = np.asarray(Us, np.float64)
        self.Uw = self.U if Uw is None else np.asarray(Uw, np.float64)
        self.Lw = self.Uw.T @ (model.H @ self.Uw)
        self.p = params
        self.g = np.asarray(gravity, np.float64)
        self.obs = obstacles or []
        self.Lam = self.U.T @ (model.H @ self.U)
        self.x = model.rest.copy()
        self.v = np.zeros_like(self.x)
        self.free = ~model.pinned
        self.pin_pos = model.rest.copy()
        self.omega = chebyshev_weights(max(params.iters_inner, params.rf_iters, 1), params.cheb_rho,
                                       params.cheb_delay)
        self.rf_dx = np.zeros_like(self.x)   # residual forwarded to the next step (2 dx term of z)
        self.last = StepStats()

    # ---- state
    def set_state(self, x, v):
        self.x = np.array(x, np.float64)
        self.v = np.array(v, np.float64)
        self.pin_pos = self.x.copy()
        self.rf_dx = np.zeros_like(self.x)

    # ---- constraint bookkeeping
    def _weights(self, a: np.ndarray) -> np.ndarray:
        return np.ldexp(self.m.k_contact, a.astype(np.int64)) if self.p.K_base == 2.0 else \
            self.m.k_contact * self.p.K_base ** a

    def _collision_terms(self, C: Constraints, x: np.ndarray, xs: Optional[np.ndarray] = None):
        """Per-vertex W = sum w_p and WY = sum w_p y_{p,v} over constraints.
        VT/EE: half-space projection with the normal and closest-point
        parameters frozen at x-; obstacles: projection onto the surface offset
        by d_hat, plus the lagged friction term (`obstacle_friction`, slip
        measured from the step's start xs) when the friction coefficient is
        positive."""
        nv = self.m.nv
        W = np.zeros(nv)
        WY = np.zeros((nv, 3))
        dh = self.p.d_hat
        mov = self.free.astype(np.float64)
        if len(C.vt):
            tri = self.m.tris[C.vt[:, 1]]
            ids = np.concatenate([C.vt[:, :1], tri], axis=1)          # (P,4)
            l1, l2 = C.lam_vt[:, 0], C.lam_vt[:, 1]
            coef = np.stack([np.ones_like(l1), -(1 - l1 - l2), -l1, -l2], 1)
            self._half_space(ids, coef, C.n_vt, self._weights(C.a_vt), x, mov, dh, W, WY)
        if len(C.ee):
            ids = np.concatenate([self.m.edges[C.ee[:, 0]], self.m.edges[C.ee[:, 1]]], axis=1)
            s, t = C.lam_ee[:, 0], C.lam_ee[:, 1]
            coef = np.stack([-(1 - s), -s, 1 - t, t], 1)
            self._half_space(ids, coef, C.n_ee, self._weights(C.a_ee), x, mov, dh, W, WY)
        if len(C.ob):
            w = self._weights(C.a_ob)
            for j, ob in enumerate(self.obs):
                sel = C.ob[:, 1] == j
                if not sel.any():
                    continue
                v = C.ob[sel, 0]
                phi, o, rad = obstacle_phi(ob, x[v])
                y = x[v].copy()
                inside = (phi < dh) & (rad > 0)
                y[inside] = x[v][inside] - o[inside] + \
                    o[inside] * ((ob.radius + dh) / rad[inside])[:, None]
                np.add.at(W, v, w[sel])
                np.add.at(WY, v, w[sel][:, None] * y)
                if self.p.friction > 0:
                    wf, uT = obstacle_friction(ob, x[v], (self.x if xs is None else xs)[v], w[sel], self.m.h,
                                               dh, self.p.friction, self.p.friction_eps_v)
                    np.add.at(W, v, wf)
                    np.add.at(WY, v, wf[:, None] * (x[v] - uT))
        return W, WY

    @staticmethod
    def _half_space(ids, coef, nrm, w, x, mov, dh, W, WY):
        # g(y) = sum_k c_k n . y_k - d_hat >= 0; minimum-norm correction over movable vertices
        cm = coef * mov[ids]
        gx = np.einsum("pk,pkd,pd->p", coef, x[ids], nrm) - dh
        den = np.einsum("pk,pk->p", cm, cm)
        delta = np.where((gx < 0) & (den > 0), -gx / np.where(den > 0, den, 1.0), 0.0)
        y = x[ids] + cm[:, :, None] * delta[:, None, None] * nrm[:, None, :]
        np.add.at(W, ids.ravel(), np.repeat(w, 4))
        np.add.at(WY, ids.ravel(), (w[:, None, None] * y).reshape(-1, 3))

    def _partial_ccd(self, C: Constraints, xm: np.ndarray, xp: np.ndarray):
        """Life-span update a <- active ? min(a+1, a_max) : 0, active when
        Q(lambda) <= 0 at some sample (Eq. (query)); obstacles: active when
        the end position is closer than d_hat."""
        amax = self.p.a_max
        if len(C.vt):
            lam = np.concatenate([np.broadcast_to(VT_SAMPLES, (len(C.vt), 3, 2)),
                                  C.lam_vt[:, None, :]], axis=1)          # (P,4,2)
            Q = query_vt(xm, xp, C.vt[:, 0], self.m.tris[C.vt[:, 1]], lam)
            act = (Q <= 0).any(1)
            if self.p.adaptive_samples:
                ids = np.concatenate([C.vt[:, :1], self.m.tris[C.vt[:, 1]]], axis=1)
                act = self._refine(act, xm, xp, ids, True, C.lam_vt,
                                   lambda sel, lam: query_vt(xm, xp, C.vt[sel, 0], self.m.tris[C.vt[sel, 1]], lam))
            C.a_vt = np.where(act, np.minimum(C.a_vt + 1, amax), 0).astype(np.int32)
        if len(C.ee):
            lam = np.concatenate([np.broadcast_to(EE_SAMPLES, (len(C.ee), 3, 2)),
                                  C.lam_ee[:, None, :]], axis=1)
            e1, e2 = self.m.edges[C.ee[:, 0]], self.m.edges[C.ee[:, 1]]
            Q = query_ee(xm, xp, e1, e2, lam)
            act = (Q <= 0).any(1)
            if self.p.adaptive_samples:
                ids = np.concatenate([e1, e2], axis=1)
                act = self._refine(act, xm, xp, ids, False, C.lam_ee,
                                   lambda sel, lam: query_ee(xm, xp, e1[sel], e2[sel], lam))
            C.a_ee = np.where(act, np.minimum(C.a_ee + 1, amax), 0).astype(np.int32)
        if len(C.ob):
            act = np.zeros(len(C.ob), bool)
            for j, ob in enumerate(self.obs):
                sel = C.ob[:, 1] == j
                phi, _, _ = obstacle_phi(ob, xp[C.ob[sel, 0]])
                act[sel] = phi < self.p.d_hat
            C.a_ob = np.where(act, np.minimum(C.a_ob + 1, amax), 0).astype(np.int32)

    @staticmethod
    def _refine(act, xm, xp, ids, vt, lam_frozen, query):
        """Adaptive density (end of section 4.1): pairs whose rho* shrank
        (stretch or fast motion) are queried on the refined sample set of
        their level instead of the fixed one (the frozen closest point is
        always a sample)."""
        level = adaptive_level(rho_star_ratio(xm[ids], xp[ids], vt))
        out = act.copy()
        for m in np.unique(level[level > ADAPT_M0]):
            sel = np.flatnonzero(level == m)
            smp = refined_samples(int(m), vt)
            lam = np.concatenate([np.broadcast_to(smp, (len(sel),) + smp.shape), lam_frozen[sel][:, None, :]],
                                 axis=1)
            out[sel] = (query(sel, lam) <= 0).any(1)
        return out

    def _outer_ccd(self, xm: np.ndarray, xp: np.ndarray, prev: Constraints, st: StepStats):
        """Broad phase + full CCD on (x-, x+): returns (s, new constraint set).
        C_o = {candidates with TOI <= 1} U (C_{o-1} intersect candidates);
        surviving entries keep their life span, new ones start at 0."""
        m = self.m
        xm32 = xm.astype(np.float32)
        xp32 = xp.astype(np.float32)
        vt, ee = native.broad_phase(xm32, xp32, m.edges, m.tris, self.p.d_hat, self.p.self_contact)
        tv, te, nf = native.toi_pairs(xm, xp, m.tris, m.edges, vt, ee)
        st.fallbacks += nf
        st.n_candidates = len(vt) + len(ee)
        tmin = min(tv.min(initial=NO_HIT), te.min(initial=NO_HIT))
        C = Constraints()
        C.vt, C.a_vt = _merge(vt, tv <= 1.0, prev.vt, prev.a_vt)
        C.ee, C.a_ee = _merge(ee, te <= 1.0, prev.ee, prev.a_ee)
        obs_rows = []
        for j, ob in enumerate(self.obs):
            toi = obstacle_toi(ob, xm, xp)
            tmin = min(tmin, toi.min(initial=NO_HIT))
            phim, _, _ = obstacle_phi(ob, xm)
            phip, _, _ = obstacle_phi(ob, xp)
            mem = (toi <= 1.0) | (phim < self.p.d_hat) | (phip < self.p.d_hat)
            mem &= self.free
            v = np.flatnonzero(mem).astype(np.int32)
            obs_rows.append(np.stack([v, np.full_like(v, j)], 1))
        ob = np.concatenate(obs_rows) if obs_rows else np.zeros((0, 2), np.int32)
        ob = ob[np.lexsort((ob[:, 1], ob[:, 0]))] if len(ob) else ob
        cand_ob = np.ones(len(ob), bool)
        C.ob, C.a_ob = _merge(ob, cand_ob, prev.ob, prev.a_ob)
        st.min_toi = min(st.min_toi, tmin)
        s = 1.0 if tmin > 1.0 else self.p.alpha * tmin
        return s, C

    def _freeze(self, C: Constraints, xm: np.ndarray):
        C.lam_vt, C.n_vt = native.frozen_vt(xm, self.m.tris, C.vt)
        C.lam_ee, C.n_ee = native.frozen_ee(xm, self.m.edges, C.ee)

    # ---- one implicit step
    def step(self) -> StepStats:
        m, p = self.m, self.p
        h = m.h
        st = StepStats()
        xs = self.x
        # Eq. (z_rf): z = x* + h v* + h^2 (M^{-1} f_ext + M^{-1} delta f), with
        # h^2 M^{-1} delta f = 2 dx forwarded by the previous step
        z = xs + h * self.v + h * h * self.g + 2.0 * self.rf_dx
        z[m.pinned] = self.pin_pos[m.pinned]
        self.rf_dx = np.zeros_like(xs)
        inertia = (m.mass / (h * h))[:, None] * z
        xw = self.warm_start(z, inertia) if p.warm_iters > 0 else z
        xm = xs.copy()
        s, C = self._outer_ccd(xm, xw, Constraints(), st)
        x = xm + s * (xw - xm)
        xm = x.copy()
        self._freeze(C, xm)
        t_exit = NO_HIT
        for o in range(p.iters_outer):
            # outer loop condition (Algorithm 1, section 7): stop once the
            # previous block moved no vertex by tol_outer or more
            if o > 0 and p.tol_outer > 0 and st.outer_dx[-1] < p.tol_outer:
                break
            st.outer_iters += 1
            st.block_iters.append(0)
            xk = x.copy()
            xkm1 = x.copy()
            for k in range(p.iters_inner):
                # inner loop condition: the previous iteration's max change
                if k > 0 and p.tol_inner > 0 and st.dx[-1] < p.tol_inner:
                    break
                xk1 = self.iterate(xk, xkm1, k, C, inertia, xm)
                self._partial_ccd(C, xm, xk1)
                st.dx.append(float(np.linalg.norm(xk1 - xk, axis=1).max()))
                st.inner_iters += 1
                st.block_iters[-1] += 1
                xkm1, xk = xk, xk1
            xp = xk
            st_o = StepStats()
            s, C = self._outer_ccd(xm, xp, C, st_o)
            st.min_toi = min(st.min_toi, st_o.min_toi)
            st.n_candidates = st_o.n_candidates
            st.fallbacks += st_o.fallbacks
            t_exit = st_o.min_toi
            x = xm + s * (xp - xm)
            st.outer_dx.append(float(np.linalg.norm(x - xm, axis=1).max()))
            xm = x.copy()
            self._freeze(C, xm)
        st.n_constraints = len(C.vt) + len(C.ee) + len(C.ob)
        st.t_exit = t_exit
        if p.rf_iters > 0 and t_exit < p.rf_toi:
            self.rf_dx = self.residual_forward(x, C, inertia)
        self.v = (x - xs) / h
        self.x = x
        self.last = st
        return st

    def warm_start(self, z, inertia):
        """Modal warm start (Algorithm 1 before the first full CCD): local
        projections of the elastic terms and the global solve restricted to
        span(Uw), collisions ignored: q = Lw^{-1} Uw^T (b - H x), x += Uw q
        with Lw = Uw^T H Uw (the diagonal of eigenvalues for an exact
        eigenbasis), warm_iters times from x = z."""
        m = self.m
        cf = sla.cho_factor(self.Lw)
        x = z.copy()
        for _ in range(self.p.warm_iters):
            b = inertia + elastic_rhs(m, x)
            r = b - m.H @ x
            r[~self.free] = 0
            x = x + self.Uw @ sla.cho_solve(cf, self.Uw.T @ r)
        return x

    def residual_forward(self, x, C, inertia):
        """Residual forwarding (section 6): with every collision weight at k
        (a = 0, the quadratic approximation of the barrier) and no CCD filter,
        rf_iters inner iterations from x approximate one more Newton-like
        solve; their displacement dx is forwarded as delta f = 2 M dx / h^2,
        i.e. z of the next step gains 2 dx."""
        Crf = Constraints(vt=C.vt, ee=C.ee, ob=C.ob, a_vt=np.zeros_like(C.a_vt), a_ee=np.zeros_like(C.a_ee),
                          a_ob=np.zeros_like(C.a_ob), lam_vt=C.lam_vt, n_vt=C.n_vt, lam_ee=C.lam_ee, n_ee=C.n_ee)
        xk = x.copy()
        xkm1 = x.copy()
        dx_prev = np.inf
        for k in range(self.p.rf_iters):
            # the inner loop condition applies here too (Algorithm 1, end)
            if k > 0 and self.p.tol_inner > 0 and dx_prev < self.p.tol_inner:
                break
            xk1 = self.iterate(xk, xkm1, k, Crf, inertia, x)
            dx_prev = float(np.linalg.norm(xk1 - xk, axis=1).max())
            xkm1, xk = xk, xk1
        dx = xk - x
        dx[~self.free] = 0
        return dx

    def iterate(self, xk, xkm1, k, C, inertia, xm, frozen=None, xs=None):
        """One inner PD iteration from x^k (history x^{k-1}) -> x^{k+1}.
        `frozen` = (b, W) replaces the local step by a fixed right-hand side
        and diagonal (used to check the global solve on its own); xs: the
        step's start for the friction slip (default: the current state)."""
        m, p = self.m, self.p
        free = self.free
        if frozen is None:
            W, WY = self._collision_terms(C, xk, xs)
            b = inertia + elastic_rhs(m, xk) + WY
        else:
            b, W = frozen
        r0 = b - m.H @ xk - W[:, None] * xk
        r0[~free] = 0
        g = self.U.T @ r0
        A = self.Lam + self.U.T @ (W[:, None] * self.U)
        Q = sla.cho_solve(sla.cho_factor(A), g)
        xt = xk + self.U @ Q
        r1 = b - m.H @ xt - W[:, None] * xt
        r1[~free] = 0
        xhat = xt + r1 / (m.diagH + W)[:, None]
        self.trace = dict(r0=r0, g=g, A=A, Q=Q, xt=xt, r1=r1, xhat=xhat, b=b, W=W)
        if p.smoother == "ajacobi2":
            # rank-2 A-Jacobi (sec. 8.1): two Jacobi steps per iteration, each
            # damped by gamma, the first from the subspace-corrected x~
            y1 = xk + p.cheb_gamma * (xhat - xk)
            r2 = b - m.H @ y1 - W[:, None] * y1
            r2[~free] = 0
            return y1 + p.cheb_gamma * r2 / (m.diagH + W)[:, None]
        om = self.omega[min(k, len(self.omega) - 1)]
        return om * (p.cheb_gamma * (xhat - xk) + xk - xkm1) + xkm1


def _merge(cand: np.ndarray, hit: np.ndarray, prev: np.ndarray, prev_a: np.ndarray):
    """Rows of `cand` (sorted) kept when hit or present in `prev`; life spans
    carried over from `prev`, 0 for new rows."""
    if len(cand) == 0:
        return np.zeros((0, 2), np.int32), np.zeros(0, np.int32)
    key = cand[:, 0].astype(np.int64) * (1 << 31) + cand[:, 1]
    pkey = prev[:, 0].astype(np.int64) * (1 << 31) + prev[:, 1] if len(prev) else np.zeros(0, np.int64)
    pos = np.searchsorted(pkey, key)
    pos_c = np.minimum(pos, max(len(pkey) - 1, 0))
    inprev = (len(pkey) > 0) & (pkey[pos_c] == key) if len(pkey) else np.zeros(len(key), bool)
    keep = hit | inprev
    a = np.where(inprev, prev_a[pos_c] if len(pkey) else 0, 0)
    return cand[keep].astype(np.int32), a[keep].astype(np.int32)
