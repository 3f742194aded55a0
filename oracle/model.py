"""Oracle precompute: rest data, lumped mass, the PD system matrix and the
rest-shape eigenbasis, all in FP64 (TEST INFRASTRUCTURE ONLY).

Follows the paper's projective-dynamics setting (section 3):
  * implicit Euler as an energy, Eq. (var), with z from Eq. (z);
  * per-element projections, Eq. (local), and the global system, Eq. (global):
        H = M/h^2 + sum_i w_i S_i^T A_i^T A_i S_i.
Element models (the paper only says "a differential operator computing the
deformation gradient of a triangle"): triangle strain with the deformation
gradient F = D_s D_m^{-1} projected onto rotations, weight k_stretch * area;
hinge bending with the cotangent edge stencil of quadratic bending, weight
k_bend * 3 / (A_1 + A_2).  Lumped mass: density * area / 3 per corner.
The subspace U (section 5): the r eigenvectors of H restricted to the free
vertices with smallest eigenvalues, zero on pinned rows.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def unique_edges(tris: np.ndarray) -> np.ndarray:
    """Undirected edges (i < j), sorted lexicographically."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def hinges(tris: np.ndarray) -> np.ndarray:
    """Interior edges as rows (x0, x1, x2, x3): the edge (x0 < x1) and the
    opposite vertices of its two triangles, x2 in the lower-index triangle.
    Sorted by edge."""
    tris = np.asarray(tris, np.int64)
    T = tris.shape[0]
    a = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    b = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    o = np.concatenate([tris[:, 2], tris[:, 0], tris[:, 1]])
    t = np.concatenate([np.arange(T)] * 3)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.lexsort((t, hi, lo))
    lo, hi, o = lo[order], hi[order], o[order]
    same = (lo[1:] == lo[:-1]) & (hi[1:] == hi[:-1])
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold edge")
    i = np.flatnonzero(same)
    return np.stack([lo[i], hi[i], o[i], o[i + 1]], 1).astype(np.int64).reshape(-1, 4)


def triangle_rest(X: np.ndarray, tris: np.ndarray):
    """Per triangle: rest area and the corner gradient vectors g_c (2-vectors)
    with F = sum_c x_c g_c^T = D_s D_m^{-1}, D_m holding the rest edges in an
    in-plane orthonormal frame (u1 along the first edge, u2 = n x u1)."""
    P = X[tris]
    e1 = P[:, 1] - P[:, 0]
    e2 = P[:, 2] - P[:, 0]
    nrm = np.cross(e1, e2)
    a2 = np.linalg.norm(nrm, axis=1)
    area = 0.5 * a2
    n = nrm / a2[:, None]
    u1 = e1 / np.linalg.norm(e1, axis=1)[:, None]
    u2 = np.cross(n, u1)
    Dm = np.empty((len(tris), 2, 2))
    Dm[:, 0, 0] = np.einsum("ij,ij->i", e1, u1)
    Dm[:, 0, 1] = np.einsum("ij,ij->i", e2, u1)
    Dm[:, 1, 0] = np.einsum("ij,ij->i", e1, u2)
    Dm[:, 1, 1] = np.einsum("ij,ij->i", e2, u2)
    Dminv = np.linalg.inv(Dm)
    g = np.empty((len(tris), 3, 2))
    g[:, 1] = Dminv[:, 0]
    g[:, 2] = Dminv[:, 1]
    g[:, 0] = -Dminv[:, 0] - Dminv[:, 1]
    return area, g


def _cot(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """cot of the angle between rows of a and b."""
    return np.einsum("ij,ij->i", a, b) / np.linalg.norm(np.cross(a, b), axis=1)


def hinge_rest(X: np.ndarray, hg: np.ndarray, area_of_pair=None):
    """Cotangent stencil K (4 coefficients on x0..x3) and rest areas sum per
    hinge; K annihilates affine fields of the flat rest hinge."""
    p0, p1, p2, p3 = X[hg[:, 0]], X[hg[:, 1]], X[hg[:, 2]], X[hg[:, 3]]
    cA0 = _cot(p1 - p0, p2 - p0)   # angle at x0 in triangle (x0, x1, x2)
    cA1 = _cot(p0 - p1, p2 - p1)   # angle at x1 in triangle (x0, x1, x2)
    cB0 = _cot(p1 - p0, p3 - p0)
    cB1 = _cot(p0 - p1, p3 - p1)
    K = np.stack([cA1 + cB1, cA0 + cB0, -cA0 - cA1, -cB0 - cB1], 1)
    aA = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)
    aB = 0.5 * np.linalg.norm(np.cross(p1 - p0, p3 - p0), axis=1)
    return K, aA + aB


@dataclass
class Model:
    nv: int
    tris: np.ndarray
    edges: np.ndarray
    hinges: np.ndarray
    rest: np.ndarray          # FP64
    pinned: np.ndarray        # bool
    h: float
    mass: np.ndarray
    area: np.ndarray
    g: np.ndarray             # (T,3,2)
    w_tri: np.ndarray
    K: np.ndarray             # (E_h,4)
    w_hinge: np.ndarray
    rest_bend: np.ndarray     # |sum_k K_k X_k| per hinge (0 for flat)
    H: sp.csr_matrix          # scalar N x N
    diagH: np.ndarray
    k_contact: float
    sigma_min: float = 1.0    # strain limits of the triangle projection
    sigma_max: float = 1.0


def build_model(tris, rest, pinned, dt, density, k_stretch, k_bend, k_contact=0.0, sigma_min=1.0,
                sigma_max=1.0) -> Model:
    tris = np.asarray(tris, np.int64)
    X = np.asarray(rest, np.float64)
    nv = X.shape[0]
    pinned = np.asarray(pinned).astype(bool) if pinned is not None else np.zeros(nv, bool)
    area, g = triangle_rest(X, tris)
    w_tri = k_stretch * area
    mass = np.zeros(nv)
    np.add.at(mass, tris.ravel(), np.repeat(density * area / 3.0, 3))
    hg = hinges(tris)
    K, asum = hinge_rest(X, hg, None)
    w_h = k_bend * 3.0 / asum
    rb = np.linalg.norm(np.einsum("ek,ekd->ed", K, X[hg]), axis=1)
    scale = np.abs(K).sum(1) * np.abs(X[hg] - X[hg[:, :1]]).max(axis=(1, 2))
    rb[rb <= 1e-12 * scale] = 0.0
    h2 = 1.0 / (dt * dt)
    rows = [np.arange(nv)]
    cols = [np.arange(nv)]
    vals = [mass * h2]
    # triangles: w g_a . g_c on (a, c)
    gg = np.einsum("tad,tcd->tac", g, g) * w_tri[:, None, None]
    rows.append(np.repeat(tris, 3, axis=1).ravel())
    cols.append(np.tile(tris, (1, 3)).ravel())
    vals.append(gg.ravel())
    # hinges: w K_a K_c
    kk = np.einsum("ea,ec->eac", K, K) * w_h[:, None, None]
    rows.append(np.repeat(hg, 4, axis=1).ravel())
    cols.append(np.tile(hg, (1, 4)).ravel())
    vals.append(kk.ravel())
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nv, nv)).tocsr()
    H.sum_duplicates()
    H.sort_indices()
    diagH = H.diagonal().copy()
    free = ~pinned
    if k_contact <= 0:
        k_contact = float((diagH - mass * h2)[free].mean())
    return Model(nv=nv, tris=tris.astype(np.int32), edges=unique_edges(tris), hinges=hg,
                 rest=X, pinned=pinned, h=dt, mass=mass, area=area, g=g, w_tri=w_tri, K=K,
                 w_hinge=w_h, rest_bend=rb, H=H, diagH=diagH, k_contact=float(k_contact),
                 sigma_min=float(sigma_min), sigma_max=float(sigma_max))


def eigenbasis(model: Model, r: int, dense_limit: int = 4096):
    """The r smallest eigenpairs of H on the free vertices (FP64); U has zero
    rows at pinned vertices and orthonormal columns."""
    free = np.flatnonzero(~model.pinned)
    Hff = model.H[free][:, free]
    if len(free) <= dense_limit:
        lam, V = np.linalg.eigh(Hff.toarray())
        lam, V = lam[:r], V[:, :r]
    else:
        lam, V = spla.eigsh(Hff.tocsc(), k=r, sigma=0.0, which="LM")
        o = np.argsort(lam)
        lam, V = lam[o], V[:, o]
    U = np.zeros((model.nv, r))
    U[free] = V
    return lam, U


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to bfloat16 (through FP32, round to nearest even),
    returned as FP64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def stored_basis(U: np.ndarray, precision: str) -> np.ndarray:
    """The basis values the solver stores: FP32 ("fp32") or BF16 ("mixed")."""
    if precision == "fp32":
        return U.astype(np.float32).astype(np.float64)
    if precision == "mixed":
        return round_bf16(U)
    if precision == "fp64":
        return np.array(U, np.float64)
    raise ValueError(precision)


def reduced_matrix(model: Model, Us: np.ndarray) -> np.ndarray:
    """Lambda~ = Us^T H Us in FP64 (diagonal when Us are exact eigenvectors)."""
    return Us.T @ (model.H @ Us)


def spectral_radius(model: Model, Us: np.ndarray, gamma: float, iters: int = 200,
                    seed: int = 0) -> float:
    """Power-iteration estimate of the spectral radius of the error operator
    of one coarse-corrected, damped Jacobi sweep at rest (no contact):
        E = (I - gamma D^{-1} H)(I - Us A^{-1} Us^T H)   on free rows."""
    rng = np.random.default_rng(seed)
    free = ~model.pinned
    A = reduced_matrix(model, Us)
    cf = sla.cho_factor(A)
    e = rng.standard_normal(model.nv)
    e[~free] = 0
    lam = 0.0
    for _ in range(iters):
        e = e - Us @ sla.cho_solve(cf, Us.T @ (model.H @ e))
        e = e - gamma * (model.H @ e) / model.diagH
        e[~free] = 0
        nrm = np.linalg.norm(e)
        lam = nrm
        e /= nrm
    return float(lam)
