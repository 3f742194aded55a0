"""Builders shared by the tests: the same seeded scene on both sides.

The oracle computes the rest eigenbasis from its own system matrix; that
FP64 basis is handed to both sides, and each rounds it to the storage
precision itself.  Chebyshev parameters come from the oracle's estimate and
are passed to both sides explicitly, as is the contact weight k.
"""
import numpy as np

from oracle import model as M
from oracle import step as S

K_CONTACT = 100.0


def oracle_side(sc, precision, gamma=0.9, k_contact=K_CONTACT, rho=None, iters_inner=None,
                iters_outer=None, U=None, sigma=(1.0, 1.0), tol=(0.0, 0.0)):
    m = M.build_model(sc.tris, sc.rest, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend,
                      k_contact=k_contact, sigma_min=sigma[0], sigma_max=sigma[1])
    if U is None:
        _, U = M.eigenbasis(m, sc.r)
    Us = M.stored_basis(U, precision)
    if rho is None:
        rho = min(0.999 * M.spectral_radius(m, Us, gamma, 150), 0.999)
    p = S.Params(iters_outer=iters_outer or sc.iters_outer, iters_inner=iters_inner or sc.iters_inner,
                 cheb_rho=rho, cheb_gamma=gamma, cheb_delay=3, d_hat=sc.d_hat,
                 self_contact=sc.self_contact, tol_inner=tol[0], tol_outer=tol[1])
    obs = [S.Obst(o.kind, np.array(o.center, float), o.radius, np.array(o.axis, float))
           for o in sc.obstacles]
    o = S.Oracle(m, Us, p, sc.gravity, obs)
    o.set_state(sc.x0, sc.v0)
    return o, U, rho


def gpu_side(sc, U, precision, rho, gamma=0.9, k_contact=K_CONTACT, iters_inner=None,
             iters_outer=None, pair_capacity=0, **kw):
    import paper_2403_19272_amd as P
    prec = P.CLOTH_MIXED if precision == "mixed" else P.CLOTH_PLAIN_FP32
    g = P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                     k_bend=sc.k_bend, k_contact=k_contact, d_hat=sc.d_hat, pinned=sc.pinned,
                     r=sc.r, iters_inner=iters_inner or sc.iters_inner,
                     iters_outer=iters_outer or sc.iters_outer, cheb_rho=rho, cheb_gamma=gamma,
                     cheb_delay=3, precision=prec, self_contact=sc.self_contact,
                     pair_capacity=pair_capacity, **kw)
    for ob in sc.obstacles:
        g.add_obstacle(ob.kind, ob.center, ob.radius, axis=ob.axis, half_length=ob.half_length,
                       omega=ob.omega)
    g.set_basis(U)
    g.set_state(sc.x0, sc.v0)
    return g


def bbox_diag(x):
    return float(np.linalg.norm(x.max(0) - x.min(0)))
