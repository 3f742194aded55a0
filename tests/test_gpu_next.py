"""GPU parity of the optional parts of Algorithm 1: the modal warm start and
residual forwarding (MI355X only)."""
import numpy as np
import pytest

import scenegen
from helpers import bbox_diag, gpu_side, oracle_side

pytestmark = pytest.mark.gpu


def vertex_err(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64), axis=1).max())


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_warm_start_hanging_cloth(precision):
    sc = scenegen.config(0)
    o, U, rho = oracle_side(sc, precision)
    o.p.warm_iters = 3
    g = gpu_side(sc, U, precision, rho)
    g.set_step_options(warm_iters=3)
    for _ in range(sc.steps):
        o.step()
        g.step(sc.gravity)
    x, _ = g.get_state()
    err = vertex_err(x, o.x) / bbox_diag(o.x)
    print(f"[warm {precision}] err/diag={err:.3e}", flush=True)
    assert err <= 1e-5


def test_residual_forwarding_after_a_filtered_step():
    """A cloth 1.5 mm above a sphere falling at 2 m/s: the exiting filter cuts
    the step (t_TOI about 0.49 < rf_toi), the forwarded dx and the next step
    agree."""
    sc = scenegen.drop_cloth(20, seed=9, obstacle="sphere", r=8, steps=2, drop=0.0015, d_hat=1e-3,
                             iters_outer=2, iters_inner=5)
    sc.v0[:] = np.array([0.0, -2.0, 0.0], np.float32)
    o, U, rho = oracle_side(sc, "fp32", gamma=0.6)
    o.p.rf_iters, o.p.rf_toi = 4, 1.5
    g = gpu_side(sc, U, "fp32", rho, gamma=0.6)
    g.set_step_options(rf_iters=4, rf_toi=1.5)
    st_o = o.step()
    st_g = g.step(sc.gravity)
    x, _ = g.get_state()
    diag = bbox_diag(o.x)
    print(f"[rf] t_exit={st_o.t_exit:.4f} min_toi={st_g['min_toi']:.4f} cons={st_o.n_constraints}/"
          f"{st_g['n_constraints']} |dx_rf|={np.abs(o.rf_dx).max():.3e}", flush=True)
    assert st_o.t_exit < 1.5 and np.abs(o.rf_dx).max() > 0
    assert vertex_err(x, o.x) / diag <= 1e-5
    assert vertex_err(g.forwarded(), o.rf_dx) / diag <= 1e-5
    o.step()
    g.step(sc.gravity)
    x, _ = g.get_state()
    assert vertex_err(x, o.x) / diag <= 1e-5


def warm_pair(sc, precision, r_warm, warm_iters, rho=None, gamma=0.9):
    """Oracle and library scenes whose warm start has its own r_warm-mode
    basis (the oracle's eigenvectors, the same FP64 values on both sides)."""
    from oracle import model as M
    from oracle import step as S
    o, U, rho = oracle_side(sc, precision, rho=rho, gamma=gamma)
    _, Uw = M.eigenbasis(o.m, r_warm)
    o2 = S.Oracle(o.m, M.stored_basis(U, precision), o.p, sc.gravity, o.obs, Uw=M.stored_basis(Uw, precision))
    o2.set_state(sc.x0, sc.v0)
    o2.p.warm_iters = warm_iters
    g = gpu_side(sc, U, precision, rho, gamma=gamma, r_warm=r_warm)
    g.set_warm_basis(Uw)
    g.set_step_options(warm_iters=warm_iters)
    return o2, g


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_warm_start_with_a_wider_basis_hanging_cloth(precision):
    """Hanging cloth, warm start in 32 modes against 16 for the reuse (the
    paper's 120 | 30 split of section 8.1, scaled)."""
    sc = scenegen.config(0)
    o, g = warm_pair(sc, precision, r_warm=32, warm_iters=3)
    for _ in range(sc.steps):
        o.step()
        g.step(sc.gravity)
    x, _ = g.get_state()
    err = vertex_err(x, o.x) / bbox_diag(o.x)
    print(f"[warm r_warm=32 {precision}] err/diag={err:.3e}", flush=True)
    assert err <= 1e-5


def test_warm_start_with_a_wider_basis_on_contact():
    """A cloth falling onto a sphere with self contact, warm start in 24
    modes against 8: the warm-started predictor feeds the first full CCD."""
    sc = scenegen.drop_cloth(20, seed=9, obstacle="sphere", r=8, steps=3, drop=0.0015, d_hat=1e-3,
                             iters_outer=2, iters_inner=5)
    sc.v0[:] = np.array([0.0, -2.0, 0.0], np.float32)
    o, g = warm_pair(sc, "fp32", r_warm=24, warm_iters=3, gamma=0.6)
    diag = None
    for s in range(sc.steps):
        so = o.step()
        sg = g.step(sc.gravity)
        x, _ = g.get_state()
        diag = diag or bbox_diag(o.x)
        err = vertex_err(x, o.x) / diag
        print(f"[warm contact] step {s} constraints {so.n_constraints}/{sg['n_constraints']} err/diag={err:.2e}",
              flush=True)
        assert err <= 1e-5
    assert sg["n_constraints"] > 0


def _shuffled(sc, seed):
    """The same scene with its vertices renumbered at random: natural vertex
    i becomes shuf[i]; returns the scene and inv (caller j = natural inv[j])."""
    import dataclasses
    rng = np.random.default_rng(seed)
    shuf = rng.permutation(sc.nv)
    inv = np.argsort(shuf)
    sc2 = dataclasses.replace(sc, tris=shuf[sc.tris].astype(np.int32), rest=sc.rest[inv], x0=sc.x0[inv],
                              v0=sc.v0[inv], pinned=sc.pinned[inv])
    return sc2, inv


def test_reordered_scene_matches_the_natural_order():
    """The small hanging cloth (corners pinned, no contact) with shuffled
    vertex numbers, stepped with the vertex reorder on, gives in the
    caller's numbering the natural-order scene's result to FP32 rounding
    after 10 steps: positions, velocities, pins, the basis and H cross the
    boundary in the caller's order.  With contact the two differ beyond
    rounding once a near-threshold contact decision flips (summation orders
    differ), so there only the outcome is checked.  The stage-level calls
    refuse a reordered scene."""
    import paper_2403_19272_amd as P
    sc = scenegen.config(0)
    o, U, rho = oracle_side(sc, "fp32")
    sc2, inv = _shuffled(sc, 9)
    assert sc2.pinned.sum() == 2 and not np.array_equal(sc2.pinned, sc.pinned)
    a = gpu_side(sc, U, "fp32", rho)
    b = gpu_side(sc2, U[inv], "fp32", rho, reorder=True)
    Ha, Hb = a.system_matrix(), b.system_matrix()
    assert abs(Hb - Ha[inv][:, inv]).max() <= 1e-12 * abs(Ha).max()
    for s in range(sc.steps):
        a.step(sc.gravity)
        b.step(sc.gravity)
    xa, va = a.get_state()
    xb, vb = b.get_state()
    diag = np.linalg.norm(xa.max(0) - xa.min(0))
    err = np.linalg.norm(xb - xa[inv], axis=1).max() / diag
    moved = np.linalg.norm(xa - sc.x0, axis=1).max() / diag
    print(f"[reorder] err/diag={err:.2e} moved/diag={moved:.2e}", flush=True)
    assert moved > 5e-3 and err <= 1e-5
    assert np.array_equal(xb[sc2.pinned == 1], sc2.x0[sc2.pinned == 1])
    with pytest.raises(P.ClothError) as e:
        b.stage_partial_ccd(xb)
    assert e.value.code == P.CLOTH_E_INVALID
    # a contact scene: the reordered steps stay finite and in contact
    cc = scenegen.drop_cloth(48, seed=31, obstacle="cylinder", r=16, steps=3, d_hat=1e-3, side=47 / 127.0)
    oc, Uc, _ = oracle_side(cc, "mixed", rho=0.95, gamma=0.6)
    cc2, inv2 = _shuffled(cc, 11)
    g = gpu_side(cc2, Uc[inv2], "mixed", 0.95, gamma=0.6, reorder=True)
    x0 = scenegen.draped_state(cc, seed=5)[inv2]
    g.set_state(x0, np.zeros_like(x0))
    st = g.step(cc.gravity, n=3)
    x, v = g.get_state()
    assert np.isfinite(x).all() and st["n_constraints"] > 0


def test_reorder_restores_sweep_speed_on_a_shuffled_grid():
    """Timing only (printed): a 256 x 256 grid with shuffled numbering,
    stepped in free fall with and without the reorder, beside the natural
    order; the reordered scene matches the natural one to FP32 rounding."""
    import time

    import paper_2403_19272_amd as P
    sc = scenegen.drop_cloth(256, seed=1, obstacle="sphere", r=64, steps=3, d_hat=1e-3)
    sc2, inv = _shuffled(sc, 10)

    def make(s, **kw):
        g = P.ClothScene(s.tris, s.rest, dt=s.dt, density=s.density, k_stretch=s.k_stretch, k_bend=s.k_bend,
                         d_hat=s.d_hat, r=s.r, iters_inner=10, iters_outer=3, cheb_rho=0.99, cheb_gamma=0.6,
                         precision=P.CLOTH_MIXED, self_contact=True, **kw)
        return g

    nat = make(sc)
    U = nat.compute_basis(degree=200, max_passes=8, tol=5e-2, return_basis=True)["U"]
    shuf, reo = make(sc2), make(sc2, reorder=True)
    for g in (shuf, reo):
        g.set_basis(U[inv])
    times = {}
    for name, g, x0 in (("natural", nat, sc.x0), ("shuffled", shuf, sc2.x0), ("reordered", reo, sc2.x0)):
        g.set_state(x0, np.zeros_like(x0))
        g.step(sc.gravity, n=2)   # (reading the statistics waits for the steps)
        t0 = time.perf_counter()
        g.step(sc.gravity, n=5)
        times[name] = (time.perf_counter() - t0) / 5 * 1e3
    print("[reorder timing] ms/step " + " ".join(f"{k} {v:.3f}" for k, v in times.items()), flush=True)
    xn, _ = nat.get_state()
    xr, _ = reo.get_state()
    err = np.linalg.norm(xr - xn[inv], axis=1).max() / np.linalg.norm(xn.max(0) - xn.min(0))
    assert err <= 1e-5


def test_spinning_cylinder_drags_the_cloth_with_friction():
    """Lagged obstacle friction on the device against the oracle: a small
    flat cloth laid half d_hat above the top line of a cylinder spinning at
    2 rad/s (self contact off), 4 steps of 2 x 6 iterations.  With friction
    the cloth picks up the surface's velocity along +z, and the positions
    match the oracle's to FP32 rounding; without friction it does not move
    along z."""
    import paper_2403_19272_amd as P
    from oracle import model as M
    from oracle import step as S
    sc = scenegen.drop_cloth(9, seed=2, obstacle="cylinder", r=8, steps=4, drop=0.0, d_hat=1e-3, side=0.05,
                             iters_outer=2, iters_inner=6)
    ob = sc.obstacles[0]
    x0 = sc.rest.astype(np.float64).copy()
    x0[:, 1] = ob.radius + 0.5e-3
    x0 = x0.astype(np.float32)
    m = M.build_model(sc.tris, x0, sc.pinned, sc.dt, sc.density, sc.k_stretch, sc.k_bend)
    _, U = M.eigenbasis(m, sc.r)
    out = {}
    for mu in (0.0, 0.6):
        p = S.Params(iters_outer=2, iters_inner=6, cheb_rho=0.9, cheb_gamma=0.6, d_hat=sc.d_hat,
                     self_contact=False, friction=mu)
        o = S.Oracle(m, M.stored_basis(U, "fp32"), p, sc.gravity,
                     [S.Obst(ob.kind, np.array(ob.center, float), ob.radius, np.array(ob.axis, float), omega=2.0)])
        o.set_state(x0, np.zeros_like(x0))
        g = P.ClothScene(sc.tris, x0, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch, k_bend=sc.k_bend,
                         k_contact=m.k_contact, d_hat=sc.d_hat, r=sc.r, iters_inner=6, iters_outer=2,
                         cheb_rho=0.9, cheb_gamma=0.6, cheb_delay=3, precision=P.CLOTH_PLAIN_FP32,
                         self_contact=False, friction=mu)
        g.add_obstacle(ob.kind, ob.center, ob.radius, axis=ob.axis, half_length=ob.half_length, omega=2.0)
        g.set_basis(U)
        g.set_state(x0, np.zeros_like(x0))
        for _ in range(sc.steps):
            o.step()
            g.step(sc.gravity)
        x, v = g.get_state()
        diag = bbox_diag(o.x)
        err = float(np.linalg.norm(x - o.x, axis=1).max()) / diag
        out[mu] = (float(v[:, 2].mean()), float(o.v[:, 2].mean()), err)
        print(f"[friction mu={mu}] vz gpu {out[mu][0]:.5f} oracle {out[mu][1]:.5f} err/diag {err:.2e}", flush=True)
        g.close()
    assert abs(out[0.0][0]) < 1e-4 and out[0.6][0] > 0.01   # (v = dx / h carries FP32 noise x 200)
    assert out[0.6][2] <= 1e-5 and out[0.0][2] <= 1e-5
    assert abs(out[0.6][0] - out[0.6][1]) <= 0.02 * out[0.6][1]
