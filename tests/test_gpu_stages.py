"""GPU parity of the contact stages on the paths and sizes the other tests
leave out (MI355X only):

  * the sampled TOI fallback: a cloth moving in its own plane makes every
    coplanarity cubic vanish identically, so every pair takes the sampled
    fallback, more per chunk than the wavefront queue holds;
  * the outer stage at full size (600 x 600) from a state lying on the
    cylinder, with jittered end positions so that self-contact pairs arise,
    and a carried constraint set: sets and spans bit-exact, step length
    within 1e-6;
  * the sphere drape (256 x 256): per-stage parity at a shared mid-run state
    and no intersecting triangles after any step;
  * the cylinder drape (600 x 600) from the 0.3 m drop through its
    contact steps: no intersecting triangles (exact check every 10th step
    and the last, the device check after every step).
"""
import numpy as np
import pytest

import scenegen
from helpers import bbox_diag, gpu_side, oracle_side
from oracle import exact, native
from oracle import model as M
from oracle import step as S

pytestmark = pytest.mark.gpu


def vertex_err(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64), axis=1).max())


def test_sampled_toi_fallback_in_plane_motion():
    n = 24
    sc = scenegen.drop_cloth(n, seed=5, obstacle="sphere", r=8, steps=1, d_hat=1e-3)
    rng = np.random.default_rng(5)
    xm = sc.rest.copy()
    h = 1.0 / (n - 1)
    xp = xm.copy()
    xp[:, 0] += rng.normal(0, 0.6 * h, sc.nv).astype(np.float32)
    xp[:, 2] += rng.normal(0, 0.6 * h, sc.nv).astype(np.float32)
    edges = M.unique_edges(sc.tris)
    vt, ee = native.broad_phase(xm, xp, edges, sc.tris, sc.d_hat)
    otv, ote, nf = native.toi_pairs(xm.astype(np.float64), xp.astype(np.float64), sc.tris, edges, vt, ee)
    o, U, rho = oracle_side(sc, "fp32", rho=0.9)
    g = gpu_side(sc, U, "fp32", 0.9)
    tv, te = g.stage_toi(xm, xp, vt, ee)
    print(f"[toi fallback] pairs {len(vt)}+{len(ee)} fallbacks {nf} hits {(otv <= 1).sum()}+{(ote <= 1).sum()}",
          flush=True)
    assert nf == len(vt) + len(ee) and nf > 32 * 8   # every pair; beyond the per-chunk queue
    assert (otv <= 1).sum() > 100 and (ote <= 1).sum() > 100
    assert np.array_equal(tv <= 1, otv <= 1) and np.array_equal(te <= 1, ote <= 1)
    h1 = otv <= 1
    assert np.abs(tv[h1] - otv[h1]).max() <= 1e-6
    h1 = ote <= 1
    assert np.abs(te[h1] - ote[h1]).max() <= 1e-6


def drape_state(sc, U, steps, precision):
    """The library's own state after `steps` steps from the seeded drop
    (library Chebyshev estimate), for stage inputs."""
    import paper_2403_19272_amd as P
    g = P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                     k_bend=sc.k_bend, d_hat=sc.d_hat, r=sc.r, iters_inner=sc.iters_inner,
                     iters_outer=sc.iters_outer, precision=P.CLOTH_MIXED if precision == "mixed" else P.CLOTH_PLAIN_FP32,
                     self_contact=True)
    ob = sc.obstacles[0]
    g.add_obstacle(ob.kind, ob.center, ob.radius, axis=ob.axis, half_length=ob.half_length, omega=ob.omega)
    g.set_basis(U)
    g.set_state(sc.x0, sc.v0)
    return g


def outer_pair(o, g, xm, xp, prev, first, nob=1):
    """One outer stage on both sides; returns (gpu set, oracle set, s's)."""
    if not first:
        ob_a = np.full((nob, o.m.nv), -1, np.int32)
        ob_a[prev.ob[:, 1], prev.ob[:, 0]] = prev.a_ob
        g.stage_load_block(xm, xm, xm, xm, prev.vt, prev.a_vt, prev.ee, prev.a_ee, ob_a)
    x_gpu, s_gpu = g.stage_outer(xm, xp, first)
    got = g.stage_read_set(nob=nob, cap=8 * o.m.nv)
    s_or, C = o._outer_ccd(xm.astype(np.float64), xp.astype(np.float64), S.Constraints() if first else prev,
                           S.StepStats())
    return x_gpu, s_gpu, got, s_or, C


def assert_same_set(got, C, nv):
    assert np.array_equal(got["vt"], C.vt) and np.array_equal(got["a_vt"], C.a_vt)
    assert np.array_equal(got["ee"], C.ee) and np.array_equal(got["a_ee"], C.a_ee)
    ob = np.full(nv, -1, np.int32)
    ob[C.ob[:, 0]] = C.a_ob
    assert np.array_equal(got["ob_a"][0], ob)


def test_full_size_outer_stage_past_first_contact():
    from paper_2403_19272_amd import basis as B
    sc = scenegen.config(2)
    import paper_2403_19272_amd as P
    probe = P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                         k_bend=sc.k_bend, r=sc.r, iters_inner=1, iters_outer=1, cheb_rho=0.9, cheb_gamma=0.5)
    U = B.rest_eigenbasis(probe.system_matrix(), sc.pinned, sc.r)
    probe.close()
    g = drape_state(sc, U, 0, "mixed")
    g.step(sc.gravity, n=70, stats=False)
    st = g.step(sc.gravity, n=0)
    x, v = g.get_state()
    assert st["n_constraints"] > 1000    # lying on the cylinder
    # the drape itself makes no self contact within its 200 steps (the
    # flaps hang apart), so the end positions get an in-plane jitter of
    # about half an edge: neighbouring triangles and edges then cross
    rng = np.random.default_rng(14)
    xm = x
    xp = (x + sc.dt * v + sc.dt ** 2 * np.array(sc.gravity, np.float32)
          + rng.normal(0, 8e-4, x.shape)).astype(np.float32)
    o, _, _ = oracle_side(sc, "mixed", rho=0.95, U=U)
    # first stage of a step, then a second stage carrying the first one's
    # set with drawn life spans
    x1, s1, got1, s1o, C1 = outer_pair(o, g, xm, xp, None, True)
    print(f"[full outer] first: s={s1:.6f}/{s1o:.6f} vt={len(C1.vt)} ee={len(C1.ee)} ob={len(C1.ob)}", flush=True)
    assert len(C1.vt) + len(C1.ee) > 1000 and len(C1.ob) > 1000
    assert_same_set(got1, C1, sc.nv)
    assert abs(s1 - s1o) <= 1e-6
    C1.a_vt = rng.integers(0, 21, len(C1.vt)).astype(np.int32)
    C1.a_ee = rng.integers(0, 21, len(C1.ee)).astype(np.int32)
    C1.a_ob = rng.integers(0, 21, len(C1.ob)).astype(np.int32)
    xm2 = x1
    xp2 = (xp + rng.normal(0, 3e-4, x.shape)).astype(np.float32)
    x2, s2, got2, s2o, C2 = outer_pair(o, g, xm2, xp2, C1, False)
    carried = int((C2.a_vt > 0).sum() + (C2.a_ee > 0).sum() + (C2.a_ob > 0).sum())
    print(f"[full outer] second: s={s2:.6f}/{s2o:.6f} vt={len(C2.vt)} ee={len(C2.ee)} ob={len(C2.ob)} "
          f"carried={carried}", flush=True)
    assert carried > 100
    assert_same_set(got2, C2, sc.nv)
    assert abs(s2 - s2o) <= 1e-6
    x2o = xm2.astype(np.float64) + s2o * (xp2.astype(np.float64) - xm2)
    assert vertex_err(x2, x2o) <= 1e-6 * bbox_diag(x2o)


def test_sphere_drape_stages_and_no_tangles():
    """256 x 256 cloth onto the sphere, the bench's solver settings: no
    intersecting triangles after any of 100 steps; at step 70 the broad
    phase, the TOI, the outer stage and one inner iteration match the oracle
    on the shared state."""
    from paper_2403_19272_amd import basis as B
    sc = scenegen.config(1)
    import paper_2403_19272_amd as P
    probe = P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                         k_bend=sc.k_bend, r=sc.r, iters_inner=1, iters_outer=1, cheb_rho=0.9, cheb_gamma=0.5)
    U = B.rest_eigenbasis(probe.system_matrix(), sc.pinned, sc.r)
    probe.close()
    g = drape_state(sc, U, 0, "fp32")
    assert exact.count_tangles(sc.x0, sc.tris) == 0
    mid = None
    for s in range(sc.steps):
        st = g.step(sc.gravity)
        x, v = g.get_state()
        assert np.isfinite(x).all()
        nt = exact.count_tangles(x, sc.tris)
        if s % 10 == 9:
            print(f"[sphere drape] step {s + 1} constraints={st['n_constraints']} min_toi={st['min_toi']:.3f} "
                  f"tangles={nt}", flush=True)
        assert nt == 0, s
        if s + 1 == 70:
            mid = (x.copy(), v.copy(), st)
    assert st["n_constraints"] > 0
    x, v, st = mid
    assert st["n_constraints"] > 0
    # stage parity at the shared state, with a fresh scene and the oracle
    o, _, rho = oracle_side(sc, "fp32", rho=0.97, gamma=0.5, U=U)
    g2 = gpu_side(sc, U, "fp32", rho, gamma=0.5)
    xp = (x + sc.dt * v + sc.dt ** 2 * np.array(sc.gravity, np.float32)).astype(np.float32)
    vt, ee = g2.stage_broad_phase(x, xp, cap=64 * sc.nv)
    ovt, oee = native.broad_phase(x, xp, o.m.edges, o.m.tris, sc.d_hat, cap=64 * sc.nv)
    assert len(ovt) > 0 and np.array_equal(vt, ovt) and np.array_equal(ee, oee)
    tv, te = g2.stage_toi(x, xp, vt, ee)
    otv, ote, _ = native.toi_pairs(x.astype(np.float64), xp.astype(np.float64), o.m.tris, o.m.edges, vt, ee)
    assert np.array_equal(tv <= 1, otv <= 1) and np.array_equal(te <= 1, ote <= 1)
    assert np.abs(tv[otv <= 1] - otv[otv <= 1]).max(initial=0) <= 1e-6
    assert np.abs(te[ote <= 1] - ote[ote <= 1]).max(initial=0) <= 1e-6
    x1, s1, got, s1o, C = outer_pair(o, g2, x, xp, None, True)
    assert_same_set(got, C, sc.nv)
    assert abs(s1 - s1o) <= 1e-6
    # one inner iteration on the new set from the filtered state
    C.a_vt = np.random.default_rng(3).integers(0, 21, len(C.vt)).astype(np.int32)
    C.a_ee = np.random.default_rng(4).integers(0, 21, len(C.ee)).astype(np.int32)
    ob_a = np.full((1, sc.nv), -1, np.int32)
    ob_a[0, C.ob[:, 0]] = C.a_ob
    xm = x1
    xk = x1
    z = xp
    g2.stage_load_block(xm, xk, xk, z, C.vt, C.a_vt, C.ee, C.a_ee, ob_a)
    g2.stage_inner(0)
    res = g2.stage_read_block(nob=1)
    o._freeze(C, xm.astype(np.float64))
    inertia = (o.m.mass / o.m.h ** 2)[:, None] * z.astype(np.float64)
    xk1 = o.iterate(xk.astype(np.float64), xk.astype(np.float64), 0, C, inertia, xm.astype(np.float64))
    diag = bbox_diag(xk1)
    err = vertex_err(res["xk"], xk1) / diag
    upd = vertex_err(xk1, xk) / diag
    print(f"[sphere drape] step 70 stages: vt={len(vt)} ee={len(ee)} set={len(C.vt)}+{len(C.ee)}+{len(C.ob)} "
          f"s={s1:.4f} inner err/diag={err:.2e} update/diag={upd:.2e}", flush=True)
    assert upd > 1e-6
    assert err <= 1e-5


def test_cylinder_drape_heavy_contact_stays_tangle_free():
    """The bench workload from the 0.3 m drop through 200 steps (contact
    from step 48 on, up to about 200,000 vertex-cylinder constraints): the
    device check after every step and the exact check every 10th step and at
    the end find no intersecting triangles."""
    import paper_2403_19272_amd as P
    from paper_2403_19272_amd import basis as B
    sc = scenegen.config(2)
    g = P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                     k_bend=sc.k_bend, d_hat=sc.d_hat, r=sc.r, iters_inner=10, iters_outer=3,
                     precision=P.CLOTH_MIXED, self_contact=True, debug_tangles=True)
    ob = sc.obstacles[0]
    g.add_obstacle(ob.kind, ob.center, ob.radius, axis=ob.axis, half_length=ob.half_length, omega=ob.omega)
    g.set_basis(B.rest_eigenbasis(g.system_matrix(), sc.pinned, sc.r))
    g.set_state(sc.x0, sc.v0)
    peak = 0
    for s in range(sc.steps):
        st = g.step(sc.gravity)   # raises CLOTH_E_TANGLED if the device check trips
        peak = max(peak, st["n_constraints"])
        if s % 10 == 9 or s == sc.steps - 1:
            x, _ = g.get_state()
            assert np.isfinite(x).all()
            nt = exact.count_tangles(x, sc.tris)
            print(f"[cylinder drape] step {s + 1} constraints={st['n_constraints']} "
                  f"contact vertices={st['n_contact_vertices']} min_toi={st['min_toi']:.3f} tangles={nt}",
                  flush=True)
            assert nt == 0, s
    assert peak > 100000
