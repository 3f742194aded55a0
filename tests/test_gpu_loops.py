"""GPU parity of Algorithm 1's loop conditions (tolerance mode), of the
strain-limited projection, and of the failed-step contract (MI355X only).

Tolerance mode: the inner and outer loop conditions are decided on the
device, so the executed counts must equal the oracle's.  The tolerances are
picked from the oracle's own runs so that every decision sits at least 10 %
away from its threshold (the FP32 norms differ from the FP64 ones by far
less) and both loops stop early at least once.

Failed steps: a capacity overflow or a non-finite iterate rolls the step back
on the device; the state stays bitwise what it was, the next stats read
reports the failure once, and a server ticket carries it.
"""
import itertools

import numpy as np
import pytest

import scenegen
from helpers import bbox_diag, gpu_side, oracle_side

pytestmark = pytest.mark.gpu


def vertex_err(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64), axis=1).max())


def decision_margin(st, tol_in, tol_out, budget_in, budget_out):
    """Smallest |log(norm / tolerance)| over the loop decisions of one oracle
    step, and whether an inner block and the outer loop stopped early."""
    m = np.inf
    pos = 0
    inner_stop = False
    for n in st.block_iters:
        blk = st.dx[pos:pos + n]
        pos += n
        for k in range(1, n + 1 if n < budget_in else n):
            m = min(m, abs(np.log(blk[k - 1] / tol_in)))
        inner_stop |= n < budget_in
    outer_stop = st.outer_iters < budget_out
    for o in range(1, st.outer_iters + 1 if outer_stop else st.outer_iters):
        m = min(m, abs(np.log(st.outer_dx[o - 1] / tol_out)))
    return m, inner_stop, outer_stop


def pick_tolerances(sc, precision, U, rho, gamma, steps, budget_in, budget_out, cand_in, cand_out):
    best = None
    for ti, to in itertools.product(cand_in, cand_out):
        o, _, _ = oracle_side(sc, precision, gamma=gamma, rho=rho, U=U, iters_inner=budget_in,
                              iters_outer=budget_out, tol=(ti, to))
        margin, stop_in, stop_out = np.inf, False, False
        for _ in range(steps):
            m, a, b = decision_margin(o.step(), ti, to, budget_in, budget_out)
            margin, stop_in, stop_out = min(margin, m), stop_in or a, stop_out or b
        if stop_in and stop_out and (best is None or margin > best[0]):
            best = (margin, ti, to)
    assert best is not None and best[0] > np.log(1.1), best
    return best[1], best[2], best[0]


def tolerance_run(sc, precision, steps, budget_in, budget_out, cand_in, cand_out, gamma, tag):
    o0, U, rho = oracle_side(sc, precision, gamma=gamma, iters_inner=budget_in, iters_outer=budget_out)
    ti, to, margin = pick_tolerances(sc, precision, U, rho, gamma, steps, budget_in, budget_out, cand_in, cand_out)
    o, _, _ = oracle_side(sc, precision, gamma=gamma, rho=rho, U=U, iters_inner=budget_in, iters_outer=budget_out,
                          tol=(ti, to))
    g = gpu_side(sc, U, precision, rho, gamma=gamma, iters_inner=budget_in, iters_outer=budget_out,
                 tol_inner=ti, tol_outer=to)
    diag = bbox_diag(o.x)
    for s in range(steps):
        so = o.step()
        sg = g.step(sc.gravity)
        x, _ = g.get_state()
        err = vertex_err(x, o.x) / diag
        print(f"[{tag}] step {s} tol_in={ti:.1e} tol_out={to:.1e} margin={np.exp(margin):.2f}x inner "
              f"{sg['inner_iters']}/{so.inner_iters} outer {sg['outer_iters']}/{so.outer_iters} err/diag={err:.2e} "
              f"dx={sg['dx_norm']:.3e}/{so.dx[-1]:.3e} outer_dx={sg['outer_dx']:.3e}/{so.outer_dx[-1]:.3e}",
              flush=True)
        assert sg["inner_iters"] == so.inner_iters and sg["outer_iters"] == so.outer_iters
        assert err <= 1e-5
        # the device norms are differences of FP32 positions: beside the 2 %
        # relative bound, each may be off by a few roundings of a coordinate
        ulp = 4 * float(np.spacing(np.float32(np.abs(o.x).max())))
        assert abs(sg["dx_norm"] - so.dx[-1]) <= 0.02 * so.dx[-1] + ulp
        assert abs(sg["outer_dx"] - so.outer_dx[-1]) <= 0.02 * so.outer_dx[-1] + ulp
    return g


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_tolerance_mode_hanging_cloth(precision):
    """Small hanging cloth thrown at 1 m/s, 3 blocks x 10 iterations."""
    sc = scenegen.config(0)
    sc.v0[:] = np.array([0.3, -1.0, 0.2], np.float32)
    sc.v0[sc.pinned.astype(bool)] = 0
    tolerance_run(sc, precision, 3, 10, 3, [2e-5, 3e-5, 5e-5, 8e-5, 1.2e-4, 1.6e-4],
                  [4e-5, 6e-5, 1e-4, 1.6e-4, 2.5e-4, 4e-4], 0.9, f"tol c0 {precision}")


def test_tolerance_mode_with_contact():
    """A cloth falling onto a sphere with self contact: skipped blocks also
    skip their CCD stages."""
    sc = scenegen.drop_cloth(20, seed=9, obstacle="sphere", r=8, steps=3, drop=0.0015, d_hat=1e-3,
                             iters_outer=3, iters_inner=6)
    sc.v0[:] = np.array([0.0, -2.0, 0.0], np.float32)
    g = tolerance_run(sc, "fp32", 3, 6, 3, [1.5e-3, 2.2e-3, 3e-3, 4.5e-3], [3e-3, 5e-3, 7e-3], 0.6,
                      "tol contact")
    assert g.step(sc.gravity)["n_constraints"] > 0


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_strain_limited_hanging_cloth(precision):
    """Strain limits [0.95, 1.05] in the local step (nearest matrix with the
    singular values in range), ten steps against the oracle's SVD form."""
    sc = scenegen.config(0)
    sc.v0[:] = np.array([0.3, -1.0, 0.2], np.float32)
    sc.v0[sc.pinned.astype(bool)] = 0
    o, U, rho = oracle_side(sc, precision, sigma=(0.95, 1.05))
    g = gpu_side(sc, U, precision, rho, sigma_min=0.95, sigma_max=1.05)
    ref, _, _ = oracle_side(sc, precision, U=U, rho=rho)
    for _ in range(sc.steps):
        o.step()
        ref.step()
        g.step(sc.gravity)
    x, _ = g.get_state()
    diag = bbox_diag(o.x)
    err = vertex_err(x, o.x) / diag
    eff = vertex_err(o.x, ref.x) / diag
    print(f"[strain {precision}] err/diag={err:.2e} effect of the limits/diag={eff:.2e}", flush=True)
    assert err <= 1e-5
    assert eff > 1e-4   # the limits change the motion


def test_capacity_overflow_rolls_back_the_step():
    """pair_capacity below the candidate count of the first contact step: the
    step fails with CLOTH_E_CAPACITY and leaves x and v bitwise unchanged;
    the failure is reported once; steps without a stats read also roll back
    and are reported at the next read."""
    import paper_2403_19272_amd as P
    sc = scenegen.drop_cloth(20, seed=9, obstacle="sphere", r=8, steps=1, drop=0.0015, d_hat=1e-3,
                             iters_outer=2, iters_inner=4)
    sc.v0[:] = np.array([0.0, -2.0, 0.0], np.float32)
    o, U, rho = oracle_side(sc, "fp32", gamma=0.6)
    wide = gpu_side(sc, U, "fp32", rho, gamma=0.6)
    st = wide.step(sc.gravity)
    peak = st["peak_candidates"]
    print(f"[capacity] peak candidates per list {peak}", flush=True)
    assert peak > 64
    g = gpu_side(sc, U, "fp32", rho, gamma=0.6, pair_capacity=peak // 2)
    x0, v0 = g.get_state()
    with pytest.raises(P.ClothError) as e:
        g.step(sc.gravity)
    assert e.value.code == P.CLOTH_E_CAPACITY
    x1, v1 = g.get_state()
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    # reported once
    st = g.step(sc.gravity, n=0)
    assert st is not None
    # three steps without reading: all roll back, one report
    g.step(sc.gravity, n=3, stats=False)
    x2, v2 = g.get_state()
    assert np.array_equal(x0, x2) and np.array_equal(v0, v2)
    with pytest.raises(P.ClothError) as e:
        g.step(sc.gravity, n=0)
    assert e.value.code == P.CLOTH_E_CAPACITY
    # the wide scene stepped on
    assert not np.array_equal(wide.get_state()[0], x0)


def test_divergence_rolls_back_the_step():
    """A damping far beyond the Jacobi stability limit makes the iterate blow
    up to Inf/NaN within a step: CLOTH_E_DIVERGED, state unchanged."""
    import paper_2403_19272_amd as P
    sc = scenegen.config(0)
    o, U, rho = oracle_side(sc, "fp32")
    g = gpu_side(sc, U, "fp32", 0.999, gamma=40.0, iters_inner=20, iters_outer=3)
    x0, v0 = g.get_state()
    with pytest.raises(P.ClothError) as e:
        g.step(sc.gravity)
    assert e.value.code == P.CLOTH_E_DIVERGED
    x1, v1 = g.get_state()
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    assert np.isfinite(x1).all()


def test_graph_recorded_again_after_add_obstacle():
    """An obstacle added after graph-replayed steps takes part in the next
    steps: graph replay and eager launches stay bitwise equal."""
    sc = scenegen.drop_cloth(24, seed=7, obstacle="sphere", r=16, steps=6, drop=0.003, d_hat=1e-3)
    o, U, rho = oracle_side(sc, "mixed", rho=0.95)
    ob = sc.obstacles[0]
    sc.obstacles = []
    a = gpu_side(sc, U, "mixed", 0.95)
    b = gpu_side(sc, U, "mixed", 0.95)
    a.set_graph(False)
    b.set_graph(True)
    for s in range(sc.steps):
        if s == 2:
            for g in (a, b):
                g.add_obstacle(ob.kind, ob.center, ob.radius, axis=ob.axis)
        sa = a.step(sc.gravity)
        sb = b.step(sc.gravity)
        xa, va = a.get_state()
        xb, vb = b.get_state()
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), s
        assert sa["n_constraints"] == sb["n_constraints"], s
    print(f"[graph+obstacle] constraints={sb['n_constraints']}", flush=True)
    assert sb["n_constraints"] > 0


def test_server_ticket_reports_a_rolled_back_step():
    import paper_2403_19272_amd as P
    sc = scenegen.drop_cloth(20, seed=9, obstacle="sphere", r=8, steps=1, drop=0.0015, d_hat=1e-3,
                             iters_outer=2, iters_inner=4)
    sc.v0[:] = np.array([0.0, -2.0, 0.0], np.float32)
    o, U, rho = oracle_side(sc, "fp32", gamma=0.6)
    g = gpu_side(sc, U, "fp32", rho, gamma=0.6, pair_capacity=48)
    ok = gpu_side(sc, U, "fp32", rho, gamma=0.6)
    x0, _ = g.get_state()
    srv = P.StepServer(slots=2)
    assert srv.admit(g) and srv.admit(ok)
    t_bad = srv.submit(g, sc.gravity)
    t_ok = srv.submit(ok, sc.gravity)
    with pytest.raises(P.ClothError) as e:
        srv.wait(t_bad)
    assert e.value.code == P.CLOTH_E_CAPACITY
    srv.wait(t_ok)
    srv.close()
    assert np.array_equal(g.get_state()[0], x0)
    assert not np.array_equal(ok.get_state()[0], x0)


def folded_states(n=16):
    """A cloth folded over itself (two layers 1 cm apart, no intersection)
    and the same with one upper vertex pushed 3 cm down through the lower
    layer (its triangles cross the lower ones)."""
    sc = scenegen.drop_cloth(n, seed=4, obstacle="sphere", r=8, steps=1, drop=0.05, d_hat=1e-3)
    X = sc.x0.astype(np.float64).copy()
    side = X[:, 0] > 0.5
    X[side, 0] = 1.0 - X[side, 0]
    X[side, 1] += 0.01 + 0.02 * (X[side, 0] - 0.5) ** 2
    Y = X.copy()
    k = np.flatnonzero(side)[len(np.flatnonzero(side)) // 2]
    Y[k, 1] -= 0.03
    return sc, X.astype(np.float32), Y.astype(np.float32)


def test_tangle_check_flags_a_tangled_state_and_rolls_back():
    """debug_tangles: a step that ends with edges crossing triangles fails
    with CLOTH_E_TANGLED and keeps its start state; an untangled fold steps
    on.  The oracle's exact count decides which state is which."""
    import paper_2403_19272_amd as P
    from oracle import exact
    sc, X, Y = folded_states()
    assert exact.count_tangles(X, sc.tris) == 0 and exact.count_tangles(Y, sc.tris) > 0
    o, U, rho = oracle_side(sc, "fp32", gamma=0.6)
    g = gpu_side(sc, U, "fp32", rho, gamma=0.6, debug_tangles=True)
    g.set_state(Y)
    with pytest.raises(P.ClothError) as e:
        g.step(sc.gravity)
    print(f"[tangle] {e.value}", flush=True)
    assert e.value.code == P.CLOTH_E_TANGLED
    x1, v1 = g.get_state()
    assert np.array_equal(x1, Y) and not v1.any()
    g.set_state(X)
    for _ in range(3):
        st = g.step(sc.gravity)
    x2, _ = g.get_state()
    assert exact.count_tangles(x2, sc.tris) == 0
    assert not np.array_equal(x2, X)
