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
