"""GPU parity against the FP64 oracle (MI355X only).

End to end on the small hanging cloth (10 steps x 20 iterations, both
precisions): max vertex error / bbox diagonal <= 1e-5.  Stage level on
identical FP32 inputs: broad-phase pair lists and life spans bit-exact, TOI
within 1e-6, one inner iteration with contact within 1e-5 of the bbox
diagonal.
"""
import numpy as np
import pytest

import scenegen
from helpers import K_CONTACT, bbox_diag, gpu_side, oracle_side
from oracle import model as M
from oracle import native
from oracle import step as S

pytestmark = pytest.mark.gpu


def vertex_err(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64), axis=1).max())


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_hanging_cloth_ten_steps(precision):
    sc = scenegen.config(0)
    o, U, rho = oracle_side(sc, precision)
    g = gpu_side(sc, U, precision, rho)
    print(f"[c0 {precision}] rho={rho:.6f}", flush=True)
    for s in range(sc.steps):
        o.step()
        st = g.step(sc.gravity)
    xg, vg = g.get_state()
    diag = bbox_diag(o.x)
    err = vertex_err(xg, o.x) / diag
    print(f"[c0 {precision}] err/diag={err:.3e} dx={st['dx_norm']:.3e} moved={vertex_err(o.x, sc.x0):.3e}", flush=True)
    assert err <= 1e-5
    assert vertex_err(o.x, sc.x0) > 1e-3   # the cloth actually moved
    assert np.abs(vg - o.v).max() <= 1e-5 * diag / sc.dt


def crumpled(sc, seed, amp=0.02, step=0.01):
    rng = np.random.default_rng(seed)
    xm = (sc.x0 + rng.normal(0, amp, sc.x0.shape)).astype(np.float32)
    xp = (xm + rng.normal(0, step, xm.shape)).astype(np.float32)
    return xm, xp


@pytest.mark.parametrize("n,seed", [(12, 0), (24, 1), (64, 2)])
def test_broad_phase_and_toi_bit_exact(n, seed):
    sc = scenegen.drop_cloth(n, seed=seed, obstacle="sphere", r=8, steps=1, d_hat=1e-3)
    xm, xp = crumpled(sc, seed, amp=0.3 / n, step=0.2 / n)
    o, U, rho = oracle_side(sc, "fp32", rho=0.9)
    g = gpu_side(sc, U, "fp32", 0.9)
    vt, ee = g.stage_broad_phase(xm, xp)
    ovt, oee = native.broad_phase(xm, xp, o.m.edges, o.m.tris, sc.d_hat)
    print(f"[bp n={n}] vt={len(vt)} ee={len(ee)}", flush=True)
    assert len(ovt) > 0 and len(oee) > 0
    assert np.array_equal(vt, ovt)
    assert np.array_equal(ee, oee)
    tv, te = g.stage_toi(xm, xp, vt, ee)
    otv, ote, nf = native.toi_pairs(xm.astype(np.float64), xp.astype(np.float64), o.m.tris, o.m.edges, vt, ee)
    hit = (otv <= 1) | (tv <= 1)
    assert np.array_equal(otv <= 1, tv <= 1)
    assert np.abs(tv[hit] - otv[hit]).max(initial=0) <= 1e-6
    hit = (ote <= 1) | (te <= 1)
    assert np.array_equal(ote <= 1, te <= 1)
    assert np.abs(te[hit] - ote[hit]).max(initial=0) <= 1e-6


def contact_block(n=20, seed=3, precision="fp32"):
    """A block state with pair and obstacle constraints on identical FP32 inputs."""
    sc = scenegen.drop_cloth(n, seed=seed, obstacle="sphere", r=8, steps=1, d_hat=2e-3, drop=0.002)
    rng = np.random.default_rng(seed)
    xm, xp = crumpled(sc, seed, amp=0.2 / n, step=0.1 / n)
    o, U, rho = oracle_side(sc, precision, rho=0.95)
    vt, ee = native.broad_phase(xm, xp, o.m.edges, o.m.tris, sc.d_hat)
    vt = vt[rng.random(len(vt)) < 0.3]
    ee = ee[rng.random(len(ee)) < 0.3]
    a_vt = rng.integers(0, 6, len(vt)).astype(np.int32)
    a_ee = rng.integers(0, 6, len(ee)).astype(np.int32)
    ob_a = np.where(rng.random(sc.nv) < 0.3, rng.integers(0, 6, sc.nv), -1).astype(np.int32)[None]
    ob_a[0, sc.pinned.astype(bool)] = -1
    xk = (xm + rng.normal(0, 0.05 / n, xm.shape)).astype(np.float32)
    xkm1 = (xk + rng.normal(0, 0.02 / n, xm.shape)).astype(np.float32)
    z = (xk + rng.normal(0, 0.05 / n, xm.shape)).astype(np.float32)
    return sc, o, U, dict(xm=xm, xp=xp, xk=xk, xkm1=xkm1, z=z, vt=vt, ee=ee, a_vt=a_vt, a_ee=a_ee, ob_a=ob_a)


def oracle_constraints(o, blk):
    C = S.Constraints()
    C.vt, C.ee = blk["vt"], blk["ee"]
    C.a_vt, C.a_ee = blk["a_vt"].copy(), blk["a_ee"].copy()
    v = np.flatnonzero(blk["ob_a"][0] >= 0).astype(np.int32)
    C.ob = np.stack([v, np.zeros_like(v)], 1)
    C.a_ob = blk["ob_a"][0][v].copy()
    o._freeze(C, blk["xm"].astype(np.float64))
    return C


def test_partial_ccd_life_spans_bit_exact():
    sc, o, U, blk = contact_block()
    g = gpu_side(sc, U, "fp32", 0.95)
    g.stage_load_block(blk["xm"], blk["xk"], blk["xkm1"], blk["z"], blk["vt"], blk["a_vt"], blk["ee"],
                       blk["a_ee"], blk["ob_a"])
    g.stage_partial_ccd(blk["xp"])
    got = g.stage_read_block(nob=1)
    C = oracle_constraints(o, blk)
    o._partial_ccd(C, blk["xm"].astype(np.float64), blk["xp"].astype(np.float64))
    print(f"[pccd] vt={len(C.vt)} ee={len(C.ee)} ob={len(C.ob)} active_vt={int((C.a_vt > 0).sum())}", flush=True)
    assert np.array_equal(got["a_vt"], C.a_vt)
    assert np.array_equal(got["a_ee"], C.a_ee)
    ob = np.full(sc.nv, -1, np.int32)
    ob[C.ob[:, 0]] = C.a_ob
    assert np.array_equal(got["ob_a"][0], ob)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_inner_iteration_with_contact(precision):
    sc, o, U, blk = contact_block(precision=precision)
    g = gpu_side(sc, U, precision, 0.95)
    g.stage_load_block(blk["xm"], blk["xk"], blk["xkm1"], blk["z"], blk["vt"], blk["a_vt"], blk["ee"],
                       blk["a_ee"], blk["ob_a"])
    k = 4
    g.stage_inner(k)
    got = g.stage_read_block(nob=1)
    C = oracle_constraints(o, blk)
    inertia = (o.m.mass / o.m.h ** 2)[:, None] * blk["z"].astype(np.float64)
    xk1 = o.iterate(blk["xk"].astype(np.float64), blk["xkm1"].astype(np.float64), k, C, inertia,
                    blk["xm"].astype(np.float64))
    diag = bbox_diag(xk1)
    err = vertex_err(got["xk"], xk1) / diag
    upd = vertex_err(xk1, blk["xk"]) / diag
    qerr = np.abs(got["Q"] - o.trace["Q"]).max() / np.abs(o.trace["Q"]).max()
    print(f"[inner {precision}] err/diag={err:.3e} update/diag={upd:.3e} Q rel={qerr:.2e}", flush=True)
    assert upd > 1e-4
    assert err <= 1e-5
