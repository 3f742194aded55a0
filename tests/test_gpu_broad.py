"""The broad phase's reusable candidate superset (broad_reuse; MI355X only): candidate
lists are filtered from a superset built on grown boxes and kept while every
stage box stays inside its grown box.  The lists must equal the oracle's
brute-force-checked broad phase whether a stage rebuilt the superset or
reused it, and a stage whose boxes stay inside must not rebuild."""
import numpy as np
import pytest

import scenegen
from helpers import gpu_side, oracle_side
from oracle import native

pytestmark = pytest.mark.gpu


def rebuilds(g, sc):
    """Superset rebuilds since the previous read (the stats read resets them)."""
    return g.step(sc.gravity, n=0)["n_broad_rebuilds"]


@pytest.mark.parametrize("n,seed", [(24, 11), (64, 12)])
def test_superset_reuse_and_rebuild_bit_exact(n, seed):
    sc = scenegen.drop_cloth(n, seed=seed, obstacle="sphere", r=8, steps=1, d_hat=1e-3)
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    xm = (sc.x0 + rng.normal(0, 0.3 * h, sc.x0.shape)).astype(np.float32)
    xp = (xm + rng.normal(0, 0.2 * h, xm.shape)).astype(np.float32)
    o, U, _ = oracle_side(sc, "fp32", rho=0.9)
    g = gpu_side(sc, U, "fp32", 0.9, broad_reuse=True)
    rebuilds(g, sc)
    # 1: first stage builds the superset
    vt, ee = g.stage_broad_phase(xm, xp)
    ovt, oee = native.broad_phase(xm, xp, o.m.edges, o.m.tris, sc.d_hat)
    assert rebuilds(g, sc) == 1
    assert len(ovt) > 0 and len(oee) > 0
    assert np.array_equal(vt, ovt) and np.array_equal(ee, oee)
    # 2: the end positions move by far less than the margin (d_hat): the
    # superset is filtered, not rebuilt
    xp2 = (xp + rng.uniform(-0.2e-3, 0.2e-3, xp.shape)).astype(np.float32)
    vt2, ee2 = g.stage_broad_phase(xm, xp2)
    ovt2, oee2 = native.broad_phase(xm, xp2, o.m.edges, o.m.tris, sc.d_hat)
    assert rebuilds(g, sc) == 0
    assert np.array_equal(vt2, ovt2) and np.array_equal(ee2, oee2)
    # 3: a smaller stage (shorter sweep): reused, fewer pairs
    xp3 = (xm + 0.5 * (xp - xm)).astype(np.float32)
    vt3, ee3 = g.stage_broad_phase(xm, xp3)
    ovt3, oee3 = native.broad_phase(xm, xp3, o.m.edges, o.m.tris, sc.d_hat)
    assert rebuilds(g, sc) == 0
    assert np.array_equal(vt3, ovt3) and np.array_equal(ee3, oee3)
    assert len(vt3) + len(ee3) < len(vt) + len(ee)
    # 4: a move past the margins rebuilds
    xm4 = (xm + rng.normal(0, 0.3 * h, xm.shape)).astype(np.float32)
    xp4 = (xm4 + rng.normal(0, 0.2 * h, xm.shape)).astype(np.float32)
    vt4, ee4 = g.stage_broad_phase(xm4, xp4)
    ovt4, oee4 = native.broad_phase(xm4, xp4, o.m.edges, o.m.tris, sc.d_hat)
    assert rebuilds(g, sc) == 1
    assert np.array_equal(vt4, ovt4) and np.array_equal(ee4, oee4)
    print(f"[superset n={n}] pairs {len(vt)}+{len(ee)} / {len(vt2)}+{len(ee2)} / {len(vt3)}+{len(ee3)} / "
          f"{len(vt4)}+{len(ee4)}", flush=True)
