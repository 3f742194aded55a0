"""The autotuner (MI355X only): every setting it may pick leaves the step's
results bitwise unchanged (so the choice is made on time at equal
accuracy), the tuned scene's state is the one it had before the trials, and
a second scene of the same size class takes the cached choice."""
import numpy as np
import pytest

import scenegen
from helpers import gpu_side, oracle_side

pytestmark = pytest.mark.gpu


def contact_scene(n=48, seed=31, broad_reuse=True):
    sc = scenegen.drop_cloth(n, seed=seed, obstacle="sphere", r=16, steps=4, drop=0.004, d_hat=1e-3,
                             side=(n - 1) / 127.0)
    o, U, rho = oracle_side(sc, "mixed", rho=0.95, gamma=0.6)
    return sc, U


def run(sc, U, steps, **tuning):
    g = gpu_side(sc, U, "mixed", 0.95, gamma=0.6, broad_reuse=True)
    g.set_tuning(**tuning)
    st = g.step(sc.gravity, n=steps)
    x, v = g.get_state()
    g.close()
    return x, v, st


def test_every_setting_gives_the_same_bits():
    sc, U = contact_scene()
    x0, v0, st0 = run(sc, U, 6)
    assert st0["n_constraints"] > 0
    for kw in (dict(query_lanes=4), dict(query_lanes=16), dict(query_lanes=8, broad_reuse=True),
               dict(query_lanes=16, broad_reuse=True, broad_margin=2e-3)):
        x, v, st = run(sc, U, 6, **kw)
        print(f"[tune] {kw}: constraints {st['n_constraints']} rebuilds {st['n_broad_rebuilds']}", flush=True)
        assert np.array_equal(x, x0) and np.array_equal(v, v0), kw


def test_autotune_restores_state_and_caches():
    sc, U = contact_scene(n=40, seed=32)
    g = gpu_side(sc, U, "mixed", 0.95, gamma=0.6, broad_reuse=True)
    g.step(sc.gravity, n=3)
    xa, va = g.get_state()
    t = g.autotune(sc.gravity, steps=3, force=True)
    print(f"[tune] choice {t}", flush=True)
    assert t["trials"] >= 3 and t["query_lanes"] in (4, 8, 16) and t["ms_per_step"] > 0
    assert t["ms_per_step"] <= t["ms_default"] + 1e-9
    xb, vb = g.get_state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    # stepping on with the tuned setting: the same bits as an untuned twin
    twin = gpu_side(sc, U, "mixed", 0.95, gamma=0.6, broad_reuse=True)
    twin.set_state(xa, va)
    g.step(sc.gravity, n=2)
    twin.step(sc.gravity, n=2)
    assert np.array_equal(g.get_state()[0], twin.get_state()[0])
    # a scene of the same size class takes the cached choice
    sc2, U2 = contact_scene(n=40, seed=33)
    g2 = gpu_side(sc2, U2, "mixed", 0.95, gamma=0.6, broad_reuse=True)
    t2 = g2.autotune(sc2.gravity, steps=3)
    assert t2["from_cache"] == 1 and t2["query_lanes"] == t["query_lanes"]
    assert t2["broad_reuse"] == t["broad_reuse"]
    for s in (g, twin, g2):
        s.close()
