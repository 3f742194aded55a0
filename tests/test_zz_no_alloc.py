"""The basis entry point that allocates no device memory
(cloth_compute_basis_static) against the allocating one
(cloth_compute_basis), called through the C ABI (MI355X only).

Two calls in a row on the fixed workspace, the second on a smaller scene
(so the array still holds the first call's larger block), each compared with
the allocating call on its own scene; then a scene whose iteration needs more
than the fixed workspace is refused before any work.
"""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


def make_scene(n, r, seed):
    import paper_2403_19272_amd as P
    sc = scenegen.hanging_cloth(n, seed=seed, r=r)
    return P.ClothScene(sc.tris, sc.rest, dt=sc.dt, density=sc.density, k_stretch=sc.k_stretch,
                        k_bend=sc.k_bend, pinned=sc.pinned, r=r, iters_inner=4, iters_outer=1,
                        cheb_rho=0.9, cheb_gamma=0.5)


def test_static_basis_equals_allocating_basis():
    cases = [(72, 24, 3), (40, 16, 4)]   # the second call is the smaller one
    scenes = [(make_scene(n, r, s), make_scene(n, r, s)) for n, r, s in cases]
    static = []
    for (n, r, _), (ga, _) in zip(cases, scenes):
        out = ga.compute_basis(degree=300, max_passes=15, tol=2e-2, return_basis=True, static=True)
        print(f"[no-alloc] static n={n} r={r} passes={out['passes']} res={out['residual']:.2e}", flush=True)
        static.append(out)
    for (n, r, _), (_, gb), st in zip(cases, scenes, static):
        ref = gb.compute_basis(degree=300, max_passes=15, tol=2e-2, return_basis=True)
        same = np.array_equal(st["U"], ref["U"]) and np.array_equal(st["ritz"], ref["ritz"])
        du = float(np.abs(st["U"] - ref["U"]).max())
        print(f"[no-alloc] n={n} r={r} bitwise={same} max|dU|={du:.2e} passes {st['passes']}/{ref['passes']}",
              flush=True)
        assert st["passes"] == ref["passes"]
        assert st["residual"] == pytest.approx(ref["residual"], rel=1e-6, abs=1e-12)
        assert np.allclose(st["ritz"], ref["ritz"], rtol=1e-6, atol=0)
        assert du <= 1e-6
    for ga, gb in scenes:
        # both scenes step the same way from the basis each entry point set
        ga.step(n=2)
        gb.step(n=2)
        xa, xb = ga.get_state()[0], gb.get_state()[0]
        assert np.abs(xa - xb).max() <= 1e-6
        ga.close()
        gb.close()


def test_static_basis_refuses_a_scene_beyond_the_workspace():
    import paper_2403_19272_amd as P
    g = make_scene(256, 64, 5)      # 4 blocks of 65,536 x 80 floats: 84 MB > 64 MiB
    with pytest.raises(P.ClothError) as e:
        g.compute_basis(degree=50, max_passes=1, static=True)
    assert e.value.code == P.CLOTH_E_INVALID and "workspace" in str(e.value)
    g.close()
