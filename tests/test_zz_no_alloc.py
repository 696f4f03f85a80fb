"""pe_solve_noalloc (the solve for callers that cannot allocate) against pe_solve, through the
C ABI: two calls in a row on the shared fixed scratch array, the second smaller, each bitwise
equal to pe_solve on the same inputs (the kernels are the same and results do not depend on
batching); a screen too large for the array is refused with PE_ENOMEM."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import torch
    import paper_2408_15583_amd as pe_mod
    assert torch.cuda.is_available()
    return pe_mod


def test_noalloc_matches_solve_twice(pe):
    sc = scenes.dihedral()
    eps = 0.5 * float(sc.radius)
    with pe.Context(0) as ctx:
        s = pe.Scene.from_scene(ctx, sc, view_res=256)
        cases = [
            dict(inc_dir=scenes.azimuth_sweep(np.arange(0, 90, 7.5), 0.0),
                 freq_hz=np.array([8e9, 10e9, 12e9]), screen=256, max_bounces=2),
            dict(inc_dir=scenes.azimuth_sweep(np.array([5.0, 45.0, 80.0]), 10.0),
                 freq_hz=np.array([10e9]), screen=128, max_bounces=1),
        ]
        for c in cases:
            E0, r0, _ = pe.solve(ctx, s, c["inc_dir"], c["freq_hz"], c["screen"],
                                 max_bounces=c["max_bounces"], eps=eps)
            used_before = ctx.footprint()[0]
            E1, r1, st = pe.solve_noalloc(ctx, s, c["inc_dir"], c["freq_hz"], c["screen"],
                                          max_bounces=c["max_bounces"], eps=eps)
            assert ctx.footprint()[0] == used_before  # nothing charged: nothing allocated
            assert np.array_equal(E0, E1)
            assert np.array_equal(r0, r1)
            assert st["ray_queries"] > 0
        with pytest.raises(pe.PEError) as e:
            pe.solve_noalloc(ctx, s, cases[0]["inc_dir"][:1], [10e9], 2048, max_bounces=2,
                             eps=eps)
        assert "PE_ENOMEM" in str(e.value)
        # the allocating path still works after the refusal
        E2, _, _ = pe.solve(ctx, s, cases[1]["inc_dir"], [10e9], 128, eps=eps)
        assert np.isfinite(E2).all()
        s.close()
