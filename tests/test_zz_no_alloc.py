"""The allocation-free design map (lbm_design_map_noalloc) against the
context form (lbm_design_init + lbm_design_map) through the C ABI: two
calls in a row on one GPU, the second on a smaller grid (the shared scratch
keeps the first call's partials), in 2D and 3D. Both forms sum the same
filter terms in the same order, so gamma and the volume fraction must agree
to the last bit; the bar is 1e-15 absolute on values in [0, 1]."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    mask = rng.random(shape) < 0.7
    base = np.where(rng.random(shape) < 0.3, 1.0, 0.0)
    x = rng.random(shape)
    return mask, base, x


@pytest.mark.parametrize("shapes", [
    (((2048, 512), 4.0), ((300, 211), 2.5)),
    (((64, 48, 40), 4.0), ((30, 21, 11), 2.0)),
], ids=["2d", "3d"])
def test_noalloc_map_matches_context_map(shapes):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_19617_amd.design import Design, map_noalloc
    for k, (shape, r) in enumerate(shapes):
        mask, base, x = _case(shape, 7 + k)
        for beta, eta in ((2.0, 0.5), (16.0, 0.35)):
            g_na, v_na = map_noalloc(shape, mask, base, x, r, beta, eta)
            torch.cuda.synchronize()
            d = Design(shape, mask, base, radius=r)
            g_ref, v_ref = d.map(x, beta, eta)
            d.close()
            diff = float((g_na - g_ref).abs().max())
            print(f"noalloc map {shape} r={r} beta={beta} eta={eta}: max |diff| {diff:.1e}, "
                  f"V {float(v_na):.15f} vs {v_ref:.15f}")
            assert diff <= 1e-15
            assert abs(float(v_na) - v_ref) <= 1e-15
