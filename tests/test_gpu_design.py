"""Parity of the design update on the GPU (through the C ABI) with the FP64
oracle: physical field and volume fraction, chain rule, and the
projected-gradient step, on ragged 2D and 3D grids that span several tiles,
with ragged design domains; plus argument errors.

Tolerances: the filter sums the same terms in a different order, so fields
agree to rounding (<= 1e-13 absolute on values in [0, 1]; chain rule <= 1e-12
relative L2); the update's bisection takes the same decisions, so its step
agrees to rounding as well."""

import numpy as np
import pytest

from oracle import design as dz

from helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Design():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_19617_amd.design import Design
    return Design


def _case(shape, seed, frac=0.7):
    rng = np.random.default_rng(seed)
    mask = rng.random(shape) < frac
    base = np.where(rng.random(shape) < 0.3, 1.0, 0.0)
    x = rng.random(shape)
    g = rng.standard_normal(shape)
    return mask, base, x, g


CASES = [((70, 37), 4.0), ((19, 13, 10), 2.5), ((21, 17, 9), 4.0), ((5, 3), 1.0)]


@pytest.mark.parametrize("shape,r", CASES, ids=lambda v: str(v))
def test_design_map_matches_oracle(Design, shape, r):
    mask, base, x, _ = _case(shape, 3)
    d = Design(shape, mask, base, radius=r)
    for beta in (2.0, 16.0):
        for eta in (0.5, 0.35):
            gam, V = d.map(x, beta, eta)
            gam_o = dz.physical_field(x, mask, base, r, beta, eta)
            assert np.max(np.abs(gam.cpu().numpy() - gam_o)) <= 1e-13
            assert abs(V - dz.volume_fraction(gam_o, mask)) <= 1e-13
    d.close()


@pytest.mark.parametrize("shape,r", CASES, ids=lambda v: str(v))
def test_design_chain_matches_oracle(Design, shape, r):
    mask, base, x, g = _case(shape, 5)
    d = Design(shape, mask, base, radius=r)
    gJ, gV = d.chain(x, 4.0, 0.5, g)
    gJ_o, gV_o = dz.chain(x, mask, r, 4.0, 0.5, g)
    assert rel_l2(gJ.cpu().numpy(), gJ_o) <= 1e-12
    assert rel_l2(gV.cpu().numpy(), gV_o) <= 1e-12
    assert np.all(gJ.cpu().numpy()[~mask] == 0.0)
    d.close()


@pytest.mark.parametrize("shape,r", CASES[:3], ids=lambda v: str(v))
def test_design_update_matches_oracle(Design, shape, r):
    mask, base, x, _ = _case(shape, 7)
    d = Design(shape, mask, base, radius=r)
    beta, eta, move = 4.0, 0.5, 0.1
    g = -1.0 + 0.3 * np.random.default_rng(8).standard_normal(shape)   # favours solid: constraint active
    gJ_o, gV_o = dz.chain(x, mask, r, beta, eta, g)
    v0 = dz.volume_fraction(dz.physical_field(x, mask, base, r, beta, eta), mask)
    for vmax in (v0 - 0.03, 1.0):
        xn, V, lam = d.update(x, gJ_o, gV_o, beta, eta, move, vmax)
        xn_o, V_o, lam_o = dz.update(x, gJ_o, gV_o, mask, base, r, beta, eta, move, vmax)
        assert np.max(np.abs(xn.cpu().numpy() - xn_o)) <= 1e-12
        assert abs(V - V_o) <= 1e-13
        assert lam == pytest.approx(lam_o, rel=1e-12, abs=0)
        if vmax < 1.0:
            assert lam > 0 and V <= vmax
        else:
            assert lam == 0.0
    d.close()


@pytest.mark.parametrize("shape,r", CASES[:3], ids=lambda v: str(v))
def test_design_update_lower_bound_matches_oracle(Design, shape, r):
    """Two-sided constraint: a sensitivity that favours fluid with V_min above
    the descent step's volume (negative multiplier), and bounds that the
    plain step meets (lam = 0), against the oracle."""
    mask, base, x, _ = _case(shape, 9)
    d = Design(shape, mask, base, radius=r)
    beta, eta, move = 4.0, 0.5, 0.1
    g = 1.0 + 0.3 * np.random.default_rng(10).standard_normal(shape)
    gJ_o, gV_o = dz.chain(x, mask, r, beta, eta, g)
    v0 = dz.volume_fraction(dz.physical_field(x, mask, base, r, beta, eta), mask)
    for vmin, vmax in ((v0 + 0.01, 1.0), (0.0, 1.0)):
        xn, V, lam = d.update(x, gJ_o, gV_o, beta, eta, move, vmax, vmin)
        xn_o, V_o, lam_o = dz.update(x, gJ_o, gV_o, mask, base, r, beta, eta, move, vmax, vmin=vmin)
        assert np.max(np.abs(xn.cpu().numpy() - xn_o)) <= 1e-12
        assert abs(V - V_o) <= 1e-13
        assert lam == pytest.approx(lam_o, rel=1e-12, abs=0)
        if vmin > 0:
            assert lam < 0 and V >= vmin
        else:
            assert lam == 0.0
    d.close()


def test_design_full_size_wake(Design):
    """Cylinder-wake grid 2048 x 512 with a 320 x 160 design window (r = 4):
    physical field, volume and chain rule against the oracle on the whole
    grid."""
    shape = (2048, 512)
    mask = np.zeros(shape, dtype=bool)
    mask[432:752, 176:336] = True
    rng = np.random.default_rng(11)
    base = np.zeros(shape)
    x = rng.random(shape)
    g = rng.standard_normal(shape)
    d = Design(shape, mask, base, radius=4.0)
    gam, V = d.map(x, 8.0, 0.5)
    gam_o = dz.physical_field(x, mask, base, 4.0, 8.0, 0.5)
    assert np.max(np.abs(gam.cpu().numpy() - gam_o)) <= 1e-13
    assert abs(V - dz.volume_fraction(gam_o, mask)) <= 1e-13
    gJ, gV = d.chain(x, 8.0, 0.5, g)
    gJ_o, gV_o = dz.chain(x, mask, 4.0, 8.0, 0.5, g)
    assert rel_l2(gJ.cpu().numpy(), gJ_o) <= 1e-12 and rel_l2(gV.cpu().numpy(), gV_o) <= 1e-12
    d.close()


def test_design_errors(Design):
    from paper_2608_19617_amd.binding import LbmError
    mask, base, x, g = _case((20, 12), 1)
    d = Design((20, 12), mask, base)
    for beta, eta in ((0.0, 0.5), (2.0, 0.0), (2.0, 1.0)):
        with pytest.raises(LbmError, match="LBM_E_INVALID"):
            d.map(x, beta, eta)
    gJ, gV = d.chain(x, 2.0, 0.5, g)
    for move, vmax, vmin in ((0.0, 0.5, 0.0), (0.1, 1.5, 0.0), (0.1, 0.4, 0.5), (0.1, 0.5, -0.1)):
        with pytest.raises(LbmError, match="LBM_E_INVALID"):
            d.update(x, gJ, gV, 2.0, 0.5, move, vmax, vmin)
    d.close()
    with pytest.raises(LbmError, match="empty"):
        Design((20, 12), np.zeros((20, 12), bool), base)


def test_optimisation_loop_matches_oracle(Design):
    """Two iterations of the GPU loop (forward windows, adjoint over the
    last window, chain rule, volume-constrained step; FP64) against the same
    iterations with the oracle's forward, adjoint and design update, with the
    projection parameter doubling after the first iteration."""
    from oracle import adjoint as ad
    from oracle import forward as fw
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.optimize import optimize
    from helpers import oracle_problem
    w = W.cylinder_channel(nx=48, ny=20, radius=3, center=(14, 10), window_len=12, sample_every=3,
                           ckpt_every=4, n_windows=2)
    w.eps = -1.0
    mask = np.zeros(w.shape, dtype=bool)
    mask[8:28, 3:17] = True
    base = np.where(mask, 0.0, w.gamma)
    x0 = np.where(mask, 0.3, 0.0)
    r, eta, beta, move = 2.5, 0.5, 2.0, 0.2
    prob = oracle_problem(w)
    Wl = w.window_len
    x, hist = optimize(w, mask, x0, prec="f64", radius=r, eta=eta, beta=beta, beta_every=1, move=move,
                       vmax=0.25, n_max=2, eps_o=0.0, base=base)
    xo, b = x0.copy(), beta
    for m in range(2):
        gam = dz.physical_field(xo, mask, base, r, b, eta)
        out = fw.run(prob, gam, 2 * Wl, keep={Wl})
        J, g, _ = ad.window_gradient(prob, gam, out["states"][Wl])
        assert hist[m]["J"] == pytest.approx(J, rel=1e-11, abs=1e-18)
        assert hist[m]["V"] == pytest.approx(dz.volume_fraction(gam, mask), abs=1e-13)
        gJ, gV = dz.chain(xo, mask, r, b, eta, g)
        xo, _, lam = dz.update(xo, gJ, gV, mask, base, r, b, eta, move, 0.25)
        assert hist[m]["lam"] == pytest.approx(lam, rel=1e-8, abs=1e-12)
        b = min(2 * b, 16.0)
    assert np.max(np.abs(x.cpu().numpy() - xo)) <= 1e-9


def test_optimisation_prescribed_window_mode(Design):
    """optimize(steps=n |W|) (a prescribed window: the last of n windows from
    t = 0) gives the same iterations as the representative-window mode when
    the criterion is off and the run is n windows long."""
    from paper_2608_19617_amd import workloads as W
    from paper_2608_19617_amd.optimize import optimize
    w = W.cylinder_channel(nx=48, ny=20, radius=3, center=(14, 10), window_len=12, sample_every=3,
                           ckpt_every=4, n_windows=2)
    w.eps = -1.0
    mask = np.zeros(w.shape, dtype=bool)
    mask[8:28, 3:17] = True
    base = np.where(mask, 0.0, w.gamma)
    x0 = np.where(mask, 0.3, 0.0)
    kw = dict(prec="f64", radius=2.5, eta=0.5, beta=2.0, beta_every=1, move=0.2, vmax=0.25, n_max=2, eps_o=0.0,
              base=base)
    x1, h1 = optimize(w, mask, x0, **kw)
    x2, h2 = optimize(w, mask, x0, steps=2 * w.window_len, **kw)
    assert [h["J"] for h in h1] == [h["J"] for h in h2]
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
