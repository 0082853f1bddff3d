"""Pins of the design-update oracle (Sec. "Topology optimization procedure",
Algorithm "Optimization iteration"): the density filter against a brute-force
pair sum and closed forms, the projection against its limits and symmetry,
the chain rule against the dot-product identity and complex-step derivatives
of the composed map, and the update against its bounds and constraint."""

import numpy as np
import pytest

from oracle import design as dz


def _brute_filter(x, mask, r):
    """x~_i = sum_j w_ij x_j / sum_j w_ij over design nodes j, every pair
    visited explicitly (no offsets, no shifts)."""
    pts = list(zip(*np.nonzero(np.ones_like(mask))))
    out = x.astype(float).copy()
    for i in pts:
        if not mask[i]:
            continue
        num = den = 0.0
        for j in pts:
            if not mask[j]:
                continue
            d = np.sqrt(sum((a - b) ** 2 for a, b in zip(i, j)))
            if d < r:
                num += (r - d) * x[j]
                den += r - d
        out[i] = num / den
    return out


def test_filter_offsets_are_the_ball():
    """Offsets are exactly the integer points with |o| < r, with even
    weights r - |o| (45 points for r = 4 in 2D)."""
    for dim, r in ((2, 4.0), (3, 4.0), (2, 2.5), (3, 1.5)):
        offs, w = dz.filter_offsets(r, dim)
        want = set()
        box = range(-6, 7)
        for o in (np.array(np.meshgrid(*([box] * dim))).reshape(dim, -1).T):
            if np.sqrt((o ** 2).sum()) < r:
                want.add(tuple(int(k) for k in o))
        assert set(offs) == want
        table = dict(zip(offs, w))
        for o, v in table.items():
            assert table[tuple(-k for k in o)] == v
            assert v == pytest.approx(r - np.sqrt(sum(k * k for k in o)), abs=0)
    assert len(dz.filter_offsets(4.0, 2)[0]) == 45


@pytest.mark.parametrize("shape", [(11, 8), (7, 6, 5)])
def test_filter_matches_brute_force(shape, rng):
    """The shifted-array filter equals the pairwise definition on a tiny grid
    with a ragged design mask (r = 4 in 2D, 2.5 in 3D)."""
    r = 4.0 if len(shape) == 2 else 2.5
    mask = rng.random(shape) < 0.7
    x = rng.random(shape)
    np.testing.assert_allclose(dz.density_filter(x, mask, r), _brute_filter(x, mask, r), rtol=0, atol=1e-14)


def test_filter_preserves_constants_and_linear_fields(rng):
    """Normalisation: a constant design stays constant on D. Symmetry of the
    cone: a linear field is reproduced at nodes whose ball lies inside an
    all-design grid."""
    shape = (24, 20)
    mask = rng.random(shape) < 0.6
    c = 0.37
    xt = dz.density_filter(np.full(shape, c), mask, 4.0)
    assert np.max(np.abs(xt[mask] - c)) < 1e-15
    full = np.ones(shape, dtype=bool)
    X, Y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    lin = 0.1 + 0.02 * X - 0.03 * Y
    xt = dz.density_filter(lin, full, 4.0)
    np.testing.assert_allclose(xt[3:-3, 3:-3], lin[3:-3, 3:-3], rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(19, 13), (9, 8, 7)])
def test_filter_transpose_dot_product(shape, rng):
    """<F a, b>_D = <a, F^T b>_D for random a, b: the transposed filter is the
    adjoint of the filter restricted to the design domain."""
    mask = rng.random(shape) < 0.65
    a = np.where(mask, rng.standard_normal(shape), 0.0)
    b = np.where(mask, rng.standard_normal(shape), 0.0)
    lhs = np.sum(np.where(mask, dz.density_filter(a, mask, 4.0), 0.0) * b)
    rhs = np.sum(a * dz.density_filter_transpose(b, mask, 4.0))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)
    assert np.all(dz.density_filter_transpose(b, mask, 4.0)[~mask] == 0.0)


def test_heaviside_limits_and_symmetry():
    """H(0) = 0, H(1) = 1, H(eta) = 1/2 at eta = 1/2, H(1 - t) = 1 - H(t), monotone,
    and a step at eta as beta grows; its derivative equals the complex-step
    derivative of H."""
    t = np.linspace(0.0, 1.0, 101)
    for beta in (2.0, 4.0, 8.0, 16.0):
        H = dz.heaviside(t, beta, 0.5)
        assert H[0] == pytest.approx(0.0, abs=1e-15) and H[-1] == pytest.approx(1.0, abs=1e-15)
        assert dz.heaviside(0.5, beta, 0.5) == pytest.approx(0.5, abs=1e-15)
        np.testing.assert_allclose(dz.heaviside(1.0 - t, beta, 0.5), 1.0 - H, atol=1e-15)
        assert np.all(np.diff(H) > 0)
        for eta in (0.5, 0.3):
            h = 1e-30
            cs = dz.heaviside(t + 1j * h, beta, eta).imag / h
            np.testing.assert_allclose(dz.heaviside_derivative(t, beta, eta), cs, rtol=1e-13, atol=1e-14)
    assert dz.heaviside(0.45, 400.0, 0.5) < 1e-8 and dz.heaviside(0.55, 400.0, 0.5) > 1 - 1e-8


@pytest.mark.parametrize("shape", [(14, 11), (8, 7, 6)])
def test_chain_rule_matches_complex_step(shape, rng):
    """dJ/dx and dV/dx of the composed map x -> gamma -> (J = <c, gamma>, V)
    against complex-step derivatives on design nodes (and 0 off the domain)."""
    mask = rng.random(shape) < 0.7
    base = np.where(rng.random(shape) < 0.5, 1.0, 0.0)
    x = rng.random(shape)
    c = rng.standard_normal(shape)
    r, beta, eta = (4.0 if len(shape) == 2 else 2.5), 4.0, 0.5
    gJ, gV = dz.chain(x, mask, r, beta, eta, c)
    idx = list(zip(*np.nonzero(mask)))
    pick = [idx[k] for k in rng.choice(len(idx), size=6, replace=False)]
    h = 1e-30
    for j in pick:
        xc = x.astype(complex)
        xc[j] += 1j * h
        g = dz.physical_field(xc, mask, base, r, beta, eta)
        dJ = np.sum(c * g).imag / h
        dV = (np.sum(np.where(mask, g, 0.0)) / np.count_nonzero(mask)).imag / h
        assert gJ[j] == pytest.approx(dJ, rel=1e-12, abs=1e-15)
        assert gV[j] == pytest.approx(dV, rel=1e-12, abs=1e-15)
    assert np.all(gJ[~mask] == 0.0) and np.all(gV[~mask] == 0.0)


def test_volume_fraction_closed_forms(rng):
    """V is the mean of gamma over D: a uniform gamma gives its value; nodes
    off the domain do not count."""
    shape = (10, 9)
    mask = rng.random(shape) < 0.5
    assert dz.volume_fraction(np.full(shape, 0.25), mask) == pytest.approx(0.25, abs=1e-16)
    g = np.where(mask, 1.0, 7.0)
    assert dz.volume_fraction(g, mask) == pytest.approx(1.0, abs=1e-16)


def test_update_bounds_and_volume_constraint(rng):
    """The step stays in [0, 1] and within the move limit, leaves nodes off the
    domain alone, meets V <= V_max with the smallest multiplier (to bisection
    accuracy), and is the plain clipped descent step when the constraint is
    inactive."""
    shape = (20, 16)
    mask = rng.random(shape) < 0.7
    base = np.zeros(shape)
    x = np.clip(0.5 + 0.2 * rng.standard_normal(shape), 0.0, 1.0)
    r, beta, eta, move = 4.0, 4.0, 0.5, 0.1
    # a sensitivity that favours solid, so that the descent step alone adds volume
    gJ, gV = dz.chain(x, mask, r, beta, eta, -1.0 + 0.3 * rng.standard_normal(shape))
    v_start = dz.volume_fraction(dz.physical_field(x, mask, base, r, beta, eta), mask)
    vmax = v_start - 0.02
    xn, v, lam = dz.update(x, gJ, gV, mask, base, r, beta, eta, move, vmax)
    assert lam > 0 and v <= vmax
    assert np.all(xn >= 0.0) and np.all(xn <= 1.0)
    assert np.all(np.abs(xn - x)[mask] <= move + 1e-15) and np.all(xn[~mask] == x[~mask])
    # a slightly smaller multiplier violates the constraint
    sJ, sV = gJ / np.max(np.abs(gJ[mask])), gV / np.max(np.abs(gV[mask]))
    lo, hi = np.maximum(0, x - move), np.minimum(1, x + move)
    t = np.where(mask, np.clip(x - move * (sJ + 0.999 * lam * sV), lo, hi), x)
    assert dz.volume_fraction(dz.physical_field(t, mask, base, r, beta, eta), mask) > vmax
    # inactive constraint: lam = 0 and the clipped descent step
    xn2, v2, lam2 = dz.update(x, gJ, gV, mask, base, r, beta, eta, move, 1.0)
    assert lam2 == 0.0
    np.testing.assert_array_equal(xn2, np.where(mask, np.clip(x - move * sJ, lo, hi), x))


def test_update_lower_volume_bound(rng):
    """Two-sided constraint: a sensitivity that favours fluid (the descent
    step alone removes volume) below V_min gives lam < 0 and V >= V_min with
    the multiplier of smallest magnitude (a slightly smaller |lam| violates
    it); inside the bounds the step is the plain clipped descent step (lam = 0);
    V(x(lam)) does not increase with lam."""
    shape = (20, 16)
    mask = rng.random(shape) < 0.7
    base = np.zeros(shape)
    x = np.clip(0.5 + 0.2 * rng.standard_normal(shape), 0.0, 1.0)
    r, beta, eta, move = 4.0, 4.0, 0.5, 0.1
    gJ, gV = dz.chain(x, mask, r, beta, eta, 1.0 + 0.3 * rng.standard_normal(shape))
    v_start = dz.volume_fraction(dz.physical_field(x, mask, base, r, beta, eta), mask)
    vmin = v_start + 0.01
    xn, v, lam = dz.update(x, gJ, gV, mask, base, r, beta, eta, move, 1.0, vmin=vmin)
    assert lam < 0 and v >= vmin
    assert np.all(np.abs(xn - x)[mask] <= move + 1e-15) and np.all(xn[~mask] == x[~mask])
    sJ, sV = gJ / np.max(np.abs(gJ[mask])), gV / np.max(np.abs(gV[mask]))
    lo, hi = np.maximum(0, x - move), np.minimum(1, x + move)

    def vol(l):
        t = np.where(mask, np.clip(x - move * (sJ + l * sV), lo, hi), x)
        return dz.volume_fraction(dz.physical_field(t, mask, base, r, beta, eta), mask)

    assert vol(0.999 * lam) < vmin
    lams = np.linspace(-4, 4, 17)
    assert np.all(np.diff([vol(l) for l in lams]) <= 1e-15)
    xn2, v2, lam2 = dz.update(x, gJ, gV, mask, base, r, beta, eta, move, 1.0, vmin=0.0)
    assert lam2 == 0.0 and v2 < v_start
