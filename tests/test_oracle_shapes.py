"""Pins of the oracle's transverse particle shapes of order 0-3 (Sec. III.B:
orders 0-3 transversely): the weights are the centred cardinal B-splines
(checked against scipy's B-spline basis elements), they sum to one,
reproduce linear functions (orders >= 1), make deposit and gather adjoint,
keep the uniform lattice exactly neutral, and their derivatives (used by the
adjoint) are those of the weights."""
import dataclasses

import numpy as np
import pytest
from scipy.interpolate import BSpline

import workloads as W
from oracle import qsp_adjoint as A
from oracle import qsp_oracle as O

ORDERS = (0, 1, 2, 3)


def cardinal(p):
    """Centred cardinal B-spline of degree p (support [-(p+1)/2, (p+1)/2])."""
    knots = np.arange(p + 2) - (p + 1) / 2.0
    b = BSpline.basis_element(knots, extrapolate=False)
    return lambda t: np.nan_to_num(b(t))


@pytest.mark.parametrize("order", ORDERS)
def test_weights_are_cardinal_bsplines(order):
    rng = np.random.default_rng(order)
    n = 32
    s = rng.uniform(3.0, n - 3.0, 2000)
    s = s[np.abs(s - np.round(s) - 0.5 * (order % 2 == 0)) > 1e-9]   # no ties at the NGP/order-2 switch
    nodes, wts = O.shape_1d(s, n, order)
    B = cardinal(order)
    for b, w in zip(nodes, wts):
        assert np.allclose(w, B(b - s), atol=1e-14, rtol=0), (order,)
    # every node outside the stencil has B = 0
    lo = np.min(np.stack(nodes), axis=0)
    hi = np.max(np.stack(nodes), axis=0)
    for off in (-1, 1):
        outside = (lo - 1) if off < 0 else (hi + 1)
        assert np.allclose(B(outside - s), 0.0, atol=1e-14)


@pytest.mark.parametrize("order", ORDERS)
def test_partition_of_unity_and_first_moment(order):
    rng = np.random.default_rng(10 + order)
    s = rng.uniform(3.0, 29.0, 1000)
    nodes, wts = O.shape_1d(s, 32, order)
    assert np.allclose(sum(wts), 1.0, atol=1e-14)
    first = sum(w * b for b, w in zip(nodes, wts))
    if order >= 1:
        assert np.allclose(first, s, atol=1e-12)
    else:
        assert np.all(np.abs(first - s) <= 0.5)


def box(order, n=24):
    cfg = W.BoxConfig(nx=n, ny=n, x_lo=-3.0, x_hi=3.0, y_lo=-3.0, y_hi=3.0, nzeta=2,
                      zeta_hi=0.0, dzeta=0.1, shape_order=order)
    return cfg


@pytest.mark.parametrize("order", ORDERS)
def test_deposit_and_gather_are_adjoint(order):
    cfg = box(order)
    rng = np.random.default_rng(20 + order)
    x = rng.uniform(cfg.x_lo, cfg.x_hi, 500)
    y = rng.uniform(cfg.y_lo, cfg.y_hi, 500)
    v = rng.normal(size=500)
    F = O.zero_boundary(rng.normal(size=(cfg.ny + 1, cfg.nx + 1)))
    lhs = np.sum(O.deposit_values(cfg, x, y, v) * F)
    rhs = np.sum(v * O.gather(cfg, F, x, y))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("ppc", [1, 2])
def test_uniform_lattice_is_neutral(order, ppc):
    # ions sit on the electrons' rest lattice: neutral at every node, the
    # ones next to the box edge included
    cfg = dataclasses.replace(box(order), ppc_x=ppc, ppc_y=ppc)
    dep = O.add_ion_background(cfg, O.plasma_deposit(cfg, O.init_plasma(cfg)))
    assert np.abs(dep["rho_mjz"]).max() < 1e-12 * cfg.n0


def edge_factor(order, ppc, i):
    """Fraction of the 1D lattice sum that node i >= 1 receives, from the
    B-spline values of the lattice points missing beyond the edge (the
    points at -(k + 1/2)/ppc, k = 0, 1, ...)."""
    miss = sum(cardinal(order)(i + (k + 0.5) / ppc) for k in range(8))
    return 1.0 - miss / ppc


@pytest.mark.parametrize("order,ppc", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (0, 2)])
def test_ion_density_edge_profile(order, ppc):
    # closed forms: interior nodes n0; node 1 of a cubic, one particle per
    # cell: n0 (1 - 1/48) per axis (the missing point at -1/2 weighs
    # B3(3/2) = 1/48); quadratic, two per cell: n0 (1 - 1/64)
    cfg = dataclasses.replace(box(order), ppc_x=ppc, ppc_y=ppc, n0=1.7)
    ion = O.ion_density(cfg)
    n = cfg.nx
    assert np.all(ion[0, :] == 0) and np.all(ion[:, 0] == 0)
    assert np.allclose(ion[3:n - 2, 3:n - 2], cfg.n0, rtol=1e-14)
    for i in (1, 2):
        fx = edge_factor(order, ppc, i)
        assert abs(ion[n // 2, i] / cfg.n0 - fx) < 1e-14
        assert abs(ion[i, i] / cfg.n0 - fx * fx) < 1e-14
    if (order, ppc) == (3, 1):
        assert abs(edge_factor(3, 1, 1) - 47 / 48) < 1e-15
    if (order, ppc) == (2, 2):
        assert abs(edge_factor(2, 2, 1) - 63 / 64) < 1e-15


@pytest.mark.parametrize("order", [1, 2, 3])
def test_weight_derivatives_match_finite_differences(order):
    rng = np.random.default_rng(30 + order)
    s = rng.uniform(3.0, 29.0, 500)
    h = 1e-6
    # stay away from the stencil switch points (integers or half-integers)
    f = s - np.floor(s)
    s = s[(np.abs(f - 0.5) > 1e-4) & (f > 1e-4) & (f < 1 - 1e-4)]
    nodes, _ = O.shape_1d(s, 32, order)
    _, wp = O.shape_1d(s + h, 32, order)
    _, wm = O.shape_1d(s - h, 32, order)
    for k, dw in enumerate(A.shape_1d_grad(s, 32, order)):
        fd = (wp[k] - wm[k]) / (2 * h)
        assert np.allclose(dw, fd, atol=1e-7), (order, k)
