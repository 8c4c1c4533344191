"""Charge conservation pins of the oracle (quasi-static continuity, Sec. II):
with zeta = z - t and d/dtau = 0, continuity of the plasma electrons reads
d_zeta (rho - Jz) = div_perp J_perp.  Per macro-particle rho - Jz = q w S
(the gamma - u_z = 1 + Psi invariant), so along the pusher's orbits
(dx_p/dzeta = -u_p/D_p) the zeta derivative of the deposited rho - Jz is the
shape's position derivative times that velocity, which is the divergence of
the continuous current sum q w (u/D) S.  Two consequences are pinned:

* the finite-difference zeta derivative of the deposit along exact orbits
  equals the shape-slope deposit of the orbit velocity (orders 1-3), and a
  plasma moving with a uniform velocity carries its deposit along exactly;
* the total of rho - Jz (electrons and ions) over a nonlinear box stays
  what it is at the head of the box, slice after slice, as long as no
  particle reaches the box edge."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import qsp_oracle as O
from test_oracle_explicit import random_plasma, smooth_fields


def orbit_fd_of_charge(cfg, p, flds, eps=1e-8):
    f, _ = O.particle_rhs(cfg, p, flds)
    out = []
    for sgn in (1.0, -1.0):
        q = p.copy()
        q.x, q.y, q.ux, q.uy, q.psi = (np.stack([p.x, p.y, p.ux, p.uy, p.psi]) + sgn * eps * f)
        out.append(O.plasma_deposit(cfg, q, ("rho_mjz",))["rho_mjz"])
    return (out[0] - out[1]) / (2 * eps), f


@pytest.mark.parametrize("order", [1, 2, 3])
def test_dzeta_charge_is_shape_slope_times_orbit_velocity(order):
    cfg, _ = W.small(n=32, nzeta=4, ppc=2)
    cfg = dataclasses.replace(cfg, shape_order=order)
    p = random_plasma(cfg, 40 + order)
    flds = smooth_fields(cfg, 17)
    fd, f = orbit_fd_of_charge(cfg, p, flds)
    qn = -p.w / (cfg.hx * cfg.hy)
    # dx_p/dzeta from the pusher's right-hand side: -u/D (absorbed
    # particles, w = 0, are frozen)
    d = O.clamp_d(cfg, p.psi)
    live = p.w > 0
    assert np.allclose(f[0][live], (-p.ux / d)[live], rtol=1e-14, atol=0.0)
    assert np.allclose(f[1][live], (-p.uy / d)[live], rtol=1e-14, atol=0.0)
    slope = O.deposit_slopes(cfg, p.x, p.y, qn * f[0], qn * f[1])
    err = np.linalg.norm(fd - slope) / np.linalg.norm(slope)
    assert err < 1e-6, err


def test_uniform_drift_carries_the_deposit():
    # every particle shifted by a whole number of cells leaves the deposit
    # of the interior shifted by exactly that many nodes
    cfg, _ = W.small(n=32, nzeta=4, ppc=1)
    p = random_plasma(cfg, 3, margin=6)
    base = O.plasma_deposit(cfg, p, ("rho_mjz",))["rho_mjz"]
    q = p.copy()
    q.x = q.x + 2 * cfg.hx
    q.y = q.y - 1 * cfg.hy
    moved = O.plasma_deposit(cfg, q, ("rho_mjz",))["rho_mjz"]
    assert np.allclose(moved[1:-2, 3:-1], base[2:-1, 1:-3], rtol=1e-12, atol=1e-12)


def boundary_charge(cfg, p):
    """Electron charge that the shape puts on the Dirichlet boundary nodes
    or past them (stencils of order 3 reach one node beyond), where the
    deposit drops it."""
    nodes, wts = O.shape_weights(cfg, p.x, p.y)
    qn = -p.w
    tot = 0.0
    for (i, j), s in zip(nodes, wts):
        edge = (i <= 0) | (i >= cfg.nx) | (j <= 0) | (j >= cfg.ny)
        tot += float(np.sum((qn * s)[edge]))
    return tot


@pytest.mark.parametrize("order", [1, 3])
def test_box_charge_is_conserved(order):
    # a strongly nonlinear wake (electrons blown out of the axis, the edge
    # plasma disturbed): slice after slice the interior total of rho - Jz
    # (electrons and ions) changes only by the electron charge that moves
    # onto or off the boundary nodes
    cfg, beam = W.small(n=64, nzeta=32, nb=8.0, sigma=0.35, extent=4.0, pc_max_iter=3)
    cfg = dataclasses.replace(cfg, shape_order=order)
    st = O.initial_state(cfg)
    totals, leaked = [], []
    for _ in range(cfg.nzeta):
        plasma = st.plasma.copy()
        st, rec = O.advance_slice(cfg, st, beam)
        totals.append(rec["rho_mjz"].sum() * cfg.hx * cfg.hy)
        leaked.append(boundary_charge(cfg, plasma))
    totals, leaked = np.array(totals), np.array(leaked)
    assert np.all(st.plasma.w > 0)                      # nothing absorbed
    p0 = O.init_plasma(cfg)
    assert np.hypot(st.plasma.x - p0.x, st.plasma.y - p0.y).max() > 5.0 * cfg.hx
    assert np.abs(totals - totals[0]).max() > 1e-3      # the interior total does move
    kept = totals + leaked
    assert np.abs(kept - kept[0]).max() < 1e-12 * st.plasma.w.sum(), np.abs(kept - kept[0]).max()
