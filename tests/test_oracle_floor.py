"""Pins of the oracle's floored 1 + Psi branch (the paper's pusher equations
divide by 1 + Psi and leave its vanishing unspecified; the reading taken:
D = max(1 + Psi, floor) wherever 1 + Psi divides, Psi itself integrated
unchanged, floored pushes counted).

What fixes the expected values without retyping the push:
* a consistent linear multistep method integrates a constant right-hand
  side exactly once its history is full, so in zero fields a floored
  particle moves by exactly dzeta * u / floor per slice;
* the deposit of one particle on a node is a four-vector (rho, J) with
  rho^2 - |J|^2 = (q w / (hx hy D))^2 (the proper density), whatever gamma
  and u_z are, so the floored divisor shows up in a Lorentz invariant;
* in a uniform Ez (and nothing else) Psi grows linearly, dPsi/dzeta = -Ez,
  so the slice where 1 + Psi crosses the floor, and with it the number of
  floored pushes, is known beforehand."""
import numpy as np

import workloads as W
from oracle import qsp_oracle as O


def cfg16():
    return W.BoxConfig(nx=16, ny=16, x_lo=-4.0, x_hi=4.0, y_lo=-4.0, y_hi=4.0,
                       nzeta=64, zeta_hi=0.0, dzeta=0.05)


def plasma_of(x, y, ux, uy, psi, w=0.25):
    n = len(x)
    a = lambda v: np.array(v, dtype=np.float64)
    return O.Plasma(x=a(x), y=a(y), ux=a(ux), uy=a(uy), psi=a(psi), w=np.full(n, w),
                    hist=np.zeros((4, 5, n)))


def zero_fields(cfg):
    z = np.zeros((cfg.ny + 1, cfg.nx + 1))
    return {k: z.copy() for k in ("exmby", "eypbx", "ez", "bx", "by", "bz")}


def test_floored_particle_drifts_with_the_floor_as_divisor():
    cfg = cfg16()
    floor = cfg.psi_floor
    # 1 + Psi = 0.3 floor, 0.9 floor (floored) and 2 floor (not floored)
    raw = np.array([0.3 * floor, 0.9 * floor, 2.0 * floor])
    p = plasma_of([-1.0, 0.0, 1.0], [0.5, -0.5, 0.0], [0.02, -0.01, 0.03], [0.01, 0.02, -0.02],
                  raw - 1.0)
    flds = zero_fields(cfg)
    xs, clamps = [p.x.copy()], []
    for _ in range(9):
        p, nc, nabs = O.ab5_push(cfg, p, flds, commit=True)
        xs.append(p.x.copy())
        clamps.append(nc)
        assert nabs == 0
    # Psi and u never change in zero fields: the two low particles stay floored
    assert np.array_equal(p.psi, raw - 1.0)
    assert clamps == [2] * 9
    d = np.maximum(raw, floor)
    ux = np.array([0.02, -0.01, 0.03])
    for k in range(5, 9):     # history full: one dzeta * u / D per slice
        step = xs[k + 1] - xs[k]
        assert np.allclose(step, cfg.dzeta * ux / d, rtol=1e-12, atol=0.0), (k, step)
    # the divisor is the floor, not the raw value
    assert not np.allclose(xs[9] - xs[8], cfg.dzeta * ux / raw)


def test_floored_deposit_has_the_floored_proper_density():
    cfg = W.BoxConfig(nx=8, ny=8, x_lo=-4.0, x_hi=4.0, y_lo=-4.0, y_hi=4.0,
                      nzeta=4, zeta_hi=0.0, dzeta=0.1)           # h = 1, nodes at integers
    floor = cfg.psi_floor
    for raw, ux, uy in ((0.3 * floor, 0.4, -0.7), (0.5, 0.4, -0.7), (0.02 * floor, 1.5, 0.2)):
        w = 0.8
        p = plasma_of([1.0], [-2.0], [ux], [uy], [raw - 1.0], w=w)   # on node (5, 2)
        dep = O.plasma_deposit(cfg, p)
        rho, jx, jy, jz = (dep[c][2, 5] for c in ("rho", "jx", "jy", "jz"))
        d = max(raw, floor)
        # rho^2 - |J|^2 cancels to (w/D)^2 from terms gamma^2 times larger
        inv = rho * rho - jx * jx - jy * jy - jz * jz
        assert abs(inv - (w / d) ** 2) <= 1e-14 * rho * rho, (raw, inv, (w / d) ** 2)
        assert abs(dep["rho_mjz"][2, 5] - (-w)) <= 1e-15
        # and the particle moves along z at less than c
        assert abs(jz) < abs(rho)


def test_psi_crosses_the_floor_at_the_predicted_slice():
    cfg = cfg16()
    floor = cfg.psi_floor
    ez0 = 0.04
    flds = zero_fields(cfg)
    flds["ez"][1:-1, 1:-1] = ez0
    p = plasma_of([0.3], [-0.2], [0.0], [0.0], [-1.0 + 0.25 * floor])
    # history as if the particle had seen the same field before: every
    # step then adds exactly dzeta * Ez to Psi
    p.hist[:, 4, 0] = -ez0
    psi0 = p.psi[0]
    total = 0
    for k in range(12):
        p, nc, _ = O.ab5_push(cfg, p, flds, commit=True)
        total += nc
        assert abs(p.psi[0] - (psi0 + (k + 1) * cfg.dzeta * ez0)) <= 1e-13
        assert p.x[0] == 0.3 and p.ux[0] == 0.0
    # pushes with 1 + Psi_k < floor: Psi_k = psi0 + k dzeta Ez, k = 0, 1, ...
    expect = sum(1 for k in range(12) if 1.0 + psi0 + k * cfg.dzeta * ez0 < floor)
    assert total == expect == 4
