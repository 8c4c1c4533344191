"""Pins of the oracle's macro-particle beam (Sec. III.A: beam particles
sorted per slice, deposited and pushed inside the slice loop; Sec. III.B:
second-order symplectic beam push; zeroth-order longitudinal deposit)."""
import numpy as np
from scipy.integrate import solve_ivp

import workloads as W
from oracle import qsp_oracle as O


def one_particle(cfg, x, y, zeta, ux, uy, uz, w=1.0, dt=1.0):
    a = lambda v: np.array([float(v)])
    return W.ParticleBeam(a(x), a(y), a(zeta), a(ux), a(uy), a(uz), a(w), dt=dt)


def uniform_fields(cfg, Ex, Ey, Ez, Bx, By, Bz):
    sh = (cfg.ny + 1, cfg.nx + 1)
    f = lambda v: O.zero_boundary(np.full(sh, float(v)))
    return {"exmby": f(Ex - By), "eypbx": f(Ey + Bx), "ez": f(Ez),
            "bx": f(Bx), "by": f(By), "bz": f(Bz)}


def box():
    return W.BoxConfig(nx=16, ny=16, x_lo=-50.0, x_hi=50.0, y_lo=-50.0, y_hi=50.0,
                       nzeta=4, zeta_hi=0.0, dzeta=1.0)


def test_magnetic_rotation_preserves_momentum():
    cfg = box()
    b = one_particle(cfg, 0.1, -0.2, 0.0, 3.0, -1.0, 20.0, dt=0.7)
    F = uniform_fields(cfg, 0, 0, 0, 0.3, -0.4, 1.1)
    u0 = np.sqrt(b.ux ** 2 + b.uy ** 2 + b.uz ** 2)
    for _ in range(50):
        O.beam_push_slice(cfg, b, 0, F, b.dt)
    assert abs(np.sqrt(b.ux ** 2 + b.uy ** 2 + b.uz ** 2)[0] / u0[0] - 1) < 1e-13


def test_free_drift_of_zeta():
    cfg = box()
    b = one_particle(cfg, 0.0, 0.0, -0.3, 0.0, 0.0, np.sqrt(2000.0 ** 2 - 1), dt=6.0)
    F = uniform_fields(cfg, 0, 0, 0, 0, 0, 0)
    O.beam_push_slice(cfg, b, 0, F, 6.0)
    vz = np.sqrt(2000.0 ** 2 - 1) / 2000.0
    assert abs(b.zeta[0] - (-0.3 + 6.0 * (vz - 1.0))) < 1e-15
    assert b.x[0] == 0.0 and b.ux[0] == 0.0


def lorentz(t, s, E, B):
    u = s[3:6]
    g = np.sqrt(1 + u @ u)
    v = u / g
    du = -(E + np.cross(v, B))
    return np.concatenate([v[:2], [v[2] - 1.0], du])


def test_second_order_against_lorentz_ode():
    cfg = box()
    E = np.array([0.2, -0.1, 0.05])
    B = np.array([0.15, 0.25, -0.3])
    F = uniform_fields(cfg, *E, *B)
    s0 = np.array([0.5, -0.3, -0.25, 1.5, -0.5, 4.0])
    T = 4.0
    ref = solve_ivp(lorentz, (0, T), s0, args=(E, B), rtol=1e-12, atol=1e-14,
                    method="DOP853").y[:, -1]
    errs = []
    for nsteps in (20, 40, 80):
        dt = T / nsteps
        b = one_particle(cfg, *s0[:3], *s0[3:], dt=dt)
        for _ in range(nsteps):
            O.beam_push_slice(cfg, b, int(O.beam_slice_index(cfg, b.zeta)[0]), F, dt)
        got = np.array([b.x[0], b.y[0], b.zeta[0], b.ux[0], b.uy[0], b.uz[0]])
        errs.append(np.linalg.norm(got - ref))
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(r - 2.0) < 0.2), (errs, r)


def test_beam_deposit_charge_and_identity():
    cfg, beam = W.small_particle_beam()
    k = 16
    src = O.particle_beam_source(cfg, beam, k)
    sel = O.beam_slice_index(cfg, beam.zeta) == k
    inner = sel & (np.abs(beam.x) < 7) & (np.abs(beam.y) < 7)
    assert inner.sum() == sel.sum() > 100
    total = src["rho"].sum() * cfg.hx * cfg.hy * cfg.dzeta
    assert abs(total + beam.w[sel].sum()) < 1e-12 * beam.w[sel].sum()
    g = np.sqrt(1 + beam.ux ** 2 + beam.uy ** 2 + beam.uz ** 2)
    # rho - Jz = rho (1 - v_z) for every particle, written without cancellation
    vz = beam.uz / g
    one_m_vz = (1 + beam.ux ** 2 + beam.uy ** 2) / (g * (g + beam.uz))
    assert np.allclose(one_m_vz[sel], 1 - vz[sel], rtol=1e-6, atol=1e-16)
    assert np.allclose(src["rho"] - src["jz"], src["rho_mjz"], atol=1e-12 * np.abs(src["rho"]).max())


def test_nearest_slice_assignment():
    cfg = box()
    z = np.array([0.0, -0.49, -0.51, -1.0, -2.6])
    assert list(O.beam_slice_index(cfg, z)) == [0, 0, 1, 1, 3]
