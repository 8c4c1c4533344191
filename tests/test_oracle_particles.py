"""Pins of the oracle's deposit, gather and plasma pusher (Sec. III.B:
CIC current deposition, zeroth order in zeta; the pusher equations and the
Lorentz factor; fifth-order Adams-Bashforth in zeta)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import qsp_oracle as O


def box(n=16, ext=4.0, ppc=1):
    return W.BoxConfig(nx=n, ny=n, x_lo=-ext, x_hi=ext, y_lo=-ext, y_hi=ext,
                       nzeta=8, zeta_hi=0.0, dzeta=0.1, ppc_x=ppc, ppc_y=ppc)


def test_single_particle_hand_weights():
    cfg = box(8, 4.0)                       # h = 1, nodes at -4..4
    x, y = np.array([0.25]), np.array([-1.5])  # cell (4, 2), fx = .25, fy = .5
    dep = O.deposit_values(cfg, x, y, np.array([2.0]))
    expect = np.zeros((9, 9))
    expect[2, 4] = 2 * 0.75 * 0.5
    expect[2, 5] = 2 * 0.25 * 0.5
    expect[3, 4] = 2 * 0.75 * 0.5
    expect[3, 5] = 2 * 0.25 * 0.5
    assert np.array_equal(dep, expect)


def test_partition_of_unity_and_adjointness():
    cfg = box(16, 4.0)
    rng = np.random.default_rng(5)
    n = 500
    x = rng.uniform(cfg.x_lo + cfg.hx, cfg.x_hi - cfg.hx, n)
    y = rng.uniform(cfg.y_lo + cfg.hy, cfg.y_hi - cfg.hy, n)
    c = rng.normal(size=n)
    dep = O.deposit_values(cfg, x, y, c)
    assert abs(dep.sum() - c.sum()) < 1e-12 * np.abs(c).sum()
    F = O.zero_boundary(rng.normal(size=dep.shape))
    assert abs(np.sum(dep * F) - np.sum(c * O.gather(cfg, F, x, y))) < 1e-11


def test_gather_reproduces_bilinear_fields():
    cfg = box(16, 4.0)
    xn, yn = O.node_coords(cfg)
    X, Y = np.meshgrid(xn, yn)
    F = 0.3 + 1.1 * X - 0.6 * Y + 0.2 * X * Y
    rng = np.random.default_rng(6)
    x, y = rng.uniform(-3.9, 3.9, 50), rng.uniform(-3.9, 3.9, 50)
    assert np.allclose(O.gather(cfg, F, x, y), 0.3 + 1.1 * x - 0.6 * y + 0.2 * x * y,
                       atol=1e-12)


@pytest.mark.parametrize("ppc", [1, 2, 3])
def test_uniform_lattice_is_neutral(ppc):
    cfg = box(16, 4.0, ppc)
    p = O.init_plasma(cfg)
    dep = O.add_ion_background(cfg, O.plasma_deposit(cfg, p))
    assert np.abs(dep["rho_mjz"][1:-1, 1:-1]).max() < 1e-13
    assert np.abs(dep["rho"][1:-1, 1:-1]).max() < 1e-13
    for c in ("jx", "jy", "jz"):
        assert np.abs(dep[c]).max() == 0.0


def test_rho_minus_jz_identity():
    # rho - Jz from the separate rho and Jz channels equals the q*w channel
    cfg = box(16, 4.0)
    p = O.init_plasma(cfg)
    rng = np.random.default_rng(7)
    p.x = p.x + rng.uniform(-0.3, 0.3, p.x.size)
    p.y = p.y + rng.uniform(-0.3, 0.3, p.y.size)
    p.x = np.clip(p.x, cfg.x_lo, cfg.x_hi)
    p.y = np.clip(p.y, cfg.y_lo, cfg.y_hi)
    p.ux = rng.normal(0, 0.5, p.x.size)
    p.uy = rng.normal(0, 0.5, p.x.size)
    p.psi = rng.uniform(-0.5, 1.0, p.x.size)
    d = O.plasma_deposit(cfg, p)
    assert np.abs(d["rho"] - d["jz"] - d["rho_mjz"]).max() < 1e-12 * np.abs(d["rho"]).max()


def test_gamma_identity():
    rng = np.random.default_rng(8)
    ux, uy = rng.normal(0, 2, 100), rng.normal(0, 2, 100)
    d = rng.uniform(0.05, 5, 100)
    g = O.gamma_of(ux, uy, d)
    uz = g - d
    assert np.allclose(g * g, 1 + ux * ux + uy * uy + uz * uz, rtol=1e-13)


def lorentz_zeta_rhs(state, E, B):
    """d/dzeta of (x, y, ux, uy, Psi) derived from the lab-frame Lorentz
    force on an electron, du/dt = -(E + v x B), with zeta = z - t so that
    d/dzeta = d/dt / (v_z - 1), and Psi = gamma - u_z - 1."""
    x, y, ux, uy, psi = state
    d = 1.0 + psi
    g = (1 + ux * ux + uy * uy + d * d) / (2 * d)
    uz = g - d
    v = np.array([ux, uy, uz]) / g
    dudt = -(np.asarray(E) + np.cross(v, B))
    dgdt = -np.dot(v, E)
    dzdt = v[2] - 1.0
    return np.array([v[0] / dzdt, v[1] / dzdt, dudt[0] / dzdt, dudt[1] / dzdt,
                     (dgdt - dudt[2]) / dzdt])


def test_rhs_matches_lorentz_force():
    cfg = box(16, 4.0)
    rng = np.random.default_rng(9)
    for _ in range(20):
        st = np.array([0.1, -0.2, rng.normal(0, 1), rng.normal(0, 1),
                       rng.uniform(-0.6, 2.0)])
        Ex, Ey, Ez, Bx, By, Bz = rng.normal(0, 1, 6)
        shape = (cfg.ny + 1, cfg.nx + 1)
        flds = {"exmby": np.full(shape, Ex - By), "eypbx": np.full(shape, Ey + Bx),
                "ez": np.full(shape, Ez), "bx": np.full(shape, Bx),
                "by": np.full(shape, By), "bz": np.full(shape, Bz)}
        p = O.Plasma(*(np.array([v]) for v in st), w=np.array([1.0]),
                     hist=np.zeros((4, 5, 1)))
        f, _ = O.particle_rhs(cfg, p, flds)
        ref = lorentz_zeta_rhs(st, [Ex, Ey, Ez], [Bx, By, Bz])
        assert np.allclose(f[:, 0], ref, rtol=1e-12, atol=1e-12)


def ramp(s):
    """Smooth start-up factor: zero with its first five derivatives at
    s = 0 (s = distance behind the box head)."""
    return np.where(s > 0, s ** 6 / (1 + s ** 6), 0.0)


def field_history(zeta):
    s = -zeta
    r = ramp(s)
    return dict(Ex=0.3 * r * np.cos(s), Ey=-0.2 * r, Ez=0.25 * r * np.sin(0.7 * s),
                Bx=0.15 * r, By=-0.1 * r * np.cos(1.3 * s), Bz=0.2 * r)


def run_ab5(dz, span=3.0):
    n = 8
    cfg = W.BoxConfig(nx=n, ny=n, x_lo=-40.0, x_hi=40.0, y_lo=-40.0, y_hi=40.0,
                      nzeta=int(round(span / dz)), zeta_hi=0.0, dzeta=dz)
    p = O.Plasma(*(np.array([v]) for v in (0.3, -0.2, 0.0, 0.0, 0.0)),
                 w=np.array([1.0]), hist=np.zeros((4, 5, 1)))
    shape = (n + 1, n + 1)
    for k in range(cfg.nzeta):
        F = field_history(cfg.zeta_hi - k * dz)
        flds = {"exmby": np.full(shape, F["Ex"] - F["By"]),
                "eypbx": np.full(shape, F["Ey"] + F["Bx"]),
                "ez": np.full(shape, F["Ez"]), "bx": np.full(shape, F["Bx"]),
                "by": np.full(shape, F["By"]), "bz": np.full(shape, F["Bz"])}
        p, _, _ = O.ab5_push(cfg, p, flds, commit=True)
    return np.array([p.x[0], p.y[0], p.ux[0], p.uy[0], p.psi[0]]), -cfg.nzeta * dz


def test_ab5_fifth_order():
    def rhs(zeta, st):
        F = field_history(np.array(zeta))
        return lorentz_zeta_rhs(st, [F["Ex"], F["Ey"], F["Ez"]],
                                [F["Bx"], F["By"], F["Bz"]])
    errs = []
    dzs = [0.05, 0.025, 0.0125]
    for dz in dzs:
        y, zend = run_ab5(dz)
        ref = solve_ivp(rhs, (0.0, zend), [0.3, -0.2, 0.0, 0.0, 0.0],
                        rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
        errs.append(np.linalg.norm(y - ref))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 5.0) < 0.3), (errs, slopes)


def test_ion_column_betatron_frequency():
    # inside an electron-free ion column Ex - By = x/2; a slow electron
    # oscillates as x'' = -x/2 in zeta, i.e. with wavenumber 1/sqrt(2)
    cfg = W.BoxConfig(nx=64, ny=64, x_lo=-4, x_hi=4, y_lo=-4, y_hi=4,
                      nzeta=2000, zeta_hi=0.0, dzeta=0.01)
    x, y = O.node_coords(cfg)
    X, Y = np.meshgrid(x, y)
    flds = {"exmby": O.zero_boundary(X / 2), "eypbx": O.zero_boundary(Y / 2),
            "ez": 0 * X, "bx": 0 * X, "by": 0 * X, "bz": 0 * X}
    a = 1e-3
    # start the multistep history on the analytic orbit x = a cos(s/sqrt 2),
    # s = -zeta, u_x = dx/ds, so the test measures the frequency only
    hist = np.zeros((4, 5, 1))
    for m in range(4):
        sm = -(m + 1) * cfg.dzeta
        xm, um = a * np.cos(sm / np.sqrt(2)), -a / np.sqrt(2) * np.sin(sm / np.sqrt(2))
        hist[m, :, 0] = [-um, 0.0, xm / 2, 0.0, um * xm / 2]
    p = O.Plasma(np.array([a]), np.array([0.0]), np.zeros(1), np.zeros(1),
                 np.zeros(1), np.ones(1), hist)
    xs = []
    for k in range(cfg.nzeta):
        p, _, _ = O.ab5_push(cfg, p, flds, commit=True)
        xs.append(p.x[0])
    s = cfg.dzeta * np.arange(1, cfg.nzeta + 1)
    assert np.allclose(xs, a * np.cos(s / np.sqrt(2)), atol=1e-5 * a)


def test_absorbed_particles_are_frozen():
    cfg = box(8, 4.0)
    p = O.Plasma(np.array([3.99]), np.array([0.0]), np.array([5.0]),
                 np.zeros(1), np.zeros(1), np.ones(1), np.zeros((4, 5, 1)))
    shape = (9, 9)
    z = {k: np.zeros(shape) for k in ("exmby", "eypbx", "ez", "bx", "by", "bz")}
    q, _, nabs = O.ab5_push(cfg, p, z, commit=True)
    assert nabs == 1 and q.w[0] == 0 and q.x[0] == 3.99 and q.ux[0] == 5.0
    q2, _, nabs2 = O.ab5_push(cfg, q, z, commit=True)
    assert nabs2 == 0 and q2.x[0] == 3.99
