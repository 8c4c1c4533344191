"""Pins of the oracle's explicit Bx/By solver (Sec. III.B, second option of
the Bx/By field solver): the analytic d_zeta J_perp against finite
differences of the deposited current along the pusher's orbits, the
-chi B coupling, the linear-regime magnetic field against its closed form
(for both Bx/By solvers), and agreement with the predictor-corrector as the
slices get thinner."""
import dataclasses

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import j1

import workloads as W
from oracle import qsp_oracle as O
from test_oracle_loop import linear_theory, rel


def random_plasma(cfg, seed, margin=3):
    """A plasma slice with random displacements, momenta and Psi, a few
    particles on the 1+Psi floor; particles within `margin` cells of the
    edge are absorbed (weight 0) so that every stencil stays inside."""
    rng = np.random.default_rng(seed)
    p = O.init_plasma(cfg)
    n = p.x.size
    p.x = p.x + rng.uniform(-0.4, 0.4, n) * cfg.hx
    p.y = p.y + rng.uniform(-0.4, 0.4, n) * cfg.hy
    inner = ((p.x > cfg.x_lo + margin * cfg.hx) & (p.x < cfg.x_hi - margin * cfg.hx) &
             (p.y > cfg.y_lo + margin * cfg.hy) & (p.y < cfg.y_hi - margin * cfg.hy))
    p.w[~inner] = 0.0
    p.ux = rng.normal(0.0, 0.3, n)
    p.uy = rng.normal(0.0, 0.3, n)
    p.psi = rng.uniform(-0.5, 0.6, n)
    p.psi[::17] = -1.0 + 0.3 * cfg.psi_floor        # floored 1 + Psi
    p.w[::23] = 0.0                                 # absorbed particles
    return p


def smooth_fields(cfg, seed, bperp=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(*O.node_coords(cfg))
    out = {}
    for k in ("exmby", "eypbx", "ez", "bz"):
        a, x0, y0 = rng.normal(), rng.uniform(-2, 2), rng.uniform(-2, 2)
        out[k] = O.zero_boundary(a * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / 4.0))
    out["bx"] = np.full_like(X, bperp[0])
    out["by"] = np.full_like(X, bperp[1])
    out["psi"] = np.zeros_like(X)
    return out


def dzeta_current_fd(cfg, p, flds, eps=1e-8):
    """(J(zeta + eps) - J(zeta - eps)) / (2 eps) with the particles moved
    along the exact right-hand side of the pusher equations (eps small
    enough that hardly any particle crosses a kink of the linear shape)."""
    f, _ = O.particle_rhs(cfg, p, flds)
    js = []
    for sgn in (1.0, -1.0):
        q = p.copy()
        q.x, q.y, q.ux, q.uy, q.psi = (np.stack([p.x, p.y, p.ux, p.uy, p.psi]) + sgn * eps * f)
        js.append(O.plasma_deposit(cfg, q, ("jx", "jy")))
    return {c: (js[0][c] - js[1][c]) / (2 * eps) for c in ("jx", "jy")}


@pytest.mark.parametrize("order", [1, 2, 3])
def test_analytic_dzeta_current_matches_finite_differences(order):
    cfg, _ = W.small(n=32, nzeta=4, ppc=2)
    cfg = dataclasses.replace(cfg, shape_order=order)
    p = random_plasma(cfg, 3 + order)
    flds = smooth_fields(cfg, 11)
    fd = dzeta_current_fd(cfg, p, flds)
    src = O.explicit_sources(cfg, p, flds)
    for c, dj in (("jx", "djx"), ("jy", "djy")):
        err = np.linalg.norm(src[dj] - fd[c]) / np.linalg.norm(fd[c])
        assert err < 1e-6, (c, err)


def test_bperp_enters_as_minus_chi_b():
    # a uniform B_perp is gathered exactly, so its whole effect on
    # d_zeta J_perp is the node term (-chi By, +chi Bx)
    cfg, _ = W.small(n=32, nzeta=4, ppc=2)
    p = random_plasma(cfg, 8)
    b = (0.37, -0.61)
    fd0 = dzeta_current_fd(cfg, p, smooth_fields(cfg, 12))
    fd1 = dzeta_current_fd(cfg, p, smooth_fields(cfg, 12, bperp=b))
    chi = O.explicit_sources(cfg, p, smooth_fields(cfg, 12))["chi"]
    scale = np.abs(chi).max() * max(abs(b[0]), abs(b[1]))
    assert np.abs((fd1["jx"] - fd0["jx"]) - (-chi * b[1])).max() < 1e-7 * scale
    assert np.abs((fd1["jy"] - fd0["jy"]) - (chi * b[0])).max() < 1e-7 * scale
    # an unperturbed plasma has chi = n0 at every interior node
    q = O.init_plasma(cfg)
    chi0 = O.explicit_sources(cfg, q, smooth_fields(cfg, 12))["chi"]
    assert np.allclose(chi0[1:-1, 1:-1], cfg.n0, rtol=1e-13)


# ------------------------------------------------------- linear-regime B_perp
# Cold linear response to an electron beam n_b = nb f(r) g(zeta): at first
# order the plasma Jz is n0 psi (u_z = -Psi), d_zeta u_perp = E_perp and
# J_perp = -n0 u_perp, so eq. (bxby) becomes (lap - 1) By = -d_x n_b: the
# plasma return current screens the beam's magnetic field,
#   By = -nb g(zeta) d_x R(r),  R = (lap - 1)^-1 f,
#   dR/dr = s^2 int_0^inf k^2 J1(kr) exp(-k^2 s^2/2) / (1 + k^2) dk.

def dR_closed(r, s):
    return quad(lambda k: s * s * k * k * j1(k * r) * np.exp(-k * k * s * s / 2) / (1 + k * k),
                0, 40, limit=400)[0]


def test_closed_form_radial_derivative():
    # dR/dr of R = (lap - 1)^-1 exp(-r^2/2) by a finite difference of the
    # radial ODE solution R'' + R'/r - R = f, checked at one radius
    from test_oracle_loop import R_closed
    r, h = 1.3, 1e-4
    fd = (R_closed(r + h, 1.0) - R_closed(r - h, 1.0)) / (2 * h)
    assert abs(dR_closed(r, 1.0) - fd) < 1e-7


@pytest.mark.parametrize("solver", ["pc", "explicit"])
def test_linear_magnetic_field_matches_theory(solver):
    nb = 0.01
    cfg, _ = W.c1(nb)
    cfg.nx = cfg.ny = 64
    cfg.nzeta, cfg.dzeta = 64, 8.0 / 64
    cfg.bxby_solver = solver
    if solver == "pc":
        cfg.pc_max_iter, cfg.pc_tol = 20, 1e-12
    beam = W.GaussianBeam(W.gaussian_envelope(cfg, nb, -2.0, 1.0), 1.0, 1.0)
    j = cfg.ny // 2
    recs, _ = O.run_box(cfg, beam, keep=lambda k, r: (r["by"][j].copy(), r["bx"][j].copy(),
                                                     r["ez"][j].copy(), r["psi"][j].copy()))
    by = np.stack([r[0] for r in recs])
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    dr = np.array([np.sign(v) * dR_closed(abs(v), 1.0) for v in x])
    g = np.exp(-(cfg.zeta() + 2.0) ** 2 / 2.0)
    by_th = -nb * g[:, None] * dr[None, :]
    assert rel(by, by_th) < 0.04, rel(by, by_th)
    assert np.abs(np.stack([r[1] for r in recs])).max() < 1e-12   # Bx = 0 on y = 0
    ez_th, psi_th = linear_theory(cfg, nb)
    assert rel(np.stack([r[2] for r in recs]), ez_th) < 0.05
    assert rel(np.stack([r[3] for r in recs]), psi_th) < 0.05


def test_explicit_and_predictor_corrector_converge_together():
    # both solve eq. (bxby); their difference shrinks with the slice spacing
    def fields(nzeta, solver):
        cfg, beam = W.small(n=64, nzeta=nzeta, nb=1.0, pc_max_iter=40, pc_tol=1e-13)
        cfg.bxby_solver = solver
        recs, _ = O.run_box(cfg, beam)
        s = nzeta // 24
        return {q: O.stack(recs, q)[s - 1::s] for q in ("psi", "ez", "bx", "by")}
    d = []
    for nz in (24, 96):
        a, b = fields(nz, "pc"), fields(nz, "explicit")
        d.append({q: rel(b[q], a[q]) for q in a})
    assert all(v < 0.05 for v in d[0].values()), d
    for q in ("psi", "ez", "bx", "by"):
        assert d[1][q] < 0.5 * d[0][q], (q, d)
