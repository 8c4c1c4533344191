"""Plain FP64 CPU oracle of the quasi-static PIC per-slice loop.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the only common dependency is the input description in ``workloads``.

What it computes (HiPACE++, arXiv:2109.10277), in normalised units
(c = eps0 = mu0 = 1, lengths in k_p^-1, densities in n0, fields in E0):

* field equations, Sec. II eqs. (psi), (exmby), (ez), (bxby), (bz):
    lap psi = -(rho - Jz);  Ex-By = -d_x psi;  Ey+Bx = -d_y psi
    lap Ez  = d_x Jx + d_y Jy
    lap Bx  = -d_y Jz + d_zeta Jy;  lap By = d_x Jz - d_zeta Jx
    lap Bz  = d_y Jx - d_x Jy
* the 2D slice routine, Sec. II (enumerated steps 1-7), head to tail;
* the plasma pusher, Sec. III.B eqs. for d_zeta x_perp, d_zeta u_perp,
  d_zeta Psi and the Lorentz factor gamma(u_perp, Psi), for electrons
  (q = -1, M = m_e) with a fifth-order Adams-Bashforth step in zeta;
* deposition zeroth order in zeta with a transverse shape of order 0-3
  (centred B-splines; order 1, CIC, by default), Sec. III.B, the ions
  deposited from the electrons' rest lattice with the same shape;
* Dirichlet fast Poisson solves by a type-I discrete sine transform plus
  finite-difference operators, Sec. III.B ("solving a transverse Poisson
  equation");
* the Bx/By predictor-corrector, Sec. III.B, with the initial guess built
  from Bx/By of the two previous slices (Sec. V.B, the list of per-cell
  quantities S_cell), or the explicit Bx/By solver (Sec. III.B, second
  option): d_zeta J_perp integrated along the pusher's orbits and the
  resulting Helmholtz-like equation solved by a sparse factorisation;
* beams: rigid Gaussian sources or macro-particles sorted by slice once per
  time step and pushed once per slice, and the multi-time-step loop.

Where the paper is silent, this file takes the readings listed beside each
function (node-centred grid, centred differences, linear-extrapolation
initial guess, relative-L2 P-C criterion, 1+Psi floor, absorbing box edge).

Every step is a plain array expression or a library primitive
(``numpy.bincount`` for scatter-add, ``scipy.fft.dstn`` for the sine
transform).  Array layout: node fields are float64 arrays of shape
(ny+1, nx+1) indexed [j, i] (row = y).  Boundary rows/columns are zero.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence

import numpy as np
import scipy.fft

# fifth-order Adams-Bashforth weights for f_k, f_{k-1}, ..., f_{k-4}
# (standard textbook values, denominator 720)
AB5 = np.array([1901.0, -2774.0, 2616.0, -1274.0, 251.0]) / 720.0

FIELDS = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz")
DEPOSITS = ("rho_mjz", "jx", "jy", "jz", "rho")


# --------------------------------------------------------------------------
# Grid helpers
# --------------------------------------------------------------------------

def node_coords(cfg):
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    y = cfg.y_lo + cfg.hy * np.arange(cfg.ny + 1)
    return x, y


def zero_boundary(f: np.ndarray) -> np.ndarray:
    """Homogeneous Dirichlet nodes (index 0 and n on each axis) are zero."""
    f[0, :] = 0.0
    f[-1, :] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    return f


# --------------------------------------------------------------------------
# Plasma particles
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Plasma:
    """One slice of plasma electrons plus the Adams-Bashforth history.

    ``w`` is the macro-particle weight n0*hx*hy/(ppc_x*ppc_y) (charge per
    unit zeta is q*w); w = 0 marks an absorbed particle.  ``hist[m]`` holds
    the right-hand side f_{k-1-m} (m = 0..3) of the five integrated
    quantities (x, y, ux, uy, Psi).
    """
    x: np.ndarray
    y: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    psi: np.ndarray
    w: np.ndarray
    hist: np.ndarray          # [4, 5, N]

    def copy(self) -> "Plasma":
        return Plasma(*(np.array(getattr(self, f.name), copy=True)
                        for f in dataclasses.fields(Plasma)))


def init_plasma(cfg) -> Plasma:
    """Unperturbed plasma ahead of the box (Sec. II: "a slice of unperturbed
    plasma is initialized ahead of the beams"): electrons at rest on a
    uniform lattice, Psi = 0 and zero history (exact for a plasma that has
    not yet met any field)."""
    nX, nY = cfg.nx * cfg.ppc_x, cfg.ny * cfg.ppc_y
    I, J = np.meshgrid(np.arange(nX), np.arange(nY))
    x = cfg.x_lo + (I.ravel() + 0.5) * cfg.hx / cfg.ppc_x
    y = cfg.y_lo + (J.ravel() + 0.5) * cfg.hy / cfg.ppc_y
    n = x.size
    w = np.full(n, cfg.n0 * cfg.hx * cfg.hy / (cfg.ppc_x * cfg.ppc_y))
    z = np.zeros(n)
    return Plasma(x=x, y=y, ux=z.copy(), uy=z.copy(), psi=z.copy(), w=w,
                  hist=np.zeros((4, 5, n)))


def shape_1d(s, n: int, order: int):
    """Transverse particle shape of order 0-3 (Sec. III.B: orders 0-3 are
    available transversely) along one axis: the centred B-spline of degree
    ``order`` (the box function convolved with itself ``order`` times)
    evaluated at the node offsets, for positions s in node units
    (0 <= s <= n).  Returns (node index arrays, weight arrays); nodes may fall
    outside 0..n, where the field is zero and deposits are dropped.

      order 0 (NGP): nearest node b = floor(s + 1/2)
      order 1 (CIC): b = floor(s) (b = n - 1 at s = n), d = s - b:
                     (1 - d, d) on (b, b + 1)
      order 2:       b = floor(s + 1/2), d = s - b in [-1/2, 1/2):
                     ((1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2) on b-1 .. b+1
      order 3:       b = floor(s), d = s - b in [0, 1):
                     ((1-d)^3, 4 - 6d^2 + 3d^3, 1 + 3d + 3d^2 - 3d^3, d^3) / 6 on b-1 .. b+2
    """
    s = np.asarray(s, dtype=np.float64)
    if order == 0:
        b = np.floor(s + 0.5).astype(np.int64)
        return [b], [np.ones_like(s)]
    if order == 1:
        b = np.clip(np.floor(s).astype(np.int64), 0, n - 1)
        d = s - b
        return [b, b + 1], [1.0 - d, d]
    if order == 2:
        b = np.floor(s + 0.5).astype(np.int64)
        d = s - b
        return [b - 1, b, b + 1], [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
    if order == 3:
        b = np.floor(s).astype(np.int64)
        d = s - b
        return ([b - 1, b, b + 1, b + 2],
                [(1.0 - d) ** 3 / 6.0, (4.0 - 6.0 * d * d + 3.0 * d ** 3) / 6.0,
                 (1.0 + 3.0 * d + 3.0 * d * d - 3.0 * d ** 3) / 6.0, d ** 3 / 6.0])
    raise ValueError("shape order must be 0, 1, 2 or 3")


def shape_1d_slope(s, n: int, order: int):
    """Derivatives d w / d s of the ``shape_1d`` weights, in the same node
    order (orders 1-3; the order-0 shape is piecewise constant)."""
    s = np.asarray(s, dtype=np.float64)
    if order == 1:
        return [-np.ones_like(s), np.ones_like(s)]
    if order == 2:
        d = s - np.floor(s + 0.5)
        return [-(0.5 - d), -2.0 * d, 0.5 + d]
    if order == 3:
        d = s - np.floor(s)
        return [-0.5 * (1.0 - d) ** 2, (-12.0 * d + 9.0 * d * d) / 6.0,
                (3.0 + 6.0 * d - 9.0 * d * d) / 6.0, 0.5 * d * d]
    raise ValueError("shape slopes exist for orders 1, 2 and 3")


def shape_order(cfg) -> int:
    return int(getattr(cfg, "shape_order", 1))


def shape_weights(cfg, x, y):
    """2D tensor-product shape of the configured order: lists of node index
    pairs and weights (one entry per stencil node)."""
    o = shape_order(cfg)
    ni, wi = shape_1d((x - cfg.x_lo) / cfg.hx, cfg.nx, o)
    nj, wj = shape_1d((y - cfg.y_lo) / cfg.hy, cfg.ny, o)
    nodes, wts = [], []
    for j, wy in zip(nj, wj):
        for i, wx in zip(ni, wi):
            nodes.append((i, j))
            wts.append(wx * wy)
    return nodes, wts


def _valid(cfg, i, j):
    return (i >= 0) & (i <= cfg.nx) & (j >= 0) & (j <= cfg.ny)


def deposit_values(cfg, x, y, values: np.ndarray) -> np.ndarray:
    """Scatter-add per-particle density ``values`` to the nodes with the
    configured transverse shape (zeroth order in zeta); deposits on or
    beyond the boundary nodes are dropped."""
    out = np.zeros((cfg.ny + 1) * (cfg.nx + 1))
    nodes, wts = shape_weights(cfg, x, y)
    for (i, j), s in zip(nodes, wts):
        ok = _valid(cfg, i, j)
        out += np.bincount((j * (cfg.nx + 1) + i)[ok], weights=(values * s)[ok],
                           minlength=out.size)
    return zero_boundary(out.reshape(cfg.ny + 1, cfg.nx + 1))


def deposit_slopes(cfg, x, y, ax: np.ndarray, ay: np.ndarray) -> np.ndarray:
    """Scatter-add of ax dS/dx_p + ay dS/dy_p per particle: the rate of
    change of a deposit when the particle moves with velocity (ax, ay) per
    unit of its weight (the shape's derivative with respect to the particle
    position, tensor product of ``shape_1d_slope`` and ``shape_1d``)."""
    o = shape_order(cfg)
    sx = (x - cfg.x_lo) / cfg.hx
    sy = (y - cfg.y_lo) / cfg.hy
    ni, wi = shape_1d(sx, cfg.nx, o)
    nj, wj = shape_1d(sy, cfg.ny, o)
    gi = shape_1d_slope(sx, cfg.nx, o)
    gj = shape_1d_slope(sy, cfg.ny, o)
    out = np.zeros((cfg.ny + 1) * (cfg.nx + 1))
    for j, wy, dwy in zip(nj, wj, gj):
        for i, wx, dwx in zip(ni, wi, gi):
            ok = _valid(cfg, i, j)
            v = ax * dwx * wy / cfg.hx + ay * wx * dwy / cfg.hy
            out += np.bincount((j * (cfg.nx + 1) + i)[ok], weights=v[ok], minlength=out.size)
    return zero_boundary(out.reshape(cfg.ny + 1, cfg.nx + 1))


def gather(cfg, field: np.ndarray, x, y) -> np.ndarray:
    """Interpolate a node field to the particles with the same shape (the
    transpose of ``deposit_values`` up to the 1/(hx hy) density
    normalisation); nodes beyond the box read zero."""
    nodes, wts = shape_weights(cfg, x, y)
    total = 0.0
    for (i, j), s in zip(nodes, wts):
        ok = _valid(cfg, i, j)
        total = total + np.where(ok, field[np.clip(j, 0, cfg.ny), np.clip(i, 0, cfg.nx)], 0.0) * s
    return total


def clamp_d(cfg, psi):
    """D = 1 + Psi, floored at cfg.psi_floor (the paper's equations are
    singular at 1 + Psi = 0 and it does not say how that is handled)."""
    return np.maximum(1.0 + psi, cfg.psi_floor)


def gamma_of(ux, uy, d):
    """Lorentz factor from the transverse momentum and 1 + Psi, Sec. III.B
    eq. for gamma_p."""
    return (1.0 + ux * ux + uy * uy + d * d) / (2.0 * d)


def plasma_deposit(cfg, p: Plasma, channels: Sequence[str] = DEPOSITS):
    """Charge and current densities of the plasma electrons (q = -1).

    A macro-particle crossing the slice contributes q*w*S/(hx hy) times
    1/(1 - v_z) = gamma/(1 + Psi) to rho, and rho*v to J.  Hence
    rho - Jz = q*w*S/(hx hy) exactly (the quasi-static invariant
    gamma - u_z = 1 + Psi), which is deposited on its own channel so the
    psi source never forms the difference of two large numbers.
    """
    d = clamp_d(cfg, p.psi)
    g = gamma_of(p.ux, p.uy, d)
    uz = g - d
    qn = -p.w / (cfg.hx * cfg.hy)          # q * w / cell area
    per = {"rho_mjz": qn,
           "jx": qn * p.ux / d,
           "jy": qn * p.uy / d,
           "jz": qn * uz / d,
           "rho": qn * g / d}
    return {c: deposit_values(cfg, p.x, p.y, per[c]) for c in channels}


def ion_density(cfg) -> np.ndarray:
    """Density of the immobile ions (Sec. II: ions remain practically
    immobile).  They are taken as a neutralising species sitting on the
    electrons' rest lattice and deposited with the same transverse shape, so
    the unperturbed plasma is neutral node by node for every shape order,
    also next to the box edge where a stencil of order >= 2 reaches past it.
    For order 1 this is n0 at every interior node."""
    key = (cfg.nx, cfg.ny, cfg.ppc_x, cfg.ppc_y, cfg.x_lo, cfg.y_lo, cfg.hx,
           cfg.hy, cfg.n0, shape_order(cfg))
    ion = _ION_CACHE.get(key)
    if ion is None:
        p = init_plasma(cfg)
        ion = deposit_values(cfg, p.x, p.y, p.w / (cfg.hx * cfg.hy))
        _ION_CACHE[key] = ion
    return ion


_ION_CACHE: dict = {}


def add_ion_background(cfg, dep: dict) -> dict:
    """Add the ion charge density to rho and rho - Jz (the ions carry no
    current)."""
    ion = ion_density(cfg)
    for c in ("rho_mjz", "rho"):
        if c in dep:
            dep[c] = dep[c] + ion
    return dep


def particle_rhs(cfg, p: Plasma, flds: dict):
    """d/dzeta of (x, y, ux, uy, Psi) for electrons (q = -1, M = m_e, so
    -q/M = +1 and -q m_e/(M e) = +1), Sec. III.B pusher equations:

      dx/dzeta   = -ux / D
      dux/dzeta  = gamma/D (Ex-By) + By + Bz uy / D
      duy/dzeta  = gamma/D (Ey+Bx) - Bx - Bz ux / D
      dPsi/dzeta = (ux (Ex-By) + uy (Ey+Bx)) / D - Ez

    with D = 1 + Psi (floored) and the six fields gathered at the particle.
    Returns (f [5, N], number of particles whose D was floored).
    """
    g = {k: gather(cfg, flds[k], p.x, p.y)
         for k in ("exmby", "eypbx", "ez", "bx", "by", "bz")}
    raw = 1.0 + p.psi
    d = np.maximum(raw, cfg.psi_floor)
    gam = gamma_of(p.ux, p.uy, d)
    f = np.empty((5, p.x.size))
    f[0] = -p.ux / d
    f[1] = -p.uy / d
    f[2] = gam / d * g["exmby"] + g["by"] + g["bz"] * p.uy / d
    f[3] = gam / d * g["eypbx"] - g["bx"] - g["bz"] * p.ux / d
    f[4] = (p.ux * g["exmby"] + p.uy * g["eypbx"]) / d - g["ez"]
    alive = p.w > 0
    f[:, ~alive] = 0.0
    nclamp = int(np.count_nonzero(alive & (raw < cfg.psi_floor)))
    return f, nclamp


def ab5_push(cfg, p: Plasma, flds: dict, commit: bool):
    """Advance the slice from zeta_k to zeta_{k+1} = zeta_k - dzeta with the
    fifth-order Adams-Bashforth formula (Sec. III.B; history zero before
    the first slice):

      y_{k+1} = y_k - dzeta * sum_m AB5[m] f_{k-m}

    A particle that ends outside the box is absorbed: its weight becomes 0
    and its state keeps the last in-box values.  With ``commit`` the new
    f_k is pushed onto the history (the real push); without it (the
    predictor-corrector trial push) the history is left alone.
    Returns (new plasma, clamp count, newly absorbed count).
    """
    f, nclamp = particle_rhs(cfg, p, flds)
    incr = AB5[0] * f
    for m in range(4):
        incr = incr + AB5[m + 1] * p.hist[m]
    q = p.copy()
    new = np.stack([p.x, p.y, p.ux, p.uy, p.psi]) - cfg.dzeta * incr
    alive = p.w > 0
    inside = ((new[0] >= cfg.x_lo) & (new[0] <= cfg.x_hi) &
              (new[1] >= cfg.y_lo) & (new[1] <= cfg.y_hi))
    move = alive & inside
    q.x[move], q.y[move], q.ux[move], q.uy[move], q.psi[move] = new[:, move]
    absorbed = alive & ~inside
    q.w[absorbed] = 0.0
    if commit:
        q.hist = np.concatenate([f[None], p.hist[:3]], axis=0)
    return q, nclamp, int(np.count_nonzero(absorbed))


# --------------------------------------------------------------------------
# Field solve
# --------------------------------------------------------------------------

def laplacian_eigenvalues(cfg) -> np.ndarray:
    """Eigenvalues of the 5-point Laplacian with zero Dirichlet nodes on the
    sine modes sin(pi p i / nx) sin(pi q j / ny), shape (ny-1, nx-1)."""
    p = np.arange(1, cfg.nx)
    q = np.arange(1, cfg.ny)
    lx = -4.0 / cfg.hx ** 2 * np.sin(np.pi * p / (2 * cfg.nx)) ** 2
    ly = -4.0 / cfg.hy ** 2 * np.sin(np.pi * q / (2 * cfg.ny)) ** 2
    return ly[:, None] + lx[None, :]


def poisson_solve(cfg, src: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """Solve (lap_h - shift) u = src on the interior nodes with u = 0 on the
    boundary (fast Poisson solver by a type-I DST, Sec. III.B): transform,
    divide by the eigenvalues, transform back.  shift = 0 is the Poisson
    problem of the field equations; the predictor-corrector uses shift > 0."""
    s = src[1:-1, 1:-1]
    shat = scipy.fft.dstn(s, type=1)
    u = np.zeros_like(src)
    u[1:-1, 1:-1] = scipy.fft.idstn(
        shat / (laplacian_eigenvalues(cfg) - shift), type=1)
    return u


def ddx(cfg, f: np.ndarray) -> np.ndarray:
    """Centred x difference at interior nodes; boundary result set to 0."""
    out = np.zeros_like(f)
    out[1:-1, 1:-1] = (f[1:-1, 2:] - f[1:-1, :-2]) / (2.0 * cfg.hx)
    return out


def ddy(cfg, f: np.ndarray) -> np.ndarray:
    out = np.zeros_like(f)
    out[1:-1, 1:-1] = (f[2:, 1:-1] - f[:-2, 1:-1]) / (2.0 * cfg.hy)
    return out


def solve_psi_ez_bz(cfg, dep: dict) -> dict:
    """Steps 4-6 of the slice routine: psi from eq. (psi), Ex-By and Ey+Bx
    from eq. (exmby), Ez from eq. (ez), Bz from eq. (bz)."""
    psi = poisson_solve(cfg, -dep["rho_mjz"])
    ez = poisson_solve(cfg, ddx(cfg, dep["jx"]) + ddy(cfg, dep["jy"]))
    bz = poisson_solve(cfg, ddy(cfg, dep["jx"]) - ddx(cfg, dep["jy"]))
    return {"psi": psi, "exmby": -ddx(cfg, psi), "eypbx": -ddy(cfg, psi),
            "ez": ez, "bz": bz}


def pc_shift(cfg) -> float:
    """Screening shift s of the predictor-corrector iteration.  A change dB
    of Bx/By at slice k changes the trial u_perp at k+1 by
    -dzeta*AB5[0]*dB, hence J_perp(k+1) and the centred d_zeta J_perp term
    of the Bx/By source by (AB5[0]/2) * n/D * dB; for the unperturbed
    plasma (n/D = n0) that is s = (1901/1440) n0."""
    if getattr(cfg, "pc_shift", None) is not None:
        return float(cfg.pc_shift)
    return 0.5 * AB5[0] * cfg.n0


def bxby_sources(cfg, jz_k, jx_prev, jy_prev, jx_next, jy_next):
    """Right-hand sides of eq. (bxby) with d_zeta J_perp at slice k taken as
    the centred difference (J_{k-1} - J_{k+1}) / (2 dzeta) (slice k-1 lies
    at zeta + dzeta, slice k+1 at zeta - dzeta)."""
    dz2 = 2.0 * cfg.dzeta
    sbx = -ddy(cfg, jz_k) + (jy_prev - jy_next) / dz2
    sby = ddx(cfg, jz_k) - (jx_prev - jx_next) / dz2
    return zero_boundary(sbx), zero_boundary(sby)


def solve_bxby(cfg, jz_k, jx_prev, jy_prev, jx_next, jy_next, bx_old, by_old):
    """One corrector solve of eq. (bxby).  The equation lap B = S(B) is
    written as (lap - s) B_new = S(B_old) - s B_old: it has the same
    solution at the fixed point B_new = B_old, but the iteration contracts
    (the unshifted map multiplies the longest sine modes by ~1.32/k^2 and
    diverges)."""
    s = pc_shift(cfg)
    sbx, sby = bxby_sources(cfg, jz_k, jx_prev, jy_prev, jx_next, jy_next)
    return (poisson_solve(cfg, sbx - s * bx_old, s),
            poisson_solve(cfg, sby - s * by_old, s))


# --------------------------------------------------------------------------
# Beams
# --------------------------------------------------------------------------

def gaussian_beam_density(cfg, beam, k: int) -> np.ndarray:
    """n_b of a rigid Gaussian beam sampled at the nodes of slice k (point
    sample in zeta: zeroth-order longitudinal deposition)."""
    x, y = node_coords(cfg)
    gx = np.exp(-(x - beam.x0) ** 2 / (2.0 * beam.sigma_x ** 2))
    gy = np.exp(-(y - beam.y0) ** 2 / (2.0 * beam.sigma_y ** 2))
    return zero_boundary(beam.amp[k] * gy[:, None] * gx[None, :])


def gaussian_beam_source(cfg, beam, k: int) -> dict:
    """Rigid ultra-relativistic electron beam (v = c along z):
    rho_b = Jz_b = -n_b, J_perp = 0, so rho_b - Jz_b = 0."""
    nb = gaussian_beam_density(cfg, beam, k)
    return {"rho": -nb, "jz": -nb}


def beam_slice_index(cfg, zeta: np.ndarray) -> np.ndarray:
    """Nearest slice of each beam particle (zeroth order in zeta)."""
    return np.rint((cfg.zeta_hi - zeta) / cfg.dzeta).astype(np.int64)


def beam_slices(cfg, b) -> np.ndarray:
    """Slice of each beam particle for the current time step.  The beam is
    sorted per slice once per time step, before the loop over slices
    (Sec. III.A), so a particle keeps the slice it had at the start of the
    box for its deposit and its push even if the push moves it across a
    slice boundary; ``run_box`` fixes this assignment.  Outside a box the
    assignment is taken from the current positions."""
    frozen = getattr(b, "_slice_of_step", None)
    return frozen if frozen is not None else beam_slice_index(cfg, b.zeta)


def particle_beam_source(cfg, b, k: int) -> dict:
    """Deposit of the macro-particles of slice k (NGP in zeta, CIC
    transversely): rho = q w S / (hx hy dzeta), Jz = rho v_z, with
    rho - Jz = rho (1 + u_perp^2) / (gamma (gamma + u_z)) written so it does
    not cancel; the transverse beam current is neglected."""
    sel = (beam_slices(cfg, b) == k)
    x, y = b.x[sel].astype(np.float64), b.y[sel].astype(np.float64)
    ux, uy, uz = (b.ux[sel].astype(np.float64), b.uy[sel].astype(np.float64),
                  b.uz[sel].astype(np.float64))
    w = b.w[sel].astype(np.float64)
    inside = (x >= cfg.x_lo) & (x <= cfg.x_hi) & (y >= cfg.y_lo) & (y <= cfg.y_hi)
    x, y, ux, uy, uz, w = (a[inside] for a in (x, y, ux, uy, uz, w))
    g = np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
    rho = -w / (cfg.hx * cfg.hy * cfg.dzeta)
    return {"rho": deposit_values(cfg, x, y, rho),
            "jz": deposit_values(cfg, x, y, rho * uz / g),
            "rho_mjz": deposit_values(cfg, x, y,
                                      rho * (1.0 + ux * ux + uy * uy) /
                                      (g * (g + uz)))}


def beam_push_slice(cfg, b, k: int, flds: dict, dt: float) -> None:
    """Advance the macro-particles of slice k by one time step dt with the
    slice-k fields (Sec. III.A: beam gather and push run per slice inside the
    loop; Sec. III.B: a second-order symplectic integrator).  Reading:
    drift - kick - drift, the kick a Boris step (electric half kick,
    magnetic rotation, electric half kick) for an electron (q = -1):

      x_h   = x + dt/2 u_perp/gamma,   zeta_h = zeta + dt/2 (u_z/gamma - 1)
      E, B gathered (CIC) at x_h from the slice's fields, with
      E_perp = (Ex-By + By, Ey+Bx - Bx); zero outside the box
      u-    = u + q dt/2 E;  t = q dt/2 B/gamma(u-);  s = 2t/(1+t.t)
      u'    = u- + u- x t;   u+ = u- + u' x s;   u_new = u+ + q dt/2 E
      x_new = x_h + dt/2 u_perp_new/gamma_new,  zeta likewise.

    The particle keeps its slice for the gather.  Mutates ``b`` in place."""
    sel = np.nonzero(beam_slices(cfg, b) == k)[0]
    if sel.size == 0:
        return
    x, y, z = b.x[sel].astype(np.float64), b.y[sel].astype(np.float64), b.zeta[sel].astype(np.float64)
    u = np.stack([b.ux[sel], b.uy[sel], b.uz[sel]]).astype(np.float64)
    g0 = np.sqrt(1.0 + np.sum(u * u, axis=0))
    xh = x + 0.5 * dt * u[0] / g0
    yh = y + 0.5 * dt * u[1] / g0
    zh = z + 0.5 * dt * (u[2] / g0 - 1.0)
    inside = (xh >= cfg.x_lo) & (xh <= cfg.x_hi) & (yh >= cfg.y_lo) & (yh <= cfg.y_hi)
    xs, ys = np.clip(xh, cfg.x_lo, cfg.x_hi), np.clip(yh, cfg.y_lo, cfg.y_hi)
    gat = {k2: np.where(inside, gather(cfg, flds[k2], xs, ys), 0.0)
           for k2 in ("exmby", "eypbx", "ez", "bx", "by", "bz")}
    E = np.stack([gat["exmby"] + gat["by"], gat["eypbx"] - gat["bx"], gat["ez"]])
    B = np.stack([gat["bx"], gat["by"], gat["bz"]])
    q = -1.0
    um = u + 0.5 * q * dt * E
    gm = np.sqrt(1.0 + np.sum(um * um, axis=0))
    t = 0.5 * q * dt * B / gm
    sv = 2.0 * t / (1.0 + np.sum(t * t, axis=0))
    up = um + np.cross(um, t, axis=0)
    upl = um + np.cross(up, sv, axis=0)
    un = upl + 0.5 * q * dt * E
    g1 = np.sqrt(1.0 + np.sum(un * un, axis=0))
    b.x[sel] = xh + 0.5 * dt * un[0] / g1
    b.y[sel] = yh + 0.5 * dt * un[1] / g1
    b.zeta[sel] = zh + 0.5 * dt * (un[2] / g1 - 1.0)
    b.ux[sel], b.uy[sel], b.uz[sel] = un


def beam_source(cfg, beam, k: int) -> dict:
    if beam is None:
        return {}
    if hasattr(beam, "amp"):
        return gaussian_beam_source(cfg, beam, k)
    if callable(beam):
        return beam(k)
    return particle_beam_source(cfg, beam, k)


# --------------------------------------------------------------------------
# Explicit Bx/By solver
# --------------------------------------------------------------------------

def explicit_sources(cfg, p: Plasma, flds: dict) -> dict:
    """Explicit d_zeta J_perp (Sec. III.B, the explicit Bx/By solver: the
    longitudinal derivative is integrated analytically instead of iterated).

    The plasma current is J_perp = sum_p q w_p S(x - x_p) u_p / D_p (per
    cell area), so along the particle orbits of the Sec. III.B pusher
      d_zeta J_perp = sum_p q w_p [ S d(u/D)/dzeta + (u/D) dS/dzeta ],
      d(u/D)/dzeta  = (du/dzeta) / D - u (dPsi/dzeta) / D^2,
      dS/dzeta      = grad_p S . dx_p/dzeta = -grad_p S . u / D.
    du_x/dzeta = a_x + By and du_y/dzeta = a_y - Bx, where
    a_x = gamma/D (Ex-By) + Bz u_y/D and a_y = gamma/D (Ey+Bx) - Bz u_x/D
    hold only quantities known before the Bx/By solve.  Hence
      d_zeta Jx = DJx - chi By,   d_zeta Jy = DJy + chi Bx,
      chi = sum_p w_p S / D  (> 0 for electrons, q = -1),
    with DJ the deposit of everything else.  The B_perp terms, gathered at
    the particles, are taken at the node (chi B) so that the Bx/By equation
    stays linear on the grid.  A floored D is constant along the orbit.
    Returns {"chi", "djx", "djy"} (node arrays, boundary zero)."""
    g = {k: gather(cfg, flds[k], p.x, p.y) for k in ("exmby", "eypbx", "ez", "bz")}
    raw = 1.0 + p.psi
    d = np.maximum(raw, cfg.psi_floor)
    gam = gamma_of(p.ux, p.uy, d)
    ax = gam / d * g["exmby"] + g["bz"] * p.uy / d
    ay = gam / d * g["eypbx"] - g["bz"] * p.ux / d
    apsi = np.where(raw < cfg.psi_floor, 0.0,
                    (p.ux * g["exmby"] + p.uy * g["eypbx"]) / d - g["ez"])
    wa = p.w / (cfg.hx * cfg.hy)
    qn = -wa                                  # q w / cell area
    vx, vy = p.ux / d, p.uy / d
    djx = deposit_values(cfg, p.x, p.y, qn * (ax / d - p.ux * apsi / d ** 2))
    djy = deposit_values(cfg, p.x, p.y, qn * (ay / d - p.uy * apsi / d ** 2))
    djx = djx + deposit_slopes(cfg, p.x, p.y, -qn * vx * vx, -qn * vx * vy)
    djy = djy + deposit_slopes(cfg, p.x, p.y, -qn * vy * vx, -qn * vy * vy)
    chi = deposit_values(cfg, p.x, p.y, wa / d)
    return {"chi": chi, "djx": djx, "djy": djy}


def helmholtz_solve(cfg, rhs: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """Solve (lap_h - chi) u = rhs on the interior nodes, u = 0 on the
    boundary, by a sparse direct factorisation of the 5-point operator
    (a library primitive; chi varies from node to node)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    mx, my = cfg.nx - 1, cfg.ny - 1
    lx = sp.diags([np.ones(mx - 1), -2.0 * np.ones(mx), np.ones(mx - 1)], [-1, 0, 1]) / cfg.hx ** 2
    ly = sp.diags([np.ones(my - 1), -2.0 * np.ones(my), np.ones(my - 1)], [-1, 0, 1]) / cfg.hy ** 2
    a = sp.kron(sp.identity(my), lx) + sp.kron(ly, sp.identity(mx))
    a = (a - sp.diags(chi[1:-1, 1:-1].ravel())).tocsc()
    u = np.zeros_like(rhs)
    u[1:-1, 1:-1] = spl.spsolve(a, rhs[1:-1, 1:-1].ravel()).reshape(my, mx)
    return u


def explicit_bxby(cfg, jz_k: np.ndarray, src: dict):
    """Eq. (bxby) with the explicit d_zeta J_perp of ``explicit_sources``:
      lap Bx = -d_y Jz + DJy + chi Bx  ->  (lap - chi) Bx = -d_y Jz + DJy
      lap By =  d_x Jz - DJx + chi By  ->  (lap - chi) By =  d_x Jz - DJx
    a Helmholtz-like equation with a node-dependent coefficient."""
    rx = zero_boundary(-ddy(cfg, jz_k) + src["djy"])
    ry = zero_boundary(ddx(cfg, jz_k) - src["djx"])
    return helmholtz_solve(cfg, rx, src["chi"]), helmholtz_solve(cfg, ry, src["chi"])


def bxby_solver(cfg) -> str:
    return getattr(cfg, "bxby_solver", "pc")


# --------------------------------------------------------------------------
# One slice and the box
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SliceState:
    """Everything slice k needs from earlier slices (Sec. V.B: J_perp of the
    previous slice and Bx/By of the two previous slices, plus one slice of
    plasma particles with its Adams-Bashforth history)."""
    k: int
    plasma: Plasma
    jx_prev: np.ndarray
    jy_prev: np.ndarray
    bx_prev1: np.ndarray
    by_prev1: np.ndarray
    bx_prev2: np.ndarray
    by_prev2: np.ndarray

    def copy(self) -> "SliceState":
        return SliceState(self.k, self.plasma.copy(),
                          *(np.array(getattr(self, n), copy=True) for n in
                            ("jx_prev", "jy_prev", "bx_prev1", "by_prev1",
                             "bx_prev2", "by_prev2")))


def initial_state(cfg) -> SliceState:
    z = np.zeros((cfg.ny + 1, cfg.nx + 1))
    return SliceState(0, init_plasma(cfg), z, z.copy(), z.copy(), z.copy(),
                      z.copy(), z.copy())


def total_deposit(cfg, p: Plasma, beam, k: int) -> dict:
    """Steps 2-3 of the slice routine: plasma deposit, ion background and
    the beam source of slice k."""
    dep = add_ion_background(cfg, plasma_deposit(cfg, p))
    for c, v in beam_source(cfg, beam, k).items():
        dep[c] = dep[c] + v
    return dep


def predictor_corrector(cfg, st: SliceState, flds: dict, dep: dict):
    """Bx/By predictor-corrector (Sec. III.B).  Initial guess by linear
    extrapolation from the two previous slices, B0 = 2 B_{k-1} - B_{k-2}.
    Each iteration trial-pushes a copy of the particles to slice k+1 with
    the current B, deposits Jx, Jy there, solves eq. (bxby) (in the
    screened form of ``solve_bxby``) and measures
    r = ||B_new - B_old|| / ||B_new|| over both components (FP64).  It stops
    when r < pc_tol (pc_tol > 0) or after pc_max_iter iterations.
    Returns (bx, by, iterations, residual list, clamp count of the trials)."""
    bx = 2.0 * st.bx_prev1 - st.bx_prev2
    by = 2.0 * st.by_prev1 - st.by_prev2
    res = []
    nclamp = 0
    it = 0
    for it in range(1, cfg.pc_max_iter + 1):
        trial_flds = dict(flds, bx=bx, by=by)
        trial, nc, _ = ab5_push(cfg, st.plasma, trial_flds, commit=False)
        nclamp += nc
        jn = plasma_deposit(cfg, trial, ("jx", "jy"))
        bx_new, by_new = solve_bxby(cfg, dep["jz"], st.jx_prev, st.jy_prev,
                                    jn["jx"], jn["jy"], bx, by)
        num = np.sum((bx_new - bx) ** 2) + np.sum((by_new - by) ** 2)
        den = np.sum(bx_new ** 2) + np.sum(by_new ** 2)
        r = np.sqrt(num / den) if den > 0 else (0.0 if num == 0 else np.inf)
        res.append(float(r))
        bx, by = bx_new, by_new
        if cfg.pc_tol > 0 and r < cfg.pc_tol:
            break
    return bx, by, it, res, nclamp


def advance_slice(cfg, st: SliceState, beam):
    """Compute the fields of slice st.k and push the plasma to slice k+1
    (the 2D slice routine of Sec. II, with the predictor-corrector or the
    explicit solver as step 7).  A macro-particle beam with a non-zero ``dt`` also has its
    slice-k particles pushed by one time step once the slice's fields are
    final (mutating the beam).  Returns (state at k+1, record of slice k)."""
    k = st.k
    dep = total_deposit(cfg, st.plasma, beam, k)
    flds = solve_psi_ez_bz(cfg, dep)
    if bxby_solver(cfg) == "explicit":
        bx, by = explicit_bxby(cfg, dep["jz"], explicit_sources(cfg, st.plasma, flds))
        its, res, nclamp_pc = 0, [], 0
    else:
        bx, by, its, res, nclamp_pc = predictor_corrector(cfg, st, flds, dep)
    flds["bx"], flds["by"] = bx, by
    if beam is not None and hasattr(beam, "zeta") and getattr(beam, "dt", 0.0):
        beam_push_slice(cfg, beam, k, flds, beam.dt)
    new_plasma, nclamp, nabs = ab5_push(cfg, st.plasma, flds, commit=True)
    rec = dict(flds)
    rec.update(dep)
    rec["pc_iters"] = its
    rec["pc_residuals"] = res
    rec["n_clamped"] = nclamp
    rec["n_absorbed"] = nabs
    nxt = SliceState(k + 1, new_plasma, dep["jx"], dep["jy"], bx, by,
                     st.bx_prev1, st.by_prev1)
    return nxt, rec


def run_box(cfg, beam, keep: Optional[Callable[[int, dict], dict]] = None,
            state: Optional[SliceState] = None, k_end: Optional[int] = None):
    """Run slices st.k .. k_end-1 (default: the whole box from the head).
    ``keep(k, rec)`` selects what to retain per slice (default: all fields
    and deposits).  Returns (list of kept records, final state)."""
    st = initial_state(cfg) if state is None else state
    k_end = cfg.nzeta if k_end is None else k_end
    out = []
    particle_beam = beam is not None and hasattr(beam, "zeta")
    if particle_beam:
        beam._slice_of_step = beam_slice_index(cfg, beam.zeta)
    try:
        while st.k < k_end:
            k = st.k
            st, rec = advance_slice(cfg, st, beam)
            out.append(rec if keep is None else keep(k, rec))
    finally:
        if particle_beam:
            beam._slice_of_step = None
    return out, st


def run_steps(cfg, beam, nsteps: int, state_fn: Optional[Callable[[], "SliceState"]] = None,
              after_step: Optional[Callable[[int, list], None]] = None):
    """Multi-time-step loop (Sec. II): each time step runs the whole box
    from the head with a fresh plasma (``state_fn()``, default the
    unperturbed plasma) while the beam macro-particles advance by their
    time step dt in every slice; ``after_step(step, records)`` sees each
    box.  Mutates ``beam``."""
    for step in range(nsteps):
        st = state_fn() if state_fn is not None else None
        recs, _ = run_box(cfg, beam, keep=lambda k, r: {}, state=st)
        if after_step is not None:
            after_step(step, recs)


def stack(records: Sequence[dict], name: str) -> np.ndarray:
    return np.stack([r[name] for r in records])
