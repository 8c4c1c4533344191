"""Seeded synthetic workloads for the quasi-static PIC slice loop.

This module only *describes inputs*: grid and box geometry, plasma lattice
density, beam envelopes and seeded random draws.  It holds none of the
method's arithmetic (no deposit, push, source or solve), so both the FP64
oracle under ``oracle/`` and the HIP product path may use it.

The workloads follow the paper's reference setup (Sec. IV and the Appendix:
Gaussian driver and witness beams in a uniform plasma with immobile ions,
normalised units, domain (-8,8)^2 x (-7,5) k_p^-1, dt = 6 / omega_p) scaled to
the five configurations the hot path is exercised on:

* ``c1``  64^2 x 64 linear wake (n_b/n0 = 0.01), 3 fixed P-C iterations
* ``c2``  512^2 x 1024 blowout wake (n_b/n0 = 10), P-C to 1e-4, <= 5 iterations
* ``c3``  1024^2 x 1024 paper-scale step with 2 x 2^21 macro-particle beams
* ``c4``  256^2 x 512 adjoint workload, per-slice amplitudes with 5% noise
* ``c5``  1024^2 x 1024, 2x2 plasma lattice, adjoint with memory pressure

All lengths are in units of k_p^-1, densities in units of n0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED = 210910277

# Floor applied to 1 + Psi before it is used as a divisor (the paper leaves the
# singular limit unspecified; both implementations clamp the same way).
ONE_PLUS_PSI_FLOOR = 0.01


@dataclasses.dataclass
class BoxConfig:
    """Geometry, plasma and solver parameters of one simulation box.

    Nodes are x_i = x_lo + i*hx for i = 0..nx (same in y); nodes 0 and nx
    carry the homogeneous Dirichlet boundary.  Slice k sits at
    zeta_k = zeta_hi - k*dzeta, k = 0..nzeta-1 (slice 0 is the box head).
    The plasma electrons start on a uniform lattice of (nx*ppc_x) x (ny*ppc_y)
    sites at the centres of a ppc-times refined cell grid.
    """
    nx: int
    ny: int
    x_lo: float
    x_hi: float
    y_lo: float
    y_hi: float
    nzeta: int
    zeta_hi: float
    dzeta: float
    ppc_x: int = 1
    ppc_y: int = 1
    n0: float = 1.0
    pc_max_iter: int = 3
    pc_tol: float = 0.0          # <= 0: always pc_max_iter iterations
    pc_shift: Optional[float] = None   # None: the method's default screening
    psi_floor: float = ONE_PLUS_PSI_FLOOR
    shape_order: int = 1         # transverse particle shape: 0 NGP, 1 CIC, 2 and 3 B-splines
    bxby_solver: str = "pc"      # "pc" predictor-corrector or "explicit"

    @property
    def hx(self) -> float:
        return (self.x_hi - self.x_lo) / self.nx

    @property
    def hy(self) -> float:
        return (self.y_hi - self.y_lo) / self.ny

    @property
    def n_particles(self) -> int:
        return self.nx * self.ppc_x * self.ny * self.ppc_y

    def zeta(self) -> np.ndarray:
        return self.zeta_hi - self.dzeta * np.arange(self.nzeta)


@dataclasses.dataclass
class GaussianBeam:
    """Rigid, ultra-relativistic electron beam with a Gaussian transverse
    profile and an arbitrary per-slice peak density ``amp[k]`` (n_b/n0)."""
    amp: np.ndarray          # [nzeta] float64
    sigma_x: float
    sigma_y: float
    x0: float = 0.0
    y0: float = 0.0


@dataclasses.dataclass
class ParticleBeam:
    """Macro-particle electron beam (SoA, float32 like the GPU storage)."""
    x: np.ndarray
    y: np.ndarray
    zeta: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    w: np.ndarray            # number of physical electrons (units n0 k_p^-3)
    dt: float = 0.0          # time step of the per-slice beam push (0: no push)

    def soa(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.zeta, self.ux, self.uy,
                         self.uz, self.w]).astype(np.float32)


def gaussian_envelope(cfg: BoxConfig, peak: float, zeta_c: float,
                      sigma_z: float) -> np.ndarray:
    z = cfg.zeta()
    return peak * np.exp(-(z - zeta_c) ** 2 / (2.0 * sigma_z ** 2))


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def c1(nb: float = 0.01) -> tuple[BoxConfig, GaussianBeam]:
    """64^2 x 64 linear wake: x,y in [-8,8], zeta in (-8,0], 1 ppc, rigid
    driver n_b/n0 = nb, sigma = 1, centred 2 behind the head, 3 P-C steps."""
    cfg = BoxConfig(nx=64, ny=64, x_lo=-8.0, x_hi=8.0, y_lo=-8.0, y_hi=8.0,
                    nzeta=64, zeta_hi=0.0, dzeta=8.0 / 64,
                    pc_max_iter=3, pc_tol=0.0)
    beam = GaussianBeam(gaussian_envelope(cfg, nb, -2.0, 1.0), 1.0, 1.0)
    return cfg, beam


def c2(n: int = 512, nzeta: int = 1024) -> tuple[BoxConfig, GaussianBeam]:
    """Blowout wake: [-6,6]^2, zeta in (-6,4], driver n_b/n0 = 10,
    sigma_r = 0.3, sigma_z = 1.41 at zeta = 0, P-C to 1e-4 (max 5)."""
    cfg = BoxConfig(nx=n, ny=n, x_lo=-6.0, x_hi=6.0, y_lo=-6.0, y_hi=6.0,
                    nzeta=nzeta, zeta_hi=4.0, dzeta=10.0 / nzeta,
                    pc_max_iter=5, pc_tol=1e-4)
    beam = GaussianBeam(gaussian_envelope(cfg, 10.0, 0.0, 1.41), 0.3, 0.3)
    return cfg, beam


C3_DRIVER = dict(peak=5.0, sigma_r=0.25, sigma_z=1.0, zeta_c=0.0)
C3_WITNESS = dict(peak=20.0, sigma_r=0.1, sigma_z=0.2, zeta_c=-5.0)
C3_GAMMA = 2000.0
BEAM_DT = 6.0     # beam time step, omega_p^-1 (Appendix)


def explicit_currents(cfg: BoxConfig, peak: float = 0.8, seed: int = SEED) -> np.ndarray:
    """Per-slice beam current planes Jz (node layout, zero on the boundary)
    that no Gaussian describes: an off-axis elliptical driver plus a weaker
    displaced satellite, with a seeded per-slice amplitude jitter.  Shape
    [nzeta, ny+1, nx+1]; Jz < 0 (electrons moving along +z)."""
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    y = cfg.y_lo + cfg.hy * np.arange(cfg.ny + 1)
    X, Y = np.meshgrid(x, y)
    main = np.exp(-(X - 0.4) ** 2 / 0.5 - Y ** 2 / 0.9)
    sat = 0.3 * np.exp(-((X + 1.0) ** 2 + (Y - 0.7) ** 2) / 0.3)
    rng = np.random.default_rng(seed + 1)
    env = gaussian_envelope(cfg, peak, -1.0, 0.7) * (1.0 + 0.1 * rng.uniform(-1, 1, cfg.nzeta))
    J = -env[:, None, None] * (main + sat)[None]
    J[:, 0, :] = J[:, -1, :] = 0.0
    J[:, :, 0] = J[:, :, -1] = 0.0
    return J


def emittance_study(n: int = 256, nzeta: int = 256, n_per_beam: int = 2 ** 15,
                    witness_zeta: float = -4.0,
                    seed: int = SEED) -> tuple[BoxConfig, ParticleBeam]:
    """Reduced reference setup for a precision study: the C3 geometry at
    n x n x nzeta, driver and witness macro-particle beams (gamma = 2000),
    the witness with zero initial emittance (u_perp = 0) and its centroid
    offset transversely by one sigma_x.  The witness sits inside the first
    bubble (zeta = -4: focusing Ex - By = x/2 and accelerating); at the C3
    position zeta = -5 it would straddle the back of the bubble, where the
    field defocuses.  Driver and witness carry different macro weights,
    which identify them after the beam has been re-sorted."""
    cfg = c3_config(n, nzeta)
    rng = np.random.default_rng(seed + 7)
    d = gaussian_particle_beam(n_per_beam, C3_DRIVER["peak"], C3_DRIVER["sigma_r"],
                               C3_DRIVER["sigma_z"], C3_DRIVER["zeta_c"], C3_GAMMA, rng)
    w = gaussian_particle_beam(n_per_beam, C3_WITNESS["peak"], C3_WITNESS["sigma_r"],
                               C3_WITNESS["sigma_z"], witness_zeta, C3_GAMMA, rng)
    w.x = w.x + C3_WITNESS["sigma_r"]
    beam = ParticleBeam(*(np.concatenate([getattr(d, f.name), getattr(w, f.name)])
                          for f in dataclasses.fields(ParticleBeam)[:7]), dt=BEAM_DT)
    return cfg, beam


def ion_column(n: int = 64, nzeta: int = 4, extent: float = 4.0, x0: float = 0.2,
               gamma: float = 2000.0, dt: float = BEAM_DT, w: float = 1e-8):
    """Beam test particles in a pure ion column: the box holds ions of
    density n0 = 1 and no plasma electrons (their weights are zeroed by the
    caller), so Ex - By = x/2 and Ey + Bx = y/2 inside.  One test electron
    per slice at (x0, 0), (0, x0), (x0, x0/2) and (-x0/2, x0) in turn, at
    rest transversally, u_z = gamma, negligible charge w.  Returns
    (BoxConfig, ParticleBeam)."""
    cfg = BoxConfig(nx=n, ny=n, x_lo=-extent, x_hi=extent, y_lo=-extent, y_hi=extent,
                    nzeta=nzeta, zeta_hi=0.0, dzeta=1.0 / nzeta, pc_max_iter=2, pc_tol=0.0)
    pts = [(x0, 0.0), (0.0, x0), (x0, 0.5 * x0), (-0.5 * x0, x0)]
    x = np.array([pts[k % 4][0] for k in range(nzeta)], dtype=np.float32)
    y = np.array([pts[k % 4][1] for k in range(nzeta)], dtype=np.float32)
    zeta = np.asarray(cfg.zeta(), dtype=np.float32)
    uz = np.full(nzeta, np.sqrt(gamma * gamma - 1.0), dtype=np.float32)
    zero = np.zeros(nzeta, dtype=np.float32)
    beam = ParticleBeam(x, y, zeta, zero.copy(), zero.copy(), uz, np.full(nzeta, w, np.float32), dt)
    return cfg, beam


def witness_factors(cfg: BoxConfig, rel_cut: float = 1e-10):
    """Separable factors of ``witness_profile`` restricted to the slices
    where the longitudinal factor exceeds rel_cut * peak: returns
    (k_lo, gz [k_hi-k_lo+1], gy [ny+1], gx [nx+1]) with
    n_w[k, j, i] = gz[k - k_lo] * gy[j] * gx[i]."""
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    y = cfg.y_lo + cfg.hy * np.arange(cfg.ny + 1)
    z = cfg.zeta()
    p = C3_WITNESS
    gz = p["peak"] * np.exp(-(z - p["zeta_c"]) ** 2 / (2 * p["sigma_z"] ** 2))
    keep = np.nonzero(gz > rel_cut * p["peak"])[0]
    k_lo, k_hi = int(keep[0]), int(keep[-1])
    gx = np.exp(-x ** 2 / (2 * p["sigma_r"] ** 2))
    gy = np.exp(-y ** 2 / (2 * p["sigma_r"] ** 2))
    return k_lo, gz[k_lo:k_hi + 1], gy, gx


def c3_config(n: int = 1024, nzeta: int = 1024) -> BoxConfig:
    return BoxConfig(nx=n, ny=n, x_lo=-8.0, x_hi=8.0, y_lo=-8.0, y_hi=8.0,
                     nzeta=nzeta, zeta_hi=5.0, dzeta=12.0 / nzeta,
                     pc_max_iter=5, pc_tol=1e-4)


def gaussian_particle_beam(n: int, peak: float, sigma_r: float,
                           sigma_z: float, zeta_c: float, gamma: float,
                           rng: np.random.Generator) -> ParticleBeam:
    """n fixed-weight macro-particles with normally distributed positions
    whose density peaks at ``peak`` (n_b/n0); momenta ux = uy = 0,
    uz = sqrt(gamma^2 - 1)."""
    x = rng.normal(0.0, sigma_r, n)
    y = rng.normal(0.0, sigma_r, n)
    z = rng.normal(zeta_c, sigma_z, n)
    total = peak * (2.0 * math.pi) ** 1.5 * sigma_r * sigma_r * sigma_z
    uz = math.sqrt(gamma * gamma - 1.0)
    return ParticleBeam(x=x, y=y, zeta=z, ux=np.zeros(n), uy=np.zeros(n),
                        uz=np.full(n, uz), w=np.full(n, total / n))


def copy_beam(b: ParticleBeam) -> ParticleBeam:
    return ParticleBeam(*(np.array(getattr(b, f.name), copy=True)
                          if isinstance(getattr(b, f.name), np.ndarray) else getattr(b, f.name)
                          for f in dataclasses.fields(ParticleBeam)))


def c3(n: int = 1024, nzeta: int = 1024, n_per_beam: int = 2 ** 21,
       seed: int = SEED) -> tuple[BoxConfig, ParticleBeam]:
    """Paper-scale step: 1024^2 x 1024, 1 ppc, driver + witness beams of
    ``n_per_beam`` macro-particles each, gamma = 2000."""
    cfg = c3_config(n, nzeta)
    rng = np.random.default_rng(seed)
    d = gaussian_particle_beam(n_per_beam, C3_DRIVER["peak"],
                               C3_DRIVER["sigma_r"], C3_DRIVER["sigma_z"],
                               C3_DRIVER["zeta_c"], C3_GAMMA, rng)
    w = gaussian_particle_beam(n_per_beam, C3_WITNESS["peak"],
                               C3_WITNESS["sigma_r"], C3_WITNESS["sigma_z"],
                               C3_WITNESS["zeta_c"], C3_GAMMA, rng)
    beam = ParticleBeam(*(np.concatenate([getattr(d, f.name), getattr(w, f.name)])
                          for f in dataclasses.fields(ParticleBeam)[:7]), dt=BEAM_DT)
    return cfg, beam


def small_particle_beam(n: int = 64, nzeta: int = 64, n_per_beam: int = 4096,
                        seed: int = SEED) -> tuple[BoxConfig, ParticleBeam]:
    """A reduced C3 for tests: 64^2 nodes over [-8,8]^2, zeta in (-3,5]
    (dzeta = 0.125), driver (peak 2, sigma_r 0.6, sigma_z 0.8 at 3) and
    witness (peak 5, sigma_r 0.4, sigma_z 0.3 at 0) with n_per_beam
    macro-particles each, gamma = 2000, values representable in float32,
    4 fixed P-C iterations."""
    cfg = BoxConfig(nx=n, ny=n, x_lo=-8.0, x_hi=8.0, y_lo=-8.0, y_hi=8.0,
                    nzeta=nzeta, zeta_hi=5.0, dzeta=8.0 / nzeta,
                    pc_max_iter=4, pc_tol=0.0)
    rng = np.random.default_rng(seed)
    d = gaussian_particle_beam(n_per_beam, 2.0, 0.6, 0.8, 3.0, C3_GAMMA, rng)
    w = gaussian_particle_beam(n_per_beam, 5.0, 0.4, 0.3, 0.0, C3_GAMMA, rng)
    beam = ParticleBeam(*(np.concatenate([getattr(d, f.name), getattr(w, f.name)])
                          .astype(np.float32).astype(np.float64)
                          for f in dataclasses.fields(ParticleBeam)[:7]), dt=BEAM_DT)
    return cfg, beam


def c4(n: int = 256, nzeta: int = 512, seed: int = SEED
       ) -> tuple[BoxConfig, GaussianBeam]:
    """Adjoint workload: [-6,6]^2, zeta in (-10,0], driver amplitudes
    2*exp(-(zeta+3)^2/2)*(1 + 0.05 u), u ~ U(-1,1) seeded, sigma_r = 0.4,
    3 fixed P-C iterations."""
    cfg = BoxConfig(nx=n, ny=n, x_lo=-6.0, x_hi=6.0, y_lo=-6.0, y_hi=6.0,
                    nzeta=nzeta, zeta_hi=0.0, dzeta=10.0 / nzeta,
                    pc_max_iter=3, pc_tol=0.0)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, nzeta)
    amp = gaussian_envelope(cfg, 2.0, -3.0, 1.0) * (1.0 + 0.05 * u)
    return cfg, GaussianBeam(amp, 0.4, 0.4)


C4_LOSS_SLICES = (400, 420)   # inclusive range of witness slices


def c5(n: int = 1024, nzeta: int = 1024) -> tuple[BoxConfig, GaussianBeam]:
    """Large adjoint: C3 geometry, 2x2 plasma lattice, driver 5*exp(-zeta^2/2),
    sigma_x = sigma_y = 0.25, 3 fixed P-C iterations."""
    cfg = c3_config(n, nzeta)
    cfg.ppc_x = cfg.ppc_y = 2
    cfg.pc_max_iter, cfg.pc_tol = 3, 0.0
    amp = gaussian_envelope(cfg, C3_DRIVER["peak"], C3_DRIVER["zeta_c"],
                            C3_DRIVER["sigma_z"])
    return cfg, GaussianBeam(amp, 0.25, 0.25)


def witness_profile(cfg: BoxConfig) -> np.ndarray:
    """Loss weights n_w(x_i, y_j, zeta_k) of the C3 witness (peak 20,
    sigma_r 0.1, sigma_z 0.2, centre -5), shape [nzeta, ny+1, nx+1]."""
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    y = cfg.y_lo + cfg.hy * np.arange(cfg.ny + 1)
    z = cfg.zeta()
    p = C3_WITNESS
    gz = p["peak"] * np.exp(-(z - p["zeta_c"]) ** 2 / (2 * p["sigma_z"] ** 2))
    gx = np.exp(-x ** 2 / (2 * p["sigma_r"] ** 2))
    gy = np.exp(-y ** 2 / (2 * p["sigma_r"] ** 2))
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def small(n: int = 32, nzeta: int = 24, ppc: int = 1, nb: float = 0.5,
          sigma: float = 0.8, pc_max_iter: int = 3, pc_tol: float = 0.0,
          extent: float = 6.0) -> tuple[BoxConfig, GaussianBeam]:
    """A tiny moderately nonlinear box for fast unit and parity tests."""
    cfg = BoxConfig(nx=n, ny=n, x_lo=-extent, x_hi=extent, y_lo=-extent,
                    y_hi=extent, nzeta=nzeta, zeta_hi=0.0,
                    dzeta=4.0 / nzeta, ppc_x=ppc, ppc_y=ppc,
                    pc_max_iter=pc_max_iter, pc_tol=pc_tol)
    beam = GaussianBeam(gaussian_envelope(cfg, nb, -1.0, 0.7), sigma, sigma)
    return cfg, beam


def blowout_slice_state(cfg: BoxConfig, seed: int = SEED, r_bubble: float = 1.2,
                        n_floored: int = 64, n_leaving: int = 64, n_dead: int = 32,
                        psi_floor: float = ONE_PLUS_PSI_FLOOR) -> dict:
    """A seeded plasma slice shaped like the inside of a blowout, for
    importing the same state into both implementations at full grid size
    without running the box up to a nonlinear slice.

    Particles keep their lattice order.  Each lattice site at radius r0 is
    moved radially to r0 + (sqrt(r0^2 + r_bubble^2) - r0) exp(-r0^2/12.5)
    (an electron-free column of radius ~r_bubble with a dense sheath), plus
    a uniform jitter of +-0.3 cells; every position stays one cell inside
    the box.  Momenta point outward with amplitude 0.6 exp(-(r0/1.5)^2)
    plus N(0, 0.05) noise; Psi = -0.4 exp(-r^2/4.5) + N(0, 0.02).
    Special particles, chosen at random without overlap:
      n_floored  in the annulus 3 < r0 < 5 with 1 + Psi = 0.3 psi_floor
                 (below the floor) and |u| <= 0.05;
      n_leaving  on the lattice rows and columns next to the box edge, with
                 an outward momentum of 3 (they leave the box in one slice);
      n_dead     weight 0 (absorbed earlier).
    History slots hold N(0, 0.05) values.  The macro weight of a live
    particle is n0 hx hy / (ppc_x ppc_y).

    Returns a dict of float64 arrays: x, y, ux, uy, psi, w [N];
    hist [4, 5, N]; index arrays floored, leaving, dead."""
    rng = np.random.default_rng(seed)
    nX, nY = cfg.nx * cfg.ppc_x, cfg.ny * cfg.ppc_y
    I, J = np.meshgrid(np.arange(nX), np.arange(nY))
    I, J = I.ravel(), J.ravel()
    x0 = cfg.x_lo + (I + 0.5) * cfg.hx / cfg.ppc_x
    y0 = cfg.y_lo + (J + 0.5) * cfg.hy / cfg.ppc_y
    n = x0.size
    r0 = np.hypot(x0, y0)
    push = (np.sqrt(r0 * r0 + r_bubble * r_bubble) - r0) * np.exp(-r0 * r0 / 12.5)
    ang = np.arctan2(y0, x0)
    cx, cy = np.cos(ang), np.sin(ang)
    x = x0 + push * cx + rng.uniform(-0.3, 0.3, n) * cfg.hx
    y = y0 + push * cy + rng.uniform(-0.3, 0.3, n) * cfg.hy
    x = np.clip(x, cfg.x_lo + cfg.hx, cfg.x_hi - cfg.hx)
    y = np.clip(y, cfg.y_lo + cfg.hy, cfg.y_hi - cfg.hy)
    amp = 0.6 * np.exp(-(r0 / 1.5) ** 2)
    ux = amp * cx + rng.normal(0.0, 0.05, n)
    uy = amp * cy + rng.normal(0.0, 0.05, n)
    r = np.hypot(x, y)
    psi = -0.4 * np.exp(-r * r / 4.5) + rng.normal(0.0, 0.02, n)
    w = np.full(n, cfg.n0 * cfg.hx * cfg.hy / (cfg.ppc_x * cfg.ppc_y))
    hist = rng.normal(0.0, 0.05, (4, 5, n))

    taken = np.zeros(n, dtype=bool)

    def pick(mask, count):
        cand = np.nonzero(mask & ~taken)[0]
        sel = np.sort(rng.choice(cand, size=min(count, cand.size), replace=False))
        taken[sel] = True
        return sel

    floored = pick((r0 > 3.0) & (r0 < 5.0), n_floored)
    psi[floored] = -1.0 + 0.3 * psi_floor
    ux[floored] = rng.uniform(-0.05, 0.05, floored.size)
    uy[floored] = rng.uniform(-0.05, 0.05, floored.size)
    edge = (I < cfg.ppc_x) | (I >= nX - cfg.ppc_x) | (J < cfg.ppc_y) | (J >= nY - cfg.ppc_y)
    leaving = pick(edge, n_leaving)
    x[leaving] = np.clip(x0[leaving], cfg.x_lo + 0.5 * cfg.hx, cfg.x_hi - 0.5 * cfg.hx)
    y[leaving] = np.clip(y0[leaving], cfg.y_lo + 0.5 * cfg.hy, cfg.y_hi - 0.5 * cfg.hy)
    out_x = np.where(I[leaving] < nX // 2, -1.0, 1.0)
    out_y = np.where(J[leaving] < nY // 2, -1.0, 1.0)
    on_x = (I[leaving] < cfg.ppc_x) | (I[leaving] >= nX - cfg.ppc_x)
    ux[leaving] = np.where(on_x, 3.0 * out_x, 0.0)
    uy[leaving] = np.where(on_x, 0.0, 3.0 * out_y)
    psi[leaving] = 0.0
    hist[:, :, leaving] = 0.0
    dead = pick(np.ones(n, dtype=bool), n_dead)
    w[dead] = 0.0
    return {"x": x, "y": y, "ux": ux, "uy": uy, "psi": psi, "w": w, "hist": hist,
            "floored": floored, "leaving": leaving, "dead": dead}


def smooth_planes(cfg: BoxConfig, seed: int = SEED, scale: float = 0.2) -> dict:
    """Seeded smooth node planes for the quantities a slice takes over from
    the two slices before it (transverse currents of slice k-1, Bx and By of
    slices k-1 and k-2): sums of a few random Gaussians of width 0.5-2 near
    the axis, amplitude ~scale, zero on the boundary nodes."""
    rng = np.random.default_rng(seed)
    x = cfg.x_lo + cfg.hx * np.arange(cfg.nx + 1)
    y = cfg.y_lo + cfg.hy * np.arange(cfg.ny + 1)
    X, Y = np.meshgrid(x, y)
    out = {}
    for name in ("jx_prev", "jy_prev", "bx_prev1", "by_prev1", "bx_prev2", "by_prev2"):
        f = np.zeros_like(X)
        for _ in range(4):
            a = rng.normal(0.0, scale)
            xc, yc = rng.uniform(-1.5, 1.5, 2)
            s = rng.uniform(0.5, 2.0)
            f += a * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2 * s * s))
        f[0, :] = f[-1, :] = 0.0
        f[:, 0] = f[:, -1] = 0.0
        out[name] = f
    return out


def witness_slice_beam(cfg: BoxConfig, k: int, n: int, peak: float = C3_WITNESS["peak"],
                       sigma_r: float = C3_WITNESS["sigma_r"],
                       sigma_z: float = C3_WITNESS["sigma_z"], gamma: float = C3_GAMMA,
                       dt: float = BEAM_DT, seed: int = SEED) -> ParticleBeam:
    """n macro-particles of a Gaussian beam (peak n_b/n0 `peak`, transverse
    sigma_r, longitudinal sigma_z) that all sit within slice k (|zeta -
    zeta_k| < dzeta/4): the density of one slice at the peak of the C3
    witness.  Weights carry the full beam's charge per slice (peak density x
    2 pi sigma_r^2 x dzeta spread over n particles); values are float32
    representable.  u_perp = 0 plus N(0, 0.01), u_z = sqrt(gamma^2 - 1)."""
    rng = np.random.default_rng(seed)
    zk = cfg.zeta_hi - k * cfg.dzeta
    x = rng.normal(0.0, sigma_r, n)
    y = rng.normal(0.0, sigma_r, n)
    z = zk + rng.uniform(-0.25, 0.25, n) * cfg.dzeta
    total = peak * 2.0 * math.pi * sigma_r * sigma_r * cfg.dzeta
    uz = math.sqrt(gamma * gamma - 1.0)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return ParticleBeam(x=f32(x), y=f32(y), zeta=f32(z), ux=f32(rng.normal(0.0, 0.01, n)),
                        uy=f32(rng.normal(0.0, 0.01, n)), uz=f32(np.full(n, uz)),
                        w=f32(np.full(n, total / n)), dt=dt)


PRESETS = {"c1": c1, "c2": c2, "c4": c4, "c5": c5}
