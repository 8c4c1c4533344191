"""FP64 adjoint (reverse mode) of the oracle's slice loop.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The loss is L = sum_k sum_F <W_{F,k}, F_k> for fields F in (psi, Ex-By,
Ey+Bx, Ez, Bx, By, Bz) of slice k with given cotangent weights W.  The
parameters are the per-slice amplitudes a_k and the transverse sizes
(sigma_x, sigma_y) of a rigid Gaussian drive beam.  The predictor-corrector
is unrolled with the iteration count the forward pass used on each slice.

Every forward step of ``qsp_oracle.advance_slice`` is transposed here:
  * deposit (CIC, with the particle values q w / cell, q w u/D, q w u_z/D)
    -> gather of the adjoint planes with S and, for the positions, grad S;
  * field gather -> deposit of the adjoint of the gathered values, plus the
    grad S position terms;
  * the pusher right-hand side -> its explicit Jacobian (transposed);
  * the Adams-Bashforth step -> adjoint history: lam_f_k collects -dzeta b0
    lam_y_{k+1} and the shifted history adjoints;
  * (lap - s)^-1 is symmetric -> the same solve;
  * centred differences with zero Dirichlet nodes satisfy D^T = -D.
Absorption and the 1+Psi floor are treated as locally constant.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Optional

import numpy as np

from . import qsp_oracle as O

FIELD_KEYS = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz")


# --------------------------------------------------------------------------
# Forward with a tape
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SliceTape:
    plasma: O.Plasma               # state at the start of the slice
    flds: dict                     # exmby, eypbx, ez, bz, psi of the slice
    b_iter: List[tuple]            # (bx, by) iterates B^0 .. B^M
    m: int                         # predictor-corrector iterations used


def forward_with_tape(cfg, beam):
    """Runs the box like ``qsp_oracle.run_box`` and records what the reverse
    pass needs.  Returns (records, tape)."""
    st = O.initial_state(cfg)
    tape, recs = [], []
    for k in range(cfg.nzeta):
        p0 = st.plasma.copy()
        dep = O.total_deposit(cfg, st.plasma, beam, k)
        flds = O.solve_psi_ez_bz(cfg, dep)
        # predictor-corrector, recording every iterate
        bx = 2.0 * st.bx_prev1 - st.bx_prev2
        by = 2.0 * st.by_prev1 - st.by_prev2
        iters = [(bx, by)]
        res = []
        for m in range(cfg.pc_max_iter):
            trial, _, _ = O.ab5_push(cfg, st.plasma, dict(flds, bx=bx, by=by), commit=False)
            jn = O.plasma_deposit(cfg, trial, ("jx", "jy"))
            bxn, byn = O.solve_bxby(cfg, dep["jz"], st.jx_prev, st.jy_prev, jn["jx"], jn["jy"],
                                    bx, by)
            num = np.sum((bxn - bx) ** 2) + np.sum((byn - by) ** 2)
            den = np.sum(bxn ** 2) + np.sum(byn ** 2)
            r = np.sqrt(num / den) if den > 0 else (0.0 if num == 0 else np.inf)
            res.append(r)
            bx, by = bxn, byn
            iters.append((bx, by))
            if cfg.pc_tol > 0 and r < cfg.pc_tol:
                break
        flds["bx"], flds["by"] = bx, by
        new_plasma, _, _ = O.ab5_push(cfg, st.plasma, flds, commit=True)
        tape.append(SliceTape(p0, {q: flds[q] for q in ("psi", "exmby", "eypbx", "ez", "bz")},
                              iters, len(iters) - 1))
        rec = dict(flds)
        rec.update(dep)
        rec["pc_iters"] = len(iters) - 1
        rec["pc_residuals"] = res
        recs.append(rec)
        st = O.SliceState(k + 1, new_plasma, dep["jx"], dep["jy"], bx, by,
                          st.bx_prev1, st.by_prev1)
    return recs, tape


# --------------------------------------------------------------------------
# Transposed building blocks
# --------------------------------------------------------------------------

def shape_1d_grad(s, n: int, order: int):
    """Derivatives d w / d s of the ``shape_1d`` weights (orders 1-3; the
    order-0 shape is discontinuous and has no adjoint)."""
    if order not in (1, 2, 3):
        raise ValueError("the adjoint needs a shape of order 1, 2 or 3")
    return O.shape_1d_slope(s, n, order)


def cic_grad(cfg, x, y):
    """Nodes, weights S and their derivatives dS/dx, dS/dy for the
    configured shape (tensor products of ``shape_1d`` and its derivative)."""
    o = O.shape_order(cfg)
    sx = (x - cfg.x_lo) / cfg.hx
    sy = (y - cfg.y_lo) / cfg.hy
    ni, wi = O.shape_1d(sx, cfg.nx, o)
    nj, wj = O.shape_1d(sy, cfg.ny, o)
    di = shape_1d_grad(sx, cfg.nx, o)
    dj = shape_1d_grad(sy, cfg.ny, o)
    nodes, wts, dx, dy = [], [], [], []
    for j, wy, dwy in zip(nj, wj, dj):
        for i, wx, dwx in zip(ni, wi, di):
            nodes.append((i, j))
            wts.append(wx * wy)
            dx.append(dwx * wy / cfg.hx)
            dy.append(wx * dwy / cfg.hy)
    return nodes, wts, dx, dy


def gather_grad(cfg, F, x, y):
    """Value of the shape interpolant of F at the particles and its gradient."""
    nodes, wts, dx, dy = cic_grad(cfg, x, y)
    v = gx = gy = 0.0
    for (i, j), s, ddx, ddy in zip(nodes, wts, dx, dy):
        ok = O._valid(cfg, i, j)
        f = np.where(ok, F[np.clip(j, 0, cfg.ny), np.clip(i, 0, cfg.nx)], 0.0)
        v = v + f * s
        gx = gx + f * ddx
        gy = gy + f * ddy
    return v, gx, gy


def scatter(cfg, x, y, vals):
    """Transpose of ``gather``: sum_p vals_p S_p at the nodes (boundary
    nodes, which carry no unknown, dropped)."""
    return O.deposit_values(cfg, x, y, vals)


GATHERED = ("exmby", "eypbx", "ez", "bx", "by", "bz")


def rhs_vjp(cfg, p: O.Plasma, F: dict, lam_f: np.ndarray, lam_y: np.ndarray,
            lam_F: dict):
    """Adds (d f / d y)^T lam_f to lam_y (positions through the gather) and
    the gather transpose to lam_F, for f = particle_rhs(p, F)."""
    alive = p.w > 0
    lf = np.where(alive[None, :], lam_f, 0.0)
    vals = {}
    grads = {}
    for q in GATHERED:
        v, gx, gy = gather_grad(cfg, F[q], p.x, p.y)
        vals[q], grads[q] = v, (gx, gy)
    e1, e2, ez, bx, by, bz = (vals[q] for q in GATHERED)
    ux, uy = p.ux, p.uy
    raw = 1.0 + p.psi
    d = np.maximum(raw, cfg.psi_floor)
    dd_dpsi = (raw >= cfg.psi_floor).astype(np.float64)
    u2 = 1.0 + ux * ux + uy * uy
    G = u2 / (2 * d * d) + 0.5                     # gamma / D
    l0, l1, l2, l3, l4 = lf
    # d f / d ux, uy, D
    lam_ux = -l0 / d + l2 * (ux / d ** 2) * e1 + l3 * ((ux / d ** 2) * e2 - bz / d) + l4 * e1 / d
    lam_uy = -l1 / d + l2 * ((uy / d ** 2) * e1 + bz / d) + l3 * (uy / d ** 2) * e2 + l4 * e2 / d
    lam_d = (l0 * ux / d ** 2 + l1 * uy / d ** 2 +
             l2 * (-u2 / d ** 3 * e1 - bz * uy / d ** 2) +
             l3 * (-u2 / d ** 3 * e2 + bz * ux / d ** 2) +
             l4 * (-(ux * e1 + uy * e2) / d ** 2))
    lam_y[2] += lam_ux
    lam_y[3] += lam_uy
    lam_y[4] += lam_d * dd_dpsi
    # d f / d gathered fields
    lg = {"exmby": l2 * G + l4 * ux / d,
          "eypbx": l3 * G + l4 * uy / d,
          "ez": -l4,
          "bx": -l3,
          "by": l2,
          "bz": l2 * uy / d - l3 * ux / d}
    for q in GATHERED:
        gx, gy = grads[q]
        lam_y[0] += lg[q] * gx
        lam_y[1] += lg[q] * gy
        lam_F[q] = lam_F[q] + scatter(cfg, p.x, p.y, lg[q])


def deposit_vjp(cfg, p: O.Plasma, lam_dep: dict, lam_y: np.ndarray):
    """Adds the transpose of ``plasma_deposit`` (channels given in lam_dep
    among rho_mjz, jx, jy, jz) to lam_y."""
    alive = p.w > 0
    d_raw = 1.0 + p.psi
    d = np.maximum(d_raw, cfg.psi_floor)
    dd_dpsi = (d_raw >= cfg.psi_floor).astype(np.float64)
    qn = -p.w / (cfg.hx * cfg.hy)
    ux, uy = p.ux, p.uy
    u2 = 1.0 + ux * ux + uy * uy
    val = {"rho_mjz": qn, "jx": qn * ux / d, "jy": qn * uy / d,
           "jz": qn * (u2 / (2 * d * d) - 0.5)}
    # derivatives of the values w.r.t. ux, uy, D
    dval = {"rho_mjz": (0 * qn, 0 * qn, 0 * qn),
            "jx": (qn / d, 0 * qn, -qn * ux / d ** 2),
            "jy": (0 * qn, qn / d, -qn * uy / d ** 2),
            "jz": (qn * ux / d ** 2, qn * uy / d ** 2, -qn * u2 / d ** 3)}
    for c, lam in lam_dep.items():
        g, gx, gy = gather_grad(cfg, lam, p.x, p.y)
        lam_y[0] += np.where(alive, val[c] * gx, 0.0)
        lam_y[1] += np.where(alive, val[c] * gy, 0.0)
        dux, duy, dd = dval[c]
        lam_y[2] += np.where(alive, dux * g, 0.0)
        lam_y[3] += np.where(alive, duy * g, 0.0)
        lam_y[4] += np.where(alive, dd * g * dd_dpsi, 0.0)


def trial_state(cfg, p: O.Plasma, F: dict) -> O.Plasma:
    trial, _, _ = O.ab5_push(cfg, p, F, commit=False)
    return trial


def ab5_vjp(cfg, p: O.Plasma, F: dict, lam_new: np.ndarray, lam_hist_new0: Optional[np.ndarray],
            lam_y: np.ndarray, lam_h: np.ndarray, lam_F: dict):
    """Transpose of one AB5 step y' = y - dzeta (b0 f(y, F) + sum b_j h_j)
    taken from state p.  lam_new: adjoint of y'; lam_hist_new0: adjoint of
    the new history slot holding f (real push) or None (trial).  Particles
    the step absorbs, or already dead, pass nothing on."""
    ab = O.AB5
    new = np.stack([p.x, p.y, p.ux, p.uy, p.psi])
    f, _ = O.particle_rhs(cfg, p, F)
    stepped = new - cfg.dzeta * (ab[0] * f + sum(ab[m + 1] * p.hist[m] for m in range(4)))
    inside = ((stepped[0] >= cfg.x_lo) & (stepped[0] <= cfg.x_hi) &
              (stepped[1] >= cfg.y_lo) & (stepped[1] <= cfg.y_hi))
    moved = (p.w > 0) & inside
    ln = np.where(moved[None, :], lam_new, 0.0)
    lam_y += ln
    lam_f = -cfg.dzeta * ab[0] * ln
    if lam_hist_new0 is not None:
        lam_f = lam_f + np.where(moved[None, :], lam_hist_new0, 0.0)
    for m in range(4):
        lam_h[m] += -cfg.dzeta * ab[m + 1] * ln
    rhs_vjp(cfg, p, F, lam_f, lam_y, lam_F)


def gaussian_profile(cfg, beam):
    x, y = O.node_coords(cfg)
    gx = np.exp(-(x - beam.x0) ** 2 / (2 * beam.sigma_x ** 2))
    gy = np.exp(-(y - beam.y0) ** 2 / (2 * beam.sigma_y ** 2))
    dgx = gx * (x - beam.x0) ** 2 / beam.sigma_x ** 3
    dgy = gy * (y - beam.y0) ** 2 / beam.sigma_y ** 3
    prof = O.zero_boundary(gy[:, None] * gx[None, :])
    dsx = O.zero_boundary(gy[:, None] * dgx[None, :])
    dsy = O.zero_boundary(dgy[:, None] * gx[None, :])
    return prof, dsx, dsy


# --------------------------------------------------------------------------
# The reverse slice loop
# --------------------------------------------------------------------------

def adjoint_box(cfg, beam, tape: List[SliceTape],
                cotangent: Callable[[int], Dict[str, np.ndarray]]):
    """Gradient of L = sum_k sum_F <cotangent(k)[F], F_k> with respect to
    the beam amplitudes a_k and (sigma_x, sigma_y).  Returns
    (grad_amp [nzeta], grad_sigma_x, grad_sigma_y)."""
    s = O.pc_shift(cfg)
    prof, dprof_x, dprof_y = gaussian_profile(cfg, beam)
    shape = (cfg.ny + 1, cfg.nx + 1)
    zeros = lambda: np.zeros(shape)
    n = tape[0].plasma.x.size
    ab = O.AB5
    lam_y_next = np.zeros((5, n))
    lam_h_next = np.zeros((4, 5, n))
    lam_jprev = (zeros(), zeros())        # adjoint of J_perp_{k} held by state k+1
    lam_b1 = (zeros(), zeros())           # adjoint of B_k held by state k+1
    lam_b2 = (zeros(), zeros())           # adjoint of B_{k-1} held by state k+1
    g_amp = np.zeros(cfg.nzeta)
    g_sx = g_sy = 0.0
    dz2 = 2.0 * cfg.dzeta
    for k in range(cfg.nzeta - 1, -1, -1):
        T = tape[k]
        p = T.plasma
        lam_F = {q: zeros() for q in GATHERED}
        lam_psi = zeros()
        for q, w in cotangent(k).items():
            w = O.zero_boundary(np.array(w, dtype=np.float64))   # boundary nodes are fixed
            if q == "psi":
                lam_psi = lam_psi + w
            else:
                lam_F[q] = lam_F[q] + w
        lam_F["bx"] = lam_F["bx"] + lam_b1[0]
        lam_F["by"] = lam_F["by"] + lam_b1[1]
        lam_b1_k = [lam_b2[0].copy(), lam_b2[1].copy()]
        lam_b2_k = [zeros(), zeros()]
        lam_jx_dep, lam_jy_dep = lam_jprev[0].copy(), lam_jprev[1].copy()
        lam_y = np.zeros((5, n))
        lam_h = np.zeros((4, 5, n))
        # real push k -> k+1 (history: new slot 0 = f_k, slots shift)
        lam_h[0] += lam_h_next[1]
        lam_h[1] += lam_h_next[2]
        lam_h[2] += lam_h_next[3]
        bxM, byM = T.b_iter[T.m]
        F_real = dict(T.flds, bx=bxM, by=byM)
        lam_Fr = {q: zeros() for q in GATHERED}
        ab5_vjp(cfg, p, F_real, lam_y_next, lam_h_next[0], lam_y, lam_h, lam_Fr)
        for q in GATHERED:
            lam_F[q] = lam_F[q] + lam_Fr[q]
        # predictor-corrector, unrolled in reverse
        lam_B = (lam_F["bx"], lam_F["by"])
        lam_jz = zeros()
        jp_x, jp_y = zeros(), zeros()       # adjoint of J_perp_{k-1} (state k)
        for m in range(T.m - 1, -1, -1):
            # B^{m+1} = (lap - s)^-1 [ -d_y Jz + (Jy_{k-1} - Jy~)/2dz - s Bx^m,
            #                          d_x Jz - (Jx_{k-1} - Jx~)/2dz - s By^m ]
            lsx = O.poisson_solve(cfg, lam_B[0], s)
            lsy = O.poisson_solve(cfg, lam_B[1], s)
            lam_jz = lam_jz + O.ddy(cfg, lsx) - O.ddx(cfg, lsy)
            jp_x = jp_x - lsy / dz2
            jp_y = jp_y + lsx / dz2
            lam_jt = {"jx": lsy / dz2, "jy": -lsx / dz2}
            bxm, bym = T.b_iter[m]
            Fm = dict(T.flds, bx=bxm, by=bym)
            # trial deposit transposed, then the trial AB5 step transposed
            trial = trial_state(cfg, p, Fm)
            lam_tr = np.zeros((5, n))
            deposit_vjp(cfg, trial, lam_jt, lam_tr)
            lam_Fm = {q: zeros() for q in GATHERED}
            ab5_vjp(cfg, p, Fm, lam_tr, None, lam_y, lam_h, lam_Fm)
            for q in ("exmby", "eypbx", "ez", "bz"):
                lam_F[q] = lam_F[q] + lam_Fm[q]
            lam_B = (-s * lsx + lam_Fm["bx"], -s * lsy + lam_Fm["by"])
        # initial guess B^0 = 2 B_{k-1} - B_{k-2}
        lam_b1_k[0] += 2.0 * lam_B[0]
        lam_b1_k[1] += 2.0 * lam_B[1]
        lam_b2_k[0] += -lam_B[0]
        lam_b2_k[1] += -lam_B[1]
        # psi, Ez, Bz solves and their sources
        lam_psi = lam_psi + O.ddx(cfg, lam_F["exmby"]) + O.ddy(cfg, lam_F["eypbx"])
        l_spsi = O.poisson_solve(cfg, lam_psi)
        l_sez = O.poisson_solve(cfg, lam_F["ez"])
        l_sbz = O.poisson_solve(cfg, lam_F["bz"])
        lam_dep = {"rho_mjz": -l_spsi,
                   "jx": lam_jx_dep - O.ddx(cfg, l_sez) - O.ddy(cfg, l_sbz),
                   "jy": lam_jy_dep - O.ddy(cfg, l_sez) + O.ddx(cfg, l_sbz),
                   "jz": lam_jz}
        # beam parameters: Jz_beam = -a_k * profile
        a = beam.amp[k]
        g_amp[k] = -np.sum(lam_jz * prof)
        g_sx += -a * np.sum(lam_jz * dprof_x)
        g_sy += -a * np.sum(lam_jz * dprof_y)
        deposit_vjp(cfg, p, lam_dep, lam_y)
        # hand state k's adjoints to slice k-1
        lam_y_next, lam_h_next = lam_y, lam_h
        lam_jprev = (jp_x, jp_y)
        lam_b1 = (lam_b1_k[0], lam_b1_k[1])
        lam_b2 = (lam_b2_k[0], lam_b2_k[1])
    return g_amp, g_sx, g_sy


def loss_value(recs, cotangent: Callable[[int], Dict[str, np.ndarray]]) -> float:
    total = 0.0
    for k, r in enumerate(recs):
        for q, w in cotangent(k).items():
            total += float(np.sum(w * r[q]))
    return total
