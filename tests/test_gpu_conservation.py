"""Charge conservation of the GPU path through a blowout (quasi-static
continuity, Sec. II): slice after slice the interior total of the deposited
rho - Jz (electrons and ions) changes only by the electron charge that the
particles' shapes put on or past the Dirichlet boundary nodes, computed here
from the particle states the GPU exports.  This holds whatever the field
solves do, so it checks the deposit and the particle bookkeeping on their
own.  FP64: exact to rounding (1e-11 of the electron charge).  FP32: the
kernels place a particle at its FP32 offset inside its lattice cell while
the exported position is that offset widened to FP64, which moves the
weights at the boundary by FP32 rounding (bar 1e-6); a lost stencil node
or particle would show at the 1e-3 level."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from test_oracle_continuity import boundary_charge

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class _P:
    def __init__(self, x, y, w):
        self.x, self.y, self.w = x, y, w


@pytest.mark.parametrize("order,prec", [(1, "fp64"), (1, "fp32"), (3, "fp32")])
def test_blowout_box_conserves_charge(order, prec):
    from paper_2109_10277_amd import qsp
    cfg, beam = W.small(n=64, nzeta=32, nb=8.0, sigma=0.35, extent=4.0, pc_max_iter=5,
                        pc_tol=1e-4)
    cfg = dataclasses.replace(cfg, shape_order=order)
    print(f"charge conservation order {order} {prec}", flush=True)
    totals, leaked = [], []
    with qsp.Box(cfg, prec) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.init_plasma()
        out = {"rho_mjz": box.empty("rho_mjz")}
        for _ in range(cfg.nzeta):
            s = box.get_state()
            p = _P(s["x"], s["y"], s["w"] * cfg.hx * cfg.hy)
            box.advance_slice(out)
            torch.cuda.synchronize()
            totals.append(float(out["rho_mjz"].double().sum()) * cfg.hx * cfg.hy)
            leaked.append(boundary_charge(cfg, p))
        stats = box.stats()
    totals, leaked = np.array(totals), np.array(leaked)
    electrons = float(np.sum(p.w))
    print("  interior total moves by", np.abs(totals - totals[0]).max(),
          "deposits outside their tile", stats["n_deposit_global"])
    assert stats["n_absorbed"] == 0
    assert stats["n_deposit_global"] > 0                  # a real blowout
    assert np.abs(totals - totals[0]).max() > 1e-3        # the edge plasma moves
    kept = totals + leaked
    tol = 1e-11 if prec == "fp64" else 1e-6
    assert np.abs(kept - kept[0]).max() < tol * electrons, np.abs(kept - kept[0]).max()
