"""Pins of the oracle's adjoint of the slice loop: FP64 central differences
of the loss, causality (amplitudes behind the last loss slice have exactly
zero gradient) and the linear-regime identity g . a = L."""
import numpy as np
import pytest

import workloads as W
from oracle import qsp_adjoint as A
from oracle import qsp_oracle as O


def cot_all_fields(cfg, k_lo, k_hi):
    c = cfg.nx // 2
    rng = np.random.default_rng(11)
    weights = {}
    for k in range(k_lo, k_hi + 1):
        d = {}
        for q in A.FIELD_KEYS:
            w = np.zeros((cfg.ny + 1, cfg.nx + 1))
            w[c - 2:c + 3, c - 2:c + 3] = rng.normal(size=(5, 5))
            d[q] = w
        weights[k] = d
    return lambda k: weights.get(k, {})


def loss(cfg, beam, cot):
    recs, _ = O.run_box(cfg, beam)
    return A.loss_value(recs, cot)


@pytest.mark.parametrize("ppc,nb,order", [(1, 0.8, 1), (2, 1.5, 1), (1, 0.8, 2), (1, 0.8, 3)])
def test_adjoint_matches_central_differences(ppc, nb, order):
    cfg, beam = W.small(n=16, nzeta=14, ppc=ppc, nb=nb, sigma=0.9, pc_max_iter=2,
                        pc_tol=0.0, extent=4.0)
    cfg.shape_order = order
    cot = cot_all_fields(cfg, 7, 11)
    recs, tape = A.forward_with_tape(cfg, beam)
    ga, gsx, gsy = A.adjoint_box(cfg, beam, tape, cot)
    for k in (1, 4, 7, 10):
        h = 1e-6 * max(abs(beam.amp[k]), 1e-2)
        ap, am = beam.amp.copy(), beam.amp.copy()
        ap[k] += h
        am[k] -= h
        fd = (loss(cfg, W.GaussianBeam(ap, beam.sigma_x, beam.sigma_y), cot) -
              loss(cfg, W.GaussianBeam(am, beam.sigma_x, beam.sigma_y), cot)) / (2 * h)
        assert abs(ga[k] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(ga).max()), (k, ga[k], fd)
    h = 1e-6
    for g, which in ((gsx, "x"), (gsy, "y")):
        bp = W.GaussianBeam(beam.amp, beam.sigma_x + h * (which == "x"), beam.sigma_y + h * (which == "y"))
        bm = W.GaussianBeam(beam.amp, beam.sigma_x - h * (which == "x"), beam.sigma_y - h * (which == "y"))
        fd = (loss(cfg, bp, cot) - loss(cfg, bm, cot)) / (2 * h)
        assert abs(g - fd) <= 1e-5 * abs(fd), (which, g, fd)


def test_adjoint_causality():
    cfg, beam = W.small(n=16, nzeta=14, nb=0.8, pc_max_iter=2, pc_tol=0.0, extent=4.0)
    cot = cot_all_fields(cfg, 5, 8)
    _, tape = A.forward_with_tape(cfg, beam)
    ga, _, _ = A.adjoint_box(cfg, beam, tape, cot)
    assert np.all(ga[9:] == 0.0)
    assert np.all(ga[:9] != 0.0)


def test_linear_regime_gradient_reproduces_loss():
    # for a vanishing beam every field is linear in the amplitudes and
    # L(0) = 0, so L = sum_k g_k a_k
    cfg, beam = W.small(n=16, nzeta=14, nb=1e-7, pc_max_iter=3, pc_tol=0.0, extent=4.0)
    cot = cot_all_fields(cfg, 4, 12)
    recs, tape = A.forward_with_tape(cfg, beam)
    ga, _, _ = A.adjoint_box(cfg, beam, tape, cot)
    L = A.loss_value(recs, cot)
    assert abs(np.dot(ga, beam.amp) - L) < 1e-6 * abs(L)
