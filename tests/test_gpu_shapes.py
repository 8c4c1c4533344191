"""GPU parity of the transverse shape orders 0, 2 and 3 (Sec. III.B: orders
0-3 transversely) against the FP64 oracle: the rest plasma with its ion
background, one slice from an oracle state, whole boxes with a Gaussian and
with a macro-particle beam, and the adjoint for orders 2 and 3.

Bars as for the linear shape: FP64 to 1e-9 (one slice) / 1e-8 (a nonlinear
box: rounding differences carried through the slices), FP32 to 1e-4 (one
slice) / 1e-3 (a box).  Order 0 runs with two particles per cell, so that
the rest lattice is off the rounding edges of the nearest-node assignment."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import qsp_adjoint as A
from oracle import qsp_oracle as O
from parity_util import DEPOSIT_NAMES, FIELD_NAMES, field_errors, oracle_state_to_abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Q():
    from paper_2109_10277_amd import qsp
    return qsp


def to_np(t):
    return t.double().cpu().numpy()


def with_order(cfg, order):
    cfg = dataclasses.replace(cfg, shape_order=order)
    if order == 0:
        cfg = dataclasses.replace(cfg, ppc_x=2, ppc_y=2)
    return cfg


@pytest.mark.parametrize("order", [0, 1, 2, 3])
@pytest.mark.parametrize("ppc", [1, 2])
def test_rest_plasma_is_neutral_and_stays_at_rest(order, ppc):
    # no beam: the ions cancel the electrons node by node, edges included,
    # so no field arises and nothing moves
    cfg, _ = W.small(n=32, nzeta=6, ppc=ppc)
    cfg = dataclasses.replace(cfg, shape_order=order)
    print(f"rest plasma order {order} ppc {ppc}", flush=True)
    with Q().Box(cfg, "fp64") as box:
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in ("psi", "ez", "bx", "rho_mjz", "rho")}
        stats = box.run_box(stack=stack)
        got = {q: to_np(t) for q, t in stack.items()}
        st = box.get_state()
    for q in ("psi", "ez", "bx", "rho_mjz", "rho"):
        assert np.abs(got[q]).max() < 1e-12, (q, np.abs(got[q]).max())
    p0 = O.init_plasma(cfg)
    # positions come back as lattice site + displacement: equal up to rounding
    assert np.abs(st["x"] - p0.x).max() < 1e-12 * cfg.hx
    assert np.abs(st["ux"]).max() < 1e-12
    assert stats["n_absorbed"] == 0


CASE_ORDERS = [(0, "fp64"), (2, "fp64"), (3, "fp64"), (2, "fp32"), (3, "fp32"), (0, "fp32")]


@pytest.mark.parametrize("order,prec", CASE_ORDERS)
def test_one_slice_from_oracle_state(order, prec):
    cfg, beam = W.small(n=32, nzeta=24, nb=1.0)
    cfg = with_order(cfg, order)
    k = 12
    print(f"one slice order {order} {prec}", flush=True)
    _, st = O.run_box(cfg, beam, keep=lambda kk, r: None, k_end=k)
    st_k = st.copy()
    st_next, rec = O.advance_slice(cfg, st, beam)
    with Q().Box(cfg, prec) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.set_state(k, oracle_state_to_abi(cfg, st_k))
        outs = {q: box.empty(q) for q in FIELD_NAMES + DEPOSIT_NAMES}
        box.advance_slice(outs)
        torch.cuda.synchronize()
        got = {q: to_np(t) for q, t in outs.items()}
        after = box.get_state()
    errs = field_errors(got, {q: rec[q] for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert all(e < tol for e in errs.values()), errs
    p = st_next.plasma
    for name, ref in (("x", p.x), ("y", p.y), ("ux", p.ux), ("uy", p.uy), ("psi", p.psi)):
        d = np.abs(after[name] - ref).max()
        scale = max(np.abs(ref).max(), 1e-30) if name not in ("x", "y") else cfg.hx
        assert d / scale < (1e-10 if prec == "fp64" else 2e-5), (name, d)


def run_box_gpu(cfg, beam, prec):
    with Q().Box(cfg, prec) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
        iters = torch.zeros(cfg.nzeta, dtype=torch.int32, device="cuda")
        stats = box.run_box(stack=stack, pc_iters=iters)
        return {q: to_np(t) for q, t in stack.items()}, iters.cpu().numpy(), stats


@pytest.mark.parametrize("order", [0, 2, 3])
def test_nonlinear_box_fp64_matches_oracle(order):
    cfg, beam = W.small(n=32, nzeta=24, nb=1.0, pc_max_iter=5, pc_tol=1e-4)
    cfg = with_order(cfg, order)
    print(f"nonlinear box order {order}", flush=True)
    recs, _ = O.run_box(cfg, beam)
    got, iters, _ = run_box_gpu(cfg, beam, "fp64")
    errs = field_errors(got, {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    assert all(e < 1e-8 for e in errs.values()), errs
    assert list(iters) == [r["pc_iters"] for r in recs]


@pytest.mark.parametrize("order", [2, 3])
def test_linear_box_fp32_matches_oracle(order):
    cfg, beam = W.c1()
    cfg = with_order(cfg, order)
    print(f"c1 box order {order} fp32", flush=True)
    recs, _ = O.run_box(cfg, beam)
    got, _, stats = run_box_gpu(cfg, beam, "fp32")
    errs = field_errors(got, {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    assert all(e < 1e-3 for e in errs.values()), errs
    assert stats["n_absorbed"] == 0


@pytest.mark.parametrize("order,prec", [(3, "fp64"), (3, "fp32"), (0, "fp64")])
def test_particle_beam_box_matches_oracle(order, prec):
    cfg, beam = W.small_particle_beam()
    cfg = with_order(cfg, order)
    print(f"particle beam box order {order} {prec}", flush=True)
    keys = O.beam_slice_index(cfg, beam.zeta)
    perm = np.argsort(np.where((keys >= 0) & (keys < cfg.nzeta), keys, cfg.nzeta), kind="stable")
    b = W.copy_beam(beam)
    recs, _ = O.run_box(cfg, b)
    with Q().Box(cfg, prec) as box:
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), beam.dt)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
        box.run_box(stack=stack)
        got = {q: to_np(t) for q, t in stack.items()}
        after = box.get_beam_particles().double().cpu().numpy()
    errs = field_errors(got, {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    tol = 1e-9 if prec == "fp64" else 1e-3
    assert all(e < tol for e in errs.values()), errs
    ref_b = np.stack([getattr(b, n)[perm] for n in ("x", "y", "zeta", "ux", "uy", "uz", "w")])
    for c, name in enumerate(("x", "y", "zeta", "ux", "uy", "uz", "w")):
        scale = np.abs(ref_b[c]).max()
        d = np.abs(after[c] - ref_b[c]).max()
        assert d <= (2e-6 if prec == "fp64" else 2e-4) * scale + 1e-12, (name, d, scale)


def cotangents(cfg, k_lo, k_hi, seed=5):
    rng = np.random.default_rng(seed)
    cx, cy = cfg.nx // 2, cfg.ny // 2
    w = np.zeros((k_hi - k_lo + 1, len(A.FIELD_KEYS), cfg.ny + 1, cfg.nx + 1))
    w[:, :, cy - 3:cy + 4, cx - 3:cx + 4] = rng.normal(size=(k_hi - k_lo + 1, len(A.FIELD_KEYS),
                                                             7, 7))
    return w


@pytest.mark.parametrize("order,prec,tol", [(2, "fp64", 1e-9), (3, "fp64", 1e-9), (3, "fp32", 1e-3)])
def test_adjoint_matches_oracle(order, prec, tol):
    cfg, beam = W.small(n=32, nzeta=14, ppc=1, nb=0.9, sigma=0.8, pc_max_iter=3, pc_tol=0.0,
                        extent=5.0)
    cfg = with_order(cfg, order)
    k_lo, k_hi = cfg.nzeta // 2, cfg.nzeta - 2
    w = cotangents(cfg, k_lo, k_hi)
    recs, tape = A.forward_with_tape(cfg, beam)

    def cot(k):
        if k < k_lo or k > k_hi:
            return {}
        return {q: w[k - k_lo, i] for i, q in enumerate(A.FIELD_KEYS)}
    ga_o, gsx, gsy = A.adjoint_box(cfg, beam, tape, cot)
    gs_o = np.array([gsx, gsy])
    L_o = A.loss_value(recs, cot)
    print(f"adjoint order {order} {prec}", flush=True)
    with Q().Box(cfg, prec) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        box.record(k_hi + 1, 4)
        c = {q: torch.tensor(w[:, i], dtype=box.fdtype, device="cuda")
             for i, q in enumerate(A.FIELD_KEYS)}
        ga, gs, loss = box.adjoint(k_lo, c)
        torch.cuda.synchronize()
        ga, gs, L = ga.cpu().numpy(), gs.cpu().numpy(), float(loss.cpu()[0])
    scale = np.abs(ga_o).max()
    assert scale > 0
    assert np.abs(ga - ga_o).max() / scale <= tol, (ga, ga_o)
    assert np.all(np.abs(gs - gs_o) <= tol * np.abs(gs_o)), (gs, gs_o)
    assert abs(L - L_o) <= tol * max(abs(L_o), 1e-30) + 1e-12, (L, L_o)


def test_adjoint_rejects_the_nearest_node_shape():
    qsp = Q()
    cfg, beam = W.small(n=16, nzeta=4, ppc=2)
    cfg = dataclasses.replace(cfg, shape_order=0)
    with qsp.Box(cfg, "fp64") as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        with pytest.raises(qsp.QspError) as e:
            box.record(cfg.nzeta, 2)
        assert e.value.status == qsp.QSP_ERR_INVALID_ARG
