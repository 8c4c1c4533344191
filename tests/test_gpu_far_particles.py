"""GPU parity of the plasma deposit when many particles have left their push
tile, as in the sheath around a blown-out bubble (Sec. III.B deposition):
far stencils go to global atomics beside the tile histograms, both for
tiles of one particle per thread and for the 16-row tiles whose threads
loop over several particles.  Each is checked against the FP64 oracle and
against direct global atomics (the same sums in another order).

Bars as for every one-slice case: FP64 to 1e-9, FP32 to 1e-4 per field;
tiled against direct atomics in FP64 to 1e-12."""
import dataclasses
import os

import numpy as np
import pytest

import workloads as W
from oracle import qsp_oracle as O
from parity_util import DEPOSIT_NAMES, FIELD_NAMES, field_errors, oracle_state_to_abi, rel_l2

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


def scattered_state(cfg, beam, k, seed, reach):
    """The oracle's state at slice k with every particle moved by up to
    `reach` cells in x and y (kept one cell inside the box) and given small
    random transverse momenta: with reach above the tile halo most
    particles deposit outside their tile, spread over a window of about
    (2 reach)^2 nodes per workgroup."""
    _, st = O.run_box(cfg, beam, keep=lambda kk, r: None, k_end=k)
    rng = np.random.default_rng(seed)
    p = st.plasma
    n = p.x.size
    p.x = np.clip(p.x + rng.uniform(-reach, reach, n) * cfg.hx, cfg.x_lo + cfg.hx,
                  cfg.x_hi - cfg.hx)
    p.y = np.clip(p.y + rng.uniform(-reach, reach, n) * cfg.hy, cfg.y_lo + cfg.hy,
                  cfg.y_hi - cfg.hy)
    p.ux = p.ux + rng.normal(0.0, 0.05, n)
    p.uy = p.uy + rng.normal(0.0, 0.05, n)
    return st


def gpu_slice(cfg, beam, k, st, prec, deposit_mode=0, tile_rows=None):
    old = os.environ.get("QSP_TILE_ROWS")
    if tile_rows is not None:
        os.environ["QSP_TILE_ROWS"] = str(tile_rows)
    try:
        with Q().Box(cfg, prec, deposit_mode=deposit_mode) as box:
            box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
            box.set_state(k, oracle_state_to_abi(cfg, st))
            outs = {q: box.empty(q) for q in FIELD_NAMES + DEPOSIT_NAMES}
            box.advance_slice(outs)
            torch.cuda.synchronize()
            got = {q: to_np(t) for q, t in outs.items()}
            return got, box.get_state(), box.stats()
    finally:
        if tile_rows is not None:
            if old is None:
                del os.environ["QSP_TILE_ROWS"]
            else:
                os.environ["QSP_TILE_ROWS"] = old


def check_against_oracle(cfg, beam, k, st, prec, **kw):
    st_k = st.copy()
    st_next, rec = O.advance_slice(cfg, st, beam)
    got, after, stats = gpu_slice(cfg, beam, k, st_k, prec, **kw)
    errs = field_errors(got, {q: rec[q] for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()},
          "deposits outside their tile", stats["n_deposit_global"])
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert all(e < tol for e in errs.values()), errs
    p = st_next.plasma
    for name, ref in (("x", p.x), ("y", p.y), ("ux", p.ux), ("uy", p.uy), ("psi", p.psi)):
        d = np.abs(after[name] - ref).max()
        scale = max(np.abs(ref).max(), 1e-30) if name not in ("x", "y") else cfg.hx
        assert d / scale < (1e-10 if prec == "fp64" else 2e-5), (name, d)
    return got, stats


# reach 3: far stencils just outside the halo; 12: most particles far,
# spread over ~25 x 25 nodes per workgroup; 40: spread over most of the box
@pytest.mark.parametrize("reach", [3, 12, 40])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_scattered_plasma_one_slice(reach, prec):
    cfg, beam = W.small(n=64, nzeta=24, nb=1.0, extent=4.0)
    k = 10
    print(f"scattered plasma reach {reach} {prec}", flush=True)
    st = scattered_state(cfg, beam, k, seed=reach, reach=reach)
    _, stats = check_against_oracle(cfg, beam, k, st, prec)
    # the deposit-only pass at import and the real push both see far particles
    assert stats["n_deposit_global"] > (cfg.nx * cfg.ny // 4 if reach >= 12 else 0)


@pytest.mark.parametrize("order", [0, 2, 3])
def test_scattered_plasma_shape_orders(order):
    cfg, beam = W.small(n=64, nzeta=24, nb=1.0, extent=4.0)
    cfg = dataclasses.replace(cfg, shape_order=order)
    if order == 0:
        cfg = dataclasses.replace(cfg, ppc_x=2, ppc_y=2)
    k = 10
    print(f"scattered plasma order {order}", flush=True)
    st = scattered_state(cfg, beam, k, seed=7 + order, reach=12)
    check_against_oracle(cfg, beam, k, st, "fp64")


def test_scattered_plasma_two_by_two_lattice():
    # 2 x 2 particles per cell: a 64-site tile row spans 32 cells
    cfg, beam = W.small(n=32, nzeta=24, ppc=2, nb=1.0, extent=4.0)
    k = 10
    print("scattered plasma ppc 2", flush=True)
    st = scattered_state(cfg, beam, k, seed=21, reach=12)
    check_against_oracle(cfg, beam, k, st, "fp64")


@pytest.mark.parametrize("reach", [12, 40])
def test_tiled_direct_atomics_and_looping_form_agree(reach):
    cfg, beam = W.small(n=64, nzeta=24, nb=1.0, extent=4.0)
    k = 10
    st = scattered_state(cfg, beam, k, seed=3 + reach, reach=reach)
    print(f"tiled / direct / 16-row tiles, reach {reach}", flush=True)
    a, _, sa = gpu_slice(cfg, beam, k, st.copy(), "fp64")
    b, _, _ = gpu_slice(cfg, beam, k, st.copy(), "fp64", deposit_mode=1)
    c, _, sc = gpu_slice(cfg, beam, k, st.copy(), "fp64", tile_rows=16)
    assert sa["n_deposit_global"] > 0 and sc["n_deposit_global"] > 0
    for q in FIELD_NAMES + DEPOSIT_NAMES:
        assert rel_l2(a[q], b[q]) < 1e-12, (q, rel_l2(a[q], b[q]))
        assert rel_l2(a[q], c[q]) < 1e-12, (q, rel_l2(a[q], c[q]))


def test_blowout_box_fp64_matches_oracle():
    # a narrow dense driver blows the plasma out well beyond the tile halo
    cfg, beam = W.small(n=64, nzeta=32, nb=8.0, sigma=0.35, extent=4.0, pc_max_iter=5,
                        pc_tol=1e-4)
    print("blowout box", flush=True)
    recs, _ = O.run_box(cfg, beam)
    with Q().Box(cfg, "fp64") as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
        iters = torch.zeros(cfg.nzeta, dtype=torch.int32, device="cuda")
        stats = box.run_box(stack=stack, pc_iters=iters)
        got = {q: to_np(t) for q, t in stack.items()}
    errs = field_errors(got, {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()},
          "deposits outside their tile", stats["n_deposit_global"])
    assert all(e < 1e-8 for e in errs.values()), errs
    assert list(iters.cpu().numpy()) == [r["pc_iters"] for r in recs]
    assert stats["n_deposit_global"] > 0
