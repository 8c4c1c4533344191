"""GPU parity of the HIP slice loop against the FP64 oracle, through the C ABI.

Tolerances: FP64 kernels agree with the oracle to round-off amplified by the
loop (<= 1e-9 rel-L2); FP32 kernels meet the stated bars, <= 1e-4 rel-L2 per
field for one slice from an oracle state and <= 1e-3 over a linear-regime
box (the C1 workload).  Bz is measured against ||(Bx, By)||."""
import numpy as np
import pytest

import workloads as W
from oracle import qsp_oracle as O
from parity_util import (DEPOSIT_NAMES, FIELD_NAMES, field_errors,
                         oracle_state_to_abi, rel_l2)

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
    return t.detach().double().cpu().numpy()


# ------------------------------------------------------------------ DST solve

@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (32, 128), (256, 256), (512, 512),
                                   (1024, 1024), (1024, 512), (2048, 2048)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_poisson_solve_matches_oracle(nx, ny, prec):
    cfg = W.BoxConfig(nx=nx, ny=ny, x_lo=-3.0, x_hi=3.0, y_lo=-2.0, y_hi=2.5,
                      nzeta=2, zeta_hi=0.0, dzeta=0.1)
    print(f"poisson {nx}x{ny} {prec}", flush=True)
    rng = np.random.default_rng(nx * 7 + ny)
    nb = 3
    src = O.zero_boundary(rng.normal(size=(ny + 1, nx + 1)))
    src2 = O.zero_boundary(np.cos(np.arange(ny + 1))[:, None] * np.ones(nx + 1))
    src3 = O.zero_boundary(np.zeros((ny + 1, nx + 1)) + 1.0)
    srcs = np.stack([src, src2, src3])
    with Q().Box(cfg, prec) as box:
        dt = box.fdtype
        s = torch.tensor(srcs, dtype=dt, device="cuda")
        for shift in (0.0, 1.32):
            d = torch.zeros_like(s)
            box.solve_poisson(s, d, shift)
            torch.cuda.synchronize()
            got = to_np(d)
            # Round-off of the transforms is amplified ~n times in the solution
            # of a white-noise source (its low modes carry ~1/n of its norm and
            # are divided by the smallest eigenvalues): tolerance eps_n n log2 n.
            n = max(nx, ny)
            fast = prec == "fp32" and all(256 <= m <= 1024 for m in (nx, ny))
            for b in range(nb):
                ref = O.poisson_solve(cfg, srcs[b], shift)
                err = rel_l2(got[b], ref)
                if fast and b != 1:
                    # transforms without the prefix-sum recurrence: plain FFT
                    # round-off (a float32 model of the solve gives 1.4e-7 to
                    # 2.5e-7 for these sources, the recurrence 1.2e-6 to
                    # 3.9e-6); the rapidly oscillating source 1 loses ~1e-5
                    # in any float32 transform
                    unit = 2e-6
                else:
                    unit = (1e-15 if prec == "fp64" else 1e-7) * n * np.log2(n)
                print(f"  source {b} shift {shift}: rel-L2 {err:.2e} (tol {unit:.1e})")
                assert err < unit, (b, shift, err)
                assert np.all(got[b][0] == 0) and np.all(got[b][:, -1] == 0)


# ------------------------------------------------------------------ one slice

def one_slice_case(cfg, beam, k, prec, deposit_mode=0):
    """Oracle runs to slice k; the GPU imports the oracle state and computes
    slice k.  Returns (gpu outputs, oracle record, gpu state after,
    oracle state after)."""
    _, st = O.run_box(cfg, beam, keep=lambda kk, r: None, k_end=k)
    st_k = st.copy()
    st_next, rec = O.advance_slice(cfg, st, beam)
    with Q().Box(cfg, prec, deposit_mode=deposit_mode) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.set_state(k, oracle_state_to_abi(cfg, st_k))
        outs = {q: box.empty(q) for q in FIELD_NAMES + DEPOSIT_NAMES}
        box.advance_slice(outs)
        torch.cuda.synchronize()
        got = {q: to_np(t) for q, t in outs.items()}
        after = box.get_state()
    return got, rec, after, st_next


def rect_box():
    """64 x 16 nodes with hx != hy."""
    cfg, beam = W.small(n=64, nzeta=24, nb=1.0)
    cfg.ny, cfg.y_lo, cfg.y_hi = 16, -3.0, 3.0
    return cfg, beam


CASES = {
    "c1_k20": (lambda: W.c1(), 20),
    "small_nonlinear_k12": (lambda: W.small(n=32, nzeta=24, nb=1.0), 12),
    "small_ppc2_k10": (lambda: W.small(n=32, nzeta=24, ppc=2, nb=1.0), 10),
    "rect_k9": (lambda: rect_box(), 9),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_slice_from_oracle_state(case, prec):
    make, k = CASES[case]
    cfg, beam = make()
    print(f"one-slice {case} {prec}", flush=True)
    got, rec, after, st_next = one_slice_case(cfg, beam, k, prec)
    errs = field_errors({q: got[q] for q in FIELD_NAMES + DEPOSIT_NAMES},
                        {q: rec[q] for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    tol = 1e-9 if prec == "fp64" else 1e-4
    bad = {q: e for q, e in errs.items() if e > tol}
    assert not bad, (errs, rec["pc_iters"])
    # state after the real push (positions, momenta, Psi, history)
    p = st_next.plasma
    for name, ref in (("x", p.x), ("y", p.y), ("ux", p.ux), ("uy", p.uy), ("psi", p.psi)):
        d = np.abs(after[name] - ref).max()
        scale = max(np.abs(ref).max(), 1e-30) if name not in ("x", "y") else cfg.hx
        assert d / scale < (1e-10 if prec == "fp64" else 2e-5), (name, d)
    assert np.abs(after["hist"][0] - p.hist[0]).max() <= \
        (1e-9 if prec == "fp64" else 1e-4) * max(np.abs(p.hist[0]).max(), 1e-30)


def test_tiled_and_global_deposits_agree():
    cfg, beam = W.small(n=32, nzeta=24, nb=2.0)
    a = one_slice_case(cfg, beam, 14, "fp64", deposit_mode=0)[0]
    b = one_slice_case(cfg, beam, 14, "fp64", deposit_mode=1)[0]
    for q in FIELD_NAMES + DEPOSIT_NAMES:
        assert rel_l2(a[q], b[q]) < 1e-12, q


# ------------------------------------------------------------------ whole box

def run_box_gpu(cfg, beam, prec, deposit_mode=0):
    with Q().Box(cfg, prec, deposit_mode=deposit_mode) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
        iters = torch.zeros(cfg.nzeta, dtype=torch.int32, device="cuda")
        resid = torch.zeros(cfg.nzeta, dtype=torch.float64, device="cuda")
        stats = box.run_box(stack=stack, pc_iters=iters, pc_resid=resid)
        return ({q: to_np(t) for q, t in stack.items()}, iters.cpu().numpy(),
                resid.cpu().numpy(), stats)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c1_box_matches_oracle(prec):
    cfg, beam = W.c1()
    print(f"c1 box {prec}", flush=True)
    recs, _ = O.run_box(cfg, beam)
    got, iters, resid, stats = run_box_gpu(cfg, beam, prec)
    ref = {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES}
    errs = field_errors(got, ref)
    tol = 1e-9 if prec == "fp64" else 1e-3
    assert all(e < tol for e in errs.values()), errs
    assert np.all(iters == 3)
    assert stats["slices"] == cfg.nzeta and stats["n_absorbed"] == 0 and stats["n_clamped"] == 0
    assert stats["pc_iterations"] == 3 * cfg.nzeta
    orc_res = np.array([r["pc_residuals"][-1] for r in recs])
    if prec == "fp64":
        assert np.allclose(resid, orc_res, rtol=1e-5, atol=1e-12)


def test_small_nonlinear_box_fp64_matches_oracle():
    cfg, beam = W.small(n=32, nzeta=24, nb=1.0, pc_max_iter=5, pc_tol=1e-4)
    recs, _ = O.run_box(cfg, beam)
    got, iters, _, stats = run_box_gpu(cfg, beam, "fp64")
    ref = {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES}
    errs = field_errors(got, ref)
    assert all(e < 1e-8 for e in errs.values()), errs
    assert list(iters) == [r["pc_iters"] for r in recs]


def test_abi_state_errors():
    qsp = Q()
    cfg, beam = W.small(n=16, nzeta=2)
    with qsp.Box(cfg, "fp32") as box:
        with pytest.raises(qsp.QspError) as e:
            box.advance_slice({})
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        box.init_plasma()
        box.advance_slice({})
        box.advance_slice({})
        with pytest.raises(qsp.QspError) as e:
            box.advance_slice({})
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        with pytest.raises(qsp.QspError) as e:
            box.set_beam_gaussian(np.full(cfg.nzeta, np.nan), 1.0, 1.0)
        assert e.value.status == qsp.QSP_ERR_INVALID_ARG


def test_mem_cap_is_enforced():
    qsp = Q()
    cfg, _ = W.small(n=64, nzeta=2)
    with pytest.raises(qsp.QspError) as e:
        qsp.Box(cfg, "fp32", mem_cap_bytes=1024)
    assert e.value.status == qsp.QSP_ERR_OUT_OF_MEMORY


# ------------------------------------------------------------------ particle beams

def run_particle_beam_box(cfg, beam, prec):
    with Q().Box(cfg, prec) as box:
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), beam.dt)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
        iters = torch.zeros(cfg.nzeta, dtype=torch.int32, device="cuda")
        box.run_box(stack=stack, pc_iters=iters)
        after = box.get_beam_particles().double().cpu().numpy()
        return {q: to_np(t) for q, t in stack.items()}, after


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_particle_beam_box_matches_oracle(prec):
    cfg, beam = W.small_particle_beam()
    print(f"particle beam box {prec}", flush=True)
    keys = O.beam_slice_index(cfg, beam.zeta)
    order = np.argsort(np.where((keys >= 0) & (keys < cfg.nzeta), keys, cfg.nzeta), kind="stable")
    b = W.copy_beam(beam)
    recs, _ = O.run_box(cfg, b)
    got, after = run_particle_beam_box(cfg, beam, prec)
    ref = {q: O.stack(recs, q) for q in FIELD_NAMES + DEPOSIT_NAMES}
    errs = field_errors(got, ref)
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    tol = 1e-9 if prec == "fp64" else 1e-3
    assert all(e < tol for e in errs.values()), errs
    # the beam after its per-slice push, in the library's slice-sorted order
    ref_b = np.stack([getattr(b, n)[order] for n in ("x", "y", "zeta", "ux", "uy", "uz", "w")])
    assert after.shape == ref_b.shape
    for c, name in enumerate(("x", "y", "zeta", "ux", "uy", "uz", "w")):
        scale = np.abs(ref_b[c]).max()
        d = np.abs(after[c] - ref_b[c]).max()
        assert d <= (2e-6 if prec == "fp64" else 2e-4) * scale + 1e-12, (name, d, scale)


@pytest.mark.parametrize("n", [1, 4095, 4096, 5 * 4096 + 123])
def test_beam_sort_stable_across_chunks(n):
    """The slice sort over several 4096-particle chunks with a ragged tail,
    keys spread over every slice, particles ahead of and behind the box and
    runs of equal keys: the sorted beam must be the stable argsort of the
    nearest-slice keys (particles outside the box last)."""
    cfg, _ = W.small_particle_beam(n=16, nzeta=300)
    rng = np.random.default_rng(1234 + n)
    zeta = rng.uniform(cfg.zeta_hi - (cfg.nzeta + 20) * cfg.dzeta, cfg.zeta_hi + 10 * cfg.dzeta, n)
    zeta[: n // 3] = cfg.zeta_hi - 7 * cfg.dzeta     # a long run of one key
    soa = np.stack([np.arange(n, dtype=np.float64)] + [rng.normal(size=n) for _ in range(6)])
    soa[2] = zeta
    soa = soa.astype(np.float32)
    with Q().Box(cfg, "fp32") as box:
        box.set_beam_particles(torch.tensor(soa, device="cuda"), 0.0)
        got = box.get_beam_particles().cpu().numpy()
    keys = O.beam_slice_index(cfg, soa[2].astype(np.float64))
    keys = np.where((keys >= 0) & (keys < cfg.nzeta), keys, cfg.nzeta)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(got, soa[:, order])


def test_beam_sort_and_counts():
    cfg, beam = W.small_particle_beam()
    with Q().Box(cfg, "fp32") as box:
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), 0.0)
        assert box.beam_count() == beam.x.size
        got = box.get_beam_particles().cpu().numpy()
    keys = O.beam_slice_index(cfg, got[2].astype(np.float64))
    keys = np.where((keys >= 0) & (keys < cfg.nzeta), keys, cfg.nzeta)
    assert np.all(np.diff(keys) >= 0)
    ref_keys = O.beam_slice_index(cfg, beam.zeta)
    ref_keys = np.where((ref_keys >= 0) & (ref_keys < cfg.nzeta), ref_keys, cfg.nzeta)
    order = np.argsort(ref_keys, kind="stable")
    assert np.array_equal(got, beam.soa()[:, order])
