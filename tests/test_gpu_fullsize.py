"""GPU parity at the grid sizes the benchmarks run: one slice from the same
imported state on the GPU and in the FP64 oracle, at 512^2 and 1024^2
nodes (8 and 16 push tiles of 64 lattice sites across x, 16-32 with the
2 x 2 lattice), so that the tile offsets, the cross-tile halo flush and
the n = 512 / 1024 transform schedules inside the slice loop all meet the
oracle.

The state is seeded and shaped like the inside of a blowout
(workloads.blowout_slice_state): an electron-free column with a dense
sheath, particles tens of cells from their lattice site (deposits outside
their tile's histogram), particles below the 1 + Psi floor (the floored
push and deposit of the method's singular limit), particles that leave
the box during the push, and absorbed particles.  The transverse currents
of the previous slice are the state's own deposit, Bx/By of the two
previous slices seeded smooth planes.

Bars as for every one-slice case: FP64 to 1e-9 and FP32 to 1e-4 rel-L2
per field and deposit, the pushed particle state to 1e-10 / 2e-5, and the
integer outcomes (predictor-corrector iterations, floored pushes,
absorbed particles) equal to the oracle's.  Tiled against direct global
atomics: 1e-12 in FP64."""
import dataclasses
import functools

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
    return t.detach().double().cpu().numpy()


def c2_cfg(**kw):
    cfg, beam = W.c2()
    return dataclasses.replace(cfg, **kw), beam


def c3_cfg(ppc=1, **kw):
    """The paper-scale grid (1024^2 over [-8, 8]^2, 1024 slices) with the
    C3/C5 rigid driver (n_b/n0 = 5, sigma_r = 0.25, sigma_z = 1)."""
    cfg, beam = W.c5()
    return dataclasses.replace(cfg, ppc_x=ppc, ppc_y=ppc, **kw), beam


# name: (config and beam, slice index, macro-particle witness particles or 0)
CASES = {
    # a 64^2 box with the same kinds of particles, for a fast first look
    "small_64_m3": (lambda: W.small(n=64, nzeta=24, nb=1.0, pc_max_iter=3), 12, 0),
    # the seeded Bx/By of the previous slices are far from this slice's, so
    # the iteration needs a looser tolerance than the C2 run's 1e-4 to stop
    # before its cap (the residuals fall ~8x per iteration here)
    "c2_512_tol": (lambda: c2_cfg(pc_max_iter=5, pc_tol=5e-3), 420, 0),
    "c2_512_m3": (lambda: c2_cfg(pc_max_iter=3, pc_tol=0.0), 420, 0),
    "c5_512_ppc2_m3": (lambda: (dataclasses.replace(c2_cfg()[0], ppc_x=2, ppc_y=2,
                                                    pc_max_iter=3, pc_tol=0.0), c2_cfg()[1]),
                       420, 0),
    "c3_1024_m3": (lambda: c3_cfg(pc_max_iter=3, pc_tol=0.0), 427, 0),
    "c3_1024_witness_m2": (lambda: c3_cfg(pc_max_iter=2, pc_tol=0.0), 853, 49152),
}


def import_state(cfg, k, seed):
    """The oracle SliceState of the seeded blowout slice (J_perp of slice
    k-1 taken as the state's own deposit)."""
    s = W.blowout_slice_state(cfg, seed=seed)
    p = O.Plasma(x=s["x"], y=s["y"], ux=s["ux"], uy=s["uy"], psi=s["psi"], w=s["w"],
                 hist=s["hist"])
    pl = W.smooth_planes(cfg, seed=seed + 1)
    j = O.plasma_deposit(cfg, p, ("jx", "jy"))
    return O.SliceState(k, p, j["jx"], j["jy"], pl["bx_prev1"], pl["by_prev1"],
                        pl["bx_prev2"], pl["by_prev2"]), s


def make_beam(name, cfg, gbeam, k, nwit):
    if not nwit:
        return gbeam
    return W.witness_slice_beam(cfg, k, nwit)


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    """(cfg, beam, state at k, oracle state at k+1, oracle record of slice k,
    oracle beam after its push, special-particle indices)."""
    make, k, nwit = CASES[name]
    cfg, gbeam = make()
    st, s = import_state(cfg, k, seed=1000 + k)
    beam = make_beam(name, cfg, gbeam, k, nwit)
    b_in = W.copy_beam(beam) if nwit else beam
    print(f"  oracle slice {k} of {name} ({cfg.nx}x{cfg.ny}, {st.plasma.x.size} particles)",
          flush=True)
    st_next, rec = O.advance_slice(cfg, st.copy(), b_in)
    return cfg, beam, st, st_next, rec, b_in if nwit else None, s


def gpu_case(cfg, beam, st, prec, deposit_mode=0):
    with Q().Box(cfg, prec, deposit_mode=deposit_mode) as box:
        if hasattr(beam, "amp"):
            box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y, beam.x0, beam.y0)
        else:
            box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), beam.dt)
        box.set_state(st.k, oracle_state_to_abi(cfg, st))
        before = box.stats()
        outs = {q: box.empty(q) for q in FIELD_NAMES + DEPOSIT_NAMES}
        box.advance_slice(outs)
        torch.cuda.synchronize()
        got = {q: to_np(t) for q, t in outs.items()}
        after = box.get_state()
        stats = box.stats()
        pushed = box.get_beam_particles().double().cpu().numpy() if not hasattr(beam, "amp") \
            else None
    d = {c: stats[c] - before[c] for c in ("n_clamped", "n_absorbed", "n_deposit_global",
                                           "pc_iterations")}
    return got, after, d, pushed


def check_state(cfg, after, st_next, prec, floored):
    """The pushed particle state against the oracle's.  A floored particle's
    momentum changes by (gamma/D) E dzeta with gamma/D ~ 1/(2 floor^2) =
    5000: its new momentum carries the relative error of the gathered
    fields, so those particles are held to the field bar (1e-4 in FP32),
    the others to 2e-5 of the largest value."""
    p = st_next.plasma
    rest = np.ones(p.x.size, dtype=bool)
    rest[floored] = False
    for name, ref in (("x", p.x), ("y", p.y), ("ux", p.ux), ("uy", p.uy), ("psi", p.psi)):
        for sel, bar in ((rest, 2e-5), (floored, 1e-4)):
            d = np.abs(after[name][sel] - ref[sel]).max()
            scale = max(np.abs(ref[sel]).max(), 1e-30) if name not in ("x", "y") else cfg.hx
            assert d / scale < (1e-10 if prec == "fp64" else bar), (name, d, scale)
    # absorbed particles: exactly the oracle's
    assert np.array_equal(after["w"] == 0, p.w == 0)
    # the newest history slot of the live particles (an absorbed particle's
    # history is never read again: it neither moves nor deposits)
    live = p.w > 0
    h = p.hist[0][:, live]
    assert np.abs(after["hist"][0][:, live] - h).max() <= \
        (1e-9 if prec == "fp64" else 1e-4) * max(np.abs(h).max(), 1e-30)


@pytest.mark.parametrize("name,prec", [
    ("small_64_m3", "fp64"),
    ("small_64_m3", "fp32"),
    ("c2_512_tol", "fp64"),
    ("c2_512_m3", "fp32"),
    ("c5_512_ppc2_m3", "fp64"),
    ("c5_512_ppc2_m3", "fp32"),
    ("c3_1024_m3", "fp64"),
    ("c3_1024_m3", "fp32"),
    ("c3_1024_witness_m2", "fp64"),
    ("c3_1024_witness_m2", "fp32"),
])
def test_full_size_slice_matches_oracle(name, prec):
    print(f"full-size slice {name} {prec}", flush=True)
    cfg, beam, st, st_next, rec, beam_after, s = oracle_case(name)
    nX = cfg.nx * cfg.ppc_x
    assert nX // 64 >= (1 if name.startswith("small") else 8)   # push tiles across x
    got, after, d, pushed = gpu_case(cfg, beam, st, prec)
    errs = field_errors(got, {q: rec[q] for q in FIELD_NAMES + DEPOSIT_NAMES})
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()}, "counters", d,
          "oracle iterations", rec["pc_iters"], "clamped", rec["n_clamped"],
          "absorbed", rec["n_absorbed"], flush=True)
    tol = 1e-9 if prec == "fp64" else 1e-4
    bad = {q: e for q, e in errs.items() if e > tol}
    assert not bad, errs
    check_state(cfg, after, st_next, prec, s["floored"])
    # integer outcomes of the slice
    assert d["pc_iterations"] == rec["pc_iters"]
    assert d["n_clamped"] == rec["n_clamped"] == s["floored"].size > 0
    assert d["n_absorbed"] == rec["n_absorbed"] > 0
    assert d["n_deposit_global"] > 0
    if pushed is not None:
        ref = beam_after
        # the library holds the beam sorted by slice (stable); all of it sits
        # in slice k, so the order is the input order
        ref_b = np.stack([getattr(ref, f) for f in ("x", "y", "zeta", "ux", "uy", "uz", "w")])
        for c in range(7):
            scale = np.abs(ref_b[c]).max()
            dd = np.abs(pushed[c] - ref_b[c]).max()
            assert dd <= (2e-6 if prec == "fp64" else 2e-4) * scale + 1e-12, (c, dd, scale)


def test_full_size_predictor_corrector_exits_early():
    # the tolerance run converges before its cap, like the C2 workload
    cfg, beam, st, st_next, rec, _, _ = oracle_case("c2_512_tol")
    assert 1 <= rec["pc_iters"] < cfg.pc_max_iter, rec["pc_residuals"]
    assert rec["pc_residuals"][-1] < cfg.pc_tol <= rec["pc_residuals"][-2]


def test_full_size_tiled_and_direct_deposits_agree():
    cfg, beam, st, _, _, _, _ = oracle_case("c2_512_m3")
    print("full-size tiled / direct", flush=True)
    a, _, da, _ = gpu_case(cfg, beam, st.copy(), "fp64")
    b, _, db, _ = gpu_case(cfg, beam, st.copy(), "fp64", deposit_mode=1)
    assert da["n_deposit_global"] > 0 and db["n_deposit_global"] == 0
    for q in FIELD_NAMES + DEPOSIT_NAMES:
        assert rel_l2(a[q], b[q]) < 1e-12, (q, rel_l2(a[q], b[q]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_lineout_and_axis_outputs(prec):
    # qsp_box_out.lineout / axis carry row ny/2 and node (nx/2, ny/2) of
    # every slice: bit-equal to the stacked planes of the same run, and equal
    # to the oracle's within the box bars when requested without planes
    cfg, beam = W.c1()
    names = FIELD_NAMES + DEPOSIT_NAMES
    jc, ic = cfg.ny // 2, cfg.nx // 2
    print(f"lineout / axis outputs {prec}", flush=True)
    with Q().Box(cfg, prec) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        stack = {q: box.empty(q, cfg.nzeta) for q in names}
        line = {q: torch.zeros(cfg.nzeta, cfg.nx + 1, dtype=box.dtype_of(q), device="cuda")
                for q in names}
        axis = {q: torch.zeros(cfg.nzeta, dtype=box.dtype_of(q), device="cuda") for q in names}
        box.run_box(stack=stack, lineout=line, axis=axis)
        torch.cuda.synchronize()
        for q in names:
            assert torch.equal(line[q], stack[q][:, jc, :]), q
            assert torch.equal(axis[q], stack[q][:, jc, ic]), q
        box.init_plasma()
        line2 = {q: torch.zeros_like(line[q]) for q in names}
        axis2 = {q: torch.zeros_like(axis[q]) for q in names}
        box.run_box(lineout=line2, axis=axis2)
        torch.cuda.synchronize()
        got_line = {q: to_np(line2[q]) for q in names}
        got_axis = {q: to_np(axis2[q]) for q in names}
    recs, _ = O.run_box(cfg, beam)
    tol = 1e-9 if prec == "fp64" else 1e-3
    rows = cfg.ny - 1
    bperp = np.linalg.norm(np.stack([O.stack(recs, "bx")[:, 1:-1, 1:-1],
                                     O.stack(recs, "by")[:, 1:-1, 1:-1]])) / np.sqrt(rows)
    for q in names:
        ref = O.stack(recs, q)
        ref_line = ref[:, jc, 1:-1]
        # scale: the field's rms row (fields odd in y vanish on the axis row)
        den = bperp if q == "bz" else max(np.linalg.norm(ref_line),
                                          np.linalg.norm(ref[:, 1:-1, 1:-1]) / np.sqrt(rows))
        err = np.linalg.norm(got_line[q][:, 1:-1] - ref_line) / den
        assert err < tol, (q, err)
        # the axis value against the same scale (fields odd in x or y vanish
        # on the axis of the round, centred beam)
        err_axis = np.linalg.norm(got_axis[q] - ref[:, jc, ic]) / den
        assert err_axis < tol, (q, err_axis)
