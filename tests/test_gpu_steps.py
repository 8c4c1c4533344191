"""Multi-time-step loop with beam evolution on the GPU (each time step runs
the whole box with a fresh plasma while the macro-particle beam advances in
every slice, re-sorted by slice between steps) against the FP64 oracle, and
the betatron oscillation of test electrons in a pure ion column against
k_beta = 1/sqrt(2 gamma)."""
import numpy as np
import pytest

import workloads as W
from oracle import qsp_oracle as O
from parity_util import FIELD_NAMES, field_errors, oracle_state_to_abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Q():
    from paper_2109_10277_amd import qsp
    return qsp


NAMES = ("x", "y", "zeta", "ux", "uy", "uz", "w")


def slice_sort(cfg, beam):
    """The library's order: stable by slice, particles outside the box last."""
    keys = O.beam_slice_index(cfg, beam.zeta)
    order = np.argsort(np.where((keys >= 0) & (keys < cfg.nzeta), keys, cfg.nzeta), kind="stable")
    for n in NAMES:
        setattr(beam, n, getattr(beam, n)[order].copy())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multistep_particle_beam_matches_oracle(prec):
    cfg, beam = W.small_particle_beam()
    nsteps = 3
    ref_beam = W.copy_beam(beam)
    slice_sort(cfg, ref_beam)
    last = {}

    def after(step, recs):
        if step == nsteps - 1:
            last.update({q: O.stack(recs, q) for q in FIELD_NAMES})
        slice_sort(cfg, ref_beam)
    print(f"multistep particle beam {prec}", flush=True)
    for step in range(nsteps):
        recs, _ = O.run_box(cfg, ref_beam)
        after(step, recs)
    with Q().Box(cfg, prec) as box:
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), beam.dt)
        for step in range(nsteps):
            box.init_plasma()
            stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES}
            box.run_box(stack=stack)
        box.init_plasma()                      # re-sorts the pushed beam
        got_b = box.get_beam_particles().double().cpu().numpy()
        got = {q: t.double().cpu().numpy() for q, t in stack.items()}
    errs = field_errors(got, last)
    print("  rel-L2", {q: f"{e:.1e}" for q, e in errs.items()})
    # both sides store the beam in FP32: a one-ulp (6e-8) difference in a
    # pushed position, from another rounding order of the same FP64 push,
    # carries into the next step's fields
    tol = 1e-7 if prec == "fp64" else 2e-3
    assert all(e < tol for e in errs.values()), errs
    ref_b = np.stack([getattr(ref_beam, n).astype(np.float64) for n in NAMES])
    for c, name in enumerate(NAMES):
        scale = np.abs(ref_b[c]).max()
        d = np.abs(got_b[c] - ref_b[c]).max()
        assert d <= (5e-6 if prec == "fp64" else 5e-4) * scale + 1e-12, (name, d, scale)


def dead_oracle_state(cfg):
    """Unperturbed plasma with every electron removed: ions only."""
    st = O.initial_state(cfg)
    st.plasma.w[:] = 0.0
    return st


def dead_state(cfg):
    return oracle_state_to_abi(cfg, dead_oracle_state(cfg))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_betatron_oscillation_in_ion_column(prec):
    gamma, dt, x0, nsteps = 2000.0, 6.0, 0.2, 200
    cfg, beam = W.ion_column(gamma=gamma, dt=dt, x0=x0)
    state = dead_state(cfg)
    print(f"betatron ion column {prec}", flush=True)
    xs = [beam.x.astype(np.float64)]
    with Q().Box(cfg, prec) as box:
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), dt)
        for step in range(nsteps):
            box.set_state(0, state)            # ions only: no plasma electrons
            box.run_box()
            xs.append(box.get_beam_particles()[0].double().cpu().numpy())
    xs = np.array(xs)
    t = dt * np.arange(nsteps + 1)
    kb = 1.0 / np.sqrt(2.0 * gamma)
    # slice 0 holds the electron started at (x0, 0); the beam keeps its order
    assert np.max(np.abs(xs[:, 0] - x0 * np.cos(kb * t))) < 0.03 * x0
    # the same trajectory as the oracle's (FP32 storage on both sides)
    ref = W.ion_column(gamma=gamma, dt=dt, x0=x0)[1]
    rx = [ref.x.astype(np.float64).copy()]
    O.run_steps(cfg, ref, nsteps, state_fn=lambda: dead_oracle_state(cfg),
                after_step=lambda s, r: rx.append(ref.x.astype(np.float64).copy()))
    rx = np.array(rx)
    tol = 1e-5 if prec == "fp64" else 2e-3
    assert np.max(np.abs(xs - rx)) < tol * x0, np.max(np.abs(xs - rx))
