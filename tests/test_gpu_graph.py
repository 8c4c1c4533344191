"""Whole-box graph replay: boxes run from HIP graphs give the results of the
same boxes launched one kernel at a time, over several replays with eager
work and synchronisations in between, with the kernel timer on, after the
beam changes (which forces a new capture), with a moving macro-particle
beam, and with the speculative predictor-corrector launch budgets (boxes
after the first launch only the iterations the slices needed before; a
slice left unconverged makes the box run again with every iteration)."""
import os

import numpy as np
import pytest

import workloads as W
from parity_util import DEPOSIT_NAMES, FIELD_NAMES, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Q():
    from paper_2109_10277_amd import qsp
    return qsp


def make_box(cfg, prec, graphs, budget=None):
    env = {"QSP_GRAPH": "1" if graphs else "0"}
    if budget is not None:
        env["QSP_PC_BUDGET"] = str(budget)
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return Q().Box(cfg, prec)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def run(box, cfg):
    box.init_plasma()
    stack = {q: box.empty(q, cfg.nzeta) for q in FIELD_NAMES + DEPOSIT_NAMES}
    iters = torch.zeros(cfg.nzeta, dtype=torch.int32, device="cuda")
    stats = box.run_box(stack=stack, pc_iters=iters)
    torch.cuda.synchronize()
    return {q: t.double().cpu().numpy() for q, t in stack.items()}, iters.cpu().numpy(), stats


def same(a, b, tol):
    for q in a:
        assert rel_l2(a[q], b[q]) <= tol, (q, rel_l2(a[q], b[q]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("solver", ["pc", "explicit"])
def test_graph_replays_match_eager_launches(prec, tol, solver):
    cfg, beam = W.small(n=64, nzeta=40, nb=1.0, pc_max_iter=4, pc_tol=1e-4)
    cfg.bxby_solver = solver
    if solver == "explicit":
        cfg.pc_max_iter, cfg.pc_tol = 6, (1e-10 if prec == "fp64" else 1e-5)
    print(f"graph replay {solver} {prec}", flush=True)
    eager = make_box(cfg, prec, graphs=False)
    eager.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    ref, ref_it, ref_st = run(eager, cfg)
    box = make_box(cfg, prec, graphs=True)
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    for rep in range(3):
        got, it, st = run(box, cfg)
        same(got, ref, tol)
        assert np.array_equal(it, ref_it)
        assert st["slices"] == ref_st["slices"] and st["particle_pushes"] == ref_st["particle_pushes"]
        assert st["pc_iterations"] == ref_st["pc_iterations"]
        # eager work in between: a few single slices on the same box
        box.init_plasma()
        for _ in range(3):
            box.advance_slice()
        torch.cuda.synchronize()
    eager.close()
    box.close()


def test_graph_with_timer_and_a_new_beam():
    cfg, beam = W.small(n=64, nzeta=32, nb=1.0, pc_max_iter=3, pc_tol=0.0)
    eager = make_box(cfg, "fp64", graphs=False)
    box = make_box(cfg, "fp64", graphs=True)
    for b in (beam, W.GaussianBeam(0.5 * beam.amp, 0.6, 0.9)):
        eager.set_beam_gaussian(b.amp, b.sigma_x, b.sigma_y)
        box.set_beam_gaussian(b.amp, b.sigma_x, b.sigma_y)
        ref, _, _ = run(eager, cfg)
        box.set_timing(4)
        for rep in range(2):
            box.set_timing(4)
            got, _, _ = run(box, cfg)
            same(got, ref, 1e-12)
            ms, n = box.kernel_times()["push"]
            assert n == len(range(0, cfg.nzeta - 1, 4)) and ms > 0.0
        box.set_timing(0)
    eager.close()
    box.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_graph_replays_with_a_moving_particle_beam(prec, tol):
    # the beam is pushed in every slice and sorted by slice again before each
    # box, so every box has other per-slice particle ranges: the replayed
    # boxes read them on the device and match eager launches box by box
    cfg, beam = W.small_particle_beam(n=64, nzeta=48, n_per_beam=3000)
    soa = torch.tensor(beam.soa(), device="cuda")
    print(f"graph replay moving beam {prec}", flush=True)
    eager = make_box(cfg, prec, graphs=False)
    box = make_box(cfg, prec, graphs=True)
    eager.set_beam_particles(soa.clone(), beam.dt)
    box.set_beam_particles(soa.clone(), beam.dt)
    for step in range(3):
        ref, ref_it, _ = run(eager, cfg)
        got, it, _ = run(box, cfg)
        same(got, ref, tol)
        assert np.array_equal(it, ref_it)
        b_ref = eager.get_beam_particles().double().cpu().numpy()
        b_got = box.get_beam_particles().double().cpu().numpy()
        assert np.abs(b_got - b_ref).max() <= tol * max(1.0, np.abs(b_ref).max()), step
    eager.close()
    box.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_pc_budgets_give_the_full_launch_results(prec, tol):
    # predictor-corrector to a tolerance: slices converge after 2-5
    # iterations; boxes after the first launch the learned counts only
    cfg, beam = W.small(n=64, nzeta=40, nb=1.0, pc_max_iter=5, pc_tol=1e-4)
    print(f"pc budgets {prec}", flush=True)
    eager = make_box(cfg, prec, graphs=False)
    eager.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    ref, ref_it, ref_st = run(eager, cfg)
    assert ref_it.min() < cfg.pc_max_iter    # there are launches to save
    box = make_box(cfg, prec, graphs=True)
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    for rep in range(3):
        got, it, st = run(box, cfg)
        same(got, ref, tol)
        assert np.array_equal(it, ref_it)
        assert st["pc_iterations"] == ref_st["pc_iterations"]
        assert st["pc_not_converged"] == ref_st["pc_not_converged"]
        assert st["box_reruns"] == 0, rep
    eager.close()
    box.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_pc_budget_shortfall_reruns_the_box(prec, tol):
    # budgets one short of what the slices need (QSP_PC_BUDGET=-1): every
    # box after the first leaves slices unconverged, is reset (plasma at
    # rest, the moving beam restored) and runs again with every iteration;
    # the results, iteration counts and the pushed beam are those of eager
    # launches box by box
    cfg, beam = W.small_particle_beam(n=64, nzeta=48, n_per_beam=3000)
    cfg.pc_max_iter, cfg.pc_tol = 5, 1e-4
    soa = torch.tensor(beam.soa(), device="cuda")
    print(f"pc budget rerun {prec}", flush=True)
    eager = make_box(cfg, prec, graphs=False)
    box = make_box(cfg, prec, graphs=True, budget=-1)
    eager.set_beam_particles(soa.clone(), beam.dt)
    box.set_beam_particles(soa.clone(), beam.dt)
    for step in range(3):
        ref, ref_it, ref_st = run(eager, cfg)
        got, it, st = run(box, cfg)
        same(got, ref, tol)
        assert np.array_equal(it, ref_it)
        assert st["pc_iterations"] == ref_st["pc_iterations"]
        assert st["box_reruns"] == (1 if step > 0 else 0), (step, st["box_reruns"])
        b_ref = eager.get_beam_particles().double().cpu().numpy()
        b_got = box.get_beam_particles().double().cpu().numpy()
        assert np.abs(b_got - b_ref).max() <= tol * max(1.0, np.abs(b_ref).max()), step
    eager.close()
    box.close()
