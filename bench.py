#!/usr/bin/env python3
"""Benchmark of the quasi-static PIC slice loop on one MI355X.

Headline: one full time step of the paper-scale box (Sec. VI, the single-GPU
table): 1024 x 1024 transverse cells over [-8, 8]^2 k_p^-1, 1024 slices over
zeta in (-7, 5], 1 plasma electron per cell (1,048,576 particles), a driver
(n_b/n0 = 5, sigma_r = 0.25, sigma_z = 1) and a witness (n_b/n0 = 20,
sigma_r = 0.1, sigma_z = 0.2, 5 behind it) of 2^21 FP32 macro-particles
each with seeded normal positions and gamma = 2000, pushed in every slice
(dt = 6), Bx/By predictor-corrector to 1e-4 (at most 5 iterations), FP32
particles and fields with FP64 deposition sums.  One step = re-sort the
beam by slice, reset the plasma ahead of the box, compute every slice
(deposit, beam deposit, psi/Ez/Bz solves, predictor-corrector, beam push,
real plasma push).  Inputs are synthetic and resident on the GPU before the
timed region; the beam evolves from step to step as in a run.

Prints one JSON line: particle-slice updates/s (whole job), DST solves/s,
the per-kernel-class device time, the roofline of the real push (the fused
gather + push + deposit, the largest HBM stream; timed with HIP events on
the library's stream inside the timed region) and the time-dominant kernel
class, the FP64 CPU oracle on the first slices of the same box, and extra
legs: FP64 and the explicit Bx/By solver on the same step, the 512^2
blowout box (C2) and the 4-ppc box (C5) replayed from HIP graphs, the
FP32-against-FP64 accuracy, and the adjoint (forward+backward / forward).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
METRIC = "plasma particle-slice updates/s + DST solves/s; FP32 vs FP64; fwd+bwd/fwd ratio"
KCLASSES = ("push", "trial", "row_fwd", "col", "row_inv", "other")

# HBM bytes per real-push launch from the FETCH_SIZE / WRITE_SIZE counter
# runs (each scaled by what the counter reads for a plain 256 MiB copy),
# valid while the push kernel's sources (and the runtime, which picks its
# tiles) hash to the recorded value
PUSH_SOURCES = ["paper_2109_10277_amd/csrc/particles.hip",
                "paper_2109_10277_amd/csrc/push_tile.hpp",
                "paper_2109_10277_amd/csrc/shape.hpp",
                "paper_2109_10277_amd/csrc/runtime.cpp"]
PUSH_TRAFFIC = {
    "c2": {"sha256_prefix": "6f740fbb09b747c8", "bytes": 69.54e6,
           "summary": "profiles/kernel_stats_c2_blowout_512x512x1024_fp32.md"},
    "c5": {"sha256_prefix": "6f740fbb09b747c8", "bytes": 824.48e6,
           "summary": "profiles/kernel_stats_c5_forward_1024x1024_4ppc_fp32.md"},
    "c3": {"sha256_prefix": "6f740fbb09b747c8", "bytes": 260.88e6,
           "summary": "profiles/hbm_traffic_c3_paper_step_1024x1024x1024_fp32.md"},
}


def push_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def push_traffic(key: str):
    """Counter-measured bytes per launch, or None once the kernel changed."""
    t = PUSH_TRAFFIC.get(key)
    if not t or t["bytes"] is None or not t["sha256_prefix"]:
        return None
    return t["bytes"] if push_source_hash().startswith(t["sha256_prefix"]) else None


def workload(name: str):
    """(config, beam, workload label, traffic key)."""
    import workloads as W
    if name == "c3":
        cfg, beam = W.c3()
        return cfg, beam, "c3_paper_step_1024x1024x1024_1ppc_2x2^21_beam", "c3"
    if name == "c2":
        cfg, beam = W.c2()
        return cfg, beam, "c2_blowout_512x512x1024_1ppc", "c2"
    if name == "c1":
        cfg, beam = W.c1()
        return cfg, beam, "c1_linear_64x64x64_1ppc", "c1"
    if name == "c5fwd":
        cfg, beam = W.c5()
        return cfg, beam, "c5_forward_1024x1024x1024_4ppc", "c5"
    raise SystemExit(f"unknown workload {name}")


def push_bytes(cfg, fsize: int, n_beam: int = 0) -> int:
    """Algorithmic HBM bytes of one real push launch: every particle reads
    its state (x, y, ux, uy, Psi, w), the Adams-Bashforth history part P
    (5) and 3 history slots x 5 quantities, and writes 5 state + 5 history
    values and the next P (5); the six field planes are read once and the
    four FP64 deposit planes (rho - Jz, Jx, Jy, Jz) written once.
    A launch also carries the beam work of its slice: every beam particle
    is pushed once per box (6 FP32 values read and written) and deposited
    once (6 read), 72 B, spread over the nzeta - 1 real pushes."""
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    plane = cfg.nx * cfg.ny
    beam = n_beam * 72 // max(cfg.nzeta - 1, 1)
    return n_p * (26 + 15) * fsize + 6 * plane * fsize + 4 * plane * 8 + beam


def make_box(cfg, beam, precision, soa=None):
    from paper_2109_10277_amd import qsp
    box = qsp.Box(cfg, precision)
    if hasattr(beam, "amp"):
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    else:
        box.set_beam_particles(soa.clone(), beam.dt)
    return box


def run_gpu(cfg, beam, precision: str, steps: int, warmup: int, timing_every: int, soa=None):
    """Warm-up boxes, then `steps` timed boxes (each from the plasma reset;
    a macro-particle beam is re-sorted by slice at the reset and pushed in
    every slice).  Returns (box, seconds, per-box stats, kernel times)."""
    import torch
    box = make_box(cfg, beam, precision, soa)
    # the sampling period is set before the warm-up so that box graphs
    # captured there are the ones the timed boxes replay
    box.set_timing(timing_every)
    for _ in range(warmup):
        box.init_plasma()
        box.run_box()
    torch.cuda.synchronize()
    box.set_timing(timing_every)      # clears the warm-up's samples
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        box.init_plasma()
        stats.append(box.run_box())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = box.kernel_times()
    box.set_timing(0)
    return box, (t1 - t0), stats, kt


def graph_replayed(cfg, beam) -> bool:
    """Boxes are replayed from HIP graphs (QSP_GRAPH=0 launches eagerly);
    in a replay only the real push is timed with events."""
    return os.environ.get("QSP_GRAPH", "1") != "0"


def eager_breakdown(cfg, beam, precision: str, every: int, soa=None) -> dict:
    """Kernel classes of one box launched kernel by kernel (a graph replay
    times only the real push): device ms per box from the events of every
    `every`-th slice, scaled by `every`, and the eager box's own time."""
    import torch
    old = os.environ.get("QSP_GRAPH")
    os.environ["QSP_GRAPH"] = "0"
    try:
        box = make_box(cfg, beam, precision, soa)
    finally:
        if old is None:
            del os.environ["QSP_GRAPH"]
        else:
            os.environ["QSP_GRAPH"] = old
    box.set_timing(every)
    box.init_plasma()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    box.run_box()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = box.kernel_times()
    box.close()
    return {"kernel_ms_per_box": kernel_summary(kt, 1, every, False),
            "ms_per_box": (t1 - t0) * 1e3}


def kernel_summary(kt, steps: int, every: int, graphs: bool) -> dict:
    """Device ms per step by kernel class, scaled from the sampled slices;
    None for the classes a graph replay does not time."""
    out = {}
    for c in KCLASSES:
        ms, n = kt[c]
        if graphs and c != "push":
            out[c] = None
        else:
            out[c] = ms / steps * every if every else None
    return out


def standalone_solves(box, cfg, reps: int = 50) -> float:
    """Batched (3-field) Dirichlet solves per second through the C ABI."""
    import torch
    src = torch.randn(3, cfg.ny + 1, cfg.nx + 1, dtype=box.fdtype, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        box.solve_poisson(src, dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        box.solve_poisson(src, dst)
    torch.cuda.synchronize()
    return 3 * reps / (time.perf_counter() - t0)


def note(msg: str) -> None:
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def leg(cfg, beam, label, key, precision, steps, warmup, every, soa=None, solves=False,
        breakdown=False) -> dict:
    """One timed workload: throughput, kernel classes and the real push's
    event-timed roofline (breakdown: also the kernel classes of one eagerly
    launched box, after the timed boxes)."""
    note(f"{label} {precision}: {warmup} warm-up + {steps} timed boxes")
    graphs = graph_replayed(cfg, beam)
    box, dt, stats, kt = run_gpu(cfg, beam, precision, steps, warmup, every, soa)
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    fsize = 4 if precision == "fp32" else 8
    push_ms, push_n = kt["push"]
    avg = push_ms / push_n if push_n else float("nan")
    nbytes = push_bytes(cfg, fsize, 0 if soa is None else int(soa.shape[1]))
    achieved = nbytes / (avg * 1e-3) / 1e9
    out = {"workload": label, "precision": precision, "steps": steps,
           "value": n_p * cfg.nzeta * steps / dt, "ms_per_step": dt / steps * 1e3,
           "dst_solves_per_s": sum(s["dst_solves"] for s in stats) / dt,
           "pc_iterations_per_slice": sum(s["pc_iterations"] for s in stats) / (cfg.nzeta * steps),
           "n_clamped_per_step": sum(s["n_clamped"] for s in stats) / steps,
           "box_reruns": sum(s["box_reruns"] for s in stats),
           "graph_replay": graphs,
           "kernel_ms_per_step": kernel_summary(kt, steps, every, graphs),
           "push": {"achieved": achieved, "frac": achieved / HBM_PEAK_GBS,
                    "bytes_per_launch": nbytes, "avg_launch_ms": avg, "launches_timed": push_n,
                    "traffic": push_traffic(key) if precision == "fp32" else None}}
    if solves:
        out["dst_solves_per_s_standalone_batch3"] = standalone_solves(box, cfg)
    box.close()
    if breakdown and graphs and every:
        if soa is not None:   # the same beam as the timed boxes started from
            import torch
            soa = torch.tensor(beam.soa(), device="cuda")
        out["eager_box"] = eager_breakdown(cfg, beam, precision, every, soa)
    return out


ACC_FIELDS = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz", "rho_mjz", "jx", "jy", "jz")


def fp32_vs_fp64(cfg, beam, every: int = 8) -> dict:
    """Relative L2 difference of the FP32 box from the FP64 box, per field,
    over interior nodes of every `every`-th slice: over all those slices
    together and the largest and median per slice (slices where the FP64
    field is non-zero).  Bz is measured against the norm of (Bx, By), which
    it is second order small against for a round beam."""
    import torch
    from paper_2109_10277_amd import qsp
    note("FP32 against FP64 fields")
    stacks = {}
    n_stack = (cfg.nzeta + every - 1) // every
    for prec in ("fp64", "fp32"):
        with qsp.Box(cfg, prec) as box:
            box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
            box.init_plasma()
            st = {q: box.empty(q, n_stack) for q in ACC_FIELDS}
            box.run_box(stack=st, stack_every=every)
            torch.cuda.synchronize()
        stacks[prec] = st
    ref, got = stacks["fp64"], stacks["fp32"]

    def norms(t):   # per-slice L2 norm over interior nodes
        return torch.linalg.vector_norm(t[:, 1:-1, 1:-1].double(), dim=(1, 2))

    bperp = torch.sqrt(norms(ref["bx"]) ** 2 + norms(ref["by"]) ** 2)
    out = {}
    for q in ACC_FIELDS:
        d = norms(got[q].double() - ref[q])
        den = bperp if q == "bz" else norms(ref[q])
        ok = den > 0
        per = (d[ok] / den[ok]).cpu()
        box_rel = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(den))
        out[q] = {"box": box_rel, "max_slice": float(per.max()) if per.numel() else 0.0,
                  "median_slice": float(per.median()) if per.numel() else 0.0}
    del stacks, ref, got
    torch.cuda.empty_cache()
    return {"slices_compared": n_stack, "every": every, "rel_l2": out}


# one time step of the paper's single-GPU table (Sec. VI, A100): 1024^2 x 1024
# cells, 1 ppc, driver + witness macro-particle beams, seconds per step
PAPER_A100_STEP_S = {"fp32_pc": 12.9, "fp64_pc": 16.6, "fp32_explicit": 20.6,
                     "fp64_explicit": 23.8}


def c3_variants(cfg, beam, soa, steps: int) -> dict:
    """Seconds per time step of the paper-scale box in both precisions and
    with both Bx/By solvers (one untimed step first)."""
    import workloads as W
    out = {"step_s": {}, "updates_per_s": {}, "paper_a100_step_s": PAPER_A100_STEP_S}
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    for solver in ("pc", "explicit"):
        c = W.BoxConfig(**{f: getattr(cfg, f) for f in cfg.__dataclass_fields__})
        if solver == "explicit":
            c.bxby_solver, c.pc_max_iter, c.pc_tol = "explicit", 6, 1e-5
        for prec in ("fp32", "fp64"):
            note(f"paper-scale step {prec} {solver}")
            box, dt, _, _ = run_gpu(c, beam, prec, steps, 1, 0, soa)
            box.close()
            out["step_s"][f"{prec}_{solver}"] = dt / steps
            out["updates_per_s"][f"{prec}_{solver}"] = n_p * cfg.nzeta * steps / dt
    return out


def adjoint_leg(name: str, precision: str, ckpt_every: int, reps: int = 2,
                fp64_check: bool = False) -> dict:
    """Forward+backward / forward on the adjoint workloads.

    c4: 256 x 256 nodes, 512 slices, 1 plasma electron per cell, loss = mean
    on-axis Ez over slices 400..420, gradients over 512 amplitudes and the
    two beam sizes.  c5: 1024 x 1024 nodes, 2 x 2 electrons per cell (4.19M),
    loss = witness-weighted Ez integral over the slices the witness covers.
    Forward = the plain slice loop over the same slices; forward+backward =
    checkpointed record + reverse pass (with the per-chunk recompute).
    With fp64_check the gradient is also computed in FP64 and the FP32
    gradient's largest deviation reported relative to its largest entry."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp

    def weights(cfg, dtype):
        if name == "c4":
            k_lo, k_hi = W.C4_LOSS_SLICES
            n = k_hi + 1
            wts = torch.zeros(n - k_lo, cfg.ny + 1, cfg.nx + 1, dtype=dtype, device="cuda")
            wts[:, cfg.ny // 2, cfg.nx // 2] = 1.0 / (n - k_lo)
            return k_lo, n, wts
        k_lo, gz, gy, gx = W.witness_factors(cfg)
        n = k_lo + len(gz)
        dv = cfg.hx * cfg.hy * cfg.dzeta
        t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        wts = (t(gz * dv)[:, None, None] * t(gy)[None, :, None] * t(gx)[None, None, :]).to(dtype)
        return k_lo, n, wts

    cfg, beam = W.c4() if name == "c4" else W.c5()
    note(f"adjoint {name} {precision} K={ckpt_every}")
    box_dtype = torch.float32 if precision == "fp32" else torch.float64
    k_lo, n, wts = weights(cfg, box_dtype)
    box = qsp.Box(cfg, precision)
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    cot = {"ez": wts}
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y

    def forward():
        box.init_plasma()
        for _ in range(n):
            box.advance_slice()

    def fwd_bwd():
        box.init_plasma()
        box.record(n, ckpt_every)
        return box.adjoint(k_lo, cot)

    fwd_bwd()                                    # allocation + warm-up
    forward()
    torch.cuda.synchronize()
    t_f = t_r = t_a = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        box.init_plasma()
        box.record(n, ckpt_every)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ga, gs, loss = box.adjoint(k_lo, cot)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t_f, t_r, t_a = t_f + t1 - t0, t_r + t2 - t1, t_a + t3 - t2
    mem = box.stats()["device_bytes"]
    box.close()
    out = {"workload": f"{name}_{cfg.nx}x{cfg.ny}_{n}slices_{n_p}particles",
           "precision": precision, "ckpt_every": ckpt_every,
           "fwd_ms": t_f / reps * 1e3, "record_ms": t_r / reps * 1e3,
           "reverse_ms": t_a / reps * 1e3,
           "fwd_bwd_over_fwd": (t_r + t_a) / t_f,
           "fwd_bwd_updates_per_s": n_p * n / ((t_r + t_a) / reps),
           "device_bytes": mem, "loss": float(loss.cpu()[0]),
           "grad_sigma": gs.cpu().tolist()}
    if fp64_check and precision == "fp32":
        _, _, w64 = weights(cfg, torch.float64)
        with qsp.Box(cfg, "fp64") as b64:
            b64.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
            b64.init_plasma()
            b64.record(n, ckpt_every)
            g64, s64, l64 = b64.adjoint(k_lo, {"ez": w64})
            torch.cuda.synchronize()
        g32, g64 = ga.cpu().numpy(), g64.cpu().numpy()
        out["fp32_vs_fp64_grad"] = {
            "amp_max_rel": float(np.abs(g32 - g64).max() / np.abs(g64).max()),
            "sigma_rel": (np.abs(gs.cpu().numpy() - s64.cpu().numpy()) /
                          np.abs(s64.cpu().numpy())).tolist(),
            "loss_rel": abs(out["loss"] - float(l64.cpu()[0])) / abs(float(l64.cpu()[0]))}
    return out


def emittance_study(nsteps: int, solver: str = "pc") -> dict:
    """FP32 versus FP64 drift of the witness emittance over nsteps time steps
    on a reduced reference setup (256^2 x 256 slices, driver + witness
    macro-particle beams, witness with zero initial emittance and a
    transverse centroid offset of one sigma_x), with the predictor-corrector
    or the explicit Bx/By solver (the two solvers of Fig. 7).  Each time
    step runs the box with a fresh plasma while the beams advance by dt = 6
    in every slice.  A progress line goes to stderr every 50 steps."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp
    cfg, beam = W.emittance_study()
    cfg.bxby_solver = solver
    w_wit = float(beam.w[-1])
    every = max(1, nsteps // 30)
    out = {}
    for prec in ("fp32", "fp64"):
        box = qsp.Box(cfg, prec)
        box.set_beam_particles(torch.tensor(beam.soa(), device="cuda"), beam.dt)
        series = []
        t0 = time.perf_counter()
        for step in range(nsteps + 1):
            if step % every == 0 or step == nsteps:
                b = box.get_beam_particles().double()
                m = torch.isclose(b[6], torch.tensor(w_wit, dtype=torch.float64, device=b.device))
                x, ux = b[0][m], b[3][m]
                x, ux = x - x.mean(), ux - ux.mean()
                emit = torch.sqrt(torch.clamp((x * x).mean() * (ux * ux).mean() - (x * ux).mean() ** 2,
                                              min=0.0))
                series.append((step, float(emit), float(b[0][m].mean()), int(m.sum())))
            if step % 50 == 0:
                print(f"emittance study {prec}: step {step}/{nsteps}, "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
            if step < nsteps:
                box.init_plasma()
                box.run_box()
        torch.cuda.synchronize()
        out[prec] = {"seconds": time.perf_counter() - t0, "series": series}
        box.close()
    e32 = np.array([s[1] for s in out["fp32"]["series"]])
    e64 = np.array([s[1] for s in out["fp64"]["series"]])
    rel = np.abs(e32 - e64) / np.maximum(e64, 1e-300)
    return {"study": "witness emittance, FP32 vs FP64", "bxby_solver": solver, "steps": nsteps, "dt": beam.dt,
            "config": {"nx": cfg.nx, "ny": cfg.ny, "slices": cfg.nzeta,
                       "beam_particles": int(beam.x.size)},
            "steps_sampled": [s[0] for s in out["fp64"]["series"]],
            "emittance_fp64": e64.tolist(), "emittance_fp32": e32.tolist(),
            "rel_error_fp32_final": float(rel[-1]), "rel_error_fp32_max_after_first": float(rel[1:].max()),
            "centroid_x_fp64": [s[2] for s in out["fp64"]["series"]],
            "witness_particles_fp64": [s[3] for s in out["fp64"]["series"]],
            "witness_particles_fp32": [s[3] for s in out["fp32"]["series"]],
            "seconds": {p: out[p]["seconds"] for p in out}}


def solve_bench(reps: int = 200) -> dict:
    """Standalone batched Dirichlet solves (row pass, column pass, inverse
    row pass, with the node conversions) at 512^2 and 1024^2, batches of 2
    and 3 FP32 planes: microseconds per batched solve."""
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp
    out = {}
    for n in (512, 1024):
        for nb in (2, 3):
            cfg = W.BoxConfig(nx=n, ny=n, x_lo=-8.0, x_hi=8.0, y_lo=-8.0, y_hi=8.0, nzeta=2,
                              zeta_hi=0.0, dzeta=0.1)
            with qsp.Box(cfg, "fp32") as box:
                src = torch.randn(nb, n + 1, n + 1, dtype=torch.float32, device="cuda")
                dst = torch.empty_like(src)
                for _ in range(5):
                    box.solve_poisson(src, dst, 1.3)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    box.solve_poisson(src, dst, 1.3)
                torch.cuda.synchronize()
                out[f"{n}x{n}_batch{nb}"] = (time.perf_counter() - t0) / reps * 1e6
    return {"us_per_batched_solve": out, "reps": reps}


def cpu_baseline(cfg, beam, n_slices: int) -> dict:
    """The FP64 oracle on the host cores: the first n_slices slices of the
    same box, from the unperturbed plasma (a macro-particle beam is
    deposited and pushed in its slices as on the GPU)."""
    import workloads as W
    from oracle import qsp_oracle as O
    note(f"oracle on the first {n_slices} slices")
    b = W.copy_beam(beam) if hasattr(beam, "zeta") else beam
    st = O.initial_state(cfg)
    c0, w0 = time.process_time(), time.perf_counter()
    _, st = O.run_box(cfg, b, keep=lambda k, r: None, state=st, k_end=n_slices)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    return {"value": n_p * n_slices / wall, "unit": "particle-slice updates/s",
            "cores": max(1, round(cpu / wall)), "kind": "oracle",
            "sample": f"first {n_slices} of {cfg.nzeta} slices of the same box "
                      f"({n_p} plasma particles), FP64 NumPy/SciPy, {wall:.1f} s wall, "
                      f"{len(os.sched_getaffinity(0))} host cores visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=("c3", "c2", "c1", "c5fwd"))
    ap.add_argument("--timing-every", type=int, default=4,
                    help="time the kernels of every n-th slice with HIP events")
    ap.add_argument("--cpu-slices", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (for profiler runs)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-against-FP64 field comparison (C2)")
    ap.add_argument("--shape-order", type=int, default=1, choices=(0, 1, 2, 3),
                    help="transverse particle shape of the timed workload (1: linear)")
    ap.add_argument("--solver", default="pc", choices=("pc", "explicit"),
                    help="Bx/By field solver: predictor-corrector or explicit "
                         "(conjugate gradients to a relative residual of 1e-5, at most 6)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference kernel for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--solve-bench", action="store_true",
                    help="time standalone batched solves at 512^2 and 1024^2 and exit")
    ap.add_argument("--emittance-study", type=int, default=0, metavar="STEPS",
                    help="only run the FP32-vs-FP64 witness emittance study for STEPS time steps")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint legs and print their JSON")
    ap.add_argument("--adjoint-c5", default="",
                    help="comma-separated checkpoint intervals for the c5 adjoint leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the slice loop of one box runs on a "
              "single GPU and is not split across GPUs; rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return
    if args.solve_bench:
        print(json.dumps(solve_bench()))
        return
    if args.emittance_study:
        print(json.dumps(emittance_study(args.emittance_study, args.solver)))
        return
    if args.adjoint_only:
        legs = [] if args.no_adjoint else [adjoint_leg("c4", "fp32", 32, fp64_check=True)]
        legs += [adjoint_leg("c5", "fp32", int(K), reps=1)
                 for K in filter(None, args.adjoint_c5.split(","))]
        print(json.dumps({"adjoint": legs}))
        return

    cfg, beam, wname, key = workload(args.workload)
    if args.shape_order != 1:
        cfg.shape_order = args.shape_order
        wname += f"_order{args.shape_order}"
    if args.solver == "explicit":
        cfg.bxby_solver = "explicit"
        cfg.pc_max_iter, cfg.pc_tol = 6, 1e-5
        wname += "_explicit"
        key = ""
    soa = None if hasattr(beam, "amp") else torch.tensor(beam.soa(), device="cuda")
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    head = leg(cfg, beam, wname, key, "fp32", args.steps, args.warmup, args.timing_every, soa,
               solves=True, breakdown=True)
    kms = head["kernel_ms_per_step"]
    eb = head.get("eager_box")
    timed = {c: v for c, v in (eb["kernel_ms_per_box"] if eb else kms).items() if v is not None}
    dominant = max(timed, key=timed.get) if timed else None
    p = head["push"]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "particle-slice updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "nx": cfg.nx, "ny": cfg.ny,
                   "slices": cfg.nzeta, "particles": n_p,
                   "beam_particles": None if soa is None else int(soa.shape[1]),
                   "bxby_iterations": f"<= {cfg.pc_max_iter}, tol {cfg.pc_tol}",
                   "shape_order": cfg.shape_order, "bxby_solver": cfg.bxby_solver,
                   "deposit_sums": "f64"},
        "dst_solves_per_s": head["dst_solves_per_s"],
        "dst_solves_per_s_standalone_batch3": head["dst_solves_per_s_standalone_batch3"],
        "pc_iterations_per_slice": head["pc_iterations_per_slice"],
        "graph_replay": head["graph_replay"],
        "kernel_ms_per_step": kms,
        "kernel_ms_per_step_eager_box": None if eb is None else eb["kernel_ms_per_box"],
        "eager_box_ms": None if eb is None else eb["ms_per_box"],
        "kernel_timing": (f"device time of the launches of every {args.timing_every}-th slice "
                          f"(HIP events on the library stream), scaled by {args.timing_every}; "
                          "null: not timed (HIP graph replay times only the real push); "
                          "kernel_ms_per_step_eager_box: every class, from one more box of the "
                          "same workload launched kernel by kernel after the timed boxes"),
        "time_dominant_kernel_class": None if dominant is None else {
            "class": dominant, "ms_per_step": timed[dominant],
            "share_of_step": timed[dominant] / (eb["ms_per_box"] if eb else head["ms_per_step"]),
            "from": "eager box" if eb else "timed boxes"},
        "roofline": {"bound": "hbm",
                     "kernel": "k_push real (gather + AB5 push + deposit, with the slice's beam work)",
                     "achieved": p["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": p["frac"], "traffic": p["traffic"],
                     "bytes_per_launch": p["bytes_per_launch"],
                     "avg_launch_ms": p["avg_launch_ms"], "launches_timed": p["launches_timed"]},
        "fwd_bwd_over_fwd": None, "adjoint": None,
    }
    if not args.no_extras:
        extras = {}
        if args.workload == "c3" and args.solver == "pc" and not args.no_fp64:
            extras["c3_variants"] = c3_variants(cfg, beam, soa, 2)
            out["fp64_value"] = extras["c3_variants"]["updates_per_s"]["fp64_pc"]
            out["fp32_over_fp64"] = (extras["c3_variants"]["step_s"]["fp64_pc"] /
                                     extras["c3_variants"]["step_s"]["fp32_pc"])
        for wl in ("c2", "c5fwd"):
            if wl == args.workload:
                continue
            c2cfg, c2beam, c2name, c2key = workload(wl)
            extras[wl] = leg(c2cfg, c2beam, c2name, c2key, "fp32", 3 if wl == "c2" else 1, 1,
                             args.timing_every)
            if wl == "c2" and not args.no_fp64:
                extras["c2_fp64"] = leg(c2cfg, c2beam, c2name, "", "fp64", 2, 1, 0)
        if not args.no_accuracy:
            c2cfg, c2beam, _, _ = workload("c2")
            extras["c2_fp32_vs_fp64"] = fp32_vs_fp64(c2cfg, c2beam)
        out["extras"] = extras
        if not args.no_adjoint:
            adj = adjoint_leg("c4", "fp32", 32, fp64_check=True)
            out["fwd_bwd_over_fwd"] = adj["fwd_bwd_over_fwd"]
            out["adjoint"] = [adj]
            for K in filter(None, args.adjoint_c5.split(",")):
                out["adjoint"].append(adjoint_leg("c5", "fp32", int(K), reps=1))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, beam, args.cpu_slices)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
