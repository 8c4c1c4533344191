#!/usr/bin/env python3
"""Benchmark of the quasi-static PIC slice loop on one MI355X.

One step = one full box of the per-slice loop (plasma reset to the lattice,
then every slice: deposit, beam source, psi/Ez/Bz solves, Bx/By
predictor-corrector, real push) on the blowout workload: 512 x 512 nodes
over [-6, 6]^2, 1024 slices over 10 k_p^-1, 1 plasma electron per cell
(262,144 particles), rigid Gaussian driver n_b/n0 = 10, sigma_r = 0.3,
sigma_z = 1.41, predictor-corrector to 1e-4 (at most 5 iterations), FP32
with FP64 deposition sums.  Inputs are synthetic and resident on the GPU
before the timed region.

Prints one JSON line: particle-slice updates/s (whole job), DST solves/s,
the FP64 rate and FP32/FP64 ratio, the roofline of the dominant kernel (the
fused gather + push + deposit, timed with HIP events on the library's stream
inside the timed region) and the FP64 CPU oracle timed on a bounded sample
of the same workload.
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

# HBM bytes per real-push launch at c2 FP32 from the FETCH_SIZE / WRITE_SIZE
# counter runs (scaled by a 256 MiB copy), valid while the push kernel's
# sources hash to this value
PUSH_TRAFFIC = {"sources": ["paper_2109_10277_amd/csrc/particles.hip",
                            "paper_2109_10277_amd/csrc/push_tile.hpp",
                            "paper_2109_10277_amd/csrc/shape.hpp"],
                "sha256_prefix": "5d1424f6cf536825", "workload": "c2", "bytes": 64.24e6,
                "summary": "profiles/hbm_traffic_c2_blowout_512x512x1024_fp32.md"}


def push_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in PUSH_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def push_traffic(workload_name: str):
    """Counter-measured bytes per launch, or None once the kernel changed."""
    if PUSH_TRAFFIC["bytes"] is None or not PUSH_TRAFFIC["sha256_prefix"]:
        return None
    if not workload_name.startswith(PUSH_TRAFFIC["workload"] + "_"):
        return None
    return PUSH_TRAFFIC["bytes"] if push_source_hash().startswith(PUSH_TRAFFIC["sha256_prefix"]) else None


def workload(name: str):
    import workloads as W
    if name == "c2":
        cfg, beam = W.c2()
        return cfg, beam, "c2_blowout_512x512x1024_1ppc"
    if name == "c1":
        cfg, beam = W.c1()
        return cfg, beam, "c1_linear_64x64x64_1ppc"
    if name == "c5fwd":
        cfg, beam = W.c5()
        return cfg, beam, "c5_forward_1024x1024x1024_4ppc"
    raise SystemExit(f"unknown workload {name}")


def push_bytes(cfg, fsize: int) -> int:
    """Algorithmic HBM bytes of one real push launch: every particle reads
    its state (x, y, ux, uy, Psi, w) and 4 history slots x 5 quantities and
    writes 5 state + 5 history values; the six field planes are read once
    and the four FP64 deposit planes (rho - Jz, Jx, Jy, Jz) written once."""
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    plane = cfg.nx * cfg.ny
    return n_p * (26 + 10) * fsize + 6 * plane * fsize + 4 * plane * 8


def run_gpu(cfg, beam, precision: str, steps: int, warmup: int, timing_every: int):
    import torch
    from paper_2109_10277_amd import qsp
    box = qsp.Box(cfg, precision)
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    # the sampling period is set before the warm-up so that the box graphs
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


ACC_FIELDS = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz", "rho_mjz", "jx", "jy", "jz")


def fp32_vs_fp64(cfg, beam, every: int = 8) -> dict:
    """Relative L2 difference of the FP32 box from the FP64 box, per field,
    over interior nodes of every `every`-th slice: over all those slices
    together and the largest and median per slice (slices where the FP64
    field is non-zero).  Bz is measured against the norm of (Bx, By), which
    it is second order small against for a round beam."""
    import torch
    from paper_2109_10277_amd import qsp
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


def c3_leg() -> dict:
    """Wall time of one full time step of the paper-scale box (1024^2 x 1024,
    1 ppc, 2 x 2^21 beam macro-particles pushed in every slice), from the
    beam sort to the last slice, for both precisions and both Bx/By solvers.
    One untimed step first."""
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp
    cfg, beam = W.c3()
    soa = torch.tensor(beam.soa(), device="cuda")
    out = {"workload": "c3_paper_step_1024x1024x1024_1ppc_2x2^21_beam", "step_s": {},
           "updates_per_s": {}, "paper_a100_step_s": PAPER_A100_STEP_S}
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    for solver in ("pc", "explicit"):
        c = W.BoxConfig(**{f: getattr(cfg, f) for f in cfg.__dataclass_fields__})
        if solver == "explicit":
            c.bxby_solver, c.pc_max_iter, c.pc_tol = "explicit", 6, 1e-5
        for prec in ("fp32", "fp64"):
            box = qsp.Box(c, prec)
            box.set_beam_particles(soa.clone(), beam.dt)
            box.init_plasma()
            box.run_box()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            box.init_plasma()
            box.run_box()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            box.close()
            out["step_s"][f"{prec}_{solver}"] = dt
            out["updates_per_s"][f"{prec}_{solver}"] = n_p * cfg.nzeta / dt
    return out


def adjoint_leg(name: str, precision: str, ckpt_every: int, reps: int = 2) -> dict:
    """Forward+backward / forward on the adjoint workloads.

    c4: 256 x 256 nodes, 512 slices, 1 plasma electron per cell, loss = mean
    on-axis Ez over slices 400..420, gradients over 512 amplitudes and the
    two beam sizes.  c5: 1024 x 1024 nodes, 2 x 2 electrons per cell (4.19M),
    loss = witness-weighted Ez integral over the slices the witness covers.
    Forward = the plain slice loop over the same slices; forward+backward =
    checkpointed record + reverse pass (with the per-chunk recompute)."""
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp
    box_dtype = torch.float32 if precision == "fp32" else torch.float64
    if name == "c4":
        cfg, beam = W.c4()
        k_lo, k_hi = W.C4_LOSS_SLICES
        n = k_hi + 1
        wts = torch.zeros(n - k_lo, cfg.ny + 1, cfg.nx + 1, dtype=box_dtype, device="cuda")
        wts[:, cfg.ny // 2, cfg.nx // 2] = 1.0 / (n - k_lo)
    else:
        cfg, beam = W.c5()
        k_lo, gz, gy, gx = W.witness_factors(cfg)
        n = k_lo + len(gz)
        dv = cfg.hx * cfg.hy * cfg.dzeta
        t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        wts = (t(gz * dv)[:, None, None] * t(gy)[None, :, None] * t(gx)[None, None, :]).to(box_dtype)
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
    return {"workload": f"{name}_{cfg.nx}x{cfg.ny}_{n}slices_{n_p}particles",
            "precision": precision, "ckpt_every": ckpt_every,
            "fwd_ms": t_f / reps * 1e3, "record_ms": t_r / reps * 1e3,
            "reverse_ms": t_a / reps * 1e3,
            "fwd_bwd_over_fwd": (t_r + t_a) / t_f,
            "fwd_bwd_updates_per_s": n_p * n / ((t_r + t_a) / reps),
            "device_bytes": mem, "loss": float(loss.cpu()[0]),
            "grad_sigma": gs.cpu().tolist()}


def emittance_study(nsteps: int) -> dict:
    """FP32 versus FP64 drift of the witness emittance over nsteps time steps
    on a reduced reference setup (256^2 x 256 slices, driver + witness
    macro-particle beams, witness with zero initial emittance and a
    transverse centroid offset of one sigma_x).  Each time step runs the box
    with a fresh plasma while the beams advance by dt = 6 in every slice."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2109_10277_amd import qsp
    cfg, beam = W.emittance_study()
    w_wit = float(beam.w[-1])
    every = max(1, nsteps // 20)
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
                series.append((step, float(emit), float(b[0][m].mean())))
            if step < nsteps:
                box.init_plasma()
                box.run_box()
        torch.cuda.synchronize()
        out[prec] = {"seconds": time.perf_counter() - t0, "series": series}
        box.close()
    e32 = np.array([s[1] for s in out["fp32"]["series"]])
    e64 = np.array([s[1] for s in out["fp64"]["series"]])
    rel = np.abs(e32 - e64) / np.maximum(e64, 1e-300)
    return {"study": "witness emittance, FP32 vs FP64", "steps": nsteps, "dt": beam.dt,
            "config": {"nx": cfg.nx, "ny": cfg.ny, "slices": cfg.nzeta,
                       "beam_particles": int(beam.x.size)},
            "steps_sampled": [s[0] for s in out["fp64"]["series"]],
            "emittance_fp64": e64.tolist(), "emittance_fp32": e32.tolist(),
            "rel_error_fp32_final": float(rel[-1]), "rel_error_fp32_max_after_first": float(rel[1:].max()),
            "centroid_x_fp64": [s[2] for s in out["fp64"]["series"]],
            "seconds": {p: out[p]["seconds"] for p in out}}


def cpu_baseline(cfg, beam, n_slices: int) -> dict:
    """The FP64 oracle on the host cores: the first n_slices slices of the
    same box, from the unperturbed plasma."""
    from oracle import qsp_oracle as O
    st = O.initial_state(cfg)
    c0, w0 = time.process_time(), time.perf_counter()
    for _ in range(n_slices):
        st, _ = O.advance_slice(cfg, st, beam)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    return {"value": n_p * n_slices / wall, "unit": "particle-slice updates/s",
            "cores": max(1, round(cpu / wall)), "kind": "oracle",
            "sample": f"first {n_slices} of {cfg.nzeta} slices of the same box "
                      f"({n_p} particles), FP64 NumPy/SciPy, {wall:.1f} s wall, "
                      f"{len(os.sched_getaffinity(0))} host cores visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--timing-every", type=int, default=4,
                    help="time the kernels of every n-th slice with HIP events")
    ap.add_argument("--cpu-slices", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-against-FP64 field comparison of the timed box")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the paper-scale time step (1024^2 x 1024 with beams)")
    ap.add_argument("--shape-order", type=int, default=1, choices=(0, 1, 2, 3),
                    help="transverse particle shape of the timed workload (1: linear)")
    ap.add_argument("--solver", default="pc", choices=("pc", "explicit"),
                    help="Bx/By field solver: predictor-corrector or explicit "
                         "(conjugate gradients to a relative residual of 1e-5, at most 6)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference kernel for the FETCH_SIZE/WRITE_SIZE counters)")
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

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return
    if args.emittance_study:
        print(json.dumps(emittance_study(args.emittance_study)))
        return
    if args.adjoint_only:
        legs = [] if args.no_adjoint else [adjoint_leg("c4", "fp32", 32)]
        legs += [adjoint_leg("c5", "fp32", int(K), reps=1)
                 for K in filter(None, args.adjoint_c5.split(","))]
        print(json.dumps({"adjoint": legs}))
        return
    cfg, beam, wname = workload(args.workload)
    if args.shape_order != 1:
        cfg.shape_order = args.shape_order
        wname += f"_order{args.shape_order}"
    if args.solver == "explicit":
        cfg.bxby_solver = "explicit"
        cfg.pc_max_iter, cfg.pc_tol = 6, 1e-5
        wname += "_explicit"
    n_p = cfg.nx * cfg.ppc_x * cfg.ny * cfg.ppc_y
    box, dt, stats, kt = run_gpu(cfg, beam, "fp32", args.steps, args.warmup,
                                 args.timing_every)
    updates = n_p * cfg.nzeta * args.steps
    value = updates / dt
    solves = sum(s["dst_solves"] for s in stats)
    dst_ms = sum(kt[c][0] for c in ("row_fwd", "col", "row_inv"))
    push_ms, push_n = kt["push"]
    push_avg_ms = push_ms / max(push_n, 1) if push_n else float("nan")
    bytes_launch = push_bytes(cfg, 4)
    achieved = bytes_launch / (push_avg_ms * 1e-3) / 1e9
    standalone = standalone_solves(box, cfg)
    box.close()

    out = {
        "metric": METRIC, "value": value, "unit": "particle-slice updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "nx": cfg.nx, "ny": cfg.ny,
                   "slices": cfg.nzeta, "particles": n_p,
                   "bxby_iterations": f"<= {cfg.pc_max_iter}, tol {cfg.pc_tol}",
                   "shape_order": cfg.shape_order, "bxby_solver": cfg.bxby_solver,
                   "deposit_sums": "f64"},
        "dst_solves_per_s": solves / dt,
        "dst_solves_per_s_standalone_batch3": standalone,
        "pc_iterations_per_slice": sum(s["pc_iterations"] for s in stats) / (cfg.nzeta * args.steps),
        "kernel_ms_per_step": {c: kt[c][0] / args.steps * args.timing_every for c in kt},
        "fwd_bwd_over_fwd": None,
        "adjoint": None,
        "roofline": {"bound": "hbm", "kernel": "gather+push+deposit (real push)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": push_traffic(wname),
                     "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": push_avg_ms, "launches_timed": push_n},
    }
    if not args.no_fp64:
        box64, dt64, _, _ = run_gpu(cfg, beam, "fp64", max(1, args.steps // 2), 1, 0)
        box64.close()
        v64 = n_p * cfg.nzeta * max(1, args.steps // 2) / dt64
        out["fp64_value"] = v64
        out["fp32_over_fp64"] = value / v64
        if not args.no_accuracy:
            out["fp32_vs_fp64"] = fp32_vs_fp64(cfg, beam)
    if not args.no_adjoint:
        adj = adjoint_leg("c4", "fp32", 32)
        out["fwd_bwd_over_fwd"] = adj["fwd_bwd_over_fwd"]
        out["adjoint"] = [adj]
        for K in filter(None, args.adjoint_c5.split(",")):
            out["adjoint"].append(adjoint_leg("c5", "fp32", int(K), reps=1))
    if not args.no_c3:
        out["c3_paper_step"] = c3_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, beam, args.cpu_slices)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
