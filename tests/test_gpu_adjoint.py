"""GPU adjoint of the slice loop (checkpointed record + reverse pass through
the C ABI) against the FP64 oracle adjoint and against central differences
of the GPU's own FP64 forward pass.

Bars: FP64 gradients agree with the oracle's to 1e-9 of the largest
component (round-off of two FP64 evaluations of the same sums in another
order); FP32 gradients to 1e-3.  The predictor-corrector runs a fixed number
of iterations so that the loss is a smooth function of the parameters."""
import numpy as np
import pytest

import workloads as W
from oracle import qsp_adjoint as A

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Q():
    from paper_2109_10277_amd import qsp
    return qsp


FIELDS = A.FIELD_KEYS   # psi, exmby, eypbx, ez, bx, by, bz


def rect_case():
    cfg = W.BoxConfig(nx=64, ny=32, x_lo=-5.0, x_hi=5.0, y_lo=-3.0, y_hi=3.0,
                      nzeta=12, zeta_hi=0.0, dzeta=4.0 / 12, ppc_x=1, ppc_y=2,
                      pc_max_iter=2, pc_tol=0.0)
    beam = W.GaussianBeam(W.gaussian_envelope(cfg, 0.9, -1.0, 0.7), 0.7, 0.5)
    return cfg, beam


def wide_case():
    """256 x 32 lattice sites (128 x 32 cells, 2 x 1 per cell): four push
    tiles across x, so the reverse pass's tile transposes meet tile edges
    and their halo flush in x, with a driver strong enough to move the
    plasma across them."""
    cfg = W.BoxConfig(nx=128, ny=32, x_lo=-6.0, x_hi=6.0, y_lo=-3.0, y_hi=3.0,
                      nzeta=12, zeta_hi=0.0, dzeta=4.0 / 12, ppc_x=2, ppc_y=1,
                      pc_max_iter=2, pc_tol=0.0)
    beam = W.GaussianBeam(W.gaussian_envelope(cfg, 1.5, -1.0, 0.7), 0.6, 0.5)
    return cfg, beam


CASES = {
    "wide128x32_ppc2x1": wide_case,
    "n32_ppc1": lambda: W.small(n=32, nzeta=14, ppc=1, nb=0.9, sigma=0.8, pc_max_iter=3,
                                pc_tol=0.0, extent=5.0),
    "n16_ppc2": lambda: W.small(n=16, nzeta=12, ppc=2, nb=1.5, sigma=0.9, pc_max_iter=2,
                                pc_tol=0.0, extent=4.0),
    "rect64x32": rect_case,
}


def cotangents(cfg, k_lo, k_hi, seed=5):
    """Seeded weights on a patch around the axis for every field."""
    rng = np.random.default_rng(seed)
    cx, cy = cfg.nx // 2, cfg.ny // 2
    w = np.zeros((k_hi - k_lo + 1, len(FIELDS), cfg.ny + 1, cfg.nx + 1))
    w[:, :, cy - 3:cy + 4, cx - 3:cx + 4] = rng.normal(size=(k_hi - k_lo + 1, len(FIELDS), 7, 7))
    w[:, :, 0, :] = w[:, :, -1, :] = 0.0
    w[:, :, :, 0] = w[:, :, :, -1] = 0.0
    return w


def oracle_grad(cfg, beam, k_lo, w):
    recs, tape = A.forward_with_tape(cfg, beam)
    k_hi = k_lo + w.shape[0] - 1

    def cot(k):
        if k < k_lo or k > k_hi:
            return {}
        return {q: w[k - k_lo, i] for i, q in enumerate(FIELDS)}
    ga, gsx, gsy = A.adjoint_box(cfg, beam, tape, cot)
    return ga, np.array([gsx, gsy]), A.loss_value(recs, cot)


def gpu_grad(box, cfg, beam, n_slices, k_lo, w, ckpt_every):
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    box.init_plasma()
    box.record(n_slices, ckpt_every)
    cot = {q: torch.tensor(w[:, i], dtype=box.fdtype, device="cuda") for i, q in enumerate(FIELDS)}
    ga, gs, loss = box.adjoint(k_lo, cot)
    torch.cuda.synchronize()
    return ga.cpu().numpy(), gs.cpu().numpy(), float(loss.cpu()[0])


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
def test_adjoint_matches_oracle(case, prec, tol):
    cfg, beam = CASES[case]()
    k_lo, k_hi = cfg.nzeta // 2, cfg.nzeta - 2
    w = cotangents(cfg, k_lo, k_hi)
    ga_o, gs_o, L_o = oracle_grad(cfg, beam, k_lo, w)
    print(f"adjoint {case} {prec}", flush=True)
    with Q().Box(cfg, prec) as box:
        ga, gs, L = gpu_grad(box, cfg, beam, k_hi + 1, k_lo, w, ckpt_every=4)
    scale = np.abs(ga_o).max()
    assert scale > 0
    err = np.abs(ga - ga_o).max() / scale
    assert err <= tol, (err, ga, ga_o)
    assert np.all(np.abs(gs - gs_o) <= tol * np.abs(gs_o)), (gs, gs_o)
    assert abs(L - L_o) <= tol * max(abs(L_o), 1e-30) + 1e-12, (L, L_o)
    # slices behind the last loss slice never influence it
    assert np.all(ga[k_hi + 1:] == 0.0)


@pytest.mark.parametrize("ckpt_every", [1, 3, 5, 64])
def test_checkpoint_interval_does_not_change_the_gradient(ckpt_every):
    cfg, beam = CASES["n32_ppc1"]()
    k_lo, k_hi = 4, cfg.nzeta - 1
    w = cotangents(cfg, k_lo, k_hi, seed=9)
    print(f"adjoint ckpt {ckpt_every}", flush=True)
    with Q().Box(cfg, "fp64") as box:
        ref = gpu_grad(box, cfg, beam, k_hi + 1, k_lo, w, ckpt_every=k_hi + 1)
        got = gpu_grad(box, cfg, beam, k_hi + 1, k_lo, w, ckpt_every=ckpt_every)
    scale = np.abs(ref[0]).max()
    assert np.abs(got[0] - ref[0]).max() <= 1e-11 * scale
    assert np.all(np.abs(got[1] - ref[1]) <= 1e-11 * np.abs(ref[1]))


def test_adjoint_causality_on_a_full_record():
    # record the whole box, loss only up to slice 7: later amplitudes get
    # exactly zero gradient, earlier ones do not
    cfg, beam = CASES["n32_ppc1"]()
    k_lo, k_hi = 3, 7
    w = np.zeros((cfg.nzeta - k_lo, len(FIELDS), cfg.ny + 1, cfg.nx + 1))
    w[: k_hi - k_lo + 1] = cotangents(cfg, k_lo, k_hi, seed=3)
    print("adjoint causality", flush=True)
    with Q().Box(cfg, "fp64") as box:
        ga, _, _ = gpu_grad(box, cfg, beam, cfg.nzeta, k_lo, w, ckpt_every=4)
    assert np.all(ga[k_hi + 1:] == 0.0)
    assert np.all(ga[: k_hi + 1] != 0.0)


def gpu_loss(box, cfg, amp, sx, sy, n_slices, k_lo, w):
    box.set_beam_gaussian(amp, sx, sy)
    box.init_plasma()
    stack = {q: box.empty(q, n_slices) for q in FIELDS}
    box.record(n_slices, n_slices, stack=stack)
    torch.cuda.synchronize()
    return sum(float(np.sum(w[:, i] * stack[q][k_lo:].cpu().numpy()))
               for i, q in enumerate(FIELDS))


def test_adjoint_matches_central_differences_fp64():
    cfg, beam = CASES["n16_ppc2"]()
    k_lo, k_hi = 5, cfg.nzeta - 1
    w = cotangents(cfg, k_lo, k_hi, seed=21)
    n = k_hi + 1
    print("adjoint central differences", flush=True)
    with Q().Box(cfg, "fp64") as box:
        ga, gs, L = gpu_grad(box, cfg, beam, n, k_lo, w, ckpt_every=4)
        L0 = gpu_loss(box, cfg, beam.amp, beam.sigma_x, beam.sigma_y, n, k_lo, w)
        assert abs(L - L0) <= 1e-10 * abs(L0)
        for k in (0, 3, 6, 9):
            h = 1e-5 * max(abs(beam.amp[k]), 1e-2)
            ap, am = beam.amp.copy(), beam.amp.copy()
            ap[k] += h
            am[k] -= h
            fd = (gpu_loss(box, cfg, ap, beam.sigma_x, beam.sigma_y, n, k_lo, w) -
                  gpu_loss(box, cfg, am, beam.sigma_x, beam.sigma_y, n, k_lo, w)) / (2 * h)
            assert abs(ga[k] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(ga).max()), (k, ga[k], fd)
        h = 1e-5
        fd = (gpu_loss(box, cfg, beam.amp, beam.sigma_x + h, beam.sigma_y, n, k_lo, w) -
              gpu_loss(box, cfg, beam.amp, beam.sigma_x - h, beam.sigma_y, n, k_lo, w)) / (2 * h)
        assert abs(gs[0] - fd) <= 1e-5 * abs(fd), (gs[0], fd)
        fd = (gpu_loss(box, cfg, beam.amp, beam.sigma_x, beam.sigma_y + h, n, k_lo, w) -
              gpu_loss(box, cfg, beam.amp, beam.sigma_x, beam.sigma_y - h, n, k_lo, w)) / (2 * h)
        assert abs(gs[1] - fd) <= 1e-5 * abs(fd), (gs[1], fd)


def test_autograd_function_backward():
    cfg, beam = CASES["n32_ppc1"]()
    k_lo = 6
    n = cfg.nzeta
    w = cotangents(cfg, k_lo, n - 1, seed=2)[:, [3, 4]]    # Ez and Bx only
    print("adjoint autograd", flush=True)
    with Q().Box(cfg, "fp64") as box:
        amp = torch.tensor(beam.amp, dtype=torch.float64, requires_grad=True)
        sx = torch.tensor(beam.sigma_x, dtype=torch.float64, requires_grad=True)
        sy = torch.tensor(beam.sigma_y, dtype=torch.float64, requires_grad=True)
        out = Q().wake_fields(amp, sx, sy, box, n, k_lo=k_lo, fields=("ez", "bx"), ckpt_every=5)
        assert out.shape == (n - k_lo, 2, cfg.ny + 1, cfg.nx + 1)
        loss = (out * torch.tensor(w, device="cuda")).sum()
        loss.backward()
    wf = np.zeros((n - k_lo, len(FIELDS), cfg.ny + 1, cfg.nx + 1))
    wf[:, 3], wf[:, 4] = w[:, 0], w[:, 1]
    ga_o, gs_o, L_o = oracle_grad(cfg, beam, k_lo, wf)
    assert abs(float(loss.detach()) - L_o) <= 1e-9 * abs(L_o)
    assert np.abs(amp.grad.numpy() - ga_o).max() <= 1e-9 * np.abs(ga_o).max()
    assert abs(float(sx.grad) - gs_o[0]) <= 1e-9 * abs(gs_o[0])
    assert abs(float(sy.grad) - gs_o[1]) <= 1e-9 * abs(gs_o[1])


def test_adjoint_state_errors():
    qsp = Q()
    cfg, beam = CASES["n16_ppc2"]()
    with qsp.Box(cfg, "fp32") as box:
        w = {"ez": box.empty("ez", cfg.nzeta)}
        with pytest.raises(qsp.QspError) as e:
            box.adjoint(0, w)                      # nothing recorded
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        box.init_plasma()
        with pytest.raises(qsp.QspError) as e:
            box.record(cfg.nzeta, 4)               # no Gaussian beam
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        box.advance_slice()
        with pytest.raises(qsp.QspError) as e:
            box.record(cfg.nzeta, 4)               # cursor is not 0
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        box.init_plasma()
        for bad in ((0, 4), (cfg.nzeta + 1, 4), (cfg.nzeta, 0)):
            with pytest.raises(qsp.QspError) as e:
                box.record(*bad)
            assert e.value.status == qsp.QSP_ERR_INVALID_ARG
        box.record(cfg.nzeta, 4)
        with pytest.raises(qsp.QspError) as e:
            box.adjoint(cfg.nzeta, w)              # k_lo past the record
        assert e.value.status == qsp.QSP_ERR_INVALID_ARG
        ga, _, _ = box.adjoint(0, w)
        torch.cuda.synchronize()
        assert torch.all(ga == 0)                  # zero cotangent, zero gradient
        with pytest.raises(qsp.QspError) as e:
            box.adjoint(0, w)                      # the record was consumed
        assert e.value.status == qsp.QSP_ERR_BAD_STATE
        with pytest.raises(qsp.QspError) as e:
            box.advance_slice()                    # plasma must be re-initialised
        assert e.value.status == qsp.QSP_ERR_BAD_STATE


def test_adjoint_memory_cap():
    qsp = Q()
    cfg, beam = CASES["n16_ppc2"]()
    # 1024 particles: a slice state is ~115 kB; checkpoints every slice need
    # ~1.6 MB, every 4th slice ~0.9 MB, the box itself ~0.1-0.2 MB
    with qsp.Box(cfg, "fp32", mem_cap_bytes=1_400_000) as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        with pytest.raises(qsp.QspError) as e:
            box.record(cfg.nzeta, 1)
        assert e.value.status == qsp.QSP_ERR_OUT_OF_MEMORY
        box.record(cfg.nzeta, 4)
        assert box.stats()["device_bytes"] <= 1_400_000


@pytest.mark.parametrize("tol", [0.03, 0.0036])
def test_adjoint_with_early_exit_matches_oracle(tol):
    # predictor-corrector to a tolerance: the slices take different numbers
    # of iterations (1-3 at 0.03, 2-4 at 0.0036; every recorded residual is
    # at least a factor 1.4 from the tolerance), and the transpose follows
    # the recorded counts
    cfg, beam = W.small(n=32, nzeta=14, ppc=1, nb=0.9, sigma=0.8, pc_max_iter=4, pc_tol=tol,
                        extent=5.0)
    k_lo, k_hi = cfg.nzeta // 2, cfg.nzeta - 2
    w = cotangents(cfg, k_lo, k_hi)
    recs, tape = A.forward_with_tape(cfg, beam)
    counts = [r["pc_iters"] for r in recs[:k_hi + 1]]
    assert len(set(counts)) >= 3, counts

    def cot(k):
        if k < k_lo or k > k_hi:
            return {}
        return {q: w[k - k_lo, i] for i, q in enumerate(FIELDS)}
    ga_o, gsx, gsy = A.adjoint_box(cfg, beam, tape, cot)
    gs_o = np.array([gsx, gsy])
    print(f"adjoint with early exit, tol {tol}, counts {counts}", flush=True)
    with Q().Box(cfg, "fp64") as box:
        box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
        box.init_plasma()
        iters = torch.zeros(k_hi + 1, dtype=torch.int32, device="cuda")
        box.record(k_hi + 1, 4, pc_iters=iters)
        c = {q: torch.tensor(w[:, i], dtype=box.fdtype, device="cuda") for i, q in enumerate(FIELDS)}
        ga, gs, _ = box.adjoint(k_lo, c)
        torch.cuda.synchronize()
        ga, gs = ga.cpu().numpy(), gs.cpu().numpy()
    assert list(iters.cpu().numpy()) == counts
    err = np.abs(ga - ga_o).max() / np.abs(ga_o).max()
    assert err <= 1e-9, err
    assert np.all(np.abs(gs - gs_o) <= 1e-9 * np.abs(gs_o)), (gs, gs_o)


def c4_axis_loss(box, cfg, amp, sx, sy, n_loss):
    """C4 loss (mean on-axis Ez over slices k_lo..k_hi) of one forward box."""
    k_lo, k_hi = W.C4_LOSS_SLICES
    box.set_beam_gaussian(amp, sx, sy)
    box.init_plasma()
    ax = torch.zeros(cfg.nzeta, dtype=box.fdtype, device="cuda")
    box.run_box(axis={"ez": ax})
    torch.cuda.synchronize()
    return float(ax[k_lo:k_hi + 1].double().mean())


def c4_gradient(box, cfg, beam, ckpt_every=32):
    k_lo, k_hi = W.C4_LOSS_SLICES
    n = k_hi + 1
    w = torch.zeros(n - k_lo, cfg.ny + 1, cfg.nx + 1, dtype=box.fdtype, device="cuda")
    w[:, cfg.ny // 2, cfg.nx // 2] = 1.0 / (n - k_lo)
    box.set_beam_gaussian(beam.amp, beam.sigma_x, beam.sigma_y)
    box.init_plasma()
    box.record(n, ckpt_every)
    ga, gs, loss = box.adjoint(k_lo, {"ez": w})
    torch.cuda.synchronize()
    return ga.cpu().numpy(), gs.cpu().numpy(), float(loss.cpu()[0])


def test_c4_gradient_matches_central_differences():
    # the C4 workload at its own size: 256^2 nodes, the loss over slices
    # 400-420, checkpoints every 32 slices; FP64 central differences with
    # h = 1e-6 for sigma_r (sigma_x = sigma_y move together) and for
    # amplitudes ahead of, inside and behind the loss window
    cfg, beam = W.c4()
    print("c4 gradient vs central differences", flush=True)
    with Q().Box(cfg, "fp64") as box:
        ga, gs, L = c4_gradient(box, cfg, beam)
        L0 = c4_axis_loss(box, cfg, beam.amp, beam.sigma_x, beam.sigma_y, None)
        print(f"  loss {L:.12e} forward {L0:.12e}", flush=True)
        assert abs(L - L0) <= 1e-10 * abs(L0)
        gmax = np.abs(ga).max()
        h = 1e-6
        for k in (100, 250, 380, 405, 410, 419):
            ap, am = beam.amp.copy(), beam.amp.copy()
            ap[k] += h
            am[k] -= h
            fd = (c4_axis_loss(box, cfg, ap, beam.sigma_x, beam.sigma_y, None) -
                  c4_axis_loss(box, cfg, am, beam.sigma_x, beam.sigma_y, None)) / (2 * h)
            print(f"  d/da_{k}: adjoint {ga[k]:.9e} differences {fd:.9e}", flush=True)
            assert abs(ga[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * gmax), (k, ga[k], fd)
        s = beam.sigma_x
        fd = (c4_axis_loss(box, cfg, beam.amp, s + h, s + h, None) -
              c4_axis_loss(box, cfg, beam.amp, s - h, s - h, None)) / (2 * h)
        g_sr = gs[0] + gs[1]
        print(f"  d/dsigma_r: adjoint {g_sr:.9e} differences {fd:.9e}", flush=True)
        assert abs(g_sr - fd) <= 1e-4 * abs(fd), (g_sr, fd)
        # nothing behind the last loss slice matters
        assert np.all(ga[W.C4_LOSS_SLICES[1] + 1:] == 0.0)


def test_c4_fp32_gradient_matches_fp64():
    cfg, beam = W.c4()
    print("c4 gradient FP32 vs FP64", flush=True)
    with Q().Box(cfg, "fp64") as box:
        g64, s64, L64 = c4_gradient(box, cfg, beam)
    with Q().Box(cfg, "fp32") as box:
        g32, s32, L32 = c4_gradient(box, cfg, beam)
    err = np.abs(g32 - g64).max() / np.abs(g64).max()
    print(f"  amplitudes max rel {err:.2e}, sigma {s32} vs {s64}, loss {L32} vs {L64}", flush=True)
    assert err <= 1e-3, err
    assert np.all(np.abs(s32 - s64) <= 1e-3 * np.abs(s64)), (s32, s64)
    assert abs(L32 - L64) <= 1e-4 * abs(L64)
