"""The context-free, allocation-free Dirichlet solve
(qsp_solve_poisson_noalloc) against the context's qsp_solve_poisson on the
same inputs: two calls in a row on the same GPU, the second smaller (the
static scratch keeps the first call's contents), both precisions.  The two
entry points run the same transform kernels; only their tables are computed
differently (on the host with std::sin/cos for the context, on the device
with sincospi here), so FP64 agrees to round-off and FP32 to ~1e-6."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Q():
    from paper_2109_10277_amd import qsp
    return qsp


def grid(nx, ny):
    return W.BoxConfig(nx=nx, ny=ny, x_lo=-3.0, x_hi=3.0, y_lo=-2.0, y_hi=2.5,
                       nzeta=2, zeta_hi=0.0, dzeta=0.1)


def sources(cfg, nb, seed, dtype):
    rng = np.random.default_rng(seed)
    s = rng.normal(size=(nb, cfg.ny + 1, cfg.nx + 1))
    s[:, 0, :] = s[:, -1, :] = 0.0
    s[:, :, 0] = s[:, :, -1] = 0.0
    return torch.tensor(s, dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_solve_matches_context_solve_twice(prec):
    qsp = Q()
    dtype = torch.float32 if prec == "fp32" else torch.float64
    tol = 1e-12 if prec == "fp64" else 5e-6
    # the second call is smaller than the first
    for (nx, ny, nb, shift) in ((1024, 512, 4, 0.0), (256, 128, 2, 1.32)):
        cfg = grid(nx, ny)
        print(f"noalloc {prec} {nx}x{ny} batch {nb} shift {shift}", flush=True)
        src = sources(cfg, nb, nx + ny, dtype)
        got = torch.full_like(src, float("nan"))
        qsp.solve_poisson_noalloc(cfg, src, got, shift, prec)
        with qsp.Box(cfg, prec) as box:
            ref = torch.zeros_like(src)
            box.solve_poisson(src, ref, shift)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        err = float(torch.linalg.vector_norm((got - ref).double()) /
                    torch.linalg.vector_norm(ref.double()))
        print(f"  rel-L2 against the context solve {err:.2e}", flush=True)
        assert err < tol, err
        assert torch.all(got[:, 0, :] == 0) and torch.all(got[:, :, -1] == 0)


def test_noalloc_rejects_oversize_and_bad_arguments():
    qsp = Q()
    cfg = grid(2048, 2048)
    src = torch.zeros(2, 2049, 2049, dtype=torch.float64, device="cuda")
    with pytest.raises(qsp.QspError) as e:      # 2 x 2048^2 doubles = 64 MiB > 16 MiB
        qsp.solve_poisson_noalloc(cfg, src, src.clone(), 0.0, "fp64")
    assert e.value.status == qsp.QSP_ERR_INVALID_ARG
    small = grid(64, 64)
    s = torch.zeros(5, 65, 65, dtype=torch.float32, device="cuda")
    with pytest.raises(qsp.QspError) as e:      # nbatch 5
        qsp.solve_poisson_noalloc(small, s, s.clone(), 0.0, "fp32")
    assert e.value.status == qsp.QSP_ERR_INVALID_ARG
    with pytest.raises(qsp.QspError) as e:      # negative shift
        qsp.solve_poisson_noalloc(small, s[:1], s[:1].clone(), -1.0, "fp32")
    assert e.value.status == qsp.QSP_ERR_INVALID_ARG
