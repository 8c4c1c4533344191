"""ctypes binding of libqsp (include/qsp.h).

Argument marshalling only: every step of the slice loop runs in the HIP
kernels of libqsp.so.  PyTorch supplies device memory (tensors whose
``data_ptr()`` is passed across the C ABI) and the HIP stream.  The library
must have been built (``paper_2109_10277_amd/build.py``); loading fails
loudly otherwise - there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsp.so")

QSP_OK, QSP_ERR_INVALID_ARG, QSP_ERR_BAD_STATE, QSP_ERR_OUT_OF_MEMORY, \
    QSP_ERR_DEVICE, QSP_ERR_NONFINITE = range(6)
QSP_FP32, QSP_FP64 = 0, 1
QSP_BXBY_PC, QSP_BXBY_EXPLICIT = 0, 1

QUANTITIES = ("psi", "exmby", "eypbx", "ez", "bx", "by", "bz",
              "rho_mjz", "jx", "jy", "jz", "rho")
QID = {q: i for i, q in enumerate(QUANTITIES)}
NQ = len(QUANTITIES)
FIELD_QUANTITIES = QUANTITIES[:7]


class QspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


def _status_name(s: int) -> str:
    return {0: "QSP_OK", 1: "QSP_ERR_INVALID_ARG", 2: "QSP_ERR_BAD_STATE",
            3: "QSP_ERR_OUT_OF_MEMORY", 4: "QSP_ERR_DEVICE",
            5: "QSP_ERR_NONFINITE"}.get(s, f"status {s}")


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("y_lo", C.c_double), ("y_hi", C.c_double),
                ("nzeta", C.c_int32), ("precision", C.c_int32),
                ("zeta_hi", C.c_double), ("dzeta", C.c_double),
                ("ppc_x", C.c_int32), ("ppc_y", C.c_int32),
                ("n0", C.c_double),
                ("pc_max_iter", C.c_int32), ("deposit_mode", C.c_int32),
                ("pc_tol", C.c_double), ("pc_shift", C.c_double),
                ("psi_floor", C.c_double), ("mem_cap_bytes", C.c_int64),
                ("shape_order", C.c_int32), ("bxby_solver", C.c_int32)]


class SliceOut(C.Structure):
    _fields_ = [("q", C.c_void_p * NQ)]


class BoxOut(C.Structure):
    _fields_ = [("stack", C.c_void_p * NQ), ("stack_every", C.c_int32),
                ("reserved0", C.c_int32), ("lineout", C.c_void_p * NQ),
                ("axis", C.c_void_p * NQ), ("pc_iters", C.c_void_p),
                ("pc_resid", C.c_void_p)]


class Cotangent(C.Structure):
    _fields_ = [("k_lo", C.c_int32), ("reserved0", C.c_int32), ("w", C.c_void_p * 7)]


class Stats(C.Structure):
    _fields_ = [("slices", C.c_int64), ("particle_pushes", C.c_int64),
                ("pc_iterations", C.c_int64), ("pc_not_converged", C.c_int64),
                ("n_clamped", C.c_int64), ("n_absorbed", C.c_int64),
                ("n_deposit_global", C.c_int64), ("dst_solves", C.c_int64),
                ("max_pc_residual", C.c_double), ("elapsed_ms", C.c_double),
                ("device_bytes", C.c_int64), ("box_reruns", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_DP = C.POINTER(C.c_double)

KERNEL_CLASSES = ("push", "trial", "row_fwd", "col", "row_inv", "other")


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_int64 * 6)]


class SliceState(C.Structure):
    _fields_ = [("k", C.c_int32), ("reserved0", C.c_int32), ("np", C.c_int64),
                ("x", _DP), ("y", _DP), ("ux", _DP), ("uy", _DP), ("psi", _DP),
                ("w", _DP), ("hist", _DP), ("jx_prev", _DP), ("jy_prev", _DP),
                ("bx_prev1", _DP), ("by_prev1", _DP), ("bx_prev2", _DP),
                ("by_prev2", _DP)]


_lib = None


def lib() -> C.CDLL:
    """Load libqsp.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2109_10277_amd/build.py`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "qsp_validate_config": [C.POINTER(Config), C.c_char_p, C.c_size_t],
            "qsp_create": [C.POINTER(Config), C.c_int, vp, C.POINTER(vp)],
            "qsp_destroy": [vp],
            "qsp_init_plasma": [vp],
            "qsp_set_beam_gaussian": [vp, _DP, d, d, d, d],
            "qsp_set_beam_particles": [vp, i64, vp, d],
            "qsp_set_beam_current": [vp, i32, vp],
            "qsp_get_beam_particles": [vp, i64, vp],
            "qsp_get_beam_count": [vp, C.POINTER(i64)],
            "qsp_advance_slice": [vp, C.POINTER(SliceOut)],
            "qsp_run_box": [vp, C.POINTER(BoxOut), C.POINTER(Stats)],
            "qsp_get_stats": [vp, C.POINTER(Stats)],
            "qsp_get_slice_state": [vp, C.POINTER(SliceState)],
            "qsp_set_slice_state": [vp, C.POINTER(SliceState)],
            "qsp_solve_poisson": [vp, i32, vp, vp, d],
            "qsp_solve_poisson_noalloc": [C.POINTER(Config), C.c_int, vp, i32, vp, vp, d],
            "qsp_get_info": [vp, C.POINTER(i64), C.POINTER(i32)],
            "qsp_set_timing": [vp, i32],
            "qsp_get_kernel_times": [vp, C.POINTER(KernelTimes)],
            "qsp_run_box_record": [vp, i32, i32, C.POINTER(BoxOut), C.POINTER(Stats)],
            "qsp_run_box_adjoint": [vp, C.POINTER(Cotangent), vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.qsp_status_string.argtypes = [C.c_int]
        L.qsp_status_string.restype = C.c_char_p
        L.qsp_last_error.argtypes = [vp]
        L.qsp_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def make_config(cfg, precision: str = "fp32", deposit_mode: int = 0,
                mem_cap_bytes: int = 0) -> Config:
    """Build the C config from any object with the BoxConfig attributes."""
    c = Config()
    c.nx, c.ny = cfg.nx, cfg.ny
    c.x_lo, c.x_hi, c.y_lo, c.y_hi = cfg.x_lo, cfg.x_hi, cfg.y_lo, cfg.y_hi
    c.nzeta = cfg.nzeta
    c.precision = {"fp32": QSP_FP32, "fp64": QSP_FP64}[precision]
    c.zeta_hi, c.dzeta = cfg.zeta_hi, cfg.dzeta
    c.ppc_x, c.ppc_y = cfg.ppc_x, cfg.ppc_y
    c.n0 = cfg.n0
    c.pc_max_iter = cfg.pc_max_iter
    c.deposit_mode = deposit_mode
    c.pc_tol = cfg.pc_tol
    shift = getattr(cfg, "pc_shift", None)
    c.pc_shift = -1.0 if shift is None else float(shift)
    c.psi_floor = cfg.psi_floor
    c.mem_cap_bytes = mem_cap_bytes
    c.shape_order = int(getattr(cfg, "shape_order", 1))
    c.bxby_solver = {"pc": QSP_BXBY_PC, "explicit": QSP_BXBY_EXPLICIT}[
        getattr(cfg, "bxby_solver", "pc")]
    return c


def validate_config(cfg, precision: str = "fp32", **kw) -> tuple[bool, str]:
    c = make_config(cfg, precision, **kw) if not isinstance(cfg, Config) else cfg
    buf = C.create_string_buffer(256)
    st = lib().qsp_validate_config(C.byref(c), buf, 256)
    return st == QSP_OK, buf.value.decode()


def _check(st: int, ctx=None):
    if st != QSP_OK:
        msg = lib().qsp_last_error(ctx).decode()
        raise QspError(st, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


# Boxes still open are closed by an exit handler registered when the first
# box is made, after torch has been imported: exit handlers run
# last-registered first, so the contexts go before torch and the HIP runtime
# are torn down, and none is destroyed from a late finaliser.
_LIVE: "weakref.WeakSet[Box]" = weakref.WeakSet()
_EXIT_HOOK = False
_FINALIZING = sys.is_finalizing   # kept: module globals may be cleared at shutdown


def _close_live_boxes():
    for box in list(_LIVE):
        box.close()


class Box:
    """One simulation box on one GPU (a libqsp context).

    ``cfg`` is any object with the attributes of ``workloads.BoxConfig``.
    All device tensors passed in must live on this machine's device and be
    contiguous; fields use the box precision, deposits float64.
    """

    def __init__(self, cfg, precision: str = "fp32", device: int = 0,
                 stream=None, deposit_mode: int = 0, mem_cap_bytes: int = 0):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.fdtype = torch.float32 if precision == "fp32" else torch.float64
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._c = make_config(cfg, precision, deposit_mode, mem_cap_bytes)
        h = C.c_void_p()
        st = lib().qsp_create(C.byref(self._c), device, C.c_void_p(stream.cuda_stream),
                              C.byref(h))
        _check(st, None)
        self._h = h
        self.record_id = 0      # bumped by every record(); ties a backward to its forward
        global _EXIT_HOOK
        if not _EXIT_HOOK:
            atexit.register(_close_live_boxes)
            _EXIT_HOOK = True
        _LIVE.add(self)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().qsp_destroy(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be finalised:
        # leave the context to the process exit rather than call into it
        if _FINALIZING is None or _FINALIZING():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers
    def _call(self, name, *args):
        _check(getattr(lib(), name)(self._h, *args), self._h)

    def node_shape(self):
        return (self.cfg.ny + 1, self.cfg.nx + 1)

    def dtype_of(self, q: str):
        return self.fdtype if QID[q] < 7 else self.torch.float64

    def empty(self, q: str, *lead):
        return self.torch.zeros(*lead, *self.node_shape(), dtype=self.dtype_of(q),
                                device=self.device)

    @property
    def n_particles(self) -> int:
        n = C.c_int64()
        k = C.c_int32()
        self._call("qsp_get_info", C.byref(n), C.byref(k))
        return n.value

    @property
    def cursor(self) -> int:
        n = C.c_int64()
        k = C.c_int32()
        self._call("qsp_get_info", C.byref(n), C.byref(k))
        return k.value

    # -- entry points
    def init_plasma(self):
        self._call("qsp_init_plasma")

    def set_beam_gaussian(self, amp, sx, sy, x0=0.0, y0=0.0):
        a = np.ascontiguousarray(amp, dtype=np.float64)
        if a.shape != (self.cfg.nzeta,):
            raise ValueError("amp must have shape [nzeta]")
        self._call("qsp_set_beam_gaussian", a.ctypes.data_as(_DP), float(sx), float(sy),
                   float(x0), float(y0))

    def set_beam_particles(self, soa, dt: float = 0.0):
        """soa: contiguous float32 device tensor [7, n] (x, y, zeta, ux, uy, uz, w)."""
        if soa is None:
            self._call("qsp_set_beam_particles", 0, None, float(dt))
            return
        if soa.dtype != self.torch.float32 or soa.dim() != 2 or soa.shape[0] != 7:
            raise ValueError("soa must be float32 [7, n]")
        self._call("qsp_set_beam_particles", int(soa.shape[1]), C.c_void_p(_ptr(soa)), float(dt))

    def set_beam_current(self, k: int, jz=None):
        """Explicit Jz (= rho) of slice k: float64 device tensor [ny+1, nx+1]
        (None removes it; k = -1 with None removes all)."""
        if jz is not None:
            if jz.dtype != self.torch.float64 or tuple(jz.shape) != self.node_shape():
                raise ValueError("jz must be float64 [ny+1, nx+1]")
            if jz.device != self.device:
                raise ValueError("jz must be on the box device")
        self._call("qsp_set_beam_current", int(k), C.c_void_p(_ptr(jz)))

    def beam_count(self) -> int:
        n = C.c_int64()
        self._call("qsp_get_beam_count", C.byref(n))
        return n.value

    def get_beam_particles(self):
        n = self.beam_count()
        out = self.torch.empty(7, n, dtype=self.torch.float32, device=self.device)
        self._call("qsp_get_beam_particles", n, C.c_void_p(_ptr(out)))
        return out

    def advance_slice(self, outputs: Optional[Dict[str, object]] = None):
        so = SliceOut()
        for q, t in (outputs or {}).items():
            self._check_out(q, t, self.node_shape())
            so.q[QID[q]] = _ptr(t)
        self._call("qsp_advance_slice", C.byref(so))

    def run_box(self, stack=None, stack_every: int = 1, lineout=None, axis=None,
                pc_iters=None, pc_resid=None) -> dict:
        bo = self._box_out(stack, stack_every, lineout, axis, pc_iters, pc_resid)
        st = Stats()
        self._call("qsp_run_box", C.byref(bo), C.byref(st))
        return st.as_dict()

    @staticmethod
    def _box_out(stack, stack_every, lineout, axis, pc_iters, pc_resid) -> BoxOut:
        bo = BoxOut()
        bo.stack_every = stack_every
        for q, t in (stack or {}).items():
            bo.stack[QID[q]] = _ptr(t)
        for q, t in (lineout or {}).items():
            bo.lineout[QID[q]] = _ptr(t)
        for q, t in (axis or {}).items():
            bo.axis[QID[q]] = _ptr(t)
        bo.pc_iters = _ptr(pc_iters)
        bo.pc_resid = _ptr(pc_resid)
        return bo

    def record(self, n_slices: int, ckpt_every: int, stack=None, stack_every: int = 1,
               lineout=None, axis=None, pc_iters=None, pc_resid=None) -> dict:
        """Checkpointed forward pass of slices 0 .. n_slices-1 for ``adjoint``
        (outputs as in ``run_box``)."""
        bo = self._box_out(stack, stack_every, lineout, axis, pc_iters, pc_resid)
        st = Stats()
        self.record_id += 1
        self._call("qsp_run_box_record", int(n_slices), int(ckpt_every), C.byref(bo),
                   C.byref(st))
        return st.as_dict()

    def adjoint(self, k_lo: int, cot: Dict[str, object]):
        """Reverse pass of the last ``record``.  ``cot[q]``: device tensor
        [n_slices - k_lo, ny+1, nx+1] (box precision) for field q.  Returns
        (grad_amp [nzeta], grad_sigma [2], loss [1]) as float64 tensors."""
        torch = self.torch
        c = Cotangent()
        c.k_lo = int(k_lo)
        for q, t in cot.items():
            if QID[q] >= 7:
                raise ValueError(f"{q} is not a field")
            if t.dtype != self.fdtype or t.device != self.device:
                raise ValueError(f"cotangent {q}: wrong dtype/device")
            c.w[QID[q]] = _ptr(t)
        ga = torch.empty(self.cfg.nzeta, dtype=torch.float64, device=self.device)
        gs = torch.empty(2, dtype=torch.float64, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        self._call("qsp_run_box_adjoint", C.byref(c), C.c_void_p(_ptr(ga)), C.c_void_p(_ptr(gs)),
                   C.c_void_p(_ptr(loss)))
        return ga, gs, loss

    def stats(self) -> dict:
        st = Stats()
        self._call("qsp_get_stats", C.byref(st))
        return st.as_dict()

    def set_timing(self, every: int):
        self._call("qsp_set_timing", int(every))

    def kernel_times(self) -> dict:
        kt = KernelTimes()
        self._call("qsp_get_kernel_times", C.byref(kt))
        return {c: (kt.ms[i], kt.launches[i]) for i, c in enumerate(KERNEL_CLASSES)}

    def solve_poisson(self, src, dst, shift: float = 0.0):
        nb = src.shape[0]
        self._call("qsp_solve_poisson", int(nb), C.c_void_p(_ptr(src)),
                   C.c_void_p(_ptr(dst)), float(shift))

    def _state_struct(self, arrs: dict, k: int) -> SliceState:
        s = SliceState()
        s.k = k
        s.np = arrs["x"].size
        for name in ("x", "y", "ux", "uy", "psi", "w", "hist", "jx_prev", "jy_prev",
                     "bx_prev1", "by_prev1", "bx_prev2", "by_prev2"):
            a = arrs[name]
            assert a.dtype == np.float64 and a.flags.c_contiguous
            setattr(s, name, a.ctypes.data_as(_DP))
        return s

    def get_state(self) -> dict:
        n = self.n_particles
        nn = self.node_shape()
        arrs = {k: np.zeros(n) for k in ("x", "y", "ux", "uy", "psi", "w")}
        arrs["hist"] = np.zeros((4, 5, n))
        for k in ("jx_prev", "jy_prev", "bx_prev1", "by_prev1", "bx_prev2", "by_prev2"):
            arrs[k] = np.zeros(nn)
        s = self._state_struct(arrs, 0)
        self._call("qsp_get_slice_state", C.byref(s))
        arrs["k"] = s.k
        return arrs

    def set_state(self, k: int, arrs: dict):
        a = {name: np.ascontiguousarray(v, dtype=np.float64) for name, v in arrs.items()
             if name != "k"}
        s = self._state_struct(a, k)
        self._call("qsp_set_slice_state", C.byref(s))

    def _check_out(self, q, t, shape):
        if tuple(t.shape[-2:]) != tuple(shape):
            raise ValueError(f"output {q}: expected trailing shape {shape}")
        if t.dtype != self.dtype_of(q) or t.device != self.device:
            raise ValueError(f"output {q}: wrong dtype/device")


def solve_poisson_noalloc(cfg, src, dst, shift: float = 0.0, precision: str = "fp32",
                          device: int = 0, stream=None):
    """Batched Dirichlet solve without a context or device allocation
    (qsp_solve_poisson_noalloc): src, dst contiguous device tensors
    [nbatch, ny+1, nx+1] of the given precision."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(torch.device("cuda", device))
    c = make_config(cfg, precision)
    st = lib().qsp_solve_poisson_noalloc(C.byref(c), int(device), C.c_void_p(stream.cuda_stream),
                                         int(src.shape[0]), C.c_void_p(_ptr(src)),
                                         C.c_void_p(_ptr(dst)), float(shift))
    _check(st, None)


def status_string(s: int) -> str:
    return lib().qsp_status_string(s).decode()


def _wake_fn():
    import torch

    class WakeFn(torch.autograd.Function):
        """Wakefields of slices k_lo .. n_slices-1 as a differentiable
        function of the Gaussian drive beam: per-slice amplitudes ``amp``
        [nzeta] and transverse sizes ``sigma_x``, ``sigma_y``.

        forward: set the beam, reset the plasma, checkpointed forward pass
        (``Box.record``); returns [n_slices - k_lo, len(fields), ny+1, nx+1]
        in the box precision.  backward: ``Box.adjoint`` with the incoming
        gradient as cotangent.  One backward per forward (the record is
        consumed), before the box records anything else: a backward whose
        forward's record has been replaced raises."""

        @staticmethod
        def forward(ctx, amp, sigma_x, sigma_y, box, n_slices, k_lo, fields, ckpt_every,
                    x0=0.0, y0=0.0):
            box.set_beam_gaussian(amp.detach().double().cpu().numpy(), float(sigma_x),
                                  float(sigma_y), x0, y0)
            box.init_plasma()
            stack = {q: box.empty(q, n_slices) for q in fields}
            box.record(n_slices, ckpt_every, stack=stack)
            out = torch.stack([stack[q][k_lo:] for q in fields], dim=1)
            ctx.box, ctx.fields, ctx.k_lo = box, tuple(fields), k_lo
            ctx.record_id = box.record_id
            ctx.amp_meta = (amp.dtype, amp.device)
            ctx.sig_meta = [(s.dtype, s.device) if torch.is_tensor(s) else None
                            for s in (sigma_x, sigma_y)]
            return out

        @staticmethod
        def backward(ctx, g):
            if ctx.box.record_id != ctx.record_id:
                raise RuntimeError("wake_fields backward: the box has recorded another forward "
                                   "pass since this one; its gradient is no longer available")
            cot = {q: g[:, i].contiguous().to(ctx.box.fdtype) for i, q in enumerate(ctx.fields)}
            ga, gs, _ = ctx.box.adjoint(ctx.k_lo, cot)
            dt, dev = ctx.amp_meta
            gsig = []
            for i, meta in enumerate(ctx.sig_meta):
                gsig.append(None if meta is None else gs[i].to(dtype=meta[0], device=meta[1]))
            return (ga.to(dtype=dt, device=dev), gsig[0], gsig[1], None, None, None, None, None,
                    None, None)

    return WakeFn


_WAKE = None


def wake_fields(amp, sigma_x, sigma_y, box: "Box", n_slices: int, k_lo: int = 0,
                fields=("ez",), ckpt_every: int = 16, x0: float = 0.0, y0: float = 0.0):
    """Differentiable wakefields (see WakeFn)."""
    global _WAKE
    if _WAKE is None:
        _WAKE = _wake_fn()
    return _WAKE.apply(amp, sigma_x, sigma_y, box, n_slices, k_lo, tuple(fields), ckpt_every,
                       x0, y0)
