"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/qsp.h is exported by libqsp.so, the ctypes structs match the C layout
(checked against a gcc-compiled probe), and configuration validation rejects
bad inputs without touching a device."""
import ctypes
import dataclasses
import os
import re
import subprocess
import tempfile

import pytest

import workloads as W
from paper_2109_10277_amd import qsp as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsp.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(qsp_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "qsp_create" in names and "qsp_run_box" in names and len(names) >= 15
    lib = ctypes.CDLL(Q.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


STRUCTS = {
    "qsp_config": Q.Config, "qsp_slice_out": Q.SliceOut, "qsp_box_out": Q.BoxOut,
    "qsp_stats": Q.Stats, "qsp_slice_state": Q.SliceState,
    "qsp_kernel_times": Q.KernelTimes, "qsp_box_cotangent": Q.Cotangent,
}


def test_ctypes_layout_matches_c_header():
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qsp.h"', 'int main(void){']
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        cname, field, val = line.split()
        py = STRUCTS[cname]
        if field == "size":
            assert ctypes.sizeof(py) == int(val), cname
        else:
            assert getattr(py, field).offset == int(val), (cname, field)


def good():
    return W.c1()[0]


@pytest.mark.parametrize("mutate,expect", [
    (lambda c: setattr(c, "nx", 48), "nx"),
    (lambda c: setattr(c, "ny", 8), "ny"),
    (lambda c: setattr(c, "nx", 4096), "nx"),
    (lambda c: setattr(c, "x_hi", c.x_lo), "x_lo"),
    (lambda c: setattr(c, "y_lo", float("nan")), "y_lo"),
    (lambda c: setattr(c, "nzeta", 0), "nzeta"),
    (lambda c: setattr(c, "dzeta", -0.1), "dzeta"),
    (lambda c: setattr(c, "ppc_x", 3), "ppc_x"),
    (lambda c: setattr(c, "n0", 0.0), "n0"),
    (lambda c: setattr(c, "pc_max_iter", 0), "pc_max_iter"),
    (lambda c: setattr(c, "pc_tol", float("inf")), "pc_tol"),
    (lambda c: setattr(c, "psi_floor", 1.5), "psi_floor"),
])
def test_validation_rejects(mutate, expect):
    c = good()
    mutate(c)
    ok, msg = Q.validate_config(c)
    assert not ok and expect in msg


def test_validation_accepts_presets():
    for f in (W.c1, W.c2, W.c4, W.c5):
        cfg = f()[0]
        for prec in ("fp32", "fp64"):
            assert Q.validate_config(cfg, prec) == (True, "")
    assert Q.validate_config(W.c3_config())[0]


def test_bad_precision_and_deposit_mode():
    c = Q.make_config(good())
    c.precision = 7
    assert not Q.validate_config(c)[0]
    c = Q.make_config(good())
    c.deposit_mode = 2
    assert not Q.validate_config(c)[0]


@pytest.mark.parametrize("order,ok", [(0, True), (1, True), (2, True), (3, True), (4, False),
                                      (-1, False)])
def test_shape_order_validation(order, ok):
    c = Q.make_config(good())
    c.shape_order = order
    assert Q.validate_config(c)[0] == ok
    c = Q.make_config(dataclasses.replace(good(), shape_order=2))
    assert c.shape_order == 2
    c.bxby_solver = 2
    assert not Q.validate_config(c)[0]


def test_explicit_solver_validation():
    c = Q.make_config(dataclasses.replace(good(), bxby_solver="explicit"))
    assert c.bxby_solver == Q.QSP_BXBY_EXPLICIT
    assert Q.validate_config(c)[0]
    c.shape_order = 0
    ok, msg = Q.validate_config(c)
    assert not ok and "explicit" in msg


def test_status_strings():
    for s in range(6):
        assert Q.status_string(s)
    assert Q.status_string(99) == "unknown status"


def test_null_context_is_an_error_not_a_crash():
    lib = Q.lib()
    assert lib.qsp_init_plasma(None) == Q.QSP_ERR_INVALID_ARG
    assert lib.qsp_run_box_record(None, 1, 1, None, None) == Q.QSP_ERR_INVALID_ARG
    assert lib.qsp_run_box_adjoint(None, None, None, None, None) == Q.QSP_ERR_INVALID_ARG
    assert lib.qsp_destroy(None) == Q.QSP_OK
    assert lib.qsp_last_error(None)
