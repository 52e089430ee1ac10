"""C-ABI checks that need no GPU: symbols, host-only routines, argument validation."""
import ctypes as C
import os
import re

import pytest

import synth
from oracle.lattice import mu_from_filling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_1604_06296_amd as tf
    return tf.load_library()


def test_library_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "tufrg.h")).read()
    declared = set(re.findall(r"\b(tufrg_[a-z_0-9]+)\s*\(", hdr))
    assert {"tufrg_init", "tufrg_bubbles", "tufrg_project", "tufrg_rhs", "tufrg_flow"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    import paper_1604_06296_amd.binding as b
    assert set(b.EXPORTS) == declared


def test_native_mu_from_filling_matches_oracle():
    import paper_1604_06296_amd as tf
    for (t, tp, n, T, L) in [(1.0, -0.25, 0.85, 1e-3, 256), (1.0, 0.0, 1.0, 0.01, 64),
                             (1.0, -0.35, 0.72, 0.01, 128)]:
        assert abs(tf.mu_from_filling(t, tp, n, T, L) - mu_from_filling(n, t, tp, T, L)) < 1e-12


def test_native_mu_rejects_bad_filling(lib):
    out = C.c_double()
    assert lib.tufrg_mu_from_filling(1.0, 0.0, 2.5, 0.1, 16, C.byref(out)) == -1
    assert lib.tufrg_mu_from_filling(1.0, 0.0, 0.5, 0.0, 16, C.byref(out)) == -1


@pytest.mark.parametrize("kw,msg", [
    (dict(Lq=7), "Lq"), (dict(Lq=4, shells=1), "Lq"), (dict(Lq=8, shells=3), "Lq"),
    (dict(Lk=9), "Lk"), (dict(Lk=2), "Lk"), (dict(shells=5), "shells"), (dict(t=0.0), "t must"),
    (dict(Lk=1024), "Lk"),
])
def test_init_validation_without_gpu(lib, kw, msg):
    """Invalid points are rejected before any device call."""
    from paper_1604_06296_amd.binding import _Options, _Point
    p = dict(t=1.0, tp=-0.2, mu=-0.3, U=3.0, Lq=10, Lk=16, shells=1)
    p.update(kw)
    arr = (_Point * 1)(_Point(p["t"], p["tp"], p["mu"], p["U"], p["Lq"], p["Lk"], p["shells"], 0))
    h = C.c_void_p()
    st = lib.tufrg_init(arr, 1, C.byref(_Options(0, 0)), None, C.byref(h))
    assert st == -1 and not h.value
    assert msg in lib.tufrg_last_error(None).decode()


def test_workload_definitions():
    w2 = synth.cfg2()
    assert w2.points[0].nq == 576 and w2.points[0].nff == 13 and w2.points[0].Lk == 96
    w3 = synth.cfg3()
    assert -1.2 <= w3.points[0].mu <= 0.0 and w3.points[0].nff == 21
    w4 = synth.cfg4()
    assert len(w4.points) == 64
    assert {p.Lk for p in w4.points} == {4 * p.Lq for p in w4.points}
    assert all(16 <= p.Lq <= 40 and p.Lq % 2 == 0 for p in w4.points)


def test_mlp_and_surrogate_calls_validate_arguments(lib):
    """Argument errors are reported before any device call."""
    out = C.c_void_p()
    w = (C.c_int32 * 3)(9, 0, 4)
    assert lib.tufrg_mlp_create(w, 3, 64, 0, None, C.byref(out)) == -1
    assert "widths" in lib.tufrg_mlp_last_error(None).decode()
    w = (C.c_int32 * 1)(9)
    assert lib.tufrg_mlp_create(w, 1, 64, 0, None, C.byref(out)) == -1
    w = (C.c_int32 * 2)(9, 4)
    assert lib.tufrg_mlp_create(w, 2, 0, 0, None, C.byref(out)) == -1
    assert lib.tufrg_mlp_forward(None, None, None, 1) == -1
    assert lib.tufrg_surrogate_attach(None, None, None, 1e-3, 8) == -1
    assert lib.tufrg_loop_harmonics(None, None, None) == -1
    n = C.c_int32()
    assert lib.tufrg_harmonics(None, 0, C.byref(n), None, None) == -1


def test_flag_values_match_header(lib):
    """The binding's flag bits are the header's, and unknown bits are rejected."""
    import paper_1604_06296_amd.binding as b
    from paper_1604_06296_amd.binding import _Options, _Point
    hdr = open(os.path.join(ROOT, "include", "tufrg.h")).read()
    bits = {m.group(1): 1 << int(m.group(2)) for m in re.finditer(r"TUFRG_([A-Z_]+)\s*=\s*1u\s*<<\s*(\d+)", hdr)}
    for name in ("NO_CROSS", "AUTOTUNE", "NO_SYMMETRY", "LOOP_QUEUE", "NO_FUSE", "OMEGA_CUTOFF",
                 "SYMMETRIC_STATE", "DENSE_PROJECTION", "NO_LOOP_REUSE"):
        assert getattr(b, name) == bits[name], name
    assert b.REGULATORS == {"T": 0, "omega": bits["OMEGA_CUTOFF"]}
    arr = (_Point * 1)(_Point(1.0, -0.2, -0.3, 3.0, 10, 16, 1, 0))
    h = C.c_void_p()
    assert lib.tufrg_init(arr, 1, C.byref(_Options(0, 1 << 9)), None, C.byref(h)) == -1
    assert "flag" in lib.tufrg_last_error(None).decode()


def test_omega_workload_definition():
    w, w2 = synth.cfg2_omega(), synth.cfg2()
    assert w.regulator == "omega" and w2.regulator == "T"
    assert w.points[0] == w2.points[0]
    assert w.T0 == 100 * 8.0 and w.Xmax == 10 * 8.0    # bandwidth 8t, t = 1


@pytest.mark.parametrize("case,msg", [
    ("wsum", "sum to 1"), ("zone", "[-pi, pi)"), ("wneg", "weights must be finite"), ("sym", "uniform transfer grid"),
])
def test_mesh_validation_without_gpu(lib, case, msg):
    """Invalid transfer meshes (and a mesh with symmetric states) are rejected
    before any device call."""
    import numpy as np
    from paper_1604_06296_amd.binding import _Mesh, _Options, _Point
    mesh = synth.refined_mesh(8, 3, [(0.0, 0.0)], radius=1)
    qx, qy, w = mesh.qx.copy(), mesh.qy.copy(), mesh.w.copy()
    flags = 0
    if case == "wsum":
        w *= 1.001
    elif case == "zone":
        qx[3] = 3.5
    elif case == "wneg":
        w[0] = -w[0]
    elif case == "sym":
        flags = 64    # TUFRG_SYMMETRIC_STATE
    arr = (_Point * 1)(_Point(1.0, -0.2, -0.3, 3.0, 8, 16, 1, 0))
    dpp = C.POINTER(C.c_double)
    m = (_Mesh * 1)(_Mesh(qx.size, qx.ctypes.data_as(dpp), qy.ctypes.data_as(dpp), w.ctypes.data_as(dpp)))
    h = C.c_void_p()
    st = lib.tufrg_init_mesh(arr, m, 1, C.byref(_Options(0, flags)), None, C.byref(h))
    assert st in (-1, -5) and not h.value
    assert msg in lib.tufrg_last_error(None).decode()


def test_dense_projection_option_validation_without_gpu(lib):
    """The dense projection operator is FP64 per-momentum only (rejected before
    any device call)."""
    from paper_1604_06296_amd.binding import DENSE_PROJECTION, SYMMETRIC_STATE, _Options, _Point
    arr = (_Point * 1)(_Point(1.0, -0.2, -0.3, 3.0, 8, 16, 1, 0))
    h = C.c_void_p()
    assert lib.tufrg_init(arr, 1, C.byref(_Options(1, DENSE_PROJECTION)), None, C.byref(h)) == -5
    assert lib.tufrg_init(arr, 1, C.byref(_Options(0, DENSE_PROJECTION | SYMMETRIC_STATE)), None,
                          C.byref(h)) == -5
    assert "dense projection" in lib.tufrg_last_error(None).decode()
