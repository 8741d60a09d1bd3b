"""The C-ABI library loads, exports every function include/grf.h declares,
and validates its inputs on the host (CPU only: no compute call)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2605_02670_amd import grf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "grf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["grf_graph_create", "grf_graph_info", "grf_graph_destroy", "grf_noise", "grf_sample",
              "grf_solve_shifted", "grf_sample_batched", "grf_last_error", "grf_opts_init", "grf_shift_count"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(grf.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    bound = {s[0] for s in grf._SIGS}
    assert set(_declared()) <= bound, "binding misses a declared function"


def test_struct_layouts_match_header():
    # grf_opts: double, 10 x int32, int64, 3 pointers
    assert C.sizeof(grf.Opts) == 8 + 10 * 4 + 8 + 3 * 8
    # grf_stats: 4 int32, int64, double, 4 int32, 16 double, 16 int32 (per kernel id),
    # then 7 double, 7 int32 (per PCG size class), int32 n_nonfinite, 7 int64, 7 int64 (per class)
    assert C.sizeof(grf.Stats) == 4 * 4 + 8 + 8 + 4 * 4 + 16 * 8 + 16 * 4 + 7 * 8 + 8 * 4 + 2 * 7 * 8
    assert grf.Stats.pcg_class_ms.offset == 240
    assert len(grf.KERNELS) == 13  # GRF_K_COUNT


def test_status_and_flag_constants_match_header():
    text = open(os.path.join(ROOT, "include", "grf.h")).read()
    status = dict((k, int(v)) for k, v in re.findall(r"\b(GRF_E[A-Z]+|GRF_OK)\s*=\s*(-?\d+)", text))
    for name in ("GRF_OK", "GRF_EINVAL", "GRF_ENOMEM", "GRF_EDEVICE", "GRF_ENOCONV", "GRF_EUNSUP", "GRF_ENONFINITE"):
        assert status[name] == getattr(grf, name), name
    flags = dict((k, int(v)) for k, v in re.findall(r"#define\s+(GRF_[A-Z_]+)\s+(\d+)u", text))
    assert flags["GRF_MESH_ROUND"] == grf.MESH["round"] and flags["GRF_MESH_CEIL"] == grf.MESH["ceil"]
    assert flags["GRF_MASS_CONSISTENT_SYS"] == grf.MASS["consistent"]
    assert flags["GRF_NOISE_CONSISTENT"] == grf.NOISE["consistent"]


def test_opts_defaults():
    o = grf.Opts()
    grf.load().grf_opts_init(C.byref(o))
    assert o.tol == 1e-12 and o.maxit == 10000 and o.precision == 0 and o.precond == 0
    assert o.k_minus == -1 and o.k_plus == -1 and o.sample_offset == 0


@pytest.mark.parametrize("case", ["isolated", "endpoint", "length", "h", "flags", "nan"])
def test_graph_create_rejects_bad_input(case):
    lib = grf.load()
    V, e, L, h, flags = 3, np.array([[0, 1], [1, 2]], dtype=np.int64), np.array([1.0, 0.5]), 0.1, 0
    if case == "isolated":
        V = 4
    elif case == "endpoint":
        e = np.array([[0, 1], [1, 3]], dtype=np.int64)
    elif case == "length":
        L = np.array([1.0, 0.0])
    elif case == "h":
        h = -1.0
    elif case == "flags":
        flags = 8  # no such flag
    elif case == "nan":
        L = np.array([1.0, np.nan])
    out = C.c_void_p()
    rc = lib.grf_graph_create(V, e.shape[0], e.ctypes.data, L.ctypes.data, h, flags, C.byref(out))
    assert rc == grf.GRF_EINVAL
    assert out.value is None
    assert len(lib.grf_last_error()) > 0


def test_null_handles_are_rejected():
    lib = grf.load()
    assert lib.grf_graph_destroy(None) == grf.GRF_OK
    assert lib.grf_sample(None, 1.0, 0.5, 0.3, 1, 0, None, None) == grf.GRF_EINVAL
    assert lib.grf_noise(None, 1, 0, None, None) == grf.GRF_EINVAL
    assert lib.grf_solve_shifted(None, 1.0, 1.0, 1.0, 1, None, None, None) == grf.GRF_EINVAL


def test_class_mode_encoding():
    """pcg_class_modes: GRF_PCG_MODES_SET | (variant of class c) << 2c, decoded back by
    class_modes (3 is reported for classes that run the global-memory kernel)."""
    modes = ["op", "guess", "jacobi", "op", "guess", "jacobi"]
    o = grf.make_opts(pcg_class_modes=modes, stream=False)
    assert o.pcg_class_modes == grf.PCG_MODES_SET | 0 | 1 << 2 | 2 << 4 | 0 << 6 | 1 << 8 | 2 << 10
    assert grf.class_modes(o.pcg_class_modes) == modes
    assert grf.class_modes(3 << 10) == ["op"] * 5 + ["global"]
    assert grf.make_opts(stream=False).pcg_class_modes == 0
    assert grf.make_opts(precond="nn", stream=False).precond == 2


def test_shift_count_bounds():
    """The shift schedule rejects overrides that overflow the shift count or the
    coefficients c_I = pi/(2k sin(pi beta)) e^{-2 beta l k}, c_L = c_I e^{2 l k}."""
    lib = grf.load()
    km, kp, k = C.c_int32(), C.c_int32(), C.c_double()

    def count(k_minus=-1, k_plus=-1, beta=0.75, step=0.5):
        o = grf.make_opts(k_minus=k_minus, k_plus=k_plus, stream=False)
        return lib.grf_shift_count(None, beta, step, C.byref(o), C.byref(km), C.byref(kp), C.byref(k))

    # the paper's rule at k = 0.5, beta = 0.75: K- = ceil(pi^2/(4 k^2 beta)) = 14, K+ = ceil(pi^2/(4 k^2/4)) = 40
    assert count() == grf.GRF_OK and (km.value, kp.value, k.value) == (14, 40, 0.5)
    assert count(k_minus=3, k_plus=5) == grf.GRF_OK and (km.value, kp.value) == (3, 5)
    assert count(k_plus=2 ** 31 - 1) == grf.GRF_EINVAL
    assert count(k_minus=600000, k_plus=600000) == grf.GRF_EINVAL
    # e^{2 y} overflows at y = 1000 * 0.5 ... for l k > 354
    assert count(k_plus=1000) == grf.GRF_EINVAL
    assert b"not finite" in lib.grf_last_error()
    # e^{-2 beta y} overflows for y -> -infinity too
    assert count(k_minus=1000, beta=0.9) == grf.GRF_EINVAL
    assert count(beta=1.0) == grf.GRF_EINVAL
    # without a graph the paper's step rule (quad_step = 0) needs h
    assert count(step=0.0) == grf.GRF_EINVAL


def test_binding_checks_arrays():
    """The binding refuses any array the library would read or write past: the
    wrong dtype, shape, layout or device (checked before any library call)."""
    import torch

    good = torch.zeros((3, 10), dtype=torch.float64)
    with pytest.raises(ValueError, match="float64"):
        grf.check_array(good.float(), 3, 10, "out")
    with pytest.raises(ValueError, match="shape"):
        grf.check_array(good[:2], 3, 10, "out")
    with pytest.raises(ValueError, match="shape"):
        grf.check_array(good.reshape(-1), 3, 10, "out")
    with pytest.raises(ValueError, match="contiguous"):
        grf.check_array(torch.zeros((10, 3), dtype=torch.float64).t(), 3, 10, "out")
    with pytest.raises(ValueError, match="device"):
        grf.check_array(good, 3, 10, "out")
    with pytest.raises(ValueError, match="tensor"):
        grf.check_array(np.zeros((3, 10)), 3, 10, "out")
