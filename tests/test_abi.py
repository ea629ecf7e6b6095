"""The C-ABI library: loads, exports every declared symbol, validates arguments (CPU only)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2511_09165_amd import dmas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmas.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmas_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dmas.LIB_PATH):
        from paper_2511_09165_amd import build
        build.build()
    return dmas.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert set(names) == set(dmas.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in dmas.version()


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, from a C probe compiled against include/dmas.h."""
    src = tmp_path / "probe.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dmas.h"', "int main(void) {",
             f'printf("%zu\\n", sizeof({struct}));']
    lines += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    return vals[0], vals[1:]


@pytest.mark.parametrize("struct,mirror", [("dmas_plan_desc_t", dmas.PlanDesc), ("dmas_plan_info_t", dmas.PlanInfo),
                                           ("dmas_server_desc_t", dmas.ServerDesc),
                                           ("dmas_frame_info_t", dmas.FrameInfo),
                                           ("dmas_server_stats_t", dmas.ServerStats)])
def test_struct_layouts_match_header(lib, tmp_path, struct, mirror):
    """The ctypes mirrors have the C layout: same size and field offsets as the header."""
    fields = [name for name, _ in mirror._fields_]
    size, offsets = _c_layout(struct, fields, tmp_path)
    assert ctypes.sizeof(mirror) == size
    assert [getattr(mirror, f).offset for f in fields] == offsets


def test_desc_defaults(lib):
    d = dmas.PlanDesc()
    assert lib.dmas_plan_desc_init(ctypes.byref(d)) == 0
    assert d.order == 1 and d.use_cf == 1 and d.c == 343.0 and d.cf_eps == 1e-20
    assert d.fir_len == 63 and d.fir_fc == 5000.0 and d.in_dtype == 0 and d.delay_mode == 0


def test_default_lowpass_matches_oracle(lib):
    for L, fc, fs in ((63, 5000.0, 450e3), (31, 10e3, 192e3), (1, 5000.0, 450e3), (255, 5000.0, 450e3)):
        np.testing.assert_allclose(dmas.design_lowpass(L, fc, fs), oracle.lowpass_taps(L, fc, fs),
                                   rtol=1e-6, atol=1e-9)
    with pytest.raises(dmas.DmasError) as e:
        dmas.design_lowpass(64)
    assert e.value.status == 1


def _desc(lib, M=4, D=3, T=100, n=2, **kw):
    d = dmas.PlanDesc()
    lib.dmas_plan_desc_init(ctypes.byref(d))
    mic = np.zeros((M, 3))
    dirs = np.tile([0.0, 0.0, 1.0], (D, 1))
    d.num_mics, d.num_dirs, d.num_samples, d.order, d.fs = M, D, T, n, 450e3
    keep = [mic, dirs]
    d.mic_pos = mic.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.dirs = dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for k, v in kw.items():
        if k == "dirs_array":
            keep.append(v)
            d.dirs = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("field,value", [
    ("order", 5),            # n > M
    ("order", 0),
    ("order", 9),
    ("num_mics", 0),
    ("num_samples", 0),
    ("num_dirs", 0),
    ("fir_len", 64),         # even
    ("fir_len", 257),
    ("fs", 0.0),
    ("c", -1.0),
    ("use_cf", 2),
    ("geometry", 3),
    ("in_dtype", 7),
    ("delay_mode", 2),
    ("ng_fp64", 3),
    ("cf_eps", -1.0),
])
def test_invalid_descriptors_rejected_before_device(lib, field, value):
    d, keep = _desc(lib)
    setattr(d, field, value)
    h = ctypes.c_void_p()
    st = lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h))
    assert st == 1, (field, value, lib.dmas_last_error())
    assert h.value is None
    assert lib.dmas_last_error()


def test_non_unit_direction_and_nan_rejected(lib):
    bad = np.array([[0.0, 0.0, 1.5]] * 3)
    d, keep = _desc(lib, dirs_array=bad)
    h = ctypes.c_void_p()
    assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert b"unit vector" in lib.dmas_last_error()
    nan = np.array([[0.0, np.nan, 1.0]] * 3)
    d, keep = _desc(lib, dirs_array=nan)
    assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.dmas_plan_create(None, ctypes.byref(h)) == 1
    assert lib.dmas_plan_destroy(None) == 0
    assert lib.dmas_beamform(None, None, None, ctypes.c_float(1.0), None) == 1
    assert lib.dmas_envelope(None, None, None, ctypes.c_float(1.0), None) == 1
    assert lib.dmas_envelope_noalloc(None, None, None, ctypes.c_float(1.0), None) == 1
    assert lib.dmas_steering_delays(None, None, None, None) == 1
    assert lib.dmas_plan_query(None, None) == 1
    d, keep = _desc(lib)
    d.mic_pos = None
    assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1


def test_unbuilt_combinations_reported(lib):
    h = ctypes.c_void_p()
    for acc in (1, 2):
        d, keep = _desc(lib, geometry=1, compensated=acc)
        assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 2
        d, keep = _desc(lib, use_cf=0, compensated=acc)
        assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 2
    d, keep = _desc(lib, compensated=3)
    assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert b"compensated" in lib.dmas_last_error()


def test_delay_span_limit(lib):
    """Geometry whose delays would not fit the kernel's integer sample offsets is rejected."""
    far = np.array([[1.0e6, 0.0, 0.0]] * 4)
    d, keep = _desc(lib)
    keep.append(far)
    d.mic_pos = far.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert b"samples of delay" in lib.dmas_last_error()
