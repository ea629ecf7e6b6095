"""FP64 CPU oracle for DMAS-n beamforming with coherence-factor weighting.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package to check and time the GPU library. The product
library never imports it, and it imports nothing from the product library.

``liboracle.so`` (built from ``dmas_oracle.c`` by ``oracle/build.py``) holds the
plain evaluation of the paper's definitions; ``newton_girard`` holds the paper's
closed forms (eqs. (3), (5), (8)-(12)) in plain Python, used as independent pins.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from . import newton_girard  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DIAG_FIELDS = ("E", "CF", "h", "sum_x", "sum_x2", "sum_abs")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_delays.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, _i64p]
    lib.oracle_delays_frac.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, _i64p, _dp]
    lib.oracle_dmas_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     _i64p, _dp, _dp]
    lib.oracle_envelope.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
    lib.oracle_lowpass_taps.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
    lib.oracle_matched_filter.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp]
    for f in (lib.oracle_delays, lib.oracle_delays_frac, lib.oracle_dmas_rows,
              lib.oracle_envelope, lib.oracle_lowpass_taps, lib.oracle_matched_filter):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray, typ=_dp):
    return a.ctypes.data_as(typ)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for later oracle calls (timing only; results do not depend on it)."""
    _load().oracle_set_num_threads(int(n))


def delays(mic_pos, dirs, fs: float, c: float, nearfield: bool = False) -> np.ndarray:
    """Whole-sample steering delays floor(fs*tau + 1/2), shape (D, M), eq. (1)."""
    mic = _f64(mic_pos)
    dv = _f64(dirs)
    M, D = mic.shape[0], dv.shape[0]
    out = np.zeros((D, M), dtype=np.int64)
    rc = _load().oracle_delays(M, D, _ptr(mic), _ptr(dv), int(nearfield), fs, c, _ptr(out, _i64p))
    if rc:
        raise ValueError("oracle_delays: invalid arguments")
    return out


def delays_frac(mic_pos, dirs, fs: float, c: float, nearfield: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """Fractional steering delays: (floor(fs*tau), fs*tau - floor(fs*tau)), each (D, M)."""
    mic = _f64(mic_pos)
    dv = _f64(dirs)
    M, D = mic.shape[0], dv.shape[0]
    whole = np.zeros((D, M), dtype=np.int64)
    frac = np.zeros((D, M), dtype=np.float64)
    rc = _load().oracle_delays_frac(M, D, _ptr(mic), _ptr(dv), int(nearfield), fs, c,
                                    _ptr(whole, _i64p), _ptr(frac))
    if rc:
        raise ValueError("oracle_delays_frac: invalid arguments")
    return whole, frac


def dmas_rows(x, mic_pos, dirs, fs: float, c: float, order: int, use_cf: bool = True,
              nearfield: bool = False, rows: Optional[Sequence[int]] = None,
              cf_eps: float = 1e-20, interp: bool = False, diag: bool = False):
    """DMAS-n (+CF) image rows in FP64, eqs. (1), (4)-(6), (13), (14).

    ``x`` is (M, T). Returns ``y`` of shape (len(rows), T) (all D rows by
    default); with ``diag`` also a dict of per-pixel diagnostics
    (E, CF, h, sum_x, sum_x2, sum_abs), each (len(rows), T).
    """
    xv = _f64(x)
    mic = _f64(mic_pos)
    dv = _f64(dirs)
    M, T = xv.shape
    D = dv.shape[0]
    if mic.shape != (M, 3) or dv.shape[1] != 3:
        raise ValueError("shape mismatch")
    r = np.arange(D, dtype=np.int64) if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    y = np.zeros((r.size, T), dtype=np.float64)
    dg = np.zeros((r.size, T, len(DIAG_FIELDS)), dtype=np.float64) if diag else None
    rc = _load().oracle_dmas_rows(M, T, D, _ptr(xv), _ptr(mic), _ptr(dv), int(nearfield), fs, c,
                                  int(order), int(bool(use_cf)), cf_eps, int(bool(interp)),
                                  int(r.size), _ptr(r, _i64p), _ptr(y),
                                  _ptr(dg) if dg is not None else None)
    if rc:
        raise ValueError(f"oracle_dmas_rows failed ({rc})")
    if diag:
        return y, {k: dg[..., j] for j, k in enumerate(DIAG_FIELDS)}
    return y


def envelope(y, taps) -> np.ndarray:
    """Zero-phase FIR envelope of |y| along time: env[t] = sum_k h[k] |y[t + (L-1)/2 - k]|."""
    yv = _f64(y)
    if yv.ndim == 1:
        yv = yv[None, :]
    h = _f64(taps)
    R, T = yv.shape
    out = np.zeros_like(yv)
    rc = _load().oracle_envelope(R, T, _ptr(yv), int(h.size), _ptr(h), _ptr(out))
    if rc:
        raise ValueError("oracle_envelope: invalid arguments (taps must have odd length)")
    return out


def lowpass_taps(num_taps: int = 63, cutoff_hz: float = 5000.0, fs: float = 450e3) -> np.ndarray:
    """Hamming-windowed sinc low-pass, unit DC gain (the oracle's own design)."""
    taps = np.zeros(num_taps, dtype=np.float64)
    rc = _load().oracle_lowpass_taps(int(num_taps), float(cutoff_hz), float(fs), _ptr(taps))
    if rc:
        raise ValueError("oracle_lowpass_taps: invalid arguments")
    return taps


def frame_rows(frame, rows=None, diag: bool = False, interp: bool = False, x=None, cf_eps: float = 1e-20):
    """Convenience: run ``dmas_rows`` on a ``synth.Frame`` (optionally on other channel data ``x``)."""
    return dmas_rows(frame.x if x is None else x, frame.mic_pos, frame.dirs, frame.fs, frame.c,
                     frame.order, frame.use_cf, frame.nearfield, rows=rows, diag=diag,
                     interp=interp, cf_eps=cf_eps)


def matched_filter(raw, pulse) -> np.ndarray:
    """Pulse compression (Section II, pipeline step 1): r[t] = sum_k m[t + k] p[k], m = 0 beyond the record."""
    rv = _f64(raw)
    if rv.ndim == 1:
        rv = rv[None, :]
    pv = _f64(pulse)
    M, T = rv.shape
    out = np.zeros_like(rv)
    rc = _load().oracle_matched_filter(M, T, _ptr(rv), int(pv.size), _ptr(pv), _ptr(out))
    if rc:
        raise ValueError("oracle_matched_filter: invalid arguments")
    return out
