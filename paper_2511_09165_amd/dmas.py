"""ctypes binding of libdmas.so (the C ABI in include/dmas.h).

Argument marshalling only: every step of the beamformer runs in the HIP
kernels of libdmas.so. PyTorch supplies device memory and the current HIP
stream. If the library is missing this module raises; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmas.so")

DMAS_OK = 0
STATUS_NAMES = {0: "DMAS_OK", 1: "DMAS_ERR_INVALID_ARG", 2: "DMAS_ERR_UNSUPPORTED",
                3: "DMAS_ERR_OUT_OF_MEMORY", 4: "DMAS_ERR_DEVICE", 5: "DMAS_ERR_BUSY", 6: "DMAS_ERR_TIMEOUT"}
SUBMIT_ENVELOPE = 1
SUBMIT_AUTO_RELEASE = 2
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
ACCUMULATE = {"f32": 0, "kahan": 1, "f64": 2}   # dmas_accumulate_t
EXPORTED = ("dmas_plan_desc_init", "dmas_plan_create", "dmas_plan_destroy", "dmas_plan_query",
            "dmas_beamform", "dmas_envelope", "dmas_envelope_noalloc", "dmas_steering_delays",
            "dmas_design_lowpass", "dmas_matched_filter", "dmas_last_error", "dmas_version",
            "dmas_server_clock", "dmas_server_create", "dmas_server_submit", "dmas_server_query",
            "dmas_server_wait", "dmas_server_release", "dmas_server_fetch", "dmas_server_completed",
            "dmas_server_drain", "dmas_server_stats", "dmas_server_destroy")


class DmasError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("num_mics", ctypes.c_int32), ("num_samples", ctypes.c_int32), ("num_dirs", ctypes.c_int32),
        ("order", ctypes.c_int32), ("use_cf", ctypes.c_int32), ("geometry", ctypes.c_int32),
        ("mic_pos", ctypes.POINTER(ctypes.c_double)), ("dirs", ctypes.POINTER(ctypes.c_double)),
        ("fs", ctypes.c_double), ("c", ctypes.c_double), ("cf_eps", ctypes.c_double),
        ("fir_taps", ctypes.POINTER(ctypes.c_float)), ("fir_len", ctypes.c_int32), ("fir_fc", ctypes.c_double),
        ("in_dtype", ctypes.c_int32), ("ng_fp64", ctypes.c_int32), ("compensated", ctypes.c_int32),
        ("delay_mode", ctypes.c_int32), ("env_decimation", ctypes.c_int32),
        ("mf_pulse", ctypes.POINTER(ctypes.c_float)), ("mf_len", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "num_mics", "num_samples", "num_dirs", "order", "dirs_per_tile", "num_tiles", "samples_per_lane",
        "chunk", "segment", "num_segments", "window_halo", "mics_per_block", "lds_bytes", "fir_len")]
    _fields_ += [("workgroups", ctypes.c_int64), ("delay_table_bytes", ctypes.c_int64),
                 ("device_bytes", ctypes.c_int64)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("staging_bytes", ctypes.c_int64),
                ("num_streams", ctypes.c_int32), ("max_batch_frames", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FrameInfo(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("state", ctypes.c_int32), ("batch_frames", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double), ("d_out", ctypes.c_void_p), ("pixels", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "failed", "launches", "batched_frames", "queued", "admitted_not_launched",
        "in_flight", "hbm_in_use", "hbm_peak", "hbm_budget", "resident_launches", "resident_frames")]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libdmas.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(p)
    st = ctypes.c_int
    vp = ctypes.c_void_p
    lib.dmas_plan_desc_init.argtypes = [ctypes.POINTER(PlanDesc)]
    lib.dmas_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    lib.dmas_plan_destroy.argtypes = [vp]
    lib.dmas_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.dmas_beamform.argtypes = [vp, vp, vp, ctypes.c_float, vp]
    lib.dmas_envelope.argtypes = [vp, vp, vp, ctypes.c_float, vp]
    lib.dmas_envelope_noalloc.argtypes = [vp, vp, vp, ctypes.c_float, vp]
    lib.dmas_steering_delays.argtypes = [vp, vp, vp, vp]
    lib.dmas_matched_filter.argtypes = [vp, vp, vp, vp]
    lib.dmas_matched_filter.restype = st
    lib.dmas_design_lowpass.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_float)]
    for name in ("dmas_plan_desc_init", "dmas_plan_create", "dmas_plan_destroy", "dmas_plan_query",
                 "dmas_beamform", "dmas_envelope", "dmas_envelope_noalloc", "dmas_steering_delays",
                 "dmas_design_lowpass"):
        getattr(lib, name).restype = st
    lib.dmas_server_clock.restype = ctypes.c_double
    lib.dmas_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(vp)]
    lib.dmas_server_submit.argtypes = [vp, vp, vp, ctypes.c_float, ctypes.c_int32, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.dmas_server_query.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(FrameInfo)]
    lib.dmas_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(FrameInfo)]
    lib.dmas_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.dmas_server_fetch.argtypes = [vp, ctypes.c_uint64, vp]
    lib.dmas_server_completed.argtypes = [vp, ctypes.POINTER(FrameInfo), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.dmas_server_drain.argtypes = [vp, ctypes.c_double]
    lib.dmas_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.dmas_server_destroy.argtypes = [vp]
    for name in ("dmas_server_create", "dmas_server_submit", "dmas_server_query", "dmas_server_wait",
                 "dmas_server_release", "dmas_server_fetch", "dmas_server_completed", "dmas_server_drain",
                 "dmas_server_stats", "dmas_server_destroy"):
        getattr(lib, name).restype = st
    lib.dmas_last_error.restype = ctypes.c_char_p
    lib.dmas_version.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(status: int) -> None:
    if status != DMAS_OK:
        msg = load_library().dmas_last_error().decode(errors="replace")
        raise DmasError(status, msg)


def version() -> str:
    return load_library().dmas_version().decode()


def design_lowpass(num_taps: int = 63, cutoff_hz: float = 5000.0, fs: float = 450e3) -> np.ndarray:
    """The library's default envelope low-pass (host-side design)."""
    out = np.zeros(num_taps, dtype=np.float32)
    _check(load_library().dmas_design_lowpass(int(num_taps), float(cutoff_hz), float(fs),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Plan:
    """A beamforming plan: geometry and taps resident on the current device.

    Parameters follow ``dmas_plan_desc_t``. ``mic_pos`` is (M, 3) metres;
    ``dirs`` is (D, 3) unit vectors (far field) or voxel centres (near field).
    ``accumulate`` is "f32", "kahan" or "f64" (``compensated=True`` is "kahan").
    """

    def __init__(self, mic_pos, dirs, num_samples: int, order: int, fs: float, c: float = 343.0,
                 use_cf: bool = True, nearfield: bool = False, fir_taps=None, fir_len: int = 63,
                 fir_fc: float = 5000.0, in_dtype: str = "f32", ng_fp64: bool = False,
                 compensated: bool = False, linear: bool = False, cf_eps: float = 1e-20,
                 env_decimation: int = 1, mf_pulse=None, accumulate: Optional[str] = None):
        lib = load_library()
        self._lib = lib
        self._handle = ctypes.c_void_p()
        mic = np.ascontiguousarray(np.asarray(mic_pos, dtype=np.float64))
        dv = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64))
        if mic.ndim != 2 or mic.shape[1] != 3 or dv.ndim != 2 or dv.shape[1] != 3:
            raise ValueError("mic_pos and dirs must be (N, 3)")
        if in_dtype not in DTYPES:
            raise ValueError(f"in_dtype must be one of {sorted(DTYPES)}")
        d = PlanDesc()
        _check(lib.dmas_plan_desc_init(ctypes.byref(d)))
        d.num_mics, d.num_samples, d.num_dirs = mic.shape[0], int(num_samples), dv.shape[0]
        d.order, d.use_cf, d.geometry = int(order), int(bool(use_cf)), int(bool(nearfield))
        d.mic_pos = mic.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.dirs = dv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.fs, d.c, d.cf_eps = float(fs), float(c), float(cf_eps)
        taps = None
        if fir_taps is not None:
            taps = np.ascontiguousarray(np.asarray(fir_taps, dtype=np.float32))
            d.fir_taps = taps.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            d.fir_len = taps.size
        else:
            d.fir_len = int(fir_len)
        d.fir_fc = float(fir_fc)
        d.in_dtype = DTYPES[in_dtype]
        if accumulate is None:
            accumulate = "kahan" if compensated else "f32"
        elif compensated and accumulate != "kahan":
            raise ValueError("compensated=True asks for accumulate='kahan'")
        if accumulate not in ACCUMULATE:
            raise ValueError(f"accumulate must be one of {sorted(ACCUMULATE)}")
        d.ng_fp64, d.compensated, d.delay_mode = int(bool(ng_fp64)), ACCUMULATE[accumulate], int(bool(linear))
        d.env_decimation = int(env_decimation)
        pulse = None
        if mf_pulse is not None:
            pulse = np.ascontiguousarray(np.asarray(mf_pulse, dtype=np.float32))
            d.mf_pulse = pulse.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            d.mf_len = pulse.size
        _check(lib.dmas_plan_create(ctypes.byref(d), ctypes.byref(self._handle)))
        self.env_decimation = max(1, int(env_decimation))
        self.env_samples = -(-int(num_samples) // self.env_decimation)
        self.num_mics, self.num_samples, self.num_dirs = d.num_mics, d.num_samples, d.num_dirs
        self.order, self.in_dtype = int(order), in_dtype
        self.use_cf, self.nearfield, self.linear = bool(use_cf), bool(nearfield), bool(linear)

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            self._lib.dmas_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        return int(self._handle.value or 0)

    def info(self) -> dict:
        inf = PlanInfo()
        _check(self._lib.dmas_plan_query(self._handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in PlanInfo._fields_}

    # -- launches -----------------------------------------------------------
    def _check_input(self, x):
        import torch
        want = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.in_dtype]
        if not x.is_cuda or x.dtype != want or tuple(x.shape) != (self.num_mics, self.num_samples) \
                or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous {want} device tensor of shape "
                             f"({self.num_mics}, {self.num_samples}); got {x.dtype} {tuple(x.shape)}")
        # the library checks that the current device is the plan's; the data must be there too
        if x.device.index != torch.cuda.current_device():
            raise ValueError(f"x is on {x.device} but device {torch.cuda.current_device()} is current")

    def _out(self, x, out, samples=None):
        import torch
        shape = (self.num_dirs, self.num_samples if samples is None else samples)
        if out is None:
            return torch.empty(shape, dtype=torch.float32, device=x.device)
        if out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous() \
                or out.device != x.device:
            raise ValueError(f"out must be a contiguous float32 {shape} tensor on the input's device")
        return out

    def beamform(self, x, out=None, in_scale: float = 1.0, stream=None):
        """DMAS-n (+CF) image, (D, T) float32."""
        self._check_input(x)
        out = self._out(x, out)
        _check(self._lib.dmas_beamform(self._handle, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), float(in_scale),
                                       ctypes.c_void_p(_stream_handle(stream))))
        return out

    def envelope(self, x, out=None, in_scale: float = 1.0, stream=None):
        """DMAS-n (+CF) image followed by the envelope filter, (D, ceil(T / env_decimation)) float32."""
        self._check_input(x)
        out = self._out(x, out, self.env_samples)
        _check(self._lib.dmas_envelope(self._handle, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), float(in_scale),
                                       ctypes.c_void_p(_stream_handle(stream))))
        return out

    def envelope_noalloc(self, x, out, in_scale: float = 1.0, stream=None):
        """``envelope`` through dmas_envelope_noalloc: the root plane lives in the library's fixed
        per-device scratch, so the call allocates nothing; ``out`` must be given. Calls that
        overlap on one device race on that scratch."""
        self._check_input(x)
        out = self._out(x, out, self.env_samples)
        _check(self._lib.dmas_envelope_noalloc(self._handle, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), float(in_scale),
                                               ctypes.c_void_p(_stream_handle(stream))))
        return out

    def matched_filter(self, raw, out=None, stream=None):
        """Pulse compression of raw (M, T) float32 device channels with the plan's pulse."""
        import torch
        if not raw.is_cuda or raw.dtype != torch.float32 or tuple(raw.shape) != (self.num_mics, self.num_samples) \
                or not raw.is_contiguous():
            raise ValueError("raw must be a contiguous float32 (M, T) device tensor")
        if raw.device.index != torch.cuda.current_device():
            raise ValueError(f"raw is on {raw.device} but device {torch.cuda.current_device()} is current")
        if out is None:
            out = torch.empty_like(raw)
        elif out.dtype != torch.float32 or tuple(out.shape) != tuple(raw.shape) or not out.is_contiguous() \
                or out.device != raw.device:
            raise ValueError("out must be a contiguous float32 (M, T) tensor on raw's device")
        _check(self._lib.dmas_matched_filter(self._handle, ctypes.c_void_p(raw.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(_stream_handle(stream))))
        return out

    def steering_delays(self, stream=None):
        """(whole, frac) device tensors of shape (D, M): the delays the kernels use."""
        import torch
        whole = torch.empty((self.num_dirs, self.num_mics), dtype=torch.int32, device="cuda")
        frac = torch.empty((self.num_dirs, self.num_mics), dtype=torch.float32, device="cuda")
        _check(self._lib.dmas_steering_delays(self._handle, ctypes.c_void_p(whole.data_ptr()),
                                              ctypes.c_void_p(frac.data_ptr()),
                                              ctypes.c_void_p(_stream_handle(stream))))
        return whole, frac


def plan_for_frame(frame, **kw) -> Plan:
    """Plan for a ``synth.Frame``-like object (mic_pos, dirs, fs, c, order, use_cf, nearfield)."""
    args = dict(mic_pos=frame.mic_pos, dirs=frame.dirs, num_samples=frame.num_samples, order=frame.order,
                fs=frame.fs, c=frame.c, use_cf=frame.use_cf, nearfield=frame.nearfield)
    args.update(kw)
    return Plan(**args)


def server_clock() -> float:
    return float(load_library().dmas_server_clock())


class Server:
    """Continuous-batching request loop on the current device (dmas_server_* in include/dmas.h).

    ``hbm_budget`` bytes of device memory hold admitted frames' inputs and
    outputs; frames are queued by ``submit`` and launched in multi-frame
    batches of up to ``max_batch`` on ``num_streams`` streams
    (``max_batch=1, num_streams=1`` gives one plain launch per frame); with
    ``resident=True`` the frames that have a resident worker are served by one.
    """

    def __init__(self, hbm_budget: int, staging: int = 0, num_streams: int = 2, max_batch: int = 64,
                 resident: bool = False):
        self._lib = load_library()
        d = ServerDesc(int(hbm_budget), int(staging), int(num_streams), int(max_batch), int(bool(resident)), 0)
        self._h = ctypes.c_void_p()
        self._shapes = {}   # ticket -> result shape, for frames whose result stays on the device
        # the library keeps a pointer to each frame's plan: hold the Plan objects until the
        # server is closed, so that a frame in flight never outlives its plan by garbage collection
        self._plans = {}
        _check(self._lib.dmas_server_create(ctypes.byref(d), ctypes.byref(self._h)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dmas_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._plans = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, plan: Plan, x: np.ndarray, in_scale: float = 1.0, envelope: bool = True,
               auto_release: bool = False, arrival: float = -1.0) -> int:
        """Queue a frame (host array of the plan's dtype, shape (M, T)); returns its ticket."""
        want = {"f32": np.float32, "f16": np.float16, "bf16": np.uint16}[plan.in_dtype]
        xa = np.ascontiguousarray(x)
        if xa.dtype != want or xa.shape != (plan.num_mics, plan.num_samples):
            raise ValueError(f"x must be a contiguous {np.dtype(want)} array of shape "
                             f"({plan.num_mics}, {plan.num_samples})")
        flags = (SUBMIT_ENVELOPE if envelope else 0) | (SUBMIT_AUTO_RELEASE if auto_release else 0)
        self._plans[id(plan)] = plan
        t = ctypes.c_uint64()
        _check(self._lib.dmas_server_submit(self._h, ctypes.c_void_p(plan.handle),
                                            xa.ctypes.data_as(ctypes.c_void_p), float(in_scale), flags,
                                            float(arrival), ctypes.byref(t)))
        if not auto_release:
            # the result's shape, for fetch: the library copies the whole result
            self._shapes[int(t.value)] = (plan.num_dirs, plan.env_samples if envelope else plan.num_samples)
        return int(t.value)

    def query(self, ticket: int) -> dict:
        info = FrameInfo()
        _check(self._lib.dmas_server_query(self._h, ticket, ctypes.byref(info)))
        return info.as_dict()

    def wait(self, ticket: int, timeout: float = 60.0) -> dict:
        info = FrameInfo()
        _check(self._lib.dmas_server_wait(self._h, ticket, float(timeout), ctypes.byref(info)))
        return info.as_dict()

    def fetch(self, ticket: int, shape=None) -> np.ndarray:
        """The done frame's result as a (D, T) float32 array ((D, ceil(T / k)) for an envelope
        decimated by k); ``shape``, if given, must be that shape."""
        want = self._shapes.get(int(ticket))
        if want is None:
            raise ValueError(f"no result to fetch for ticket {ticket} (unknown, released or auto-released)")
        if shape is not None and tuple(shape) != want:
            raise ValueError(f"the result of ticket {ticket} has shape {want}, not {tuple(shape)}")
        out = np.empty(want, dtype=np.float32)
        _check(self._lib.dmas_server_fetch(self._h, ticket, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def release(self, ticket: int) -> None:
        _check(self._lib.dmas_server_release(self._h, ticket))
        self._shapes.pop(int(ticket), None)

    def completed(self, max_records: int = 4096) -> list:
        buf = (FrameInfo * max_records)()
        n = ctypes.c_int32()
        _check(self._lib.dmas_server_completed(self._h, buf, max_records, ctypes.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def drain(self, timeout: float = 300.0) -> None:
        _check(self._lib.dmas_server_drain(self._h, float(timeout)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.dmas_server_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}
