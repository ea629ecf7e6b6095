"""Throughput benchmark: order-5 DMAS + CF + envelope on an eRTIS-like frame.

Workload (one "step" = one pass of the whole path over one frame): 32
microphones in a 12 cm sparse planar aperture, 91 x 46 azimuth/elevation
directions (2 deg steps), 16384 samples at 450 kHz of matched-filtered chirp
echoes from 20 reflectors (synthetic, seeded). One step is one
dmas_envelope() call: steering delays, channel staging, signed roots, power
sums, Newton-Girard, coherence factor, envelope FIR and store, all in one
kernel. Inputs are resident in HBM before the timed region.

Prints one JSON line: throughput in direction*samples/s, the dominant kernel's
roofline position (VALU issue bound; the envelope FIR, which runs on the matrix
cores, as its own leg), the FP64 CPU oracle timed on a sample of the same
workload, a short serving run (Poisson arrivals of mixed frames at 2000
frames/s: p50/p99 frame latency beside throughput), and the same frame and the
1024-microphone near-field frame with steering delays evaluated on the device
instead of read from the plan's tables.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-serving]
"""

from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 VALU lane-instruction
# issue slots per second (the FP32 vector peak of 157.3 TFLOP/s counts an FMA
# as 2 flops and packed dual-FP32 as 2 lanes; packed FP32 is not used here).
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Issue cost of the gfx950 transcendentals (v_exp_f32 / v_log_f32 / v_sqrt_f32)
# in full-rate slots, measured (half rate).
TRANS_SLOTS = 2
# Dense FP32 matrix-core peak of MI355X (published), for the matched filter.
MFMA_F32_FLOPS = 157.3e12


def mic_slots(n: int, cf: bool) -> int:
    """VALU issue slots per microphone per output pixel for order n (the method's minimum).

    With whole-sample delays the signed root of a delayed sample is the root of
    a channel sample, so roots are counted once per channel sample
    (``root_slots``), not per pixel. Per microphone and pixel remain: the
    intermediate powers that cannot be fused into an FMA accumulation, n
    power-sum accumulations (P_n is sum x or sum |x|), and for CF sum x^2 (and
    sum x for even n).
    """
    powers = {1: 0, 2: 0, 3: 0, 4: 1, 5: 1, 6: 2, 7: 2, 8: 3}[n]
    accum = n + ((1 + (n % 2 == 0)) if cf else 0)
    return powers + accum


def root_slots(n: int) -> int:
    """Slots per channel sample for its signed n-th root: none (n = 1), sqrt + sign (n = 2),
    log2 + scale + exp2 + sign (n >= 3); transcendentals at TRANS_SLOTS."""
    return 0 if n == 1 else (TRANS_SLOTS + 1 if n == 2 else 2 * TRANS_SLOTS + 2)


def pixel_slots(M: int, n: int, cf: bool) -> int:
    """VALU slots per output pixel: microphone loop + Newton-Girard + CF + scale. The envelope FIR
    runs on the matrix cores and is counted apart (``fir_flops``)."""
    ng = {1: 0, 2: 3, 3: 7, 4: 11, 5: 15, 6: 21, 7: 28, 8: 36}[n]
    cf_ops = (4 + TRANS_SLOTS) if cf else 0      # square, fma, rcp, 2 mul
    return M * mic_slots(n, cf) + ng + cf_ops + 1


def launch_slots(M: int, T: int, D: int, n: int, cf: bool) -> int:
    """Algorithmic VALU slots of one frame: every pixel, plus every channel sample's root."""
    return D * T * pixel_slots(M, n, cf) + M * T * root_slots(n)


def fir_flops(D: int, T_out: int, fir_len: int) -> float:
    """Algorithmic flops of the envelope FIR: fir_len multiply-adds (2 flops) per output."""
    return 2.0 * D * T_out * fir_len


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed (what the compiler sees)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the code (comments and layout ignored) that the headline kernel is built from; the
    committed HBM counter record applies only while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_09165_amd", "csrc")
    for name in ("dmas_api.hip", "dmas_internal.hpp", "dmas_kernel.hpp", "dmas_order5.hip", "dmas_plan.hpp"):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update((name + _code_only(f.read())).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches this kernel."""
    path = os.path.join(ROOT, "profiles", "dmas_envelope_order5_erti32_traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source") != kernel_source_hash() or rec.get("workload") != workload_key:
        return None
    return rec.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frame, fir_len: int, min_seconds: float = 10.0, max_seconds: float = 30.0) -> dict:
    """Time the FP64 oracle (rows + envelope) on the same frame with all its threads: whole frames
    repeated until at least ``min_seconds`` of wall time (a frame that would push the total past
    ``max_seconds`` is not counted); then on one thread over every 64th direction."""
    import oracle
    taps = oracle.lowpass_taps(fir_len, 5000.0, frame.fs)
    x64 = frame.x_f32().astype(np.float64)
    rows = list(range(frame.num_dirs))
    frames, elapsed = 0, 0.0
    while elapsed < min_seconds:
        t0 = time.perf_counter()
        y = oracle.frame_rows(frame, x=x64, rows=rows)
        oracle.envelope(y, taps)
        dt = time.perf_counter() - t0
        if frames and elapsed + dt > max_seconds:
            break
        frames += 1
        elapsed += dt
    threads = oracle.num_threads()
    sub = rows[::64]
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        y = oracle.frame_rows(frame, x=x64, rows=sub)
        oracle.envelope(y, taps)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    pix = frames * frame.num_dirs * frame.num_samples
    return {"value": pix / elapsed, "unit": "direction*samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{frames} whole frames ({frame.num_dirs} directions x {frame.num_samples} samples each), "
                      f"order-5 DMAS+CF+envelope, FP64, {elapsed:.1f} s wall",
            "cpu_model": _cpu_model(),
            "one_thread": {"value": len(sub) * frame.num_samples / dt1, "unit": "direction*samples/s",
                           "sample": f"every 64th direction ({len(sub)}) x {frame.num_samples} samples, "
                                     f"{dt1:.1f} s wall"}}


def _launch_stats(launch, reps: int, stream) -> dict:
    """Per-launch device times (HIP events around each launch on the launch stream)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return {"launches": reps, "median_ms": float(np.median(t)), "mean_ms": float(t.mean()),
            "p95_ms": float(np.percentile(t, 95)), "min_ms": float(t.min()), "max_ms": float(t.max())}


def _timed(launch, steps: int, warmup: int, stream):
    """(wall ms per step, kernel ms per launch from HIP events on the launch stream)."""
    import torch
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall * 1e3 / steps, ev0.elapsed_time(ev1) / steps


def _roofline(slots: int, pixels: int, kernel_ms: float, traffic=None, fir=None) -> dict:
    """VALU-issue roofline of one step: ``slots`` algorithmic slots over the step's kernel time
    (root pass + beamformer, HIP events on the launch stream). ``fir`` = flops of the envelope FIR,
    which runs on the matrix cores, reported against the FP32 matrix-core peak over the same time."""
    achieved = slots / (kernel_ms * 1e-3)
    rec = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_SLOTS_PER_S / 1e12, "unit": "TOP/s",
           "frac": achieved / VALU_SLOTS_PER_S, "traffic": traffic, "kernel_ms": kernel_ms,
           "ops_per_pixel": slots / pixels,
           "op": "VALU lane-instruction issue slot (transcendental = 2); the envelope FIR is not in this count"}
    if traffic is not None:
        rec["traffic_source"] = ("replayed: HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / "
                                 "WRITE_SIZE record (profiles/dmas_envelope_order5_erti32_traffic.txt), "
                                 "valid while the kernel source hashes to the recorded value")
    if fir is not None:
        fa = fir / (kernel_ms * 1e-3)
        rec["mfma_fir"] = {"bound": "mfma", "achieved": fa / 1e12, "peak": MFMA_F32_FLOPS / 1e12,
                           "unit": "TFLOP/s", "frac": fa / MFMA_F32_FLOPS, "flops_per_pixel": fir / pixels,
                           "op": "envelope FIR multiply-add (2 flops) on the FP32 matrix cores, same step time"}
    return rec


def _base_record(args, value, ms_per_step, dtype, config) -> dict:
    return {"metric": "direction*samples/sec, order-5 DMAS+CF, 32 mics", "value": value,
            "unit": "direction*samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic (seeded)", "config": config}


def _settle(launch, stream, ms: float = 250.0, batch: int = 16) -> int:
    """Untimed launches until ``ms`` of device time have passed, so the GPU clocks have ramped up
    before the warmup steps (a handful of steps after plan creation still runs at lower clocks).
    Returns the number of launches (reported in the JSON line as clock_settle)."""
    import torch
    done, t0 = 0, time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(batch):
            launch()
        torch.cuda.synchronize()
        done += batch
    return done


def _computed_delay_ms(frame, fir_len: int, reps: int, stream, x, out) -> dict:
    """Envelope time of the same frame with plan-time delay tables (the default) and with the delays
    of eq. (1) evaluated on the device from the geometry (DMAS_NO_DELAY_TABLE, read at plan creation)."""
    from paper_2511_09165_amd import plan_for_frame
    res = {}
    for key, env in (("table", None), ("computed", "1")):
        old = os.environ.pop("DMAS_NO_DELAY_TABLE", None)
        if env:
            os.environ["DMAS_NO_DELAY_TABLE"] = env
        try:
            with plan_for_frame(frame, fir_len=fir_len) as p:
                info = p.info()
                _settle(lambda: p.envelope(x, out=out), stream, 50.0, batch=min(16, reps))   # clocks, caches
                res[f"{key}_ms"] = _timed(lambda: p.envelope(x, out=out), reps, 2, stream)[1]
                res[f"{key}_delay_table_bytes"] = info["delay_table_bytes"]
        finally:
            os.environ.pop("DMAS_NO_DELAY_TABLE", None)
            if old is not None:
                os.environ["DMAS_NO_DELAY_TABLE"] = old
    res["computed_over_table"] = res["computed_ms"] / res["table_ms"]
    return res


def bench_headline(args) -> dict:
    """Order-5 DMAS + CF + envelope on the eRTIS-like frame (the headline line)."""
    import torch

    import synth
    from paper_2511_09165_amd import plan_for_frame

    frame = synth.ertis_frame()
    M, D, T, n = frame.num_mics, frame.num_dirs, frame.num_samples, frame.order
    fir_len = 63
    plan = plan_for_frame(frame, fir_len=fir_len)
    x = torch.from_numpy(frame.x_f32()).cuda()
    out = torch.empty((D, T), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    settle = _settle(lambda: plan.envelope(x, out=out), stream)
    ms_per_step, kernel_ms = _timed(lambda: plan.envelope(x, out=out), args.steps, args.warmup, stream)
    pixels = D * T
    workload_key = f"ertis32 M={M} D={D} T={T} n={n} cf=1 env L={fir_len}"
    rec = _base_record(args, pixels / (ms_per_step * 1e-3), ms_per_step, "f32", {
        "workload": "eRTIS-like frame: order-5 DMAS+CF+envelope, M=32 mics (12 cm sparse disc), "
                    "91x46 az/el directions, T=16384 samples at 450 kHz, 63-tap envelope FIR",
        "M": M, "D": D, "T": T, "order": n, "cf": True, "fir_len": fir_len})
    rec["data"] = "synthetic (seeded eRTIS-like pulse-echo frame)"
    rec["clock_settle"] = {"launches": settle, "ms": 250,
                           "note": "untimed launches before the warmup steps while the GPU clocks ramp up"}
    rec["roofline"] = _roofline(launch_slots(M, T, D, n, True), pixels, kernel_ms,
                                measured_traffic(workload_key), fir=fir_flops(D, T, fir_len))
    # per-launch statistics of the same call, then the RF image and CF off (the paper's Table III
    # ratio); each of these legs settles the clocks again (plan creation and host waits let them
    # drop) and times at least 100 launches, whatever --steps is
    reps = max(100, args.steps // 2)
    rec["launch_stats"] = _launch_stats(lambda: plan.envelope(x, out=out), reps, stream)
    _settle(lambda: plan.beamform(x, out=out), stream, 50.0)
    extra = {"rf_ms": _timed(lambda: plan.beamform(x, out=out), reps, 2, stream)[1]}
    with plan_for_frame(frame, fir_len=fir_len, use_cf=False) as p2:
        _settle(lambda: p2.envelope(x, out=out), stream, 50.0)
        extra["no_cf_env_ms"] = _timed(lambda: p2.envelope(x, out=out), reps, 2, stream)[1]
    extra["cf_cost"] = kernel_ms / extra["no_cf_env_ms"] - 1.0
    if not args.no_delay_modes:
        extra["delays_erti32"] = _computed_delay_ms(frame, fir_len, reps, stream, x, out)
        near = synth.nearfield_frame()
        xn = torch.from_numpy(near.x_f32()).cuda()
        outn = torch.empty((near.num_dirs, near.num_samples), dtype=torch.float32, device="cuda")
        extra["delays_nearfield1024"] = _computed_delay_ms(near, fir_len, 3, stream, xn, outn)
        del xn, outn
        torch.cuda.empty_cache()
    if args.extra:
        with plan_for_frame(frame, fir_len=fir_len, ng_fp64=True) as p3:
            extra["ng_fp64_env_ms"] = _timed(lambda: p3.envelope(x, out=out), reps, 2, stream)[1]
        extra["plan"] = plan.info()
    rec["extra"] = extra
    plan.close()
    del out
    torch.cuda.empty_cache()
    if not args.no_serving:
        rec["serving"] = serving_summary(args)
    rec["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(frame, fir_len)
    return rec


def bench_nearfield(args) -> dict:
    """Near-field order-3 DMAS + CF + envelope: 1024 microphones, 64 x 64 x 32 voxels, 2048 samples."""
    import torch

    import synth
    from paper_2511_09165_amd import plan_for_frame

    frame = synth.nearfield_frame()
    M, D, T, n = frame.num_mics, frame.num_dirs, frame.num_samples, frame.order
    fir_len = 63
    with plan_for_frame(frame, fir_len=fir_len) as plan:
        x = torch.from_numpy(frame.x_f32()).cuda()
        out = torch.empty((D, T), dtype=torch.float32, device="cuda")
        steps = max(3, args.steps // 10)
        warmup = max(2, args.warmup // 20)
        ms_per_step, kernel_ms = _timed(lambda: plan.envelope(x, out=out), steps, warmup,
                                        torch.cuda.current_stream())
        info = plan.info()
    pixels = D * T
    rec = _base_record(args, pixels / (ms_per_step * 1e-3), ms_per_step, "f32", {
        "workload": "near-field passive imaging: order-3 DMAS+CF+envelope, 32x32 grid M=1024, "
                    "64x64x32 voxels, T=2048 at 192 kHz", "M": M, "D": D, "T": T, "order": n, "cf": True,
        "fir_len": fir_len})
    rec["metric"] = "direction*samples/sec, order-3 DMAS+CF, 1024 mics, near field"
    rec["steps"] = steps
    rec["warmup"] = warmup
    rec["roofline"] = _roofline(launch_slots(M, T, D, n, True), pixels, kernel_ms, fir=fir_flops(D, T, fir_len))
    rec["extra"] = {"plan": info}
    return rec


def linear_pixel_slots(M: int, n: int, cf: bool) -> int:
    """Slots per pixel with linear fractional delays: per microphone the interpolation (subtract,
    FMA) and the signed root of the interpolated value (a root of a channel sample cannot be
    reused), then the same powers and sums, Newton-Girard, CF and scale as ``pixel_slots``."""
    return pixel_slots(M, n, cf) + M * (2 + root_slots(n))


def bench_linear(args) -> dict:
    """Order-5 DMAS + CF + envelope on the eRTIS-like frame with linear fractional delays."""
    import torch

    import synth
    from paper_2511_09165_amd import plan_for_frame

    frame = synth.ertis_frame()
    M, D, T, n = frame.num_mics, frame.num_dirs, frame.num_samples, frame.order
    fir_len = 63
    with plan_for_frame(frame, fir_len=fir_len, linear=True) as plan:
        x = torch.from_numpy(frame.x_f32()).cuda()
        out = torch.empty((D, T), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream()
        steps = max(5, args.steps // 5)
        settle = _settle(lambda: plan.envelope(x, out=out), stream)
        ms_per_step, kernel_ms = _timed(lambda: plan.envelope(x, out=out), steps, args.warmup, stream)
        info = plan.info()
    pixels = D * T
    rec = _base_record(args, pixels / (ms_per_step * 1e-3), ms_per_step, "f32", {
        "workload": "eRTIS-like frame with linear fractional delays: order-5 DMAS+CF+envelope, M=32, "
                    "91x46 az/el directions, T=16384 at 450 kHz, 63-tap envelope FIR",
        "M": M, "D": D, "T": T, "order": n, "cf": True, "fir_len": fir_len, "delays": "linear"})
    rec["metric"] = "direction*samples/sec, order-5 DMAS+CF, 32 mics, linear fractional delays"
    rec["steps"] = steps
    rec["clock_settle"] = {"launches": settle, "ms": 250}
    rec["roofline"] = _roofline(D * T * linear_pixel_slots(M, n, True), pixels, kernel_ms,
                                fir=fir_flops(D, T, fir_len))
    rec["extra"] = {"plan": info}
    return rec


def bench_pipeline(args) -> dict:
    """Raw channels -> matched filter (450-tap chirp) -> order-5 DMAS + CF -> envelope kept every
    20th sample, on the eRTIS-like frame: the steps either side of the beamformer."""
    import torch

    import synth
    from paper_2511_09165_amd import plan_for_frame

    frame = synth.ertis_frame(matched=False)
    M, D, T, n = frame.num_mics, frame.num_dirs, frame.num_samples, frame.order
    fir_len, decim = 63, 20
    pulse = frame.truth["pulse"].astype(np.float32)
    P = pulse.size
    with plan_for_frame(frame, fir_len=fir_len, mf_pulse=pulse, env_decimation=decim) as plan:
        raw = torch.from_numpy(frame.x_f32()).cuda()
        x = torch.empty_like(raw)
        out = torch.empty((D, -(-T // decim)), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream()

        def step():
            plan.matched_filter(raw, out=x)
            plan.envelope(x, out=out)

        steps = max(5, args.steps // 5)
        settle = _settle(step, stream)
        ms_per_step, step_ms = _timed(step, steps, args.warmup, stream)
        mf_ms = _timed(lambda: plan.matched_filter(raw, out=x), steps, 2, stream)[1]
        env_ms = _timed(lambda: plan.envelope(x, out=out), steps, 2, stream)[1]
        info = plan.info()
    pixels = D * T
    env_slots = D * T * pixel_slots(M, n, True) + M * T * root_slots(n)
    rec = _base_record(args, pixels / (ms_per_step * 1e-3), ms_per_step, "f32", {
        "workload": "raw eRTIS-like frame -> matched filter (450-sample 25-75 kHz chirp) -> order-5 DMAS+CF -> "
                    "63-tap envelope kept every 20th sample; M=32, 91x46 directions, T=16384 at 450 kHz",
        "M": M, "D": D, "T": T, "order": n, "cf": True, "fir_len": fir_len, "env_decimation": decim,
        "mf_len": P})
    rec["metric"] = "direction*samples/sec, raw -> matched filter -> order-5 DMAS+CF -> decimated envelope"
    rec["steps"] = steps
    rec["clock_settle"] = {"launches": settle, "ms": 250}
    # the FIR runs at full rate (every sample) on the matrix cores; the algorithmic count keeps
    # only the stored outputs
    rec["roofline"] = _roofline(env_slots, pixels, env_ms, fir=fir_flops(D, -(-T // decim), fir_len))
    mf_flops = 2.0 * M * T * P
    rec["matched_filter"] = {"kernel_ms": mf_ms, "bound": "mfma", "achieved": mf_flops / (mf_ms * 1e-3) / 1e12,
                             "peak": MFMA_F32_FLOPS / 1e12, "unit": "TFLOP/s",
                             "frac": mf_flops / (mf_ms * 1e-3) / MFMA_F32_FLOPS,
                             "op": "FP32 multiply-add of the correlation, 2 flops"}
    rec["extra"] = {"step_kernel_ms": step_ms, "envelope_ms": env_ms, "plan": info}
    return rec


def bench_precision(args) -> list:
    """Throughput of the precision forms at the eRTIS-like frame's shape, orders 2..7."""
    import torch

    import synth
    from paper_2511_09165_amd import plan_for_frame

    base = synth.ertis_frame()
    D, T, M = base.num_dirs, base.num_samples, base.num_mics
    x32 = base.x_f32()
    amax = float(np.abs(x32).max())
    f16_scale = 2.0 ** np.floor(np.log2(amax / 16384.0))
    inputs = {"f32": (torch.from_numpy(x32).cuda(), 1.0),
              "f16": (torch.from_numpy(x32 / f16_scale).to(torch.float16).cuda(), f16_scale),
              "bf16": (torch.from_numpy(x32).to(torch.bfloat16).cuda(), 1.0)}
    out = torch.empty((D, T), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    recs = []
    steps = max(5, args.steps // 5)
    base.order = 5
    with plan_for_frame(base) as plan:     # bring clocks up before the first timed form
        _timed(lambda: plan.envelope(inputs["f32"][0], out=out), 200, 0, stream)
    for n in (2, 3, 4, 5, 6, 7):
        base.order = n
        for dt in ("f32", "f16", "bf16"):
            for acc, ng64 in (("f32", False), ("f32", True), ("kahan", False), ("kahan", True), ("f64", True)):
                xin, sc = inputs[dt]
                with plan_for_frame(base, in_dtype=dt, ng_fp64=ng64, accumulate=acc) as plan:
                    # plan creation idles the GPU: let the clocks come back before timing
                    _settle(lambda: plan.envelope(xin, out=out, in_scale=sc), stream, ms=50.0)
                    # median of three timed runs: a single short run is at the mercy of one stall
                    kms = float(np.median([_timed(lambda: plan.envelope(xin, out=out, in_scale=sc), steps, 2,
                                                  stream)[1] for _ in range(3)]))
                recs.append({"order": n, "storage": dt, "accumulate": acc, "ng_fp64": ng64, "kernel_ms": kms,
                             "value": D * T / (kms * 1e-3)})
    for r in recs:
        plain = next(q for q in recs if q["order"] == r["order"] and q["storage"] == "f32" and not q["ng_fp64"]
                     and q["accumulate"] == "f32")
        r["speedup_vs_plain_f32"] = plain["kernel_ms"] / r["kernel_ms"]
    return recs


SERVING_MODES = {"batched": dict(num_streams=2, max_batch=64),
                 "one_launch_per_frame": dict(num_streams=1, max_batch=1),
                 "resident": dict(num_streams=2, max_batch=64, resident=True)}


def _serve_trace(mode: str, plans, xs, pix, arrivals_gaps, picks, rate: float) -> dict:
    """One server of ``mode`` fed the Poisson trace (gaps between arrivals, pool index per frame).
    Latency = completion - scheduled arrival; throughput and latency count completed frames only,
    failed frames are counted apart."""
    from paper_2511_09165_amd import DmasError, Server, server_clock

    n_frames = len(picks)
    with Server(hbm_budget=64 << 30, staging=2 << 30, **SERVING_MODES[mode]) as srv:
        # warm up every kernel the trace can use: each plan alone, then all at once
        for k in range(len(plans)):
            srv.submit(plans[k], xs[k], envelope=True, auto_release=True)
            srv.drain(600)
        for k in range(len(plans)):
            srv.submit(plans[k], xs[k], envelope=True, auto_release=True)
        srv.drain(600)
        srv.completed(100000)
        st0 = srv.stats()
        launches0 = st0["launches"]
        t0 = server_clock() + 0.05
        arrivals = t0 + np.cumsum(arrivals_gaps)
        busy_retries = 0
        late = []
        gc.collect()
        gc.disable()   # keep collector pauses of the load generator out of the latencies
        try:
            for a, k in zip(arrivals, picks):
                while server_clock() < a:
                    pass
                late.append(server_clock() - a)
                while True:
                    try:
                        srv.submit(plans[k], xs[k], envelope=True, auto_release=True, arrival=float(a))
                        break
                    except DmasError as e:
                        if e.status != 5:
                            raise
                        busy_retries += 1
        finally:
            gc.enable()
        srv.drain(600)
        recs = srv.completed(n_frames + 10)
        st = srv.stats()
    ok = [r for r in recs if r["state"] == 3]
    failed = max(st["failed"] - st0["failed"], len(recs) - len(ok))
    lat = np.array([r["t_done"] - r["t_arrival"] for r in ok]) * 1e3
    slow = sorted(ok, key=lambda r: r["t_done"] - r["t_arrival"])[-3:]
    slowest = [{"ms": round((r["t_done"] - r["t_arrival"]) * 1e3, 2),
                "queued_ms": round((r["t_admit"] - r["t_arrival"]) * 1e3, 2),
                "wait_launch_ms": round((r["t_launch"] - r["t_admit"]) * 1e3, 2),
                "run_ms": round((r["t_done"] - r["t_launch"]) * 1e3, 2),
                "frames_in_launch": r["batch_frames"], "pixels": r["pixels"]} for r in slow]
    done = np.array([r["t_done"] for r in ok])
    ok_pix = float(sum(r["pixels"] for r in ok))
    span = float(done.max() - arrivals[0]) if ok else float("nan")
    return {"workload": "serving", "mode": mode, "offered_frames_per_s": rate, "offered_frames": n_frames,
            "frames": len(ok), "failed": int(failed),
            "achieved_frames_per_s": len(ok) / span, "direction_samples_per_s": ok_pix / span,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "launches": st["launches"] - launches0,
            "mean_frames_per_launch": len(ok) / max(1, st["launches"] - launches0),
            "resident_launches": st["resident_launches"] - st0["resident_launches"],
            "resident_frames": st["resident_frames"] - st0["resident_frames"],
            "hbm_peak_gb": st["hbm_peak"] / 1e9, "busy_retries": busy_retries,
            "client_late_max_ms": float(max(late)) * 1e3, "slowest": slowest}


def _serving_pool(args, orders=(3, 5)):
    import synth
    from paper_2511_09165_amd import plan_for_frame
    pool = synth.serving_pool(n_arrays_per_m=4, max_frames=args.serving_pool, orders=orders)
    plans = [plan_for_frame(f) for f in pool]
    return pool, plans, [f.x_f32() for f in pool], [f.num_dirs * f.num_samples for f in pool]


def serving_summary(args) -> dict:
    """The serving leg of the headline line: the mixed-frame pool (16/32/64 microphones, 1024-8192
    directions, orders 3 and 5, 4096-16384 samples) under Poisson arrivals at 2000 frames/s for
    ``--serving-summary-s`` seconds, through the batched server and through one plain launch per
    frame on the same trace."""
    pool, plans, xs, pix = _serving_pool(args)
    rate = 2000.0
    rng = np.random.default_rng(2511091654)
    n_frames = max(20, int(rate * args.serving_summary_s))
    gaps = rng.exponential(1.0 / rate, size=n_frames)
    picks = rng.integers(0, len(pool), size=n_frames)
    res = {"workload": f"{len(pool)} distinct frames (M in 16/32/64, D 1024-8192, n in 3/5, T 4096-16384, "
                       f"CF, envelope), Poisson arrivals", "offered_frames_per_s": rate,
           "duration_s": args.serving_summary_s, "frames": n_frames, "hbm_budget_gb": 64 * 2**30 / 1e9}
    try:
        for mode in ("batched", "one_launch_per_frame"):
            r = _serve_trace(mode, plans, xs, pix, gaps, picks, rate)
            res[mode] = {k: r[k] for k in ("p50_ms", "p99_ms", "max_ms", "achieved_frames_per_s",
                                           "direction_samples_per_s", "frames", "failed", "launches",
                                           "mean_frames_per_launch", "client_late_max_ms", "busy_retries")}
    finally:
        for p in plans:
            p.close()
    res["p50_ms"] = res["batched"]["p50_ms"]
    res["p99_ms"] = res["batched"]["p99_ms"]
    return res


def bench_serving(args) -> list:
    """Serving: Poisson arrivals of heterogeneous pulse-echo frames; batched server, one launch per frame,
    and resident workers (persistent launches fed by a job queue).

    Frames: arrays of 16/32/64 microphones (6-20 cm discs), az/el grids of
    1024-8192 directions, orders 3 and 5, 4096-16384 samples, FP32, envelope
    output kept on the device (released at completion). Each rate point
    offers ``rate * duration`` frames; latency = completion - scheduled arrival.
    """
    orders = tuple(int(n) for n in args.serving_orders.split(","))
    pool, plans, xs, pix = _serving_pool(args, orders)
    rng = np.random.default_rng(2511091654)
    rates = [float(r) for r in args.serving_rates.split(",")]
    out = []
    try:
        for rate in rates:
            n_frames = max(20, int(rate * args.serving_duration))
            gaps = rng.exponential(1.0 / rate, size=n_frames)
            picks = rng.integers(0, len(pool), size=n_frames)
            for mode in args.serving_modes.split(","):
                out.append(_serve_trace(mode, plans, xs, pix, gaps, picks, rate))
                print(json.dumps(out[-1]), flush=True)
    finally:
        for p in plans:
            p.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200, help="untimed steps first (clocks settle in ~100 ms)")
    ap.add_argument("--serving-rates", default="500,1000,2000,3000,4000", help="offered frames/s (serving)")
    ap.add_argument("--serving-modes", default="batched,one_launch_per_frame,resident",
                    help="servers to compare (serving): batched, one_launch_per_frame, resident")
    ap.add_argument("--serving-orders", default="3,5", help="DMAS orders in the serving pool")
    ap.add_argument("--serving-duration", type=float, default=2.0, help="seconds of arrivals per rate (serving)")
    ap.add_argument("--serving-pool", type=int, default=48, help="distinct frames in the serving pool")
    ap.add_argument("--workload", default="erti32",
                    choices=["erti32", "nearfield", "precision", "serving", "linear", "pipeline"],
                    help="erti32: the headline frame (default); nearfield: 1024-mic voxel imaging; "
                         "precision: FP16/BF16 storage, FP64 Newton-Girard and Kahan sums, orders 2-7; "
                         "linear: the headline frame with linear fractional delays; pipeline: raw channels "
                         "-> matched filter -> DMAS+CF -> decimated envelope")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="headline line without its serving leg")
    ap.add_argument("--serving-summary-s", type=float, default=3.0,
                    help="seconds of 2000 frames/s arrivals in the headline line's serving leg")
    ap.add_argument("--no-delay-modes", action="store_true",
                    help="headline line without the computed-delay timings (plan tables vs eq. (1) on the device)")
    ap.add_argument("--extra", action="store_true", help="also time FP64 Newton-Girard and print the plan")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, --steps times (HBM counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the beamformer shards by direction with no communication, and this "
              "build runs on a single MI355X; use --gpus 1.", file=sys.stderr)
        return 2

    import torch

    from paper_2511_09165_amd import load_library

    load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": args.steps}), flush=True)
        return 0
    if args.workload == "erti32":
        print(json.dumps(bench_headline(args)), flush=True)
    elif args.workload == "nearfield":
        print(json.dumps(bench_nearfield(args)), flush=True)
    elif args.workload == "serving":
        bench_serving(args)
    elif args.workload == "linear":
        print(json.dumps(bench_linear(args)), flush=True)
    elif args.workload == "pipeline":
        print(json.dumps(bench_pipeline(args)), flush=True)
    else:
        for r in bench_precision(args):
            print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
