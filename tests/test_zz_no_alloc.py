"""dmas_envelope_noalloc (root plane in the library's fixed per-device scratch) against dmas_envelope.

Both entry points run the same kernels, so the results must agree bit for bit;
the second call of a pair uses a smaller frame, so stale roots left in the
scratch by the first call would show. Calls go through the C ABI (ctypes).
"""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from _parity import check_t1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DMAS_OK, DMAS_ERR_UNSUPPORTED = 0, 2


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _lib():
    from paper_2511_09165_amd import dmas
    return dmas.load_library()


def _stream():
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def _envelopes(plan, x32, in_scale=1.0):
    """(dmas_envelope, dmas_envelope_noalloc) results for the same input, both on the device."""
    lib = _lib()
    x = torch.from_numpy(np.ascontiguousarray(x32)).cuda()
    shape = (plan.num_dirs, plan.env_samples)
    ref = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
    out = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
    h = ctypes.c_void_p(plan.handle)
    st = lib.dmas_envelope(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                           ctypes.c_float(in_scale), _stream())
    assert st == DMAS_OK, lib.dmas_last_error()
    st = lib.dmas_envelope_noalloc(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_float(in_scale), _stream())
    assert st == DMAS_OK, lib.dmas_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    ((32, 96, 4096, 5), (16, 40, 1500, 3)),    # order 5 then a smaller order-3 frame
    ((24, 64, 3000, 3), (8, 24, 700, 2)),      # order 3 then a smaller order-2 frame
])
def test_noalloc_matches_envelope_two_calls(first, second):
    from paper_2511_09165_amd import plan_for_frame
    rng = np.random.default_rng(2511091700)
    for k, (M, D, T, n) in enumerate((first, second)):
        _say(f"noalloc call {k}: M={M} D={D} T={T} n={n}")
        f = synth.random_frame(rng, M, D, T, n)
        x32 = f.x_f32()
        taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
        with plan_for_frame(f, fir_taps=taps) as plan:
            ref, out = _envelopes(plan, x32)
        assert np.isfinite(out).all()
        assert np.array_equal(ref.view(np.uint32), out.view(np.uint32)), f"call {k} differs from dmas_envelope"
        # and the oracle's envelope within T1
        y_ref = oracle.frame_rows(f, x=x32.astype(np.float64))
        env_ref = oracle.envelope(y_ref, taps.astype(np.float64))
        check_t1(out.astype(np.float64), env_ref)


def test_noalloc_half_storage_and_order_one():
    """FP16 storage with a scale (roots of 16-bit samples) and order 1 (no root plane, no scratch)."""
    from paper_2511_09165_amd import plan_for_frame
    rng = np.random.default_rng(2511091701)
    f = synth.random_frame(rng, 20, 48, 2000, 4)
    scale = 2.0 ** -3
    x16 = (f.x / scale).astype(np.float16)
    _say("noalloc f16 M=20 D=48 T=2000 n=4")
    with plan_for_frame(f, in_dtype="f16") as plan:
        ref, out = _envelopes(plan, x16, in_scale=scale)
    assert np.array_equal(ref.view(np.uint32), out.view(np.uint32))
    f1 = synth.random_frame(rng, 12, 30, 900, 1)
    _say("noalloc order 1 M=12 D=30 T=900")
    with plan_for_frame(f1) as plan:
        ref, out = _envelopes(plan, f1.x_f32())
    assert np.array_equal(ref.view(np.uint32), out.view(np.uint32))


def test_noalloc_rejects_planes_beyond_the_scratch():
    """M * T * 8 bytes above DMAS_NOALLOC_SCRATCH_BYTES (16 MiB) is refused before any launch."""
    from paper_2511_09165_amd import plan_for_frame
    rng = np.random.default_rng(2511091702)
    M, T = 64, 32769            # 64 * 32769 * 8 bytes > 16 MiB
    f = synth.random_frame(rng, M, 4, T, 3)
    lib = _lib()
    _say(f"noalloc limit M={M} T={T}")
    with plan_for_frame(f) as plan:
        x = torch.zeros((M, T), dtype=torch.float32, device="cuda")
        out = torch.full((plan.num_dirs, plan.env_samples), 7.0, dtype=torch.float32, device="cuda")
        st = lib.dmas_envelope_noalloc(ctypes.c_void_p(plan.handle), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_float(1.0), _stream())
        torch.cuda.synchronize()
        assert st == DMAS_ERR_UNSUPPORTED
        assert b"scratch" in lib.dmas_last_error()
        assert bool((out == 7.0).all()), "a refused call must not write its output"
