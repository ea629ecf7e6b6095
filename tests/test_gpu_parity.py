"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (see tests/_parity.py): T1 peak-normalised <= 1e-4, T2 per-pixel
rounding bound from the oracle's conditioning diagnostics, T3 envelope dB
deviation. Integer work (steering delays) is compared bit for bit.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from _parity import check_t1, check_t2, check_t3, env_bound, root_rel_error, y_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _plan(frame, **kw):
    from paper_2511_09165_amd import plan_for_frame
    return plan_for_frame(frame, **kw)


def _run(frame, x32, env=False, taps=None, rows=None, **kw):
    """GPU image (float64 copy), restricted to ``rows`` if given."""
    with _plan(frame, fir_taps=taps, **kw) as plan:
        x = torch.from_numpy(np.ascontiguousarray(x32)).cuda()
        out = plan.envelope(x) if env else plan.beamform(x)
        torch.cuda.synchronize()
        out = out if rows is None else out[torch.as_tensor(rows, device="cuda")]
        return out.cpu().numpy().astype(np.float64)


def _compare(frame, x32, rows=None, check_env=True, taps=None, t2=True, interp=False, **kw):
    n, M = frame.order, frame.num_mics
    x64 = x32.astype(np.float64) if x32.dtype != np.float64 else x32
    y_ref, dg = oracle.frame_rows(frame, x=x64, rows=rows, diag=True, interp=interp)
    y = _run(frame, x32, rows=rows, linear=interp, **kw)
    e1 = check_t1(y, y_ref)
    worst = None
    if t2:
        tol = y_bound(dg, M, n, frame.use_cf, root_rel_error(x64))
        worst = check_t2(y, y_ref, tol)
    res = dict(t1=e1, t2=worst)
    if check_env:
        taps = oracle.lowpass_taps(63, 5000.0, frame.fs) if taps is None else taps
        taps32 = np.asarray(taps, dtype=np.float32)
        env_ref = oracle.envelope(y_ref, taps32.astype(np.float64))
        env = _run(frame, x32, env=True, taps=taps32, rows=rows, linear=interp, **kw)
        res["env_t1"] = check_t1(env, env_ref)
        if t2:
            res["env_t2"] = check_t2(env, env_ref, env_bound(tol, np.abs(y_ref), taps32, oracle.envelope))
        res["env_db"] = check_t3(env, env_ref)
    return res


# ---------------------------------------------------------------------------
# Steering delays: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["ertis_far", "nearfield_near", "random_far_linear", "random_near_linear"])
def test_steering_delays_bit_exact(case):
    _say(f"delays {case}")
    if case == "ertis_far":
        f = synth.ertis_frame()
        linear = False
    elif case == "nearfield_near":
        f = synth.nearfield_frame(voxels=(32, 32, 8))
        linear = False
    else:
        f = synth.random_frame(np.random.default_rng(3), 37, 300, 64, 3, nearfield=case.endswith("near_linear"))
        linear = True
    with _plan(f, linear=linear) as plan:
        whole, frac = plan.steering_delays()
        torch.cuda.synchronize()
        whole, frac = whole.cpu().numpy(), frac.cpu().numpy()
    if linear:
        w_ref, f_ref = oracle.delays_frac(f.mic_pos, f.dirs, f.fs, f.c, f.nearfield)
        assert np.array_equal(whole, w_ref.astype(np.int32))
        assert np.array_equal(frac, f_ref.astype(np.float32))
    else:
        d_ref = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c, f.nearfield)
        assert np.array_equal(whole, d_ref.astype(np.int32))
        assert np.all(frac == 0)


def test_delays_at_rounding_ties():
    """Geometry where fs*tau + 1/2 fused into one FMA would round to the other sample: the delay
    table and the beamformer's own delays both follow the unfused IEEE sequence of the oracle."""
    from _parity import delay_rounding_ties
    ties = delay_rounding_ties()
    mic = np.array([[x, 0.0, 0.0] for x, _, _ in ties])
    rng = np.random.default_rng(41)
    dirs = np.vstack([[1.0, 0.0, 0.0], synth.unit_vectors(rng.uniform(-80, 80, 20), rng.uniform(-20, 20, 20))])
    f = synth.Frame(name="delay-ties", x=rng.standard_normal((len(ties), 700)), mic_pos=mic, dirs=dirs, fs=450e3, c=343.0,
                    order=3, use_cf=False, nearfield=False)
    _say(f"delay ties M={len(ties)}")
    with _plan(f) as plan:
        whole, _ = plan.steering_delays()
        whole = whole.cpu().numpy()
    d_ref = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c)
    assert np.array_equal(whole, d_ref.astype(np.int32))
    assert [int(v) for v in whole[0]] == [u for _, u, _ in ties]
    # a one-sample slip of any microphone would move this noise image by far more than T1
    _compare(f, f.x_f32(), check_env=False, t2=False)


# ---------------------------------------------------------------------------
# Whole images at small sizes (several tiles, ragged tails)
# ---------------------------------------------------------------------------

def test_burst_frame_parity():
    """Order-2 DMAS+CF, 8 mics, 64 azimuths, 1024 samples: every pixel, RF and envelope."""
    f = synth.burst_frame()
    _say("burst frame n=2 cf")
    res = _compare(f, f.x_f32())
    _say(f"burst frame {res}")


@pytest.mark.parametrize("nearfield", [False, True])
@pytest.mark.parametrize("use_cf", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_orders(n, use_cf, nearfield):
    rng = np.random.default_rng(100 * n + 10 * use_cf + nearfield)
    f = synth.random_frame(rng, 12, 21, 777, n, nearfield=nearfield, use_cf=use_cf)
    _say(f"orders n={n} cf={use_cf} near={nearfield}")
    _compare(f, f.x_f32())


@pytest.mark.parametrize("nearfield", [False, True])
def test_microphone_blocks(nearfield):
    """M = 150 spans three LDS microphone blocks (64 + 64 + 22)."""
    f = synth.random_frame(np.random.default_rng(7), 150, 13, 600, 3, nearfield=nearfield)
    _say(f"mic blocks near={nearfield}")
    _compare(f, f.x_f32())


@pytest.mark.parametrize("M", [24, 150])
@pytest.mark.parametrize("nearfield", [False, True])
@pytest.mark.parametrize("n", [1, 3, 5])
def test_delay_table_matches_per_block_delays(n, nearfield, M, monkeypatch):
    """Plans with whole-sample delays keep per-tile delay tables; the images equal, bit for bit,
    those of a plan that evaluates eq. (1) on the device instead (DMAS_NO_DELAY_TABLE): once per
    workgroup for M <= 64, per microphone block beyond."""
    f = synth.random_frame(np.random.default_rng(8 + n + M), M, 37, 900, n, nearfield=nearfield)
    _say(f"delay table n={n} near={nearfield} M={M}")
    with _plan(f) as plan:
        info = plan.info()
    assert info["delay_table_bytes"] == info["num_tiles"] * M * 9 * 4
    a = _run(f, f.x_f32(), env=True)
    monkeypatch.setenv("DMAS_NO_DELAY_TABLE", "1")
    with _plan(f) as plan:
        assert plan.info()["delay_table_bytes"] == 0
    b = _run(f, f.x_f32(), env=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("mb", [4, 8, 12, 24, 33])
@pytest.mark.parametrize("nearfield", [False, True])
def test_device_delays_any_block_size(mb, nearfield, monkeypatch):
    """Delays evaluated on the device for more microphones than lanes are computed for a group of
    blocks at a time (sixteen to one blocks of mb microphones, the last group partial at M = 150): the
    envelope equals, bit for bit, that of the plan-time tables, and with linear delays that of the
    default block size."""
    f = synth.random_frame(np.random.default_rng(300 + mb + 7 * nearfield), 150, 29, 700, 3, nearfield=nearfield)
    _say(f"device delays mb={mb} near={nearfield}")
    ref = _run(f, f.x_f32(), env=True)
    lin_ref = _run(f, f.x_f32(), env=True, linear=True)
    monkeypatch.setenv("DMAS_MIC_BLOCK", str(mb))
    monkeypatch.setenv("DMAS_NO_DELAY_TABLE", "1")
    with _plan(f) as plan:
        info = plan.info()
        assert info["mics_per_block"] == mb and info["delay_table_bytes"] == 0
    np.testing.assert_array_equal(_run(f, f.x_f32(), env=True), ref)
    np.testing.assert_array_equal(_run(f, f.x_f32(), env=True, linear=True), lin_ref)


@pytest.mark.parametrize("M", [32, 100])
@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_table_layouts_give_the_same_bits(n, M, monkeypatch):
    """Every way a kernel can read the delay tables and place the envelope rings gives the same
    envelope bit for bit: offsets one microphone ahead or a block at a time, rings per wave or in
    the window region, and delays evaluated on the device instead; and it agrees with the oracle (T1)."""
    f = synth.random_frame(np.random.default_rng(90 + 7 * n + M), M, 45, 1300, n)
    _say(f"table layouts n={n} M={M}")
    ref = _run(f, f.x_f32(), env=True)
    combos = [{"DMAS_RING_SHARING": "0"}, {"DMAS_RING_SHARING": "1"}, {"DMAS_NO_DELAY_TABLE": "1"}]
    if M <= 64:
        combos.append({"DMAS_BLOCK_TABLES": "0"})
    lds = {}
    for env in combos:
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        with _plan(f) as plan:
            lds[tuple(env.items())] = plan.info()["lds_bytes"]
        got = _run(f, f.x_f32(), env=True)
        for k in env:
            monkeypatch.delenv(k)
        assert np.array_equal(got, ref), env
    # the two ring layouts really are different launches
    assert lds[(("DMAS_RING_SHARING", "0"),)] != lds[(("DMAS_RING_SHARING", "1"),)]
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32).astype(np.float64)
    check_t1(ref, oracle.envelope(oracle.frame_rows(f, x=f.x_f32().astype(np.float64)), taps))


@pytest.mark.parametrize("M,D,T,n", [(1, 1, 1, 1), (3, 1, 2, 3), (5, 9, 63, 2), (8, 8, 255, 5), (8, 8, 256, 5),
                                     (8, 8, 257, 5), (9, 17, 513, 4), (6, 3, 1000, 6)])
def test_edge_sizes(M, D, T, n):
    f = synth.random_frame(np.random.default_rng(M * 1000 + D * 10 + T), M, D, T, n)
    _say(f"edge M={M} D={D} T={T} n={n}")
    _compare(f, f.x_f32())


@pytest.mark.parametrize("T", [1, 2, 3])
def test_tiny_records_at_broadside(T):
    """Records of 1-3 samples with every delay zero (microphones on the z axis, broadside direction)."""
    rng = np.random.default_rng(T)
    M = 4
    mic = np.zeros((M, 3))
    f = synth.Frame("tiny", rng.standard_normal((M, T)), mic, np.array([[0.0, 0.0, 1.0]] * 3), 450e3, 343.0,
                    3, True, False)
    res = _compare(f, f.x_f32())


def test_zero_and_constant_channels():
    """All-zero input gives 0 (CF guard); identical channels at broadside give C(M,n)|x|."""
    M, T = 16, 300
    mic = synth.disc_array(np.random.default_rng(1), M, 0.1)
    dirs = np.array([[0.0, 0.0, 1.0], [0.3, 0.0, np.sqrt(1 - 0.09)]])
    f = synth.Frame("zeros", np.zeros((M, T)), mic, dirs, 450e3, 343.0, 5, True, False)
    assert np.all(_run(f, f.x_f32()) == 0.0)
    assert np.all(_run(f, f.x_f32(), env=True) == 0.0)
    row = np.random.default_rng(2).standard_normal(T)
    f.x = np.tile(row, (M, 1))
    y = _run(f, f.x_f32())
    want = math.comb(16, 5) * row.astype(np.float32).astype(np.float64)  # C(M,n) sgn(x)^5 |x|
    np.testing.assert_allclose(y[0], want, rtol=2e-5)


# ---------------------------------------------------------------------------
# Full-size workloads in the benchmark's launch configuration, sampled rows
# ---------------------------------------------------------------------------

def _sample_rows(f, k, seed):
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(f.num_dirs, size=k, replace=False).tolist())
    rows.update([0, f.num_dirs - 1])
    return sorted(rows)


def test_ertis_frame_full_size_sampled_rows():
    """eRTIS-like frame: M=32, D=4186, T=16384, order 5 + CF; full launch, oracle on sampled rows."""
    f = synth.ertis_frame()
    rows = _sample_rows(f, 22, 5)
    # also the direction with the strongest DAS response (a bright pixel)
    das = oracle.dmas_rows(f.x, f.mic_pos, f.dirs, f.fs, f.c, 1, use_cf=False, rows=rows)
    _say(f"eRTIS-like frame full size, rows {rows[:4]}...")
    res = _compare(f, f.x_f32(), rows=rows)
    _say(f"eRTIS-like frame {res} (das peak {np.abs(das).max():.3g})")


@pytest.mark.parametrize("n", [2, 3, 7, 8])
def test_ertis_frame_other_orders_full_size_sampled_rows(n):
    """The eRTIS-like frame at other orders, full launch, oracle on sampled rows. Each order takes a
    different kernel layout: orders 2 and 3 the per-block tables with the rings in the window region
    (four workgroups per CU), order 7 per-block tables with per-wave rings, order 8 tables read one
    microphone ahead."""
    f = synth.ertis_frame(order=n)
    rows = _sample_rows(f, 8, 40 + n)
    _say(f"eRTIS-like frame order {n} full size, rows {rows[:4]}...")
    res = _compare(f, f.x_f32(), rows=rows)
    _say(f"eRTIS-like frame order {n} {res}")


def test_nearfield_frame_full_size_sampled_rows():
    """Near field: M=1024 (16 LDS blocks), 64x64x32 voxels, T=2048, order 3 + CF; oracle on sampled rows."""
    f = synth.nearfield_frame()
    rows = _sample_rows(f, 10, 6)
    _say(f"near-field frame full size, rows {rows[:4]}...")
    res = _compare(f, f.x_f32(), rows=rows, taps=oracle.lowpass_taps(63, 5000.0, f.fs))
    _say(f"near-field frame {res}")


def test_ertis_frame_linear_full_size_sampled_rows():
    """The eRTIS-like frame with linear fractional delays (bench.py --workload linear); sampled rows."""
    f = synth.ertis_frame()
    rows = _sample_rows(f, 12, 7)
    _say(f"eRTIS-like frame linear full size, rows {rows[:4]}...")
    res = _compare(f, f.x_f32(), rows=rows, interp=True, t2=False)
    _say(f"eRTIS-like frame linear {res}")


def test_pipeline_full_size_sampled_rows():
    """Raw eRTIS-like frame -> matched filter -> order-5 DMAS+CF -> envelope every 20th sample
    (bench.py --workload pipeline) against the same chain in the oracle on sampled rows."""
    f = synth.ertis_frame(matched=False)
    pulse = f.truth["pulse"].astype(np.float32)
    raw32 = f.x_f32()
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
    rows = _sample_rows(f, 12, 8)
    _say(f"pipeline full size, rows {rows[:4]}...")
    with _plan(f, mf_pulse=pulse, fir_taps=taps, env_decimation=20) as plan:
        x = plan.matched_filter(torch.from_numpy(raw32).cuda())
        env = plan.envelope(x)
        torch.cuda.synchronize()
        env = env[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    x_ref = oracle.matched_filter(raw32.astype(np.float64), pulse.astype(np.float64))
    env_ref = oracle.envelope(oracle.frame_rows(f, x=x_ref, rows=rows), taps.astype(np.float64))[:, ::20]
    assert env.shape == env_ref.shape
    _say(f"pipeline t1 {check_t1(env, env_ref):.3g}")


# ---------------------------------------------------------------------------
# Invariants (bitwise)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5])
def test_sign_flip_bitwise(n):
    """S(-x) = (-1)^n S(x) bit for bit (every term has degree n; the envelope sees |y|)."""
    f = synth.random_frame(np.random.default_rng(50 + n), 16, 24, 900, n)
    x = f.x_f32()
    y = _run(f, x)
    yn = _run(f, -x)
    assert np.array_equal(yn, (-1) ** n * y)
    assert np.array_equal(_run(f, x, env=True), _run(f, -x, env=True))


def test_power_of_two_scale_bitwise():
    """in_scale multiplies the result; a power of two is exact."""
    f = synth.random_frame(np.random.default_rng(60), 10, 16, 500, 3)
    x = torch.from_numpy(f.x_f32()).cuda()
    with _plan(f) as plan:
        a = plan.beamform(x).cpu().numpy()
        b = plan.beamform(x, in_scale=4.0).cpu().numpy()
    assert np.array_equal(b, 4.0 * a)


def test_determinism_and_streams():
    """Same bits on repeated runs and on two concurrent streams sharing one plan."""
    f = synth.random_frame(np.random.default_rng(61), 24, 40, 2000, 5)
    x = torch.from_numpy(f.x_f32()).cuda()
    with _plan(f) as plan:
        ref = plan.envelope(x).cpu().numpy()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            a = plan.envelope(x, stream=s1)
        with torch.cuda.stream(s2):
            b = plan.envelope(x, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), ref) and np.array_equal(b.cpu().numpy(), ref)


def _shifted(x, k):
    """Every channel delayed by k samples: xs[:, t] = x[:, t - k], zero before sample k."""
    xs = np.zeros_like(x)
    xs[:, k:] = x[:, :x.shape[1] - k]
    return xs


@pytest.mark.parametrize("k", [1, 37, 64, 1000])
@pytest.mark.parametrize("nearfield", [False, True])
def test_time_shift_bitwise(k, nearfield):
    """Shifting every channel by k samples shifts the RF image by k bit for bit, wherever neither
    image reads a delayed sample outside the record (eq. (1): pixel (t, p) reads m_i(t + d_ip) only)."""
    f = synth.random_frame(np.random.default_rng(70 + k), 20, 30, 2100, 5, nearfield=nearfield)
    _say(f"time shift k={k} near={nearfield}")
    x = f.x_f32()
    y = _run(f, x)
    ys = _run(f, _shifted(x, k))
    d = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c, f.nearfield)
    lo, hi = k - int(d.min()), f.num_samples - int(d.max())
    assert hi - lo > 1000
    np.testing.assert_array_equal(ys[:, lo:hi], y[:, lo - k:hi - k])


@pytest.mark.parametrize("k", [256, 768])
def test_time_shift_envelope_bitwise(k, monkeypatch):
    """With one time segment per tile the envelope FIR groups its products by the output's position
    within a 256-sample chunk, so a shift by a multiple of 256 moves the envelope bit for bit in the
    interior (where the FIR window of both images stays inside the shift-covariant RF interior)."""
    monkeypatch.setenv("DMAS_SEGMENT", "4096")
    f = synth.random_frame(np.random.default_rng(80 + k), 20, 30, 3000, 3)
    _say(f"envelope time shift k={k}")
    x = f.x_f32()
    e = _run(f, x, env=True)
    es = _run(f, _shifted(x, k), env=True)
    d = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c, f.nearfield)
    H = 31
    lo, hi = k - int(d.min()) + H, f.num_samples - int(d.max()) - H
    assert hi - lo > 1000
    np.testing.assert_array_equal(es[:, lo:hi], e[:, lo - k:hi - k])
    check_t1(es, oracle.envelope(oracle.frame_rows(f, x=_shifted(x, k).astype(np.float64)),
                                 oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32).astype(np.float64)))


@pytest.mark.parametrize("n", [2, 3, 5, 8])
@pytest.mark.parametrize("use_cf", [False, True])
def test_n_minus_one_channels_cancel(n, use_cf):
    """Exactly n - 1 non-zero channels: E_n has no term without a zero root (eq. (5)), so the exact
    image is 0; the Newton-Girard evaluation leaves only rounding, within the per-pixel bound T2."""
    rng = np.random.default_rng(90 + n)
    f = synth.random_frame(rng, 16, 24, 900, n, use_cf=use_cf)
    keep = rng.choice(16, size=n - 1, replace=False)
    mask = np.zeros((16, 1))
    mask[keep] = 1.0
    f.x = f.x * mask
    x32 = f.x_f32()
    x64 = x32.astype(np.float64)
    _say(f"n-1 channels n={n} cf={use_cf}")
    y_ref, dg = oracle.frame_rows(f, x=x64, diag=True)
    assert np.all(y_ref == 0.0)
    y = _run(f, x32)
    tol = y_bound(dg, 16, n, use_cf, root_rel_error(x64))
    worst = check_t2(y, y_ref, tol)
    env = _run(f, x32, env=True)
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
    check_t2(env, np.zeros_like(env), env_bound(tol, np.abs(y_ref), taps, oracle.envelope))
    _say(f"n-1 channels n={n} cf={use_cf}: worst |y| at {worst:.3g} of its bound, max |y| {np.abs(y).max():.3g}")


def _with_subnormals(rng, x, frac=0.3):
    """FP32 channels with a fraction of the samples replaced by values below the normal range,
    each channel's replaced samples at one random exponent in [-149, -127]."""
    x = x.astype(np.float32).copy()
    for i in range(x.shape[0]):
        pick = rng.random(x.shape[1]) < frac
        mag = np.float32(2.0 ** rng.integers(-149, -126)) * rng.uniform(1.0, 2.0, pick.sum()).astype(np.float32)
        x[i, pick] = np.copysign(mag, rng.standard_normal(pick.sum())).astype(np.float32)
    assert np.any((x != 0) & (np.abs(x) < np.float32(2.0 ** -126)))
    return x


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_subnormal_samples(n):
    """Channels mixing normal and subnormal samples, and channels of subnormal samples only: the root
    pass takes every finite sample's root per eq. (4), so the image matches the oracle on the same
    FP32 values within T1 and T2 (with the root error bound at the smallest exponent present)."""
    rng = np.random.default_rng(110 + n)
    f = synth.random_frame(rng, 12, 21, 700, n)
    x32 = _with_subnormals(rng, f.x_f32())
    x32[:3] = _with_subnormals(rng, np.zeros((3, 700)), frac=1.0)   # three channels below the normal range only
    _say(f"subnormal samples n={n}")
    res = _compare(f, x32)
    _say(f"subnormal samples n={n}: {res}")
    # a frame of subnormal samples only (no CF, so the image is not squared away): still eq. (4)
    f.use_cf = False
    tiny = _with_subnormals(rng, np.zeros((12, 700)), frac=1.0)
    y_ref = oracle.frame_rows(f, x=tiny.astype(np.float64))
    assert np.abs(y_ref).max() > 0
    res = _compare(f, tiny, check_env=False)
    _say(f"subnormal-only frame n={n}: {res}")


def test_subnormal_samples_linear_delays():
    """Linear delays take a root per microphone and pixel without the subnormal step: an interpolated
    value below 2^-126 enters the root as 0. On a frame mixing normal and subnormal samples that stays
    within T1 of the oracle."""
    rng = np.random.default_rng(120)
    f = synth.random_frame(rng, 12, 21, 700, 3)
    x32 = _with_subnormals(rng, f.x_f32())
    _say("subnormal samples, linear delays")
    res = _compare(f, x32, interp=True, t2=False)
    _say(f"subnormal samples linear: {res}")


# ---------------------------------------------------------------------------
# Precision forms and linear delays
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("env", [False, True])
def test_graph_capture_replays(env):
    """dmas_beamform / dmas_envelope captured in a HIP graph (the root plane's stream-ordered pool
    allocation, the root pass, the beamformer and the free): every replay, with eager work between
    replays, gives the eager result bit for bit."""
    f = synth.random_frame(np.random.default_rng(5), 16, 40, 700, 5)
    _say(f"graph capture env={env}")
    with _plan(f) as plan:
        run = plan.envelope if env else plan.beamform
        x = torch.from_numpy(f.x_f32()).cuda()
        out = torch.empty((f.num_dirs, f.num_samples), device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            run(x, out=out)
            torch.cuda.synchronize()
            ref = out.clone()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                run(x, out=out, stream=s)
        torch.cuda.synchronize()
        for _ in range(4):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            run(x, out=torch.empty_like(out))   # eager work between replays
            torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_precision_storage(dtype):
    """FP16/BF16 channels with a per-frame scale: parity against the oracle on the dequantised values."""
    f = synth.precision_frame(order=5)
    tdt = torch.float16 if dtype == "f16" else torch.bfloat16
    amax = np.abs(f.x).max()
    scale = 2.0 ** np.floor(np.log2(amax / 16384.0)) if dtype == "f16" else 1.0
    xq = torch.from_numpy(f.x / scale).to(tdt)
    x_deq = xq.float().numpy().astype(np.float64) * scale
    rows = list(range(f.num_dirs))
    y_ref, dg = oracle.frame_rows(f, x=x_deq, diag=True)
    with _plan(f, in_dtype=dtype) as plan:
        y = plan.beamform(xq.cuda(), in_scale=scale).cpu().numpy().astype(np.float64)
    check_t1(y, y_ref)
    check_t2(y, y_ref, y_bound(dg, f.num_mics, 5, True, root_rel_error(x_deq)))
    assert rows


@pytest.mark.parametrize("variant", [dict(ng_fp64=True), dict(compensated=True),
                                     dict(ng_fp64=True, compensated=True), dict(accumulate="f64")])
@pytest.mark.parametrize("n", [2, 5, 7])
def test_precision_variants(n, variant):
    f = synth.precision_frame(order=n)
    _say(f"precision n={n} {variant}")
    _compare(f, f.x_f32(), **variant)


@pytest.mark.parametrize("dtype,variant", [("f32", dict(accumulate="f64")), ("f32", dict(compensated=True)),
                                           ("f16", dict(ng_fp64=True)), ("bf16", dict())])
def test_precision_forms_full_size_sampled_rows(dtype, variant):
    """The precision forms at the eRTIS-like frame's full size, as bench.py --workload precision times
    them (order 5, CF, envelope): oracle on sampled rows of the same (dequantised) channel values."""
    f = synth.ertis_frame()
    rows = _sample_rows(f, 8, 9)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    amax = np.abs(f.x_f32()).max()
    scale = 2.0 ** np.floor(np.log2(amax / 16384.0)) if dtype == "f16" else 1.0
    xq = torch.from_numpy(f.x_f32() / np.float32(scale)).to(tdt)
    x_deq = xq.float().numpy().astype(np.float64) * scale
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
    _say(f"precision full size {dtype} {variant}")
    with _plan(f, in_dtype=dtype, fir_taps=taps, **variant) as plan:
        env = plan.envelope(xq.cuda(), in_scale=scale)
        torch.cuda.synchronize()
        env = env[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    env_ref = oracle.envelope(oracle.frame_rows(f, x=x_deq, rows=rows), taps.astype(np.float64))
    _say(f"precision full size {dtype} {variant} t1 {check_t1(env, env_ref):.3g}")


@pytest.mark.parametrize("nearfield", [False, True])
@pytest.mark.parametrize("n", [1, 3, 5])
def test_linear_delays(n, nearfield):
    """Linear fractional delays (interpolation between the two neighbouring samples)."""
    f = synth.random_frame(np.random.default_rng(70 + n), 14, 19, 640, n, nearfield=nearfield)
    _say(f"linear n={n} near={nearfield}")
    _compare(f, f.x_f32(), interp=True, t2=False)


def test_bad_inputs_rejected():
    from paper_2511_09165_amd import DmasError
    f = synth.random_frame(np.random.default_rng(80), 4, 3, 50, 2)
    with _plan(f) as plan:
        with pytest.raises(ValueError):
            plan.beamform(torch.zeros((4, 50), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            plan.beamform(torch.zeros((4, 49), dtype=torch.float32, device="cuda"))
        with pytest.raises(DmasError):
            plan.beamform(torch.zeros((4, 50), dtype=torch.float32, device="cuda"), in_scale=0.0)


# ---------------------------------------------------------------------------
# Steps either side of the beamformer: matched filter and envelope decimation
# ---------------------------------------------------------------------------

def _raw_frame(M=16, D=60, T=3000, n=3, seed=90):
    rng = np.random.default_rng(seed)
    mics = synth.disc_array(rng, M, 0.1)
    dirs = synth.az_el_grid(np.linspace(-60, 60, D // 3), [-10.0, 0.0, 10.0])
    return synth.echo_frame(rng, mics, dirs, T, 6, n, r_range=(0.3, 1.2), apply_matched_filter=False)


def test_matched_filter_parity():
    """GPU pulse compression vs the oracle: per element |d| <= 2 (P + 2) u sum_k |m[t+k] p[k]|."""
    f = _raw_frame()
    pulse = f.truth["pulse"].astype(np.float32)
    raw32 = f.x_f32()
    with _plan(f, mf_pulse=pulse) as plan:
        got = plan.matched_filter(torch.from_numpy(raw32).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.matched_filter(raw32.astype(np.float64), pulse.astype(np.float64))
    scale = oracle.matched_filter(np.abs(raw32.astype(np.float64)), np.abs(pulse.astype(np.float64)))
    bound = 2 * (pulse.size + 2) * 2.0 ** -24 * scale + 1e-30
    assert np.all(np.abs(got - ref) <= bound), float((np.abs(got - ref) / bound).max())
    check_t1(got, ref, tol=1e-5)


@pytest.mark.parametrize("M,T,P", [(3, 1000, 1), (2, 2100, 2500), (1, 700, 4200), (5, 4097, 5), (4, 1024, 64),
                                   (2, 3000, 8192)])
def test_matched_filter_shapes(M, T, P):
    """Pulse lengths 1 .. DMAS_MAX_MF_LEN (several pieces of taps), records not a multiple of the
    1024-output workgroup or of 4 (unaligned rows), against the oracle within the dot-product bound."""
    rng = np.random.default_rng(1000 + P + T)
    raw32 = rng.normal(size=(M, T)).astype(np.float32)
    pulse = rng.normal(size=P).astype(np.float32)
    mics = synth.disc_array(rng, M, 0.05)
    _say(f"matched filter M={M} T={T} P={P}")
    from paper_2511_09165_amd import Plan
    with Plan(mics, synth.az_el_grid(np.array([0.0]), np.array([0.0])), T, 1, 450e3, mf_pulse=pulse) as plan:
        got = plan.matched_filter(torch.from_numpy(raw32).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.matched_filter(raw32.astype(np.float64), pulse.astype(np.float64))
    scale = oracle.matched_filter(np.abs(raw32.astype(np.float64)), np.abs(pulse.astype(np.float64)))
    bound = 2 * (P + 2) * 2.0 ** -24 * scale + 1e-30
    assert np.all(np.abs(got - ref) <= bound), float((np.abs(got - ref) / bound).max())


def test_matched_filter_full_frame_sampled():
    """The 32 x 16384 eRTIS-like raw frame with its 450-sample chirp: sampled channels vs the oracle."""
    f = synth.ertis_frame()
    pulse = synth.linear_chirp(f.fs, 25e3, 75e3, 1e-3).astype(np.float32)
    rng = np.random.default_rng(1100)
    raw32 = rng.normal(size=(f.num_mics, f.num_samples)).astype(np.float32)
    rows = [0, 7, 31]
    _say("matched filter full frame")
    with _plan(f, mf_pulse=pulse) as plan:
        got = plan.matched_filter(torch.from_numpy(raw32).cuda()).cpu().numpy().astype(np.float64)[rows]
    sub = raw32[rows].astype(np.float64)
    ref = oracle.matched_filter(sub, pulse.astype(np.float64))
    scale = oracle.matched_filter(np.abs(sub), np.abs(pulse.astype(np.float64)))
    bound = 2 * (pulse.size + 2) * 2.0 ** -24 * scale + 1e-30
    assert np.all(np.abs(got - ref) <= bound), float((np.abs(got - ref) / bound).max())


@pytest.mark.parametrize("n", [3, 5])
def test_raw_to_envelope_pipeline(n):
    """raw -> matched filter -> DMAS-n+CF -> envelope on the GPU vs the same chain in the oracle."""
    f = _raw_frame(n=n, seed=91 + n)
    pulse = f.truth["pulse"].astype(np.float32)
    raw32 = f.x_f32()
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
    with _plan(f, mf_pulse=pulse, fir_taps=taps) as plan:
        x = plan.matched_filter(torch.from_numpy(raw32).cuda())
        env = plan.envelope(x).cpu().numpy().astype(np.float64)
    x_ref = oracle.matched_filter(raw32.astype(np.float64), pulse.astype(np.float64))
    env_ref = oracle.envelope(oracle.frame_rows(f, x=x_ref), taps.astype(np.float64))
    check_t1(env, env_ref)


@pytest.mark.parametrize("k", [2, 7, 16])
def test_envelope_decimation(k):
    """Every k-th envelope sample: the full-rate envelope's exactly (the same FIR), and the oracle's within T1."""
    f = synth.random_frame(np.random.default_rng(95 + k), 24, 30, 5000, 5)
    taps = oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32)
    full = _run(f, f.x_f32(), env=True, taps=taps)
    dec = _run(f, f.x_f32(), env=True, taps=taps, env_decimation=k)
    assert dec.shape == (f.num_dirs, -(-f.num_samples // k))
    np.testing.assert_array_equal(dec, full[:, ::k])
    env_ref = oracle.envelope(oracle.frame_rows(f, x=f.x_f32().astype(np.float64)), taps.astype(np.float64))
    check_t1(dec, env_ref[:, ::k])


@pytest.mark.parametrize("T,k", [(700, 700), (700, 699), (33, 5), (1, 1), (2, 2), (300, 256)])
def test_decimation_extremes(T, k):
    """Decimation up to k = T (one kept sample per direction) and records shorter than the FIR:
    the kept samples are the full-rate envelope's, bitwise."""
    f = synth.random_frame(np.random.default_rng(700 + T + k), 6, 11, T, 3)
    _say(f"decimation T={T} k={k}")
    full = _run(f, f.x_f32(), env=True)
    dec = _run(f, f.x_f32(), env=True, env_decimation=k)
    assert dec.shape == (f.num_dirs, -(-T // k))
    np.testing.assert_array_equal(dec, full[:, ::k])


@pytest.mark.parametrize("T", [1000, 997])
@pytest.mark.parametrize("L", [1, 3, 5, 7, 9, 61, 63, 65, 127, 255])
def test_envelope_fir_lengths(L, T):
    """Envelope with arbitrary odd-length taps (both residues of (L-1)/2 mod 2, L mod 4 all classes),
    on records whose rows are and are not 16-byte aligned in the output."""
    f = synth.random_frame(np.random.default_rng(200 + L), 12, 21, T, 3)
    taps = np.random.default_rng(300 + L).normal(size=L).astype(np.float32)
    _say(f"fir L={L} T={T}")
    env = _run(f, f.x_f32(), env=True, taps=taps)
    y_ref = oracle.frame_rows(f, x=f.x_f32().astype(np.float64))
    env_ref = oracle.envelope(y_ref, taps.astype(np.float64))
    check_t1(env, env_ref)
    dec = _run(f, f.x_f32(), env=True, taps=taps, env_decimation=3)
    np.testing.assert_array_equal(dec, env[:, ::3])   # the same FIR, only every 3rd sample kept


@pytest.mark.parametrize(
    "L,T,seg",
    [(255, 997, 32), (255, 997, 96), (127, 1000, 160), (63, 2048, 2240), (63, 2048, 992), (31, 700, 160),
     (1, 300, 64), (63, 33, 32)],
)
def test_envelope_segment_walks(L, T, seg, monkeypatch):
    """Envelope over forced segment lengths: segments that start before the FIR lead (walk clipped
    at sample 0), envelope-only passes after the last computed chunk, one-segment records."""
    monkeypatch.setenv("DMAS_SEGMENT", str(seg))
    f = synth.random_frame(np.random.default_rng(500 + L + T), 12, 21, T, 3)
    taps = np.random.default_rng(600 + L).normal(size=L).astype(np.float32)
    _say(f"segment walk L={L} T={T} seg={seg}")
    with _plan(f, fir_taps=taps) as plan:
        assert plan.info()["segment"] == seg
    env = _run(f, f.x_f32(), env=True, taps=taps)
    y_ref = oracle.frame_rows(f, x=f.x_f32().astype(np.float64))
    env_ref = oracle.envelope(y_ref, taps.astype(np.float64))
    check_t1(env, env_ref)
    dec = _run(f, f.x_f32(), env=True, taps=taps, env_decimation=5)
    np.testing.assert_array_equal(dec, env[:, ::5])


@pytest.mark.parametrize("seed", list(range(24)))
def test_random_configurations(seed):
    """Random combinations of the plan's options (sizes, order, CF, geometry, delay mode, accumulation,
    FIR length, decimation) against the oracle: envelope within T1, and the RF image within T1."""
    rng = np.random.default_rng(4000 + seed)
    M = int(rng.integers(1, 100))
    n = int(rng.integers(1, min(8, M) + 1))
    near = bool(rng.random() < 0.3)
    f = synth.random_frame(rng, M, int(rng.integers(1, 200)), int(rng.integers(1, 2500)), n, nearfield=near)
    f.use_cf = bool(rng.random() < 0.8)
    linear = bool(rng.random() < 0.2)
    acc = "f32"
    if f.use_cf and not near and not linear and rng.random() < 0.3:
        acc = str(rng.choice(["kahan", "f64"]))
    L = int(rng.choice([1, 3, 31, 63, 127]))
    dec = int(rng.choice([1, 1, 1, 3, 8]))
    taps = rng.normal(size=L).astype(np.float32)
    _say(f"random #{seed}: M={M} D={f.num_dirs} T={f.num_samples} n={n} cf={f.use_cf} near={near} "
         f"linear={linear} acc={acc} L={L} dec={dec}")
    kw = dict(linear=linear, accumulate=acc)
    y = _run(f, f.x_f32(), **kw)
    env = _run(f, f.x_f32(), env=True, taps=taps, env_decimation=dec, **kw)
    y_ref = oracle.frame_rows(f, x=f.x_f32().astype(np.float64), interp=linear)
    env_ref = oracle.envelope(y_ref, taps.astype(np.float64))[:, ::dec]
    assert env.shape == env_ref.shape
    check_t1(y, y_ref)
    check_t1(env, env_ref)


@pytest.mark.parametrize("seed", list(range(12)))
def test_random_storage_and_precision(seed):
    """Random plans over input storage (FP32, FP16 with a power-of-two scale, BF16) and FP64
    Newton-Girard, with random sizes, order, CF, geometry, delay mode, FIR length and decimation:
    image and envelope within T1 of the oracle on the dequantised input."""
    rng = np.random.default_rng(7000 + seed)
    M = int(rng.integers(2, 90))
    n = int(rng.integers(2, min(8, M) + 1))
    near = bool(rng.random() < 0.3)
    f = synth.random_frame(rng, M, int(rng.integers(1, 150)), int(rng.integers(1, 2000)), n, nearfield=near)
    f.use_cf = bool(rng.random() < 0.8)
    linear = bool(f.use_cf and rng.random() < 0.25)
    dtype = str(rng.choice(["f32", "f16", "bf16"]))
    ng = bool(rng.random() < 0.5)
    L = int(rng.choice([1, 7, 63]))
    dec = int(rng.choice([1, 2, 5]))
    taps = rng.normal(size=L).astype(np.float32)
    _say(f"random storage #{seed}: M={M} D={f.num_dirs} T={f.num_samples} n={n} cf={f.use_cf} near={near} "
         f"linear={linear} dtype={dtype} ng_fp64={ng} L={L} dec={dec}")
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    amax = float(np.abs(f.x).max())
    scale = 2.0 ** np.floor(np.log2(amax / 16384.0)) if dtype == "f16" else 1.0
    xq = torch.from_numpy(f.x / scale).to(tdt)
    x_deq = xq.float().numpy().astype(np.float64) * scale
    with _plan(f, in_dtype=dtype, ng_fp64=ng, linear=linear, fir_taps=taps, env_decimation=dec) as plan:
        xd = xq.cuda()
        y = plan.beamform(xd, in_scale=scale).cpu().numpy().astype(np.float64)
        env = plan.envelope(xd, in_scale=scale).cpu().numpy().astype(np.float64)
    y_ref = oracle.frame_rows(f, x=x_deq, interp=linear)
    env_ref = oracle.envelope(y_ref, taps.astype(np.float64))[:, ::dec]
    check_t1(y, y_ref)
    check_t1(env, env_ref)


def test_bad_output_buffers_rejected():
    """Output tensors of the wrong shape, type, layout or device are refused before any launch."""
    f = synth.random_frame(np.random.default_rng(97), 8, 5, 100, 2)
    pulse = np.ones(7, dtype=np.float32)
    with _plan(f, mf_pulse=pulse) as plan:
        x = torch.zeros((8, 100), dtype=torch.float32, device="cuda")
        for bad in (torch.zeros((8, 99), device="cuda"), torch.zeros((8, 100), dtype=torch.float64, device="cuda"),
                    torch.zeros((100, 8), device="cuda").t(), torch.zeros((8, 100))):
            with pytest.raises(ValueError):
                plan.matched_filter(x, out=bad)
        for bad in (torch.zeros((5, 99), device="cuda"), torch.zeros((5, 100), dtype=torch.float16, device="cuda")):
            with pytest.raises(ValueError):
                plan.beamform(x, out=bad)
            with pytest.raises(ValueError):
                plan.envelope(x, out=bad)


def test_plan_rejects_bad_pipeline_options():
    from paper_2511_09165_amd import DmasError
    f = synth.random_frame(np.random.default_rng(96), 8, 5, 100, 2)
    with pytest.raises(DmasError):
        _plan(f, env_decimation=101)
    with _plan(f) as plan:
        with pytest.raises(DmasError):
            plan.matched_filter(torch.zeros((8, 100), dtype=torch.float32, device="cuda"))


@pytest.mark.parametrize("pick", [0, 1, 2])
def test_serving_mix_full_size_sampled_rows(pick):
    """Full-size frames of the serving mix (16/32/64 mics, up to 8192 x 16384), oracle on sampled rows."""
    rng = np.random.default_rng(200 + pick)
    M, D, T, n = [(64, 8192, 16384, 5), (16, 1024, 16384, 3), (32, 4096, 8192, 3)][pick]
    dia = [0.20, 0.06, 0.12][pick]
    mics = synth.disc_array(rng, M, dia, min_spacing=0.003)
    n_el = {8192: 64, 1024: 16, 4096: 32}[D]
    dirs = synth.az_el_grid(np.linspace(-90, 90, D // n_el), np.linspace(-45, 45, n_el))
    f = synth.echo_frame(rng, mics, dirs, T, 10, n)
    rows = _sample_rows(f, 8, 300 + pick)
    _say(f"serving-mix frame M={M} D={D} T={T} n={n}")
    res = _compare(f, f.x_f32(), rows=rows)
    _say(f"serving-mix frame {res}")
