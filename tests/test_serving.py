"""Serving runtime (dmas_server_*): continuous batching of heterogeneous frames.

Every frame must give the same bits alone (a plain dmas_envelope /
dmas_beamform launch) and inside a multi-frame batch, whatever else is in the
mix; admission must respect the HBM budget; rejected requests must not be
queued.
"""

import numpy as np
import pytest

import oracle
import synth
from _parity import check_t1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _mix(seed=0, count=10):
    """Heterogeneous small frames: arrays of 16/32/64 mics, mixed grids, lengths, orders, geometry."""
    rng = np.random.default_rng(seed)
    frames = []
    for k in range(count):
        M = int(rng.choice([16, 32, 64]))
        D = int(rng.integers(40, 400))
        T = int(rng.choice([900, 2048, 3000]))
        n = int(rng.choice([2, 3, 5]))
        near = bool(k % 4 == 3)
        f = synth.random_frame(rng, M, D, T, n, nearfield=near)
        f.env = bool(k % 3 != 1)
        frames.append(f)
    return frames


def _standalone(plan, x32, env):
    x = torch.from_numpy(x32).cuda()
    out = plan.envelope(x) if env else plan.beamform(x)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _run_server(frames, plans, **server_kw):
    from paper_2511_09165_amd import Server
    outs, infos = [], []
    with Server(**server_kw) as srv:
        tickets = [srv.submit(p, f.x_f32(), envelope=f.env) for f, p in zip(frames, plans)]
        for f, p, t in zip(frames, plans, tickets):
            infos.append(srv.wait(t, timeout=120))
            outs.append(srv.fetch(t, (f.num_dirs, p.env_samples if f.env else f.num_samples)))
            srv.release(t)
        stats = srv.stats()
    return outs, infos, stats


def _blocker():
    """A large frame submitted first, so that the small frames behind it queue up and get batched."""
    f = synth.random_frame(np.random.default_rng(99), 32, 4096, 16384, 5)
    f.env = True
    return f


def test_batched_equals_alone_bitwise(monkeypatch):
    from paper_2511_09165_amd import plan_for_frame
    # no small launches beside the blocker: the frames behind it wait for the gate and are packed
    monkeypatch.setenv("DMAS_SMALL_LAUNCH_WGS", "0")
    frames = [_blocker()] + _mix(1, 12)
    plans = [plan_for_frame(f, env_decimation=(4 if k % 5 == 2 else 1)) for k, f in enumerate(frames)]
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    _say("serving: 12 frames, batching server")
    outs, infos, stats = _run_server(frames, plans, hbm_budget=8 << 30, num_streams=2, max_batch=64)
    for k, (a, b) in enumerate(zip(alone, outs)):
        assert np.array_equal(a, b), f"frame {k} differs between alone and batched"
    assert max(i["batch_frames"] for i in infos) > 1, "no batching happened"
    assert stats["completed"] == len(frames) and stats["failed"] == 0
    assert stats["launches"] < len(frames)
    for i in infos:
        assert i["t_arrival"] <= i["t_admit"] <= i["t_launch"] <= i["t_done"]
    # and one of them against the oracle
    f = frames[1]
    y_ref = oracle.frame_rows(f, x=f.x_f32().astype(np.float64))
    if f.env:
        y_ref = oracle.envelope(y_ref, oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32).astype(np.float64))
    check_t1(outs[1].astype(np.float64)[:, :y_ref.shape[1]] if plans[1].env_decimation == 1 else
             outs[1].astype(np.float64), y_ref if plans[1].env_decimation == 1 else y_ref[:, ::plans[1].env_decimation])
    for p in plans:
        p.close()


def test_large_arrays_batched_bitwise(monkeypatch):
    """Frames of more than 64 microphones (delay offsets read per microphone block) in multi-frame
    launches: the same bits as alone, next to frames of 64 or fewer microphones."""
    from paper_2511_09165_amd import plan_for_frame
    monkeypatch.setenv("DMAS_SMALL_LAUNCH_WGS", "0")   # pack the frames that queue behind the blocker
    rng = np.random.default_rng(7)
    frames = [_blocker()]
    # runs of the same kernel class (order, geometry), which the server packs together
    for M, n, near in [(100, 3, False), (150, 3, False), (72, 3, False), (130, 5, True), (100, 5, True),
                       (32, 3, False)]:
        # few directions and samples: frames that do not fill the device alone, so they are packed
        f = synth.random_frame(rng, M, int(rng.integers(8, 24)), int(rng.choice([256, 300])), n,
                               nearfield=near)
        f.env = True
        frames.append(f)
    plans = [plan_for_frame(f) for f in frames]
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    _say("serving: frames of 72-150 microphones, batching server")
    outs, infos, stats = _run_server(frames, plans, hbm_budget=8 << 30, num_streams=2, max_batch=64)
    for k, (a, b) in enumerate(zip(alone, outs)):
        assert np.array_equal(a, b), f"frame {k} differs between alone and batched"
    assert stats["completed"] == len(frames) and stats["failed"] == 0
    assert max(i["batch_frames"] for i in infos[1:]) > 1, "no batching happened"
    for p in plans:
        p.close()


def test_small_frames_start_beside_a_long_one():
    """While a long frame runs its main body, small frames (here at most one device round of
    workgroups) start on the idle stream instead of waiting for it, and give the same bits as alone."""
    from paper_2511_09165_amd import plan_for_frame
    long_frame = synth.random_frame(np.random.default_rng(98), 64, 8192, 16384, 5)
    long_frame.env = True
    rng = np.random.default_rng(11)
    small = []
    for _ in range(6):
        f = synth.random_frame(rng, 16, int(rng.integers(16, 64)), 2048, 3)
        f.env = True
        small.append(f)
    frames = [long_frame] + small
    plans = [plan_for_frame(f) for f in frames]
    for p in plans[1:]:
        assert p.info()["workgroups"] <= 3 * 256, "not a small frame"
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    _say("serving: small frames beside a long one")
    outs, infos, stats = _run_server(frames, plans, hbm_budget=8 << 30, num_streams=2, max_batch=64)
    for k, (a, b) in enumerate(zip(alone, outs)):
        assert np.array_equal(a, b), f"frame {k} differs between alone and beside the long frame"
    assert stats["completed"] == len(frames) and stats["failed"] == 0
    t0, t1 = infos[0]["t_launch"], infos[0]["t_done"]
    early = [i for i in infos[1:] if i["t_done"] < t0 + 0.5 * (t1 - t0)]
    assert early, ("no small frame finished in the first half of the long one", t0, t1,
                   [(i["t_launch"], i["t_done"]) for i in infos[1:]])
    for p in plans:
        p.close()


def test_budget_limits_admission():
    """A budget that holds about two frames: every frame still completes, peak use stays within it."""
    from paper_2511_09165_amd import plan_for_frame
    frames = _mix(2, 8)
    plans = [plan_for_frame(f) for f in frames]
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    # input, root plane ((root, sample) FP32 pairs for n >= 2), output and the plan's device memory
    need = max(f.num_mics * f.num_samples * (4 + (8 if f.order >= 2 else 0)) + f.num_dirs * f.num_samples * 4
               + p.info()["device_bytes"] for f, p in zip(frames, plans))
    budget = 2 * need + 4096
    _say(f"serving: budget {budget} bytes")
    outs, infos, stats = _run_server(frames, plans, hbm_budget=budget, num_streams=2, max_batch=64)
    assert stats["hbm_peak"] <= stats["hbm_budget"]
    assert stats["completed"] == len(frames)
    for a, b in zip(alone, outs):
        assert np.array_equal(a, b)
    # admission is in arrival order
    admits = [i["t_admit"] for i in infos]
    assert admits == sorted(admits)
    for p in plans:
        p.close()


def test_one_launch_per_frame_mode():
    from paper_2511_09165_amd import plan_for_frame
    frames = _mix(3, 5)
    plans = [plan_for_frame(f) for f in frames]
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    outs, infos, stats = _run_server(frames, plans, hbm_budget=2 << 30, num_streams=1, max_batch=1)
    assert stats["launches"] == len(frames)
    assert all(i["batch_frames"] == 1 for i in infos)
    for a, b in zip(alone, outs):
        assert np.array_equal(a, b)
    for p in plans:
        p.close()


def test_unbatchable_plans_in_the_mix():
    """Linear-delay, Kahan and FP64-accumulation plans are launched one by one among batched frames."""
    from paper_2511_09165_amd import plan_for_frame
    frames = _mix(4, 6)
    opts = [dict(), dict(linear=True), dict(), dict(compensated=True), dict(), dict(accumulate="f64")]
    plans = []
    for f, o in zip(frames, opts):
        if o.get("compensated") or o.get("accumulate"):
            f.nearfield = False
            f.dirs = synth.unit_vectors(np.linspace(-50, 50, f.num_dirs), np.zeros(f.num_dirs))
        plans.append(plan_for_frame(f, **o))
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    outs, infos, stats = _run_server(frames, plans, hbm_budget=2 << 30, num_streams=2, max_batch=64)
    for a, b in zip(alone, outs):
        assert np.array_equal(a, b)
    assert infos[1]["batch_frames"] == 1 and infos[3]["batch_frames"] == 1 and infos[5]["batch_frames"] == 1
    for p in plans:
        p.close()


def test_rejections_and_release_rules():
    from paper_2511_09165_amd import DmasError, Server, plan_for_frame
    f = synth.random_frame(np.random.default_rng(5), 16, 100, 4096, 3)
    plan = plan_for_frame(f)
    x = f.x_f32()
    frame_bytes = 16 * 4096 * 4 + 100 * 4096 * 4
    with Server(hbm_budget=frame_bytes // 2) as srv:
        with pytest.raises(DmasError) as e:
            srv.submit(plan, x)
        assert e.value.status == 1                    # larger than the budget: never admissible
        assert srv.stats()["submitted"] == 0
    with Server(hbm_budget=1 << 30, staging=16 * 4096 * 4 + 512) as srv:
        with pytest.raises(ValueError):
            srv.submit(plan, np.zeros((16, 4095), dtype=np.float32))   # wrong shape (binding check)
        t1 = srv.submit(plan, x)
        try:
            t2 = srv.submit(plan, x)                   # staging holds one input at a time
            srv.wait(t2)
            srv.release(t2)
        except DmasError as err:
            assert err.status == 5                    # DMAS_ERR_BUSY
        srv.wait(t1, timeout=float("inf"))           # no limit: capped, not overflowed
        for bad in (float("nan"), -1.0):
            with pytest.raises(DmasError) as e:
                srv.wait(t1, timeout=bad)
            assert e.value.status == 1
            with pytest.raises(DmasError):
                srv.drain(bad)
        srv.drain(float("inf"))
        with pytest.raises(ValueError):
            srv.fetch(t1, (100, 4095))                # not the result's shape (binding check)
        assert srv.fetch(t1).shape == (100, 4096)     # the envelope's (D, T)
        srv.release(t1)
        with pytest.raises(ValueError):
            srv.fetch(t1)                             # released: nothing to fetch
        with pytest.raises(DmasError):
            srv.release(t1)                           # unknown ticket now
        with pytest.raises(DmasError):
            srv.query(12345)
    plan.close()


def test_auto_release_records():
    from paper_2511_09165_amd import Server, plan_for_frame
    frames = _mix(6, 6)
    plans = [plan_for_frame(f) for f in frames]
    with Server(hbm_budget=2 << 30) as srv:
        for f, p in zip(frames, plans):
            srv.submit(p, f.x_f32(), envelope=f.env, auto_release=True)
        srv.drain(120)
        recs = srv.completed()
        st = srv.stats()
    assert len(recs) == len(frames)
    assert st["hbm_in_use"] == 0 and st["completed"] == len(frames)
    for r in recs:
        assert r["state"] == 3 and r["d_out"] is None
        assert r["t_arrival"] <= r["t_admit"] <= r["t_launch"] <= r["t_done"]
    for p in plans:
        p.close()


def test_server_holds_its_plans():
    """A frame submitted with a Plan that the caller no longer references still runs on a live
    plan (the binding holds it until the server closes) and gives the plain launch's bits."""
    import gc
    from paper_2511_09165_amd import Server, plan_for_frame
    f = synth.random_frame(np.random.default_rng(17), 16, 40, 2048, 3)
    _say("server holds plans")
    with plan_for_frame(f) as p:
        ref = _standalone(p, f.x_f32(), True)
    with Server(hbm_budget=1 << 28) as srv:
        t = srv.submit(plan_for_frame(f), f.x_f32())
        gc.collect()
        srv.wait(t)
        np.testing.assert_array_equal(srv.fetch(t), ref)
        srv.release(t)


# ---------------------------------------------------------------------------
# Resident workers: a persistent launch per kernel class fed by a job queue
# ---------------------------------------------------------------------------

def _resident_capable(f):
    return f.order in (3, 5)


def test_resident_equals_alone_bitwise():
    """Frames served by resident workers (orders 3 and 5; tables of either mode) give the same bits
    as plain launches, in a mix with frames that go through launches (order 2) and with decimation."""
    from paper_2511_09165_amd import plan_for_frame
    rng = np.random.default_rng(31)
    frames = [_blocker()] + _mix(3, 14)
    for M, n in [(100, 3), (72, 5)]:          # more than 64 microphones: offsets per microphone block
        f = synth.random_frame(rng, M, 40, 2048, n)
        f.env = True
        frames.append(f)
    plans = [plan_for_frame(f, env_decimation=(3 if k % 6 == 4 else 1)) for k, f in enumerate(frames)]
    alone = [_standalone(p, f.x_f32(), f.env) for f, p in zip(frames, plans)]
    _say(f"resident: {len(frames)} frames")
    outs, infos, stats = _run_server(frames, plans, hbm_budget=8 << 30, resident=True)
    for k, (a, b) in enumerate(zip(alone, outs)):
        assert np.array_equal(a, b), f"frame {k} differs between alone and the resident worker"
    n_res = sum(_resident_capable(f) for f in frames)
    assert 0 < n_res < len(frames)
    assert stats["resident_frames"] == n_res and stats["resident_launches"] >= 1
    assert stats["completed"] == len(frames) and stats["failed"] == 0
    for i in infos:
        assert i["t_arrival"] <= i["t_admit"] <= i["t_launch"] <= i["t_done"]
    f = frames[1]
    y_ref = oracle.frame_rows(f, x=f.x_f32().astype(np.float64))
    if f.env:
        y_ref = oracle.envelope(y_ref, oracle.lowpass_taps(63, 5000.0, f.fs).astype(np.float32).astype(np.float64))
    check_t1(outs[1].astype(np.float64), y_ref)
    for p in plans:
        p.close()


def test_resident_worker_exits_when_idle_and_relaunches():
    """A worker that ran out of work exits by itself; the next frame gets a new worker. A plan
    created after a worker was launched is served by a later worker, with the same bits."""
    import time
    from paper_2511_09165_amd import Server, plan_for_frame
    f = synth.random_frame(np.random.default_rng(41), 32, 300, 4096, 5)
    g = synth.random_frame(np.random.default_rng(42), 16, 200, 3000, 3)
    with plan_for_frame(f) as pf:
        ref_f = _standalone(pf, f.x_f32(), True)
        _say("resident: idle exit and relaunch")
        with Server(hbm_budget=1 << 30, resident=True) as srv:
            t1 = srv.submit(pf, f.x_f32())
            srv.wait(t1, timeout=60)
            time.sleep(0.05)                       # well past the idle limit of the worker
            t2 = srv.submit(pf, f.x_f32())
            srv.wait(t2, timeout=60)
            assert srv.stats()["resident_launches"] >= 2
            with plan_for_frame(g) as pg:          # a plan newer than every worker so far
                ref_g = _standalone(pg, g.x_f32(), True)
                t3 = srv.submit(pg, g.x_f32())
                srv.wait(t3, timeout=60)
                np.testing.assert_array_equal(srv.fetch(t3), ref_g)
                srv.release(t3)
            for t in (t1, t2):
                np.testing.assert_array_equal(srv.fetch(t), ref_f)
                srv.release(t)
            st = srv.stats()
        assert st["resident_frames"] == 3 and st["failed"] == 0 and st["hbm_in_use"] == 0


def test_resident_auto_release_and_drain():
    """Auto-released frames through resident workers: every record arrives, the arena empties."""
    from paper_2511_09165_amd import Server, plan_for_frame
    frames = _mix(8, 10)
    plans = [plan_for_frame(f) for f in frames]
    with Server(hbm_budget=2 << 30, resident=True) as srv:
        for f, p in zip(frames, plans):
            srv.submit(p, f.x_f32(), envelope=f.env, auto_release=True)
        srv.drain(120)
        recs = srv.completed()
        st = srv.stats()
    assert len(recs) == len(frames) and all(r["state"] == 3 for r in recs)
    assert st["hbm_in_use"] == 0 and st["completed"] == len(frames)
    assert st["resident_frames"] == sum(_resident_capable(f) for f in frames)
    for p in plans:
        p.close()


def test_resident_destroy_with_frames_in_flight():
    """Closing a resident server with frames still queued or running returns promptly: the worker
    finishes what it has claimed and exits; a new server afterwards serves frames normally."""
    import time
    from paper_2511_09165_amd import Server, plan_for_frame
    frames = _mix(9, 8)
    plans = [plan_for_frame(f) for f in frames]
    _say("resident: destroy with frames in flight")
    t0 = time.time()
    with Server(hbm_budget=2 << 30, resident=True) as srv:
        for f, p in zip(frames, plans):
            srv.submit(p, f.x_f32(), envelope=f.env)
    assert time.time() - t0 < 30
    f, p = frames[0], plans[0]
    ref = _standalone(p, f.x_f32(), f.env)
    with Server(hbm_budget=1 << 30, resident=True) as srv:
        t = srv.submit(p, f.x_f32(), envelope=f.env)
        srv.wait(t, timeout=60)
        np.testing.assert_array_equal(srv.fetch(t), ref)
        srv.release(t)
    for q in plans:
        q.close()


def test_resident_half_precision_inputs_bitwise():
    """FP16 and BF16 frames through resident workers (the roots job reads 16-bit samples from the
    staging memory) give the same bits as plain launches, next to FP32 frames."""
    from paper_2511_09165_amd import Server, plan_for_frame
    rng = np.random.default_rng(51)
    cases = []
    for k, (dtype, n) in enumerate([("f16", 3), ("bf16", 5), ("f32", 5), ("bf16", 3), ("f16", 5)]):
        f = synth.random_frame(rng, int(rng.choice([16, 32, 72])), int(rng.integers(20, 200)),
                               int(rng.choice([900, 2048])), n)
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
        scale = 2.0 ** -8 if dtype == "f16" else 1.0
        xq = torch.from_numpy(f.x / scale).to(tdt)
        host = xq.view(torch.int16).numpy().view(np.uint16) if dtype == "bf16" else xq.numpy()
        plan = plan_for_frame(f, in_dtype=dtype)
        ref = plan.envelope(xq.cuda(), in_scale=scale).cpu().numpy()
        cases.append((plan, host, scale, ref))
    _say("resident: FP16/BF16 frames")
    with Server(hbm_budget=1 << 30, resident=True) as srv:
        tickets = [srv.submit(p, h, in_scale=s) for p, h, s, _ in cases]
        for t, (p, _, _, ref) in zip(tickets, cases):
            srv.wait(t, timeout=60)
            np.testing.assert_array_equal(srv.fetch(t), ref)
            srv.release(t)
        assert srv.stats()["resident_frames"] == len(cases)
    for p, _, _, _ in cases:
        p.close()
