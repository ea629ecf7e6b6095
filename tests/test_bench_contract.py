"""bench.py's contract on the host: one GPU only, and the algorithmic VALU counts it reports."""

import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_slot_counts():
    # per microphone and pixel: intermediate powers + n power sums + CF sums (roots counted per channel sample)
    assert [bench.mic_slots(n, True) for n in range(1, 9)] == [2, 4, 4, 7, 7, 10, 10, 13]
    assert [bench.mic_slots(n, False) for n in range(1, 9)] == [1, 2, 3, 5, 6, 8, 9, 11]
    assert [bench.root_slots(n) for n in (1, 2, 3, 5, 8)] == [0, 3, 6, 6, 6]
    # eRTIS-like frame: 32 * 7 + 15 (Newton-Girard) + 6 (CF) + 1 (scale) VALU slots per pixel; the
    # 63-tap envelope FIR runs on the matrix cores and is counted as flops apart
    assert bench.pixel_slots(32, 5, True) == 246
    D, T, M = 4186, 16384, 32
    assert bench.launch_slots(M, T, D, 5, True) == D * T * 246 + M * T * 6
    assert bench.fir_flops(D, T, 63) == 2.0 * D * T * 63


def test_linear_delay_slot_count():
    # linear delays: per microphone the interpolation (2) and the root of the interpolated value (6)
    # on top of the powers and sums: 32 * (2 + 6 + 7) + 15 + 6 + 1
    assert bench.linear_pixel_slots(32, 5, True) == 32 * 15 + 22


def test_roofline_fields():
    r = bench._roofline(246 * 1000, 1000, 1e-3, traffic=5.0, fir=126.0 * 1000)
    assert r["bound"] == "alu" and abs(r["frac"] - 246e9 / bench.VALU_SLOTS_PER_S) < 1e-12
    assert "replayed" in r["traffic_source"]
    assert r["mfma_fir"]["bound"] == "mfma" and r["mfma_fir"]["flops_per_pixel"] == 126.0


def test_unknown_workload_is_rejected(capsys):
    import pytest
    with pytest.raises(SystemExit):
        bench.main(["--workload", "nope"])
