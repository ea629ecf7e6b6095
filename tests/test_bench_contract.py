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
    # eRTIS-like frame: 32 * 7 + 15 (Newton-Girard) + 6 (CF) + 1 (scale) + 63 (FIR) per pixel
    assert bench.pixel_slots(32, 5, True, 63) == 309
    D, T, M = 4186, 16384, 32
    assert bench.launch_slots(M, T, D, 5, True, 63) == D * T * 309 + M * T * 6


def test_linear_delay_slot_count():
    # linear delays: per microphone the interpolation (2) and the root of the interpolated value (6)
    # on top of the powers and sums: 32 * (2 + 6 + 7) + 15 + 6 + 1 + 63
    assert bench.linear_pixel_slots(32, 5, True, 63) == 32 * 15 + 85


def test_unknown_workload_is_rejected(capsys):
    import pytest
    with pytest.raises(SystemExit):
        bench.main(["--workload", "nope"])
