"""The paper's qualitative image-quality claims, reproduced on synthetic data.

Section III-A reports that the point-spread function's dynamic range grows
with the DMAS order and further with CF (Fig. 2), that the image SNR at 0 dB
microphone SNR grows with the order and with CF (eqs. (15)-(18), Table I), and
that the range resolution does not change in the far field (Fig. 3). The
paper's array and data are not available, so only these trends are checked
(absolute values depend on the geometry): on the FP64 oracle here, and on the
GPU path in the GPU test below.

Metrics (on the envelope image normalised to a maximum of 1):
  PSF dynamic range: -20 log10 of the largest angular-profile value more than
    15 deg from the peak direction (noise-free point reflector);
  image SNR, eq. (18): 20 log10(1 / mean of off-target pixels), off-target =
    more than 15 deg and more than 600 samples from the peak (0 dB mic SNR);
  range width: -6 dB width in samples along time at the peak direction.
"""

import numpy as np
import pytest

import oracle
import synth

TAPS = oracle.lowpass_taps(63, 5000.0, 450e3)


def _env(frame, n, cf, x=None):
    y = oracle.dmas_rows(frame.x if x is None else x, frame.mic_pos, frame.dirs, frame.fs, frame.c, n, use_cf=cf)
    env = oracle.envelope(y, TAPS)
    return env / env.max()


def metrics(img, az):
    pk = np.unravel_index(int(np.argmax(img)), img.shape)
    prof = img.max(axis=1)
    far = np.abs(az - az[pk[0]]) > 15
    dr = -20 * np.log10(prof[far].max())
    off = np.ones_like(img, dtype=bool)
    off[~far, :] = False
    off[:, max(0, pk[1] - 600):pk[1] + 600] = False
    snr = 20 * np.log10(1.0 / img[off].mean())
    above = np.nonzero(img[pk[0]] >= 0.5)[0]
    return dict(dr=dr, snr=snr, range_width=int(above.max() - above.min()), peak_az=float(az[pk[0]]))


@pytest.fixture(scope="module")
def frames():
    return synth.point_echo_frame(), synth.point_echo_frame(snr_db=0.0, seed_salt=1)


@pytest.fixture(scope="module")
def table(frames):
    clean, noisy = frames
    az = clean.truth["az"]
    out = {}
    for n in range(1, 6):
        for cf in (False, True):
            m = metrics(_env(clean, n, cf), az)
            m["snr"] = metrics(_env(noisy, n, cf), az)["snr"]
            out[(n, cf)] = m
    return out


def test_psf_dynamic_range_grows_with_order_and_cf(table):
    for cf in (False, True):
        drs = [table[(n, cf)]["dr"] for n in range(1, 6)]
        assert all(b > a + 5.0 for a, b in zip(drs, drs[1:])), drs
    for n in range(1, 6):
        assert table[(n, True)]["dr"] > table[(n, False)]["dr"] + 10.0
    # DMAS5 with CF reaches a dynamic range of the order the paper reports (almost 80 dB
    # for its array); the exact value depends on the array geometry
    assert table[(5, True)]["dr"] > 60.0


def test_image_snr_grows_with_order_and_cf(table):
    for cf in (False, True):
        snrs = [table[(n, cf)]["snr"] for n in range(1, 6)]
        assert all(b > a for a, b in zip(snrs, snrs[1:])), snrs
    for n in range(1, 6):
        assert table[(n, True)]["snr"] > table[(n, False)]["snr"]


def test_range_resolution_unchanged_and_target_found(table):
    widths = {table[(n, cf)]["range_width"] for n in range(1, 6) for cf in (False, True)}
    assert max(widths) - min(widths) <= 0.1 * max(widths), widths
    assert all(table[k]["peak_az"] == 0.0 for k in table)


@pytest.mark.gpu
def test_gpu_images_give_the_same_metrics(frames, table):
    torch = pytest.importorskip("torch")
    from paper_2511_09165_amd import plan_for_frame
    clean, noisy = frames
    az = clean.truth["az"]
    for n in (1, 3, 5):
        for cf in (False, True):
            imgs = []
            for fr in (clean, noisy):
                fr.order, fr.use_cf = n, cf
                with plan_for_frame(fr, fir_taps=TAPS.astype(np.float32)) as plan:
                    env = plan.envelope(torch.from_numpy(fr.x_f32()).cuda()).cpu().numpy().astype(np.float64)
                imgs.append(env / env.max())
            m = metrics(imgs[0], az)
            m["snr"] = metrics(imgs[1], az)["snr"]
            ref = table[(n, cf)]
            assert abs(m["dr"] - ref["dr"]) < 0.05 and abs(m["snr"] - ref["snr"]) < 0.05, (n, cf, m, ref)
            assert m["range_width"] == ref["range_width"]
