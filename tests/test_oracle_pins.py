"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle (``oracle/liboracle.so``) against something other
than itself: the combinatorial definition evaluated by brute force (eq. (5)),
the special cases n = 1 (DAS, eq. (2)) and n = 2 (eq. (3)), the paper's
Newton-Girard forms (eqs. (8)-(12)) in exact arithmetic, closed forms,
textbook values (tests/golden), library routines (numpy convolution, scipy's
window design) and physical alignment of synthetic plane and spherical waves.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import newton_girard as ng
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _direct_pixelwise(x, mic, dirs, fs, c, n, use_cf, nearfield=False, eps=1e-20):
    """Brute-force image: delays from the physical arrival model, eq. (5) per pixel."""
    M, T = x.shape
    out = np.zeros((dirs.shape[0], T))
    for p in range(dirs.shape[0]):
        v = dirs[p]
        if nearfield:
            lag = (np.linalg.norm(v[None, :] - mic, axis=1) - np.linalg.norm(v)) / c
        else:
            lag = -(mic @ v) / c
        d = np.floor(fs * lag + 0.5).astype(np.int64)
        for t in range(T):
            idx = t + d
            xs = [x[i, idx[i]] if 0 <= idx[i] < T else 0.0 for i in range(M)]
            out[p, t] = ng.pixel(xs, n, use_cf, eps)[1]
    return out


# ---------------------------------------------------------------------------
# E_n: definition, textbook values, Newton-Girard forms
# ---------------------------------------------------------------------------

def _golden_cases():
    cases = []
    with open(os.path.join(GOLDEN, "stirling_esp.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, xs, want = (part.strip() for part in line.split("|"))
            cases.append((int(n), [float(v) for v in xs.split()], float(want)))
    return cases


@pytest.mark.parametrize("n,xs,want", _golden_cases())
def test_golden_elementary_symmetric(n, xs, want):
    """Textbook E_n values (Stirling numbers of the first kind, hand expansions)."""
    M = len(xs)
    x = np.array(xs, dtype=np.float64)[:, None]        # T = 1
    mic = np.zeros((M, 3))                             # all delays zero
    dirs = np.array([[0.0, 0.0, 1.0]])
    y = oracle.dmas_rows(x, mic, dirs, 450e3, 343.0, n, use_cf=False)
    assert y.shape == (1, 1)
    assert abs(y[0, 0] - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("M,n", [(m, n) for m in range(1, 11) for n in range(1, min(m, 7) + 1)])
def test_oracle_matches_bruteforce_definition(M, n):
    """Eq. (5) by enumeration of all n-subsets equals the oracle, random mixed-sign samples."""
    rng = np.random.default_rng(1000 + 17 * M + n)
    T = 6
    x = rng.standard_normal((M, T))
    x[rng.random((M, T)) < 0.15] = 0.0                 # exact zeros: sgn(0) = 0
    if M >= 3:
        x[0, 2] = 40.0                                  # one dominant channel
    mic = np.zeros((M, 3))
    dirs = np.array([[0.0, 0.0, 1.0]])
    for use_cf in (False, True):
        y, dg = oracle.dmas_rows(x, mic, dirs, 450e3, 343.0, n, use_cf=use_cf, diag=True)
        for t in range(T):
            xs = list(x[:, t])
            e_ref, y_ref = ng.pixel(xs, n, use_cf)
            s = [ng.signed_root(v, n) for v in xs]
            h_ref = ng.complete_homogeneous([abs(v) for v in s], n)
            scale = ng.complete_homogeneous([abs(v) for v in s], n) + 1e-300
            assert abs(dg["E"][0, t] - e_ref) <= 1e-12 * scale
            assert abs(y[0, t] - y_ref) <= 1e-12 * scale
            assert dg["h"][0, t] == pytest.approx(h_ref, rel=1e-12, abs=1e-300)
            assert dg["sum_x"][0, t] == pytest.approx(sum(xs), rel=1e-12, abs=1e-12)
            assert dg["sum_x2"][0, t] == pytest.approx(sum(v * v for v in xs), rel=1e-12)
            assert dg["sum_abs"][0, t] == pytest.approx(sum(abs(v) for v in xs), rel=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_newton_girard_forms_exact(n):
    """Eq. (8), eqs. (9)-(12) and the Newton recurrence equal E_n exactly (rational arithmetic)."""
    rng = np.random.default_rng(77 + n)
    for trial in range(5):
        M = n + trial + 1
        s = [Fraction(int(v), int(w)) for v, w in zip(rng.integers(-9, 10, M), rng.integers(1, 7, M))]
        e_true = ng.elementary_bruteforce(s, n)
        P = ng.power_sums(s, n)
        assert ng.ng_partitions(P, n) == e_true
        assert ng.newton_recurrence(P, n) == e_true
        if 1 <= n <= 5:
            assert ng.ng_explicit(P, n) == e_true


def test_partition_count():
    """Eq. (8) sums over integer partitions: p(n) = 1, 2, 3, 5, 7, 11, 15, 22 for n = 1..8."""
    assert [sum(1 for _ in ng.partitions(n)) for n in range(1, 9)] == [1, 2, 3, 5, 7, 11, 15, 22]


# ---------------------------------------------------------------------------
# Special cases: DAS (n = 1), eq. (3) (n = 2), closed forms
# ---------------------------------------------------------------------------

def test_order1_is_das():
    """n = 1: eq. (5) reduces to eq. (2); with CF it is DAS * CF (eq. (14))."""
    f = synth.random_frame(np.random.default_rng(5), 7, 9, 80, 1)
    d = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c)
    y0 = oracle.dmas_rows(f.x, f.mic_pos, f.dirs, f.fs, f.c, 1, use_cf=False)
    y1 = oracle.dmas_rows(f.x, f.mic_pos, f.dirs, f.fs, f.c, 1, use_cf=True)
    T = f.num_samples
    for p in range(f.num_dirs):
        for t in range(T):
            idx = t + d[p]
            xs = [f.x[i, j] if 0 <= j < T else 0.0 for i, j in enumerate(idx)]
            assert y0[p, t] == pytest.approx(ng.das(xs), rel=1e-12, abs=1e-12)
            assert y1[p, t] == pytest.approx(ng.das(xs) * ng.coherence_factor(xs, 1e-20), rel=1e-12, abs=1e-12)


def test_order2_is_classic_dmas():
    """n = 2 equals the double loop of eq. (3)."""
    f = synth.random_frame(np.random.default_rng(6), 6, 5, 60, 2)
    d = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c)
    y = oracle.dmas_rows(f.x, f.mic_pos, f.dirs, f.fs, f.c, 2, use_cf=False)
    T = f.num_samples
    for p in range(f.num_dirs):
        for t in range(T):
            idx = t + d[p]
            xs = [f.x[i, j] if 0 <= j < T else 0.0 for i, j in enumerate(idx)]
            assert y[p, t] == pytest.approx(ng.dmas2_pairwise(xs), rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("M", [8, 32])
def test_identical_channels_closed_form(n, M):
    """All channels equal, broadside direction (all delays 0): E_n = C(M,n) sgn(x)^n |x|, CF = 1."""
    rng = np.random.default_rng(n * 100 + M)
    T = 50
    row = rng.standard_normal(T) * 3.0
    row[::7] = 0.0
    x = np.tile(row, (M, 1))
    mic = synth.disc_array(rng, M, 0.1)
    dirs = np.array([[0.0, 0.0, 1.0]])
    y, dg = oracle.dmas_rows(x, mic, dirs, 450e3, 343.0, n, use_cf=True, diag=True)
    want_e = math.comb(M, n) * np.sign(row) ** n * np.abs(row)
    np.testing.assert_allclose(dg["E"][0], want_e, rtol=1e-12, atol=0)
    nz = row != 0
    np.testing.assert_allclose(dg["CF"][0][nz], 1.0, rtol=1e-14)
    assert np.all(dg["CF"][0][~nz] == 0.0)
    # h_n of identical |s| = a: C(M+n-1, n) a^n = C(M+n-1, n) |x|
    np.testing.assert_allclose(dg["h"][0], math.comb(M + n - 1, n) * np.abs(row), rtol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_n_minus_one_nonzero_channels_gives_zero(n):
    """With only n-1 non-zero delayed samples no n-subset is all non-zero: E_n = 0 exactly."""
    M, T = 9, 20
    rng = np.random.default_rng(n)
    x = np.zeros((M, T))
    x[: n - 1] = rng.standard_normal((n - 1, T))
    y = oracle.dmas_rows(x, np.zeros((M, 3)), np.array([[0, 0, 1.0]]), 450e3, 343.0, n, use_cf=False)
    assert np.all(y == 0.0)


def test_coherence_factor_bounds():
    """Eq. (13): 0 <= CF <= 1 (Cauchy-Schwarz), CF = 1 exactly when all x_i are equal and non-zero."""
    rng = np.random.default_rng(9)
    f = synth.random_frame(rng, 12, 6, 300, 3)
    _, dg = oracle.frame_rows(f, diag=True)
    cf = dg["CF"]
    assert np.all(cf >= 0.0) and np.all(cf <= 1.0 + 1e-15)
    x = np.full((5, 4), -2.5)
    _, dg = oracle.dmas_rows(x, np.zeros((5, 3)), np.array([[0, 0, 1.0]]), 450e3, 343.0, 2, diag=True)
    np.testing.assert_allclose(dg["CF"], 1.0, rtol=1e-15)


# ---------------------------------------------------------------------------
# Symmetries
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_sign_flip_and_scaling(n):
    """S(-x) = (-1)^n S(x) exactly; S(a x) = a S(x) for a > 0 (degree-1 homogeneity)."""
    f = synth.random_frame(np.random.default_rng(11 + n), 10, 7, 200, n)
    y = oracle.frame_rows(f)
    yn = oracle.frame_rows(f, x=-f.x)
    assert np.array_equal(yn, (-1) ** n * y)
    ys = oracle.frame_rows(f, x=3.7 * f.x)
    np.testing.assert_allclose(ys, 3.7 * y, rtol=1e-12, atol=1e-12 * np.abs(y).max())


def test_time_shift_equivariance():
    """Shifting every channel by k samples shifts the image by k (away from the edges)."""
    f = synth.random_frame(np.random.default_rng(12), 8, 5, 400, 3)
    k = 17
    xs = np.zeros_like(f.x)
    xs[:, k:] = f.x[:, :-k]
    y = oracle.frame_rows(f)
    ysh = oracle.frame_rows(f, x=xs)
    d = oracle.delays(f.mic_pos, f.dirs, f.fs, f.c)
    lo, hi = k + int(np.abs(d).max()) + 1, f.num_samples - int(np.abs(d).max()) - 1
    assert np.array_equal(ysh[:, lo:hi], y[:, lo - k:hi - k])


# ---------------------------------------------------------------------------
# Delays: physical alignment (eq. (1))
# ---------------------------------------------------------------------------

def test_farfield_plane_wave_alignment():
    """A noise-free integer-sample plane wave from a grid direction is perfectly aligned: DAS peak = M * pulse."""
    rng = np.random.default_rng(21)
    fs, c, T, M = 450e3, 343.0, 600, 16
    mic = synth.disc_array(rng, M, 0.12)
    dirs = synth.az_el_grid(np.arange(-60, 61, 4.0), [-10.0, 0.0, 10.0])
    pulse = synth.hann_burst(fs, 40e3, 0.2e-3)
    target = 47
    u = dirs[target]
    lead = np.floor(fs * (mic @ u) / c + 0.5).astype(int)
    x = np.zeros((M, T))
    onset = 250
    for i in range(M):
        x[i, onset - lead[i]: onset - lead[i] + pulse.size] = pulse
    y = oracle.dmas_rows(x, mic, dirs, fs, c, 1, use_cf=False)
    np.testing.assert_allclose(y[target, onset:onset + pulse.size], M * pulse, rtol=1e-12, atol=1e-12)
    peak = np.abs(y).max(axis=1)
    assert int(np.argmax(peak)) == target
    # the same wave is not aligned for the mirrored steering sign
    y_bad = oracle.dmas_rows(x, mic, -dirs, fs, c, 1, use_cf=False)
    assert np.abs(y_bad[target]).max() < 0.9 * M * np.abs(pulse).max()


def test_nearfield_spherical_wave_alignment():
    """A spherical wave from a voxel aligns at that voxel; far-away voxels along u give far-field delays."""
    rng = np.random.default_rng(22)
    fs, c, T, M = 192e3, 343.0, 500, 25
    mic = synth.grid_array(5, 5, 0.02)
    vox = np.stack([rng.uniform(-0.3, 0.3, 12), rng.uniform(-0.3, 0.3, 12), rng.uniform(0.5, 1.2, 12)], -1)
    target = 5
    v = vox[target]
    arrive = np.floor(fs * (np.linalg.norm(v[None] - mic, axis=1) - np.linalg.norm(v)) / c + 0.5).astype(int)
    x = np.zeros((M, T))
    x[np.arange(M), 200 + arrive] = 1.0
    y = oracle.dmas_rows(x, mic, vox, fs, c, 1, use_cf=False, nearfield=True)
    assert y[target, 200] == M
    assert np.abs(y[np.arange(12) != target]).max() < M
    # far-field limit: v = R u with R -> large gives the plane-wave delays
    u = synth.unit_vectors(rng.uniform(-50, 50, 30), rng.uniform(-30, 30, 30))
    far = oracle.delays(mic, u, fs, c)
    near = oracle.delays(mic, 1e7 * u, fs, c, nearfield=True)
    assert np.array_equal(far, near)


def test_delay_table_matches_rows():
    """The delay table (used for bit-exact GPU delay checks) matches a brute-force image built from it."""
    f = synth.random_frame(np.random.default_rng(23), 5, 4, 40, 2)
    y = oracle.frame_rows(f)
    yb = _direct_pixelwise(f.x, f.mic_pos, f.dirs, f.fs, f.c, 2, True)
    np.testing.assert_allclose(y, yb, rtol=1e-11, atol=1e-12)
    fn = synth.random_frame(np.random.default_rng(24), 5, 4, 40, 3, nearfield=True)
    y = oracle.frame_rows(fn)
    yb = _direct_pixelwise(fn.x, fn.mic_pos, fn.dirs, fn.fs, fn.c, 3, True, nearfield=True)
    np.testing.assert_allclose(y, yb, rtol=1e-11, atol=1e-12)


def test_delays_follow_unfused_ieee_sequence():
    """Eq. (1) rounded to the nearest sample as separately rounded IEEE double operations:
    tau = -(r . u)/c, f = fs * tau, d = floor(f + 1/2). Geometries where a fused fs*tau + 1/2
    would land on the other side of an integer pin the oracle to the unfused sequence."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from _parity import delay_rounding_ties
    ties = delay_rounding_ties()
    assert len(ties) >= 8
    mic = np.array([[x, 0.0, 0.0] for x, _, _ in ties])
    d = oracle.delays(mic, np.array([[1.0, 0.0, 0.0]]), 450e3, 343.0)[0]
    assert [int(v) for v in d] == [u for _, u, _ in ties]
    assert all(u != fz for _, u, fz in ties)


def test_zero_outside_record():
    """Samples steered outside [0, T) are zero: a one-sample record with a large delay sees nothing."""
    x = np.ones((3, 4))
    mic = np.array([[0.0, 0, 0], [0.05, 0, 0], [-0.05, 0, 0]])
    dirs = np.array([[1.0, 0, 0]])          # endfire: delays -66, 0, +66 samples at 450 kHz
    d = oracle.delays(mic, dirs, 450e3, 343.0)
    assert list(d[0]) == [0, -66, 66]
    y = oracle.dmas_rows(x, mic, dirs, 450e3, 343.0, 1, use_cf=False)
    np.testing.assert_array_equal(y, np.ones((1, 4)))


def test_linear_interpolation_is_exact_on_ramps():
    """Linear fractional delay reproduces a linear ramp exactly: x_i(t) = a (t + fs tau_i) + b."""
    rng = np.random.default_rng(25)
    M, T = 6, 300
    mic = synth.disc_array(rng, M, 0.1)
    dirs = synth.unit_vectors(rng.uniform(-60, 60, 5), rng.uniform(-20, 20, 5))
    a, b = 0.01, -1.3
    x = np.tile(a * np.arange(T) + b, (M, 1))
    y = oracle.dmas_rows(x, mic, dirs, 450e3, 343.0, 1, use_cf=False, interp=True)
    lag = -(dirs @ mic.T) / 343.0 * 450e3                      # (D, M) in samples
    t = np.arange(50, 250)
    want = (a * (t[None, :, None] + lag[:, None, :]) + b).sum(axis=2)
    np.testing.assert_allclose(y[:, 50:250], want, rtol=1e-12, atol=1e-12)
    whole, frac = oracle.delays_frac(mic, dirs, 450e3, 343.0)
    np.testing.assert_allclose(whole + frac, lag, rtol=0, atol=1e-12)
    assert np.all((frac >= 0) & (frac < 1))


# ---------------------------------------------------------------------------
# Envelope and its default low-pass
# ---------------------------------------------------------------------------

def test_envelope_matches_numpy_convolution():
    """The envelope equals numpy's centred ('same') convolution of |y| with the taps (odd L)."""
    rng = np.random.default_rng(31)
    y = rng.standard_normal((4, 257))
    for L in (1, 3, 63, 101):
        h = rng.standard_normal(L)
        env = oracle.envelope(y, h)
        for r in range(4):
            np.testing.assert_allclose(env[r], np.convolve(np.abs(y[r]), h, mode="same"), rtol=1e-12, atol=1e-12)


def test_envelope_impulse_and_dc():
    """An impulse at t0 gives the taps in order starting at t0 - (L-1)/2; a constant gives sum(h) inside."""
    h = np.arange(1.0, 8.0)                  # L = 7, asymmetric
    y = np.zeros((1, 40))
    y[0, 20] = -2.0
    env = oracle.envelope(y, h)
    np.testing.assert_allclose(env[0, 17:24], 2.0 * h)
    assert np.count_nonzero(env) == 7
    env = oracle.envelope(np.full((1, 40), -3.0), h)
    np.testing.assert_allclose(env[0, 3:37], 3.0 * h.sum())


def test_lowpass_matches_scipy_firwin():
    """The default envelope filter equals scipy's Hamming-window firwin design at unit DC gain."""
    scipy_signal = pytest.importorskip("scipy.signal")
    for L, fc, fs in ((63, 5000.0, 450e3), (31, 10e3, 192e3), (127, 5000.0, 450e3)):
        want = scipy_signal.firwin(L, fc, fs=fs, window="hamming", scale=True)
        np.testing.assert_allclose(oracle.lowpass_taps(L, fc, fs), want, rtol=1e-12, atol=1e-15)
    with pytest.raises(ValueError):
        oracle.lowpass_taps(64)


def test_invalid_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.dmas_rows(np.ones((3, 5)), np.zeros((3, 3)), np.array([[0, 0, 1.0]]), 450e3, 343.0, 4)
    with pytest.raises(ValueError):
        oracle.envelope(np.ones((1, 5)), np.ones(4))


def test_matched_filter_matches_numpy_and_fft():
    """Pulse compression equals numpy's 'valid' correlation of the zero-padded channel and an FFT correlation."""
    rng = np.random.default_rng(41)
    raw = rng.standard_normal((3, 500))
    pulse = synth.linear_chirp(450e3, 25e3, 75e3, 1e-4)
    out = oracle.matched_filter(raw, pulse)
    for i in range(3):
        padded = np.concatenate([raw[i], np.zeros(pulse.size - 1)])
        np.testing.assert_allclose(out[i], np.correlate(padded, pulse, mode="valid"), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out, synth.matched_filter(raw, pulse), rtol=1e-9, atol=1e-9)
    # an echo of the pulse at sample 100 peaks at 100 with the pulse energy
    echo = np.zeros((1, 400))
    echo[0, 100:100 + pulse.size] = pulse
    r = oracle.matched_filter(echo, pulse)[0]
    assert int(np.argmax(r)) == 100 and r[100] == pytest.approx(np.sum(pulse ** 2), rel=1e-12)
