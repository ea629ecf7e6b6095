"""Seeded synthetic sonar workloads.

This module builds microphone recordings and imaging grids for the workloads
the beamformer is measured and tested on. It holds scene physics only (array
layouts, direction and voxel grids, emitted pulses, echo arrival times, noise,
and the upstream matched filter); it contains none of the beamformer's own
arithmetic (no steering, roots, power sums, symmetric polynomials, coherence
factor or envelope). Both the FP64 oracle and the GPU path consume the arrays it
returns, so they see identical data.

The paper's own data (an eRTIS array and recorded frames) are not available, so
every input here is synthetic with the shapes and structure the paper describes:
a planar MEMS array, azimuth/elevation direction grids, broadband chirp echoes
after matched filtering (Section III-B), and near-field broadband sources.

Coordinate frame: the array lies in the z = 0 plane and +z is the forward axis.
A direction with azimuth ``az`` and elevation ``el`` has unit vector
``(cos el * sin az, sin el, cos el * cos az)``.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 2511091650
SPEED_OF_SOUND = 343.0


@dataclasses.dataclass
class Frame:
    """One beamforming job: recordings plus the geometry to image them with."""

    name: str
    x: np.ndarray            # (M, T) float64 recordings (already matched-filtered)
    mic_pos: np.ndarray      # (M, 3) float64 metres
    dirs: np.ndarray         # (D, 3) float64: unit vectors (far field) or voxel centres (near field)
    fs: float
    c: float
    order: int
    use_cf: bool
    nearfield: bool
    truth: dict = dataclasses.field(default_factory=dict)

    @property
    def num_mics(self) -> int:
        return int(self.x.shape[0])

    @property
    def num_samples(self) -> int:
        return int(self.x.shape[1])

    @property
    def num_dirs(self) -> int:
        return int(self.dirs.shape[0])

    def x_f32(self) -> np.ndarray:
        return np.ascontiguousarray(self.x.astype(np.float32))


def rng_for(stream: int, salt: int = 0) -> np.random.Generator:
    """Seeded generator of workload ``stream`` (a fixed small integer per workload)."""
    return np.random.default_rng(SEED_BASE + stream + 1000 * salt)


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------

def unit_vectors(az_deg: np.ndarray, el_deg: np.ndarray) -> np.ndarray:
    az = np.deg2rad(np.asarray(az_deg, dtype=np.float64))
    el = np.deg2rad(np.asarray(el_deg, dtype=np.float64))
    return np.stack([np.cos(el) * np.sin(az), np.sin(el), np.cos(el) * np.cos(az)], axis=-1)


def az_el_grid(az_deg: Sequence[float], el_deg: Sequence[float]) -> np.ndarray:
    """Direction grid with azimuth varying fastest; returns (len(el)*len(az), 3)."""
    az = np.asarray(az_deg, dtype=np.float64)
    el = np.asarray(el_deg, dtype=np.float64)
    ee, aa = np.meshgrid(el, az, indexing="ij")
    return unit_vectors(aa.ravel(), ee.ravel())


def disc_array(rng: np.random.Generator, m: int, diameter: float,
               min_spacing: float = 0.0, max_tries: int = 200000) -> np.ndarray:
    """M points uniform in a disc (z = 0), rejecting draws closer than ``min_spacing``."""
    r = diameter / 2.0
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < m:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("disc_array: cannot place microphones with this spacing")
        p = rng.uniform(-r, r, size=2)
        if p @ p > r * r:
            continue
        if min_spacing > 0 and any(np.hypot(*(p - q)) < min_spacing for q in pts):
            continue
        pts.append(p)
    out = np.zeros((m, 3))
    out[:, :2] = np.array(pts)
    return out


def grid_array(nx: int, ny: int, pitch: float) -> np.ndarray:
    """Centred uniform rectangular array in the z = 0 plane, x fastest."""
    xs = (np.arange(nx) - (nx - 1) / 2.0) * pitch
    ys = (np.arange(ny) - (ny - 1) / 2.0) * pitch
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    out = np.zeros((nx * ny, 3))
    out[:, 0] = xx.ravel()
    out[:, 1] = yy.ravel()
    return out


def hex_disc_array(radius: float, edge: float = 0.005) -> np.ndarray:
    """Microphones on a hexagonal lattice (edge length ``edge``) inside a disc."""
    n = int(math.ceil(radius / edge)) + 2
    pts = []
    for j in range(-2 * n, 2 * n + 1):
        for i in range(-2 * n, 2 * n + 1):
            x = edge * (i + 0.5 * j)
            y = edge * (math.sqrt(3.0) / 2.0) * j
            if x * x + y * y <= radius * radius * (1 + 1e-12):
                pts.append((x, y, 0.0))
    return np.array(pts, dtype=np.float64)


def voxel_grid(nx: int, ny: int, nz: int, xr, yr, zr) -> np.ndarray:
    """Cell-centred voxel grid, x fastest; returns (nx*ny*nz, 3)."""
    def centres(n, lo_hi):
        lo, hi = lo_hi
        step = (hi - lo) / n
        return lo + step * (np.arange(n) + 0.5)
    xs, ys, zs = centres(nx, xr), centres(ny, yr), centres(nz, zr)
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=-1)


# ----------------------------------------------------------------------------
# Signals
# ----------------------------------------------------------------------------

def hann_burst(fs: float, f0: float, duration: float) -> np.ndarray:
    n = int(round(duration * fs))
    t = np.arange(n) / fs
    w = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n) / (n - 1))
    return np.sin(2 * np.pi * f0 * t) * w


def linear_chirp(fs: float, f_lo: float, f_hi: float, duration: float) -> np.ndarray:
    n = int(round(duration * fs))
    t = np.arange(n) / fs
    k = (f_hi - f_lo) / duration
    return np.sin(2 * np.pi * (f_lo * t + 0.5 * k * t * t))


def place_fractional(out: np.ndarray, pulse: np.ndarray, start: float, amp: float) -> None:
    """Add ``amp * pulse`` to ``out`` starting at fractional sample ``start``.

    The pulse is resampled by linear interpolation between its samples; it is
    zero outside its own support.
    """
    T = out.shape[0]
    L = pulse.shape[0]
    lo = int(math.floor(start))
    hi = int(math.ceil(start + L - 1))
    idx = np.arange(max(lo, 0), min(hi + 1, T))
    if idx.size == 0:
        return
    pos = idx - start
    k0 = np.floor(pos).astype(np.int64)
    frac = pos - k0
    padded = np.concatenate([[0.0], pulse, [0.0]])
    v0 = padded[np.clip(k0, -1, L) + 1]
    v1 = padded[np.clip(k0 + 1, -1, L) + 1]
    out[idx] += amp * ((1.0 - frac) * v0 + frac * v1)


def matched_filter(m: np.ndarray, pulse: np.ndarray) -> np.ndarray:
    """Cross-correlate each channel with the emitted pulse (pulse compression).

    r[t] = sum_k m[t + k] * pulse[k], zero beyond the record, so the output peak
    sits at the echo onset. Computed in FP64 with an FFT.
    """
    M, T = m.shape
    L = pulse.shape[0]
    nfft = 1 << int(math.ceil(math.log2(T + L)))
    Mf = np.fft.rfft(m, nfft, axis=1)
    Pf = np.fft.rfft(pulse, nfft)
    r = np.fft.irfft(Mf * np.conj(Pf)[None, :], nfft, axis=1)
    return np.ascontiguousarray(r[:, :T])


def bandlimited_noise(rng: np.random.Generator, n: int, fs: float, f_lo: float, f_hi: float) -> np.ndarray:
    """Unit-variance Gaussian noise restricted to [f_lo, f_hi] by an FFT mask."""
    w = rng.standard_normal(n)
    W = np.fft.rfft(w)
    f = np.fft.rfftfreq(n, 1.0 / fs)
    W[(f < f_lo) | (f > f_hi)] = 0.0
    out = np.fft.irfft(W, n)
    return out / np.std(out)


def fractional_delay(sig: np.ndarray, delay_samples: float) -> np.ndarray:
    """Delay a periodic-extended signal by a fractional number of samples (FFT phase ramp)."""
    n = sig.shape[0]
    S = np.fft.rfft(sig)
    k = np.arange(S.shape[0])
    return np.fft.irfft(S * np.exp(-2j * np.pi * k * delay_samples / n), n)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def burst_frame(seed_salt: int = 0, order: int = 2) -> Frame:
    """8 mics in a 5 cm disc, 64 azimuths over +-60 deg, 1024 samples at 450 kHz.

    Three point reflectors in the horizontal plane, each a Hann-windowed 40 kHz
    tone burst of 0.5 ms, arriving as integer-sample plane waves with random
    amplitude in [0.2, 1]; additive white noise with sigma 0.05.
    """
    rng = rng_for(1, seed_salt)
    fs, c, T = 450e3, SPEED_OF_SOUND, 1024
    mics = disc_array(rng, 8, 0.05)
    dirs = az_el_grid(np.linspace(-60.0, 60.0, 64), [0.0])
    burst = hann_burst(fs, 40e3, 0.5e-3)
    x = np.zeros((8, T))
    refl = []
    max_shift = int(math.ceil(fs * np.max(np.linalg.norm(mics, axis=1)) / c)) + 1
    for _ in range(3):
        az = rng.uniform(-60.0, 60.0)
        amp = rng.uniform(0.2, 1.0)
        onset = int(rng.integers(max_shift, T - burst.size - max_shift))
        u = unit_vectors(az, 0.0)
        # A plane wave from direction u reaches microphone r earlier by (r.u)/c.
        lead = np.floor(fs * (mics @ u) / c + 0.5).astype(np.int64)
        for i in range(8):
            s0 = onset - lead[i]
            x[i, s0:s0 + burst.size] += amp * burst
        refl.append(dict(az=az, el=0.0, amp=amp, onset=onset))
    x += rng.normal(0.0, 0.05, size=x.shape)
    return Frame("burst8", x, mics, dirs, fs, c, order, True, False,
                 truth=dict(reflectors=refl, pulse_len=burst.size))


def echo_frame(rng: np.random.Generator, mics: np.ndarray, dirs: np.ndarray, T: int,
               n_reflectors: int, order: int, fs: float = 450e3, c: float = SPEED_OF_SOUND,
               az_range=(-90.0, 90.0), el_range=(-45.0, 45.0), r_range=(0.3, 5.0),
               chirp=(25e3, 75e3, 1e-3), snr_db: float = 20.0, name: str = "echo",
               apply_matched_filter: bool = True) -> Frame:
    """Pulse-echo frame: a chirp from an emitter at the origin, point reflectors, noise, matched filter.

    Reflector p at range r has amplitude 1/r^2; its echo reaches microphone i after
    (|p| + |p - r_i|)/c and is placed by linear interpolation of the sampled chirp.
    White noise has sigma = RMS(strongest echo over its duration) / 10**(snr/20).
    The matched-filtered FP64 channels are returned.
    """
    M = mics.shape[0]
    pulse = linear_chirp(fs, chirp[0], chirp[1], chirp[2])
    raw = np.zeros((M, T))
    refl = []
    r_hi = min(r_range[1], 0.5 * c * (T - pulse.size - 4) / fs - 0.2)
    for _ in range(n_reflectors):
        r = rng.uniform(r_range[0], r_hi)
        az = rng.uniform(*az_range)
        el = rng.uniform(*el_range)
        p = r * unit_vectors(az, el)
        amp = 1.0 / (r * r)
        dist = np.linalg.norm(p) + np.linalg.norm(p[None, :] - mics, axis=1)
        for i in range(M):
            place_fractional(raw[i], pulse, fs * dist[i] / c, amp)
        refl.append(dict(r=r, az=az, el=el, amp=amp))
    strongest = max(d["amp"] for d in refl) if refl else 1.0
    sigma = strongest * np.sqrt(np.mean(pulse ** 2)) / 10 ** (snr_db / 20.0)
    raw += rng.normal(0.0, sigma, size=raw.shape)
    x = matched_filter(raw, pulse) if apply_matched_filter else raw
    return Frame(name, x, mics, dirs, fs, c, order, True, False,
                 truth=dict(reflectors=refl, pulse_len=pulse.size, sigma=sigma, pulse=pulse))


def ertis_frame(seed_salt: int = 0, order: int = 5, num_samples: int = 16384, matched: bool = True) -> Frame:
    """eRTIS-like pulse-echo frame: 32 mics, 91 x 46 az/el grid, 16384 samples at 450 kHz.

    32 microphones uniform in a 12 cm disc with 4 mm minimum spacing; azimuth
    -90..90 deg and elevation -45..45 deg in 2 deg steps (azimuth fastest);
    25-75 kHz linear chirp of 1 ms; 20 reflectors at 0.3-5 m with 1/r^2
    amplitude; 20 dB SNR; matched filtered (``matched=False``: the raw
    channels of the same scene, the chirp in ``truth["pulse"]``).
    """
    rng = rng_for(2, seed_salt)
    mics = disc_array(rng, 32, 0.12, min_spacing=0.004)
    dirs = az_el_grid(np.arange(-90.0, 90.0 + 1e-9, 2.0), np.arange(-45.0, 45.0 + 1e-9, 2.0))
    return echo_frame(rng, mics, dirs, num_samples, 20, order, name="ertis32", apply_matched_filter=matched)


def precision_frame(seed_salt: int = 0, order: int = 5) -> Frame:
    """Mixed-precision sweep input: ``burst_frame``'s geometry and scene at a chosen order."""
    f = burst_frame(seed_salt, order=order)
    f.name = "precision_sweep"
    return f


def serving_pool(seed_salt: int = 0, n_arrays_per_m: int = 4, frames_per_combo: int = 1,
                 sample_choices=(4096, 8192, 16384), dir_choices=(1024, 2048, 4096, 8192),
                 mic_choices=(16, 32, 64), orders=(3, 5), max_frames: Optional[int] = None) -> List[Frame]:
    """Heterogeneous pulse-echo frames for the serving workload.

    Arrays: ``n_arrays_per_m`` random discs per microphone count, diameter
    U[6, 20] cm. Direction grids: az/el rectangles over +-90/+-45 deg with the
    requested direction counts. Orders and sample counts drawn uniformly.
    """
    rng = rng_for(4, seed_salt)
    arrays = []
    for m in mic_choices:
        for _ in range(n_arrays_per_m):
            dia = rng.uniform(0.06, 0.20)
            arrays.append(disc_array(rng, m, dia, min_spacing=min(0.004, dia / (2.5 * math.sqrt(m)))))
    grids = {}
    for d in dir_choices:
        n_el = int(round(math.sqrt(d / 2.0)))
        n_az = d // n_el
        while n_az * n_el != d:
            n_el -= 1
            n_az = d // n_el
        grids[d] = az_el_grid(np.linspace(-90, 90, n_az), np.linspace(-45, 45, n_el))
    frames = []
    count = (len(arrays) * frames_per_combo) if max_frames is None else max_frames
    for k in range(count):
        mics = arrays[k % len(arrays)]
        d = int(rng.choice(dir_choices))
        T = int(rng.choice(sample_choices))
        n = int(rng.choice(orders))
        fr = echo_frame(rng, mics, grids[d], T, 10, n, name=f"serve{k}")
        frames.append(fr)
    return frames


def nearfield_frame(seed_salt: int = 0, order: int = 3, voxels=(64, 64, 32), num_samples: int = 2048) -> Frame:
    """Near-field passive imaging: 32 x 32 grid (1 cm pitch), 64 x 64 x 32 voxels, 2048 samples at 192 kHz.

    Five broadband sources (unit-variance Gaussian noise band-limited to
    20-80 kHz) at random points of the voxel volume, each reaching microphone i
    after |p - r_i|/c with amplitude 1/|p - r_i| (FFT fractional delay), plus
    uncorrelated sensor noise at 0 dB SNR per channel.
    """
    rng = rng_for(5, seed_salt)
    fs, c, T = 192e3, SPEED_OF_SOUND, num_samples
    mics = grid_array(32, 32, 0.01)
    vox = voxel_grid(voxels[0], voxels[1], voxels[2], (-0.5, 0.5), (-0.5, 0.5), (1.0, 1.5))
    M = mics.shape[0]
    sig = np.zeros((M, T))
    srcs = []
    for _ in range(5):
        p = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(1.0, 1.5)])
        src = bandlimited_noise(rng, T, fs, 20e3, 80e3)
        dist = np.linalg.norm(p[None, :] - mics, axis=1)
        # All channels share one FFT of the source; each gets its own phase ramp.
        S = np.fft.rfft(src)
        k = np.arange(S.shape[0])
        ramps = np.exp(-2j * np.pi * np.outer(fs * dist / c, k) / T)
        sig += np.fft.irfft(S[None, :] * ramps, T, axis=1) / dist[:, None]
        srcs.append(dict(pos=p))
    power = np.mean(sig ** 2, axis=1, keepdims=True)
    x = sig + rng.standard_normal(sig.shape) * np.sqrt(power)
    return Frame("nearfield1024", x, mics, vox, fs, c, order, True, True, truth=dict(sources=srcs))


def random_frame(rng: np.random.Generator, M: int, D: int, T: int, order: int,
                 nearfield: bool = False, use_cf: bool = True, fs: float = 450e3,
                 scale: float = 1.0) -> Frame:
    """Small unstructured frame for edge-case tests: Gaussian channels and random geometry."""
    mics = disc_array(rng, M, 0.08)
    if nearfield:
        dirs = np.stack([rng.uniform(-0.4, 0.4, D), rng.uniform(-0.4, 0.4, D), rng.uniform(0.5, 1.5, D)], axis=-1)
    else:
        dirs = unit_vectors(rng.uniform(-80, 80, D), rng.uniform(-40, 40, D))
    x = rng.standard_normal((M, T)) * scale
    return Frame("random", x, mics, dirs, fs, SPEED_OF_SOUND, order, use_cf, nearfield)



def point_scene_frame(mics: np.ndarray, reflectors: Sequence[tuple], az_deg: Sequence[float],
                      num_samples: int, lead_samples: int, snr_db: Optional[float] = None,
                      stream: int = 7, seed_salt: int = 0, order: int = 5, name: str = "scene") -> Frame:
    """Point reflectors in the horizontal plane imaged by ``mics`` (Section III-A simulations).

    ``reflectors`` holds (azimuth in degrees, range in metres, amplitude) at
    elevation 0. An emitter at the origin sends the 25-75 kHz chirp of 1 ms; the
    echo of reflector p reaches microphone i after (|p| + |p - r_i|)/c with the
    given amplitude in every channel (no spreading loss, the paper's
    normalisation of a unit echo), placed by linear interpolation of the sampled
    chirp. The record starts ``lead_samples`` after emission. With ``snr_db``
    white noise of standard deviation 10**(-snr_db/20) is added before matched
    filtering, eqs. (15)-(16). Directions: the azimuths ``az_deg`` at elevation 0.
    """
    rng = rng_for(stream, seed_salt)
    fs, c, T = 450e3, SPEED_OF_SOUND, num_samples
    M = mics.shape[0]
    pulse = linear_chirp(fs, 25e3, 75e3, 1e-3)
    raw = np.zeros((M, T))
    onsets = []
    for az, rng_m, amp in reflectors:
        p = rng_m * unit_vectors(az, 0.0)
        dist = np.linalg.norm(p) + np.linalg.norm(p[None, :] - mics, axis=1)
        for i in range(M):
            place_fractional(raw[i], pulse, fs * dist[i] / c - lead_samples, amp)
        onsets.append(int(round(fs * 2.0 * rng_m / c)) - lead_samples)
    if snr_db is not None:
        raw += rng.standard_normal(raw.shape) * 10 ** (-snr_db / 20.0)
    x = matched_filter(raw, pulse)
    az = np.asarray(az_deg, dtype=np.float64)
    return Frame(name, x, mics, az_el_grid(az, [0.0]), fs, c, order, True, False,
                 truth=dict(az=az, reflectors=list(reflectors), onsets=onsets, pulse_len=pulse.size))


def two_reflector_frame(half_angle_deg: float, order: int = 5, az_step: float = 0.25) -> Frame:
    """Two unit reflectors at 1.5 m, symmetric about the forward axis at azimuths +-half_angle
    (the spatial-resolution experiment of Section III-A), seen by the 32-microphone 12 cm disc
    of ``point_echo_frame``; azimuths -30..30 deg, 1024 samples with the echoes near sample 300."""
    mics = disc_array(np.random.default_rng(SEED_BASE + 6), 32, 0.12, min_spacing=0.004)
    lead = int(round(450e3 * 2.0 * 1.5 / SPEED_OF_SOUND)) - 300
    refl = [(-half_angle_deg, 1.5, 1.0), (half_angle_deg, 1.5, 1.0)]
    return point_scene_frame(mics, refl, np.arange(-30.0, 30.0 + 1e-9, az_step), 1024, lead,
                             stream=8, order=order, name="two_reflectors")


def hex_psf_frame(radius: float, order: int = 5, az_step: float = 0.25) -> Frame:
    """Noise-free broadside reflector at 1 m seen by a hexagonal-lattice disc array of 5 mm edge and
    the given radius (the beamwidth experiment of Section III-A, 19-513 microphones for radii of
    1-6 cm); azimuths -45..45 deg, 1024 samples with the echo near sample 300."""
    mics = hex_disc_array(radius, 0.005)
    lead = int(round(450e3 * 2.0 / SPEED_OF_SOUND)) - 300
    return point_scene_frame(mics, [(0.0, 1.0, 1.0)], np.arange(-45.0, 45.0 + 1e-9, az_step), 1024, lead,
                             stream=9, order=order, name=f"hex_r{radius * 100:.0f}cm")


def point_echo_frame(order: int = 5, snr_db: Optional[float] = None, seed_salt: int = 0,
                     num_samples: int = 2048, az_step: float = 1.0, lead_samples: int = 600) -> Frame:
    """Single point reflector at 1 m broadside, for point-spread and image-SNR studies.

    32 microphones in a 12 cm disc (4 mm minimum spacing), a 25-75 kHz chirp of
    1 ms, echo amplitude 1 in every channel; with ``snr_db`` white noise of
    standard deviation 10**(-snr_db/20) is added before matched filtering (the
    paper's image-SNR procedure, Section III-A). The record starts
    ``lead_samples`` after emission so the echo lies inside it. Directions:
    azimuths -90..90 deg at elevation 0.
    """
    rng = rng_for(6, seed_salt)
    fs, c, T = 450e3, SPEED_OF_SOUND, num_samples
    mics = disc_array(np.random.default_rng(SEED_BASE + 6), 32, 0.12, min_spacing=0.004)
    az = np.arange(-90.0, 90.0 + 1e-9, az_step)
    dirs = az_el_grid(az, [0.0])
    pulse = linear_chirp(fs, 25e3, 75e3, 1e-3)
    raw = np.zeros((32, T))
    p = unit_vectors(0.0, 0.0)
    dist = np.linalg.norm(p) + np.linalg.norm(p[None, :] - mics, axis=1)
    for i in range(32):
        place_fractional(raw[i], pulse, fs * dist[i] / c - lead_samples, 1.0)
    if snr_db is not None:
        raw += rng.standard_normal(raw.shape) * 10 ** (-snr_db / 20.0)
    x = matched_filter(raw, pulse)
    return Frame("psf", x, mics, dirs, fs, c, order, True, False,
                 truth=dict(az=az, target_az=0.0, onset=int(round(fs * 2.0 / c)) - lead_samples))
