"""Tolerances for comparing the FP32 GPU path with the FP64 oracle.

T1 (the stated relative tolerance): max |y - y_ref| / max |y_ref| <= 1e-4 over
   the image (peak-normalised, the display normalisation of the paper's images).
T2 (per pixel, conditioning-aware): a first-order rounding-error bound of the
   FP32 evaluation, built from the oracle's per-pixel diagnostics:
     root:   s = exp2(log2|x| / n) has relative error rho <= (4 + 2 max|log2|x||) u
     sums:   |dP_k| <= (M u + k (rho + u)) Q_k,  Q_k = sum |s_i|^k
     NG:     sum over partitions (eq. (8)) of |coef| prod Q  =  h_n(|s|)
             so |dE| <= (n (M + n) u + n^2 rho + 10 u) h_n
     CF:     |dCF| <= 2 |A| M u sum|x| / (M B + eps) + (M + 3) u CF
     y:      |dy| <= |dE| CF + |E| |dCF| + 3 u |y|
   with a safety factor of 4. u = 2^-24.
T3 (envelope, dB): pixels above -60 dB of the peak agree within 0.01 dB.
"""

from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def root_rel_error(x: np.ndarray) -> float:
    ax = np.abs(x[np.isfinite(x) & (x != 0)])
    lg = float(np.abs(np.log2(ax)).max()) if ax.size else 0.0
    return (4.0 + 2.0 * lg) * U32


def y_bound(diag: dict, M: int, n: int, use_cf: bool, rho: float, cf_eps: float = 1e-20,
            safety: float = 4.0) -> np.ndarray:
    h = diag["h"]
    E = diag["E"]
    cf = diag["CF"] if use_cf else np.ones_like(E)
    dE = (n * (M + n) * U32 + n * n * rho + 10 * U32) * h
    if use_cf:
        A, B, S = diag["sum_x"], diag["sum_x2"], diag["sum_abs"]
        dcf = 2 * np.abs(A) * M * U32 * S / (M * B + cf_eps) + (M + 3) * U32 * cf
    else:
        dcf = 0.0
    y = E * cf
    return safety * (dE * cf + np.abs(E) * dcf + 3 * U32 * np.abs(y)) + 1e-37


def env_bound(y_tol: np.ndarray, y_ref: np.ndarray, taps: np.ndarray, envelope_fn) -> np.ndarray:
    """Propagate per-pixel y bounds through env = sum |h| |y| plus FP32 accumulation of L terms."""
    ah = np.abs(np.asarray(taps, dtype=np.float64))
    L = ah.size
    return envelope_fn(y_tol, ah) + 2 * L * U32 * envelope_fn(y_ref, ah) + 1e-37


def check_t1(got: np.ndarray, ref: np.ndarray, tol: float = 1e-4) -> float:
    peak = np.abs(ref).max()
    err = float(np.abs(got - ref).max() / peak) if peak > 0 else float(np.abs(got).max())
    assert err <= tol, f"T1 peak-normalised error {err:.3e} > {tol:.1e}"
    return err


def check_t2(got: np.ndarray, ref: np.ndarray, bound: np.ndarray) -> float:
    excess = np.abs(got - ref) / bound
    worst = float(excess.max())
    if worst > 1.0:
        idx = np.unravel_index(int(np.argmax(excess)), excess.shape)
        raise AssertionError(f"T2 per-pixel bound exceeded by {worst:.2f}x at {idx}: "
                             f"got {got[idx]!r} ref {ref[idx]!r} bound {bound[idx]!r}")
    return worst


def check_t3(env: np.ndarray, env_ref: np.ndarray, floor_db: float = -60.0, tol_db: float = 0.01) -> float:
    peak = np.abs(env_ref).max()
    if peak == 0:
        assert np.all(env == 0), "reference envelope is zero but the result is not"
        return 0.0
    mask = env_ref >= peak * 10 ** (floor_db / 20.0)
    if not mask.any():
        return 0.0
    db = np.abs(20 * np.log10(np.maximum(env[mask], 1e-300) / env_ref[mask]))
    worst = float(db.max())
    assert worst <= tol_db, f"T3 envelope deviation {worst:.4f} dB > {tol_db} dB"
    return worst


def delay_rounding_ties(fs: float = 450e3, c: float = 343.0, count: int = 24, span: int = 3000):
    """Mic x-coordinates (metres, far-field direction (1, 0, 0)) whose whole-sample delay
    floor(fs * tau + 1/2), tau = -x / c, evaluated as separately rounded IEEE double
    operations differs from the value a fused multiply-add fs * tau + 1/2 would give.
    Returns [(x, unfused, fused)]; used to check that delays follow the unfused sequence."""
    import math
    from fractions import Fraction
    out = []
    half = Fraction(1, 2)
    for k in range(-60, 60):
        x0 = (k + 0.5) * c / fs
        cand = [x0]
        for direction in (-math.inf, math.inf):
            v = x0
            for _ in range(span):
                v = float(np.nextafter(v, direction))
                cand.append(v)
        for x in cand:
            tau = -x / c
            unfused = math.floor(fs * tau + 0.5)
            fused = math.floor(Fraction(fs) * Fraction(tau) + half)
            if unfused != fused:
                out.append((x, unfused, fused))
                break
        if len(out) >= count:
            break
    return out
