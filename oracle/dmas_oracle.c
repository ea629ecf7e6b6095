/*
 * FP64 CPU oracle for n-th order Delay-Multiply-and-Sum beamforming with
 * Coherence-Factor weighting and envelope detection.
 *
 * TEST INFRASTRUCTURE ONLY. This file exists to check the GPU library against
 * a plain, slow, obviously correct evaluation of the paper's definitions. Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load it;
 * the product library neither links nor calls it, and it shares no code with
 * the GPU path.
 *
 * What it computes, in the paper's order (Jansen, Daems, Steckel, "Delay-
 * Multiply-And-Sum Beamforming for Real-Time In-Air Acoustic Imaging"):
 *   1. Pre-steering, Section II, eq. (1): x_i(t, psi) = m_i(t + tau_{i,psi}).
 *      The delay is rounded to the nearest sample (round half up) in FP64,
 *      or, with linear interpolation selected, split into whole and fractional
 *      samples. Samples outside the record are zero.
 *   2. Signed n-th root, eq. (4): s_i = sgn(x_i) |x_i|^(1/n), sgn(0) = 0.
 *   3. DMAS of order n, eqs. (5)/(6): the n-th elementary symmetric polynomial
 *      E_n of s_1..s_M. Evaluated here from its generating function: E_n is
 *      the coefficient of z^n in prod_i (1 + s_i z). This reaches the same
 *      number as the sum over all n-subsets, with no cancellation beyond what
 *      the definition itself carries. (The Newton-Girard power-sum route of
 *      eqs. (7)-(12) is what the GPU path uses; it is not used here.)
 *   4. Coherence factor, eq. (13), on the delayed signals x_i:
 *      CF = (sum x_i)^2 / (M sum x_i^2 + eps), and eq. (14): y = E_n * CF.
 *   5. Envelope (Section II, step 3 of the pipeline): |y| filtered by a
 *      zero-phase FIR, env[t] = sum_k h[k] |y[t + (L-1)/2 - k]|, y = 0 outside
 *      the record.
 * Upstream of the beamformer (pipeline step 1 of Section II), the matched
 * filter correlates each raw channel with the emitted pulse:
 * r[t] = sum_k m[t + k] p[k], m = 0 beyond the record.
 * Diagnostics (optional): per pixel E_n, CF, the complete homogeneous
 * symmetric polynomial h_n(|s|) (the error-amplification scale of any
 * power-sum evaluation of E_n), sum x, sum x^2 and sum |x|.
 *
 * Build: plain C11, -O2 -ffp-contract=off -fopenmp, libm only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_ORDER 16
#define ORACLE_DIAG 6

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later calls (n >= 1); timing only, results do not depend on it. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Steering delay of eq. (1) in samples, before rounding: fs * tau.
 * Far field (v is a unit vector toward the source): a plane wave from v
 * reaches microphone r earlier by (r . v)/c than it reaches the origin, so
 * tau = -(r . v)/c re-aligns it.
 * Near field (v is a point): tau = (|v - r| - |v|)/c aligns a spherical wave
 * from v to its arrival time at the origin.
 * The arithmetic is written as a fixed sequence of IEEE operations (no fused
 * multiply-add) so that the result is reproducible.
 */
static double steer_samples(const double *r, const double *v, int nearfield,
                            double fs, double c)
{
    double tau;
    if (!nearfield) {
        double dot = r[0] * v[0];
        dot = dot + r[1] * v[1];
        dot = dot + r[2] * v[2];
        tau = -dot / c;
    } else {
        double dx = v[0] - r[0];
        double dy = v[1] - r[1];
        double dz = v[2] - r[2];
        double q = dx * dx;
        q = q + dy * dy;
        q = q + dz * dz;
        double q0 = v[0] * v[0];
        q0 = q0 + v[1] * v[1];
        q0 = q0 + v[2] * v[2];
        tau = (sqrt(q) - sqrt(q0)) / c;
    }
    return fs * tau;
}

/* Nearest-sample delay: floor(fs*tau + 1/2). */
static int64_t steer_nearest(const double *r, const double *v, int nearfield,
                             double fs, double c)
{
    return (int64_t)floor(steer_samples(r, v, nearfield, fs, c) + 0.5);
}

/* Whole-sample delay table, D x M, row-major. */
int oracle_delays(int M, int D, const double *mic_pos, const double *dirs,
                  int nearfield, double fs, double c, int64_t *out)
{
    if (M < 1 || D < 1 || !mic_pos || !dirs || !out)
        return 1;
    for (int p = 0; p < D; ++p)
        for (int i = 0; i < M; ++i)
            out[(int64_t)p * M + i] =
                steer_nearest(mic_pos + 3 * i, dirs + 3 * p, nearfield, fs, c);
    return 0;
}

/* Fractional delay table: whole part q = floor(fs*tau) and fraction
 * phi = fs*tau - q, both D x M. */
int oracle_delays_frac(int M, int D, const double *mic_pos, const double *dirs,
                       int nearfield, double fs, double c, int64_t *whole,
                       double *frac)
{
    if (M < 1 || D < 1 || !mic_pos || !dirs || !whole || !frac)
        return 1;
    for (int p = 0; p < D; ++p)
        for (int i = 0; i < M; ++i) {
            double f = steer_samples(mic_pos + 3 * i, dirs + 3 * p, nearfield, fs, c);
            double q = floor(f);
            whole[(int64_t)p * M + i] = (int64_t)q;
            frac[(int64_t)p * M + i] = f - q;
        }
    return 0;
}

/* Signed n-th root, eq. (4), with sgn(0) = 0. */
static double signed_root(double x, int n)
{
    if (n == 1)
        return x;
    if (x == 0.0)
        return 0.0;
    return copysign(pow(fabs(x), 1.0 / (double)n), x);
}

static double sample_or_zero(const double *ch, int64_t T, int64_t idx)
{
    return (idx >= 0 && idx < T) ? ch[idx] : 0.0;
}

/*
 * DMAS-n (+CF) image rows. For each requested direction index rows[r], writes
 * y_out[r*T + t] for every t in [0, T). x is M x T row-major FP64.
 * interp = 0: nearest-sample delays; interp = 1: linear interpolation between
 * the two samples around t + fs*tau.
 * diag (optional): ORACLE_DIAG doubles per pixel:
 *   {E_n, CF (1 if disabled), h_n(|s|), sum x, sum x^2, sum |x|}.
 */
int oracle_dmas_rows(int M, int T, int D, const double *x, const double *mic_pos,
                     const double *dirs, int nearfield, double fs, double c,
                     int order, int use_cf, double cf_eps, int interp,
                     int n_rows, const int64_t *rows, double *y_out, double *diag)
{
    if (M < 1 || T < 1 || D < 1 || order < 1 || order > ORACLE_MAX_ORDER ||
        order > M || n_rows < 0 || !x || !mic_pos || !dirs || !rows || !y_out)
        return 1;
    for (int r = 0; r < n_rows; ++r)
        if (rows[r] < 0 || rows[r] >= D)
            return 1;

    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rows; ++r) {
        const double *v = dirs + 3 * rows[r];
        int64_t *dw = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
        double *df = (double *)malloc(sizeof(double) * (size_t)M);
        if (!dw || !df) {
            free(dw);
            free(df);
#pragma omp atomic write
            err = 2;
            continue;
        }
        for (int i = 0; i < M; ++i) {
            double f = steer_samples(mic_pos + 3 * i, v, nearfield, fs, c);
            if (interp) {
                double q = floor(f);
                dw[i] = (int64_t)q;
                df[i] = f - q;
            } else {
                dw[i] = (int64_t)floor(f + 0.5);
                df[i] = 0.0;
            }
        }
        for (int64_t t = 0; t < T; ++t) {
            double e[ORACLE_MAX_ORDER + 1];
            double h[ORACLE_MAX_ORDER + 1];
            double sum_x = 0.0, sum_x2 = 0.0, sum_abs = 0.0;
            e[0] = 1.0;
            h[0] = 1.0;
            for (int k = 1; k <= order; ++k) {
                e[k] = 0.0;
                h[k] = 0.0;
            }
            for (int i = 0; i < M; ++i) {
                const double *ch = x + (int64_t)i * T;
                double xi;
                if (interp) {
                    double a = sample_or_zero(ch, T, t + dw[i]);
                    double b = sample_or_zero(ch, T, t + dw[i] + 1);
                    xi = (1.0 - df[i]) * a + df[i] * b;
                } else {
                    xi = sample_or_zero(ch, T, t + dw[i]);
                }
                double s = signed_root(xi, order);
                /* coefficient of z^k in prod (1 + s z): descending k */
                for (int k = order; k >= 1; --k)
                    e[k] += s * e[k - 1];
                /* complete homogeneous polynomial of |s|: ascending k */
                double a = fabs(s);
                for (int k = 1; k <= order; ++k)
                    h[k] += a * h[k - 1];
                sum_x += xi;
                sum_x2 += xi * xi;
                sum_abs += fabs(xi);
            }
            double cf = 1.0;
            if (use_cf)
                cf = (sum_x * sum_x) / ((double)M * sum_x2 + cf_eps);
            double y = e[order] * cf;
            y_out[(int64_t)r * T + t] = y;
            if (diag) {
                double *dg = diag + ((int64_t)r * T + t) * ORACLE_DIAG;
                dg[0] = e[order];
                dg[1] = cf;
                dg[2] = h[order];
                dg[3] = sum_x;
                dg[4] = sum_x2;
                dg[5] = sum_abs;
            }
        }
        free(dw);
        free(df);
    }
    return err;
}

/* Envelope of R rows of length T: env[t] = sum_k h[k] |y[t + (L-1)/2 - k]|. */
int oracle_envelope(int R, int T, const double *y, int L, const double *taps,
                    double *env)
{
    if (R < 0 || T < 1 || L < 1 || (L % 2) == 0 || !y || !taps || !env)
        return 1;
    int64_t H = (L - 1) / 2;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
        const double *row = y + (int64_t)r * T;
        for (int64_t t = 0; t < T; ++t) {
            double acc = 0.0;
            for (int k = 0; k < L; ++k) {
                int64_t j = t + H - k;
                if (j >= 0 && j < T)
                    acc += taps[k] * fabs(row[j]);
            }
            env[(int64_t)r * T + t] = acc;
        }
    }
    return 0;
}

/*
 * Default envelope low-pass (the paper states a 5 kHz low-pass without its
 * design): Hamming-windowed ideal low-pass of odd length L and cut-off fc,
 * normalised to unit gain at DC.
 */
int oracle_lowpass_taps(int L, double fc, double fs, double *taps)
{
    if (L < 1 || (L % 2) == 0 || !(fc > 0.0) || !(fs > 0.0) || fc >= 0.5 * fs || !taps)
        return 1;
    const double pi = 3.14159265358979323846;
    int H = (L - 1) / 2;
    double wc = 2.0 * fc / fs; /* cut-off as a fraction of Nyquist */
    double sum = 0.0;
    for (int k = 0; k < L; ++k) {
        double m = (double)(k - H);
        double ideal = (m == 0.0) ? wc : sin(pi * wc * m) / (pi * m);
        double w = (L == 1) ? 1.0 : 0.54 - 0.46 * cos(2.0 * pi * k / (double)(L - 1));
        taps[k] = ideal * w;
        sum += taps[k];
    }
    for (int k = 0; k < L; ++k)
        taps[k] /= sum;
    return 0;
}

/* Matched filter (pulse compression): out[i*T + t] = sum_{k<P} raw[i*T + t + k] * pulse[k],
 * with raw = 0 beyond the record. */
int oracle_matched_filter(int M, int T, const double *raw, int P, const double *pulse, double *out)
{
    if (M < 1 || T < 1 || P < 1 || !raw || !pulse || !out)
        return 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < M; ++i) {
        const double *ch = raw + (int64_t)i * T;
        for (int64_t t = 0; t < T; ++t) {
            double acc = 0.0;
            for (int k = 0; k < P && t + k < T; ++k)
                acc += ch[t + k] * pulse[k];
            out[(int64_t)i * T + t] = acc;
        }
    }
    return 0;
}
