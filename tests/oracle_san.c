/* The FP64 oracle (oracle/dmas_oracle.c) on the CPU, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py:
 * every entry point on small seeded inputs (edges: one microphone, one sample,
 * delays that reach past both ends of the record, all orders, FIR length 1,
 * pulses longer than the record, row subsets, nearest and linear delays, near
 * and far field, CF on and off) and on invalid arguments. Prints "ok <calls>"
 * or the first failure and exits with status 1. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_delays(int M, int D, const double *mic_pos, const double *dirs, int nearfield, double fs, double c,
                  int64_t *out);
int oracle_delays_frac(int M, int D, const double *mic_pos, const double *dirs, int nearfield, double fs, double c,
                       int64_t *whole, double *frac);
int oracle_dmas_rows(int M, int T, int D, const double *x, const double *mic_pos, const double *dirs, int nearfield,
                     double fs, double c, int order, int use_cf, double cf_eps, int interp, int n_rows,
                     const int64_t *rows, double *y_out, double *diag);
int oracle_envelope(int R, int T, const double *y, int L, const double *taps, double *env);
int oracle_lowpass_taps(int L, double fc, double fs, double *taps);
int oracle_matched_filter(int M, int T, const double *raw, int P, const double *pulse, double *out);

static int calls = 0;
static uint64_t state = 2511091650u;

static double urand(void)
{
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

#define MUST(expr, want)                                                 \
    do {                                                                 \
        ++calls;                                                         \
        if ((expr) != (want)) {                                          \
            printf("failed: %s returned %d, want %d\n", #expr, (int)(expr), (int)(want)); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void)
{
    enum { MMAX = 9, DMAX = 6, TMAX = 40 };
    double mic[3 * MMAX], dirs[3 * DMAX], vox[3 * DMAX], x[MMAX * TMAX], y[DMAX * TMAX], env[DMAX * TMAX];
    double diag[DMAX * TMAX * 6], taps[255], frac[DMAX * MMAX], pulse[60], mf[MMAX * TMAX];
    int64_t whole[DMAX * MMAX], rows[DMAX];
    for (int i = 0; i < MMAX; ++i) {
        mic[3 * i] = 0.02 * urand();
        mic[3 * i + 1] = 0.02 * urand();
        mic[3 * i + 2] = 0.0;
    }
    for (int p = 0; p < DMAX; ++p) {
        double az = 1.2 * urand(), el = 0.5 * urand();
        dirs[3 * p] = cos(el) * sin(az);
        dirs[3 * p + 1] = sin(el);
        dirs[3 * p + 2] = cos(el) * cos(az);
        vox[3 * p] = 0.2 * urand();
        vox[3 * p + 1] = 0.2 * urand();
        vox[3 * p + 2] = 0.3 + 0.1 * urand();
        rows[p] = DMAX - 1 - p;
    }
    for (int k = 0; k < MMAX * TMAX; ++k) x[k] = (k % 7 == 0) ? 0.0 : urand();
    for (int k = 0; k < 60; ++k) pulse[k] = urand();

    /* fs large enough that delays reach past both ends of the short records */
    const double fs = 4.0e6, c = 343.0;
    for (int near = 0; near < 2; ++near) {
        const double *g = near ? vox : dirs;
        MUST(oracle_delays(MMAX, DMAX, mic, g, near, fs, c, whole), 0);
        MUST(oracle_delays_frac(MMAX, DMAX, mic, g, near, fs, c, whole, frac), 0);
        for (int M = 1; M <= MMAX; M += 4)
            for (int T = 1; T <= TMAX; T += 13)
                for (int n = 1; n <= M && n <= 8; ++n)
                    for (int cf = 0; cf < 2; ++cf)
                        for (int interp = 0; interp < 2; ++interp) {
                            MUST(oracle_dmas_rows(M, T, DMAX, x, mic, g, near, fs, c, n, cf, 1e-20, interp, DMAX,
                                                  rows, y, diag),
                                 0);
                            MUST(oracle_dmas_rows(M, T, DMAX, x, mic, g, near, fs, c, n, cf, 1e-20, interp, 2, rows,
                                                  y, NULL),
                                 0);
                        }
    }
    for (int L = 1; L <= 255; L += 62) {
        MUST(oracle_lowpass_taps(L, 5000.0, 450e3, taps), 0);
        MUST(oracle_envelope(DMAX, TMAX, y, L, taps, env), 0);
        MUST(oracle_envelope(DMAX, 1, y, L, taps, env), 0);
    }
    MUST(oracle_matched_filter(MMAX, TMAX, x, 60, pulse, mf), 0);   /* pulse longer than the record */
    MUST(oracle_matched_filter(1, 1, x, 1, pulse, mf), 0);
    /* invalid arguments are refused without touching memory */
    MUST(oracle_dmas_rows(0, TMAX, DMAX, x, mic, dirs, 0, fs, c, 1, 1, 1e-20, 0, DMAX, rows, y, NULL), 1);
    MUST(oracle_dmas_rows(2, TMAX, DMAX, x, mic, dirs, 0, fs, c, 3, 1, 1e-20, 0, DMAX, rows, y, NULL), 1);
    MUST(oracle_dmas_rows(MMAX, TMAX, DMAX, x, mic, dirs, 0, fs, c, 17, 1, 1e-20, 0, DMAX, rows, y, NULL), 1);
    rows[0] = DMAX;
    MUST(oracle_dmas_rows(MMAX, TMAX, DMAX, x, mic, dirs, 0, fs, c, 2, 1, 1e-20, 0, DMAX, rows, y, NULL), 1);
    rows[0] = -1;
    MUST(oracle_dmas_rows(MMAX, TMAX, DMAX, x, mic, dirs, 0, fs, c, 2, 1, 1e-20, 0, DMAX, rows, y, NULL), 1);
    MUST(oracle_envelope(DMAX, TMAX, y, 64, taps, env), 1);
    MUST(oracle_lowpass_taps(63, 225e3, 450e3, taps), 1);
    MUST(oracle_lowpass_taps(0, 5000.0, 450e3, taps), 1);
    MUST(oracle_matched_filter(MMAX, TMAX, x, 0, pulse, mf), 1);
    MUST(oracle_delays(0, DMAX, mic, dirs, 0, fs, c, whole), 1);
    MUST(oracle_delays_frac(MMAX, DMAX, mic, dirs, 0, fs, c, whole, NULL), 1);
    printf("ok %d\n", calls);
    return 0;
}
